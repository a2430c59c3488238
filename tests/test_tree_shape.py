"""The shape of the tree, pinned on the CPU through the instrumented mirror
of Eq. (5) and Eq. (6) in tests/tree_mirror.py (not the oracle, not the
product): the level-1 pairing printed in the Fig. 1 caption, the operation
count of Eq. (8) for every radix-2 window up to 32 x 32, and the last level
equal to numpy.fft.fft2 of each window (so the mirror that does the counting
computes the transform the paper defines)."""
import json
import os

import numpy as np
import pytest

from tests.tree_mirror import TreeMirror

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_values.json")))

SIDES = (1, 2, 4, 8, 16, 32)


def test_fig1_level1_pairing():
    """Fig. 1 caption (butterfly diagram, n = 8): the first calculation on
    the bottom left multiplies x_7 by omega^4 and adds it to x_3. In the tree
    this is level 1 of the tree under x_7: node i = 1 combines x_{7 - n/2}
    (added) and x_7 (multiplied by Omega[1 * n/2] = omega^4 = -1), and no
    other input. Read off by feeding impulses (the node is linear in x)."""
    g = GOLDEN["fig1_level1_pairing"]
    n, p = g["n"], g["tree_position"]
    coef = np.zeros(n + 1, dtype=np.complex128)
    for j in range(n + 1):
        x = np.zeros((1, n + 1))
        x[0, j] = 1.0
        m = TreeMirror(x, 1, n).run()
        coef[j] = m.levels[1][0, p, 0, 1]
    nz = [j for j in range(n + 1) if abs(coef[j]) > 1e-12]
    assert sorted(nz) == sorted([g["added_input"], g["multiplied_input"]])
    assert coef[g["added_input"]] == 1.0  # added without a multiply
    # multiplied by omega^twiddle_power with omega = exp(-2 pi i / n): -1 at power n/2
    assert np.isclose(coef[g["multiplied_input"]], np.exp(-2j * np.pi * g["twiddle_power"] / n),
                      atol=1e-15)
    assert g["twiddle_power"] == n // 2 and g["added_input"] == p - n // 2
    # node i = 0 of the same tree is the plain sum of the same two inputs
    x = np.zeros((1, n + 1))
    x[0, g["added_input"]] = 2.0
    x[0, g["multiplied_input"]] = 3.0
    assert TreeMirror(x, 1, n).run().levels[1][0, p, 0, 0] == 5.0


@pytest.mark.parametrize("n0", SIDES)
@pytest.mark.parametrize("n1", SIDES)
def test_ops_per_complete_tree(n0, n1):
    """Eq. (8): every complete tree (one per window) takes exactly
    2(n0 n1 - 1) node operations: 2(n1 - 1) at the row levels and
    2 n1 (n0 - 1) at the column levels. The level-l node count of a complete
    tree is 2^l along the row levels and n1 2^u along the column levels."""
    rng = np.random.default_rng(100 * n0 + n1)
    N0, N1 = n0 + 2, n1 + 3
    x = rng.standard_normal((N0, N1))
    m = TreeMirror(x, n0, n1).run()
    full = m.complete_trees()
    assert len(full) == (N0 - n0 + 1) * (N1 - n1 + 1)
    for (a, b) in full:
        assert m.ops[a, b] == 2 * (n0 * n1 - 1), (a, b)
    # per level, at one complete tree: nodes that exist there
    a, b = full[-1]
    for lvl in range(1, m.m1 + m.m0 + 1):
        nodes = np.count_nonzero(~np.isnan(m.levels[lvl][a, b].real))
        want = (1 << lvl) if lvl <= m.m1 else n1 << (lvl - m.m1)
        assert nodes == want, lvl


def test_ops_per_window_golden_cases():
    """The worked values of Eq. (8) recorded in the golden file, counted by
    the mirror (not recomputed from the formula)."""
    for n0, n1, ops in GOLDEN["ops_per_window"]["cases"]:
        x = np.random.default_rng(n0 * 64 + n1).standard_normal((n0 + 1, n1 + 1))
        m = TreeMirror(x, n0, n1).run()
        counts = {int(m.ops[a, b]) for (a, b) in m.complete_trees()}
        assert counts == {ops}, (n0, n1, counts)


@pytest.mark.parametrize("n0,n1", [(1, 8), (4, 4), (2, 8), (8, 2), (16, 4), (4, 32), (32, 8),
                                   (32, 32)])
def test_last_level_is_fft2_of_each_window(n0, n1):
    """The mirror's last level at the tree under (q0 + n0 - 1, q1 + n1 - 1) is
    numpy.fft.fft2 of the window with top-left corner (q0, q1), bins in
    natural order (no bit reversal)."""
    rng = np.random.default_rng(7 * n0 + n1)
    N0, N1 = n0 + 3, n1 + 2
    x = rng.standard_normal((N0, N1)) + 1j * rng.standard_normal((N0, N1))
    m = TreeMirror(x, n0, n1).run()
    for q0 in range(N0 - n0 + 1):
        for q1 in range(N1 - n1 + 1):
            ref = np.fft.fft2(x[q0:q0 + n0, q1:q1 + n1])
            got = m.window(q0, q1)
            assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_incomplete_trees_hold_no_top_level():
    """Sec. 4.7: trees near the top and left edges never reach the last
    level; exactly P0 x P1 trees do."""
    n0, n1 = 4, 8
    m = TreeMirror(np.ones((9, 13)), n0, n1).run()
    has_top = ~np.isnan(m.top[:, :, 0, 0].real)
    assert has_top.sum() == (9 - n0 + 1) * (13 - n1 + 1)
    assert not has_top[: n0 - 1, :].any() and not has_top[:, : n1 - 1].any()


class _ShiftOffByOne(TreeMirror):
    def shift(self, n, level):
        s = n >> level
        return s + 1 if level == 1 and n >= 4 else s


class _ConjugateTwiddles(TreeMirror):
    def twiddles(self, n):
        return np.conj(super().twiddles(n))


class _SwappedOperands(TreeMirror):
    def combine(self, added, multiplied, w):
        return multiplied + w * added


class _DroppedTwiddle(TreeMirror):
    def combine(self, added, multiplied, w):
        return added + multiplied


@pytest.mark.parametrize("broken", [_ShiftOffByOne, _ConjugateTwiddles, _SwappedOperands,
                                    _DroppedTwiddle])
def test_pins_catch_planted_mistakes(broken):
    """Each planted mistake in the mirror's node (shift, twiddle sign,
    operand order, dropped multiply) breaks the fft2 pin or the Fig. 1
    pairing, so those pins check the indexing the operation counts use."""
    rng = np.random.default_rng(5)
    n0, n1 = 4, 8
    x = rng.standard_normal((n0 + 3, n1 + 3)) + 1j * rng.standard_normal((n0 + 3, n1 + 3))
    m = broken(x, n0, n1).run()
    fft_ok = all(np.allclose(m.window(q0, q1), np.fft.fft2(x[q0:q0 + n0, q1:q1 + n1]),
                             atol=1e-9, equal_nan=False)
                 for q0 in range(4) for q1 in range(4))
    g = GOLDEN["fig1_level1_pairing"]
    n, p = g["n"], g["tree_position"]
    xi = np.zeros((1, n + 1))
    xi[0, g["multiplied_input"]] = 1.0
    pairing_ok = np.isclose(broken(xi, 1, n).run().levels[1][0, p, 0, 1],
                            np.exp(-2j * np.pi * g["twiddle_power"] / n))
    assert not (fft_ok and pairing_ok)
