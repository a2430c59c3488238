"""The priming rule of the forward tree's slabs, checked on the CPU.

A slab of the GPU tree starts at window row q and first walks the n0 - 1
input rows of that window before its first output. In that first stretch it
computes column level u (Eq. (6)) of row q + t only when t >= n0 - s_u
(s_u = n0 / 2^u), keeps in the ring the level-(u-1) value of row q + t only
when t >= n0 - 2 s_u, and emits nothing before t = n0 - 1. The reason: level
u of row p feeds level u+1 at rows p and p + s_{u+1}, hence only the windows
ending at rows p .. p + s_u - 1.

This module walks one column stream the way the kernel does (level u-1 of
the last s_u rows in a ring, slot p mod s_u, node pairs
T_u[p][i] = T_{u-1}[p-s_u][i] +/- Omega0[i s_u] T_{u-1}[p][i]), in
complex128, with the rule switched on or off. Ring slots start as NaN, so an
output that read anything the rule skipped would be NaN; every output must
equal numpy.fft.fft of its window (a library routine, independent of the
walk). It also counts the node pairs the rule drops, against the closed form
sum_u 2^(u-1) (n0 - s_u) (208 of the 225 pairs of the 15 priming rows at
n0 = 16), and walks the mixed-radix stream (levels of radix 2, then 3) under
the same rule. Test infrastructure only: the GPU kernels are checked against the
oracle by the GPU tests, on many slab layouts.
"""
from __future__ import annotations

import numpy as np
import pytest


def walk(z, n0, prune=True, compute_from=None, keep_from=None):
    """Outputs {t: n0 values} for every step t >= n0 - 1 and the number of
    node pairs computed. compute_from(u) / keep_from(u) give the first step
    at which level u is computed / level u-1 is kept in the ring (the rule
    by default; a test passes other thresholds to plant a mistake)."""
    m0 = n0.bit_length() - 1
    w = np.exp(-2j * np.pi * np.arange(n0) / n0)
    if compute_from is None:
        compute_from = lambda u: n0 - (n0 >> u)  # noqa: E731
    if keep_from is None:
        keep_from = lambda u: n0 - 2 * (n0 >> u)  # noqa: E731
    ring = {}
    outs = {}
    pairs = 0
    for t, zt in enumerate(z):
        cur = [complex(zt)]
        for u in range(1, m0 + 1):
            s, hp = n0 >> u, 1 << (u - 1)
            slot = t % s
            if prune and t < keep_from(u):
                break
            if prune and t < compute_from(u):
                ring[(u, slot)] = list(cur)
                break
            below = ring.get((u, slot), [complex(np.nan, np.nan)] * hp)
            ring[(u, slot)] = list(cur)
            nxt = [0j] * (2 * hp)
            for j in range(hp):
                tw = w[(j * s) % n0] * cur[j]
                nxt[j] = below[j] + tw
                nxt[j + hp] = below[j] - tw
                pairs += 1
            cur = nxt
        if len(cur) == n0 and t >= n0 - 1:
            outs[t] = np.array(cur)
    return outs, pairs


@pytest.mark.parametrize("n0", [2, 4, 8, 16, 32, 64])
@pytest.mark.parametrize("slab", [1, 3, 17])
def test_pruned_walk_gives_every_window(n0, slab):
    rng = np.random.default_rng(n0 * 100 + slab)
    z = rng.standard_normal(n0 - 1 + slab) + 1j * rng.standard_normal(n0 - 1 + slab)
    for prune in (False, True):
        outs, _ = walk(z, n0, prune)
        assert sorted(outs) == list(range(n0 - 1, n0 - 1 + slab))
        for t, v in outs.items():
            ref = np.fft.fft(z[t - n0 + 1:t + 1])
            assert np.all(np.isfinite(v)), (n0, slab, prune, t)
            np.testing.assert_allclose(v, ref, rtol=0, atol=1e-12 * n0)


@pytest.mark.parametrize("n0", [4, 8, 16, 32, 64])
def test_dropped_pairs_closed_form(n0):
    m0 = n0.bit_length() - 1
    steps = n0 - 1 + 5
    z = np.ones(steps, dtype=complex)
    _, full = walk(z, n0, prune=False)
    _, pruned = walk(z, n0, prune=True)
    dropped = sum((1 << (u - 1)) * (n0 - (n0 >> u)) for u in range(1, m0 + 1))
    assert full == steps * (n0 - 1)       # n0 - 1 node pairs per row (Eq. (8): 2(n0 - 1) ops)
    assert full - pruned == dropped
    if n0 == 16:
        assert dropped == 208 and (n0 - 1) ** 2 - dropped == 17


@pytest.mark.parametrize("mistake", ["compute one row late", "keep one row late",
                                     "keep only computed levels"])
def test_wrong_rules_fail(mistake):
    """Each plausible slip in the rule breaks an output (NaN or a wrong
    value), so the tests above would catch it. (Computing a level a row
    early is not among them: it only wastes work, on values no output
    reads.)"""
    n0, slab = 16, 4
    rng = np.random.default_rng(5)
    z = rng.standard_normal(n0 - 1 + slab) + 1j * rng.standard_normal(n0 - 1 + slab)
    kw = {}
    if mistake == "keep one row late":
        kw["keep_from"] = lambda u: n0 - 2 * (n0 >> u) + 1
    elif mistake == "compute one row late":
        kw["compute_from"] = lambda u: n0 - (n0 >> u) + 1
    else:
        kw["keep_from"] = lambda u: n0 - (n0 >> u)
    outs, _ = walk(z, n0, True, **kw)
    bad = False
    for t in range(n0 - 1, n0 - 1 + slab):
        v = outs.get(t)
        if v is None or not np.all(np.isfinite(v)) or \
                not np.allclose(v, np.fft.fft(z[t - n0 + 1:t + 1]), atol=1e-9):
            bad = True
    assert bad, mistake


def _radices(n):
    out = []
    while n % 2 == 0:
        out.append(2)
        n //= 2
    while n % 3 == 0:
        out.append(3)
        n //= 3
    assert n == 1
    return out


def walk_mixed(z, n0, prune=True):
    """The column stream of the mixed-radix tree (Sec. 5: levels of radix 2
    first, then 3): level t has L_t values per node and shift s_t = n0 / L_t,
    T_t[p][i + q L_{t-1}] = sum_j w_r^(q j) Omega0[i j s_t] T_{t-1}[p - (r-1-j) s_t][i];
    the ring of level t keeps level t-1 of the last (r_t - 1) s_t rows. With
    prune, level t is computed from T0 >= n0 - s_t and level t-1 kept from
    T0 >= n0 - s_{t-1}."""
    rad = _radices(n0)
    w = np.exp(-2j * np.pi * np.arange(n0) / n0)
    L = [1]
    for r in rad:
        L.append(L[-1] * r)
    s = [n0 // v for v in L]
    ring = {}
    outs = {}
    for t, zt in enumerate(z):
        cur = [complex(zt)]
        for u in range(1, len(rad) + 1):
            r, lp, su = rad[u - 1], L[u - 1], s[u]
            if prune and t < n0 - s[u - 1]:
                break
            length = (r - 1) * su
            if prune and t < n0 - su:
                ring[(u, t % length)] = list(cur)
                break
            nxt = [0j] * (lp * r)
            for i in range(lp):
                a = []
                for j in range(r - 1):
                    older = ring.get((u, (t - (r - 1 - j) * su) % length),
                                     [complex(np.nan, np.nan)] * lp)
                    a.append(w[(i * j * su) % n0] * older[i])
                a.append(w[(i * (r - 1) * su) % n0] * cur[i])
                for q in range(r):
                    nxt[i + q * lp] = sum(np.exp(-2j * np.pi * q * j / r) * a[j] for j in range(r))
            ring[(u, t % length)] = list(cur)
            cur = nxt
        if len(cur) == n0 and t >= n0 - 1:
            outs[t] = np.array(cur)
    return outs


@pytest.mark.parametrize("n0", [3, 6, 9, 12, 24])
@pytest.mark.parametrize("slab", [1, 5])
def test_pruned_mixed_walk_gives_every_window(n0, slab):
    rng = np.random.default_rng(n0 * 10 + slab)
    z = rng.standard_normal(n0 - 1 + slab) + 1j * rng.standard_normal(n0 - 1 + slab)
    for prune in (False, True):
        outs = walk_mixed(z, n0, prune)
        assert sorted(outs) == list(range(n0 - 1, n0 - 1 + slab))
        for t, v in outs.items():
            assert np.all(np.isfinite(v)), (n0, slab, prune, t)
            np.testing.assert_allclose(v, np.fft.fft(z[t - n0 + 1:t + 1]), rtol=0,
                                       atol=1e-12 * n0)
