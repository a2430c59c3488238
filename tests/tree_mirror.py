"""Instrumented CPU mirror of the 2D tree (Eq. (5) and Eq. (6), Sec. 4.2).

Test infrastructure only: it is neither the oracle (which evaluates Eq. (2)
window by window) nor the product (the HIP kernels). It runs the tree levels
as the paper states them, levels outermost over all trees of a small grid,
in complex128, and counts every node operation (one complex multiply and one
complex add, the unit of Eq. (8)) at the tree position it belongs to. The
tests use it to pin the shape of the tree: which inputs a node combines
(Fig. 1), how many operations one complete tree takes (Eq. (8)), and that the
last level is the DFT of the window ending at that tree (checked against
numpy.fft.fft2, a library routine, so the mirror is not pinned by itself).

Notation: a node of level l at tree position p holds the values i < 2^l of
the 2^l-point DFT of the samples p - (2^l - 1) s_l, ..., p - s_l, p (stride
s_l = n / 2^l); it exists only for p >= n - s_l (Sec. 4.7: the trees near the
top and left edges are incomplete). Twiddles Omega_n[m] = exp(-2 pi i m / n)
(the forward sign), computed here directly with numpy.
"""
from __future__ import annotations

import numpy as np


def _omega(n: int) -> np.ndarray:
    return np.exp(-2j * np.pi * np.arange(max(n, 1)) / max(n, 1))


class TreeMirror:
    """Levels of the 2D tree over an N0 x N1 array x with n0 x n1 windows.

    After run(): `levels[l]` is an array [N0, N1, 2^l0, 2^l1] (NaN where the
    node does not exist), for l = 0 .. m1 + m0 (row levels first, Eq. (5),
    then column levels, Eq. (6)); `ops[p0, p1]` counts the node operations
    performed at tree position (p0, p1); `node_ops` counts them per level."""

    def __init__(self, x: np.ndarray, n0: int, n1: int):
        self.x = np.asarray(x, dtype=np.complex128)
        self.N0, self.N1 = self.x.shape
        self.n0, self.n1 = n0, n1
        self.m0, self.m1 = n0.bit_length() - 1, n1.bit_length() - 1
        assert 1 << self.m0 == n0 and 1 << self.m1 == n1, "radix-2 windows only"
        self.ops = np.zeros((self.N0, self.N1), dtype=np.int64)
        self.node_ops: list[int] = []
        self.levels: list[np.ndarray] = []

    # The three ingredients of a node, separate so that a test can plant a
    # mistake in one of them.
    def shift(self, n: int, level: int) -> int:
        """s_l = n / 2^l: the distance between the two trees a node combines."""
        return n >> level

    def twiddles(self, n: int) -> np.ndarray:
        return _omega(n)

    def combine(self, added, multiplied, w):
        """One node operation: added + w * multiplied."""
        return added + w * multiplied

    def run(self) -> "TreeMirror":
        N0, N1, n0, n1 = self.N0, self.N1, self.n0, self.n1
        w0, w1 = self.twiddles(n0), self.twiddles(n1)
        # level 0: the data itself, one node value per position
        T = self.x[:, :, None, None].copy()
        self.levels.append(T)
        p0 = np.arange(N0)[:, None]
        p1 = np.arange(N1)[None, :]
        # row levels t = 1..m1 (Eq. (5)): T_t[p][i] = T_{t-1}[p - s][i mod h]
        #                                 + Omega1[i s] T_{t-1}[p][i mod h]
        for t in range(1, self.m1 + 1):
            s, h = self.shift(n1, t), 1 << (t - 1)
            exists = np.broadcast_to(p1 >= n1 - s, (N0, N1))
            new = np.full((N0, N1, 1, 2 * h), np.nan, dtype=np.complex128)
            count = 0
            for i in range(2 * h):
                a = np.full((N0, N1), np.nan, dtype=np.complex128)
                if s < N1:
                    a[:, s:] = T[:, :N1 - s, 0, i % h]
                val = self.combine(a, T[:, :, 0, i % h], w1[(i * s) % n1])
                new[:, :, 0, i] = np.where(exists, val, np.nan)
                self.ops += exists
                count += int(exists.sum())
            self.node_ops.append(count)
            T = new
            self.levels.append(T)
        # column levels u = 1..m0 (Eq. (6)), node index (i0 < 2^u, i1 < n1):
        # T_v[p0][i0][i1] = T_{v-1}[p0 - s][i0 mod h][i1]
        #                   + Omega0[i0 s] T_{v-1}[p0][i0 mod h][i1]
        row_done = np.broadcast_to(p1 >= n1 - 1, (N0, N1))
        for u in range(1, self.m0 + 1):
            s, h = self.shift(n0, u), 1 << (u - 1)
            exists = (p0 >= n0 - s) & row_done
            new = np.full((N0, N1, 2 * h, n1), np.nan, dtype=np.complex128)
            count = 0
            for i0 in range(2 * h):
                for i1 in range(n1):
                    a = np.full((N0, N1), np.nan, dtype=np.complex128)
                    if s < N0:
                        a[s:, :] = T[:N0 - s, :, i0 % h, i1]
                    val = self.combine(a, T[:, :, i0 % h, i1], w0[(i0 * s) % n0])
                    new[:, :, i0, i1] = np.where(exists, val, np.nan)
                    self.ops += exists
                    count += int(exists.sum())
            self.node_ops.append(count)
            T = new
            self.levels.append(T)
        self.top = T
        return self

    def window(self, q0: int, q1: int) -> np.ndarray:
        """Last level at the tree of the window with top-left corner (q0, q1),
        i.e. position (q0 + n0 - 1, q1 + n1 - 1): its n0 x n1 2D DFT."""
        return self.top[q0 + self.n0 - 1, q1 + self.n1 - 1]

    def complete_trees(self):
        """Positions whose whole tree exists (one per window, Sec. 4.1)."""
        return [(a, b) for a in range(self.n0 - 1, self.N0) for b in range(self.n1 - 1, self.N1)]
