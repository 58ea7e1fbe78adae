"""Sector footprint of the fused kernel's stencil gathers on the 256^3
single-subdomain workload (run by hand: python tests/footprint.py).

For groups of G consecutive records in pool order (G = 64: one wave's records
at a time; 256: one item of a 256x4 tile; 1024: a whole tile), counts the
distinct 64-byte sectors of each field component that the group's stage-1 and
stage-2 stencils touch, and prints the sum over groups x 3 components x 64 B:
the field bytes a cache that kept exactly one group's data would fetch.  The
stage-2 position is X + dt U(X) with U from the oracle (the step starts from
V = U(X)).  Compare with the measured FETCH_SIZE of the kernel.

The same for 128-byte lines (what the L2 fetches from memory per miss).

Then, per 64-lane gather instruction (one wave's 16-byte x-pair load of one
stencil row of one component), the mean number of distinct 64-byte lines it
touches, for the pool order and two other cell orders: the L1 tag lookups
per gather that the kernel's TCP_TOTAL_CACHE_ACCESSES counts.
"""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import oracle  # noqa: E402
from paper_2604_11008_amd import gen  # noqa: E402


def sectors(X, n, L, halo, line=64):
    """Memory lines of `line` bytes that each stencil row's x pair touches."""
    S = n + 2 * halo
    s = X * (n / L) - 0.5
    i = np.floor(s).astype(np.int64) + halo
    out = []
    for dy in (0, 1):
        for dz in (0, 1):
            row = (i[1] + dy) + S * (i[2] + dz)
            b0 = (row * S + i[0]) * 8
            out.append(b0 // line)
            out.append((b0 + 15) // line)
    return np.stack(out)


def main():
    wl = gen.make_workload("C2")
    n, L = wl.n, wl.L
    x = wl.pool.x[:, :int(wl.pool.count[0])]
    of = oracle.Field(wl.stored_field(np.float64), n, wl.halo, L)
    U, _ = oracle.interp(of, x)
    xs = x + wl.dt * U
    s1, s2 = sectors(x, n, L, wl.halo), sectors(xs, n, L, wl.halo)
    np_ = x.shape[1]
    for G in (64, 128, 256, 512, 1024, 2048, 4096):
        tot = 0
        for g0 in range(0, np_, G):
            tot += np.unique(np.concatenate([s1[:, g0:g0 + G].ravel(),
                                             s2[:, g0:g0 + G].ravel()])).size
        print(f"groups of {G:5d}: {tot * 3 * 64 / 1e9:.3f} GB "
              f"({tot * 3 * 64 / np_:.1f} B/particle)")
    allu = np.unique(np.concatenate([s1.ravel(), s2.ravel()])).size
    print(f"whole step: {allu * 3 * 64 / 1e9:.3f} GB ({allu * 3 * 64 / np_:.1f} B/particle)")
    # the L2 fetches 128-byte lines from memory
    t1, t2 = sectors(x, n, L, wl.halo, 128), sectors(xs, n, L, wl.halo, 128)
    for G in (256, 1024):
        tot = 0
        for g0 in range(0, np_, G):
            tot += np.unique(np.concatenate([t1[:, g0:g0 + G].ravel(),
                                             t2[:, g0:g0 + G].ravel()])).size
        print(f"groups of {G:5d}, 128-byte lines: {tot * 3 * 128 / 1e9:.3f} GB")

    cell = [np.clip(np.floor(x[a] * (n / L)).astype(np.int64), 0, n - 1) for a in range(3)]
    orders = {
        "pool order (Z-order over x pairs)": np.arange(np_),
        "Z-order of cells": np.argsort(gen.morton3(*cell), kind="stable"),
        "Z-order over 4-cell x runs": np.argsort(gen.morton3(cell[0] >> 2, cell[1], cell[2])
                                                 * 4 + (cell[0] & 3), kind="stable"),
    }
    nw = np_ // 64
    for name, perm in orders.items():
        tot = 0
        for s in (s1[:, perm], s2[:, perm]):
            for r in range(4):  # stencil rows (dy, dz); each spans 1 or 2 sectors
                ll = np.concatenate([s[2 * r, :nw * 64].reshape(nw, 64),
                                     s[2 * r + 1, :nw * 64].reshape(nw, 64)], axis=1)
                ll.sort(axis=1)
                tot += (1 + (np.diff(ll, axis=1) != 0).sum(axis=1)).sum()
        print(f"lines per gather instruction, {name}: {tot / (nw * 8):.1f}")


if __name__ == "__main__":
    main()
