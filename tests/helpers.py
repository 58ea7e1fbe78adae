"""Shared test helpers: small pools built by hand, record extraction and
comparison.  No step arithmetic lives here."""
from __future__ import annotations

import numpy as np

from paper_2604_11008_amd import gen

STAY = 13


def pool_from(pos, owners, nsub, vel=None, tau=None, ids=None, extra=8,
              vdtype=np.float64):
    """Pool whose segment s holds, in the given order, the particles with
    owners == s.  Capacities leave `extra` free slots."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[1]
    owners = np.asarray(owners, dtype=np.int64)
    vel = np.zeros((3, n)) if vel is None else np.asarray(vel, dtype=np.float64)
    tau = np.full(n, 0.5) if tau is None else np.asarray(tau, dtype=np.float64)
    ids = np.arange(n, dtype=np.uint64) if ids is None else np.asarray(ids, dtype=np.uint64)
    counts = np.bincount(owners, minlength=nsub).astype(np.int64)
    cap = counts + extra
    base = np.zeros(nsub, dtype=np.int64)
    base[1:] = np.cumsum(cap)[:-1]
    pool = gen.empty_pool(base, cap, vdtype)
    for s in range(nsub):
        sel = np.nonzero(owners == s)[0]
        b = int(base[s])
        c = len(sel)
        pool.x[:, b:b + c] = pos[:, sel]
        pool.v[:, b:b + c] = vel[:, sel].astype(vdtype)
        pool.tau[b:b + c] = tau[sel].astype(vdtype)
        pool.id[b:b + c] = ids[sel]
        pool.count[s] = c
    return pool


def like(pool, cap_scale=1.0, extra=0):
    """Empty pool with the same segment structure (for outputs)."""
    cap = (pool.cap * cap_scale).astype(np.int64) + extra
    base = np.zeros_like(cap)
    base[1:] = np.cumsum(cap)[:-1]
    return gen.empty_pool(base, cap, pool.v.dtype)


def send_for(nsub, cap_each=64, vdtype=np.float64):
    cap = np.full(nsub * 27, cap_each, dtype=np.int64)
    cap[STAY::27] = 0
    base = np.zeros_like(cap)
    base[1:] = np.cumsum(cap)[:-1]
    return gen.empty_pool(base, cap, vdtype)


def records(pool, q):
    """(x (3,c), v (3,c), tau (c), id (c)) of segment q, clipped to capacity."""
    b = int(pool.base[q])
    c = int(min(pool.count[q], pool.cap[q]))
    return (pool.x[:, b:b + c], pool.v[:, b:b + c], pool.tau[b:b + c],
            pool.id[b:b + c])


def ids_of(pool, q):
    return records(pool, q)[3]
