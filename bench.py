"""Benchmark of the fused particle step on one MI355X.

Default workload (the 1024^3 mixed-precision batched case): a 1024^3
periodic velocity field, 2^28 blob-clustered particles (70% around 4096
Gaussian blobs of two cells, 30% uniform), tau log-uniform in [0.01, 1],
8x8x8 subdomains, dt giving at most half a cell per step.  It runs in
float64 (field, velocities, tau: `value`, the paper's precision) and in the
mixed form (float32 field, velocities and tau; float64 positions and
ownership), and times the plain float64 three-call path beside them; then
both forms again from the same start with the field stored node-interleaved
(the three components of a node next to each other), whose final states
must be bitwise those of the split runs.

A step is the whole hot path over every particle: interpolation at two RK2
stages, the Heun drag update, classification, scan, pack/compact and the
on-device append of the migrants.  Inputs are resident in HBM before the
timed region.  The CPU-baseline leg runs the oracle on the particles with
the 2^20 lowest ids for 20 whole steps (same field and decomposition) and
compares them per id with the device's steps 1 and 20 from the same start
state: that is the error of each form against the FP64 oracle.  Prints one
JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2604_11008_amd import gen  # noqa: E402  (seeded inputs; no torch)

METRIC = "particles/sec per full step (interp+drag+scan-migrate); HBM GB/s; FP32 vs FP64"

WORKLOADS = {
    "C2": "256^3 FP64 field with a one-cell halo, 4,194,304 uniform particles, "
          "1 subdomain (26 periodic self-neighbour buffers), tau log-uniform [0.01,1], "
          "g=(0,0,-1), dt=0.5 cell/(max|u|+tau_max|g|)",
    "C1": "64^3 periodic FP64 field, 65,536 uniform particles, 2x2x2 subdomains, dt=0.01",
    "C2S": "256^3 periodic FP64 field, 4,194,304 uniform particles, 8x8x8 subdomains, "
           "dt=0.5 cell per unit speed (a few percent migrate per step)",
    "C3": "512^3 periodic FP64 field, 2^26 blob-clustered particles, 4x4x4 subdomains",
    "C4": "512^3 periodic FP64 field, lognormal per-subdomain counts (median 1e5), "
          "8x8x8 subdomains",
    "C5": "1024^3 periodic field, 2^28 blob-clustered particles (70% in 4096 Gaussian "
          "blobs of sigma 2 cells, 30% uniform), tau log-uniform [0.01,1], 8x8x8 "
          "subdomains, dt=0.5 cell/max|u|",
    "CP": "750^3 FP64 field with a one-cell halo, 52,734,375 uniform particles (750^3/8, "
          "the paper's per-rank share), 1 subdomain, tau log-uniform [0.01,1], g=(0,0,-1)",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="C5", choices=sorted(WORKLOADS))
    ap.add_argument("--order", default="canonical",
                    choices=["canonical", "morton", "rowmajor", "shuffled"],
                    help="particle order within each segment at the start: cell-sorted "
                         "(canonical: Z-order over x pairs; morton; rowmajor) or shuffled")
    ap.add_argument("--precision", default="auto", choices=["auto", "f64", "mixed", "both"],
                    help="f64; mixed (float32 field, velocities and tau; float64 positions); "
                         "both (f64 as the value, then mixed); auto: both for the 1024^3 "
                         "workload, else the workload's own")
    ap.add_argument("--drag", default="stokes", choices=["stokes", "nonlinear"],
                    help="drag law: Stokes (f = 1) or the paper's nonlinear correction "
                         "(nu = 1.5e-5, rho_p/rho = 843 in the field's units)")
    ap.add_argument("--stagger", action="store_true",
                    help="read the field as MAC-staggered (component c on the faces "
                         "normal to axis c)")
    ap.add_argument("--layout", default="auto",
                    choices=["auto", "split", "interleaved", "both"],
                    help="field storage: one array per component (split), the three "
                         "components of a node interleaved, or both (split as the value, "
                         "then interleaved from the same start); auto: both for the "
                         "1024^3 workload, else split")
    ap.add_argument("--staged", action="store_true",
                    help="migrate after each RK2 stage (the paper's scheme) instead of once "
                         "per step")
    ap.add_argument("--migration-only", action="store_true",
                    help="also time the exchange alone (classify/scan/pack + "
                         "compact/append, no advance) on the timed state")
    ap.add_argument("--graph", action="store_true", help="time graph replays (the eager "
                    "steps are then not timed per kernel)")
    ap.add_argument("--no-graph-replay", action="store_true",
                    help="skip the graph replay of the timed steps")
    ap.add_argument("--tune", default=None, help="wg,items[,blocks_per_cu[,xcd_block]] or 'auto'")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the CPU-baseline leg (oracle timing and per-id errors)")
    ap.add_argument("--resort", type=int, default=0,
                    help="re-sort the pool by cell (pm_sort) every K steps inside the "
                         "timed region (0: never, the paper's method)")
    ap.add_argument("--sample", type=int, default=1 << 20,
                    help="the CPU-baseline leg follows the particles with ids below this")
    ap.add_argument("--sample-steps", type=int, default=20)
    ap.add_argument("--copy-probe", action="store_true",
                    help="accepted for the profiling commands: the plain torch copy of "
                         "1 GiB (the counters' scaling reference and the copy-rate "
                         "figure) always runs")
    ap.add_argument("--traffic", default=None,
                    help="traffic record of the fused kernel (default: "
                         "profiles/k_step_<config>_<f64|mixed>_traffic.json)")
    ap.add_argument("--plain", default="auto", choices=["auto", "on", "off"],
                    help="time the plain three-call path too (auto: in the f64 run of "
                         "'both')")
    ap.add_argument("--side-stream", action="store_true",
                    help="run on a new (default-priority) stream instead of the null stream")
    ap.add_argument("--plain-per-sub", action="store_true",
                    help="time the plain path launched once per subdomain")
    ap.add_argument("--cpu-delegated", action="store_true",
                    help="time the CPU-delegated exchange of the paper's comparison: the "
                         "17-array records device->host, the oracle's sequential pack and "
                         "unpack on one core, host->device")
    return ap.parse_args()


# ----------------------------------------------------------------------------
# samples of the pool by id
# ----------------------------------------------------------------------------

def sample(p, nmax):
    """Records of device pool p with id < nmax, in pool order, on the host:
    (x float64, v and tau as stored, id, number per segment)."""
    import torch
    size = p.x.shape[1]
    valid = torch.zeros(size, dtype=torch.bool, device=p.x.device)
    base, count = p.base.cpu().numpy(), p.count.cpu().numpy()
    for b, c in zip(base, count):
        if c > 0:
            valid[int(b):int(b) + int(c)] = True
    sel = torch.nonzero(valid & (p.id < nmax)).squeeze(1)
    seg = torch.bucketize(sel, torch.as_tensor(base, device=sel.device), right=True) - 1
    counts = torch.bincount(seg, minlength=len(base)).cpu().numpy().astype(np.int64)
    return (p.x[:, sel].cpu().numpy(), p.v[:, sel].cpu().numpy(), p.tau[sel].cpu().numpy(),
            p.id[sel].cpu().numpy().astype(np.uint64), counts)


def host_pool(smp, vdtype=np.float64):
    x, v, tau, ids, counts = smp
    base, cap = gen.layout(counts, slack=0.5, extra=256)
    pool = gen.empty_pool(base, cap, vdtype)
    start = 0
    for q, n in enumerate(counts):
        b = int(base[q])
        pool.x[:, b:b + n] = x[:, start:start + n]
        pool.v[:, b:b + n] = v[:, start:start + n]
        pool.tau[b:b + n] = tau[start:start + n]
        pool.id[b:b + n] = ids[start:start + n]
        start += n
    pool.count[:] = counts
    return pool


def valid_records(pool):
    sl = [slice(int(b), int(b) + int(min(c, k)))
          for b, c, k in zip(pool.base, pool.count, pool.cap)]
    cat = lambda a: np.concatenate([a[..., s] for s in sl], axis=-1)  # noqa: E731
    return cat(pool.x), cat(pool.v).astype(np.float64), cat(pool.id)


def per_id_errors(got, ref, L, cell, umax):
    """Largest |dV| / |u|max and |dX| in cells (periodic images folded), per id."""
    gx, gv, gid = valid_records(got)
    rx, rv, rid = valid_records(ref)
    gi, ri = np.argsort(gid, kind="stable"), np.argsort(rid, kind="stable")
    if not np.array_equal(gid[gi], rid[ri]):
        raise SystemExit("the device and the oracle hold different ids")
    dx = np.abs(gx[:, gi] - rx[:, ri])
    dx = np.minimum(dx, L - dx)
    return (float(np.abs(gv[:, gi] - rv[:, ri]).max(initial=0.0)) / umax,
            float(dx.max(initial=0.0)) * cell)


# ----------------------------------------------------------------------------
# the CPU-baseline leg: the oracle
# ----------------------------------------------------------------------------

def cpu_leg(wl, fh, runs, params, drag, stagger, staged, steps, record_at):
    """The oracle (sequential FP64, one thread) on each run's start sample,
    whole steps with the workload's field and decomposition; returns, per
    run, the per-id errors of the device's samples after the steps in
    record_at, and the timing of the first run (comparisons excluded)."""
    import oracle
    of = oracle.Field(fh, wl.n, wl.halo, wl.L, stagger=stagger)
    od = oracle.Decomp(wl.p, wl.bounds)
    umax = max(float(np.abs(u).max()) for u in fh)
    cell = wl.n / wl.L
    out = {}
    timing = None
    for name, (start, got) in runs.items():
        host = host_pool(start)
        m = int(host.count.sum())
        osb, osc = gen.send_layout(host.count, face=0.2, edge=0.05, corner=0.03)
        errs = {}
        el = 0.0
        for k in range(1, steps + 1):
            t0 = time.perf_counter()
            nxt = gen.empty_pool(host.base, host.cap)
            if staged:
                mid = gen.empty_stage_pool(host.base, host.cap)
                msend = gen.empty_stage_pool(osb, osc)
                fl = oracle.step_staged(of, od, params.dt, params.g, host, mid, msend, nxt,
                                        gen.empty_pool(osb, osc), drag=drag, nu=params.nu,
                                        density_ratio=params.density_ratio)
            else:
                _, fl = oracle.step(of, od, params.dt, params.g, host, nxt,
                                    gen.empty_pool(osb, osc), drag=drag, nu=params.nu,
                                    density_ratio=params.density_ratio)
            el += time.perf_counter() - t0
            if fl:
                raise SystemExit(f"oracle flags {fl} in the CPU-baseline leg")
            host = nxt
            if k in record_at and k in got:
                ev, ex = per_id_errors(host_pool(got[k]), host, wl.L, cell, umax)
                errs[f"after_{k}"] = {"v_err_rel_umax": ev, "x_err_cells": ex}
        out[name] = errs
        if timing is None:
            timing = (m, steps, el)
    return out, timing


def host_cpu():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f
                          if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"cpu": model, "threads": os.cpu_count()}


def copy_rate(dev, nbytes=1 << 30, reps=10):
    """Milliseconds and GB/s (read + written) of a plain torch device copy of
    nbytes; also the reference the counter runs are scaled by."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return ms, 2 * nbytes / (ms * 1e-3) / 1e9


def single_core_triad_gbps(nbytes=1 << 28, reps=5):
    """a = b + s*c on one core (numpy, float64): 3 arrays x nbytes/8 values."""
    n = nbytes // 8
    b = np.full(n, 1.5)
    c = np.full(n, 0.25)
    a = np.empty_like(b)
    best = 1e30
    for _ in range(reps):
        t0 = time.perf_counter()
        np.multiply(c, 3.0, out=a)
        np.add(a, b, out=a)
        best = min(best, time.perf_counter() - t0)
    # the two passes move 5 arrays (c, a | a, b, a); the triad counts 3
    return 3 * nbytes / (best * 5 / 3) / 1e9


def link_gbps(torch, dev, nbytes=1 << 28):
    """Pinned host <-> device copy rates (GB/s)."""
    h = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
    d = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    for _ in range(2):
        d.copy_(h, non_blocking=True)
        h.copy_(d, non_blocking=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(4):
        d.copy_(h, non_blocking=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(4):
        h.copy_(d, non_blocking=True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return 4 * nbytes / (t1 - t0) / 1e9, 4 * nbytes / (t2 - t1) / 1e9


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def delegated_transfers(ctx, field, p, params, dev):
    """Device side of the CPU-delegated exchange (the paper's comparison in
    Sect. 3.2.2): the state advanced by one step on a copy, then its
    17-array record (x, v, x*, v*, a, tau, id: 136 bytes per particle in
    float64) copied device -> pinned host and back, timed.  Returns the
    advanced records on the host for the oracle's pack and unpack."""
    import torch
    from paper_2604_11008_amd import pm
    work = pm.DevicePool(p.x.clone(), p.v.clone(), p.tau.clone(), p.id.clone(), p.base,
                         p.cap, p.count.clone())
    ctx.interp_advance(field, work, params)
    n = work.x.shape[1]
    dev17 = torch.empty((17, n), dtype=torch.float64, device=dev)
    dev17[0:3] = work.x
    dev17[3:6] = work.v.double()
    dev17[6:9] = work.x
    dev17[9:15] = work.v.double().repeat(2, 1)
    dev17[15] = work.tau.double()
    dev17[16] = work.id.view(torch.float64)
    host17 = torch.empty((17, n), dtype=torch.float64, pin_memory=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    host17.copy_(dev17)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dev17.copy_(host17)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    if ctx.get_status():
        raise SystemExit("flags in the delegated-exchange advance")
    host = work.to_host()
    del work, dev17, host17
    return {"records": int(host.count.sum()), "bytes": 17 * 8 * n,
            "d2h_ms": (t1 - t0) * 1e3, "h2d_ms": (t2 - t1) * 1e3, "host_state": host}


def delegated_pack_unpack(wl, host):
    """Host side of the CPU-delegated exchange: the oracle's sequential pack
    (classification and per-direction counters) and unpack (compaction and
    receive) of the advanced records, one core, timed."""
    import oracle
    od = oracle.Decomp(wl.p, wl.bounds)
    pool = gen.Pool(x=host.x, v=host.v.astype(np.float64), tau=host.tau.astype(np.float64),
                    id=host.id, base=host.base, cap=host.cap, count=host.count)
    sb, sc = gen.send_layout(pool.count, face=0.05, edge=0.01, corner=0.005)
    out = gen.empty_pool(pool.base, pool.cap)
    send = gen.empty_pool(sb, sc)
    t0 = time.perf_counter()
    stay, f1 = oracle.partition(od, pool, out, send)
    t1 = time.perf_counter()
    f2 = oracle.append(od, send, stay, out)
    t2 = time.perf_counter()
    if f1 or f2:
        raise SystemExit(f"oracle flags {f1 | f2} in the delegated exchange")
    return {"pack_ms": (t1 - t0) * 1e3, "unpack_ms": (t2 - t1) * 1e3,
            "migrants": int(send.count.sum())}


# ----------------------------------------------------------------------------
# one run: a precision, its pools, its timed steps
# ----------------------------------------------------------------------------

def state_digest(p):
    """Order- and bit-sensitive 64-bit digest of a device pool's valid records
    (x, v, tau, id), computed on the device."""
    import torch
    size = p.x.shape[1]
    cnt = torch.minimum(p.count, p.cap)
    edge = torch.zeros(size + 1, dtype=torch.int32, device=p.x.device)
    edge.index_add_(0, p.base, torch.ones_like(p.base, dtype=torch.int32))
    edge.index_add_(0, p.base + cnt, -torch.ones_like(p.base, dtype=torch.int32))
    valid = edge.cumsum(0)[:size] > 0
    w = 2 * torch.arange(size, device=p.x.device)[valid] + 1
    d = 0
    for t in (p.x, p.v, p.tau.view(1, -1), p.id.view(1, -1)):
        bits = t.view(torch.int64) if t.element_size() == 8 else \
            t.view(torch.int32).to(torch.int64)
        for r in range(bits.shape[0]):
            d = (d * 1000003 + int((bits[r][valid] * w).sum().item())) & ((1 << 64) - 1)
    return f"{d:016x}"


def run(args, wl, dev, field, dc, start, pool, sb, sc, mixed, plain, label):
    """Device samples for the CPU-baseline leg (untimed steps from the start
    state), warm-up, the timed steps with per-launch kernel times, graph
    replays and the plain path.  start: device tensors (x, v, tau, id,
    count) of the start state."""
    import torch
    from paper_2604_11008_amd import accounting, pm
    vdt = torch.float32 if mixed else torch.float64
    mode = "mixed" if mixed else "f64"
    size = start[0].shape[1]
    base = torch.as_tensor(pool.base).to(dev)
    cap = torch.as_tensor(pool.cap).to(dev)
    pa = pm.DevicePool(*[t.clone() for t in start[:4]], base, cap, start[4].clone())
    pb = pm.DevicePool.empty(pool.base, pool.cap, vdtype=vdt, device=dev, size=size)
    send = pm.DevicePool.empty(sb, sc, vdtype=vdt, device=dev)
    ctx = pm.Context(size, send.size, dc.nsub, device=dev)
    params = pm.Params(wl.dt, wl.g, drag=args.drag)
    npart = int(pool.count.sum())
    mid = msend = None
    if args.staged:
        if args.tune == "auto" or args.stagger:
            raise SystemExit("--staged runs without the autotuner, on collocated fields")
        mid = pm.DeviceStagePool.empty(pool.base, pool.cap, vdtype=vdt, device=dev, size=size)
        msend = pm.DeviceStagePool.empty(sb, sc, vdtype=vdt, device=dev, size=send.size)

    def do_step(src, dst):
        if args.staged:
            ctx.step_staged(field, dc, src, mid, msend, dst, send, params)
        else:
            ctx.step(field, dc, src, dst, send, params)

    def restore(p, state):
        for t, v in zip((p.x, p.v, p.tau, p.id, p.count), state):
            t.copy_(v)

    if args.tune == "auto":
        ctx.autotune(field, dc, pa, pb, send, params, cache_path=args.tune_cache)
        restore(pa, start)
    elif args.tune:
        ctx.set_tuning(*[int(v) for v in args.tune.split(",")])
    res = {"mode": mode}

    # untimed: the device's samples for the CPU-baseline leg's comparison
    if not args.no_cpu:
        record_at = (1, args.sample_steps)
        ta = time.perf_counter()
        smp0 = sample(pa, args.sample)
        got = {}
        for k in range(1, args.sample_steps + 1):
            do_step(pa, pb)
            pa, pb = pb, pa
            if k in record_at:
                got[k] = sample(pa, args.sample)
        f = ctx.get_status()
        if f:
            raise SystemExit(f"{label}: flags in the sample steps: {pm.flag_names(f)}")
        res["samples"] = (smp0, got)
        restore(pa, start)
        log(f"{label}: {args.sample_steps} sample steps in {time.perf_counter() - ta:.1f} s")

    if args.graph:
        ctx.set_graph(True)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        do_step(pa, pb)
        pa, pb = pb, pa
    f = ctx.get_status()
    if f:
        raise SystemExit(f"{label}: warm-up flags: {pm.flag_names(f)}")

    # algorithmic bytes of a step of this state (untimed): touched field nodes
    # and migrants
    touched = ctx.touched_nodes(field, pa, params)
    do_step(pa, pb)
    migrants = int(send.count.sum().item())
    pa, pb = pb, pa
    if args.staged:
        migrants1 = int(msend.count.sum().item())
        alg = accounting.staged_algorithmic_bytes(npart, migrants1, migrants, touched, mode)
        alg["fused_kernel"] = alg["stage_kernels"]
        res["stage1_migrants_per_step"] = migrants1
    else:
        alg = accounting.step_algorithmic_bytes(npart, migrants, touched, mode)
    # the state the timed steps start from, so the graph replays start from it
    snap = [t.clone() for t in (pa.x, pa.v, pa.tau, pa.id, pa.count)]

    if not args.graph:
        ctx.set_timing(args.steps * (2 if args.staged else 1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        do_step(pa, pb)
        pa, pb = pb, pa
        if args.resort and (k + 1) % args.resort == 0:
            ctx.sort(field, pa, pb)
            pa, pb = pb, pa
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    f = ctx.get_status()
    if f:
        raise SystemExit(f"{label}: flags after the timed steps: {pm.flag_names(f)}")
    res["state_digest"] = state_digest(pa)
    ms_step = (t1 - t0) * 1e3 / args.steps
    k_total, k_each = (ctx.kernel_times() if not args.graph else (None, []))
    if args.staged and k_each:  # the two stage kernels of a step, summed
        k_each = [a + b for a, b in zip(k_each[0::2], k_each[1::2])]
    k_ms = (k_total / len(k_each)) if k_each else None
    log(f"{label}: {args.steps} steps {ms_step:.4f} ms/step; fused kernel "
        f"{k_ms if k_ms is None else round(k_ms, 4)} ms; tuning {ctx.get_tuning()}")
    res.update(ms_per_step=ms_step, particles_per_s=npart / (ms_step * 1e-3),
               touched=touched, migrants=migrants, alg=alg, tuning=list(ctx.get_tuning()))

    roof = None
    if k_ms:
        achieved = alg["fused_kernel"] / (k_ms * 1e-3) / 1e9
        from paper_2604_11008_amd import profsum
        wg, items = ctx.get_tuning()[:2]
        tf = lambda b: "true" if b else "false"  # noqa: E731
        # the last template argument: field arrangement (0 split, 1 MAC, 2 interleaved)
        arr = 1 if args.stagger else (2 if field.interleaved else 0)
        variant = (f"k_step<{wg}, {items}, {'float' if mixed else 'double'}, "
                   f"{tf(wl.halo)}, {tf(args.drag == 'nonlinear')}, {arr}>")
        lay = "_interleaved" if field.interleaved else ""
        tpath = args.traffic or os.path.join(ROOT, "profiles",
                                             f"k_step_{args.config}_{mode}{lay}_traffic.json")
        traffic = None
        # the record was taken on the canonical start order of this workload
        if os.path.exists(tpath) and json.load(open(tpath)).get("kernel") == variant \
                and not args.staged and args.order == "canonical" and not args.resort:
            traffic = profsum.load_traffic(tpath)
        roof = {"bound": "hbm", "achieved": round(achieved, 1),
                "peak": accounting.HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / accounting.HBM_PEAK_GBPS, 4), "traffic": traffic,
                "kernel": ("k_stage<1> + k_stage<2> (the two per-stage fused kernels)"
                           if args.staged else
                           f"{variant} (fused interpolate/advance/classify/scan/scatter)"),
                "kernel_ms": round(k_ms, 5),
                "kernel_ms_first_last": [round(k_each[0], 5), round(k_each[-1], 5)],
                "kernel_ms_min_median_max": [round(float(np.min(k_each)), 5),
                                             round(float(np.median(k_each)), 5),
                                             round(float(np.max(k_each)), 5)],
                "algorithmic_bytes_per_launch": alg["fused_kernel"]}
    res["roofline"] = roof

    if args.migration_only:
        # the exchange alone, one stage's worth (what the paper times as
        # packing + unpacking), on the timed state advanced by one step in
        # place on a copy, so that its leavers are still in their old owners
        ctx.set_timing(0)
        sendm = pm.DevicePool.empty(sb, sc, vdtype=vdt, device=dev)
        outm = pm.DevicePool.empty(pool.base, pool.cap, vdtype=vdt, device=dev, size=size)
        work = pm.DevicePool(pa.x.clone(), pa.v.clone(), pa.tau.clone(), pa.id.clone(),
                             pa.base, pa.cap, pa.count.clone())
        ctx.interp_advance(field, work, params)
        for _ in range(2):
            ctx.classify_scan_pack(dc, work, sendm)
            ctx.compact_append(dc, work, sendm, outm)
        torch.cuda.synchronize()
        reps = 10
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        for _ in range(reps):
            ctx.classify_scan_pack(dc, work, sendm)
        e[1].record()
        for _ in range(reps):
            ctx.compact_append(dc, work, sendm, outm)
        e[2].record()
        torch.cuda.synchronize()
        f = ctx.get_status()
        if f:
            raise SystemExit(f"flags after the exchange timing: {pm.flag_names(f)}")
        res["migration_only_ms"] = {
            "classify_scan_pack": round(e[0].elapsed_time(e[1]) / reps, 4),
            "compact_append": round(e[1].elapsed_time(e[2]) / reps, 4),
            "migrants": int(sendm.count.sum().item())}
        del sendm, outm, work
    if args.resort:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ctx.sort(field, pa, pb)
        e0.record()
        for _ in range(5):
            ctx.sort(field, pa, pb)
        e1.record()
        torch.cuda.synchronize()
        res["sort_ms"] = round(e0.elapsed_time(e1) / 5, 4)
    if not args.graph and not args.resort and not args.no_graph_replay:
        # the same steps replayed from captured HIP graphs (two graphs: A->B, B->A)
        ctx.set_timing(0)
        ctx.set_graph(True)
        restore(pa, snap)
        for _ in range(2):
            do_step(pa, pb)
            pa, pb = pb, pa
        torch.cuda.synchronize()
        tg0 = time.perf_counter()
        for _ in range(args.steps):
            do_step(pa, pb)
            pa, pb = pb, pa
        torch.cuda.synchronize()
        tg1 = time.perf_counter()
        ctx.set_graph(False)
        f = ctx.get_status()
        if f:
            raise SystemExit(f"{label}: flags after graph steps: {pm.flag_names(f)}")
        res["graph_ms_per_step"] = round((tg1 - tg0) * 1e3 / args.steps, 5)
    if args.cpu_delegated and label == args.first_mode:
        res["delegated"] = delegated_transfers(ctx, field, pa, params, dev)
    if plain:
        # the plain path: three calls per step over all subdomains, advancing
        # in place on a copy so that the step's input stays intact
        ctx.set_timing(0)
        restore(pa, snap)
        sendp = pm.DevicePool.empty(sb, sc, vdtype=vdt, device=dev)
        work = pm.DevicePool.empty(pool.base, pool.cap, vdtype=vdt, device=dev, size=size)
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        for _ in range(args.steps):
            work.x.copy_(pa.x)
            work.v.copy_(pa.v)
            work.tau.copy_(pa.tau)
            work.id.copy_(pa.id)
            work.count.copy_(pa.count)
            ctx.interp_advance(field, work, params)
            ctx.classify_scan_pack(dc, work, sendp)
            ctx.compact_append(dc, work, sendp, pb)
            pa, pb = pb, pa
        torch.cuda.synchronize()
        tp1 = time.perf_counter()
        f = ctx.get_status()
        if f:
            raise SystemExit(f"{label}: flags after the plain steps: {pm.flag_names(f)}")
        res["plain_ms_per_step_incl_copy"] = round((tp1 - tp0) * 1e3 / args.steps, 4)
        del sendp, work
    if args.plain_per_sub:
        ctx.set_timing(0)
        sendp = pm.DevicePool.empty(sb, sc, vdtype=vdt, device=dev)
        work = pm.DevicePool.empty(pool.base, pool.cap, vdtype=vdt, device=dev, size=size)
        steps = max(1, min(args.steps, 5))
        torch.cuda.synchronize()
        tq0 = time.perf_counter()
        for _ in range(steps):
            work.x.copy_(pa.x)
            work.v.copy_(pa.v)
            work.tau.copy_(pa.tau)
            work.id.copy_(pa.id)
            work.count.copy_(pa.count)
            for s in range(dc.nsub):
                ctx.interp_advance(field, work, params, s, 1)
            for s in range(dc.nsub):
                ctx.classify_scan_pack(dc, work, sendp, s, 1)
            for s in range(dc.nsub):
                ctx.compact_append(dc, work, sendp, pb, s, 1)
        torch.cuda.synchronize()
        tq1 = time.perf_counter()
        res["plain_per_subdomain_ms_per_step_incl_copy"] = round((tq1 - tq0) * 1e3 / steps, 4)
        del sendp, work
    del pa, pb, send, ctx, mid, msend
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(subdomains are virtual partitions of one device)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2604_11008_amd import accounting, pm

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.side_stream:
        torch.cuda.set_stream(torch.cuda.Stream(device=dev))
    precision = args.precision
    if precision == "auto":
        precision = "both" if args.config == "C5" else gen.CONFIGS[args.config]["mode"]
    modes = {"both": ["f64", "mixed"], "f64": ["f64"], "mixed": ["mixed"]}[precision]
    t_gen = time.perf_counter()
    big = gen.CONFIGS[args.config]["n"] >= 512
    multi = np.prod(gen.CONFIGS[args.config]["p"]) > 1
    # subdomain counts random-walk as particles migrate: leave room to grow;
    # the pool holds float64 tau (rounded for the mixed run)
    wl = gen.make_workload(args.config, field_backend="device" if big else "numpy",
                           slack=0.25 if multi else 0.05, extra=4096 if multi else 1024,
                           order=args.order, sort_device=dev if big else None,
                           mode_override="f64")
    t_gen = time.perf_counter() - t_gen
    pool = wl.pool
    npart = int(pool.count.sum())
    size = pool.x.shape[1]
    dc = pm.Decomp(wl.p, wl.bounds)
    sb, sc = gen.send_layout(pool.count, face=0.05, edge=0.01, corner=0.005)
    field64 = pm.DeviceField(wl.stored_field(np.float64), wl.n, wl.halo, wl.L, device=dev,
                             stagger=args.stagger)
    wl.field = None
    # start state: v0 = U(x0) interpolated in float64 on the device (rounded to
    # float32 for the mixed run)
    pa = pm.DevicePool.from_host(pool, dev)
    ctx0 = pm.Context(size, 1, dc.nsub, device=dev)
    pa.v.copy_(ctx0.interp(field64, pa.x))
    del ctx0
    start64 = (pa.x, pa.v, pa.tau, pa.id, pa.count)
    fh = None
    if not args.no_cpu:
        # the oracle reads the float64 field from host memory
        fh = [u.cpu().numpy() for u in field64.u]
    log(f"{args.config}: {npart} particles, field {wl.n}^3 halo={wl.halo}, "
        f"{dc.nsub} subdomains, dt={wl.dt:.4g}, gen {t_gen:.1f}s, runs {modes}")

    layout = args.layout
    if layout == "auto":
        layout = "both" if args.config == "C5" and not args.stagger else "split"
    if layout != "split" and args.stagger:
        raise SystemExit("the interleaved layout is for collocated fields")
    plain_on = args.plain == "on" or (args.plain == "auto" and precision == "both")
    args.first_mode = modes[0]
    # the interleaved runs from the same start: timed steps only (no samples,
    # graph replay or plain path), in their own default launch shape (or the
    # one --tune gives)
    ilv_args = argparse.Namespace(**vars(args))
    ilv_args.no_cpu = ilv_args.no_graph_replay = True
    ilv_args.cpu_delegated = ilv_args.migration_only = ilv_args.plain_per_sub = False
    results, ilv_results = {}, {}
    for mode in modes:
        if mode == "f64":
            field, start = field64, start64
        else:
            # the mixed form's field: float64 values rounded to float32, split
            # (timed for comparison with the interleaved rounding below)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            u32 = [u.float() for u in field64.u]
            e1.record()
            torch.cuda.synchronize()
            split_round_ms = e0.elapsed_time(e1)
            field = pm.DeviceField(u32, wl.n, wl.halo, wl.L, device=dev, stagger=args.stagger)
            del u32
            start = (start64[0], start64[1].float(), start64[2].float(), start64[3],
                     start64[4])
        if layout != "interleaved":
            results[mode] = run(args, wl, dev, field, dc, start, pool, sb, sc,
                                mode == "mixed", plain_on and mode == "f64", mode)
        if layout != "split":
            # the library's pass into the interleaved layout (component c of
            # stored node m at 3m + c): a copy of the float64 field, or the
            # float64 field rounded to float32 for the mixed form; timed on
            # its second call into the same buffer (what a caller pays per
            # field once the buffer exists)
            odt = torch.float64 if mode == "f64" else torch.float32
            fi = pm.interleave_field(field64, dtype=odt)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            pm.interleave_field(field64, out=fi.u[0], dtype=odt)
            e1.record()
            torch.cuda.synchronize()
            interleave_ms = e0.elapsed_time(e1)
            if mode != "f64":
                del field
            torch.cuda.empty_cache()
            if layout == "interleaved":
                results[mode] = run(args, wl, dev, fi, dc, start, pool, sb, sc,
                                    mode == "mixed", plain_on and mode == "f64", mode)
            else:
                ilv_results[mode] = run(ilv_args, wl, dev, fi, dc, start, pool, sb, sc,
                                        mode == "mixed", False, f"{mode} interleaved")
                ilv_results[mode]["interleave_ms"] = interleave_ms
                if mode != "f64":
                    ilv_results[mode]["split_round_ms"] = split_round_ms
                log(f"{mode}: pm_field_interleave {interleave_ms:.3f} ms")
            del fi
        field = None
        del start
        torch.cuda.empty_cache()
    head = results[modes[0]]
    del start64, pa, field64
    torch.cuda.empty_cache()

    # a plain device copy of 1 GiB: the copy rate the kernel is also compared with
    cms, copy_gbps = copy_rate(dev)
    for r in list(results.values()) + list(ilv_results.values()):
        roof = r["roofline"]
        if roof is not None:
            roof["frac_of_copy"] = round(roof["achieved"] / copy_gbps, 4)
            if roof["traffic"]:
                # measured bytes (rocprofv3 FETCH_SIZE + WRITE_SIZE) per kernel time
                tr = roof["traffic"] / (roof["kernel_ms"] * 1e-3) / 1e9
                roof["traffic_GBps"] = round(tr, 1)
                roof["traffic_frac_of_copy"] = round(tr / copy_gbps, 4)
                roof["traffic_over_algorithmic"] = round(
                    roof["traffic"] / roof["algorithmic_bytes_per_launch"], 3)

    cpu = None
    errors = {}
    if not args.no_cpu:
        runs = {m: r.pop("samples") for m, r in results.items()}
        ta = time.perf_counter()
        errors, (m, steps, el) = cpu_leg(wl, fh, runs, pm.Params(wl.dt, wl.g, drag=args.drag),
                                         args.drag, args.stagger, args.staged,
                                         args.sample_steps, (1, args.sample_steps))
        log(f"CPU-baseline leg {time.perf_counter() - ta:.1f} s: {errors}")
        h2d, d2h = link_gbps(torch, dev)
        triad = single_core_triad_gbps()
        model = accounting.cpu_delegated_model(1, accounting.record_bytes(modes[0]), npart,
                                               min(h2d, d2h), triad)
        delegated = None
        if "delegated" in head:
            d = head.pop("delegated")
            pu = delegated_pack_unpack(wl, d.pop("host_state"))
            d.update(pu)
            d["total_ms"] = d["d2h_ms"] + d["pack_ms"] + d["unpack_ms"] + d["h2d_ms"]
            d["what"] = ("one exchange as the CPU-delegated scheme does it: the 17 float64 "
                         "arrays of every record device->host (pinned), the oracle's "
                         "sequential pack and unpack of the advanced records (8 values "
                         "each) on one core, the 17 arrays host->device")
            delegated = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in d.items()}
            log(f"CPU-delegated exchange: {delegated}")
        cpu = {"value": round(m * steps / el, 1), "unit": "particles/s", "cores": 1,
               "kind": "oracle", "host": host_cpu(),
               "sample": f"{steps} whole oracle steps (sequential FP64, one thread, "
                         f"{el:.1f} s) of the {m} particles with ids below {args.sample} "
                         f"(in their pool order and subdomains, the same field), from "
                         f"the {modes[0]} run's start state",
               "cpu_delegated_model": {
                   "link_GBps_h2d": round(h2d, 1), "link_GBps_d2h": round(d2h, 1),
                   "single_core_triad_GBps": round(triad, 1),
                   "ms_per_migration": round(model["total_ms"], 2),
                   "gpu_fused_step_ms": round(head["ms_per_step"], 4)}}
        if delegated is not None:
            cpu["cpu_delegated_measured"] = delegated
    else:
        for r in results.values():
            r.pop("samples", None)

    def summary(r):
        keep = ("ms_per_step", "particles_per_s", "roofline", "graph_ms_per_step",
                "plain_ms_per_step_incl_copy", "plain_per_subdomain_ms_per_step_incl_copy",
                "migration_only_ms", "sort_ms", "stage1_migrants_per_step", "tuning")
        out = {k: r[k] for k in keep if k in r}
        out["hbm_GBps_algorithmic"] = round(r["alg"]["step"] / (r["ms_per_step"] * 1e-3)
                                            / 1e9, 1)
        if r["mode"] in errors and r is results.get(r["mode"]):
            out["error_vs_fp64_oracle"] = errors[r["mode"]]
        return out

    value = head["particles_per_s"]
    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "particles/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "mixed-f32/f64" if modes[0] == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": f"{args.config}: {WORKLOADS[args.config]}" +
                   (", migration after each RK2 stage" if args.staged else "") +
                   (", nonlinear drag" if args.drag == "nonlinear" else "") +
                   (", MAC-staggered field" if args.stagger else "") +
                   (f", {args.order} particle order" if args.order != "canonical" else "") +
                   (f", re-sorted by cell every {args.resort} steps" if args.resort else ""),
                   "particles": npart, "grid": wl.n, "halo": wl.halo,
                   "field_layout": "interleaved" if layout == "interleaved" else "split",
                   "subdomains": list(wl.p), "graph": bool(args.graph),
                   "tuning": head["tuning"],
                   "runs": {m: ("float64 field, velocities and tau" if m == "f64" else
                                "float32 field, velocities and tau; float64 positions")
                            for m in modes}},
        "hbm_GBps_algorithmic": round(head["alg"]["step"] / (head["ms_per_step"] * 1e-3)
                                      / 1e9, 1),
        "algorithmic_bytes_per_step": head["alg"]["step"], "touched_nodes": head["touched"],
        "migrants_per_step": head["migrants"],
        "roofline": head["roofline"], "cpu_baseline": cpu,
        "copy_1GiB_ms": round(cms, 4), "copy_GBps": round(copy_gbps, 1),
    }
    for k in ("graph_ms_per_step", "plain_ms_per_step_incl_copy",
              "plain_per_subdomain_ms_per_step_incl_copy", "migration_only_ms", "sort_ms",
              "stage1_migrants_per_step"):
        if k in head:
            line[k] = head[k]
    if modes[0] in errors:
        line["error_vs_fp64_oracle"] = errors[modes[0]]
    if "mixed" in results and modes[0] != "mixed":
        mx = results["mixed"]
        line["mixed"] = summary(mx)
        line["mixed"]["speedup_vs_fused_f64"] = round(head["ms_per_step"] / mx["ms_per_step"],
                                                      3)
        if "plain_ms_per_step_incl_copy" in head:
            line["mixed"]["speedup_vs_plain_f64"] = round(
                head["plain_ms_per_step_incl_copy"] / mx["ms_per_step"], 3)
    if ilv_results:
        line["interleaved"] = {}
        for m, r in ilv_results.items():
            e = summary(r)
            e["speedup_vs_split"] = round(results[m]["ms_per_step"] / r["ms_per_step"], 3)
            saved = results[m]["ms_per_step"] - r["ms_per_step"]
            e["interleave_copy_ms"] = round(r["interleave_ms"], 4)
            if "split_round_ms" in r:
                # the float32 field is written by a rounding pass either way
                e["split_round_ms"] = round(r["split_round_ms"], 4)
                extra = r["interleave_ms"] - r["split_round_ms"]
                e["steps_to_repay_the_copy"] = (max(0.0, round(extra / saved, 1))
                                                if saved > 0 else None)
            else:
                e["steps_to_repay_the_copy"] = (round(r["interleave_ms"] / saved, 1)
                                                if saved > 0 else None)
            e["bitwise_equal_to_split"] = r["state_digest"] == results[m]["state_digest"]
            line["interleaved"][m] = e
        line["interleaved"]["what"] = (
            "the same steps from the same start state with the field stored node-"
            "interleaved (component c of node m at 3m + c), as a solver that can store "
            "it would hand it over, or as pm_field_interleave writes it from the float64 "
            "split field (interleave_copy_ms, outside the timed steps: a copy, or for the "
            "mixed form the rounding to float32 that the split float32 field also needs, "
            "split_round_ms)")
        if not all(e["bitwise_equal_to_split"] for k, e in line["interleaved"].items()
                   if k != "what"):
            print(json.dumps(line), flush=True)
            raise SystemExit("interleaved layout: final state differs from the split run's")
    line["state_digest"] = head["state_digest"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
