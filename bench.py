"""Benchmark of the fused particle step on one MI355X.

Default workload (the 256^3 single-subdomain case): a 256^3 collocated FP64
velocity field stored with a one-cell halo, 4,194,304 particles uniform in the
box, tau log-uniform in [0.01, 1], gravity (0,0,-1), dt giving at most half a
cell per step; one subdomain whose 26 neighbours are its own periodic images.

A step is the whole hot path over every particle: interpolation at two RK2
stages, the Heun drag update, classification, scan, pack/compact and the
on-device append of the migrants.  Inputs are resident in HBM before the
timed region.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
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
    "C5": "1024^3 periodic FP32 field, 2^28 blob-clustered particles (FP64 positions, "
          "FP32 velocity/tau), 8x8x8 subdomains",
    "CP": "750^3 FP64 field with a one-cell halo, 52,734,375 uniform particles (750^3/8, "
          "the paper's per-rank share), 1 subdomain, tau log-uniform [0.01,1], g=(0,0,-1)",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="C2", choices=sorted(WORKLOADS))
    ap.add_argument("--order", default="canonical",
                    choices=["canonical", "morton", "rowmajor", "shuffled"],
                    help="particle order within each segment at the start: cell-sorted "
                         "(canonical: Z-order over x pairs; morton; rowmajor) or shuffled")
    ap.add_argument("--precision", default="auto", choices=["auto", "f64", "mixed"],
                    help="override the workload's arithmetic (mixed: float32 field, "
                         "velocities and tau; float64 positions)")
    ap.add_argument("--drag", default="stokes", choices=["stokes", "nonlinear"],
                    help="drag law: Stokes (f = 1) or the paper's nonlinear correction "
                         "(nu = 1.5e-5, rho_p/rho = 843 in the field's units)")
    ap.add_argument("--stagger", action="store_true",
                    help="read the field as MAC-staggered (component c on the faces "
                         "normal to axis c)")
    ap.add_argument("--staged", action="store_true",
                    help="migrate after each RK2 stage (the paper's scheme) instead of once "
                         "per step")
    ap.add_argument("--migration-only", action="store_true",
                    help="also time the exchange alone (classify/scan/pack + "
                         "compact/append, no advance) on the timed state")
    ap.add_argument("--graph", action="store_true", help="replay captured HIP graphs")
    ap.add_argument("--tune", default=None, help="wg,items[,blocks_per_cu[,xcd_block]] or 'auto'")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--resort", type=int, default=0,
                    help="re-sort the pool by cell (pm_sort) every K steps inside the "
                         "timed region (0: never, the paper's method)")
    ap.add_argument("--accuracy", action="store_true",
                    help="also run --accuracy-steps untimed steps from the start state and "
                         "report the error of the particles with the lowest ids against "
                         "the FP64 oracle after the first and the last")
    ap.add_argument("--accuracy-sample", type=int, default=1 << 20)
    ap.add_argument("--accuracy-steps", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="accepted for the profiling commands: the plain torch copy of "
                         "1 GiB (the counters' scaling reference and the copy-rate "
                         "figure) always runs")
    ap.add_argument("--traffic", default=None,
                    help="traffic record of the fused kernel (default: "
                         "profiles/k_step_<config>_traffic.json)")
    ap.add_argument("--plain", action="store_true", help="time the 3-call plain path too")
    ap.add_argument("--side-stream", action="store_true",
                    help="run on a new (default-priority) stream instead of the null stream")
    ap.add_argument("--plain-per-sub", action="store_true",
                    help="time the plain path launched once per subdomain")
    return ap.parse_args()


def host_field64(wl):
    """The stored field as float64 numpy arrays (copied off the device when the
    field was generated there)."""
    return [u if isinstance(u, np.ndarray) else u.cpu().numpy()
            for u in wl.stored_field(np.float64)]


def subsample(p, nmax):
    """Valid records of device pool p whose id is below nmax, sorted by id, on
    the host as float64 (x, v, tau, id)."""
    import torch
    size = p.x.shape[1]
    valid = torch.zeros(size, dtype=torch.bool, device=p.x.device)
    base, count = p.base.cpu().numpy(), p.count.cpu().numpy()
    for b, c in zip(base, count):
        if c > 0:
            valid[int(b):int(b) + int(c)] = True
    sel = torch.nonzero(valid & (p.id < nmax)).squeeze(1)
    ids = p.id[sel]
    order = torch.argsort(ids)
    sel = sel[order]
    return (p.x[:, sel].cpu().numpy(), p.v[:, sel].double().cpu().numpy(),
            p.tau[sel].double().cpu().numpy(), p.id[sel].cpu().numpy().astype(np.uint64))


def accuracy_report(wl, field, dc, ctx, params, pstart, pool_template, sb, sc, vdt, dev,
                    nmax, steps, drag):
    """Untimed: `steps` device steps from pstart on spare pools, and the oracle
    in FP64 (the float64 field) on the particles with id < nmax from the same
    start state (float64 positions; velocities and tau as the device holds
    them).  Particles do not interact, so the oracle follows the subsample
    alone, in one periodic subdomain.  Errors: max |dV| / max|u| and max |dX|
    in cells (across the periodic seam), after the first and the last step."""
    import oracle
    from paper_2604_11008_amd import pm
    qa = pm.DevicePool(pstart.x.clone(), pstart.v.clone(), pstart.tau.clone(),
                       pstart.id.clone(), pstart.base, pstart.cap, pstart.count.clone())
    qb = pm.DevicePool.empty(pool_template.base, pool_template.cap, vdtype=vdt, device=dev,
                             size=pstart.x.shape[1])
    qsend = pm.DevicePool.empty(sb, sc, vdtype=vdt, device=dev)
    x0, v0, tau0, id0 = subsample(qa, nmax)
    got = {}
    for k in range(1, steps + 1):
        ctx.step(field, dc, qa, qb, qsend, params)
        qa, qb = qb, qa
        if k in (1, steps):
            got[k] = subsample(qa, nmax)
    f = ctx.get_status()
    if f:
        raise SystemExit(f"accuracy run flags: {pm.flag_names(f)}")
    del qa, qb, qsend
    fh = host_field64(wl)
    umax = max(float(np.abs(u).max()) for u in fh)
    of = oracle.Field(fh, wl.n, wl.halo, wl.L)
    od = oracle.Decomp((1, 1, 1), gen.bounds((1, 1, 1), wl.L))
    m = len(id0)
    cap = np.array([m + 1024], dtype=np.int64)
    host = gen.empty_pool(np.zeros(1, dtype=np.int64), cap)
    host.x[:, :m], host.v[:, :m], host.tau[:m], host.id[:m] = x0, v0, tau0, id0
    host.count[0] = m
    osb, osc = gen.send_layout(host.count, face=0.2, edge=0.05, corner=0.03)
    out = {"subsample": m, "ids": f"below {nmax}", "steps": steps,
           "oracle": "FP64 on the float64 field, one periodic subdomain"}
    cell = wl.n / wl.L
    for k in range(1, steps + 1):
        nxt = gen.empty_pool(host.base, host.cap)
        send = gen.empty_pool(osb, osc)
        _, fl = oracle.step(of, od, params.dt, params.g, host, nxt, send, drag=drag,
                            nu=params.nu, density_ratio=params.density_ratio)
        if fl:
            raise SystemExit(f"oracle flags {fl} in the accuracy run")
        host = nxt
        if k in got:
            c = int(host.count[0])
            o = np.argsort(host.id[:c], kind="stable")
            rx, rv, rid = host.x[:, :c][:, o], host.v[:, :c][:, o], host.id[:c][o]
            gx, gv, _, gid = got[k]
            if not np.array_equal(rid, gid):
                raise SystemExit("accuracy run: the device and the oracle hold different ids")
            dx = np.abs(gx - rx)
            dx = np.minimum(dx, wl.L - dx)
            out[f"after_{k}"] = {"v_err_rel_umax": float(np.abs(gv - rv).max() / umax),
                                 "x_err_cells": float(dx.max() * cell)}
    return out


def cpu_baseline(wl, seconds, drag="stokes", stagger=False, max_particles=1 << 22):
    """The oracle, single-threaded, on whole steps of the same workload for
    about `seconds`.  Workloads above max_particles run on the first
    count * max_particles / Np particles of every segment (same field,
    decomposition and particle distribution), so one step stays short."""
    import oracle
    pool = wl.pool
    npart_all = int(pool.count.sum())
    subset = npart_all > max_particles
    if subset:
        pool = gen.Pool(x=pool.x, v=pool.v, tau=pool.tau, id=pool.id, base=pool.base,
                        cap=pool.cap, count=pool.count * max_particles // npart_all)
    of = oracle.Field(host_field64(wl), wl.n, wl.halo, wl.L, stagger=stagger)
    od = oracle.Decomp(wl.p, wl.bounds)
    sb, sc = gen.send_layout(pool.count, face=0.05, edge=0.01, corner=0.005)
    npart = int(pool.count.sum())
    done = 0
    t0 = time.perf_counter()
    steps = 0
    while True:
        out = gen.empty_pool(pool.base, pool.cap)
        send = gen.empty_pool(sb, sc)
        oracle.step(of, od, wl.dt, wl.g, pool, out, send, drag=drag)
        steps += 1
        done += npart
        if time.perf_counter() - t0 >= seconds:
            break
    el = time.perf_counter() - t0
    what = (f"the first {npart} of {npart_all} particles (the same share of every segment)"
            if subset else f"all {npart} particles")
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f
                          if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": done / el, "unit": "particles/s", "cores": 1, "kind": "oracle",
            "host": {"cpu": model, "threads": os.cpu_count()},
            "sample": f"{steps} whole oracle step(s) of the same workload on {what}, "
                      f"sequential FP64, one thread, {el:.1f} s"}


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
    t_gen = time.perf_counter()
    big = gen.CONFIGS[args.config]["n"] >= 512
    multi = np.prod(gen.CONFIGS[args.config]["p"]) > 1
    # subdomain counts random-walk as particles migrate: leave room to grow
    wl = gen.make_workload(args.config, field_backend="device" if big else "numpy",
                           slack=0.25 if multi else 0.05, extra=4096 if multi else 1024,
                           order=args.order)
    t_gen = time.perf_counter() - t_gen
    mixed = wl.mode == "mixed" if args.precision == "auto" else args.precision == "mixed"
    if mixed != (wl.mode == "mixed"):
        cast = np.float32 if mixed else np.float64
        wl.pool.v = wl.pool.v.astype(cast)
        wl.pool.tau = wl.pool.tau.astype(cast)
        wl.mode = "mixed" if mixed else "f64"
    fdt = np.float32 if mixed else np.float64
    field = pm.DeviceField(wl.stored_field(fdt), wl.n, wl.halo, wl.L, device=dev,
                           stagger=args.stagger)
    dc = pm.Decomp(wl.p, wl.bounds)
    vdt = torch.float32 if mixed else torch.float64
    pool = wl.pool
    npart = int(pool.count.sum())
    size = pool.x.shape[1]
    pa = pm.DevicePool.from_host(pool, dev)
    pb = pm.DevicePool.empty(pool.base, pool.cap, vdtype=vdt, device=dev, size=size)
    sb, sc = gen.send_layout(pool.count, face=0.05, edge=0.01, corner=0.005)
    send = pm.DevicePool.empty(sb, sc, vdtype=vdt, device=dev)
    ctx = pm.Context(size, send.size, dc.nsub, device=dev)
    # v0 = U(x0), interpolated on the device
    pa.v.copy_(ctx.interp(field, pa.x))
    params = pm.Params(wl.dt, wl.g, drag=args.drag)
    accuracy = None
    if args.accuracy:
        if args.staged or args.stagger:
            raise SystemExit("--accuracy runs the per-step path on collocated fields")
        ta = time.perf_counter()
        accuracy = accuracy_report(wl, field, dc, ctx, params, pa, pool, sb, sc, vdt, dev,
                                   args.accuracy_sample, args.accuracy_steps, args.drag)
        print(f"[bench] accuracy run {time.perf_counter() - ta:.1f} s: {accuracy}",
              file=sys.stderr, flush=True)
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

    if args.tune == "auto":
        ctx.autotune(field, dc, pa, pb, send, params, cache_path=args.tune_cache)
    elif args.tune:
        t = [int(v) for v in args.tune.split(",")]
        ctx.set_tuning(*t)
    if args.graph:
        ctx.set_graph(True)
    torch.cuda.synchronize()
    print(f"[bench] {args.config}: {npart} particles, field {wl.n}^3 halo={wl.halo}, "
          f"{dc.nsub} subdomains, dt={wl.dt:.4g}, gen {t_gen:.1f}s, tuning {ctx.get_tuning()}",
          file=sys.stderr, flush=True)

    # warm-up
    for _ in range(args.warmup):
        do_step(pa, pb)
        pa, pb = pb, pa
    f = ctx.get_status()
    if f:
        raise SystemExit(f"warm-up flags: {pm.flag_names(f)}")

    # algorithmic bytes of a step of this state (untimed): touched field nodes
    # and migrants
    touched = ctx.touched_nodes(field, pa, params)
    do_step(pa, pb)
    migrants = int(send.count.sum().item())
    pa, pb = pb, pa
    if args.staged:
        migrants1 = int(msend.count.sum().item())
        alg = accounting.staged_algorithmic_bytes(npart, migrants1, migrants, touched,
                                                  "mixed" if mixed else "f64")
        alg["fused_kernel"] = alg["stage_kernels"]
    else:
        alg = accounting.step_algorithmic_bytes(npart, migrants, touched,
                                                "mixed" if mixed else "f64")

    # the state the timed steps start from, so the graph replays below start
    # from it too (kernel time drifts as particles disperse from their sorted
    # start order)
    snap = [t.clone() for t in (pa.x, pa.v, pa.tau, pa.id, pa.count)]

    # timed region
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
        raise SystemExit(f"flags after timed steps: {pm.flag_names(f)}")
    ms_step = (t1 - t0) * 1e3 / args.steps
    k_total, k_each = (ctx.kernel_times() if not args.graph else (None, []))
    if args.staged and k_each:  # the two stage kernels of a step, summed
        k_each = [a + b for a, b in zip(k_each[0::2], k_each[1::2])]
    k_ms = (k_total / len(k_each)) if k_each else None
    print(f"[bench] {args.steps} steps: {ms_step:.4f} ms/step; fused kernel "
          f"{k_ms if k_ms is None else round(k_ms, 4)} ms", file=sys.stderr, flush=True)

    roof = None
    if k_ms:
        achieved = alg["fused_kernel"] / (k_ms * 1e-3) / 1e9
        from paper_2604_11008_amd import profsum
        wg, items = ctx.get_tuning()[:2]
        tf = lambda b: "true" if b else "false"  # noqa: E731
        variant = (f"k_step<{wg}, {items}, {'float' if mixed else 'double'}, "
                   f"{tf(wl.halo)}, {tf(args.drag == 'nonlinear')}, {tf(args.stagger)}>")
        tpath = args.traffic or os.path.join(ROOT, "profiles",
                                             f"k_step_{args.config}_traffic.json")
        traffic = None
        # the record was taken on the canonical start order of this workload
        if os.path.exists(tpath) and json.load(open(tpath)).get("kernel") == variant \
                and not args.staged and args.order == "canonical":
            traffic = profsum.load_traffic(tpath)
        roof = {"bound": "hbm", "achieved": round(achieved, 1),
                "peak": accounting.HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / accounting.HBM_PEAK_GBPS, 4), "traffic": traffic,
                "kernel": ("k_stage<1> + k_stage<2> (the two per-stage fused kernels)"
                           if args.staged else
                           "k_step (fused interpolate/advance/classify/scan/scatter)"),
                "kernel_ms": round(k_ms, 5),
                "kernel_ms_first_last": [round(k_each[0], 5), round(k_each[-1], 5)],
                "kernel_ms_min_median_max": [round(float(np.min(k_each)), 5),
                                             round(float(np.median(k_each)), 5),
                                             round(float(np.max(k_each)), 5)],
                "algorithmic_bytes_per_launch": alg["fused_kernel"]}

    extra = {}
    if args.staged:
        extra["stage1_migrants_per_step"] = migrants1
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
        extra["migration_only_ms"] = {
            "classify_scan_pack": round(e[0].elapsed_time(e[1]) / reps, 4),
            "compact_append": round(e[1].elapsed_time(e[2]) / reps, 4),
            "migrants": int(sendm.count.sum().item())}
        del sendm, outm, work
    if args.resort:
        # the re-sort alone, on the final state
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ctx.sort(field, pa, pb)
        e0.record()
        for _ in range(5):
            ctx.sort(field, pa, pb)
        e1.record()
        torch.cuda.synchronize()
        extra["sort_ms"] = round(e0.elapsed_time(e1) / 5, 4)
    if not args.graph and not args.resort:
        # the same steps replayed from captured HIP graphs (two graphs: A->B, B->A)
        ctx.set_timing(0)
        ctx.set_graph(True)
        if pa.size != snap[0].shape[1]:
            raise SystemExit("pool size changed")
        for t, v in zip((pa.x, pa.v, pa.tau, pa.id, pa.count), snap):
            t.copy_(v)
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
            raise SystemExit(f"flags after graph steps: {pm.flag_names(f)}")
        extra["graph_ms_per_step"] = round((tg1 - tg0) * 1e3 / args.steps, 5)
    if args.plain:
        ctx.set_timing(0)
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
        torch.cuda.synchronize()
        tp1 = time.perf_counter()
        extra["plain_ms_per_step_incl_copy"] = round((tp1 - tp0) * 1e3 / args.steps, 4)

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
        extra["plain_per_subdomain_ms_per_step_incl_copy"] = round((tq1 - tq0) * 1e3 / steps, 4)
    # a plain device copy of 1 GiB: the copy rate the kernel is also compared with
    cms, copy_gbps = copy_rate(dev)
    extra["copy_1GiB_ms"] = round(cms, 4)
    extra["copy_GBps"] = round(copy_gbps, 1)
    if roof is not None:
        roof["frac_of_copy"] = round(roof["achieved"] / copy_gbps, 4)
        if roof["traffic"]:
            # measured bytes (rocprofv3 FETCH_SIZE + WRITE_SIZE) per kernel time
            tr = roof["traffic"] / (roof["kernel_ms"] * 1e-3) / 1e9
            roof["traffic_GBps"] = round(tr, 1)
            roof["traffic_frac_of_copy"] = round(tr / copy_gbps, 4)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(wl, args.cpu_seconds, args.drag, args.stagger)
        # the paper's CPU-delegated estimate (Sect. 3.2.2) for this host and workload:
        # arrays out and back over the link, packed and unpacked at one core's bandwidth
        h2d, d2h = link_gbps(torch, dev)
        triad = single_core_triad_gbps()
        model = accounting.cpu_delegated_model(1, accounting.record_bytes(
            "mixed" if mixed else "f64"), npart, min(h2d, d2h), triad)
        extra["cpu_delegated_model"] = {
            "link_GBps_h2d": round(h2d, 1), "link_GBps_d2h": round(d2h, 1),
            "single_core_triad_GBps": round(triad, 1),
            "ms_per_migration": round(model["total_ms"], 2),
            "gpu_fused_step_ms": round(ms_step, 4)}

    value = npart / (ms_step * 1e-3)
    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "particles/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "mixed-f32/f64" if mixed else "f64", "data": "synthetic",
        "config": {"workload": f"{args.config}: {WORKLOADS[args.config]}" +
                   (", migration after each RK2 stage" if args.staged else "") +
                   (f" (run at {args.precision})" if args.precision != "auto" else "") +
                   (", nonlinear drag" if args.drag == "nonlinear" else "") +
                   (", MAC-staggered field" if args.stagger else "") +
                   (f", {args.order} particle order" if args.order != "canonical" else "") +
                   (f", re-sorted by cell every {args.resort} steps" if args.resort else ""),
                   "particles": npart, "grid": wl.n, "halo": wl.halo,
                   "subdomains": list(wl.p), "graph": bool(args.graph),
                   "tuning": list(ctx.get_tuning())},
        "hbm_GBps_algorithmic": round(alg["step"] / (ms_step * 1e-3) / 1e9, 1),
        "algorithmic_bytes_per_step": alg["step"], "touched_nodes": touched,
        "migrants_per_step": migrants,
        "roofline": roof, "cpu_baseline": cpu,
        **({"accuracy": accuracy} if accuracy is not None else {}),
    }
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
