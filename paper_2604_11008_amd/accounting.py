"""Byte accounting for the particle step and the paper's CPU-delegated cost
model.  Host-side bookkeeping only; no step arithmetic."""
from __future__ import annotations

# MI355X published peaks
HBM_PEAK_GBPS = 8000.0
FP64_VECTOR_TFLOPS = 78.6
FP32_VECTOR_TFLOPS = 157.3


def record_bytes(mode: str) -> int:
    """Bytes of one particle record: x,y,z (f64) + v (3) + tau + id (u64).
    "f64": velocity and tau in float64 (64 B); "mixed": in float32 (48 B)."""
    if mode == "f64":
        return 3 * 8 + 3 * 8 + 8 + 8
    if mode == "mixed":
        return 3 * 8 + 3 * 4 + 4 + 8
    raise ValueError(mode)


def field_value_bytes(mode: str) -> int:
    return 8 if mode == "f64" else 4


def step_algorithmic_bytes(n_particles, migrants, touched_nodes, mode):
    """What one full step must move at minimum: every record read once and
    written once, every migrant written to and read back from its send buffer
    once, and every field node some stencil touches read once (3 components).
    Returns a dict with the split per kernel of the fused path."""
    s_rec = record_bytes(mode)
    s_f = field_value_bytes(mode)
    fused = n_particles * 2 * s_rec + touched_nodes * 3 * s_f
    append = migrants * 2 * s_rec
    return {"step": fused + append, "fused_kernel": fused, "append_kernel": append,
            "per_particle_record": s_rec, "per_node": 3 * s_f}


def mid_record_bytes(mode):
    """Mid-step record of per-stage migration: X_n, X* (float64) and V_n, V*,
    dV/dt, tau (float64, or float32 in the mixed mode), id."""
    s = 8 if mode == "f64" else 4
    return 6 * 8 + 10 * s + 8


def staged_algorithmic_bytes(n_particles, migrants1, migrants2, touched_nodes, mode):
    """Both stage kernels of per-stage migration: stage 1 reads each plain
    record and writes a mid-step record, stage 2 reads it back and writes a
    plain record; every touched field node is read at least once (the union
    over both stages, a lower bound); leavers of each stage go to and come
    back from their send buffers."""
    s_rec, s_mid = record_bytes(mode), mid_record_bytes(mode)
    s_f = field_value_bytes(mode)
    kernels = n_particles * 2 * (s_rec + s_mid) + touched_nodes * 3 * s_f
    exchange = migrants1 * 2 * s_mid + migrants2 * 2 * s_rec
    return {"step": kernels + exchange, "stage_kernels": kernels,
            "exchange": exchange}


def cpu_delegated_model(arrays, bytes_per_value, particles, link_gbps, core_gbps):
    """Sect. 3.2.2: the full particle arrays go device->host over the link,
    are packed and unpacked sequentially at one core's memory bandwidth, and
    come back host->device; per RK2 stage t = 2 (V/link + V/core)."""
    volume = arrays * bytes_per_value * particles
    d2h = volume / (link_gbps * 1e9)
    pack = volume / (core_gbps * 1e9)
    return {"volume_GB": volume / 1e9, "d2h_ms": d2h * 1e3, "h2d_ms": d2h * 1e3,
            "pack_ms": pack * 1e3, "unpack_ms": pack * 1e3,
            "total_ms": 2 * (d2h + pack) * 1e3}
