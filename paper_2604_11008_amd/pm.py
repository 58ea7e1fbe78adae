"""Python binding of libpm.so (include/pm.h): argument marshalling only.

Every step of the particle update runs in the HIP kernels of the library;
this module turns torch tensors into the C structures and calls the entry
points of the same names on the current torch stream.  If the library is
not built, the first call raises: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpm.so")

F64, F32 = 0, 1
LAYOUT_SPLIT, LAYOUT_INTERLEAVED = 0, 1
STAY = 13
SEND_OVERFLOW, DEST_OVERFLOW, SKIP, NONFINITE, HALO, LAYOUT = 1, 2, 4, 8, 16, 32
FLAG_NAMES = {SEND_OVERFLOW: "SEND_OVERFLOW", DEST_OVERFLOW: "DEST_OVERFLOW", SKIP: "SKIP",
              NONFINITE: "NONFINITE", HALO: "HALO", LAYOUT: "LAYOUT"}
SHAPES = [(256, 1), (256, 2), (256, 4), (256, 8), (512, 1), (512, 2), (512, 4)]


class PMError(RuntimeError):
    pass


# --- C structures (pm.h) -------------------------------------------------------

class _Field(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("halo", C.c_int32), ("L", C.c_double * 3),
                ("dtype", C.c_int32), ("stagger", C.c_int32), ("u", C.c_void_p * 3),
                ("layout", C.c_int32)]


class _Decomp(C.Structure):
    _fields_ = [("p", C.c_int32 * 3), ("pad_", C.c_int32), ("bounds", C.c_void_p * 3)]


class _Particles(C.Structure):
    _fields_ = [("nsub", C.c_int32), ("vdtype", C.c_int32), ("base", C.c_void_p),
                ("cap", C.c_void_p), ("count", C.c_void_p), ("x", C.c_void_p * 3),
                ("v", C.c_void_p * 3), ("tau", C.c_void_p), ("id", C.c_void_p)]


class _Send(C.Structure):
    _fields_ = [("base", C.c_void_p), ("cap", C.c_void_p), ("count", C.c_void_p),
                ("x", C.c_void_p * 3), ("v", C.c_void_p * 3), ("tau", C.c_void_p),
                ("id", C.c_void_p)]


class _StageParticles(C.Structure):
    _fields_ = [("nsub", C.c_int32), ("vdtype", C.c_int32), ("base", C.c_void_p),
                ("cap", C.c_void_p), ("count", C.c_void_p), ("x", C.c_void_p * 3),
                ("v", C.c_void_p * 3), ("xs", C.c_void_p * 3), ("vs", C.c_void_p * 3),
                ("a", C.c_void_p * 3), ("tau", C.c_void_p), ("id", C.c_void_p)]


class _StageSend(C.Structure):
    _fields_ = [("base", C.c_void_p), ("cap", C.c_void_p), ("count", C.c_void_p),
                ("x", C.c_void_p * 3), ("v", C.c_void_p * 3), ("xs", C.c_void_p * 3),
                ("vs", C.c_void_p * 3), ("a", C.c_void_p * 3), ("tau", C.c_void_p),
                ("id", C.c_void_p)]


class _Params(C.Structure):
    _fields_ = [("dt", C.c_double), ("g", C.c_double * 3), ("drag", C.c_int32),
                ("pad_", C.c_int32), ("nu", C.c_double), ("density_ratio", C.c_double)]


DRAG = {"stokes": 0, "nonlinear": 1}


class _Tuning(C.Structure):
    _fields_ = [("wg", C.c_int32), ("items", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("xcd_block", C.c_int32)]


_lib = None


def lib():
    """The loaded library (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise PMError(f"{LIB_PATH} is not built: run python -c "
                          "'import __graft_entry__; __graft_entry__.build()'")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        sig = {
            "pm_workspace_bytes": ([i64, i64, i32], C.c_size_t),
            "pm_create": ([vp, vp, C.c_size_t, i64, i64, i32], C.c_int),
            "pm_destroy": ([vp], C.c_int),
            "pm_interp": ([vp, vp, i64, vp, vp, vp, vp, vp, vp, vp], C.c_int),
            "pm_interp_advance": ([vp, vp, vp, vp, i32, i32, vp], C.c_int),
            "pm_classify_scan_pack": ([vp, vp, vp, vp, i32, i32, vp], C.c_int),
            "pm_compact_append": ([vp, vp, vp, vp, vp, i32, i32, vp], C.c_int),
            "pm_step": ([vp, vp, vp, vp, vp, vp, vp, vp], C.c_int),
            "pm_step_staged": ([vp, vp, vp, vp, vp, vp, vp, vp, vp, vp], C.c_int),
            "pm_step_noalloc": ([vp, vp, vp, vp, vp, vp, i64, i64, vp, vp], C.c_int),
            "pm_field_interleave": ([vp, i32, vp, vp], C.c_int),
            "pm_get_status": ([vp, vp, vp], C.c_int),
            "pm_set_tuning": ([vp, vp], C.c_int),
            "pm_get_tuning": ([vp, vp], C.c_int),
            "pm_autotune": ([vp, vp, vp, vp, vp, vp, vp, vp, C.c_char_p], C.c_int),
            "pm_set_graph": ([vp, i32], C.c_int),
            "pm_set_timing": ([vp, i32], C.c_int),
            "pm_kernel_times": ([vp, vp, vp, vp, i32], C.c_int),
            "pm_touched_nodes": ([vp, vp, vp, vp, vp, i64, vp, vp], C.c_int),
            "pm_last_error": ([], C.c_char_p),
            "pm_sort_workspace_bytes": ([i64, i32], C.c_size_t),
            "pm_sort": ([vp, vp, vp, vp, vp, C.c_size_t, vp], C.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        msg = lib().pm_last_error().decode()
        raise PMError(f"{'argument' if rc == 1 else 'HIP'} error: {msg}")


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _p(t: torch.Tensor):
    return t.data_ptr()


def _rows(t: torch.Tensor):
    """Pointers of the three rows of a contiguous (3, n) tensor (computed, so
    that no row views are made on every call)."""
    p = t.data_ptr()
    step = t.stride(0) * t.element_size()
    return (C.c_void_p * 3)(p, p + step, p + 2 * step)


# --- device-side objects -------------------------------------------------------------

class DeviceField:
    """Velocity field on the device (float64 or float32).  Split layout:
    `u` is three flat tensors, one per component; stagger=True: MAC
    arrangement (component c on the faces normal to axis c).  Interleaved
    layout (interleaved=True, collocated only): `u` is one tensor of three
    values per stored node, component fastest (shape (nodes, 3) or flat)."""

    def __init__(self, u, n, halo, L, device="cuda", stagger=False, interleaved=False):
        def flat(c):
            if isinstance(c, torch.Tensor):
                return c.reshape(-1).contiguous()
            return torch.as_tensor(np.ascontiguousarray(c).reshape(-1)).to(device)

        self.interleaved = bool(interleaved)
        self.u = [flat(u)] if self.interleaved else [flat(c) for c in u]
        dt = self.u[0].dtype
        if dt not in (torch.float64, torch.float32) or any(c.dtype != dt for c in self.u):
            raise PMError("field components must all be float64 or all float32")
        self.n = (n, n, n) if np.isscalar(n) else tuple(n)
        self.halo = int(halo)
        self.L = (L, L, L) if np.isscalar(L) else tuple(L)
        st = [k + 2 * self.halo for k in self.n]
        nodes = st[0] * st[1] * st[2]
        if self.interleaved:
            if stagger:
                raise PMError("an interleaved field must be collocated")
            if self.u[0].numel() != 3 * nodes:
                raise PMError("interleaved field size does not match n and halo")
            ptrs = [_p(self.u[0]), None, None]
        else:
            if len(self.u) != 3 or any(c.numel() != nodes for c in self.u):
                raise PMError("field size does not match n and halo")
            ptrs = [_p(c) for c in self.u]
        self.dtype = F64 if dt == torch.float64 else F32
        self.stagger = int(bool(stagger))
        self.layout = LAYOUT_INTERLEAVED if self.interleaved else LAYOUT_SPLIT
        self.c = _Field((C.c_int32 * 3)(*self.n), self.halo, (C.c_double * 3)(*self.L),
                        self.dtype, self.stagger, (C.c_void_p * 3)(*ptrs), self.layout)

    @property
    def mixed(self):
        return self.dtype == F32


class Decomp:
    def __init__(self, p, bounds):
        self.p = tuple(int(k) for k in p)
        self.b = [np.ascontiguousarray(b, dtype=np.float64) for b in bounds]
        self.c = _Decomp((C.c_int32 * 3)(*self.p), 0,
                         (C.c_void_p * 3)(*[b.ctypes.data for b in self.b]))

    @property
    def nsub(self):
        return self.p[0] * self.p[1] * self.p[2]


class DevicePool:
    """Particle records on the device, in segments (also used for send buffers)."""

    def __init__(self, x, v, tau, ids, base, cap, count):
        self.x, self.v, self.tau, self.id = x, v, tau, ids
        self.base, self.cap, self.count = base, cap, count
        for t in (x, v):
            if t.dim() != 2 or t.shape[0] != 3 or not t.is_contiguous():
                raise PMError("x and v must be contiguous (3, size) tensors")
        if x.dtype != torch.float64 or ids.dtype != torch.int64:
            raise PMError("x must be float64 and id int64 (read as uint64)")
        if v.dtype != tau.dtype or v.dtype not in (torch.float64, torch.float32):
            raise PMError("v and tau must share float64 or float32")
        for t in (base, cap, count):
            if t.dtype != torch.int64 or not t.is_contiguous():
                raise PMError("base/cap/count must be contiguous int64")

    @property
    def size(self):
        return self.x.shape[1]

    @property
    def nseg(self):
        return self.base.numel()

    @property
    def vdtype(self):
        return F64 if self.v.dtype == torch.float64 else F32

    @classmethod
    def empty(cls, base, cap, vdtype=torch.float64, device="cuda", size=None):
        base = torch.as_tensor(np.asarray(base, dtype=np.int64)).to(device)
        cap = torch.as_tensor(np.asarray(cap, dtype=np.int64)).to(device)
        if size is None:
            size = int((base + cap).max().item()) if base.numel() else 0
        size = max(int(size), 1)
        return cls(torch.zeros((3, size), dtype=torch.float64, device=device),
                   torch.zeros((3, size), dtype=vdtype, device=device),
                   torch.zeros(size, dtype=vdtype, device=device),
                   torch.zeros(size, dtype=torch.int64, device=device), base, cap,
                   torch.zeros(base.numel(), dtype=torch.int64, device=device))

    @classmethod
    def from_host(cls, pool, device="cuda", size=None):
        """From a numpy pool (gen.Pool or alike); size pads the arrays."""
        n = pool.x.shape[1] if size is None else max(size, pool.x.shape[1])

        def pad(a, dtype):
            t = torch.zeros((a.shape[0], n) if a.ndim == 2 else (n,), dtype=dtype)
            src = torch.from_numpy(np.ascontiguousarray(a).astype(
                {torch.float64: np.float64, torch.float32: np.float32,
                 torch.int64: np.int64}[dtype], copy=False))
            if a.ndim == 2:
                t[:, :a.shape[1]] = src
            else:
                t[:a.shape[0]] = src
            return t.to(device)

        vd = torch.float32 if pool.v.dtype == np.float32 else torch.float64
        ids = pool.id.view(np.int64) if pool.id.dtype == np.uint64 else pool.id
        return cls(pad(pool.x, torch.float64), pad(pool.v, vd), pad(pool.tau, vd),
                   pad(ids, torch.int64),
                   torch.as_tensor(np.asarray(pool.base, dtype=np.int64)).to(device),
                   torch.as_tensor(np.asarray(pool.cap, dtype=np.int64)).to(device),
                   torch.as_tensor(np.asarray(pool.count, dtype=np.int64)).to(device))

    def to_host(self):
        """numpy copy with the attributes of gen.Pool (id as uint64)."""
        from types import SimpleNamespace
        return SimpleNamespace(
            x=self.x.cpu().numpy(), v=self.v.cpu().numpy(), tau=self.tau.cpu().numpy(),
            id=self.id.cpu().numpy().view(np.uint64), base=self.base.cpu().numpy(),
            cap=self.cap.cpu().numpy(), count=self.count.cpu().numpy())

    def particles(self):
        return _Particles(self.nseg, self.vdtype, _p(self.base), _p(self.cap), _p(self.count),
                          _rows(self.x), _rows(self.v), _p(self.tau), _p(self.id))

    def sendbufs(self):
        return _Send(_p(self.base), _p(self.cap), _p(self.count),
                     _rows(self.x), _rows(self.v), _p(self.tau), _p(self.id))

    def extent(self):
        return int((self.base + self.cap).max().item()) if self.nseg else 0


class DeviceStagePool(DevicePool):
    """Mid-step records of per-stage migration on the device: the pool's
    arrays plus xs (X*, float64), vs (V*) and a (dV/dt), like v."""

    def __init__(self, x, v, xs, vs, a, tau, ids, base, cap, count):
        super().__init__(x, v, tau, ids, base, cap, count)
        self.xs, self.vs, self.a = xs, vs, a
        if xs.shape != x.shape or xs.dtype != torch.float64 or not xs.is_contiguous():
            raise PMError("xs must be a contiguous float64 (3, size) tensor")
        for t in (vs, a):
            if t.shape != v.shape or t.dtype != v.dtype or not t.is_contiguous():
                raise PMError("vs and a must match v")

    @classmethod
    def empty(cls, base, cap, vdtype=torch.float64, device="cuda", size=None):
        p = DevicePool.empty(base, cap, vdtype=vdtype, device=device, size=size)
        return cls(p.x, p.v, torch.zeros_like(p.x), torch.zeros_like(p.v),
                   torch.zeros_like(p.v), p.tau, p.id, p.base, p.cap, p.count)

    def to_host(self):
        h = super().to_host()
        h.xs, h.vs, h.a = self.xs.cpu().numpy(), self.vs.cpu().numpy(), self.a.cpu().numpy()
        return h

    def _arr(self, t):
        return _rows(t)

    def stage_particles(self):
        return _StageParticles(self.nseg, self.vdtype, _p(self.base), _p(self.cap),
                               _p(self.count), self._arr(self.x), self._arr(self.v),
                               self._arr(self.xs), self._arr(self.vs), self._arr(self.a),
                               _p(self.tau), _p(self.id))

    def stage_sendbufs(self):
        return _StageSend(_p(self.base), _p(self.cap), _p(self.count), self._arr(self.x),
                          self._arr(self.v), self._arr(self.xs), self._arr(self.vs),
                          self._arr(self.a), _p(self.tau), _p(self.id))


@dataclass
class Params:
    """pm_params: time step, gravity, drag law ("stokes" or "nonlinear") and,
    for the nonlinear law, nu and rho_p/rho."""
    dt: float
    g: tuple = (0.0, 0.0, 0.0)
    drag: str = "stokes"
    nu: float = 1.5e-5
    density_ratio: float = 843.0

    @property
    def c(self):
        return _Params(float(self.dt), (C.c_double * 3)(*[float(x) for x in self.g]),
                       DRAG[self.drag], 0, float(self.nu), float(self.density_ratio))


def workspace_bytes(pool_extent, send_extent, nsub):
    return int(lib().pm_workspace_bytes(int(pool_extent), int(send_extent), int(nsub)))


class Context:
    """A pm_ctx with its device workspace (owned by this object)."""

    def __init__(self, pool_extent, send_extent, nsub, device="cuda"):
        self.pool_extent = int(pool_extent)
        self.send_extent = int(send_extent)
        self.nsub = int(nsub)
        nb = workspace_bytes(self.pool_extent, self.send_extent, self.nsub)
        self.workspace = torch.empty(nb, dtype=torch.uint8, device=device)
        h = C.c_void_p()
        _check(lib().pm_create(C.byref(h), _p(self.workspace), nb, self.pool_extent,
                               self.send_extent, self.nsub))
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().pm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- checks of tensor sizes against the extents the context was made for
    def _pool(self, pool, what):
        # the kernels check base+cap <= pool_extent on the device; the arrays
        # must therefore hold pool_extent records
        if pool.size < self.pool_extent:
            raise PMError(f"{what}: arrays ({pool.size}) shorter than the context's pool "
                          f"extent ({self.pool_extent})")
        if pool.nseg > self.nsub:
            raise PMError(f"{what}: {pool.nseg} segments exceed the context's {self.nsub}")
        return pool.particles()

    def _send(self, send, nsub):
        if send.nseg != nsub * 27:
            raise PMError("send buffers need nsub*27 segments")
        if send.size < self.send_extent:
            raise PMError("send arrays shorter than the context's send extent")
        return send.sendbufs()

    # -- entry points
    def interp(self, field: DeviceField, X: torch.Tensor, stream=None):
        n = X.shape[1]
        X = X.contiguous()
        dt = torch.float32 if field.mixed else torch.float64
        U = torch.empty((3, n), dtype=dt, device=X.device)
        _check(lib().pm_interp(self.h, C.byref(field.c), n, _p(X[0]), _p(X[1]), _p(X[2]),
                               _p(U[0]), _p(U[1]), _p(U[2]), _stream(stream)))
        return U

    def interp_advance(self, field, pool, params, sub_first=0, sub_count=None, stream=None):
        pc = self._pool(pool, "inout")
        sub_count = pool.nseg - sub_first if sub_count is None else sub_count
        _check(lib().pm_interp_advance(self.h, C.byref(field.c), C.byref(pc),
                                       C.byref(params.c), sub_first, sub_count,
                                       _stream(stream)))

    def classify_scan_pack(self, decomp, pin, send, sub_first=0, sub_count=None, stream=None):
        pc = self._pool(pin, "in")
        sc = self._send(send, pin.nseg)
        sub_count = pin.nseg - sub_first if sub_count is None else sub_count
        _check(lib().pm_classify_scan_pack(self.h, C.byref(decomp.c), C.byref(pc),
                                           C.byref(sc), sub_first, sub_count,
                                           _stream(stream)))

    def compact_append(self, decomp, pin, send, pout, sub_first=0, sub_count=None,
                       stream=None):
        pc = self._pool(pin, "in")
        oc = self._pool(pout, "out")
        sc = self._send(send, pin.nseg)
        sub_count = pin.nseg - sub_first if sub_count is None else sub_count
        _check(lib().pm_compact_append(self.h, C.byref(decomp.c), C.byref(pc), C.byref(sc),
                                       C.byref(oc), sub_first, sub_count, _stream(stream)))

    def step(self, field, decomp, pin, pout, send, params, stream=None):
        pc = self._pool(pin, "in")
        oc = self._pool(pout, "out")
        sc = self._send(send, pin.nseg)
        _check(lib().pm_step(self.h, C.byref(field.c), C.byref(decomp.c), C.byref(pc),
                             C.byref(oc), C.byref(sc), C.byref(params.c), _stream(stream)))

    def step_staged(self, field, decomp, pin, mid, mid_send, pout, send, params, stream=None):
        """Migration after each RK2 stage: pin -> mid (DeviceStagePool, leavers
        through mid_send) -> pout (leavers through send)."""
        pc = self._pool(pin, "in")
        oc = self._pool(pout, "out")
        sc = self._send(send, pin.nseg)
        self._pool(mid, "mid")
        self._send(mid_send, pin.nseg)
        mc, msc = mid.stage_particles(), mid_send.stage_sendbufs()
        _check(lib().pm_step_staged(self.h, C.byref(field.c), C.byref(decomp.c), C.byref(pc),
                                    C.byref(mc), C.byref(msc), C.byref(oc), C.byref(sc),
                                    C.byref(params.c), _stream(stream)))

    def get_status(self, stream=None):
        f = C.c_uint32(0)
        _check(lib().pm_get_status(self.h, _stream(stream), C.byref(f)))
        return int(f.value)

    def set_tuning(self, wg, items, blocks_per_cu=0, xcd_block=0):
        t = _Tuning(wg, items, blocks_per_cu, xcd_block)
        _check(lib().pm_set_tuning(self.h, C.byref(t)))

    def get_tuning(self):
        t = _Tuning()
        _check(lib().pm_get_tuning(self.h, C.byref(t)))
        return (t.wg, t.items, t.blocks_per_cu, t.xcd_block)

    def autotune(self, field, decomp, pin, pout, send, params, cache_path=None, stream=None):
        pc = self._pool(pin, "in")
        oc = self._pool(pout, "out")
        sc = self._send(send, pin.nseg)
        _check(lib().pm_autotune(self.h, C.byref(field.c), C.byref(decomp.c), C.byref(pc),
                                 C.byref(oc), C.byref(sc), C.byref(params.c),
                                 _stream(stream),
                                 cache_path.encode() if cache_path else None))
        return self.get_tuning()

    def set_graph(self, enable=True):
        _check(lib().pm_set_graph(self.h, 1 if enable else 0))

    def set_timing(self, max_records):
        _check(lib().pm_set_timing(self.h, int(max_records)))

    def kernel_times(self, max_ms=4096):
        n = C.c_int32(0)
        tot = C.c_double(0.0)
        ms = (C.c_float * max_ms)()
        _check(lib().pm_kernel_times(self.h, C.byref(n), C.byref(tot), ms, max_ms))
        return tot.value, list(ms[:min(n.value, max_ms)])

    def sort(self, field, pin, pout, stream=None):
        """Cell re-sort of every segment of pin into pout (pm_sort); the
        sort's workspace is allocated on first use and kept."""
        pc = self._pool(pin, "in")
        oc = self._pool(pout, "out")
        nb = int(lib().pm_sort_workspace_bytes(self.pool_extent, pin.nseg))
        if nb == 0:
            raise PMError("no re-sort for this pool extent")
        ws = getattr(self, "sort_workspace", None)
        if ws is None or ws.numel() < nb:
            ws = torch.empty(nb, dtype=torch.uint8, device=pin.x.device)
            self.sort_workspace = ws
        _check(lib().pm_sort(self.h, C.byref(field.c), C.byref(pc), C.byref(oc), _p(ws),
                             ws.numel(), _stream(stream)))

    def touched_nodes(self, field, pin, params, stream=None):
        pc = self._pool(pin, "in")
        nodes = (field.n[0] + 2 * field.halo) * (field.n[1] + 2 * field.halo) * \
            (field.n[2] + 2 * field.halo) * (3 if field.stagger else 1)
        words = (nodes + 63) // 64
        bm = torch.empty(words, dtype=torch.int64, device=field.u[0].device)
        out = C.c_int64(0)
        _check(lib().pm_touched_nodes(self.h, C.byref(field.c), C.byref(pc),
                                      C.byref(params.c), _p(bm), words * 64,
                                      _stream(stream), C.byref(out)))
        return int(out.value)


NOALLOC_SCRATCH_BYTES = 64 << 20


def step_noalloc(field, decomp, pin, pout, send, params, flags, stream=None):
    """pm_step_noalloc: the fused step with the library's fixed device scratch
    instead of a context and workspace.  flags: a device int32 tensor of one
    element that receives the step's flag bits."""
    if flags.dtype != torch.int32 or flags.numel() != 1 or not flags.is_cuda:
        raise PMError("flags must be a device int32 tensor of one element")
    pc, oc, sc = pin.particles(), pout.particles(), send.sendbufs()
    _check(lib().pm_step_noalloc(C.byref(field.c), C.byref(decomp.c), C.byref(pc),
                                 C.byref(oc), C.byref(sc), C.byref(params.c),
                                 min(pin.size, pout.size), send.size, _p(flags),
                                 _stream(stream)))


def interleave_field(field, out=None, dtype=None, stream=None):
    """pm_field_interleave: the same field stored node-interleaved, written by
    the library into `out` (a contiguous device tensor of 3 x (stored nodes)
    values) or, if None, a new one; dtype torch.float32 rounds a float64 field
    (default: the field's own dtype)."""
    nodes = field.u[0].numel()
    dtype = field.u[0].dtype if dtype is None else dtype
    if dtype not in (torch.float64, torch.float32):
        raise PMError("dtype must be torch.float64 or torch.float32")
    if out is None:
        out = torch.empty((nodes, 3), dtype=dtype, device=field.u[0].device)
    elif out.numel() != 3 * nodes or out.dtype != dtype or not out.is_contiguous():
        raise PMError("out must be a contiguous tensor of 3 values per stored node of the "
                      "requested dtype")
    _check(lib().pm_field_interleave(C.byref(field.c), F64 if dtype == torch.float64 else F32,
                                     _p(out), _stream(stream)))
    return DeviceField(out, field.n, field.halo, field.L, device=out.device, interleaved=True)


def flag_names(f):
    return [name for bit, name in FLAG_NAMES.items() if f & bit]
