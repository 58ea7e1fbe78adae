"""Sequential FP64 CPU oracle of the particle step (ctypes over liboracle.so).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may use it; the product path never does.  It shares no code
with the GPU library.  Everything here only marshals numpy arrays into the C
functions of oracle.c, which hold the arithmetic.

Pools are any objects with numpy attributes x (3,size), v (3,size), tau,
id (uint64), base, cap, count (int64), e.g. ``gen.Pool``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("PM_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

SEND_OVERFLOW, DEST_OVERFLOW, SKIP, NONFINITE, HALO = 1, 2, 4, 8, 16
STAY = 13


def build(quiet: bool = True) -> str:
    """Compile oracle.c into liboracle.so (plain gcc, no contraction)."""
    cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
           "-Wall", "-o", LIB_PATH, os.path.join(HERE, "oracle.c"), "-lm"]
    subprocess.run(cmd, check=True, capture_output=quiet)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        src = os.path.join(HERE, "oracle.c")
        if not os.environ.get("PM_ORACLE_LIB") and (not os.path.exists(LIB_PATH)
                or os.path.getmtime(LIB_PATH) < os.path.getmtime(src)):
            build()
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.orc_interp.argtypes = [vp, vp, vp]
        L.orc_interp.restype = C.c_uint
        L.orc_interp_many.argtypes = [vp, C.c_int64, vp, vp, vp, vp, vp, vp]
        L.orc_interp_many.restype = C.c_uint
        L.orc_advance.argtypes = [vp, vp, C.c_int64, vp, vp, vp]
        L.orc_advance.restype = C.c_uint
        L.orc_classify.argtypes = [vp, C.c_int, vp, vp, vp]
        L.orc_classify.restype = C.c_int
        L.orc_partition.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.orc_partition.restype = C.c_uint
        L.orc_append.argtypes = [vp, vp, vp, vp]
        L.orc_append.restype = C.c_uint
        L.orc_step.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.orc_step.restype = C.c_uint
        L.orc_step_staged.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
        L.orc_step_staged.restype = C.c_uint
        _lib = L
    return _lib


# --- C structures (mirroring oracle.h) ---------------------------------------

class _Field(C.Structure):
    _fields_ = [("n", C.c_int * 3), ("halo", C.c_int), ("stagger", C.c_int),
                ("L", C.c_double * 3), ("u", C.c_void_p * 3)]


class _Decomp(C.Structure):
    _fields_ = [("p", C.c_int * 3), ("b", C.c_void_p * 3)]


class _Pool(C.Structure):
    _fields_ = [("nseg", C.c_int), ("base", C.c_void_p), ("cap", C.c_void_p),
                ("count", C.c_void_p), ("x", C.c_void_p * 3), ("v", C.c_void_p * 3),
                ("tau", C.c_void_p), ("id", C.c_void_p)]


class _XPool(C.Structure):
    _fields_ = [("nseg", C.c_int), ("base", C.c_void_p), ("cap", C.c_void_p),
                ("count", C.c_void_p), ("x", C.c_void_p * 3), ("v", C.c_void_p * 3),
                ("xs", C.c_void_p * 3), ("vs", C.c_void_p * 3), ("a", C.c_void_p * 3),
                ("tau", C.c_void_p), ("id", C.c_void_p)]


class _Params(C.Structure):
    _fields_ = [("dt", C.c_double), ("g", C.c_double * 3), ("drag", C.c_int),
                ("nu", C.c_double), ("density_ratio", C.c_double)]


DRAG = {"stokes": 0, "nonlinear": 1}


def _params(dt, g, drag, nu, density_ratio):
    return _Params(float(dt), (C.c_double * 3)(*g), DRAG[drag], float(nu),
                   float(density_ratio))


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


class Field:
    """Velocity field as stored: three flat float64 arrays, (n or n+2)^3;
    stagger=True: MAC arrangement (component c on the faces normal to axis c)."""

    def __init__(self, u, n, halo, L=2.0 * np.pi, stagger=False):
        self.u = [_f64(np.asarray(c).reshape(-1)) for c in u]
        self.n = (n, n, n) if np.isscalar(n) else tuple(n)
        self.halo = int(halo)
        self.stagger = int(bool(stagger))
        self.L = (L, L, L) if np.isscalar(L) else tuple(L)
        st = [k + 2 * self.halo for k in self.n]
        if any(c.size != st[0] * st[1] * st[2] for c in self.u):
            raise ValueError("field size does not match n and halo")
        self._c = _Field((C.c_int * 3)(*self.n), self.halo, self.stagger,
                         (C.c_double * 3)(*self.L),
                         (C.c_void_p * 3)(*[c.ctypes.data for c in self.u]))

    @property
    def ref(self):
        return C.byref(self._c)


class Decomp:
    def __init__(self, p, bnds):
        self.p = tuple(int(k) for k in p)
        self.b = [_f64(b) for b in bnds]
        self._c = _Decomp((C.c_int * 3)(*self.p),
                          (C.c_void_p * 3)(*[b.ctypes.data for b in self.b]))

    @property
    def ref(self):
        return C.byref(self._c)


class _PoolView:
    """float64 copies (when needed) of a pool's arrays, plus the C struct.
    write_back() copies results into the original pool."""

    def __init__(self, pool, nseg=None):
        self.pool = pool
        self.x = _f64(pool.x)
        self.v = _f64(pool.v)
        self.tau = _f64(pool.tau)
        self.id = np.ascontiguousarray(pool.id, dtype=np.uint64)
        self.base = np.ascontiguousarray(pool.base, dtype=np.int64)
        self.cap = np.ascontiguousarray(pool.cap, dtype=np.int64)
        self.count = np.ascontiguousarray(pool.count, dtype=np.int64)
        n = len(self.base) if nseg is None else nseg
        self._c = _Pool(n, self.base.ctypes.data, self.cap.ctypes.data,
                        self.count.ctypes.data,
                        (C.c_void_p * 3)(*[self.x[a].ctypes.data for a in range(3)]),
                        (C.c_void_p * 3)(*[self.v[a].ctypes.data for a in range(3)]),
                        self.tau.ctypes.data, self.id.ctypes.data)

    @property
    def ref(self):
        return C.byref(self._c)

    def write_back(self):
        p = self.pool
        for name in ("x", "v", "tau", "id", "count"):
            dst = getattr(p, name)
            src = getattr(self, name)
            if dst is not src:
                dst[...] = src.astype(dst.dtype)


class _XPoolView:
    """float64 copies of a stage pool's arrays (gen.StagePool), the C struct,
    and write_back() into the original."""

    NAMES = ("x", "v", "xs", "vs", "a")

    def __init__(self, pool):
        self.pool = pool
        for n in self.NAMES:
            setattr(self, n, _f64(getattr(pool, n)))
        self.tau = _f64(pool.tau)
        self.id = np.ascontiguousarray(pool.id, dtype=np.uint64)
        self.base = np.ascontiguousarray(pool.base, dtype=np.int64)
        self.cap = np.ascontiguousarray(pool.cap, dtype=np.int64)
        self.count = np.ascontiguousarray(pool.count, dtype=np.int64)
        arr = lambda n: (C.c_void_p * 3)(*[getattr(self, n)[a].ctypes.data for a in range(3)])  # noqa: E731
        self._c = _XPool(len(self.base), self.base.ctypes.data, self.cap.ctypes.data,
                         self.count.ctypes.data, arr("x"), arr("v"), arr("xs"), arr("vs"),
                         arr("a"), self.tau.ctypes.data, self.id.ctypes.data)

    @property
    def ref(self):
        return C.byref(self._c)

    def write_back(self):
        p = self.pool
        for name in self.NAMES + ("tau", "id", "count"):
            dst = getattr(p, name)
            src = getattr(self, name)
            if dst is not src:
                dst[...] = src.astype(dst.dtype)


# --- the calls -----------------------------------------------------------------

def interp(field: Field, X):
    """U at points X (3,n): returns (U (3,n), flags)."""
    X = _f64(X)
    n = X.shape[1]
    U = np.zeros((3, n))
    flags = lib().orc_interp_many(field.ref, n, _ptr(X[0]), _ptr(X[1]), _ptr(X[2]),
                                  _ptr(U[0]), _ptr(U[1]), _ptr(U[2]))
    return U, int(flags)


def advance(field: Field, x, v, tau, dt, g=(0.0, 0.0, 0.0), drag="stokes", nu=1.5e-5,
            density_ratio=843.0):
    """One Heun step; returns new (x, v, flags), inputs untouched.  drag is
    "stokes" (f = 1) or "nonlinear" (f = 1 + 0.15 Re_p^0.687, with nu and
    rho_p/rho)."""
    x = np.array(x, dtype=np.float64, order="C", copy=True)
    v = np.array(v, dtype=np.float64, order="C", copy=True)
    tau = _f64(tau)
    pr = _params(dt, g, drag, nu, density_ratio)
    xp = (C.c_void_p * 3)(*[x[a].ctypes.data for a in range(3)])
    vp = (C.c_void_p * 3)(*[v[a].ctypes.data for a in range(3)])
    flags = lib().orc_advance(field.ref, C.byref(pr), x.shape[1], xp, vp, _ptr(tau))
    return x, v, int(flags)


def classify(decomp: Decomp, s, X):
    """Direction codes, shifted positions and flags of points X (3,n) owned by s."""
    X = _f64(X)
    n = X.shape[1]
    d = np.zeros(n, dtype=np.int32)
    Xs = np.zeros((3, n))
    flags = C.c_uint(0)
    xi = np.zeros(3)
    xo = np.zeros(3)
    for i in range(n):
        xi[:] = X[:, i]
        d[i] = lib().orc_classify(decomp.ref, int(s), _ptr(xi), _ptr(xo), C.byref(flags))
        Xs[:, i] = xo
    return d, Xs, int(flags.value)


def partition(decomp: Decomp, pin, pout, send, want_slots=False):
    """Sequential partition; fills pout (stayers) and send in place.
    Returns (stay_count, flags[, dir, slot])."""
    vin, vout, vsend = _PoolView(pin), _PoolView(pout), _PoolView(send)
    stay = np.zeros(len(vin.base), dtype=np.int64)
    size = vin.x.shape[1]
    dirs = np.full(size, -1, dtype=np.int32)
    slot = np.full(size, -1, dtype=np.int64)
    flags = lib().orc_partition(decomp.ref, vin.ref, vout.ref, vsend.ref, _ptr(stay),
                                _ptr(dirs), _ptr(slot))
    vout.write_back()
    vsend.write_back()
    if want_slots:
        return stay, int(flags), dirs, slot
    return stay, int(flags)


def append(decomp: Decomp, send, stay_count, pout):
    vsend, vout = _PoolView(send), _PoolView(pout)
    stay = np.ascontiguousarray(stay_count, dtype=np.int64)
    flags = lib().orc_append(decomp.ref, vsend.ref, _ptr(stay), vout.ref)
    vout.write_back()
    return int(flags)


def step(field: Field, decomp: Decomp, dt, g, pin, pout, send, drag="stokes", nu=1.5e-5,
         density_ratio=843.0):
    """Whole step pin -> pout (pin unchanged).  Returns (stay_count, flags)."""
    vin, vout, vsend = _PoolView(pin), _PoolView(pout), _PoolView(send)
    stay = np.zeros(len(vin.base), dtype=np.int64)
    pr = _params(dt, g, drag, nu, density_ratio)
    flags = lib().orc_step(field.ref, decomp.ref, C.byref(pr), vin.ref, vout.ref,
                           vsend.ref, _ptr(stay))
    vout.write_back()
    vsend.write_back()
    return stay, int(flags)


def step_staged(field: Field, decomp: Decomp, dt, g, pin, mid, mid_send, pout, send,
                drag="stokes", nu=1.5e-5, density_ratio=843.0):
    """Whole step with migration after each RK2 stage: pin -> mid (stage-1
    records, leavers through mid_send; gen.StagePool) -> pout (leavers through
    send).  pin is unchanged.  Returns the flags."""
    vin, vout, vsend = _PoolView(pin), _PoolView(pout), _PoolView(send)
    vmid, vms = _XPoolView(mid), _XPoolView(mid_send)
    pr = _params(dt, g, drag, nu, density_ratio)
    flags = lib().orc_step_staged(field.ref, decomp.ref, C.byref(pr), vin.ref, vmid.ref,
                                  vms.ref, vout.ref, vsend.ref)
    for v in (vmid, vms, vout, vsend):
        v.write_back()
    return int(flags)
