"""Seeded synthetic inputs for the particle step.

This module only draws inputs: a divergence-free random-Fourier-mode velocity
field, particle positions, relaxation times and ids, their initial owners and
a pool layout.  It performs none of the step's arithmetic (no interpolation,
drag, boundary classification, scan or packing), so the GPU path and the CPU
oracle can both be fed from it without sharing any of the method.

The paper's turbulence fields and particle data are not available; these
seeded stand-ins have the shapes, sizes and statistics of its workloads
(a periodic cube of side 2*pi, Sect. 2.1; particle counts of the order of the
grid count, Sect. 3.2.4).

Seeds: ``numpy.random.SeedSequence(260411008 + index)`` spawned into four
children (field, positions, tau, shuffle), each driving a PCG64 generator.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field as dc_field

import numpy as np

TWO_PI = 2.0 * math.pi
STAY = 13

# Workload recipes.  "dt": a number, or "rule" = 0.5 cell / (max|u| + tau_max |g|).
CONFIGS = {
    "C1": dict(index=0, n=64, halo=0, k0=4, kmax=8, np=65536, dist="uniform",
               tau=("uniform", 0.05, 0.5), g=(0.0, 0.0, 0.0), dt=0.01,
               p=(2, 2, 2), steps=10, mode="f64"),
    "C2": dict(index=1, n=256, halo=1, k0=8, kmax=32, np=4194304, dist="uniform",
               tau=("loguniform", 0.01, 1.0), g=(0.0, 0.0, -1.0), dt="rule",
               p=(1, 1, 1), steps=100, mode="f64"),
    "C3": dict(index=2, n=512, halo=0, k0=16, kmax=64, np=1 << 26, dist="blobs",
               tau=("loguniform", 0.01, 1.0), g=(0.0, 0.0, 0.0), dt="rule",
               p=(4, 4, 4), steps=50, mode="f64"),
    "C4": dict(index=3, n=512, halo=0, k0=16, kmax=64, np=None, dist="lognormal",
               tau=("loguniform", 0.01, 1.0), g=(0.0, 0.0, 0.0), dt="rule",
               p=(8, 8, 8), steps=20, mode="f64"),
    "C5": dict(index=4, n=1024, halo=0, k0=32, kmax=128, np=1 << 28, dist="blobs",
               tau=("loguniform", 0.01, 1.0), g=(0.0, 0.0, 0.0), dt="rule",
               p=(8, 8, 8), steps=20, mode="mixed"),
    # the 256^3 field made periodic and cut into 8x8x8 subdomains, with a
    # step of half a cell at the rms speed: a few percent migrate per step
    "C2S": dict(index=5, n=256, halo=0, k0=8, kmax=32, np=4194304, dist="uniform",
                tau=("loguniform", 0.01, 1.0), g=(0.0, 0.0, -1.0), dt="rms",
                p=(8, 8, 8), steps=20, mode="f64"),
    # the paper's per-rank share of its particle-communication measurement
    # (Sect. 3.2.2: a 1500^3 grid and 750^3 particles over 8 GPUs): a 750^3
    # field with a one-cell halo and 750^3 / 8 uniform particles in one
    # subdomain (26 periodic self-neighbours)
    "CP": dict(index=6, n=750, halo=1, k0=16, kmax=64, np=52734375, dist="uniform",
               tau=("loguniform", 0.01, 1.0), g=(0.0, 0.0, -1.0), dt="rule",
               p=(1, 1, 1), steps=20, mode="f64"),
}


def seeds(index: int):
    """Four independent child seeds (field, positions, tau, shuffle)."""
    return np.random.SeedSequence(260411008 + index).spawn(4)


def rng(seed) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ----------------------------------------------------------------------------
# velocity field
# ----------------------------------------------------------------------------

def model_spectrum(k, k0):
    """E(k) proportional to k^4 exp(-2 (k/k0)^2)."""
    k = np.asarray(k, dtype=np.float64)
    return k ** 4 * np.exp(-2.0 * (k / k0) ** 2)


def spectral_modes(k0: float, kmax: int, seed):
    """Wavevectors (m,3) of one half-space and their complex amplitudes (m,3).

    Every mode 0 < |k| <= kmax gets a random direction perpendicular to k and a
    random phase, with |u_hat|^2 = 2 E(|k|) / (4 pi |k|^2); the other half
    space holds the complex conjugates, so the field is real and k . u_hat = 0.
    """
    g = rng(seed)
    kk = np.arange(-kmax, kmax + 1)
    kz, ky, kx = np.meshgrid(kk, kk, kk, indexing="ij")
    k2 = kx * kx + ky * ky + kz * kz
    half = (k2 > 0) & (k2 <= kmax * kmax) & (
        (kz > 0) | ((kz == 0) & (ky > 0)) | ((kz == 0) & (ky == 0) & (kx > 0)))
    kv = np.stack([kx[half], ky[half], kz[half]], axis=1).astype(np.float64)
    del kx, ky, kz, k2, half
    kn = np.sqrt((kv * kv).sum(axis=1))
    unit = kv / kn[:, None]
    a = g.standard_normal(kv.shape)
    b = g.standard_normal(kv.shape)
    a -= (a * unit).sum(axis=1)[:, None] * unit
    b -= (b * unit).sum(axis=1)[:, None] * unit
    e = a + 1j * b
    e /= np.sqrt((np.abs(e) ** 2).sum(axis=1))[:, None]
    amp = np.sqrt(2.0 * model_spectrum(kn, k0) / (4.0 * math.pi * kn * kn))
    return kv.astype(np.int64), e * amp[:, None]


def _dense_spectrum(n, kv, uh, comp):
    """N^3 array with the mode amplitudes of one component, shifted by half a
    cell so that the inverse transform lands on cell centres."""
    spec = np.zeros((n, n, n), dtype=np.complex128)
    phase = np.exp(1j * math.pi * kv.sum(axis=1) / n)
    val = uh[:, comp] * phase
    iz, iy, ix = kv[:, 2] % n, kv[:, 1] % n, kv[:, 0] % n
    spec[iz, iy, ix] = val
    spec[(-kv[:, 2]) % n, (-kv[:, 1]) % n, (-kv[:, 0]) % n] = np.conj(val)
    return spec


def spectral_field(n: int, k0: float, kmax: int, seed, backend: str = "numpy"):
    """Three float64 arrays of shape (n,n,n), indexed [k][j][i] (x fastest),
    holding the velocity at cell centres, scaled so that the rms of one
    component, sqrt(<|u|^2>/3), is 1.  A single scale keeps div u = 0."""
    if kmax > n // 2 - 1:
        raise ValueError("kmax must stay below the Nyquist wavenumber")
    kv, uh = spectral_modes(k0, kmax, seed)
    comps = []
    for c in range(3):
        spec = _dense_spectrum(n, kv, uh, c)
        if backend == "torch":
            import torch
            t = torch.from_numpy(spec).cuda()
            del spec
            u = torch.fft.ifftn(t).real.mul_(float(n) ** 3).cpu().numpy()
            del t
        else:
            u = np.fft.ifftn(spec).real * float(n) ** 3
            del spec
        comps.append(np.ascontiguousarray(u))
    ms = sum(float(np.mean(u * u)) for u in comps) / 3.0
    scale = 1.0 / math.sqrt(ms)
    return [u * scale for u in comps]


def spectral_field_device(n: int, k0: float, kmax: int, seed, device="cuda"):
    """spectral_field computed with torch on a device: the same modes and
    phases, the inverse transform and scaling done there.  Returns three
    float64 device tensors (n,n,n)."""
    import torch
    if kmax > n // 2 - 1:
        raise ValueError("kmax must stay below the Nyquist wavenumber")
    kv, uh = spectral_modes(k0, kmax, seed)
    phase = np.exp(1j * math.pi * kv.sum(axis=1) / n)
    iz = torch.from_numpy(np.concatenate([kv[:, 2] % n, (-kv[:, 2]) % n])).to(device)
    iy = torch.from_numpy(np.concatenate([kv[:, 1] % n, (-kv[:, 1]) % n])).to(device)
    ix = torch.from_numpy(np.concatenate([kv[:, 0] % n, (-kv[:, 0]) % n])).to(device)
    comps = []
    for c in range(3):
        val = uh[:, c] * phase
        vals = torch.from_numpy(np.concatenate([val, np.conj(val)])).to(device)
        spec = torch.zeros((n, n, n), dtype=torch.complex128, device=device)
        spec[iz, iy, ix] = vals
        u = torch.fft.ifftn(spec).real.mul_(float(n) ** 3).contiguous()
        del spec
        comps.append(u)
    ms = sum(float((u * u).mean()) for u in comps) / 3.0
    scale = 1.0 / math.sqrt(ms)
    return [u.mul_(scale) for u in comps]


def with_halo(u: np.ndarray) -> np.ndarray:
    """Periodic copy of one cell on each side: (n+2)^3."""
    return np.pad(u, 1, mode="wrap")


def shell_spectrum(comps, kmax_out=None):
    """Energy spectrum estimator of Sect. 3.1.1: E(k) = 1/2 sum'_k |u_hat|^2,
    sum'_k = (4 pi k^2 / N_k) * sum over k-1/2 <= |k| < k+1/2, N_k the number of
    wavevectors in the shell.  u_hat is the normalised discrete transform."""
    n = comps[0].shape[0]
    f = np.fft.fftfreq(n, d=1.0 / n)
    kz, ky, kx = np.meshgrid(f, f, f, indexing="ij")
    kn = np.sqrt(kx * kx + ky * ky + kz * kz)
    e = np.zeros_like(kn)
    for u in comps:
        uh = np.fft.fftn(u) / float(n) ** 3
        e += np.abs(uh) ** 2
    kmax_out = kmax_out or n // 2
    out = np.zeros(kmax_out + 1)
    for k in range(1, kmax_out + 1):
        shell = (kn >= k - 0.5) & (kn < k + 0.5)
        nk = int(shell.sum())
        if nk:
            out[k] = 0.5 * (4.0 * math.pi * k * k / nk) * e[shell].sum()
    return out


# ----------------------------------------------------------------------------
# decomposition and particles
# ----------------------------------------------------------------------------

def bounds(p, L=TWO_PI):
    """Per axis p[a]+1 bounds a*(L/P), with the last exactly L."""
    out = []
    for P in p:
        b = np.array([a * (L / P) for a in range(P + 1)], dtype=np.float64)
        b[-1] = L
        out.append(b)
    return out


def pred(L=TWO_PI):
    return float(np.nextafter(L, 0.0))


def into_box(x, L=TWO_PI):
    """Periodic image in [0, L)."""
    x = np.mod(x, L)
    x[x >= L] = pred(L)
    return x


def owner(pos, bnds, p):
    """Initial owner subdomain of each position (half-open intervals)."""
    idx = []
    for a in range(3):
        i = np.searchsorted(bnds[a], pos[a], side="right") - 1
        idx.append(np.clip(i, 0, p[a] - 1))
    return idx[0] + p[0] * (idx[1] + p[1] * idx[2])


def draw_tau(g, n, spec):
    kind, lo, hi = spec
    if kind == "uniform":
        return g.uniform(lo, hi, n)
    if kind == "loguniform":
        return np.exp(g.uniform(math.log(lo), math.log(hi), n))
    raise ValueError(kind)


def uniform_positions(g, n, L=TWO_PI):
    return np.stack([into_box(g.uniform(0.0, L, n), L) for _ in range(3)])


def blob_positions(g, n, ncells, nblobs=4096, sigma_cells=2.0, background=0.3,
                   L=TWO_PI):
    """70% of the particles around 4096 Gaussian blobs (sigma 2 cells), 30%
    uniform, wrapped into the box."""
    centres = g.uniform(0.0, L, (3, nblobs))
    nb = int(round(n * (1.0 - background)))
    pick = g.integers(0, nblobs, nb)
    sig = sigma_cells * L / ncells
    pb = centres[:, pick] + sig * g.standard_normal((3, nb))
    pu = g.uniform(0.0, L, (3, n - nb))
    pos = np.concatenate([pb, pu], axis=1)
    return np.stack([into_box(pos[a], L) for a in range(3)])


def lognormal_positions(g, p, bnds, median=1e5, sigma=1.0):
    """Per-subdomain counts round(exp(ln median + sigma z)), positions uniform
    inside each subdomain."""
    nsub = p[0] * p[1] * p[2]
    z = g.standard_normal(nsub)
    counts = np.rint(np.exp(math.log(median) + sigma * z)).astype(np.int64)
    parts = []
    for s in range(nsub):
        sx, sy, sz = s % p[0], (s // p[0]) % p[1], s // (p[0] * p[1])
        c = int(counts[s])
        blk = []
        for a, k in enumerate((sx, sy, sz)):
            lo, hi = bnds[a][k], bnds[a][k + 1]
            x = g.uniform(lo, hi, c)
            x[x >= hi] = np.nextafter(hi, lo)
            blk.append(x)
        parts.append(np.stack(blk))
    return np.concatenate(parts, axis=1)


@dataclass
class Pool:
    """Structure-of-arrays particle records in per-segment slices."""
    x: np.ndarray            # (3, size) float64
    v: np.ndarray            # (3, size) float64 or float32
    tau: np.ndarray          # (size,)  float64 or float32
    id: np.ndarray           # (size,)  uint64
    base: np.ndarray         # (nseg,) int64
    cap: np.ndarray          # (nseg,) int64
    count: np.ndarray        # (nseg,) int64

    @property
    def size(self):
        return self.x.shape[1]

    def segment(self, q):
        b, c = int(self.base[q]), int(self.count[q])
        return slice(b, b + c)


def empty_pool(base, cap, vdtype=np.float64):
    base = np.asarray(base, dtype=np.int64)
    cap = np.asarray(cap, dtype=np.int64)
    size = int((base + cap).max()) if len(base) else 0
    return Pool(x=np.zeros((3, size)), v=np.zeros((3, size), dtype=vdtype),
                tau=np.zeros(size, dtype=vdtype), id=np.zeros(size, dtype=np.uint64),
                base=base, cap=cap, count=np.zeros(len(base), dtype=np.int64))


@dataclass
class StagePool:
    """Mid-step records of per-stage migration: X_n, V_n, X*, V*, the stage-1
    acceleration a, tau and id (structure of arrays, per-segment slices)."""
    x: np.ndarray            # (3, size) float64
    v: np.ndarray            # (3, size) float64 or float32
    xs: np.ndarray           # (3, size) float64
    vs: np.ndarray           # (3, size) like v
    a: np.ndarray            # (3, size) like v
    tau: np.ndarray
    id: np.ndarray
    base: np.ndarray
    cap: np.ndarray
    count: np.ndarray

    @property
    def size(self):
        return self.x.shape[1]

    def segment(self, q):
        b, c = int(self.base[q]), int(self.count[q])
        return slice(b, b + c)


def empty_stage_pool(base, cap, vdtype=np.float64):
    base = np.asarray(base, dtype=np.int64)
    cap = np.asarray(cap, dtype=np.int64)
    size = max(int((base + cap).max()) if len(base) else 0, 1)
    z = lambda dt: np.zeros((3, size), dtype=dt)  # noqa: E731
    return StagePool(x=z(np.float64), v=z(vdtype), xs=z(np.float64), vs=z(vdtype),
                     a=z(vdtype), tau=np.zeros(size, dtype=vdtype),
                     id=np.zeros(size, dtype=np.uint64), base=base, cap=cap,
                     count=np.zeros(len(base), dtype=np.int64))


def neighbour_max(counts, p):
    """Largest count among the 26 periodic neighbours of every subdomain."""
    c = np.asarray(counts).reshape(p[2], p[1], p[0])
    m = np.zeros_like(c)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if dx or dy or dz:
                    m = np.maximum(m, np.roll(c, (dz, dy, dx), axis=(0, 1, 2)))
    return m.reshape(-1)


def layout(counts, slack=0.05, extra=1024, align=64, p=None, inflow=0.05):
    """Segment bases and capacities with room for growth, in subdomain order.
    With the decomposition p, a segment also gets room for `inflow` times its
    most populated neighbour (uneven counts make particles flow into the
    sparse subdomains)."""
    counts = np.asarray(counts, dtype=np.int64)
    grow = counts * (1.0 + slack)
    if p is not None and int(np.prod(p)) > 1:
        grow = grow + inflow * neighbour_max(counts, p)
    cap = (grow.astype(np.int64) + extra + align - 1) // align * align
    base = np.zeros_like(cap)
    base[1:] = np.cumsum(cap)[:-1]
    return base, cap


def send_layout(counts, face=0.02, edge=0.002, corner=0.0005, extra=256):
    """Send-buffer segments s*27+d sized by the kind of neighbour."""
    counts = np.asarray(counts, dtype=np.int64)
    nsub = len(counts)
    cap = np.zeros(nsub * 27, dtype=np.int64)
    for d in range(27):
        if d == STAY:
            continue
        o = (d % 3 - 1, (d // 3) % 3 - 1, d // 9 - 1)
        kind = sum(1 for c in o if c != 0)
        frac = {1: face, 2: edge, 3: corner}[kind]
        cap[d::27] = (counts * frac).astype(np.int64) + extra
    base = np.zeros_like(cap)
    base[1:] = np.cumsum(cap)[:-1]
    return base, cap


def _int64(a):
    """int64 view of an index array: numpy arrays and scalars, or torch
    tensors (kept on their device)."""
    if hasattr(a, "device") and hasattr(a, "dtype") and not isinstance(a, np.ndarray):
        import torch
        return a.to(torch.int64)
    return np.asarray(a, dtype=np.int64)


def morton3(i, j, k, bits=11):
    """Z-order code of cell (i, j, k): bits of i, j, k interleaved, i lowest.
    Works on numpy arrays and on torch int64 tensors alike."""
    i, j, k = _int64(i), _int64(j), _int64(k)
    code = i * 0
    for b in range(bits):
        code |= ((i >> b) & 1) << (3 * b)
        code |= ((j >> b) & 1) << (3 * b + 1)
        code |= ((k >> b) & 1) << (3 * b + 2)
    return code


def cell_key(i, j, k):
    """Sort key of the canonical order: the Z-order code of (i/2, j, k), then
    the parity of i, so that the smallest blocks are two cells long in x,
    the axis along which a stencil's two nodes share memory sectors."""
    i = _int64(i)
    return morton3(i >> 1, j, k) * 2 + (i & 1)


def _order_torch(pos, p, bnds, n, L, order, device):
    """Owners and the stable order of build_pool computed with torch on
    `device` (the same permutation as the numpy lexsort: the keys below
    are unique up to ties, which a stable sort leaves in id order)."""
    import torch
    P = torch.from_numpy(np.ascontiguousarray(pos)).to(device)
    idx = []
    for a in range(3):
        b = torch.from_numpy(np.ascontiguousarray(bnds[a])).to(device)
        idx.append((torch.searchsorted(b, P[a].contiguous(), right=True) - 1)
                   .clamp_(0, p[a] - 1))
    s = idx[0] + p[0] * (idx[1] + p[1] * idx[2])
    del idx
    cell = [torch.floor(P[a] * (n / L)).to(torch.int64).clamp_(0, n - 1) for a in range(3)]
    del P
    bits = max(1, int(n - 1).bit_length())
    if order == "rowmajor":
        key = ((s * n + cell[2]) * n + cell[1]) * n + cell[0]
    elif order == "morton":
        key = (s << (3 * bits)) | morton3(cell[0], cell[1], cell[2])
    else:
        key = (s << (3 * bits + 1)) | cell_key(cell[0], cell[1], cell[2])
    del cell
    perm = torch.sort(key, stable=True).indices
    del key
    return s.cpu().numpy(), perm.cpu().numpy()


def build_pool(pos, tau, ids, p, bnds, n, L=TWO_PI, slack=0.05, extra=1024,
               vdtype=np.float64, order="canonical", shuffle_seed=None, sort_device=None):
    """Pool with each particle in its owner's segment.  Canonical order: by
    subdomain, then cell_key of the cell, then id.  order="morton" uses the
    plain Z-order code of the cell, order="rowmajor" the cell (z, y, x);
    order="shuffled" permutes each segment of the canonical order with the
    shuffle seed.  sort_device: compute owners and the order with torch on
    that device (same result; for pools of 2^26 and more particles), which
    needs ids in drawing order (ids[i] == i)."""
    nsub = p[0] * p[1] * p[2]
    if sort_device is not None:
        if not np.array_equal(ids[:16], np.arange(min(16, len(ids)), dtype=ids.dtype)):
            raise ValueError("sort_device needs ids in drawing order")
        s, perm = _order_torch(pos, p, bnds, n, L,
                               "canonical" if order == "shuffled" else order, sort_device)
    else:
        s = owner(pos, bnds, p)
        cell = [np.clip(np.floor(pos[a] * (n / L)).astype(np.int64), 0, n - 1)
                for a in range(3)]
        if order == "rowmajor":
            perm = np.lexsort((ids, cell[0], cell[1], cell[2], s))
        elif order == "morton":
            perm = np.lexsort((ids, morton3(cell[0], cell[1], cell[2]), s))
        else:
            perm = np.lexsort((ids, cell_key(cell[0], cell[1], cell[2]), s))
        del cell
    s_sorted = s[perm]
    counts = np.bincount(s_sorted, minlength=nsub).astype(np.int64)
    if order == "shuffled":
        g = rng(shuffle_seed)
        start = 0
        for q in range(nsub):
            c = int(counts[q])
            perm[start:start + c] = perm[start:start + c][g.permutation(c)]
            start += c
    base, cap = layout(counts, slack=slack, extra=extra, p=p)
    pool = empty_pool(base, cap, vdtype)
    start = 0
    for q in range(nsub):
        c = int(counts[q])
        sel = perm[start:start + c]
        b = int(base[q])
        pool.x[:, b:b + c] = pos[:, sel]
        pool.tau[b:b + c] = tau[sel].astype(vdtype)
        pool.id[b:b + c] = ids[sel]
        start += c
    pool.count[:] = counts
    return pool


@dataclass
class Workload:
    name: str
    n: int
    halo: int
    L: float
    p: tuple
    bounds: list
    field: list              # three float64 arrays (n,n,n), no halo
    pool: Pool               # positions, tau, id; v left zero
    dt: float
    g: tuple
    mode: str
    steps: int
    info: dict = dc_field(default_factory=dict)

    def stored_field(self, dtype=np.float64):
        """Field arrays as stored on the device (with the halo if any): numpy
        arrays, or device tensors when the field was generated on a device."""
        out = []
        for u in self.field:
            if isinstance(u, np.ndarray):
                a = with_halo(u) if self.halo else u
                out.append(np.ascontiguousarray(a.astype(dtype)).reshape(-1))
            else:
                import torch
                a = u
                if self.halo:
                    a = torch.cat([a[-1:], a, a[:1]], dim=0)
                    a = torch.cat([a[:, -1:], a, a[:, :1]], dim=1)
                    a = torch.cat([a[:, :, -1:], a, a[:, :, :1]], dim=2)
                tdt = torch.float32 if dtype == np.float32 else torch.float64
                out.append(a.to(tdt).contiguous().reshape(-1))
        return out


def dt_rule(field, tau_max, g, n, L=TWO_PI, kind="rule"):
    """Half a cell per step at the largest speed the particles can reach
    (max|u| + tau_max |g|); kind "rms": half a cell at the rms speed."""
    delta = L / n
    gn = math.sqrt(sum(c * c for c in g))
    if kind == "rms":
        return 0.5 * delta
    if isinstance(field[0], np.ndarray):
        umax = math.sqrt(float(np.max(field[0] ** 2 + field[1] ** 2 + field[2] ** 2)))
    else:
        umax = math.sqrt(float((field[0] ** 2 + field[1] ** 2 + field[2] ** 2).max()))
    return 0.5 * delta / (umax + tau_max * gn)


def make_workload(name, np_override=None, n_override=None, p_override=None,
                  order="canonical", field_backend="numpy", slack=0.05,
                  extra=1024, kmax_override=None, k0_override=None, sort_device=None,
                  mode_override=None):
    """Build a named workload (optionally resized for tests).  sort_device:
    order the pool with torch on that device (the same pool, faster for
    large workloads).  mode_override "f64" keeps tau in float64 for a
    workload defined in mixed precision (which rounds the same draws)."""
    cfg = dict(CONFIGS[name])
    n = n_override or cfg["n"]
    p = tuple(p_override or cfg["p"])
    k0 = k0_override or cfg["k0"]
    kmax = kmax_override or min(cfg["kmax"], n // 2 - 1)
    s_field, s_pos, s_tau, s_shuf = seeds(cfg["index"])
    L = TWO_PI
    if field_backend == "device":
        field = spectral_field_device(n, k0, kmax, s_field)
    else:
        field = spectral_field(n, k0, kmax, s_field, backend=field_backend)
    bnds = bounds(p, L)
    gp = rng(s_pos)
    npart = np_override or cfg["np"]
    if cfg["dist"] == "uniform":
        pos = uniform_positions(gp, npart, L)
    elif cfg["dist"] == "blobs":
        pos = blob_positions(gp, npart, n, L=L)
    elif cfg["dist"] == "lognormal":
        pos = lognormal_positions(gp, p, bnds,
                                  median=1e5 if np_override is None else np_override)
    else:
        raise ValueError(cfg["dist"])
    npart = pos.shape[1]
    tau = draw_tau(rng(s_tau), npart, cfg["tau"])
    ids = np.arange(npart, dtype=np.uint64)
    mode = mode_override or cfg["mode"]
    vdtype = np.float32 if mode == "mixed" else np.float64
    pool = build_pool(pos, tau, ids, p, bnds, n, L, slack=slack, extra=extra,
                      vdtype=vdtype, order=order, shuffle_seed=s_shuf,
                      sort_device=sort_device)
    if cfg["dt"] in ("rule", "rms"):
        dt = dt_rule(field, cfg["tau"][2], cfg["g"], n, L, kind=cfg["dt"])
    else:
        dt = float(cfg["dt"])
    return Workload(name=name, n=n, halo=cfg["halo"], L=L, p=p, bounds=bnds,
                    field=field, pool=pool, dt=dt, g=tuple(cfg["g"]),
                    mode=mode, steps=cfg["steps"],
                    info=dict(k0=k0, kmax=kmax, np=npart, dist=cfg["dist"]))
