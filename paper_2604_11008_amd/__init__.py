"""MI355X-native Lagrangian particle step (LCS.jl, arXiv 2604.11008).

Per step, for every particle: trilinear interpolation of a gridded fluid
velocity, a two-stage second-order Runge-Kutta advance under Stokes drag,
classification against the 26 neighbouring subdomains, and a prefix-scan
migration that packs the leavers into per-direction buffers, compacts the
stayers and appends what each subdomain receives.

The work runs in hand-written HIP kernels for gfx950 behind a C ABI
(``libpm.so``, declared in ``include/pm.h``); ``paper_2604_11008_amd.pm``
marshals torch tensors into those calls.  The library is loaded on first use
and a missing or unbuilt library is an error, never a fallback.
"""
__all__ = ["gen", "pm"]
