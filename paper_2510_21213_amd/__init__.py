"""MI355X (gfx950) DG Poisson hot path: SIPDG operator, hp-multigrid PCG and
exchange reductions as hand-written HIP kernels behind a C ABI
(include/dg_poisson.h).  ``binding`` is the thin Python layer over it."""
