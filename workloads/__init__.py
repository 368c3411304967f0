"""Seeded synthetic inputs for the DG Poisson hot path.

This package only evaluates closed-form functions (s-type Gaussian orbitals,
Gaussian densities and their full-space Coulomb potentials) at points the
caller supplies.  It contains none of the discretisation or solver arithmetic,
so it can feed both the GPU library and the CPU oracle without coupling them.
"""
