"""Plain FP64 CPU oracle for the DG Poisson hot path (test infrastructure only).

This package is the correctness reference for the GPU library.  It is slow,
unblocked and written to be checked against the paper by eye.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import it;
the product path (the HIP library and its Python binding) never does, and the
two share no code.

Contents (paper: Pan & Lindsey, "Fast adaptive discontinuous basis sets for
electronic structure"):

* ``nodes``     -- Gauss-Lobatto / Gauss-Legendre nodes, weights, derivative and
                   interpolation matrices (the nodal grid of Sec. 6.2).
* ``sipdg``     -- the symmetric interior-penalty Laplacian of eq. (sip_bilinear)
                   with the penalty of eq. (pen_poly), on a uniform hexahedral
                   auxiliary mesh, as a Kronecker sum (Sec. 3.4-3.5), with
                   Dirichlet data imposed weakly (Sec. 6.3); right-hand side
                   4*pi*rho sampled at the nodes (Sec. 6.1).  Node family GLL
                   (the library's default) or GL (the nodes Sec. 6.2 names: no
                   node on a face, exact diagonal mass); ``face_points`` gives
                   where Dirichlet data are sampled.
* ``assemble``  -- an independent element-by-element assembly of the same
                   bilinear form from 3D volume and face quadrature, used to pin
                   the Kronecker-sum construction on tiny meshes.
* ``fdm``       -- exact solve of the discrete system by fast diagonalisation.
* ``mg``        -- hp-multigrid hierarchy (Sec. 6.4): degree coarsening down to
                   1, then geometric coarsening; Chebyshev-Jacobi smoothing;
                   symmetric V-cycle.
* ``pcg``       -- V-cycle preconditioned conjugate gradients (Sec. 6.4).
* ``exchange``  -- pair densities, exchange potentials W_k and pair energies
                   K_ij (Sec. 6.1, eq. fock_poisson).
* ``boundary``  -- Dirichlet data by quadrature of the source over the grid
                   (Sec. 6.3): g(r) = sum_q W_q f(x_q)/|r - x_q| at the face points.
* ``consumers`` -- the Hartree and exchange actions projected on a basis by the
                   grid's quadrature (Sec. 6.1) and the adaptively compressed
                   exchange built from the exchange action on the occupied
                   orbitals (Sec. 7.2).
* ``layout``    -- conversion between the element-major storage order of the
                   library and the global tensor order used here.

Every function with no independent pin is marked "parity unpinned" in its
docstring; at present there is none.
"""
