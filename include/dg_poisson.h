/*
 * dg_poisson.h -- C ABI of the MI355X DG Poisson library.
 *
 * The library solves the Poisson problems of the auxiliary-grid step of the
 * DG Hartree-Fock method of Pan & Lindsey ("Fast adaptive discontinuous basis
 * sets for electronic structure", Sec. 6):
 *
 *     -Lap v = 4 pi f   in the box Omega,     v = g   on the boundary of Omega
 *
 * (eq. hartree_poisson and eq. fock_poisson, truncated to a finite box with
 * Dirichlet data as in Sec. 6.3), discretised by the symmetric interior
 * penalty method of eq. (sip_bilinear) with the penalty of eq. (pen_poly)
 * (sigma = (p+1)^2 / (eps h), eps = 1/8) on a uniform hexahedral mesh carrying
 * tensor-product Gauss-Lobatto nodal polynomials of degree p.  The nodes also
 * define the quadrature rule (Sec. 6.1): the source f is given by its values
 * at the nodes and the potential v is returned by its values at the nodes.
 * Dirichlet data are imposed weakly (symmetric Nitsche terms).  The discrete
 * system is solved by conjugate gradients preconditioned by an hp-multigrid
 * V-cycle (Sec. 6.4): degree coarsening down to 1, then geometric coarsening.
 *
 * Units are atomic (bohr, hartree).
 *
 * Storage orders
 *   field   one value per node, element-major: [ez][ey][ex][k][j][i]
 *           (elements lexicographic with x fastest; local node index i along x
 *           fastest).  n_dofs = Ex*Ey*Ez*(p+1)^3 values per right-hand side.
 *   faces   Dirichlet data at the boundary nodes: the six faces x-, x+, y-,
 *           y+, z-, z+ concatenated; an x face is [Z][Y] over global node
 *           indices (Y fastest), a y face [Z][X], a z face [Y][X], where the
 *           global node index along an axis is X = ex*(p+1) + i.
 *           n_face = 2*(NY*NZ + NX*NZ + NX*NY) values per right-hand side.
 *   batch   several right-hand sides are packed back to back in the order
 *           given, each at the offset of the sum of the sizes before it.
 *   pairs   for norb orbitals the npairs = norb(norb+1)/2 pairs (i <= j) are
 *           ordered row-major: idx(i,j) = i*norb - i(i-1)/2 + (j - i).
 *
 * Ownership and synchronisation
 *   Every field pointer below is a HIP device pointer owned by the caller
 *   unless marked "host".  The context owns its level tables and work space
 *   (grown on demand, kept until dg_poisson_destroy).  Work is enqueued on
 *   the caller's stream; calls that return statistics synchronise the stream
 *   before they return.  A context is used by one host thread at a time.
 *
 * Errors
 *   Functions return a dg_status; no C++ exception crosses the ABI.
 *   DG_ERR_ARG for bad sizes, indices or null pointers, and from the solves
 *   (dg_poisson_solve_batch, dg_exchange_apply) when a source, its Dirichlet
 *   data or a caller's initial guess holds a NaN or Inf: such a right-hand side
 *   does no iterations, the others are solved, and the outputs of the call are
 *   then not to be used; DG_ERR_HIP when a HIP runtime call fails
 *   (dg_last_error() gives the message);
 *   DG_WARN_NOT_CONVERGED when a right-hand side missed its tolerance within
 *   max_iter (its stats entry says which); DG_ERR_BREAKDOWN when the last FP64
 *   PCG pass of a right-hand side stopped on a non-positive p.Ap or r.z short
 *   of its tolerance (after restarts and, in FP32_IR, the FP64 fallback).
 */
#ifndef DG_POISSON_H
#define DG_POISSON_H

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DG_OK = 0,
    DG_WARN_NOT_CONVERGED = 1,
    DG_ERR_ARG = -1,
    DG_ERR_HIP = -2,
    DG_ERR_OOM = -3,
    DG_ERR_BREAKDOWN = -4,
    DG_ERR_STATE = -5
} dg_status;

/* Arithmetic of the iteration.  FP64: every vector and kernel in double.
 * FP32_IR: FP64 iterative refinement (FP64 right-hand side, solution and
 * residual) around an inner PCG whose vectors, operator applications and
 * smoothing are FP32; dot products, the coarsest-grid solve and all energy
 * reductions stay FP64.
 * FP32_PC: FP64 PCG (FP64 iterate, residual and search direction, FP64
 * operator application of the search direction, FP64 dot products) whose
 * preconditioner, the V-cycle, runs in FP32 (smoothing, transfers and their
 * fields; the coarsest-grid solve in FP64 arithmetic).  The iterate is FP64
 * CG's, so a solve stopped at a residual tolerance has the accuracy of an
 * FP64 solve stopped there, while most bytes moved are the V-cycle's FP32
 * ones.
 * BF16_PC: FP32_PC whose finest-level smoothing steps compute their x and y
 * line contractions on the matrix cores with BF16 operands and FP32
 * accumulation (degree-4 meshes; other degrees run the FP32 kernels).  The
 * preconditioner is then no longer exactly symmetric, so the FP64 CG takes
 * the flexible (Polak-Ribiere) beta.
 * BF16F_PC: FP32_PC whose V-cycle fields on the finest level (its source, the residual handed
 * over by the CG update, and the smoother iterates) and on the finest level's degree-2 step (when
 * that is not the coarsest level) are stored in BF16 (rounded to nearest even), read into FP32
 * arithmetic, and whose search direction p is stored in FP32 (rounded before q = A p is formed
 * from it, so q is the FP64 product of the stored direction).  Iterate, residual, q and every dot
 * stay FP64, so a solve stopped at a residual keeps the FP64 solver's accuracy.  Degree-4 finest
 * levels whose next level is their degree-2 step; other hierarchies run as FP32_PC. */
typedef enum {
    DG_PREC_FP64 = 0,
    DG_PREC_FP32_IR = 1,
    DG_PREC_FP32_PC = 2,
    DG_PREC_BF16_PC = 3,
    DG_PREC_BF16F_PC = 4
} dg_precision;

/* A uniform hexahedral mesh: ne[d] elements along axis d on [lo[d], hi[d]],
 * nodal polynomials of degree p (1 <= p <= 7) on the node family of dg_opts.node_family. */
typedef struct {
    int ne[3];
    int p;
    double lo[3], hi[3];
} dg_mesh;

typedef struct {
    int n_levels;        /* multigrid levels; 0 = automatic (coarsest <= 16 nodes per axis) */
    int cheb_degree;     /* Chebyshev smoothing steps before and after the coarse correction */
    double cheb_ratio;   /* smoothing interval [lam_hi/ratio, lam_hi] */
    double cheb_safety;  /* lam_hi = safety * Lanczos estimate of lambda_max(D^-1 A) */
    int lanczos_steps;   /* Lanczos steps of that estimate */
    double penalty_eps;  /* eps of the penalty sigma = (p+1)^2/(eps h); the paper uses 1/8 */
    double rtol;         /* stop when ||b - A v||_2 <= rtol ||b||_2 (FP64 residual) */
    int max_iter;        /* PCG iterations per right-hand side (inner iterations in FP32_IR) */
    dg_precision precision;
    double inner_rtol;   /* FP32_IR: relative tolerance of each inner solve (loosened for the last
                            step to 0.9 rtol ||b|| / ||r_k|| when that is larger) */
    int max_outer;       /* FP32_IR: refinement steps; a right-hand side still above rtol after
                            them is finished by FP64 PCG from its current iterate */
    int check_every;     /* PCG iterations per replay block (graph: rounded up to even) and
                            between host convergence checks; with a graph the first check
                            waits for as many iterations as the same PCG run of the previous
                            solve on this mesh needed (finished right-hand sides are skipped
                            on the device, so replays past convergence change nothing) */
    int use_graph;       /* 1: replay the PCG iteration as a captured HIP graph */
    int lanes;           /* solver instances per mesh (1 to 4): with more than one, a batch of
                            at least 16 right-hand sides of one mesh is solved as that many
                            consecutive parts (at least 8 right-hand sides each) on as many
                            streams at once, so that the latency-bound coarse-level phases of
                            one part overlap the bandwidth-bound phases of the others */
    int cheb_degree_h;   /* smoothing steps on the degree-1 levels below the finest (the
                            mesh-coarsening part of the hierarchy); 0 = cheb_degree */
    int fused;           /* fused small-mesh solve, FP64 precision only (other precisions ignore it):
                            1: a mesh whose every level has degree at most 4, at most 8,192 nodes
                            and at most 128 nodes per axis is solved by a single launch that runs
                            the whole PCG, one work-group per right-hand side (level fields held
                            in LDS when they fit); 2: group-persistent launch, the same solve
                            with fused_wgs work-groups per right-hand side, persistent for the
                            whole solve, the phases separated by a barrier of the group (no
                            grid-wide barrier; any level size, degree at most 4, coarsest level
                            at most 16 nodes per axis); a group whose barrier gives up waiting
                            (see fused_spin) leaves the call to solve the batch again with the
                            level kernels; 0 (default): the level-by-level kernels */
    int fused_wgs;       /* fused = 2: work-groups per right-hand side, 1..32; 0 = automatic
                            (about four finest-level nodes per thread, at most 16) */
    long long fused_spin; /* fused = 2: polls before a group barrier gives up; 0 = default
                            (2,000,000, about a second); negative: give up at the first poll
                            that finds the group incomplete (tests the fallback) */
    int node_family;     /* nodes of every element, which also define the quadrature (Sec. 6.1,
                            Sec. 6.2): 0 (default) Gauss-Lobatto-Legendre, the end points are
                            nodes and face values are node values; 1 Gauss-Legendre, the family
                            Sec. 6.2 names: no node on a face, face values and derivatives are
                            interpolated, the diagonal mass is exact.  Gauss-Legendre meshes run
                            on the general (brick) operator kernels in every precision (BF16F_PC
                            and BF16_PC then run as FP32_PC), take Dirichlet data from the caller
                            at the face points dg_mesh_coords gives (no quadrature data), no
                            learned guess and no fused solve (DG_ERR_ARG); point-Jacobi smoothing
                            sees less of their operator, so they need more iterations. */
    int learned_cgc;     /* learned coarse-grid correction: the first learned_cgc PCG iterations
                            (rounded up to even) are preconditioned by z = g c + V(r - g A c), where
                            c is the attached guess network's prediction of A^-1 r (the residual
                            given to it as the density r / (4 pi M), its degree-2 output prolonged
                            to the finest level), g = c.r / c.Ac its Galerkin multiple (0 if c.Ac
                            is not positive) and V the V-cycle; those steps restart the direction
                            (beta = 0), the later ones are plain PCG.  FP64 precision, one solver
                            lane, no fused solve (DG_ERR_ARG at set-up otherwise); a solve without
                            an attached network is DG_ERR_ARG.  0 (default): off. */
} dg_opts;

typedef struct {
    int iters;           /* PCG iterations (summed over inner solves in FP32_IR) */
    int outer_iters;     /* refinement steps (FP32_IR), 1 for FP64; one more when the FP64
                            fallback finished the right-hand side (see max_outer) */
    int status;          /* DG_OK, DG_WARN_NOT_CONVERGED, or DG_ERR_BREAKDOWN when the last FP64
                            PCG pass stopped on a non-positive p.Ap or r.z short of the
                            tolerance (after up to three restarts from the current iterate);
                            a solve returns the worst of its right-hand sides' statuses */
    int guess_used;      /* 1 if an initial guess was used: the caller's x0, or a learned guess
                            that passed the guard (residual below ||b||) */
    double rel_residual; /* ||b - A v||_2 / ||b||_2 recomputed in FP64 at exit */
} dg_rhs_stats;

typedef struct dg_ctx dg_ctx;

/* Fill *opts with the defaults: automatic levels, degree 6, ratio 60,
 * safety 1.1, 30 Lanczos steps, eps 1/8, rtol 1e-8, 500 iterations, FP64,
 * inner_rtol 1e-4, max_outer 8, check_every 2, use_graph 1, lanes 2,
 * cheb_degree_h 10, fused 0, fused_wgs 0, fused_spin 0. */
void dg_opts_default(dg_opts* opts);

/* Build the level hierarchy, operator tables, coarsest-grid eigendata and
 * smoother bounds for each of n_meshes meshes (host arrays).  *out receives
 * a new context.  Uses the current HIP device. */
dg_status dg_poisson_setup(const dg_mesh* meshes, int n_meshes, const dg_opts* opts, dg_ctx** out);
void dg_poisson_destroy(dg_ctx* ctx);
const char* dg_status_string(dg_status s);
const char* dg_last_error(void);

/* Sizes of a mesh: DOFs per field and boundary-face values per right-hand
 * side, and the number of multigrid levels built for it (host outputs). */
dg_status dg_mesh_info(const dg_ctx* ctx, int mesh_id, long long* n_dofs, long long* n_face, int* n_levels);

/* Coordinates of the nodes (host output xyz[3][n_dofs], field order) and of
 * the boundary-face nodes (host output fxyz[3][n_face], face order), so that
 * a caller can sample f and g where the library expects them. */
dg_status dg_mesh_coords(const dg_ctx* ctx, int mesh_id, double* xyz, double* fxyz);

/* Solve nrhs Poisson problems.  mesh_id (host [nrhs]) names each problem's
 * mesh.  rho: sources at the nodes (packed fields); g: Dirichlet data (packed
 * face vectors), or NULL: computed from rho by quadrature, as dg_boundary_data
 * does; x0: initial guesses (packed fields) or NULL for zero;
 * v: solutions (packed fields).  stats: host [nrhs] or NULL. */
dg_status dg_poisson_solve_batch(dg_ctx* ctx, int nrhs, const int* mesh_id, const double* rho,
                                 const double* g, const double* x0, double* v,
                                 dg_rhs_stats* stats, hipStream_t stream);

/* Exchange step for norb orbitals phi (packed fields [norb][n_dofs]) on one
 * mesh (Sec. 6.1, eq. fock_poisson): for every pair i <= j the pair density
 * rho_ij = phi_i phi_j is the source of one Poisson problem with Dirichlet
 * data g_pairs (packed face vectors, pair order; NULL: computed from the pair
 * densities by quadrature, as dg_boundary_data does); then
 *   W_k  = sum_s phi_s v_ks        (device [norb][n_dofs], the exchange action
 *                                   on u = phi_k at the nodes, positive sign),
 *   K_ij = sum_nodes w rho_ij v_ij (device [npairs], GLL quadrature),
 *   E_x  = sum_i K_ii + 2 sum_{i<j} K_ij   (host double).
 * v_pairs: device [npairs][n_dofs] receives the pair potentials, or NULL to
 * keep them in context work space.  stats: host [npairs] or NULL. */
dg_status dg_exchange_apply(dg_ctx* ctx, int mesh_id, int norb, const double* phi, const double* g_pairs,
                            double* W, double* K_pairs, double* E_x, double* v_pairs,
                            dg_rhs_stats* stats, hipStream_t stream);

/* Pair densities (Sec. 6.1: the source of the exchange Poisson problem of
 * eq. fock_poisson for u = phi_i and psi_s = phi_j is their product at the
 * nodes): rho[q - first_pair] = phi_i phi_j for the npairs pairs q =
 * first_pair .. first_pair + npairs - 1 of norb orbitals in the pair order
 * above.  phi: device [norb][n_dofs] (packed fields); rho: device
 * [npairs][n_dofs], written.  Needs no context; enqueued on `stream`.
 * Errors: DG_ERR_ARG for a pair range outside 0 .. norb(norb+1)/2, more than
 * 65535 pairs, or null pointers with work to do. */
dg_status dg_pair_densities(long long n_dofs, int norb, int first_pair, int npairs, const double* phi, double* rho,
                            hipStream_t stream);

/* Dirichlet data by quadrature (Sec. 6.3): the full-space problem -Lap u =
 * 4 pi f is restated on the mesh box with boundary values equal to the
 * Coulomb potential of f, evaluated with the quadrature rule of the mesh's
 * nodal grid (GLL weights, the lumped mass W):
 *   g_s(r) = sum over the nodes x of W(x) f_s(x) / |r - x|,  r a boundary node.
 * f: device [nsrc][n_dofs] (packed fields, field order); g: device
 * [nsrc][n_face] (packed face vectors, face order), written.  The term of a
 * node at the boundary node itself (closer than 1e-6 of the smallest element
 * width) is left out: the method has f vanish on the boundary.  FP64
 * throughout; cost n_face * n_dofs terms per source.  Enqueued on `stream`
 * (no synchronisation); work space is held by the context.  Errors:
 * DG_ERR_ARG for nsrc < 0 or null pointers with nsrc > 0. */
dg_status dg_boundary_data(dg_ctx* ctx, int mesh_id, int nsrc, const double* f, double* g, hipStream_t stream);

/* dg_boundary_data for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same Dirichlet data by quadrature, same arguments, layout and errors,
 * with no hipMalloc, hipFree or other allocation inside the call.  Its work
 * space (the packed source records and split partial sums) is a fixed array
 * of 64 MiB per GPU, held from the first dg_poisson_setup on that GPU until
 * the process ends; the node tables come from the context (built at set-up).
 * Sources go in tiles narrow enough for the records and partial sums to fit,
 * so a mesh whose n_dofs exceeds 8,388,608 values (one source's records) is
 * rejected with DG_ERR_ARG, and large batches take more passes than
 * dg_boundary_data.  Every call on a GPU shares that GPU's array: calls that
 * overlap on one GPU (two streams, or two host threads) race and must be
 * ordered by the caller.  DG_ERR_ARG also when the context's device is not
 * the current one. */
dg_status dg_boundary_data_noalloc(dg_ctx* ctx, int mesh_id, int nsrc, const double* f, double* g,
                                   hipStream_t stream);

/* ---- Consumers of the potentials: actions projected on a basis, compressed exchange ----
 * Functions on the grid are element-major fields of the mesh's finest level, packed one after
 * another ([count][n_dofs], device).  Integrals use the grid's quadrature rule (Sec. 6.1:
 * each factor evaluated at the nodes, weights = the lumped GLL mass).  Outputs are row-major
 * device matrices.  Work is enqueued on `stream` (no synchronisation unless stated). */

/* Hartree action on vectors u_a projected on basis functions phi_i (Sec. 6.1, the action of
 * eq. hartreecoulomb on an orbital): out[i*nu + a] = sum over nodes of w phi_i u_a vH, where vH
 * is a potential on the same grid (e.g. the solution of a Hartree problem from
 * dg_poisson_solve_batch).  nbasis, nu >= 1.  DG_ERR_ARG on bad sizes or null pointers. */
dg_status dg_hartree_action(dg_ctx* ctx, int mesh_id, int nbasis, const double* phi, int nu, const double* u,
                            const double* vH, double* out, hipStream_t stream);

/* Exchange action on vectors u_a projected on basis functions phi_i (Sec. 6.1, eq.
 * fock_exchange and eq. fock_poisson): for every pair (a, s) with an occupied orbital psi_s the
 * problem -Lap v_as = 4 pi u_a psi_s is solved on the grid as dg_poisson_solve_batch does (the
 * context's precision, tolerance, lanes and attached learned guess); W_a = sum_s psi_s v_as
 * (positive sign; the Hartree-Fock prefactor is the caller's) and out[i*nu + a] = sum over nodes
 * of w phi_i W_a.  g_pairs: Dirichlet data [nu*nocc][n_face] with pair (a, s) at a*nocc + s, or
 * NULL (computed by quadrature of u_a psi_s, as dg_boundary_data).  W: device [nu][n_dofs]
 * receiving W_a, or NULL.  stats: host [nu*nocc] or NULL.  1 <= nocc <= 64, nu*nocc <= 4096.
 * Returns after synchronising the stream, with the solve's worst status (dg_poisson_solve_batch). */
dg_status dg_exchange_action(dg_ctx* ctx, int mesh_id, int nbasis, const double* phi, int nu, const double* u,
                             int nocc, const double* psi, const double* g_pairs, double* out, double* W,
                             dg_rhs_stats* stats, hipStream_t stream);

/* Adaptively compressed exchange (Sec. 7.2, the construction the paper cites): from the occupied
 * orbitals psi_k and W_k, the exchange action on them (dg_exchange_apply's W, or
 * dg_exchange_action's W with u = psi), M_kl = (psi_k, W_l) (quadrature), its symmetric part
 * factored M = L L^T (Cholesky), and xi = L^-1 W: xi_k = sum_{j<=k} (L^-1)_kj W_j, device
 * [nocc][n_dofs].  The compressed operator sum_k xi_k (xi_k, .) equals the exchange operator on
 * the span of the psi_k.  1 <= nocc <= 64.  Synchronises the stream; DG_ERR_BREAKDOWN when M is
 * not positive definite (xi then not to be used). */
dg_status dg_ace_build(dg_ctx* ctx, int mesh_id, int nocc, const double* psi, const double* W, double* xi,
                       hipStream_t stream);

/* The compressed exchange applied to vectors u_a and projected on phi_i:
 * out[i*nu + a] = sum_k (phi_i, xi_k) (xi_k, u_a), inner products by quadrature. */
dg_status dg_ace_action(dg_ctx* ctx, int mesh_id, int nbasis, const double* phi, int nu, const double* u, int nocc,
                        const double* xi, double* out, hipStream_t stream);

/* Work-group tiles of the operator kernels (host only; no GPU needed).
 * The operator steps of the path run as a slab kernel on nodes-per-edge n = 2,
 * 3 and 5 (degrees 1, 2, 4): a work-group owns tx x ty elements of the x-y
 * plane and zlen element layers along z.  dg_tile_set chooses the tile of one
 * step (DG_STEP_*) for one arithmetic (fp_bytes 4: FP32, 8: FP64) and one n,
 * for every context set up afterwards (contexts set up before keep theirs).
 * Compiled shapes: n = 2: 8x8, zlen 1..2; n = 3: 4x4, zlen 1..4; n = 5: 4x2,
 * 4x4 or 2x2, zlen 1..4; anything else returns DG_ERR_ARG.  dg_tile_get
 * reports the current choice (host outputs).  The built-in defaults are
 * measured choices for gfx950; the package's tuning script times the
 * alternatives on a workload and writes a table that its binding applies. */
typedef enum {
    DG_STEP_APPLY = 0,     /* y = A u */
    DG_STEP_RESID = 1,     /* r = f - A u */
    DG_STEP_CHEB = 2,      /* Chebyshev smoothing step */
    DG_STEP_CHEBDOT = 3,   /* the same with partial sums of f.z (last post-smoothing step) */
    DG_STEP_PQ = 4,        /* p = z + beta p; q = A p; partial sums of p.q */
    DG_STEP_RESIDDOT = 5,  /* r = f - A u with partial sums of r.r */
    DG_STEP_RESTRICT = 6   /* r = f - A u restricted to the next coarser degree */
} dg_step;
dg_status dg_tile_set(int fp_bytes, int n, int step, int tx, int ty, int zlen);
dg_status dg_tile_get(int fp_bytes, int n, int step, int* tx, int* ty, int* zlen);

/* ---- single steps of the path, exposed for verification and profiling ----
 * All operate on nrhs packed FP64 fields of one mesh at multigrid level
 * `level` (0 = finest).  They return after enqueueing (no synchronisation). */

/* y = A_level u (SIPDG matrix of eq. sip_bilinear at that level). */
dg_status dg_operator_apply(dg_ctx* ctx, int mesh_id, int level, int nrhs, const double* u, double* y,
                            hipStream_t stream);
/* b = 4 pi M rho + boundary lift of g (finest level). */
dg_status dg_rhs_assemble(dg_ctx* ctx, int mesh_id, int nrhs, const double* rho, const double* g, double* b,
                          hipStream_t stream);
/* z = B r, one V-cycle of the hp-multigrid preconditioner from `level` down. */
dg_status dg_vcycle_apply(dg_ctx* ctx, int mesh_id, int level, int nrhs, const double* r, double* z,
                          hipStream_t stream);
/* The FP32 forms of the two entries above, as the inner solve of DG_PREC_FP32_IR
 * runs them: FP32 fields and FP32 arithmetic for the operator, the smoother and
 * the transfers; the coarsest solve still in FP64 arithmetic (on FP32 data).
 * Same layout, ownership and errors as the FP64 entries. */
dg_status dg_operator_apply_f32(dg_ctx* ctx, int mesh_id, int level, int nrhs, const float* u, float* y,
                                hipStream_t stream);
dg_status dg_vcycle_apply_f32(dg_ctx* ctx, int mesh_id, int level, int nrhs, const float* r, float* z,
                              hipStream_t stream);
/* y = A u with FP32 fields and the x and y line contractions on the matrix
 * cores (BF16 operands, FP32 accumulation; the z contraction in FP32 on the
 * vector units), as the smoothing steps of DG_PREC_BF16_PC run it.  Only
 * levels of degree 4; DG_ERR_ARG for others.  Layout, ownership and errors
 * as dg_operator_apply_f32. */
dg_status dg_operator_apply_mfma(dg_ctx* ctx, int mesh_id, int level, int nrhs, const float* u, float* y,
                                 hipStream_t stream);
/* Coarsest-level exact solve z = A^{-1} r (fast diagonalisation). */
dg_status dg_coarse_solve(dg_ctx* ctx, int mesh_id, int nrhs, const double* r, double* z, hipStream_t stream);
/* Transfers between `level` and `level`+1: rc = P^T r (restriction of a
 * fine field) and zf += P zc (prolongation and correction). */
dg_status dg_restrict(dg_ctx* ctx, int mesh_id, int level, int nrhs, const double* r, double* rc,
                      hipStream_t stream);
dg_status dg_prolong_add(dg_ctx* ctx, int mesh_id, int level, int nrhs, const double* zc, double* zf,
                         hipStream_t stream);
/* Timing of the dominant kernel, the finest-level Chebyshev smoothing step.
 * dg_profile_enable(ctx, 1) resets the counters and brackets every later
 * launch of that kernel by HIP events on the solve's stream; 0 stops.
 * dg_profile_read returns the launches timed (-1 if the runtime could not
 * time them), their summed duration in seconds and their algorithmic bytes:
 * every vector the step reads or writes counted once per right-hand side
 * still iterating (host outputs). */
/* Number of group-persistent solves (dg_opts.fused = 2) of this context whose group barrier gave
 * up waiting and that were therefore solved again by the level kernels. */
dg_status dg_fused_fallbacks(const dg_ctx* ctx, long long* count);

dg_status dg_profile_enable(dg_ctx* ctx, int enable);
dg_status dg_profile_read(const dg_ctx* ctx, long long* launches, double* seconds, double* bytes);

/* Smoother bounds [lam_lo, lam_hi] of a level (host outputs). */
dg_status dg_level_info(const dg_ctx* ctx, int mesh_id, int level, int* ne, int* p, double* lam_lo,
                        double* lam_hi);

/* ---- learned initial guess ----------------------------------------------
 * A 3D U-Net on the element grid gives the PCG initial guess.  Tensors are
 * FP32 channels-last [batch][z][y][x][channel] with one channel per node of
 * an element, so an element-major field is a network tensor as it is.
 * Architecture (levels L, channels C; ReLU after every convolution but the
 * last; zero padding 1 for 3x3x3):
 *   h = relu(in(x))                                   1x1x1, in_channels -> C
 *   for l = 0..L-1: e_l = relu(enc_l_b(relu(enc_l_a(h))))    3x3x3, C -> C
 *                   if l < L-1: h = relu(down_l(e_l))        3x3x3 stride 2
 *   d = e_{L-1}
 *   for l = L-2..0: u = relu(up_l(nearest_x2(d)))            3x3x3, C -> C
 *                   d = relu(merge_l(concat(u, e_l)))        3x3x3, 2C -> C
 *   y = out(d)                                        1x1x1, C -> out_channels
 * Parameters: for each convolution in that order, W[tap][ci][co]
 * (tap = (dz*3+dy)*3+dx) then bias[co].  in_channels is the number of nodes
 * of a finest-level element and out_channels that of a level-1 element.  The
 * guess for a source rho is v0 = s P C net(rho / s), s = rms(rho) (see
 * dg_net_guess).  Training minimises the relative A-norm error
 * ||v0 - v_ref||_A^2 / ||v_ref||_A^2 with Adam.  The network is not
 * part of the paper; it only changes where PCG starts, and every solve still
 * stops on the FP64 residual. */
typedef struct { int levels; int channels; int in_channels; int out_channels; } dg_net_config;
typedef struct dg_net dg_net;

dg_status dg_net_create(const dg_net_config* cfg, dg_net** out);
void dg_net_destroy(dg_net* net);
const char* dg_net_last_error(void);
long long dg_net_num_params(const dg_net* net);
/* Host float arrays of dg_net_num_params values (the optimiser state is reset). */
dg_status dg_net_set_params(dg_net* net, const float* params, long long n);
dg_status dg_net_get_params(const dg_net* net, float* params, long long n);
/* y = net(x) for `batch` tensors on an ne[0] x ne[1] x ne[2] element grid (device). */
dg_status dg_net_forward(dg_net* net, int batch, const int* ne, const float* x, float* y, hipStream_t stream);
/* y = net(x) as the guess evaluates it: convolutions on the matrix cores (BF16 operands, FP32
 * accumulation) with BF16 activations between layers (each layer's output rounded to nearest
 * even), the last layer's output in FP32; x is rounded to BF16 first.  Leaves the training
 * state alone (a backward needs dg_net_forward). */
dg_status dg_net_infer(dg_net* net, int batch, const int* ne, const float* x, float* y, hipStream_t stream);
/* Gradient of sum(y * dy) for the last forward; grad (device, may be NULL) receives it. */
dg_status dg_net_backward(dg_net* net, const float* dy, float* grad, hipStream_t stream);
/* Forward convolutions on the matrix cores with BF16 operands and FP32
 * accumulation (enable = 1, the default) or in FP32 on the vector units (0). */
dg_status dg_net_set_bf16(dg_net* net, int enable);
/* One Adam step on the gradient of the last backward. */
dg_status dg_net_adam(dg_net* net, float lr, float b1, float b2, float eps, hipStream_t stream);
/* x = rho / s, s = rms(rho) per sample (device: rho FP64 [batch][n_dofs], x FP32, scale FP64 [batch]). */
dg_status dg_net_prepare_input(dg_net* net, int batch, long long n_dofs, const double* rho, float* x, double* scale,
                               hipStream_t stream);
/* One training step on mesh mesh_id of ctx: forward on x, relative A-norm loss
 * against the scaled targets t = v_ref / s (FP64, packed fields), backward, Adam
 * with learning rate lr; *loss (host) receives the batch mean A-norm loss before
 * the step.  mode selects the output gradient: 0 the A-norm gradient
 * 2Ae/(t'At); 1 the relative nodal L2 gradient 2e/(t't); 2 the A-norm gradient
 * preconditioned by one V-cycle, 2 B A e/(t'At) (well conditioned: B A e ~ e). */
dg_status dg_net_train_step(dg_net* net, dg_ctx* ctx, int mesh_id, int batch, const float* x, const double* t, float lr,
                            int mode, double* loss, hipStream_t stream);
/* v0 = s P C net(rho / s) for batch sources rho of mesh mesh_id of ctx (device
 * FP64 packed fields).  The network's output is a field on multigrid level 1
 * (one channel per node of that level's element); C averages every node
 * shared by neighbouring elements over its copies (continuous field), P is
 * the level-1 to level-0 interpolation of the V-cycle.  With the matrix-core path on (the
 * default) the network is evaluated as dg_net_infer does: BF16 activations. */
dg_status dg_net_guess(dg_net* net, const dg_ctx* ctx, int mesh_id, int batch, const double* rho, double* v0,
                       hipStream_t stream);
/* Flat binary weight file: "DGNET001", 4 ints of configuration, count, floats. */
dg_status dg_net_save(const dg_net* net, const char* path);
dg_status dg_net_load(dg_net* net, const char* path);
/* Use net (or NULL to stop) for the initial guess of every later solve of ctx
 * that passes no x0.  A guess is kept only if ||b - A v0|| < ||b||, right-hand
 * side by right-hand side; stats.guess_used says which were kept. */
dg_status dg_poisson_attach_guess(dg_ctx* ctx, dg_net* net);

/* ---------------------------------------------------------------------------------------------
 * Adaptive octree auxiliary mesh (Sec. 6.2), its SIPDG Poisson problem with hanging faces
 * (Sec. 6.3) and MG-PCG over the refinement hierarchy (Sec. 6.4).
 *
 * Construction: a uniform box of ne[0] x ne[1] x ne[2] base elements (1 to 8 per axis) with
 * degree-q Gauss-Legendre nodes (q = 1..4); a cell of edge lengths L_d (L = max) is halved along
 * every axis with L_d >= L/2 (2, 4 or 8 children) and replaced by its children when the GL
 * integrals of the density on the cell and on its children differ by more than delta_q
 * (indicator Q of Sec. 6.2; the paper uses 1e-8); children are tested in turn, generation by
 * generation, at most max_depth times below a base element (0..8).  Elements (the leaves) are in
 * depth-first order: base elements z, y, x lexicographic with x fastest, the children of a cell
 * in z, y, x lexicographic order of their half along each split axis; each element's (q+1)^3
 * nodes [k][j][i], x fastest.  Fields: element-major FP64, right-hand side after right-hand
 * side.
 *
 * Discretisation: the SIPDG form of eq. sip_bilinear with penalty eq. pen_poly ((q+1)^2 /
 * (eps h), h the smaller width of the two elements along the normal); a hanging face is
 * integrated piece by piece (the intersections of the two sides' faces) with the piece's own
 * (q+1)^2-point GL rule; Nitsche terms carry the Dirichlet data g on the domain boundary.
 * Multigrid: degree steps q -> q/2 -> .. -> 1 on the leaves, then the tree cut at generation
 * G-1, .., 0 at degree 1; exact fast-diagonalisation solve on the base mesh; Chebyshev-Jacobi
 * smoothing with the dg_opts parameters.  Precision DG_PREC_FP64, or DG_PREC_FP32_PC: the
 * V-cycle in FP32 preconditioning the FP64 CG (residuals, iterates and stopping test in FP64). */
typedef struct dg_octree dg_octree;

/* The density: out[i] = rho(x[i], y[i], z[i]) for i < n (host arrays).  Called on the host
 * during dg_octree_create, once per generation with the GL points of every cell tested in it
 * and of its would-be children. */
typedef void (*dg_density_fn)(long long n, const double* x, const double* y, const double* z, double* out,
                              void* user);

typedef struct {
    int ne[3];              /* base elements per axis, 1..8 */
    double lo[3], hi[3];    /* the box */
    int q;                  /* degree, 1..4 */
    double delta_q;         /* refinement tolerance (> 0) */
    int max_depth;          /* refinements below a base element, 0..8 */
    long long max_elements; /* refinement beyond this many elements is DG_ERR_ARG */
} dg_octree_desc;

/* Build the mesh (rho may be NULL: no refinement), its levels and smoother bounds on the current
 * device.  opts NULL: dg_opts_default; precision DG_PREC_FP64 or DG_PREC_FP32_PC.  DG_ERR_ARG on bad sizes,
 * options, a density that is not finite, or more than max_elements elements. */
dg_status dg_octree_create(const dg_octree_desc* desc, dg_density_fn rho, void* user, const dg_opts* opts,
                           dg_octree** out);
void dg_octree_destroy(dg_octree* octree);
/* Elements, finest-level nodes (= n_elements (q+1)^3), Dirichlet points, multigrid levels, and
 * the deepest generation; any pointer may be NULL. */
dg_status dg_octree_info(const dg_octree* octree, long long* n_elements, long long* n_dofs, long long* n_boundary,
                         int* n_levels, int* max_generation);
/* Elements and degree of a multigrid level (0 finest) and its smoother interval. */
dg_status dg_octree_level_info(const dg_octree* octree, int level, long long* n_elements, int* q, double* lam_lo,
                               double* lam_hi);
/* Host arrays: lohi[6e .. 6e+5] = (x, y, z) of the lower, then the upper corner of element e;
 * generation[e] its refinement generation (either may be NULL). */
dg_status dg_octree_elements(const dg_octree* octree, double* lohi, int* generation);
/* Host arrays of n_dofs: the node coordinates, element-major. */
dg_status dg_octree_nodes(const dg_octree* octree, double* x, double* y, double* z);
/* Host arrays of n_boundary: the Dirichlet points, (q+1)^2 per boundary face of an element, in
 * element order, then face order x-, x+, y-, y+, z-, z+, each face [t2][t1] (t1 < t2 its
 * tangential axes, t1 fastest). */
dg_status dg_octree_boundary_points(const dg_octree* octree, double* x, double* y, double* z);
/* b = 4 pi M f + Nitsche lift of g (eq. hartree_poisson / fock_poisson on the auxiliary mesh):
 * device arrays f, b [nrhs][n_dofs] and g [nrhs][n_boundary]; g NULL: the Dirichlet data by
 * quadrature of f (dg_octree_boundary_data, into work space kept by the octree). */
dg_status dg_octree_rhs(dg_octree* octree, int nrhs, const double* f, const double* g, double* b, void* stream);
/* Dirichlet data by quadrature (Sec. 6.3): g_s(r) = sum_q W_q f_s(x_q) / |r - x_q| at the
 * Dirichlet points, over the finest level's nodes x_q with their GL weights W_q (no node lies on
 * the boundary).  Device arrays f [nsrc][n_dofs], g [nsrc][n_boundary]; the node tables and the
 * partial sums are kept by the octree (allocated on first use and when nsrc grows). */
dg_status dg_octree_boundary_data(dg_octree* octree, int nsrc, const double* f, double* g, void* stream);
/* y = A u on multigrid level `level` (device arrays [nrhs][level nodes]). */
dg_status dg_octree_apply(dg_octree* octree, int level, int nrhs, const double* u, double* y, void* stream);
/* y = A u on a level in FP32 arithmetic, the operator of the FP32 V-cycle (device float arrays
 * [nrhs][level nodes]). */
dg_status dg_octree_apply_f32(dg_octree* octree, int level, int nrhs, const float* u, float* y, void* stream);
/* z = V r, one FP64 V-cycle of the preconditioner on the finest level (device arrays). */
dg_status dg_octree_vcycle(dg_octree* octree, int nrhs, const double* r, double* z, void* stream);
/* Exchange on the octree grid (Sec. 6.1): for the orbitals phi [norb][n_dofs] (device, 1 <= norb
 * <= 64) solve for the potentials v_ij of the pair densities phi_i phi_j (i <= j, row-major pair
 * order) with Dirichlet data g_pairs [npairs][n_boundary] (device; NULL: by quadrature), then
 * W [norb][n_dofs] (device, may be NULL): W_k = sum_s phi_s v_ks pointwise, K [npairs] (host, may
 * be NULL): K_ij = sum_q W_q phi_i phi_j v_ij with the grid's GL weights, *e_x (host, may be NULL)
 * = sum over ordered pairs.  v_pairs [npairs][n_dofs] (device) receives the potentials if not
 * NULL.  Solves as dg_octree_solve (stats [npairs], host, may be NULL); synchronises the stream;
 * returns the worst solve status; its work space is kept by the octree (allocated on the first
 * call and when a call needs more). */
dg_status dg_octree_exchange(dg_octree* octree, int norb, const double* phi, const double* g_pairs, double* v_pairs,
                             double* W, double* K, double* e_x, dg_rhs_stats* stats, void* stream);
/* Tuning: right-hand sides per work-group of the octree operator kernels (1, 2 or 4; 0, the
 * default: 4 in FP32 and at degree 4 in FP64, 2 below, the fastest measured on MI355X):
 * the right-hand sides of a work-group share its element's geometry, pieces and tables, and
 * give each thread independent work between its barriers.  Results do not depend on it. */
dg_status dg_octree_set_rhs_per_block(dg_octree* octree, int rhs_per_block);
/* x = A^-1 b by FP64 MG-PCG from x = 0, stopping at ||r|| <= rtol ||b|| (recurrence residual) or
 * max_iter; stats (host, may be NULL) as for dg_poisson_solve_batch; returns the worst status. */
dg_status dg_octree_solve(dg_octree* octree, int nrhs, const double* b, double* x, dg_rhs_stats* stats,
                          void* stream);

#ifdef __cplusplus
}
#endif
#endif /* DG_POISSON_H */
