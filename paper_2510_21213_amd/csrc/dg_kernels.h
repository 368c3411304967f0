// Kernel launchers of the DG Poisson library (host-callable, internal).
#pragma once

#include "dg_internal.h"

namespace dg {

// Epilogues of the brick operator kernel.
enum BrickMode {
    BM_APPLY = 0,    // out = A u
    BM_RESID = 1,    // out = f - A u
    BM_CHEB = 2,     // out = u + cp (u - zprev) + cr D^-1 (f - A u)
    BM_CHEBDOT = 3,  // BM_CHEB and partial sums of f.out
    BM_PQ = 4,       // w = u + beta u2; out2 = w; out = A w; partial sums of w.out
    BM_RESIDDOT = 5,  // BM_RESID and partial sums of out.out
    BM_RESTRICT = 6,  // fc = P^T (f - A u) onto the next coarser (degree) level (launch_restrict only)
    BM_PQ32 = 7       // BM_PQ in FP64 with u an FP32 field (the preconditioned direction of FP32_PC;
                      // launch_pq_mixed only; uses the tile of BM_PQ)
};

enum FinalizeWhat {
    FIN_BB = 0,    // bb = s
    FIN_RR0 = 1,   // rr = s; active = rr > tol2 bb (start of an iteration)
    FIN_RZ = 2,    // beta = rz/rz_old (0 on the first iteration); rz = s
    FIN_PQ = 3,    // alpha = rz/s (breakdown if s <= 0)
    FIN_RR = 4,    // rr = s; iters++; active = rr > tol2 bb and iters < maxit
    FIN_TRUE = 5,  // rr_true = s (FP64 residual of the returned solution)
    FIN_OUTER = 6, // outer refinement: rr = s; scale = sqrt(s); active = rr > tol2 bb
    FIN_FLEX = 7,  // flexible CG after FIN_RZ, s = z.r_old: beta = (rz - s) / rz_prev (0 on the first iteration)
    FIN_RZ0 = 8,   // as FIN_RZ with beta = 0 (a restarted step: the direction is the preconditioned residual)
    FIN_CR = 9,    // cr = s (c.r of the learned correction)
    FIN_CAC = 10   // cac = s (c.Ac of the learned correction)
};

struct KernelCfg {
    int bricks_per_rhs;  // partial-sum slots of brick kernels
    int chunks_per_rhs;  // partial-sum slots of pointwise kernels
};

inline int chunks_of(long long ndof) { return (int)((ndof + 1023) / 1024); }
inline int bricks_of(const LevelHost& L) { return L.nbr[0] * L.nbr[1] * L.nbr[2]; }
// Slab-kernel tiles.  tile_set/tile_get edit the process-wide table from which assign_tiles
// fills a level when it is set up (false: a shape with no compiled kernel, or bad arguments).
bool tile_set(int fp_bytes, int n, int mode, int tx, int ty, int zlen);
bool tile_get(int fp_bytes, int n, int mode, int* tx, int* ty, int* zlen);
void assign_tiles(LevelHost& L);

// Partial-sum slots per right-hand side that launch_brick writes in dot mode
// `mode` (its work-groups per right-hand side).
template <typename T>
int op_blocks(const LevelHost& L, int mode);

template <typename T>
void launch_brick(int mode, const LevelHost& L, const LevelDev<T>* dev, int nrhs, const RhsState* st, const T* u,
                  const T* u2, const T* f, const T* zprev, T* out, T* out2, double* partial, int pstride, double cp,
                  double cr, hipStream_t s);

// fc = P^T (f - A z) (z may be null: fc = P^T f); optionally z1c = c0c Dc^-1 fc.
template <typename T>
void launch_restrict(const LevelHost& Lf, const LevelDev<T>* devf, const LevelHost& Lc, const LevelDev<T>* devc,
                     int nrhs, const RhsState* st, const T* z, const T* f, T* fc, T* z1c, double c0c, hipStream_t s);

// The FP32 operator step with its x and y line contractions on the matrix cores (BF16 operands,
// FP32 accumulation; modes BM_APPLY, BM_CHEB, BM_CHEBDOT).  False (nothing launched) where the
// level has no such kernel (degree 4 on 4 x 2 tiles only).
bool launch_brick_mf(int mode, const LevelHost& L, const LevelDev<float>* dev, int nrhs, const RhsState* st,
                     const float* u, const float* f, const float* zprev, float* out, double* partial, int pstride,
                     double cp, double cr, hipStream_t s);

// FP32_PC step of the FP64 PCG: p = z + beta p_old with z the FP32 V-cycle output, q = A p and
// partial sums of p.q, all in FP64.  tmp: an FP64 field buffer used only on levels whose degree
// has no slab kernel (z is widened into it first); may be null when has_pq_mixed(L).
bool has_pq_mixed(const LevelHost& L);
// zbf16: z holds BF16 values (the BF16-field V-cycle); degree-4 levels only.  The search direction
// is then stored in FP32 (pold and pnew address FP32 values; the new direction is rounded to FP32
// before q = A p is formed from it).
void launch_pq_mixed(const LevelHost& L, const LevelDev<double>* dev, int nrhs, const RhsState* st, const float* z,
                     const double* pold, double* q, double* pnew, double* tmp, double* partial, int pstride,
                     hipStream_t s, bool zbf16 = false);
// BF16-field forms of the V-cycle steps of the finest levels (FP32 arithmetic, fields stored as
// BF16 at the addresses the float pointers give): a smoothing step (BM_CHEB; BM_CHEBDOT on degree
// 4), the residual restriction of a degree step (coarse_bf16: its coarse outputs fc and z1c are
// BF16 too; degree 4 only), and the prolongation-correction of a degree step into a BF16 fine field
// (coarse_bf16: zc holds BF16 values; degree 4 only).  Degree 4 with its 4 -> 2 step, and degree 2
// with its 2 -> 1 step into FP32 coarse fields; false elsewhere, and nothing is launched then.
bool launch_brick_lp(int mode, const LevelHost& L, const LevelDev<float>* dev, int nrhs, const RhsState* st,
                     const float* u, const float* f, const float* zprev, float* out, double* partial, int pstride,
                     double cp, double cr, hipStream_t s);
bool launch_restrict_lp(const LevelHost& Lf, const LevelDev<float>* devf, const LevelHost& Lc,
                        const LevelDev<float>* devc, int nrhs, const RhsState* st, const float* z, const float* f,
                        float* fc, float* z1c, double c0c, hipStream_t s, bool coarse_bf16 = false);
bool launch_prolong_lp(const LevelHost& Lf, const LevelHost& Lc, int nrhs, const RhsState* st, const float* zc,
                       float* zf, hipStream_t s, bool coarse_bf16 = false);

// zf += P zc
// zf = scale[rhs] * P zc for a degree step (writes every fine node); false when the step
// between the two levels is not a degree step with a kernel for it (nothing launched)
bool launch_prolong_set(const LevelHost& Lf, const LevelHost& Lc, int nrhs, const double* zc, double* zf,
                        const double* scale, hipStream_t s);
template <typename T>
void launch_prolong(const LevelHost& Lf, const LevelHost& Lc, int nrhs, const RhsState* st, const T* zc, T* zf,
                    hipStream_t s);

// z = A^-1 r on the coarsest level (FP64 arithmetic for any storage type).  scratch: 2 * nrhs *
// L.ndof doubles, which spreads the solve over many work-groups in three launches; null: one
// work-group per right-hand side.
template <typename T>
void launch_coarse(const CoarseDev* C, const LevelHost& L, int nrhs, const RhsState* st, const T* r, T* z,
                   double* scratch, hipStream_t s);

// L.dinv64 / L.dinv32 = 1 / diag(A) of the level (the tables must be allocated, ndof each).
void launch_dinv(const LevelHost& L, hipStream_t s);

// z = c0 D^-1 f
template <typename T>
void launch_cheb0(const LevelHost& L, const LevelDev<T>* dev, int nrhs, const RhsState* st, const T* f, T* z,
                  double c0, hipStream_t s);

// x += alpha p; r -= alpha q; partial sums of r.r; optionally z1 = c0 D^-1 r.
template <typename T>
void launch_update(const LevelHost& L, const LevelDev<T>* dev, int nrhs, const RhsState* st, T* x, T* r, const T* p,
                   const T* q, T* z1, double c0, double* partial, int pstride, hipStream_t s);

// FP32_PC update: x += alpha p; r -= alpha q; partial sums of r.r (FP64); r32 = (float) r and
// z1 = (float) c0 D^-1 r, the source and first smoothing iterate of the FP32 V-cycle.  bf16: r32
// and z1 are BF16 fields and p holds FP32 values (the BF16-field V-cycle's search direction).
void launch_update_pc(const LevelHost& L, const LevelDev<double>* dev, int nrhs, const RhsState* st, double* x,
                      double* r, const double* p, const double* q, float* r32, float* z1, double c0, double* partial,
                      int pstride, hipStream_t s, bool bf16 = false);
// FP32_PC start: r32 = (float) r and z1 = (float) c0 D^-1 r.
void launch_to32_cheb0(const LevelHost& L, const LevelDev<double>* dev, int nrhs, const RhsState* st, const double* r,
                       float* r32, float* z1, double c0, hipStream_t s, bool bf16 = false);

// partial sums of a.b per right-hand side (FP64 accumulation).
template <typename TA, typename TB>
void launch_dot(long long ndof, int nrhs, const RhsState* st, const TA* a, const TB* b, double* partial,
                int pstride, hipStream_t s);

// Guard of an initial guess, after its FP64 residual r = b - A x and st.rr = ||r||^2: a guess
// whose residual is not below ||b|| is dropped (x = 0, r = b, rr = bb); st.guess records the
// decision.  outer: st is the refinement state (FIN_OUTER fields are updated as well).
// drop_all: every right-hand side starts from x = 0 (no residual needed, st.bb set).
void launch_guard(int nrhs, long long n, RhsState* st, const double* b, double* x, double* r, bool outer,
                  bool drop_all, hipStream_t s);
void launch_finalize(int what, int nrhs, RhsState* st, const double* partial, int pstride, int nblk,
                     hipStream_t s);

// st[i].active = 0 wherever gate[i].active == 0 (right-hand sides whose outer loop has finished).
void launch_gate(int nrhs, RhsState* st, const RhsState* gate, hipStream_t s);

// Inner FP32 state of a refinement step from the outer FP64 state: relative tolerance
// max(inner_rtol, 0.9 rtol sqrt(bb / rr)) capped at 0.5 (what the outer tolerance still
// needs), on a right-hand side of norm 1; active where the outer loop is.
void launch_inner_init(int nrhs, const RhsState* outer, RhsState* inner, double rtol, double inner_rtol, int maxit,
                       hipStream_t s);

// b = 4 pi M rho + lift(g).  If phi is non-null, rho of right-hand side q is
// phi[pi[q]] * phi[pj[q]] (pair densities) and rho is ignored.
void launch_rhs(const LevelHost& L, const LevelDev<double>* dev, int nrhs, const double* rho, const double* phi,
                const int* pi, const int* pj, const double* g, long long nface, double* b, hipStream_t s);

// Iterative refinement: r32 = r64 / st.scale, and x64 += st.scale * d32.
void launch_to_inner(long long ndof, int nrhs, const RhsState* st, const double* r64, float* r32, hipStream_t s);
void launch_correct(long long ndof, int nrhs, const RhsState* st, const float* d32, double* x64, hipStream_t s);

// Fill / copy / scale helpers.
template <typename T>
void launch_fill(T* x, T v, long long n, hipStream_t s);
void launch_copy(const double* a, double* b, long long n, hipStream_t s);
// y[i] = x[i] * D(i)^-1/2 of the level (Lanczos set-up), per right-hand side 0 only.
void launch_dscale(const LevelHost& L, const LevelDev<double>* dev, const double* x, double* y, hipStream_t s);
// y = a x + b y  (single vector)
void launch_axpby(long long n, double a, const double* x, double b, double* y, hipStream_t s);
// rho = r / (4 pi M) for nrhs fields of the level: the source whose right-hand side, without a boundary
// lift, is r (the learned coarse-grid correction hands a residual to the guess network as a density).
void launch_source_of(const LevelHost& L, const LevelDev<double>* dev, int nrhs, const double* r, double* rho,
                      hipStream_t s);
// The learned correction's Galerkin step, per active right-hand side: gamma = c.r / c.Ac (0 unless
// c.Ac > 0, from the state's cr and cac), c <- gamma c, and q <- r - gamma q (q holds A c on entry).
void launch_lcgc_scale(long long ndof, int nrhs, const RhsState* st, const double* r, double* c, double* q,
                       hipStream_t s);

// Exchange: W_k = sum_s phi_s v_ks; partial sums of w rho_ij v_ij per pair.
void launch_exchange(const LevelHost& L, const LevelDev<double>* dev, int norb, const double* phi, const double* v,
                     double* W, double* partial, int pstride, hipStream_t s);
// rho[q] = phi[pi[q]] * phi[pj[q]] for every pair q.
void launch_pair_products(long long ndof, int npairs, const double* phi, const int* pi, const int* pj, double* rho,
                          hipStream_t s);

// rho[q - first] = phi_i phi_j for the pairs q = first .. first + count - 1 (row-major pair order).
void launch_pair_densities(long long ndof, int norb, int first, int count, const double* phi, double* rho,
                           hipStream_t s);

// dst[doff[q] + i] = src[soff[q] + i] for i < len and q < nseg (offset tables on the device).
void launch_segcopy(const double* src, const long long* soff, double* dst, const long long* doff, long long len,
                    int nseg, hipStream_t s);

// K[q] = sum of partial[q][0..nblk-1] (fixed order).
void launch_sum_partials(int nq, const double* partial, int pstride, int nblk, double* K, hipStream_t s);

// Fused solve of small meshes: one work-group (FUSED_THREADS threads, a divisor of 1024) per right-hand side runs
// the whole FP64 PCG with its V-cycle, every level staged through LDS, in a single launch.
// Every level of an eligible mesh has degree at most 4, at most FUSED_MAX_DOF nodes (two FP64
// staging arrays of that size fill 128 KiB of LDS) and at most FUSED_MAX_AXIS nodes per axis.
// The group-persistent variant (launch_group_pcg) reads the same tables with no limit on the
// nodes of a level.
constexpr int FUSED_THREADS = 512;
constexpr int FUSED_MAX_DOF = 8192;
constexpr int FUSED_MAX_LEVELS = 8;
constexpr int FUSED_MAX_AXIS = 128;
constexpr int FUSED_MAX_DEG = 16;
constexpr int FUSED_LDS_DOUBLES = 20480;  // the work-group's LDS: 160 KiB
constexpr int FUSED_COARSE_SCRATCH = 16 * (16 * 17 + 2) + 3 * 16 * 16;  // coarsest solve's LDS (CMAX = 16)
struct FusedLevel {
    const LevelDev<double>* L;  // 1D blocks and masses of the level (device)
    const double* dinv;         // inverse diagonal, element-major (device)
    int E[3], n, ndof, N[3];    // elements, nodes per element edge, nodes, nodes per axis
    int deg;                    // smoothing steps (0 on the coarsest level)
    double c0, cp[FUSED_MAX_DEG], cr[FUSED_MAX_DEG];
    long long off_f, off_za, off_zb;  // fields of the level in a right-hand side's work space
    int lf, lza, lzb;                 // the same fields' offsets in LDS (resident mode)
    // transfer to the next coarser level per axis: P[d][Xf * Nc_d + Xc] (device, dense); the
    // coarse node Xc takes the fine nodes rlo .. rlo + rcnt - 1 (restriction), the fine node Xf
    // the coarse nodes plo .. plo + pcnt - 1 (prolongation)
    const double* P[3];
    short rlo[3][FUSED_MAX_AXIS], rcnt[3][FUSED_MAX_AXIS], plo[3][FUSED_MAX_AXIS], pcnt[3][FUSED_MAX_AXIS];
};
struct FusedMeshDev {
    int nl;
    int resident;  // 1: every level field lives in LDS for the whole solve
    int lsy;       // resident mode: LDS offset of the operator output (and of the coarsest solve's scratch)
    int lds_ok;    // 1: every level fits the one-work-group kernel's LDS staging (FUSED_MAX_DOF)
    FusedLevel lv[FUSED_MAX_LEVELS];
    const CoarseDev* coarse;
    long long off_x, off_r, off_p;  // level-0 PCG fields (the level-0 smoother fields are lv[0].off_za/zb)
    long long ws_per_rhs;           // doubles of work space per right-hand side
    // group-persistent solve: after the fields above, q = A p (level 0), the residual handed to a
    // restriction (largest level), two coarsest-level scratch arrays and the group's reduction slots
    long long off_q, off_t, off_g1, off_g2, off_red;
    long long ws_group;             // doubles of work space per right-hand side in that solve
};
// Solve nrhs problems b -> x of one small mesh (FP64 PCG, HS beta, up to three restarts from the
// current iterate when the recomputed residual misses the tolerance).  st: tol2 and maxit set;
// on return bb, rr (of the returned x), iters, breakdown and guess are written, active = 0.
// has_x0: x holds initial guesses (guard: a guess whose residual is not below ||b|| is dropped).
// ws: nrhs * M.ws_per_rhs doubles.
void launch_fused_pcg(const FusedMeshDev* M, int nrhs, const double* b, double* x, RhsState* st, double* ws,
                      bool has_x0, bool guard, hipStream_t s);

// Group-persistent fused solve: the same solve with K work-groups (GROUP_THREADS threads each) per
// right-hand side, persistent for the whole solve, every phase spread over the group and the phases
// separated by a group barrier (an arrival counter per right-hand side; no grid-wide barrier).  The
// group's work-groups run on one XCD.  A barrier that waits more than `spin` polls gives up: the
// right-hand side then returns with st.breakdown = GROUP_SYNC_FAILED (its outputs are not to be
// used) and the caller solves it again with the level kernels.  ws: nrhs * M.ws_group doubles;
// sync: 2 * nrhs counters (zeroed here, before the launch).
constexpr int GROUP_THREADS = 256;
constexpr int GROUP_MAX_K = 32;
constexpr int GROUP_SYNC_FAILED = 3;
void launch_group_pcg(const FusedMeshDev* M, int K, int nrhs, const double* b, double* x, RhsState* st, double* ws,
                      unsigned* sync, bool has_x0, bool guard, long long spin, hipStream_t s);

// Consumers of the grid potentials (dg_consumers.hip).  Quadrature weight of a node: the product
// of the level's three 1D lumped masses.
// out[i * nu + a] = sum_q w_q f_q phi_i(q) u_a(q) over the nodes of level L (f null: 1), fields
// packed [nbasis][ndof] and [nu][ndof]; partial: nbasis * nu * project_chunks(L.ndof) doubles.
int project_chunks(long long ndof);
void launch_project(const LevelHost& L, int nbasis, const double* phi, int nu, const double* u, const double* f,
                    double* partial, double* out, hipStream_t s);
// rho[a * nocc + s] = u_a psi_s
void launch_cross_products(long long ndof, int nu, int nocc, const double* u, const double* psi, double* rho,
                           hipStream_t s);
// W[a] = sum_s psi_s v[a * nocc + s]
void launch_cross_w(long long ndof, int nu, int nocc, const double* psi, const double* v, double* W, hipStream_t s);
// One work-group: T = L^-1 for the Cholesky factor L of the symmetric part of M (n x n, n <= 64);
// flag[0] = 1 when M is not positive definite.
void launch_ace_factor(int n, const double* M, double* T, int* flag, hipStream_t s);
// xi[k] = sum_{j <= k} T[k][j] W[j]
void launch_ace_combine(long long ndof, int n, const double* T, const double* W, double* xi, hipStream_t s);
// C = A B for small row-major matrices (ni x nk) (nk x na)
void launch_small_gemm(int ni, int nk, int na, const double* A, const double* B, double* C, hipStream_t s);

// Dirichlet data by quadrature (dg_boundary.hip): g[s][b] = sum_q W_q f_s(x_q) / |r_b - x_q| over the
// finest level's nodes, for nsrc sources f (packed fields) or, with f null, the pair products
// phi[pi[s]] phi[pj[s]].  Sources go in tiles of R; each tile is packed into rec (rec_len
// doubles) and its Z planes are split S ways (partial sums in part, part_len doubles).
struct QuadPlan {
    int R, ntile, S, zper;
    long long nface, rec_len, part_len;
};
QuadPlan quad_plan(const LevelHost& L, int nsrc);
// The same with rec_len + part_len <= capacity doubles (R = 0 if the mesh cannot fit).
QuadPlan quad_plan_bounded(const LevelHost& L, int nsrc, long long capacity);
// The fixed work space of dg_boundary_data_noalloc (a file-scope device array): look up this
// device's copy once, with the device current (quad_scratch_init), then fetch it and its size
// in doubles (quad_scratch; null before the lookup).
hipError_t quad_scratch_init(int device);
double* quad_scratch(int device, long long* capacity);
// nodes: the node coordinates per axis, x[NX] then y[NY] then z[NZ] (device).
void launch_quad_data(const LevelHost& L, const LevelDev<double>* dev, const double* nodes, const QuadPlan& P,
                      int nsrc, const double* f, const double* phi, const int* pi, const int* pj, double* rec,
                      double* part, double* g, hipStream_t s);

}  // namespace dg
