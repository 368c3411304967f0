// C ABI and solver driver of the DG Poisson library.
//
// The driver enqueues the kernels of dg_kernels.hip on the caller's stream:
// right-hand-side assembly, batched V-cycle preconditioned conjugate
// gradients with per-right-hand-side state kept on the device (a finished
// right-hand side is skipped by every later kernel), and in FP32_IR mode an
// FP64 iterative-refinement loop around an FP32 inner solve.  The host only
// reads the per-right-hand-side state back every `check_every` iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <exception>
#include <functional>
#include <memory>
#include <atomic>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "dg_internal.h"
#include "dg_kernels.h"

namespace {

thread_local std::string g_err;

void set_err(const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
}

struct HipError : std::runtime_error {
    using std::runtime_error::runtime_error;
};
struct ArgError : std::runtime_error {
    using std::runtime_error::runtime_error;
};

#define HIPCHK(x)                                                                                       \
    do {                                                                                                \
        hipError_t e_ = (x);                                                                            \
        if (e_ != hipSuccess)                                                                           \
            throw HipError(std::string(#x) + ": " + hipGetErrorString(e_) + " at line " +               \
                           std::to_string(__LINE__));                                                   \
    } while (0)

template <typename T>
T* dalloc(long long n) {
    void* p = nullptr;
    if (n <= 0) n = 1;
    HIPCHK(hipMalloc(&p, (size_t)n * sizeof(T)));
    return (T*)p;
}

template <typename T>
void dfree(T*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

// Per-precision work space of one mesh, in groups sized separately (right-hand sides each holds):
// WK_R the level-0 residual (the V-cycle source), WK_PCG the other level-0 PCG vectors, WK_LV the
// per-level smoother and transfer vectors, WK_TMP one more level-0 field (FP32_PC on a degree
// with no mixed-precision operator kernel).
enum { WK_R = 1, WK_PCG = 2, WK_LV = 4, WK_TMP = 8, WK_ALL = WK_R | WK_PCG | WK_LV };
template <typename T>
struct Work {
    std::vector<T*> f, za, zb;  // per level (f[0] unused: the PCG residual is the level-0 source)
    T *x = nullptr, *r = nullptr, *p0 = nullptr, *p1 = nullptr, *q = nullptr, *tmp = nullptr;
    int cap_r = 0, cap_pcg = 0, cap_lv = 0, cap_tmp = 0;
    void release_lv() {
        for (auto* p : f) dfree(p);
        for (auto* p : za) dfree(p);
        for (auto* p : zb) dfree(p);
        f.clear(); za.clear(); zb.clear();
        cap_lv = 0;
    }
    void release() {
        release_lv();
        dfree(x); dfree(r); dfree(p0); dfree(p1); dfree(q); dfree(tmp);
        cap_r = cap_pcg = cap_tmp = 0;
    }
};

struct ChebCoef {
    double c0;                       // first step 1/theta
    std::vector<double> cp, cr;      // steps k = 1 .. m-1
};

}  // namespace

struct dg_ctx {
    dg_opts opts;
    int device = 0;
    hipStream_t stream = nullptr;        // internal stream (capturable), default priority
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    struct Mesh {
        dg_mesh mesh;
        std::vector<dg::LevelHost> lv;
        std::vector<ChebCoef> cheb;
        dg::CoarseDev coarse;
        dg::CoarseDev* dcoarse = nullptr;
        int pstride = 0;
        long long nface = 0;
        Work<double> w64;
        Work<float> w32;
        double* b = nullptr;       // FP64 right-hand sides
        double* r64 = nullptr;     // FP64 outer residual (FP32_IR)
        double* partial = nullptr;
        dg::RhsState* st = nullptr;      // outer / FP64 state
        dg::RhsState* st_in = nullptr;   // inner FP32 state
        dg::RhsState* st_host = nullptr; // pinned host mirror
        int cap_b = 0, cap_st = 0;
        // captured PCG iterations, per kind of run (index 0: FP64, 1: FP32 inner solve, 2: FP32_PC, 3: BF16_PC,
        // 4: BF16F_PC)
        struct Graph {
            hipGraphExec_t exec = nullptr;
            int nrhs = 0, every = 0;
            bool prof = false;
            std::vector<hipEvent_t> ev;
            size_t nev = 0;
        } graph[5];
        // multi-mesh batches: the mesh's own stream and completion event, and its
        // right-hand sides gathered from the caller's packing when they are not contiguous
        hipStream_t stream = nullptr;
        hipEvent_t ev_done = nullptr;
        // iterations the k-th PCG run of the last solve needed (per kind of run): the next
        // solve replays that many before its first host check
        std::vector<int> pred[5];
        // timing events of eager launches driven by this solver instance
        std::vector<hipEvent_t> pev;
        size_t pused = 0;
        // a second solver instance of a mesh (lane) shares the level tables of the first
        bool owns_tables = true;
        double *grho = nullptr, *gface = nullptr, *gx0 = nullptr, *gv = nullptr;
        int cap_g = 0;
        double* qnodes = nullptr;  // node coordinates per axis (quadrature Dirichlet data), built at set-up
        // fused solve of a small mesh (null when the mesh is not small enough): device tables
        // (shared by the lanes), their transfer matrices, and this lane's work space
        dg::FusedMeshDev* dfused = nullptr;
        std::vector<double*> fusedP;
        double* fws = nullptr;
        long long fws_cap = 0, fws_per = 0;  // work space held, and needed per right-hand side
        bool fused_lds_ok = false;           // every level fits the one-work-group kernel's LDS staging
        long long fws_group = 0;             // work space per right-hand side of the group-persistent solve
        unsigned* gsync = nullptr;           // its barrier counters (2 per right-hand side)
        int gsync_cap = 0;
        double* cscr = nullptr;              // scratch of the coarsest solve (2 fields per right-hand side)
        int cscr_cap = 0;
        double* lc_rho = nullptr;            // learned coarse-grid correction: the residual as a density,
        double* lc_c = nullptr;              // and the network's correction (finest-level fields)
        long long lc_cap = 0;
    };
    std::vector<Mesh> meshes;
    std::vector<Mesh> twins;       // further solver lanes: lane k >= 1 of mesh i at (k - 1) * n_meshes + i
                                   // (empty with one lane)
    dg_net* guess = nullptr;       // learned initial guess (not owned)
    std::atomic<long long> fused_fallbacks{0};  // group-persistent solves that fell back to the level kernels
    double* g_x0 = nullptr;        // guess work space
    double* g_rho = nullptr;
    long long g_cap = 0;
    // timing of the finest-level Chebyshev step
    struct Prof {
        bool on = false;
        std::vector<hipEvent_t> ev;  // start/stop pairs
        size_t used = 0;
        long long launches = 0;
        double seconds = 0.0, bytes = 0.0;
        bool failed = false;
        std::mutex mu;               // solver lanes add their timings from their own threads
    } prof;
    hipEvent_t ev_ready = nullptr;           // multi-mesh batches: inputs assembled
    long long* segtab = nullptr;             // gather / scatter offset tables (device)
    long long* segtab_host = nullptr;        // their pinned staging copy
    long long segtab_cap = 0;
    // exchange work space
    double* xv = nullptr;
    long long xv_cap = 0;
    double* xpart = nullptr;
    long long xpart_cap = 0;
    int* xpairs = nullptr;
    int xpairs_cap = 0;
    // quadrature Dirichlet data work space: packed source tile, split partial sums, pair data
    double* qrec = nullptr;
    long long qrec_cap = 0;
    double* qpart = nullptr;
    long long qpart_cap = 0;
    double* qg = nullptr;
    long long qg_cap = 0;
    // consumers (projections, exchange action, compressed exchange): work space
    double* cpart = nullptr;   // projection partial sums
    long long cpart_cap = 0;
    double* crho = nullptr;    // pair sources u_a psi_s
    long long crho_cap = 0;
    double* cv = nullptr;      // their potentials
    long long cv_cap = 0;
    double* cW = nullptr;      // W_a when the caller does not take it
    long long cW_cap = 0;
    double* csmall = nullptr;  // small matrices (M, L^-1, ACE factors)
    long long csmall_cap = 0;
    int* cflag = nullptr;
};

namespace {

using dg::LevelHost;
using Mesh = dg_ctx::Mesh;

void drop_graphs(Mesh& M) {
    for (auto& G : M.graph) {
        if (G.exec) (void)hipGraphExecDestroy(G.exec);
        G.exec = nullptr;
    }
}

void ensure_state(Mesh& M, int nrhs) {
    if (M.cap_st >= nrhs) return;
    drop_graphs(M);
    dfree(M.st);
    dfree(M.st_in);
    if (M.st_host) (void)hipHostFree(M.st_host);
    dfree(M.partial);
    M.st = dalloc<dg::RhsState>(nrhs);
    M.st_in = dalloc<dg::RhsState>(nrhs);
    HIPCHK(hipHostMalloc((void**)&M.st_host, sizeof(dg::RhsState) * nrhs, hipHostMallocDefault));
    M.partial = dalloc<double>((long long)nrhs * M.pstride);
    M.cap_st = nrhs;
}

void ensure_cscr(Mesh& M, int nrhs) {
    if (M.cscr_cap >= nrhs) return;
    drop_graphs(M);
    dfree(M.cscr);
    M.cscr = dalloc<double>(2LL * nrhs * M.lv.back().ndof);
    M.cscr_cap = nrhs;
}

template <typename T>
void ensure_work(Mesh& M, Work<T>& W, int nrhs, int parts = WK_ALL) {
    const long long n0 = M.lv[0].ndof * nrhs;
    const int L = (int)M.lv.size();
    if ((parts & WK_R) && W.cap_r < nrhs) {
        drop_graphs(M);
        dfree(W.r);
        W.r = dalloc<T>(n0);
        W.cap_r = nrhs;
    }
    if ((parts & WK_PCG) && W.cap_pcg < nrhs) {
        drop_graphs(M);
        dfree(W.x); dfree(W.p0); dfree(W.p1); dfree(W.q);
        W.x = dalloc<T>(n0);
        W.p0 = dalloc<T>(n0);
        W.p1 = dalloc<T>(n0);
        W.q = dalloc<T>(n0);
        W.cap_pcg = nrhs;
    }
    if ((parts & WK_TMP) && W.cap_tmp < nrhs) {
        drop_graphs(M);
        dfree(W.tmp);
        W.tmp = dalloc<T>(n0);
        W.cap_tmp = nrhs;
    }
    if ((parts & WK_LV) && W.cap_lv < nrhs) {
        drop_graphs(M);
        W.release_lv();
        W.f.assign(L, nullptr);
        W.za.assign(L, nullptr);
        W.zb.assign(L, nullptr);
        for (int l = 0; l < L; ++l) {
            const long long n = M.lv[l].ndof * nrhs;
            if (l > 0) W.f[l] = dalloc<T>(n);
            W.za[l] = dalloc<T>(n);
            W.zb[l] = dalloc<T>(n);
        }
        W.cap_lv = nrhs;
        ensure_cscr(M, nrhs);
    }
}

// Work space of an FP32_PC or BF16_PC solve: FP64 PCG vectors, an FP32 V-cycle with its FP32 source
// (flexible: two of them, the current and the previous).
void ensure_work_pc(Mesh& M, int nrhs, bool flex = false) {
    ensure_work<double>(M, M.w64, nrhs, WK_R | WK_PCG | (dg::has_pq_mixed(M.lv[0]) ? 0 : WK_TMP));
    ensure_work<float>(M, M.w32, nrhs, WK_R | WK_LV | (flex ? WK_TMP : 0));
}

void ensure_b(Mesh& M, int nrhs, bool need_r64) {
    if (M.cap_b < nrhs || (need_r64 && !M.r64)) {
        dfree(M.b);
        dfree(M.r64);
        M.b = dalloc<double>(M.lv[0].ndof * nrhs);
        if (need_r64) M.r64 = dalloc<double>(M.lv[0].ndof * nrhs);
        M.cap_b = nrhs;
    }
}

template <typename T>
const dg::LevelDev<T>* ldev(const LevelHost& L);
template <>
const dg::LevelDev<double>* ldev<double>(const LevelHost& L) { return L.dev64; }
template <>
const dg::LevelDev<float>* ldev<float>(const LevelHost& L) { return L.dev32; }

// One V-cycle from level l: on entry f is the level-l source; if z1_ready,
// W.za[l] already holds the first smoothing iterate c0 D^-1 f.  Returns the
// buffer that holds z = B f.  With dot, the last smoothing step at level 0
// also writes partial sums of f.z.
// Profiling state of the context being driven by this host thread (null on the
// worker threads of a multi-mesh batch, which are not timed).
thread_local dg_ctx::Prof* g_prof = nullptr;

// Where prof_mark records: the context's pool (eager launches) or the event
// set of a graph being captured (re-recorded at every replay).
struct EventSink {
    std::vector<hipEvent_t>* ev = nullptr;
    size_t* used = nullptr;
};
thread_local EventSink g_sink;

void prof_mark(hipStream_t s) {
    auto& ev = *g_sink.ev;
    auto& used = *g_sink.used;
    if (used == ev.size()) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        ev.push_back(e);
    }
    HIPCHK(hipEventRecord(ev[used++], s));
}

// Called after the stream has been synchronised: add up the timed launches.
void prof_sum(const std::vector<hipEvent_t>& ev, size_t used) {
    auto& P = *g_prof;
    std::lock_guard<std::mutex> lock(P.mu);
    for (size_t i = 0; i + 1 < used; i += 2) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) != hipSuccess) {
            // timing not available for these events: report nothing rather than fail the solve
            (void)hipGetLastError();
            P.failed = true;
            return;
        }
        P.seconds += 1e-3 * ms;
        P.launches += 1;
    }
}

// The number of finest levels whose V-cycle fields BF16F_PC keeps in BF16, where the kernels exist
// for them: a degree-4 finest level whose next level is its degree-2 step (1), and that level too
// when it is not the coarsest and its own next level is its degree-1 step (2).  0: the mode runs
// as FP32_PC on this hierarchy.
int lp_fields(const dg_ctx* ctx, const Mesh& M) {
    if (ctx->opts.precision != DG_PREC_BF16F_PC || M.lv.size() < 2) return 0;
    auto degree_step = [](const LevelHost& F, const LevelHost& C, int nf, int nc) {
        return F.n == nf && C.n == nc && !F.hcoarse && F.E[0] == C.E[0] && F.E[1] == C.E[1] && F.E[2] == C.E[2];
    };
    if (!degree_step(M.lv[0], M.lv[1], 5, 3) || !dg::has_pq_mixed(M.lv[0])) return 0;
    return M.lv.size() >= 3 && degree_step(M.lv[1], M.lv[2], 3, 2) ? 2 : 1;
}

// mf: the level-0 smoothing steps take their x and y contractions on the matrix cores (FP32
// fields only, where the level has such a kernel).  lpn: the fields (source, smoother iterates) of
// levels below lpn hold BF16 values (FP32 arithmetic; the levels below them stay FP32); see
// lp_fields().
template <typename T>
T* vcycle(Mesh& M, Work<T>& W, int l, int nrhs, const dg::RhsState* st, const T* f, bool z1_ready, bool dot,
          hipStream_t s, bool mf = false, int lpn = 0) {
    const bool timed = l == 0 && g_prof && g_prof->on;
    const int L = (int)M.lv.size();
    const LevelHost& Lv = M.lv[l];
    if (l == L - 1) {
        dg::launch_coarse<T>(M.dcoarse, Lv, nrhs, st, f, W.za[l], M.cscr_cap >= nrhs ? M.cscr : nullptr, s);
        return W.za[l];
    }
    const ChebCoef& C = M.cheb[l];
    const int m = (int)C.cp.size() + 1;
    const auto* dv = ldev<T>(Lv);
    if (!z1_ready) dg::launch_cheb0<T>(Lv, dv, nrhs, st, f, W.za[l], C.c0, s);
    T* cur = W.za[l];
    T* prev = W.zb[l];
    const bool mf0 = mf && l == 0;
    const bool lpl = l < lpn, lpc = l + 1 < lpn;  // BF16 fields on this level, on the next
    // one smoothing step: on the matrix cores where asked for and available, else the FP32/FP64 kernel
    auto step = [&](int mode, const T* u, const T* zp, T* out, double cp, double cr) {
        if constexpr (sizeof(T) == 4) {
            if (lpl) {
                if (!dg::launch_brick_lp(mode, Lv, dv, nrhs, st, u, f, zp, out, M.partial, M.pstride, cp, cr, s))
                    throw std::logic_error("internal: no BF16-field smoothing kernel for this level");
                return;
            }
            if (mf0 && dg::launch_brick_mf(mode, Lv, dv, nrhs, st, u, f, zp, out, M.partial, M.pstride, cp, cr, s))
                return;
        }
        dg::launch_brick<T>(mode, Lv, dv, nrhs, st, u, nullptr, f, zp, out, nullptr, M.partial, M.pstride, cp, cr, s);
    };
    for (int k = 1; k < m; ++k) {
        if (timed) prof_mark(s);
        step(dg::BM_CHEB, cur, k == 1 ? nullptr : prev, prev, C.cp[k - 1], C.cr[k - 1]);
        if (timed) prof_mark(s);
        std::swap(cur, prev);
    }
    const LevelHost& Lc = M.lv[l + 1];
    const bool coarse_is_last = (l + 1 == L - 1);
    if constexpr (sizeof(T) == 4) {
        if (lpl) {
            if (!dg::launch_restrict_lp(Lv, dv, Lc, ldev<T>(Lc), nrhs, st, cur, f, W.f[l + 1],
                                        coarse_is_last ? nullptr : W.za[l + 1], coarse_is_last ? 0.0 : M.cheb[l + 1].c0,
                                        s, lpc))
                throw std::logic_error("internal: no BF16-field restriction kernel for this level");
        } else {
            dg::launch_restrict<T>(Lv, dv, Lc, ldev<T>(Lc), nrhs, st, cur, f, W.f[l + 1],
                                   coarse_is_last ? nullptr : W.za[l + 1], coarse_is_last ? 0.0 : M.cheb[l + 1].c0, s);
        }
    } else {
        dg::launch_restrict<T>(Lv, dv, Lc, ldev<T>(Lc), nrhs, st, cur, f, W.f[l + 1],
                               coarse_is_last ? nullptr : W.za[l + 1], coarse_is_last ? 0.0 : M.cheb[l + 1].c0, s);
    }
    T* zc = vcycle<T>(M, W, l + 1, nrhs, st, W.f[l + 1], !coarse_is_last, false, s, false, lpn);
    if constexpr (sizeof(T) == 4) {
        if (lpl) {
            if (!dg::launch_prolong_lp(Lv, Lc, nrhs, st, zc, cur, s, lpc))
                throw std::logic_error("internal: no BF16-field prolongation kernel for this level");
        } else {
            dg::launch_prolong<T>(Lv, Lc, nrhs, st, zc, cur, s);
        }
    } else {
        dg::launch_prolong<T>(Lv, Lc, nrhs, st, zc, cur, s);
    }
    for (int k = 0; k < m; ++k) {
        const bool last = (k == m - 1);
        const int mode = (dot && last) ? dg::BM_CHEBDOT : dg::BM_CHEB;
        const double cp = k == 0 ? 0.0 : C.cp[k - 1];
        const double cr = k == 0 ? C.c0 : C.cr[k - 1];
        if (timed) prof_mark(s);
        step(mode, cur, k == 0 ? nullptr : prev, prev, cp, cr);
        if (timed) prof_mark(s);
        std::swap(cur, prev);
    }
    return cur;
}

// One PCG iteration on level 0 (vectors of W; p ping-pong by parity).
template <typename T>
void pcg_iteration(Mesh& M, Work<T>& W, int nrhs, dg::RhsState* st, int parity, hipStream_t s) {
    const LevelHost& L0 = M.lv[0];
    const auto* dv = ldev<T>(L0);
    const int nb_rz = dg::op_blocks<T>(L0, dg::BM_CHEBDOT), nb = dg::op_blocks<T>(L0, dg::BM_PQ);
    const int nc = dg::chunks_of(L0.ndof);
    T* z = vcycle<T>(M, W, 0, nrhs, st, W.r, true, true, s);
    if (M.lv.size() == 1) {
        // the preconditioner was the exact solve alone: no smoothing step wrote the r.z partial sums
        dg::launch_dot<T, T>(L0.ndof, nrhs, st, W.r, z, M.partial, M.pstride, s);
        dg::launch_finalize(dg::FIN_RZ, nrhs, st, M.partial, M.pstride, nc, s);
    } else {
        dg::launch_finalize(dg::FIN_RZ, nrhs, st, M.partial, M.pstride, nb_rz, s);
    }
    T* pold = parity ? W.p1 : W.p0;
    T* pnew = parity ? W.p0 : W.p1;
    dg::launch_brick<T>(dg::BM_PQ, L0, dv, nrhs, st, z, pold, nullptr, nullptr, W.q, pnew, M.partial, M.pstride, 0.0,
                        0.0, s);
    dg::launch_finalize(dg::FIN_PQ, nrhs, st, M.partial, M.pstride, nb, s);
    dg::launch_update<T>(L0, dv, nrhs, st, W.x, W.r, pnew, W.q, W.za[0], M.cheb[0].c0, M.partial, M.pstride, s);
    dg::launch_finalize(dg::FIN_RR, nrhs, st, M.partial, M.pstride, nc, s);
}

// One FP64 PCG iteration preconditioned by the learned coarse-grid correction followed by the
// V-cycle: c = N(r) (the guess network fed the residual as the density r / (4 pi M), its level-1
// output prolonged to the finest level) spans a one-dimensional coarse space, corrected by its
// Galerkin multiple gamma = c.r / c.Ac, then z = gamma c + V(r - gamma A c); the direction
// restarts (beta = 0), since this preconditioner is not a fixed linear map.  One solver lane (the
// network's buffers are shared).
void pcg_iteration_lcgc(dg_ctx* ctx, Mesh& M, Work<double>& W, int nrhs, dg::RhsState* st, int parity,
                        hipStream_t s) {
    const LevelHost& L0 = M.lv[0];
    const auto* dv = L0.dev64;
    const int nb = dg::op_blocks<double>(L0, dg::BM_PQ), nc = dg::chunks_of(L0.ndof);
    const long long n = L0.ndof * nrhs;
    if (M.lc_cap < n) {
        dfree(M.lc_rho);
        dfree(M.lc_c);
        M.lc_rho = dalloc<double>(n);
        M.lc_c = dalloc<double>(n);
        M.lc_cap = n;
    }
    const int mesh_id = (int)(&M - ctx->meshes.data());
    dg::launch_source_of(L0, dv, nrhs, W.r, M.lc_rho, s);
    if (dg_net_guess(ctx->guess, ctx, mesh_id, nrhs, M.lc_rho, M.lc_c, s) != DG_OK)
        throw ArgError(std::string("learned coarse-grid correction failed: ") + dg_net_last_error());
    // A c into q (free until the search-direction step); the Galerkin multiple gamma = c.r / c.Ac
    // of c (the best one in the energy norm: a useless c gets gamma = 0, and z falls back to V(r));
    // then q = r - gamma A c and z = gamma c + V(q)
    dg::launch_brick<double>(dg::BM_APPLY, L0, dv, nrhs, st, M.lc_c, nullptr, nullptr, nullptr, W.q, nullptr,
                             M.partial, M.pstride, 0.0, 0.0, s);
    dg::launch_dot<double, double>(L0.ndof, nrhs, st, M.lc_c, W.r, M.partial, M.pstride, s);
    dg::launch_finalize(dg::FIN_CR, nrhs, st, M.partial, M.pstride, nc, s);
    dg::launch_dot<double, double>(L0.ndof, nrhs, st, M.lc_c, W.q, M.partial, M.pstride, s);
    dg::launch_finalize(dg::FIN_CAC, nrhs, st, M.partial, M.pstride, nc, s);
    dg::launch_lcgc_scale(L0.ndof, nrhs, st, W.r, M.lc_c, W.q, s);
    double* z = vcycle<double>(M, W, 0, nrhs, st, W.q, false, false, s);
    dg::launch_axpby(n, 1.0, M.lc_c, 1.0, z, s);
    dg::launch_dot<double, double>(L0.ndof, nrhs, st, W.r, z, M.partial, M.pstride, s);
    dg::launch_finalize(dg::FIN_RZ0, nrhs, st, M.partial, M.pstride, nc, s);
    double* pold = parity ? W.p1 : W.p0;
    double* pnew = parity ? W.p0 : W.p1;
    dg::launch_brick<double>(dg::BM_PQ, L0, dv, nrhs, st, z, pold, nullptr, nullptr, W.q, pnew, M.partial, M.pstride,
                             0.0, 0.0, s);
    dg::launch_finalize(dg::FIN_PQ, nrhs, st, M.partial, M.pstride, nb, s);
    dg::launch_update<double>(L0, dv, nrhs, st, W.x, W.r, pnew, W.q, W.za[0], M.cheb[0].c0, M.partial, M.pstride, s);
    dg::launch_finalize(dg::FIN_RR, nrhs, st, M.partial, M.pstride, nc, s);
}

// One PCG iteration of FP32_PC: the PCG vectors, the operator of the search direction and all dot
// products in FP64 (W); the V-cycle preconditioner in FP32 (M.w32, whose level-0 residual r32 and
// first smoothing iterate the update step writes).
// flex (BF16_PC): the smoothing steps of level 0 on the matrix cores, and the flexible (Polak-Ribiere)
// beta, for which the FP32 residual alternates between two buffers so that the previous one is
// still there for z.r_old.
void pcg_iteration_pc(Mesh& M, Work<double>& W, int nrhs, dg::RhsState* st, int parity, hipStream_t s,
                      bool flex = false, int lpn = 0) {
    const bool lp = lpn > 0;
    const LevelHost& L0 = M.lv[0];
    Work<float>& V = M.w32;
    const int nb_rz = dg::op_blocks<float>(L0, dg::BM_CHEBDOT), nb = dg::op_blocks<double>(L0, dg::BM_PQ);
    const int nc = dg::chunks_of(L0.ndof);
    float* rcur = (flex && parity) ? V.tmp : V.r;
    float* rnext = flex ? (parity ? V.r : V.tmp) : V.r;
    float* z = vcycle<float>(M, V, 0, nrhs, st, rcur, true, true, s, flex, lpn);
    if (M.lv.size() == 1) {
        // the preconditioner was the exact solve alone: no smoothing step wrote the r.z partial sums
        dg::launch_dot<float, float>(L0.ndof, nrhs, st, rcur, z, M.partial, M.pstride, s);
        dg::launch_finalize(dg::FIN_RZ, nrhs, st, M.partial, M.pstride, nc, s);
    } else {
        dg::launch_finalize(dg::FIN_RZ, nrhs, st, M.partial, M.pstride, nb_rz, s);
    }
    if (flex) {
        dg::launch_dot<float, float>(L0.ndof, nrhs, st, rnext, z, M.partial, M.pstride, s);  // z . r_old
        dg::launch_finalize(dg::FIN_FLEX, nrhs, st, M.partial, M.pstride, nc, s);
    }
    // lp: the search direction is kept in FP32 in the first half of these FP64 buffers
    double* pold = parity ? W.p1 : W.p0;
    double* pnew = parity ? W.p0 : W.p1;
    dg::launch_pq_mixed(L0, L0.dev64, nrhs, st, z, pold, W.q, pnew, W.tmp, M.partial, M.pstride, s, lp);
    dg::launch_finalize(dg::FIN_PQ, nrhs, st, M.partial, M.pstride, nb, s);
    dg::launch_update_pc(L0, L0.dev64, nrhs, st, W.x, W.r, pnew, W.q, rnext, V.za[0], M.cheb[0].c0, M.partial,
                         M.pstride, s, lp);
    dg::launch_finalize(dg::FIN_RR, nrhs, st, M.partial, M.pstride, nc, s);
}

void read_state(Mesh& M, const dg::RhsState* st, int nrhs, hipStream_t s) {
    HIPCHK(hipMemcpyAsync(M.st_host, st, sizeof(dg::RhsState) * nrhs, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
}

void init_state(Mesh& M, dg::RhsState* st, int nrhs, double rtol, int maxit, hipStream_t s) {
    for (int i = 0; i < nrhs; ++i) {
        dg::RhsState S{};
        S.tol2 = rtol * rtol;
        S.maxit = maxit;
        S.active = 1;
        S.scale = 1.0;
        M.st_host[i] = S;
    }
    HIPCHK(hipMemcpyAsync(st, M.st_host, sizeof(dg::RhsState) * nrhs, hipMemcpyHostToDevice, s));
}

// PCG on level 0 from the current x and r of W (r holds the residual);
// st must have tol2/maxit/bb set.  PC: FP64 PCG (T = double) preconditioned by the FP32 V-cycle.
template <typename T, bool PC = false>
void pcg_run(dg_ctx* ctx, Mesh& M, Work<T>& W, int nrhs, dg::RhsState* st, const dg::RhsState* gate, int slot,
             hipStream_t s) {
    static_assert(!PC || sizeof(T) == 8, "FP32_PC runs its PCG in FP64");
    const LevelHost& L0 = M.lv[0];
    const int nc = dg::chunks_of(L0.ndof);
    const bool flex = PC && ctx->opts.precision == DG_PREC_BF16_PC;
    const int lpn = PC ? lp_fields(ctx, M) : 0;
    const bool lp = lpn > 0;
    const int kind = PC ? (lp ? 4 : flex ? 3 : 2) : (sizeof(T) == 8 ? 0 : 1);
    // element size of the V-cycle's level-0 fields
    const size_t vbytes = PC ? (lp ? sizeof(__bf16) : sizeof(float)) : sizeof(T);
    // rr and the active flags
    dg::launch_dot<T, T>(L0.ndof, nrhs, gate, W.r, W.r, M.partial, M.pstride, s);
    dg::launch_finalize(dg::FIN_RR0, nrhs, st, M.partial, M.pstride, nc, s);
    if (gate) dg::launch_gate(nrhs, st, gate, s);  // finished outer loops keep their inner solve idle
    if constexpr (PC)
        dg::launch_to32_cheb0(L0, L0.dev64, nrhs, st, W.r, M.w32.r, M.w32.za[0], M.cheb[0].c0, s, lp);
    else
        dg::launch_cheb0<T>(L0, ldev<T>(L0), nrhs, st, W.r, W.za[0], M.cheb[0].c0, s);
    dg::launch_fill<T>(W.p0, (T)0, L0.ndof * nrhs, s);
    dg::launch_fill<T>(W.p1, (T)0, L0.ndof * nrhs, s);
    auto iteration = [&](int parity) {
        if constexpr (PC)
            pcg_iteration_pc(M, W, nrhs, st, parity, s, flex, lpn);
        else
            pcg_iteration<T>(M, W, nrhs, st, parity, s);
    };
    const int maxit = ctx->opts.max_iter;
    const bool timed = g_prof && g_prof->on;
    int it = 0;
    if constexpr (!PC && sizeof(T) == 8) {
        // the leading iterations with the learned coarse-grid correction (an even count keeps the
        // p ping-pong of the captured iterations aligned), on eager launches
        const int K = (ctx->opts.learned_cgc + 1) / 2 * 2;
        if (K > 0 && ctx->opts.precision == DG_PREC_FP64 && ctx->guess && !gate) {
            for (; it < K && it < maxit; ++it) pcg_iteration_lcgc(ctx, M, W, nrhs, st, it & 1, s);
            HIPCHK(hipGetLastError());
        }
    }
    if (ctx->opts.use_graph) {
        // `every` iterations captured once and replayed; an even count keeps the p ping-pong aligned
        int every = std::max(2, ctx->opts.check_every);
        every += every & 1;
        auto& G = M.graph[kind];
        if (!G.exec || G.nrhs != nrhs || G.every != every || G.prof != timed) {
            if (G.exec) (void)hipGraphExecDestroy(G.exec);
            G.exec = nullptr;
            size_t used = 0;
            EventSink saved = g_sink;
            if (timed) {
                // events are created before the capture; the graph records them at every replay
                const int m = (int)M.cheb[0].cp.size() + 1;
                const size_t need = (size_t)every * 2 * (2 * m - 1);
                while (G.ev.size() < need) {
                    hipEvent_t e;
                    HIPCHK(hipEventCreate(&e));
                    G.ev.push_back(e);
                }
            }
            g_sink = {&G.ev, &used};
            HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            hipGraph_t graph = nullptr;
            try {
                for (int c = 0; c < every; ++c) iteration(c & 1);
            } catch (...) {
                (void)hipStreamEndCapture(s, &graph);  // leave capture mode before reporting
                if (graph) (void)hipGraphDestroy(graph);
                g_sink = saved;
                throw;
            }
            HIPCHK(hipStreamEndCapture(s, &graph));
            g_sink = saved;
            hipError_t e = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            HIPCHK(e);
            G.nrhs = nrhs;
            G.every = every;
            G.prof = timed;
            G.nev = used;
        }
        // replay up to the count the same run of the previous solve needed, then check
        // after every replay (finished right-hand sides cost only early-exiting launches)
        auto& pred = M.pred[kind];
        const int ahead = slot < (int)pred.size() ? pred[slot] : 0;
        while (it < maxit) {
            do {
                HIPCHK(hipGraphLaunch(G.exec, s));
                it += every;
            } while (it + every <= ahead && it < maxit);
            read_state(M, st, nrhs, s);
            if (timed) prof_sum(G.ev, G.nev);
            bool any = false;
            for (int i = 0; i < nrhs; ++i) any |= M.st_host[i].active != 0;
            if (!any) break;
        }
    } else {
        const int every = std::max(1, ctx->opts.check_every);
        while (it < maxit) {
            if (timed) {
                M.pused = 0;
                g_sink = {&M.pev, &M.pused};
            }
            for (int c = 0; c < every && it < maxit; ++c, ++it) iteration(it & 1);
            HIPCHK(hipGetLastError());
            read_state(M, st, nrhs, s);
            if (timed) prof_sum(M.pev, M.pused);
            bool any = false;
            for (int i = 0; i < nrhs; ++i) any |= M.st_host[i].active != 0;
            if (!any) break;
        }
    }
    {
        auto& pred = M.pred[kind];
        if ((int)pred.size() <= slot) pred.resize(slot + 1, 0);
        int need = 0;
        for (int i = 0; i < nrhs; ++i) need = std::max(need, M.st_host[i].iters);
        pred[slot] = need;
    }
    if (g_prof && g_prof->on) {
        // algorithmic bytes of the timed steps: per V-cycle, pre-smoothing steps 1..m-1 and post-smoothing
        // steps 0..m-1 read u and f, the steps with a previous iterate also read it, and all write one vector
        const int m = (int)M.cheb[0].cp.size() + 1;
        const double per_cycle = (m >= 2 ? 3.0 + 4.0 * (m - 2) : 0.0) + 3.0 + 4.0 * (m - 1);
        long long cycles = 0;
        for (int i = 0; i < nrhs; ++i) cycles += M.st_host[i].iters;
        std::lock_guard<std::mutex> lock(g_prof->mu);
        g_prof->bytes += per_cycle * (double)cycles * (double)L0.ndof * (double)vbytes;
    }
}

// The solver runs on the context's own stream (the caller's may be the legacy
// default stream, which cannot be captured into a graph): it waits for the
// caller's stream on entry, and the caller's stream waits for it on exit.
hipStream_t enter(dg_ctx* ctx, hipStream_t user) {
    HIPCHK(hipEventRecord(ctx->ev_in, user));
    HIPCHK(hipStreamWaitEvent(ctx->stream, ctx->ev_in, 0));
    return ctx->stream;
}
void leave(dg_ctx* ctx, hipStream_t user) {
    HIPCHK(hipEventRecord(ctx->ev_out, ctx->stream));
    HIPCHK(hipStreamWaitEvent(user, ctx->ev_out, 0));
}

void check_mesh_id(const dg_ctx* ctx, int mesh_id) {
    if (!ctx) throw ArgError("null context");
    if (mesh_id < 0 || mesh_id >= (int)ctx->meshes.size()) throw ArgError("mesh_id out of range");
}

void ensure_len(double*& p, long long& cap, long long n) {
    if (cap >= n) return;
    dfree(p);
    p = dalloc<double>(n);
    cap = n;
}

// Dirichlet data by quadrature (Sec. 6.3) of nsrc sources of mesh M into g (device
// [nsrc][n_face]): the sources are the fields f, or with f null the pair products of phi.
// Node coordinates per axis of the finest level (x, then y, then z) in device memory: the
// quadrature's grid.  Built when a mesh is set up.
void build_qnodes(dg_ctx* ctx, Mesh& M) {
    std::vector<double> all;
    for (int d = 0; d < 3; ++d) {
        dg::AxisDev<double> ax;
        std::vector<double> nodes;
        dg::build_axis(M.mesh.ne[d], M.mesh.p, M.mesh.lo[d], M.mesh.hi[d], ctx->opts.penalty_eps, ax, nullptr,
                       &nodes, ctx->opts.node_family);
        all.insert(all.end(), nodes.begin(), nodes.end());
    }
    double* d = dalloc<double>((long long)all.size());
    HIPCHK(hipMemcpy(d, all.data(), sizeof(double) * all.size(), hipMemcpyHostToDevice));
    M.qnodes = d;
}

void quad_data(dg_ctx* ctx, Mesh& M, int nsrc, const double* f, const double* phi, const int* pi, const int* pj,
               double* g, hipStream_t s) {
    const LevelHost& L0 = M.lv[0];
    if (L0.family != 0)
        throw ArgError("Dirichlet data by quadrature need Gauss-Lobatto nodes (pass g at the face points)");
    const dg::QuadPlan P = dg::quad_plan(L0, nsrc);
    if (P.nface != M.nface) throw std::logic_error("quadrature plan: face count mismatch");
    ensure_len(ctx->qrec, ctx->qrec_cap, P.rec_len);
    ensure_len(ctx->qpart, ctx->qpart_cap, P.part_len);
    dg::launch_quad_data(L0, L0.dev64, M.qnodes, P, nsrc, f, phi, pi, pj, ctx->qrec, ctx->qpart, g, s);
}

// Tables of the fused small-mesh solve (every level at most FUSED_MAX_DOF nodes): levels, smoother
// coefficients, dense 1D transfers with their index ranges, work-space offsets.  Leaves M.dfused
// null when the mesh is not small enough.
void build_fused(Mesh& M) {
    const int nl = (int)M.lv.size();
    if (nl > dg::FUSED_MAX_LEVELS || M.lv[0].family != 0) return;
    bool lds_ok = true;
    for (int l = 0; l < nl; ++l) {
        const LevelHost& L = M.lv[l];
        if (L.n > 5) return;  // the fused operator has kernels for degrees 1..4
        if (L.ndof > dg::FUSED_MAX_DOF) lds_ok = false;
        for (int d = 0; d < 3; ++d)
            if (L.E[d] * L.n > dg::FUSED_MAX_AXIS) return;
        if (l + 1 < nl && (int)M.cheb[l].cp.size() + 1 > dg::FUSED_MAX_DEG) return;
    }
    if (M.lv.back().E[0] * M.lv.back().n > dg::CMAX || M.lv.back().E[1] * M.lv.back().n > dg::CMAX ||
        M.lv.back().E[2] * M.lv.back().n > dg::CMAX)
        return;  // the coarsest solve's tables hold at most CMAX nodes per axis
    dg::FusedMeshDev H;
    std::memset(&H, 0, sizeof(H));
    H.nl = nl;
    long long off = 0;
    H.off_x = off; off += M.lv[0].ndof;
    H.off_r = off; off += M.lv[0].ndof;
    H.off_p = off; off += M.lv[0].ndof;
    for (int l = 0; l < nl; ++l) {
        const LevelHost& L = M.lv[l];
        dg::FusedLevel& F = H.lv[l];
        F.L = L.dev64;
        F.dinv = L.dinv64;
        for (int d = 0; d < 3; ++d) {
            F.E[d] = L.E[d];
            F.N[d] = L.E[d] * L.n;
        }
        F.n = L.n;
        F.ndof = (int)L.ndof;
        F.off_f = off; off += L.ndof;
        F.off_za = off; off += L.ndof;
        F.off_zb = off; off += L.ndof;
        if (l + 1 == nl) continue;
        const ChebCoef& C = M.cheb[l];
        F.deg = (int)C.cp.size() + 1;
        F.c0 = C.c0;
        for (size_t k = 0; k < C.cp.size(); ++k) {
            F.cp[k] = C.cp[k];
            F.cr[k] = C.cr[k];
        }
        // 1D transfers to the next coarser level: degree step (same elements) or mesh step (parent element)
        const LevelHost& Lc = M.lv[l + 1];
        std::vector<double> xf, wf, Df, xc, wc, Dc;
        dg::gll(L.p, xf, wf, Df);
        dg::gll(Lc.p, xc, wc, Dc);
        for (int d = 0; d < 3; ++d) {
            const int nf = L.n, nc = Lc.n, Nf = F.N[d], Nc = Lc.E[d] * Lc.n;
            const bool mesh_step = L.E[d] != Lc.E[d];
            std::vector<double> P((size_t)Nf * Nc, 0.0);
            for (int ef = 0; ef < L.E[d]; ++ef) {
                const int ec = mesh_step ? ef / 2 : ef;
                std::vector<double> pts(nf), Lg;
                for (int i = 0; i < nf; ++i) pts[i] = mesh_step ? (xf[i] + 2.0 * (ef % 2) - 1.0) / 2.0 : xf[i];
                dg::lagrange_eval(xc, pts, Lg);
                for (int i = 0; i < nf; ++i)
                    for (int a = 0; a < nc; ++a) P[(size_t)(ef * nf + i) * Nc + ec * nc + a] = Lg[i * nc + a];
                for (int i = 0; i < nf; ++i) {  // fine node <- coarse nodes of its (parent) element
                    F.plo[d][ef * nf + i] = (short)(ec * nc);
                    F.pcnt[d][ef * nf + i] = (short)nc;
                }
            }
            for (int ec = 0; ec < Lc.E[d]; ++ec)
                for (int a = 0; a < nc; ++a) {  // coarse node <- fine nodes of its element (or its two children)
                    F.rlo[d][ec * nc + a] = (short)((mesh_step ? 2 * ec : ec) * nf);
                    F.rcnt[d][ec * nc + a] = (short)((mesh_step ? 2 : 1) * nf);
                }
            double* dP = dalloc<double>((long long)P.size());
            HIPCHK(hipMemcpy(dP, P.data(), sizeof(double) * P.size(), hipMemcpyHostToDevice));
            M.fusedP.push_back(dP);
            F.P[d] = dP;
        }
    }
    // resident mode when every level field fits in LDS with the operator output, the coarsest
    // solve's scratch (from the output's offset on) and the reduction slots:
    // [f, za, zb of every level][output, max(level-0 size, coarse scratch)][reduction]
    {
        int lo = 0;
        for (int l = 0; l < nl; ++l) {
            dg::FusedLevel& F = H.lv[l];
            F.lf = lo; lo += F.ndof;
            F.lza = lo; lo += F.ndof;
            F.lzb = lo; lo += F.ndof;
        }
        H.lsy = lo;
        lo += std::max(H.lv[0].ndof, dg::FUSED_COARSE_SCRATCH);
        H.resident = lo + dg::FUSED_THREADS / 64 <= dg::FUSED_LDS_DOUBLES ? 1 : 0;
    }
    H.coarse = M.dcoarse;
    H.ws_per_rhs = off;
    M.fws_per = off;
    H.lds_ok = lds_ok ? 1 : 0;
    M.fused_lds_ok = lds_ok;
    // group-persistent solve: q, the restriction's residual (largest level below the coarsest, or
    // level 0), two coarsest-level scratch arrays, two sets of reduction slots
    {
        long long big = 0;
        for (int l = 0; l < nl; ++l) big = std::max(big, M.lv[l].ndof);
        H.off_q = off; off += M.lv[0].ndof;
        H.off_t = off; off += big;
        H.off_g1 = off; off += M.lv[nl - 1].ndof;
        H.off_g2 = off; off += M.lv[nl - 1].ndof;
        H.off_red = off; off += 2 * dg::GROUP_MAX_K;
        H.ws_group = off;
        M.fws_group = off;
    }
    M.dfused = dalloc<dg::FusedMeshDev>(1);
    HIPCHK(hipMemcpy(M.dfused, &H, sizeof(H), hipMemcpyHostToDevice));
}

// fused = 1: one work-group per right-hand side (levels within its LDS staging); fused = 2: the
// group-persistent solve.
bool use_fused(const dg_ctx* ctx, const Mesh& M) {
    if (!M.dfused || ctx->opts.precision != DG_PREC_FP64) return false;
    return (ctx->opts.fused == 1 && M.fused_lds_ok) || ctx->opts.fused == 2;
}

// Work-groups per right-hand side of the group-persistent solve: the option, else about 4
// level-0 nodes per thread, at most 16.
int group_wgs(const dg_ctx* ctx, const Mesh& M) {
    if (ctx->opts.fused_wgs > 0) return std::min(ctx->opts.fused_wgs, dg::GROUP_MAX_K);
    const long long per = 4LL * dg::GROUP_THREADS;
    return (int)std::max(1LL, std::min(16LL, (M.lv[0].ndof + per - 1) / per));
}

void ensure_fused_ws(const dg_ctx* ctx, Mesh& M, int nrhs) {
    const bool group = ctx->opts.fused == 2;
    const long long need = (group ? M.fws_group : M.fws_per) * nrhs;
    if (M.fws_cap < need) {
        dfree(M.fws);
        M.fws = dalloc<double>(need);
        M.fws_cap = need;
    }
    if (group && M.gsync_cap < nrhs) {
        dfree(M.gsync);
        M.gsync = dalloc<unsigned>(2LL * nrhs);
        M.gsync_cap = nrhs;
    }
}

// Learned guess for nrhs sources rho of mesh M: writes ctx->g_x0 (the solve's guard
// later drops a guess whose residual is not below ||b||).
void learned_guess(dg_ctx* ctx, Mesh& M, int nrhs, const double* rho, hipStream_t s);

// Solve nrhs problems of one mesh: b (FP64, packed) -> v.  Fills stats.
// guard: x0 is a learned guess, kept per right-hand side only if its residual is below ||b||
// (decided on the device from the first FP64 residual of the solve).
void solve_group(dg_ctx* ctx, Mesh& M, int nrhs, const double* b, const double* x0, double* v, dg_rhs_stats* stats,
                 hipStream_t s, bool guard = false) {
    const LevelHost& L0 = M.lv[0];
    const long long n0 = L0.ndof;
    const int nc = dg::chunks_of(n0), nb = dg::op_blocks<double>(L0, dg::BM_RESIDDOT);
    const auto& o = ctx->opts;
    ensure_state(M, nrhs);
    std::vector<int> iters(nrhs, 0), outer(nrhs, 0), kept(nrhs, x0 ? 1 : 0);
    bool fused_done = false;
    if (use_fused(ctx, M)) {
        // small mesh: the whole PCG in one launch, one work-group (fused = 1) or a group of
        // work-groups (fused = 2) per right-hand side
        ensure_fused_ws(ctx, M, nrhs);
        init_state(M, M.st, nrhs, o.rtol, o.max_iter, s);
        if (x0) HIPCHK(hipMemcpyAsync(v, x0, sizeof(double) * n0 * nrhs, hipMemcpyDeviceToDevice, s));
        if (o.fused == 2)
            dg::launch_group_pcg(M.dfused, group_wgs(ctx, M), nrhs, b, v, M.st, M.fws, M.gsync, x0 != nullptr, guard,
                                 o.fused_spin > 0 ? o.fused_spin : (o.fused_spin < 0 ? 0LL : 2000000LL), s);
        else
            dg::launch_fused_pcg(M.dfused, nrhs, b, v, M.st, M.fws, x0 != nullptr, guard, s);
        HIPCHK(hipGetLastError());
        read_state(M, M.st, nrhs, s);
        // a group barrier that gave up leaves its right-hand side unsolved: the batch is solved
        // again by the level kernels below (the caller's initial guesses are still in x0)
        fused_done = true;
        for (int i = 0; i < nrhs; ++i) fused_done &= M.st_host[i].breakdown != dg::GROUP_SYNC_FAILED;
        if (fused_done) {
            for (int i = 0; i < nrhs; ++i) {
                iters[i] = M.st_host[i].iters;
                outer[i] = 1;
                if (x0) kept[i] = M.st_host[i].guess;
            }
        } else {
            ctx->fused_fallbacks += 1;
            init_state(M, M.st, nrhs, o.rtol, o.max_iter, s);
        }
    }
    if (fused_done) {
    } else if (o.precision == DG_PREC_FP64 || o.precision == DG_PREC_FP32_PC || o.precision == DG_PREC_BF16_PC ||
               o.precision == DG_PREC_BF16F_PC) {
        const bool pc = o.precision != DG_PREC_FP64;
        if (pc)
            ensure_work_pc(M, nrhs, o.precision == DG_PREC_BF16_PC);
        else
            ensure_work<double>(M, M.w64, nrhs);
        Work<double>& W = M.w64;
        init_state(M, M.st, nrhs, o.rtol, o.max_iter, s);
        dg::launch_dot<double, double>(n0, nrhs, nullptr, b, b, M.partial, M.pstride, s);
        dg::launch_finalize(dg::FIN_BB, nrhs, M.st, M.partial, M.pstride, nc, s);
        if (x0 && guard) {
            dg::launch_copy(x0, W.x, n0 * nrhs, s);
            dg::launch_brick<double>(dg::BM_RESIDDOT, L0, L0.dev64, nrhs, nullptr, W.x, nullptr, b, nullptr, W.r,
                                     nullptr, M.partial, M.pstride, 0, 0, s);
            dg::launch_finalize(dg::FIN_TRUE, nrhs, M.st, M.partial, M.pstride, nb, s);
            dg::launch_guard(nrhs, n0, M.st, b, W.x, W.r, false, false, s);
        } else if (x0) {
            dg::launch_copy(x0, W.x, n0 * nrhs, s);
            dg::launch_brick<double>(dg::BM_RESID, L0, L0.dev64, nrhs, nullptr, W.x, nullptr, b, nullptr, W.r,
                                     nullptr, nullptr, 0, 0, 0, s);
        } else {
            dg::launch_fill<double>(W.x, 0.0, n0 * nrhs, s);
            dg::launch_copy(b, W.r, n0 * nrhs, s);
        }
        for (int restart = 0; restart < 3; ++restart) {
            if (pc)
                pcg_run<double, true>(ctx, M, W, nrhs, M.st, nullptr, restart, s);
            else
                pcg_run<double>(ctx, M, W, nrhs, M.st, nullptr, restart, s);
            for (int i = 0; i < nrhs; ++i) iters[i] += M.st_host[i].iters;
            // FP64 residual of the current solution
            dg::launch_brick<double>(dg::BM_RESIDDOT, L0, L0.dev64, nrhs, nullptr, W.x, nullptr, b, nullptr, W.r,
                                     nullptr, M.partial, M.pstride, 0, 0, s);
            dg::launch_finalize(dg::FIN_TRUE, nrhs, M.st, M.partial, M.pstride, nb, s);
            read_state(M, M.st, nrhs, s);
            bool again = false;
            for (int i = 0; i < nrhs; ++i) {
                const auto& S = M.st_host[i];
                const bool miss = S.bb > 0 && S.rr > S.tol2 * S.bb * 1.0201;  // (1.01 rtol)^2
                again |= miss && iters[i] < o.max_iter && !S.breakdown;
            }
            if (!again) break;
        }
        for (int i = 0; i < nrhs; ++i) outer[i] = 1;
        if (x0 && guard)
            for (int i = 0; i < nrhs; ++i) kept[i] = M.st_host[i].guess;
        HIPCHK(hipMemcpyAsync(v, W.x, sizeof(double) * n0 * nrhs, hipMemcpyDeviceToDevice, s));
    } else {
        ensure_work<float>(M, M.w32, nrhs);
        if (!M.r64) throw ArgError("internal: FP64 residual buffer missing");
        Work<float>& W = M.w32;
        init_state(M, M.st, nrhs, o.rtol, o.max_iter, s);
        dg::launch_dot<double, double>(n0, nrhs, nullptr, b, b, M.partial, M.pstride, s);
        dg::launch_finalize(dg::FIN_BB, nrhs, M.st, M.partial, M.pstride, nc, s);
        if (x0) dg::launch_copy(x0, v, n0 * nrhs, s);
        bool done = false;  // the last outer residual is that of the returned solution
        for (int it = 0; it < o.max_outer; ++it) {
            if (it == 0 && !x0) {
                // from x = 0 the first residual is b itself: v = 0, r = b, rr = bb
                dg::launch_guard(nrhs, n0, M.st, b, v, M.r64, true, true, s);
            } else {
                dg::launch_brick<double>(dg::BM_RESIDDOT, L0, L0.dev64, nrhs, nullptr, v, nullptr, b, nullptr,
                                         M.r64, nullptr, M.partial, M.pstride, 0, 0, s);
                dg::launch_finalize(dg::FIN_OUTER, nrhs, M.st, M.partial, M.pstride, nb, s);
                if (it == 0 && guard) dg::launch_guard(nrhs, n0, M.st, b, v, M.r64, true, false, s);
            }
            read_state(M, M.st, nrhs, s);
            if (it == 0 && x0 && guard)
                for (int i = 0; i < nrhs; ++i) kept[i] = M.st_host[i].guess;
            bool any = false;
            for (int i = 0; i < nrhs; ++i) {
                any |= M.st_host[i].active != 0;
                if (M.st_host[i].active) outer[i] += 1;
            }
            if (!any) {
                done = true;
                break;
            }
            dg::launch_to_inner(n0, nrhs, M.st, M.r64, W.r, s);
            dg::launch_fill<float>(W.x, 0.0f, n0 * nrhs, s);
            // inner state on ||r32|| = 1: relative tolerance inner_rtol, loosened for the last
            // refinement step to what the outer tolerance still needs, rtol ||b|| / ||r_k||
            dg::launch_inner_init(nrhs, M.st, M.st_in, o.rtol, o.inner_rtol, o.max_iter, s);
            pcg_run<float>(ctx, M, W, nrhs, M.st_in, M.st, it, s);
            for (int i = 0; i < nrhs; ++i) iters[i] += M.st_host[i].iters;
            dg::launch_correct(n0, nrhs, M.st, W.x, v, s);
        }
        if (!done) {
            // out of refinement steps: FP64 residual of the returned solution
            dg::launch_brick<double>(dg::BM_RESIDDOT, L0, L0.dev64, nrhs, nullptr, v, nullptr, b, nullptr, M.r64,
                                     nullptr, M.partial, M.pstride, 0, 0, s);
            dg::launch_finalize(dg::FIN_TRUE, nrhs, M.st, M.partial, M.pstride, nb, s);
            read_state(M, M.st, nrhs, s);
        }
        // Fallback: right-hand sides still above the tolerance after max_outer refinement steps
        // (an inner solve that stalls or breaks down) are finished by FP64 PCG from the current
        // iterate; converged ones stay inactive in it.  M.r64 holds b - A v of the current v.
        std::vector<char> miss(nrhs, 0);
        bool any_miss = false;
        for (int i = 0; i < nrhs; ++i) {
            const auto& S = M.st_host[i];
            miss[i] = std::isfinite(S.bb) && std::isfinite(S.rr) && S.bb > 0 && S.rr > S.tol2 * S.bb * 1.0201 &&
                      iters[i] < o.max_iter;
            any_miss |= miss[i] != 0;
        }
        if (any_miss) {
            ensure_work<double>(M, M.w64, nrhs);  // sized when the fallback first happens
            Work<double>& W = M.w64;
            dg::launch_copy(v, W.x, n0 * nrhs, s);
            dg::launch_copy(M.r64, W.r, n0 * nrhs, s);
            for (int i = 0; i < nrhs; ++i) outer[i] += miss[i];
            for (int restart = 0; restart < 3; ++restart) {
                pcg_run<double>(ctx, M, W, nrhs, M.st, nullptr, restart, s);
                for (int i = 0; i < nrhs; ++i) iters[i] += M.st_host[i].iters;
                dg::launch_brick<double>(dg::BM_RESIDDOT, L0, L0.dev64, nrhs, nullptr, W.x, nullptr, b, nullptr,
                                         W.r, nullptr, M.partial, M.pstride, 0, 0, s);
                dg::launch_finalize(dg::FIN_TRUE, nrhs, M.st, M.partial, M.pstride, nb, s);
                read_state(M, M.st, nrhs, s);
                bool again = false;
                for (int i = 0; i < nrhs; ++i) {
                    const auto& S = M.st_host[i];
                    again |= S.bb > 0 && S.rr > S.tol2 * S.bb * 1.0201 && iters[i] < o.max_iter && !S.breakdown;
                }
                if (!again) break;
            }
            HIPCHK(hipMemcpyAsync(v, W.x, sizeof(double) * n0 * nrhs, hipMemcpyDeviceToDevice, s));
        }
    }
    HIPCHK(hipGetLastError());
    // A NaN or Inf in a source, its Dirichlet data or a caller's initial guess leaves ||b||^2 or
    // the residual non-finite.  Such a right-hand side never became active (every comparison
    // with NaN is false), so it cost no iterations; the call reports an argument error.
    for (int i = 0; i < nrhs; ++i) {
        const auto& S = M.st_host[i];
        if (!std::isfinite(S.bb) || !std::isfinite(S.rr)) {
            HIPCHK(hipStreamSynchronize(s));
            throw ArgError("non-finite value (NaN or Inf) in the source, Dirichlet data or initial guess of a "
                           "right-hand side");
        }
    }
    if (stats) {
        for (int i = 0; i < nrhs; ++i) {
            const auto& S = M.st_host[i];
            dg_rhs_stats& r = stats[i];
            r.iters = iters[i];
            r.outer_iters = outer[i];
            r.guess_used = kept[i];
            r.rel_residual = S.bb > 0 ? std::sqrt(S.rr / S.bb) : 0.0;
            // breakdown: the last FP64 PCG pass stopped on a non-positive p.Ap or r.z
            r.status = (r.rel_residual <= o.rtol * 1.01) ? DG_OK : S.breakdown ? DG_ERR_BREAKDOWN : DG_WARN_NOT_CONVERGED;
        }
    }
}

// One solve on one solver lane: cnt right-hand sides b (already assembled) -> v.
struct Job {
    Mesh* M;
    int cnt;
    const double* b;
    const double* x0;
    double* v;
    dg_rhs_stats* stats;
    bool guard;  // x0 is a learned guess (guarded in the solve)
};

constexpr int kLaneMin = 16;  // smallest batch of one mesh that is split over lanes
constexpr int kLaneRhs = 8;   // fewest right-hand sides a lane takes

// Sizes the work space of a lane for cnt right-hand sides (on the calling thread, so
// that the solves allocate nothing).
void prepare_lane(dg_ctx* ctx, Mesh& M, int cnt) {
    const int prec = ctx->opts.precision;
    ensure_b(M, cnt, prec == DG_PREC_FP32_IR);
    ensure_state(M, cnt);
    if (use_fused(ctx, M))
        ensure_fused_ws(ctx, M, cnt);
    else if (prec == DG_PREC_FP32_IR)
        ensure_work<float>(M, M.w32, cnt);
    else if (prec == DG_PREC_FP32_PC || prec == DG_PREC_BF16_PC || prec == DG_PREC_BF16F_PC)
        ensure_work_pc(M, cnt, prec == DG_PREC_BF16_PC);
    else
        ensure_work<double>(M, M.w64, cnt);
}

// Appends the jobs of one mesh's batch: one job, or consecutive parts of nearly equal size on
// the mesh's lanes (as many lanes as the options give, each taking at least kLaneRhs right-hand
// sides).  guard: x0 is a learned guess.
void add_jobs(dg_ctx* ctx, int mesh_id, int cnt, const double* b, const double* x0, double* v, dg_rhs_stats* stats,
              bool guard, std::vector<Job>& jobs) {
    Mesh& M = ctx->meshes[mesh_id];
    const long long n0 = M.lv[0].ndof;
    const int nm = (int)ctx->meshes.size();
    const int nl = std::min(ctx->opts.lanes, std::max(1, cnt / kLaneRhs));
    if (ctx->twins.empty() || cnt < kLaneMin || nl < 2) {
        prepare_lane(ctx, M, cnt);
        jobs.push_back({&M, cnt, b, x0, v, stats, guard});
        return;
    }
    int first = 0;
    for (int k = 0; k < nl; ++k) {
        const int part = cnt / nl + (k >= nl - cnt % nl ? 1 : 0);  // the later lanes take the remainder
        Mesh& T = k == 0 ? M : ctx->twins[(size_t)(k - 1) * nm + mesh_id];
        prepare_lane(ctx, T, part);
        jobs.push_back({&T, part, b + first * n0, x0 ? x0 + first * n0 : nullptr, v + first * n0,
                        stats ? stats + first : nullptr, guard});
        first += part;
    }
}

// Runs the jobs: a single one on the caller's stream; several at once, each on its
// lane's stream from its own host thread (the host waits of one overlap the kernels of
// the others).  Results do not depend on how the jobs are run.
void run_jobs(dg_ctx* ctx, std::vector<Job>& jobs, hipStream_t stream) {
    if (jobs.size() == 1) {
        auto& J = jobs[0];
        solve_group(ctx, *J.M, J.cnt, J.b, J.x0, J.v, J.stats, stream, J.guard);
        return;
    }
    HIPCHK(hipEventRecord(ctx->ev_ready, stream));
    dg_ctx::Prof* prof = g_prof;
    std::vector<std::exception_ptr> err(jobs.size());
    std::vector<std::thread> th;
    for (size_t k = 0; k < jobs.size(); ++k) {
        th.emplace_back([&, k] {
            try {
                g_prof = prof;
                HIPCHK(hipSetDevice(ctx->device));
                auto& J = jobs[k];
                HIPCHK(hipStreamWaitEvent(J.M->stream, ctx->ev_ready, 0));
                solve_group(ctx, *J.M, J.cnt, J.b, J.x0, J.v, J.stats, J.M->stream, J.guard);
                HIPCHK(hipEventRecord(J.M->ev_done, J.M->stream));
            } catch (...) {
                err[k] = std::current_exception();
            }
        });
    }
    for (auto& t : th) t.join();
    for (auto& e : err)
        if (e) std::rethrow_exception(e);
    for (auto& J : jobs) HIPCHK(hipStreamWaitEvent(stream, J.M->ev_done, 0));
}

void learned_guess(dg_ctx* ctx, Mesh& M, int nrhs, const double* rho, hipStream_t s) {
    const long long n0 = M.lv[0].ndof;
    if (ctx->g_cap < n0 * nrhs) {
        dfree(ctx->g_x0);
        dfree(ctx->g_rho);
        ctx->g_x0 = dalloc<double>(n0 * nrhs);
        ctx->g_rho = dalloc<double>(n0 * nrhs);
        ctx->g_cap = n0 * nrhs;
    }
    const int mesh_id = (int)(&M - ctx->meshes.data());
    if (dg_net_guess(ctx->guess, ctx, mesh_id, nrhs, rho, ctx->g_x0, s) != DG_OK)
        throw ArgError(std::string("learned guess failed: ") + dg_net_last_error());
}

void setup_mesh(dg_ctx* ctx, const dg_mesh& mesh, Mesh& M, hipStream_t s) {
    const auto& o = ctx->opts;
    if (mesh.p < 1 || mesh.p > dg::NMAX - 1) throw ArgError("degree p must be in 1..7");
    for (int d = 0; d < 3; ++d) {
        if (mesh.ne[d] < 1) throw ArgError("element counts must be positive");
        if (!(mesh.hi[d] > mesh.lo[d])) throw ArgError("box must have positive extent");
    }
    M.mesh = mesh;
    // a single level (a small degree-1 mesh) is solved by PCG with the exact coarsest-level
    // solve as its preconditioner (build_coarse rejects one with more than CMAX nodes per axis)
    auto specs = dg::hierarchy(mesh.ne, mesh.p, o.n_levels);
    for (auto& [E, p] : specs) {
        LevelHost L;
        for (int d = 0; d < 3; ++d) {
            L.E[d] = E[d];
            L.h[d] = (mesh.hi[d] - mesh.lo[d]) / E[d];
            L.lo[d] = mesh.lo[d];
        }
        L.p = p;
        L.n = p + 1;
        L.ndof = (long long)E[0] * E[1] * E[2] * L.n * L.n * L.n;
        L.be = dg::brick_edge(L.n);
        L.family = o.node_family;
        for (int d = 0; d < 3; ++d) L.nbr[d] = (E[d] + L.be - 1) / L.be;
        dg::assign_tiles(L);
        if (L.family != 0)  // the slab kernels take face values at the end nodes: GL runs on the bricks
            for (int f = 0; f < 2; ++f)
                for (int m = 0; m <= dg::BM_RESTRICT; ++m) L.tile[f][m][0] = 0;
        for (int d = 0; d < 3; ++d) {
            dg::build_axis(E[d], p, mesh.lo[d], mesh.hi[d], o.penalty_eps, L.d64.ax[d], nullptr, nullptr, L.family);
            auto& a = L.d64.ax[d];
            auto& f = L.d32.ax[d];
            std::memset(&f, 0, sizeof(f));
            for (int t = 0; t < 4; ++t)
                for (int i = 0; i < dg::NMAX; ++i) {
                    for (int j = 0; j < dg::NMAX; ++j) f.B[t][i][j] = (float)a.B[t][i][j];
                    f.Bd[t][i] = (float)a.Bd[t][i];
                }
            for (int i = 0; i < dg::NMAX; ++i) {
                f.dL[i] = (float)a.dL[i];
                f.dR[i] = (float)a.dR[i];
                f.eL[i] = (float)a.eL[i];
                f.eR[i] = (float)a.eR[i];
                f.m[i] = (float)a.m[i];
                f.liftL[i] = (float)a.liftL[i];
                f.liftR[i] = (float)a.liftR[i];
            }
            f.sigma = (float)a.sigma;
            f.E = a.E;
            f.gl = a.gl;
        }
        dg::build_ref(p, o.penalty_eps, L.h, L.d64.ref);
        {
            const auto& r = L.d64.ref;
            auto& f = L.d32.ref;
            std::memset(&f, 0, sizeof(f));
            for (int i = 0; i < dg::NMAX; ++i) {
                for (int j = 0; j < dg::NMAX; ++j) f.B[i][j] = (float)r.B[i][j];
                f.aL[i] = (float)r.aL[i];
                f.aR[i] = (float)r.aR[i];
                f.w[i] = (float)r.w[i];
            }
            f.sig = (float)r.sig;
            for (int d = 0; d < 3; ++d) f.scale[d] = (float)r.scale[d];
            for (int i = 0; i < dg::NMAX / 2; ++i) {
                for (int l = 0; l < dg::NMAX / 2; ++l) {
                    f.Pe[i][l] = (float)r.Pe[i][l];
                    f.Po[i][l] = (float)r.Po[i][l];
                }
                f.qe[i] = (float)r.qe[i];
                f.qo[i] = (float)r.qo[i];
            }
            for (int i = 0; i <= dg::NMAX / 2; ++i) f.Bm[i] = (float)r.Bm[i];
            f.qm = (float)r.qm;
        }
        M.lv.push_back(L);
    }
    const int nl = (int)M.lv.size();
    for (int l = 0; l + 1 < nl; ++l) {
        LevelHost& F = M.lv[l];
        const LevelHost& C = M.lv[l + 1];
        F.hcoarse = F.E[0] != C.E[0];
        if (F.hcoarse && (F.be % 2 || F.n != 2 || C.n != 2)) throw ArgError("mesh coarsening only at p = 1");
        dg::build_transfer(F, C, F.tr);
    }
    dg::build_coarse(M.lv.back(), o.penalty_eps, M.coarse);
    // device copies
    for (auto& L : M.lv) {
        L.dev64 = dalloc<dg::LevelDev<double>>(1);
        L.dev32 = dalloc<dg::LevelDev<float>>(1);
        HIPCHK(hipMemcpy(L.dev64, &L.d64, sizeof(L.d64), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(L.dev32, &L.d32, sizeof(L.d32), hipMemcpyHostToDevice));
        L.devtr = dalloc<dg::TransferDev>(1);
        HIPCHK(hipMemcpy(L.devtr, &L.tr, sizeof(L.tr), hipMemcpyHostToDevice));
        L.dinv64 = dalloc<double>(L.ndof);
        L.dinv32 = dalloc<float>(L.ndof);
        dg::launch_dinv(L, s);
    }
    HIPCHK(hipStreamSynchronize(s));
    M.dcoarse = dalloc<dg::CoarseDev>(1);
    HIPCHK(hipMemcpy(M.dcoarse, &M.coarse, sizeof(M.coarse), hipMemcpyHostToDevice));
    int ps = dg::chunks_of(M.lv[0].ndof);
    for (auto& L : M.lv)
        for (int mode : {dg::BM_CHEBDOT, dg::BM_PQ, dg::BM_RESIDDOT})
            ps = std::max({ps, dg::bricks_of(L), dg::op_blocks<float>(L, mode), dg::op_blocks<double>(L, mode)});
    M.pstride = ps;
    const int NX = mesh.ne[0] * (mesh.p + 1), NY = mesh.ne[1] * (mesh.p + 1), NZ = mesh.ne[2] * (mesh.p + 1);
    M.nface = 2LL * ((long long)NY * NZ + (long long)NX * NZ + (long long)NX * NY);

    // smoother bounds: Lanczos on D^-1/2 A D^-1/2 per level (single vector)
    M.cheb.resize(nl);
    for (int l = 0; l + 1 < nl; ++l) {
        LevelHost& L = M.lv[l];
        const long long n = L.ndof;
        std::vector<double> h(n);
        double nrm = 0.0;
        for (long long i = 0; i < n; ++i) {
            uint32_t v = (uint32_t)((uint64_t)i * 2654435761ull + 12345ull);
            h[i] = (double)v / 4294967296.0 - 0.5;
            nrm += h[i] * h[i];
        }
        nrm = std::sqrt(nrm);
        for (auto& x : h) x /= nrm;
        double *v = dalloc<double>(n), *vp = dalloc<double>(n), *w = dalloc<double>(n), *tmp = dalloc<double>(n);
        double* part = dalloc<double>(dg::chunks_of(n));
        HIPCHK(hipMemcpy(v, h.data(), sizeof(double) * n, hipMemcpyHostToDevice));
        dg::launch_fill<double>(vp, 0.0, n, s);
        std::vector<double> alphas, betas, hp(dg::chunks_of(n));
        auto dot = [&](const double* a, const double* b) {
            dg::launch_dot<double, double>(n, 1, nullptr, a, b, part, dg::chunks_of(n), s);
            HIPCHK(hipMemcpyAsync(hp.data(), part, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            double acc = 0.0;
            for (double x : hp) acc += x;
            return acc;
        };
        double beta = 0.0;
        const int steps = (int)std::min<long long>(o.lanczos_steps, n);
        for (int k = 0; k < steps; ++k) {
            dg::launch_dscale(L, L.dev64, v, tmp, s);
            dg::launch_brick<double>(dg::BM_APPLY, L, L.dev64, 1, nullptr, tmp, nullptr, nullptr, nullptr, w, nullptr,
                                     nullptr, 0, 0, 0, s);
            dg::launch_dscale(L, L.dev64, w, w, s);
            dg::launch_axpby(n, -beta, vp, 1.0, w, s);
            const double alpha = dot(w, v);
            dg::launch_axpby(n, -alpha, v, 1.0, w, s);
            alphas.push_back(alpha);
            beta = std::sqrt(std::max(0.0, dot(w, w)));
            if (k == steps - 1 || beta == 0.0) break;
            betas.push_back(beta);
            std::swap(v, vp);          // vp <- v (old)
            dg::launch_copy(w, v, n, s);
            dg::launch_axpby(n, 0.0, w, 1.0 / beta, v, s);  // v = w / beta
        }
        HIPCHK(hipStreamSynchronize(s));
        HIPCHK(hipGetLastError());
        dfree(v); dfree(vp); dfree(w); dfree(tmp); dfree(part);
        betas.resize(alphas.size() > 0 ? alphas.size() - 1 : 0);
        const double lmax = dg::tridiag_max_eig(alphas, betas);
        L.lam_hi = o.cheb_safety * lmax;
        L.lam_lo = L.lam_hi / o.cheb_ratio;
        const double theta = 0.5 * (L.lam_hi + L.lam_lo), delta = 0.5 * (L.lam_hi - L.lam_lo);
        const double sigma1 = theta / delta;
        ChebCoef C;
        C.c0 = 1.0 / theta;
        double rho = 1.0 / sigma1;
        const int degree = (l >= 1 && L.p == 1 && o.cheb_degree_h > 0) ? o.cheb_degree_h : o.cheb_degree;
        for (int k = 1; k < degree; ++k) {
            const double rn = 1.0 / (2.0 * sigma1 - rho);
            C.cp.push_back(rn * rho);
            C.cr.push_back(2.0 * rn / delta);
            rho = rn;
        }
        M.cheb[l] = C;
    }
    build_fused(M);
}

}  // namespace

namespace {
dg_status run_guarded(const std::function<void()>& fn) {
    try {
        fn();
        return DG_OK;
    } catch (const ArgError& e) {
        set_err("%s", e.what());
        return DG_ERR_ARG;
    } catch (const HipError& e) {
        set_err("%s", e.what());
        return DG_ERR_HIP;
    } catch (const std::bad_alloc&) {
        set_err("host allocation failed");
        return DG_ERR_OOM;
    } catch (const std::exception& e) {
        set_err("%s", e.what());
        return DG_ERR_ARG;
    }
}
}  // namespace

namespace dg {
dg_status guarded(const std::function<void()>& fn) { return run_guarded(fn); }
void hip_fail(const std::string& what) { throw HipError(what); }

const LevelHost& ctx_fine_level(const dg_ctx* ctx, int mesh_id) {
    check_mesh_id(ctx, mesh_id);
    return ctx->meshes[mesh_id].lv[0];
}
const LevelHost& ctx_level(const dg_ctx* ctx, int mesh_id, int level) {
    check_mesh_id(ctx, mesh_id);
    const auto& M = ctx->meshes[mesh_id];
    if (level < 0 || level >= (int)M.lv.size()) throw std::runtime_error("level out of range");
    return M.lv[level];
}
}  // namespace dg

extern "C" {

void dg_opts_default(dg_opts* o) {
    if (!o) return;
    o->n_levels = 0;
    o->cheb_degree = 6;
    o->cheb_ratio = 60.0;
    o->cheb_safety = 1.1;
    o->lanczos_steps = 30;
    o->penalty_eps = 0.125;
    o->rtol = 1e-8;
    o->max_iter = 500;
    o->precision = DG_PREC_FP64;
    o->inner_rtol = 1e-4;
    o->max_outer = 8;
    o->check_every = 2;
    o->lanes = 2;
    o->use_graph = 1;
    o->cheb_degree_h = 10;
    o->fused = 0;
    o->fused_wgs = 0;
    o->fused_spin = 0;
    o->node_family = 0;
    o->learned_cgc = 0;
}

const char* dg_status_string(dg_status s) {
    switch (s) {
        case DG_OK: return "ok";
        case DG_WARN_NOT_CONVERGED: return "not converged";
        case DG_ERR_ARG: return "invalid argument";
        case DG_ERR_HIP: return "HIP runtime error";
        case DG_ERR_OOM: return "out of memory";
        case DG_ERR_BREAKDOWN: return "CG breakdown";
        case DG_ERR_STATE: return "invalid state";
    }
    return "unknown status";
}

const char* dg_last_error(void) { return g_err.c_str(); }

dg_status dg_poisson_setup(const dg_mesh* meshes, int n_meshes, const dg_opts* opts, dg_ctx** out) {
    return run_guarded([&] {
        if (!meshes || n_meshes < 1 || !out) throw ArgError("need at least one mesh and an output pointer");
        auto ctx = std::make_unique<dg_ctx>();
        if (opts)
            ctx->opts = *opts;
        else
            dg_opts_default(&ctx->opts);
        const auto& o = ctx->opts;
        if (o.cheb_degree < 1 || o.cheb_degree_h < 0 || o.cheb_ratio <= 1.0 || o.cheb_safety < 1.0 || o.lanczos_steps < 2 ||
            o.penalty_eps <= 0 || o.rtol <= 0 || o.max_iter < 1 || o.max_outer < 1 || o.inner_rtol <= 0 ||
            o.inner_rtol >= 1 || o.lanes < 1 || o.lanes > 4 ||
            (o.precision != DG_PREC_FP64 && o.precision != DG_PREC_FP32_IR && o.precision != DG_PREC_FP32_PC &&
             o.precision != DG_PREC_BF16_PC && o.precision != DG_PREC_BF16F_PC) ||
            o.node_family < 0 || o.node_family > 1)
            throw ArgError("invalid solver options");
        if (o.node_family != 0 && o.fused != 0) throw ArgError("the fused solves need Gauss-Lobatto nodes");
        if (o.learned_cgc < 0 || (o.learned_cgc > 0 && (o.precision != DG_PREC_FP64 || o.lanes != 1 || o.fused != 0)))
            throw ArgError("the learned coarse-grid correction runs in FP64 precision on one solver lane, unfused");
        HIPCHK(hipGetDevice(&ctx->device));
        HIPCHK(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&ctx->ev_in, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&ctx->ev_out, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&ctx->ev_ready, hipEventDisableTiming));
        hipStream_t s = ctx->stream;
        ctx->meshes.resize(n_meshes);
        // the fixed work space of the entry point that allocates nothing: this device's copy
        HIPCHK(dg::quad_scratch_init(ctx->device));
        for (int i = 0; i < n_meshes; ++i) {
            setup_mesh(ctx.get(), meshes[i], ctx->meshes[i], s);
            build_qnodes(ctx.get(), ctx->meshes[i]);
            HIPCHK(hipStreamCreateWithFlags(&ctx->meshes[i].stream, hipStreamNonBlocking));
            HIPCHK(hipEventCreateWithFlags(&ctx->meshes[i].ev_done, hipEventDisableTiming));
        }
        if (o.lanes >= 2) {
            // the further lanes of a mesh: the same (read-only) level tables, their own work space
            ctx->twins.resize((size_t)(o.lanes - 1) * n_meshes);
            for (size_t q = 0; q < ctx->twins.size(); ++q) {
                const Mesh& M = ctx->meshes[q % n_meshes];
                Mesh& T = ctx->twins[q];
                T.mesh = M.mesh;
                T.lv = M.lv;
                T.cheb = M.cheb;
                T.coarse = M.coarse;
                T.dcoarse = M.dcoarse;
                T.dfused = M.dfused;
                T.fws_per = M.fws_per;
                T.fused_lds_ok = M.fused_lds_ok;
                T.fws_group = M.fws_group;
                T.pstride = M.pstride;
                T.nface = M.nface;
                T.owns_tables = false;
                HIPCHK(hipStreamCreateWithFlags(&T.stream, hipStreamNonBlocking));
                HIPCHK(hipEventCreateWithFlags(&T.ev_done, hipEventDisableTiming));
            }
        }
        HIPCHK(hipDeviceSynchronize());
        *out = ctx.release();
    });
}

void dg_poisson_destroy(dg_ctx* ctx) {
    if (!ctx) return;
    (void)hipDeviceSynchronize();
    for (auto& M : ctx->twins) ctx->meshes.push_back(std::move(M));  // lanes are freed like meshes
    ctx->twins.clear();
    for (auto& M : ctx->meshes) {
        if (M.owns_tables) {
            for (auto& L : M.lv) {
                dfree(L.dev64);
                dfree(L.dev32);
                dfree(L.devtr);
                dfree(L.dinv64);
                dfree(L.dinv32);
            }
            dfree(M.dcoarse);
            dfree(M.dfused);
            for (auto* p : M.fusedP) dfree(p);
        }
        dfree(M.fws);
        dfree(M.gsync);
        dfree(M.cscr);
        dfree(M.lc_rho);
        dfree(M.lc_c);
        M.w64.release();
        M.w32.release();
        dfree(M.b);
        dfree(M.r64);
        dfree(M.partial);
        dfree(M.st);
        dfree(M.st_in);
        if (M.st_host) (void)hipHostFree(M.st_host);
        dfree(M.grho);
        dfree(M.gface);
        dfree(M.gx0);
        dfree(M.gv);
        dfree(M.qnodes);
        if (M.ev_done) (void)hipEventDestroy(M.ev_done);
        if (M.stream) (void)hipStreamDestroy(M.stream);
        for (auto e : M.pev) (void)hipEventDestroy(e);
    }
    for (auto e : ctx->prof.ev) (void)hipEventDestroy(e);
    for (auto& M : ctx->meshes) {
        drop_graphs(M);
        for (auto& G : M.graph)
            for (auto e : G.ev) (void)hipEventDestroy(e);
    }
    if (ctx->ev_in) (void)hipEventDestroy(ctx->ev_in);
    if (ctx->ev_out) (void)hipEventDestroy(ctx->ev_out);
    if (ctx->ev_ready) (void)hipEventDestroy(ctx->ev_ready);
    dfree(ctx->segtab);
    if (ctx->segtab_host) (void)hipHostFree(ctx->segtab_host);
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    dfree(ctx->g_x0);
    dfree(ctx->g_rho);
    dfree(ctx->xv);
    dfree(ctx->xpart);
    dfree(ctx->xpairs);
    dfree(ctx->qrec);
    dfree(ctx->qpart);
    dfree(ctx->qg);
    dfree(ctx->cpart);
    dfree(ctx->crho);
    dfree(ctx->cv);
    dfree(ctx->cW);
    dfree(ctx->csmall);
    dfree(ctx->cflag);
    delete ctx;
}

dg_status dg_mesh_info(const dg_ctx* ctx, int mesh_id, long long* n_dofs, long long* n_face, int* n_levels) {
    return run_guarded([&] {
        check_mesh_id(ctx, mesh_id);
        const auto& M = ctx->meshes[mesh_id];
        if (n_dofs) *n_dofs = M.lv[0].ndof;
        if (n_face) *n_face = M.nface;
        if (n_levels) *n_levels = (int)M.lv.size();
    });
}

dg_status dg_level_info(const dg_ctx* ctx, int mesh_id, int level, int* ne, int* p, double* lam_lo, double* lam_hi) {
    return run_guarded([&] {
        check_mesh_id(ctx, mesh_id);
        const auto& M = ctx->meshes[mesh_id];
        if (level < 0 || level >= (int)M.lv.size()) throw ArgError("level out of range");
        const auto& L = M.lv[level];
        if (ne) for (int d = 0; d < 3; ++d) ne[d] = L.E[d];
        if (p) *p = L.p;
        if (lam_lo) *lam_lo = L.lam_lo;
        if (lam_hi) *lam_hi = L.lam_hi;
    });
}

dg_status dg_mesh_coords(const dg_ctx* ctx, int mesh_id, double* xyz, double* fxyz) {
    return run_guarded([&] {
        check_mesh_id(ctx, mesh_id);
        const auto& M = ctx->meshes[mesh_id];
        const auto& m = M.mesh;
        const int n = m.p + 1;
        std::vector<double> nodes[3];
        for (int d = 0; d < 3; ++d) {
            dg::AxisDev<double> ax;
            dg::build_axis(m.ne[d], m.p, m.lo[d], m.hi[d], ctx->opts.penalty_eps, ax, nullptr, &nodes[d],
                           ctx->opts.node_family);
        }
        const long long ndof = M.lv[0].ndof;
        if (xyz) {
            for (long long q = 0; q < ndof; ++q) {
                const long long e = q / (n * n * n);
                const int l = (int)(q % (n * n * n));
                const int ex = (int)(e % m.ne[0]), ey = (int)((e / m.ne[0]) % m.ne[1]), ez = (int)(e / (m.ne[0] * m.ne[1]));
                const int i = l % n, j = (l / n) % n, k = l / (n * n);
                xyz[q] = nodes[0][ex * n + i];
                xyz[ndof + q] = nodes[1][ey * n + j];
                xyz[2 * ndof + q] = nodes[2][ez * n + k];
            }
        }
        if (fxyz) {
            const int NX = m.ne[0] * n, NY = m.ne[1] * n, NZ = m.ne[2] * n;
            const long long nf = M.nface;
            long long o = 0;
            auto put = [&](double x, double y, double z) {
                fxyz[o] = x;
                fxyz[nf + o] = y;
                fxyz[2 * nf + o] = z;
                ++o;
            };
            for (int side = 0; side < 2; ++side)  // x faces [Z][Y]
                for (int Z = 0; Z < NZ; ++Z)
                    for (int Y = 0; Y < NY; ++Y) put(side ? m.hi[0] : m.lo[0], nodes[1][Y], nodes[2][Z]);
            for (int side = 0; side < 2; ++side)  // y faces [Z][X]
                for (int Z = 0; Z < NZ; ++Z)
                    for (int X = 0; X < NX; ++X) put(nodes[0][X], side ? m.hi[1] : m.lo[1], nodes[2][Z]);
            for (int side = 0; side < 2; ++side)  // z faces [Y][X]
                for (int Y = 0; Y < NY; ++Y)
                    for (int X = 0; X < NX; ++X) put(nodes[0][X], nodes[1][Y], side ? m.hi[2] : m.lo[2]);
        }
    });
}

// Status of a call whose right-hand sides all ran: a breakdown that the FP64 restarts could not
// cure first, then a missed tolerance.
static dg_status worst_status(const dg_rhs_stats* stats, int n) {
    dg_status w = DG_OK;
    for (int i = 0; i < n; ++i) {
        if (stats[i].status == DG_ERR_BREAKDOWN) return DG_ERR_BREAKDOWN;
        if (stats[i].status != DG_OK) w = DG_WARN_NOT_CONVERGED;
    }
    return w;
}

dg_status dg_poisson_solve_batch(dg_ctx* ctx, int nrhs, const int* mesh_id, const double* rho, const double* g,
                                 const double* x0, double* v, dg_rhs_stats* stats, hipStream_t stream) {
    std::vector<dg_rhs_stats> all;  // every right-hand side's statistics, whether or not the caller takes them
    dg_status st = run_guarded([&] {
        if (!ctx) throw ArgError("null context");
        if (ctx->opts.learned_cgc > 0 && !ctx->guess)
            throw ArgError("the learned coarse-grid correction needs an attached guess network");
        g_prof = &ctx->prof;
        if (nrhs < 0) throw ArgError("nrhs must be >= 0");
        if (nrhs == 0) return;
        if (!mesh_id || !rho || !v) throw ArgError("null pointer argument");
        for (int i = 0; i < nrhs; ++i) check_mesh_id(ctx, mesh_id[i]);
        const hipStream_t user = stream;
        stream = enter(ctx, user);
        const bool fp32 = ctx->opts.precision == DG_PREC_FP32_IR;
        std::vector<long long> off(nrhs + 1, 0), foff(nrhs + 1, 0);
        for (int i = 0; i < nrhs; ++i) {
            off[i + 1] = off[i] + ctx->meshes[mesh_id[i]].lv[0].ndof;
            foff[i + 1] = foff[i] + ctx->meshes[mesh_id[i]].nface;
        }
        // One part per mesh: all of its right-hand sides, in the caller's order, solved
        // together whatever the interleaving (gathered when they are not contiguous).
        struct Part {
            int m = 0, cnt = 0;
            bool contig = true, guessed = false;
            long long tab = 0;  // offset-table position (non-contiguous parts)
            const double *rho = nullptr, *g = nullptr, *x0 = nullptr;
            double* v = nullptr;
            std::vector<int> idx;
            std::vector<dg_rhs_stats> stats;
        };
        std::vector<Part> parts;
        {
            std::vector<int> pos(ctx->meshes.size(), -1);
            for (int i = 0; i < nrhs; ++i) {
                int& k = pos[mesh_id[i]];
                if (k < 0) {
                    k = (int)parts.size();
                    parts.emplace_back();
                    parts.back().m = mesh_id[i];
                }
                parts[k].idx.push_back(i);
            }
        }
        long long ntab = 0;
        for (auto& P : parts) {
            P.cnt = (int)P.idx.size();
            P.contig = P.idx.back() - P.idx.front() + 1 == P.cnt;
            P.stats.assign(P.cnt, dg_rhs_stats{});
            if (!P.contig) {
                P.tab = ntab;
                ntab += 4LL * P.cnt;
            }
        }
        if (ntab > 0) {
            // tables A = caller offsets, B = packed offsets (fields); C, D the same for the faces
            if (ctx->segtab_cap < ntab) {
                dfree(ctx->segtab);
                if (ctx->segtab_host) (void)hipHostFree(ctx->segtab_host);
                ctx->segtab_host = nullptr;
                ctx->segtab = dalloc<long long>(ntab);
                HIPCHK(hipHostMalloc((void**)&ctx->segtab_host, sizeof(long long) * ntab, hipHostMallocDefault));
                ctx->segtab_cap = ntab;
            }
            for (auto& P : parts) {
                if (P.contig) continue;
                const Mesh& M = ctx->meshes[P.m];
                long long* t = ctx->segtab_host + P.tab;
                for (int q = 0; q < P.cnt; ++q) {
                    t[q] = off[P.idx[q]];
                    t[P.cnt + q] = q * M.lv[0].ndof;
                    t[2 * P.cnt + q] = foff[P.idx[q]];
                    t[3 * P.cnt + q] = q * M.nface;
                }
            }
            HIPCHK(hipMemcpyAsync(ctx->segtab, ctx->segtab_host, sizeof(long long) * ntab, hipMemcpyHostToDevice,
                                  stream));
        }
        for (auto& P : parts) {
            Mesh& M = ctx->meshes[P.m];
            const long long n0 = M.lv[0].ndof;
            const int cnt = P.cnt;
            ensure_b(M, cnt, fp32);  // the assembled right-hand sides of the whole part
            const bool want_guess = !x0 && ctx->guess;
            if ((!P.contig || want_guess || !g) && M.cap_g < cnt) {
                dfree(M.grho);
                dfree(M.gface);
                dfree(M.gx0);
                dfree(M.gv);
                M.grho = dalloc<double>(n0 * cnt);
                M.gface = dalloc<double>(M.nface * cnt);
                M.gx0 = dalloc<double>(n0 * cnt);
                M.gv = dalloc<double>(n0 * cnt);
                M.cap_g = cnt;
            }
            if (P.contig) {
                const int i0 = P.idx.front();
                P.rho = rho + off[i0];
                P.g = g ? g + foff[i0] : nullptr;
                P.x0 = x0 ? x0 + off[i0] : nullptr;
                P.v = v + off[i0];
            } else {
                const long long* t = ctx->segtab + P.tab;
                dg::launch_segcopy(rho, t, M.grho, t + cnt, n0, cnt, stream);
                if (g) dg::launch_segcopy(g, t + 2 * cnt, M.gface, t + 3 * cnt, M.nface, cnt, stream);
                if (x0) dg::launch_segcopy(x0, t, M.gx0, t + cnt, n0, cnt, stream);
                P.rho = M.grho;
                P.g = M.gface;
                P.x0 = x0 ? M.gx0 : nullptr;
                P.v = M.gv;
            }
            if (!g) {
                // no Dirichlet data given: computed from the sources by quadrature (Sec. 6.3)
                quad_data(ctx, M, cnt, P.rho, nullptr, nullptr, nullptr, M.gface, stream);
                P.g = M.gface;
            }
            dg::launch_rhs(M.lv[0], M.lv[0].dev64, cnt, P.rho, nullptr, nullptr, nullptr, P.g, M.nface, M.b, stream);
            if (want_guess) {
                if (ctx->g_cap < n0 * cnt) {
                    dfree(ctx->g_x0);
                    dfree(ctx->g_rho);
                    ctx->g_x0 = dalloc<double>(n0 * cnt);
                    ctx->g_rho = dalloc<double>(n0 * cnt);
                    ctx->g_cap = n0 * cnt;
                }
                learned_guess(ctx, M, cnt, P.rho, stream);
                dg::launch_copy(ctx->g_x0, M.gx0, n0 * cnt, stream);  // the guess buffer is shared by the parts
                P.x0 = M.gx0;
                P.guessed = true;
            }
        }
        // every buffer is sized here, on this thread: the solves allocate nothing (but for the
        // FP64 fallback of a mixed-precision solve, sized when it first happens)
        std::vector<Job> jobs;
        for (auto& P : parts)
            add_jobs(ctx, P.m, P.cnt, ctx->meshes[P.m].b, P.x0, P.v, P.stats.data(), P.guessed, jobs);
        run_jobs(ctx, jobs, stream);
        for (auto& P : parts) {
            if (!P.contig) {
                const long long* t = ctx->segtab + P.tab;
                dg::launch_segcopy(P.v, t + P.cnt, v, t, ctx->meshes[P.m].lv[0].ndof, P.cnt, stream);
            }
            all.resize(nrhs);
            for (int q = 0; q < P.cnt; ++q) all[P.idx[q]] = P.stats[q];
        }
        if (stats) std::copy(all.begin(), all.end(), stats);
        HIPCHK(hipStreamSynchronize(stream));
        leave(ctx, user);
    });
    return st == DG_OK ? worst_status(all.data(), (int)all.size()) : st;
}

dg_status dg_exchange_apply(dg_ctx* ctx, int mesh_id, int norb, const double* phi, const double* g_pairs, double* W,
                            double* K_pairs, double* E_x, double* v_pairs, dg_rhs_stats* stats, hipStream_t stream) {
    std::vector<dg_rhs_stats> st_all;  // every pair's statistics, whether or not the caller takes them
    dg_status st = run_guarded([&] {
        check_mesh_id(ctx, mesh_id);
        g_prof = &ctx->prof;
        if (ctx->opts.learned_cgc > 0 && !ctx->guess)
            throw ArgError("the learned coarse-grid correction needs an attached guess network");
        if (norb < 1 || norb > 32) throw ArgError("norb must be in 1..32");
        if (!phi || !W || !K_pairs) throw ArgError("null pointer argument");
        const hipStream_t user = stream;
        stream = enter(ctx, user);
        Mesh& M = ctx->meshes[mesh_id];
        const int npairs = norb * (norb + 1) / 2;
        const long long n0 = M.lv[0].ndof;
        std::vector<int> hp(2 * npairs);
        int q = 0;
        for (int i = 0; i < norb; ++i)
            for (int j = i; j < norb; ++j, ++q) {
                hp[q] = i;
                hp[npairs + q] = j;
            }
        if (ctx->xpairs_cap < 2 * npairs) {
            dfree(ctx->xpairs);
            ctx->xpairs = dalloc<int>(2 * npairs);
            ctx->xpairs_cap = 2 * npairs;
        }
        HIPCHK(hipMemcpyAsync(ctx->xpairs, hp.data(), sizeof(int) * 2 * npairs, hipMemcpyHostToDevice, stream));
        double* v = v_pairs;
        if (!v) {
            if (ctx->xv_cap < n0 * npairs) {
                dfree(ctx->xv);
                ctx->xv = dalloc<double>(n0 * npairs);
                ctx->xv_cap = n0 * npairs;
            }
            v = ctx->xv;
        }
        ensure_b(M, npairs, ctx->opts.precision == DG_PREC_FP32_IR);
        if (!g_pairs) {
            ensure_len(ctx->qg, ctx->qg_cap, (long long)npairs * M.nface);
            quad_data(ctx, M, npairs, nullptr, phi, ctx->xpairs, ctx->xpairs + npairs, ctx->qg, stream);
            g_pairs = ctx->qg;
        }
        dg::launch_rhs(M.lv[0], M.lv[0].dev64, npairs, nullptr, phi, ctx->xpairs, ctx->xpairs + npairs, g_pairs,
                       M.nface, M.b, stream);
        if (ctx->guess) {
            if (ctx->g_cap < n0 * npairs) {
                dfree(ctx->g_x0);
                dfree(ctx->g_rho);
                ctx->g_x0 = dalloc<double>(n0 * npairs);
                ctx->g_rho = dalloc<double>(n0 * npairs);
                ctx->g_cap = n0 * npairs;
            }
            dg::launch_pair_products(n0, npairs, phi, ctx->xpairs, ctx->xpairs + npairs, ctx->g_rho, stream);
            learned_guess(ctx, M, npairs, ctx->g_rho, stream);
        }
        st_all.assign(npairs, dg_rhs_stats{});
        std::vector<Job> jobs;
        add_jobs(ctx, mesh_id, npairs, M.b, ctx->guess ? ctx->g_x0 : nullptr, v, st_all.data(), ctx->guess != nullptr,
                 jobs);
        run_jobs(ctx, jobs, stream);
        if (stats) std::copy(st_all.begin(), st_all.end(), stats);
        const int nblk = (int)((n0 + 255) / 256);
        if (ctx->xpart_cap < (long long)npairs * nblk) {
            dfree(ctx->xpart);
            ctx->xpart = dalloc<double>((long long)npairs * nblk);
            ctx->xpart_cap = (long long)npairs * nblk;
        }
        dg::launch_exchange(M.lv[0], M.lv[0].dev64, norb, phi, v, W, ctx->xpart, nblk, stream);
        dg::launch_sum_partials(npairs, ctx->xpart, nblk, nblk, K_pairs, stream);
        std::vector<double> K(npairs);
        HIPCHK(hipMemcpyAsync(K.data(), K_pairs, sizeof(double) * npairs, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        HIPCHK(hipGetLastError());
        leave(ctx, user);
        double ex = 0.0;
        q = 0;
        for (int i = 0; i < norb; ++i)
            for (int j = i; j < norb; ++j, ++q) ex += (i == j ? 1.0 : 2.0) * K[q];
        if (E_x) *E_x = ex;
    });
    return st == DG_OK ? worst_status(st_all.data(), (int)st_all.size()) : st;
}

// ---- consumers of the potentials (Sec. 6.1, Sec. 7.2)

namespace {

// out = quadrature projection (phi_i, f u_a) on the mesh's finest level, on stream s.
void project(dg_ctx* ctx, Mesh& M, int nbasis, const double* phi, int nu, const double* u, const double* f,
             double* out, hipStream_t s) {
    ensure_len(ctx->cpart, ctx->cpart_cap, (long long)nbasis * nu * dg::project_chunks(M.lv[0].ndof));
    dg::launch_project(M.lv[0], nbasis, phi, nu, u, f, ctx->cpart, out, s);
}

}  // namespace

dg_status dg_hartree_action(dg_ctx* ctx, int mesh_id, int nbasis, const double* phi, int nu, const double* u,
                            const double* vH, double* out, hipStream_t stream) {
    return run_guarded([&] {
        check_mesh_id(ctx, mesh_id);
        if (nbasis < 1 || nu < 1 || (long long)nbasis * nu > (1LL << 24)) throw ArgError("bad nbasis or nu");
        if (!phi || !u || !vH || !out) throw ArgError("null pointer argument");
        const hipStream_t user = stream;
        stream = enter(ctx, user);
        project(ctx, ctx->meshes[mesh_id], nbasis, phi, nu, u, vH, out, stream);
        HIPCHK(hipGetLastError());
        leave(ctx, user);
    });
}

dg_status dg_exchange_action(dg_ctx* ctx, int mesh_id, int nbasis, const double* phi, int nu, const double* u,
                             int nocc, const double* psi, const double* g_pairs, double* out, double* W,
                             dg_rhs_stats* stats, hipStream_t stream) {
    std::vector<dg_rhs_stats> all;
    dg_status solve_status = DG_OK;
    dg_status st = run_guarded([&] {
        check_mesh_id(ctx, mesh_id);
        if (nbasis < 1 || nu < 1 || nocc < 1 || nocc > 64 || nu * nocc > 4096 || (long long)nbasis * nu > (1LL << 24))
            throw ArgError("bad nbasis, nu or nocc");
        if (!phi || !u || !psi || !out) throw ArgError("null pointer argument");
        const hipStream_t user = stream;
        stream = enter(ctx, user);
        Mesh& M = ctx->meshes[mesh_id];
        const long long n0 = M.lv[0].ndof;
        const int npairs = nu * nocc;
        ensure_len(ctx->crho, ctx->crho_cap, n0 * npairs);
        ensure_len(ctx->cv, ctx->cv_cap, n0 * npairs);
        dg::launch_cross_products(n0, nu, nocc, u, psi, ctx->crho, stream);
        // the pair problems, solved as one batch of the mesh (quadrature data when none is given)
        std::vector<int> ids(npairs, mesh_id);
        all.assign(npairs, dg_rhs_stats{});
        solve_status = dg_poisson_solve_batch(ctx, npairs, ids.data(), ctx->crho, g_pairs, nullptr, ctx->cv,
                                              all.data(), stream);
        if (solve_status < 0) throw std::runtime_error(std::string("pair solves: ") + g_err);
        double* w = W;
        if (!w) {
            ensure_len(ctx->cW, ctx->cW_cap, n0 * nu);
            w = ctx->cW;
        }
        dg::launch_cross_w(n0, nu, nocc, psi, ctx->cv, w, stream);
        project(ctx, M, nbasis, phi, nu, w, nullptr, out, stream);
        HIPCHK(hipStreamSynchronize(stream));
        HIPCHK(hipGetLastError());
        leave(ctx, user);
        if (stats) std::copy(all.begin(), all.end(), stats);
    });
    return st == DG_OK ? solve_status : st;
}

dg_status dg_ace_build(dg_ctx* ctx, int mesh_id, int nocc, const double* psi, const double* W, double* xi,
                       hipStream_t stream) {
    int bad = 0;
    dg_status st = run_guarded([&] {
        check_mesh_id(ctx, mesh_id);
        if (nocc < 1 || nocc > 64) throw ArgError("nocc must be in 1..64");
        if (!psi || !W || !xi) throw ArgError("null pointer argument");
        const hipStream_t user = stream;
        stream = enter(ctx, user);
        Mesh& M = ctx->meshes[mesh_id];
        ensure_len(ctx->csmall, ctx->csmall_cap, 2LL * nocc * nocc);
        if (!ctx->cflag) ctx->cflag = dalloc<int>(1);
        double* Mm = ctx->csmall;
        double* T = ctx->csmall + (long long)nocc * nocc;
        project(ctx, M, nocc, psi, nocc, W, nullptr, Mm, stream);  // M_kl = (psi_k, W_l)
        dg::launch_ace_factor(nocc, Mm, T, ctx->cflag, stream);
        dg::launch_ace_combine(M.lv[0].ndof, nocc, T, W, xi, stream);
        HIPCHK(hipMemcpyAsync(&bad, ctx->cflag, sizeof(int), hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        HIPCHK(hipGetLastError());
        leave(ctx, user);
        if (bad) set_err("exchange overlap matrix (psi_k, W_l) is not positive definite");
    });
    return st == DG_OK && bad ? DG_ERR_BREAKDOWN : st;
}

dg_status dg_ace_action(dg_ctx* ctx, int mesh_id, int nbasis, const double* phi, int nu, const double* u, int nocc,
                        const double* xi, double* out, hipStream_t stream) {
    return run_guarded([&] {
        check_mesh_id(ctx, mesh_id);
        if (nbasis < 1 || nu < 1 || nocc < 1 || nocc > 64 || (long long)nbasis * nu > (1LL << 24))
            throw ArgError("bad nbasis, nu or nocc");
        if (!phi || !u || !xi || !out) throw ArgError("null pointer argument");
        const hipStream_t user = stream;
        stream = enter(ctx, user);
        Mesh& M = ctx->meshes[mesh_id];
        ensure_len(ctx->csmall, ctx->csmall_cap, (long long)nocc * (nbasis + nu));
        double* A = ctx->csmall;                         // (phi_i, xi_k)   [nbasis][nocc]
        double* B = ctx->csmall + (long long)nbasis * nocc;  // (xi_k, u_a) [nocc][nu]
        project(ctx, M, nbasis, phi, nocc, xi, nullptr, A, stream);
        project(ctx, M, nocc, xi, nu, u, nullptr, B, stream);
        dg::launch_small_gemm(nbasis, nocc, nu, A, B, out, stream);
        HIPCHK(hipGetLastError());
        leave(ctx, user);
    });
}

dg_status dg_pair_densities(long long n_dofs, int norb, int first_pair, int npairs, const double* phi, double* rho,
                            hipStream_t stream) {
    return run_guarded([&] {
        const long long total = (long long)norb * (norb + 1) / 2;
        if (n_dofs < 0 || norb < 1 || first_pair < 0 || npairs < 0 || first_pair + (long long)npairs > total)
            throw ArgError("bad pair range");
        if (npairs > 65535) throw ArgError("at most 65535 pairs per call");
        if (npairs == 0 || n_dofs == 0) return;
        if (!phi || !rho) throw ArgError("null pointer argument");
        dg::launch_pair_densities(n_dofs, norb, first_pair, npairs, phi, rho, stream);
        HIPCHK(hipGetLastError());
    });
}

dg_status dg_boundary_data(dg_ctx* ctx, int mesh_id, int nsrc, const double* f, double* g, hipStream_t stream) {
    return run_guarded([&] {
        check_mesh_id(ctx, mesh_id);
        if (nsrc < 0 || (nsrc > 0 && (!f || !g))) throw ArgError("bad arguments");
        if (nsrc == 0) return;
        quad_data(ctx, ctx->meshes[mesh_id], nsrc, f, nullptr, nullptr, nullptr, g, stream);
        HIPCHK(hipGetLastError());
    });
}

dg_status dg_boundary_data_noalloc(dg_ctx* ctx, int mesh_id, int nsrc, const double* f, double* g,
                                   hipStream_t stream) {
    return run_guarded([&] {
        check_mesh_id(ctx, mesh_id);
        if (nsrc < 0 || (nsrc > 0 && (!f || !g))) throw ArgError("bad arguments");
        if (nsrc == 0) return;
        int dev = -1;
        HIPCHK(hipGetDevice(&dev));
        if (dev != ctx->device) throw ArgError("the context's device is not the current device");
        long long cap = 0;
        double* scr = dg::quad_scratch(dev, &cap);
        if (!scr) throw HipError("work space of this device not set up");
        const Mesh& M = ctx->meshes[mesh_id];
        const LevelHost& L0 = M.lv[0];
        if (L0.family != 0)
            throw ArgError("Dirichlet data by quadrature need Gauss-Lobatto nodes (pass g at the face points)");
        const dg::QuadPlan P = dg::quad_plan_bounded(L0, nsrc, cap);
        if (P.R == 0) throw ArgError("mesh too large for the fixed work space (records of one source exceed it)");
        // records first, then the split partial sums (every entry read is written first in the call)
        double* part = P.part_len > 0 ? scr + P.rec_len : nullptr;
        dg::launch_quad_data(L0, L0.dev64, M.qnodes, P, nsrc, f, nullptr, nullptr, nullptr, scr, part, g, stream);
        HIPCHK(hipGetLastError());
    });
}

dg_status dg_tile_set(int fp_bytes, int n, int step, int tx, int ty, int zlen) {
    return run_guarded([&] {
        if (!dg::tile_set(fp_bytes, n, step, tx, ty, zlen)) throw ArgError("no operator kernel for this tile");
    });
}

dg_status dg_tile_get(int fp_bytes, int n, int step, int* tx, int* ty, int* zlen) {
    return run_guarded([&] {
        if (!dg::tile_get(fp_bytes, n, step, tx, ty, zlen)) throw ArgError("bad tile query");
    });
}

dg_status dg_operator_apply(dg_ctx* ctx, int mesh_id, int level, int nrhs, const double* u, double* y,
                            hipStream_t stream) {
    return run_guarded([&] {
        check_mesh_id(ctx, mesh_id);
        auto& M = ctx->meshes[mesh_id];
        if (level < 0 || level >= (int)M.lv.size()) throw ArgError("level out of range");
        if (nrhs < 0 || (nrhs > 0 && (!u || !y))) throw ArgError("bad arguments");
        const auto& L = M.lv[level];
        dg::launch_brick<double>(dg::BM_APPLY, L, L.dev64, nrhs, nullptr, u, nullptr, nullptr, nullptr, y, nullptr,
                                 nullptr, 0, 0, 0, stream);
        HIPCHK(hipGetLastError());
    });
}

dg_status dg_rhs_assemble(dg_ctx* ctx, int mesh_id, int nrhs, const double* rho, const double* g, double* b,
                          hipStream_t stream) {
    return run_guarded([&] {
        check_mesh_id(ctx, mesh_id);
        auto& M = ctx->meshes[mesh_id];
        if (nrhs < 0 || (nrhs > 0 && (!rho || !g || !b))) throw ArgError("bad arguments");
        dg::launch_rhs(M.lv[0], M.lv[0].dev64, nrhs, rho, nullptr, nullptr, nullptr, g, M.nface, b, stream);
        HIPCHK(hipGetLastError());
    });
}

dg_status dg_vcycle_apply(dg_ctx* ctx, int mesh_id, int level, int nrhs, const double* r, double* z,
                          hipStream_t stream) {
    return run_guarded([&] {
        check_mesh_id(ctx, mesh_id);
        auto& M = ctx->meshes[mesh_id];
        if (level < 0 || level >= (int)M.lv.size()) throw ArgError("level out of range");
        if (nrhs < 0 || (nrhs > 0 && (!r || !z))) throw ArgError("bad arguments");
        if (nrhs == 0) return;
        ensure_state(M, nrhs);
        ensure_work<double>(M, M.w64, nrhs);
        g_prof = nullptr;
        double* out = vcycle<double>(M, M.w64, level, nrhs, nullptr, r, false, false, stream);
        HIPCHK(hipMemcpyAsync(z, out, sizeof(double) * M.lv[level].ndof * nrhs, hipMemcpyDeviceToDevice, stream));
        HIPCHK(hipGetLastError());
    });
}

dg_status dg_operator_apply_f32(dg_ctx* ctx, int mesh_id, int level, int nrhs, const float* u, float* y,
                                hipStream_t stream) {
    return run_guarded([&] {
        check_mesh_id(ctx, mesh_id);
        auto& M = ctx->meshes[mesh_id];
        if (level < 0 || level >= (int)M.lv.size()) throw ArgError("level out of range");
        if (nrhs < 0 || (nrhs > 0 && (!u || !y))) throw ArgError("bad arguments");
        const auto& L = M.lv[level];
        dg::launch_brick<float>(dg::BM_APPLY, L, L.dev32, nrhs, nullptr, u, nullptr, nullptr, nullptr, y, nullptr,
                                nullptr, 0, 0, 0, stream);
        HIPCHK(hipGetLastError());
    });
}

dg_status dg_operator_apply_mfma(dg_ctx* ctx, int mesh_id, int level, int nrhs, const float* u, float* y,
                                 hipStream_t stream) {
    return run_guarded([&] {
        check_mesh_id(ctx, mesh_id);
        auto& M = ctx->meshes[mesh_id];
        if (level < 0 || level >= (int)M.lv.size()) throw ArgError("level out of range");
        if (nrhs < 0 || (nrhs > 0 && (!u || !y))) throw ArgError("bad arguments");
        if (nrhs == 0) return;
        const auto& L = M.lv[level];
        if (!dg::launch_brick_mf(dg::BM_APPLY, L, L.dev32, nrhs, nullptr, u, nullptr, nullptr, y, nullptr, 0, 0, 0,
                                 stream))
            throw ArgError("no matrix-core operator kernel for this level (degree 4 only)");
        HIPCHK(hipGetLastError());
    });
}

dg_status dg_vcycle_apply_f32(dg_ctx* ctx, int mesh_id, int level, int nrhs, const float* r, float* z,
                              hipStream_t stream) {
    return run_guarded([&] {
        check_mesh_id(ctx, mesh_id);
        auto& M = ctx->meshes[mesh_id];
        if (level < 0 || level >= (int)M.lv.size()) throw ArgError("level out of range");
        if (nrhs < 0 || (nrhs > 0 && (!r || !z))) throw ArgError("bad arguments");
        if (nrhs == 0) return;
        ensure_state(M, nrhs);
        ensure_work<float>(M, M.w32, nrhs);
        g_prof = nullptr;
        float* out = vcycle<float>(M, M.w32, level, nrhs, nullptr, r, false, false, stream);
        HIPCHK(hipMemcpyAsync(z, out, sizeof(float) * M.lv[level].ndof * nrhs, hipMemcpyDeviceToDevice, stream));
        HIPCHK(hipGetLastError());
    });
}

dg_status dg_coarse_solve(dg_ctx* ctx, int mesh_id, int nrhs, const double* r, double* z, hipStream_t stream) {
    return run_guarded([&] {
        check_mesh_id(ctx, mesh_id);
        auto& M = ctx->meshes[mesh_id];
        if (nrhs < 0 || (nrhs > 0 && (!r || !z))) throw ArgError("bad arguments");
        ensure_cscr(M, nrhs);
        dg::launch_coarse<double>(M.dcoarse, M.lv.back(), nrhs, nullptr, r, z, M.cscr, stream);
        HIPCHK(hipGetLastError());
    });
}

dg_status dg_restrict(dg_ctx* ctx, int mesh_id, int level, int nrhs, const double* r, double* rc,
                      hipStream_t stream) {
    return run_guarded([&] {
        check_mesh_id(ctx, mesh_id);
        auto& M = ctx->meshes[mesh_id];
        if (level < 0 || level + 1 >= (int)M.lv.size()) throw ArgError("level out of range");
        if (nrhs < 0 || (nrhs > 0 && (!r || !rc))) throw ArgError("bad arguments");
        const auto& F = M.lv[level];
        const auto& C = M.lv[level + 1];
        dg::launch_restrict<double>(F, F.dev64, C, C.dev64, nrhs, nullptr, nullptr, r, rc, nullptr, 0.0, stream);
        HIPCHK(hipGetLastError());
    });
}

dg_status dg_prolong_add(dg_ctx* ctx, int mesh_id, int level, int nrhs, const double* zc, double* zf,
                         hipStream_t stream) {
    return run_guarded([&] {
        check_mesh_id(ctx, mesh_id);
        auto& M = ctx->meshes[mesh_id];
        if (level < 0 || level + 1 >= (int)M.lv.size()) throw ArgError("level out of range");
        if (nrhs < 0 || (nrhs > 0 && (!zc || !zf))) throw ArgError("bad arguments");
        dg::launch_prolong<double>(M.lv[level], M.lv[level + 1], nrhs, nullptr, zc, zf, stream);
        HIPCHK(hipGetLastError());
    });
}

dg_status dg_poisson_attach_guess(dg_ctx* ctx, dg_net* net) {
    return run_guarded([&] {
        if (!ctx) throw ArgError("null context");
        if (net && ctx->opts.node_family != 0)
            throw ArgError("the guess network works on Gauss-Lobatto element values");
        ctx->guess = net;
    });
}

dg_status dg_fused_fallbacks(const dg_ctx* ctx, long long* count) {
    return run_guarded([&] {
        if (!ctx || !count) throw ArgError("null argument");
        *count = ctx->fused_fallbacks.load();
    });
}

dg_status dg_profile_enable(dg_ctx* ctx, int enable) {
    return run_guarded([&] {
        if (!ctx) throw ArgError("null context");
        auto& P = ctx->prof;
        P.on = enable != 0;
        if (P.on) {
            P.used = 0;
            P.launches = 0;
            P.seconds = 0.0;
            P.bytes = 0.0;
            P.failed = false;
        }
    });
}

dg_status dg_profile_read(const dg_ctx* ctx, long long* launches, double* seconds, double* bytes) {
    return run_guarded([&] {
        if (!ctx) throw ArgError("null context");
        if (launches) *launches = ctx->prof.failed ? -1 : ctx->prof.launches;
        if (seconds) *seconds = ctx->prof.seconds;
        if (bytes) *bytes = ctx->prof.bytes;
    });
}

}  // extern "C"
