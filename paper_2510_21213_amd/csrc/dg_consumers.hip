// Consumers of the auxiliary-grid potentials (Sec. 6.1, Sec. 7.2): quadrature-weighted
// projections of grid functions on a basis, the exchange action W_a = sum_s psi_s v_as of a set
// of vectors, and the adaptively compressed exchange (ACE) vectors.
//
// Every integral is the grid's quadrature: node q of an element-major field carries the weight
// w_q = m_x[i] m_y[j] m_z[k], the lumped GLL mass of its local indices (the same for every
// element of a uniform mesh).  These steps stream their fields once (the projection reads each
// basis function once and the vectors from L2), so they are bound by HBM bandwidth; the dense
// contractions they contain are short (a few to a few hundred outputs per node) and stay on the
// vector units.
#include <hip/hip_runtime.h>

#include <stdexcept>

#include "dg_kernels.h"

namespace dg {

namespace {

constexpr int PJ_THREADS = 256;
constexpr int PJ_NODES = 32;  // nodes per thread per chunk: a chunk is 8,192 nodes
constexpr int PJ_MAXN3 = 512;  // nodes per element (degree <= 7)

// partial[(i * nu + a) * nchunk + c] = sum over the nodes q of chunk c of w_q f_q phi_i(q) u_a(q),
// for the TI x TA block of (i, a) of this work-group (f null: 1).  Work-groups of one chunk are
// consecutive, so the chunk's u and f come from L2 after the first.  The weight of a node depends
// only on its local index in the element (the three 1D lumped masses of a uniform mesh), staged
// in LDS per work-group.  Indices within one field are 32-bit (a field has < 2^31 nodes).
template <int TI, int TA>
__global__ __launch_bounds__(PJ_THREADS) void k_project(const LevelDev<double>* __restrict__ Lp, int n, int ndof,
                                                        int nbasis, const double* __restrict__ phi, int nu,
                                                        const double* __restrict__ u, const double* __restrict__ f,
                                                        int nchunk, double* __restrict__ partial) {
    __shared__ double red[PJ_THREADS / 64][TI * TA];
    __shared__ double wloc[PJ_MAXN3];
    const int nti = (nbasis + TI - 1) / TI, nta = (nu + TA - 1) / TA;
    const int b = blockIdx.x;
    const int ti = b % nti, ta = (b / nti) % nta, c = b / (nti * nta);
    const int i0 = ti * TI, a0 = ta * TA;
    const int n3 = n * n * n;
    {
        const LevelDev<double>& L = *Lp;
        for (int l = threadIdx.x; l < n3; l += PJ_THREADS)
            wloc[l] = L.ax[0].m[l % n] * L.ax[1].m[(l / n) % n] * L.ax[2].m[l / (n * n)];
    }
    __syncthreads();
    const double* __restrict__ prow[TI];
    const double* __restrict__ urow[TA];
#pragma unroll
    for (int r = 0; r < TI; ++r) prow[r] = phi + (long long)min(i0 + r, nbasis - 1) * ndof;
#pragma unroll
    for (int k = 0; k < TA; ++k) urow[k] = u + (long long)min(a0 + k, nu - 1) * ndof;
    double acc[TI][TA];
#pragma unroll
    for (int r = 0; r < TI; ++r)
#pragma unroll
        for (int k = 0; k < TA; ++k) acc[r][k] = 0.0;
    const int q0 = c * PJ_THREADS * PJ_NODES + (int)threadIdx.x;
#pragma unroll 4
    for (int m = 0; m < PJ_NODES; ++m) {
        const int q = q0 + m * PJ_THREADS;
        const bool ok = q < ndof;
        const int qq = ok ? q : 0;
        double wq = ok ? wloc[qq % n3] : 0.0;
        if (f) wq *= f[qq];
        double uv[TA];
#pragma unroll
        for (int k = 0; k < TA; ++k) uv[k] = wq * urow[k][qq];
#pragma unroll
        for (int r = 0; r < TI; ++r) {
            const double pv = prow[r][qq];
#pragma unroll
            for (int k = 0; k < TA; ++k) acc[r][k] += pv * uv[k];
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int r = 0; r < TI; ++r)
#pragma unroll
        for (int k = 0; k < TA; ++k) {
            double v = acc[r][k];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0) red[wv][r * TA + k] = v;
        }
    __syncthreads();
    if (threadIdx.x < TI * TA) {
        const int r = threadIdx.x / TA, k = threadIdx.x % TA;
        if (i0 + r < nbasis && a0 + k < nu) {
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < PJ_THREADS / 64; ++w) s += red[w][threadIdx.x];
            partial[((long long)(i0 + r) * nu + a0 + k) * nchunk + c] = s;
        }
    }
}

// W[a][q] = sum_s psi[s][q] v[a * nocc + s][q]
__global__ __launch_bounds__(256) void k_cross_w(long long ndof, int nu, int nocc, const double* __restrict__ psi,
                                                 const double* __restrict__ v, double* __restrict__ W) {
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    const int a = blockIdx.y;
    if (q >= ndof || a >= nu) return;
    double s = 0.0;
    for (int k = 0; k < nocc; ++k) s += psi[(long long)k * ndof + q] * v[((long long)a * nocc + k) * ndof + q];
    W[(long long)a * ndof + q] = s;
}

// rho[a * nocc + s] = u[a] psi[s] on every node
__global__ __launch_bounds__(256) void k_cross_products(long long ndof, int nu, int nocc,
                                                        const double* __restrict__ u, const double* __restrict__ psi,
                                                        double* __restrict__ rho) {
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    const int pr = blockIdx.y, a = pr / nocc, s = pr % nocc;
    if (q >= ndof || a >= nu) return;
    rho[(long long)pr * ndof + q] = u[(long long)a * ndof + q] * psi[(long long)s * ndof + q];
}

// One work-group: M (nocc x nocc, row-major, M[k][l] = (psi_k, W_l)) -> its symmetric part,
// the Cholesky factor L (M = L L^T) and T = L^-1 (lower triangular, written row-major).
// flag[0] = 1 when a pivot is not positive (M not positive definite); T is then not to be used.
constexpr int ACE_MAX = 64;
__global__ __launch_bounds__(256) void k_ace_factor(int n, const double* __restrict__ Min, double* __restrict__ T,
                                                    int* flag) {
    __shared__ double L[ACE_MAX][ACE_MAX + 1];
    __shared__ double Ti[ACE_MAX][ACE_MAX + 1];
    __shared__ int bad;
    const int t = threadIdx.x;
    if (t == 0) bad = 0;
    for (int e = t; e < n * n; e += 256) {
        const int r = e / n, c = e % n;
        L[r][c] = 0.5 * (Min[r * n + c] + Min[c * n + r]);
    }
    __syncthreads();
    for (int j = 0; j < n; ++j) {  // column j: pivot, then the entries below it
        if (t == 0) {
            double d = L[j][j];
            for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
            if (!(d > 0.0)) {
                bad = 1;
                d = 1.0;
            }
            L[j][j] = sqrt(d);
        }
        __syncthreads();
        for (int r = j + 1 + t; r < n; r += 256) {
            double s = L[r][j];
            for (int k = 0; k < j; ++k) s -= L[r][k] * L[j][k];
            L[r][j] = s / L[j][j];
        }
        __syncthreads();
    }
    // T = L^-1, one column per thread by forward substitution on e_c
    for (int c = t; c < n; c += 256) {
        for (int r = 0; r < n; ++r) {
            if (r < c) {
                Ti[r][c] = 0.0;
                continue;
            }
            double s = (r == c) ? 1.0 : 0.0;
            for (int k = c; k < r; ++k) s -= L[r][k] * Ti[k][c];
            Ti[r][c] = s / L[r][r];
        }
    }
    __syncthreads();
    for (int e = t; e < n * n; e += 256) T[e] = Ti[e / n][e % n];
    if (t == 0) flag[0] = bad;
}

// xi[k][q] = sum_{j <= k} T[k][j] W[j][q]
__global__ __launch_bounds__(256) void k_ace_combine(long long ndof, int n, const double* __restrict__ T,
                                                     const double* __restrict__ W, double* __restrict__ xi) {
    __shared__ double Ts[ACE_MAX * ACE_MAX];
    for (int e = threadIdx.x; e < n * n; e += 256) Ts[e] = T[e];
    __syncthreads();
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q >= ndof) return;
    for (int k = 0; k < n; ++k) {  // W[j][q] is re-read per k from L1/L2: this step runs once per SCF rebuild
        double s = 0.0;
        for (int j = 0; j <= k; ++j) s += Ts[k * n + j] * W[(long long)j * ndof + q];
        xi[(long long)k * ndof + q] = s;
    }
}

// C[i][a] = sum_k A[i][k] B[k][a]  (small dense product, one thread per output)
__global__ __launch_bounds__(256) void k_small_gemm(int ni, int nk, int na, const double* __restrict__ A,
                                                    const double* __restrict__ B, double* __restrict__ C) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= ni * na) return;
    const int i = e / na, a = e % na;
    double s = 0.0;
    for (int k = 0; k < nk; ++k) s += A[(long long)i * nk + k] * B[(long long)k * na + a];
    C[e] = s;
}

}  // namespace

int project_chunks(long long ndof) { return (int)((ndof + PJ_THREADS * PJ_NODES - 1) / (PJ_THREADS * PJ_NODES)); }

void launch_project(const LevelHost& L, int nbasis, const double* phi, int nu, const double* u, const double* f,
                    double* partial, double* out, hipStream_t s) {
    if (nbasis == 0 || nu == 0) return;
    constexpr int TI = 8, TA = 8;
    const int nchunk = project_chunks(L.ndof);
    const long long nti = (nbasis + TI - 1) / TI, nta = (nu + TA - 1) / TA;
    const long long grid = nti * nta * nchunk;
    if (grid > 0x7fffffffLL) throw std::runtime_error("projection grid too large");
    if (L.ndof >= 0x7fffffffLL || L.n * L.n * L.n > PJ_MAXN3) throw std::runtime_error("projection: field too large");
    hipLaunchKernelGGL((k_project<TI, TA>), dim3((unsigned)grid), dim3(PJ_THREADS), 0, s, L.dev64, L.n, (int)L.ndof,
                       nbasis, phi, nu, u, f, nchunk, partial);
    launch_sum_partials(nbasis * nu, partial, nchunk, nchunk, out, s);
}

void launch_cross_products(long long ndof, int nu, int nocc, const double* u, const double* psi, double* rho,
                           hipStream_t s) {
    if (nu == 0 || nocc == 0) return;
    hipLaunchKernelGGL(k_cross_products, dim3((unsigned)((ndof + 255) / 256), nu * nocc), dim3(256), 0, s, ndof, nu,
                       nocc, u, psi, rho);
}

void launch_cross_w(long long ndof, int nu, int nocc, const double* psi, const double* v, double* W, hipStream_t s) {
    if (nu == 0) return;
    hipLaunchKernelGGL(k_cross_w, dim3((unsigned)((ndof + 255) / 256), nu), dim3(256), 0, s, ndof, nu, nocc, psi, v, W);
}

void launch_ace_factor(int n, const double* M, double* T, int* flag, hipStream_t s) {
    if (n < 1 || n > ACE_MAX) throw std::runtime_error("ACE: bad orbital count");
    hipLaunchKernelGGL(k_ace_factor, dim3(1), dim3(256), 0, s, n, M, T, flag);
}

void launch_ace_combine(long long ndof, int n, const double* T, const double* W, double* xi, hipStream_t s) {
    hipLaunchKernelGGL(k_ace_combine, dim3((unsigned)((ndof + 255) / 256)), dim3(256), 0, s, ndof, n, T, W, xi);
}

void launch_small_gemm(int ni, int nk, int na, const double* A, const double* B, double* C, hipStream_t s) {
    if (ni * na == 0) return;
    hipLaunchKernelGGL(k_small_gemm, dim3((unsigned)((ni * na + 255) / 256)), dim3(256), 0, s, ni, nk, na, A, B, C);
}

}  // namespace dg
