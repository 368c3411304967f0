// Adaptive octree auxiliary mesh (Sec. 6.2), its SIPDG Poisson operator with hanging faces
// (Sec. 6.3) and MG-PCG over the nested refinement hierarchy (Sec. 6.4).
//
// Mesh.  A uniform box of base elements is refined cell by cell: a cell of edge lengths L_d
// (L = max) is halved along every axis with L_d >= L/2, and its children replace it when the
// Gauss-Legendre integrals of the density on the cell and on its children differ by more than
// delta_q.  Cells are tested generation by generation, every generation's samples in one call
// of the caller's density function.  Elements are the leaves, in depth-first order (base cells
// z, y, x lexicographic, x fastest; children likewise by their half along each split axis);
// degree-q GL nodes [k][j][i] per element.
//
// Operator.  Matrix-free, one work-group slot per element and right-hand side: the volume term
// as three 1D contractions with the element's own scale factors, then the six faces of the
// element.  A face is tiled by "pieces", the intersections with the neighbours' faces (dyadic
// cells: along each tangential axis the piece is the smaller of the two intervals).  On a piece
// both sides' traces and normal derivatives are interpolated to the piece's (q+1)^2 GL points
// with 1D tables (interval j of 2^k of the element's face; k = 0 is the identity), the SIPDG
// flux is formed there, and its test-function side is projected back onto the element's face
// nodes.  Each element gathers its own rows (no atomics); every interior piece is computed from
// both sides.
//
// Multigrid.  Degree steps on the leaves, then mesh steps (the tree cut at generation g, g =
// G-1 .. 0) at degree 1; the coarsest level is the uniform base mesh at degree 1, solved by
// fast diagonalisation.  Chebyshev-Jacobi smoothing with the uniform mesh's parameters; the
// Chebyshev step is fused into the operator kernel's epilogue.  The V-cycle runs in FP64, or
// in FP32 under the FP64 CG (DG_PREC_FP32_PC): the kernels are templated on the field type.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <stdexcept>
#include <string>
#include <vector>

#include "dg_internal.h"
#include "dg_kernels.h"

namespace dg {
namespace oct {

constexpr int OT = 128;     // threads of an operator work-group
constexpr int KMAX = 8;     // deepest interpolation table entry (a level jump of 2^8 along an axis)
constexpr int NTAB = (2 << KMAX) - 1;

struct Piece {
    int nb;        // neighbour element, -1 on the domain boundary
    int s1, s2;    // table entries: this element's face nodes -> the piece's points, along t1 and t2
    int n1, n2;    // the same for the neighbour's face
    int face;      // face of this element: 2 d + (upper side), d the normal axis
    double sig;    // penalty of the piece
    double wsc;    // product of the piece's two tangential half-widths
    double ijn;    // 1 / (the neighbour's half-width along the normal), 0 on the boundary
};

template <int N, typename T = double>
struct Ref {
    T K1[N][N];          // D^T diag(w) D on [-1, 1]
    T w[N];
    T eL[N], eR[N];      // basis values at -1 and +1
    T dL[N], dR[N];      // basis derivatives there (reference coordinate)
};

enum { OP_APPLY = 0, OP_RESID = 1, OP_CHEB = 2 };

#define OCHK(x)                                                                                    \
    do {                                                                                           \
        hipError_t e_ = (x);                                                                       \
        if (e_ != hipSuccess)                                                                      \
            hip_fail(std::string(#x) + ": " + hipGetErrorString(e_) + " at line " + std::to_string(__LINE__)); \
    } while (0)

// y = A u (APPLY), y = f - A u (RESID), or one fused Chebyshev step (CHEB, u = the current
// correction d): z += d; r -= A d; y = c1 d + c2 D^-1 r.  Grid (element blocks, nrhs); a block
// holds EPB = 128 / N^3 element slots of N^3 threads.  The pieces of an element (all six faces,
// stored consecutively) are taken N at a time, N^2 threads per piece: traces of both sides, the
// two interpolation passes to the piece's points, the flux, the two transposed passes back onto
// the element's face nodes; then every node thread adds what the pass's pieces give its own row.
template <int N, int MODE, int RB, typename T>
__global__ __launch_bounds__(OT) void k_oct_op(Ref<N, double> Rarg, int ne, int nrhs, const double* __restrict__ J,
                                              const int* __restrict__ fstart, const Piece* __restrict__ pcs,
                                              const T* __restrict__ tab, const RhsState* __restrict__ st,
                                              const T* __restrict__ u, T* __restrict__ y,
                                              const T* __restrict__ f, T* __restrict__ r,
                                              T* __restrict__ z, const T* __restrict__ dinv, T c1, T c2) {
    constexpr int N2 = N * N, N3 = N * N * N, EPB = OT / N3;
    __shared__ T U[RB][EPB][N3];
    // per right-hand side and slot, per piece of the pass (N pieces of N^2 points): own /
    // neighbour trace and normal derivative, the interpolation scratch, the flux, and the result
    // on the face nodes
    __shared__ T A0[RB][EPB][N3], A1[RB][EPB][N3], A2[RB][EPB][N3], A3[RB][EPB][N3];
    __shared__ T B0[RB][EPB][N3], B1[RB][EPB][N3], B2[RB][EPB][N3], B3[RB][EPB][N3];
    __shared__ int npc[EPB], ncc[EPB];
    __shared__ Ref<N, T> R;  // the reference data, indexed at run time (from LDS, not the argument block)
    const int rhs0 = blockIdx.y * RB;
    bool live[RB];
    bool any = false;
#pragma unroll
    for (int q = 0; q < RB; ++q) {
        live[q] = rhs0 + q < nrhs && (!st || st[rhs0 + q].active);
        any = any || live[q];
    }
    if (!any) return;
    const int t = threadIdx.x, s = t / N3, l = t - s * N3;
    // work-groups are dealt to the 8 XCDs in turn; give each XCD a contiguous run of elements
    // (depth-first order is spatially local), so that neighbour faces are read from its own L2
    const int nbx = gridDim.x, full = nbx / 8 * 8;
    const int bx = (int)blockIdx.x < full ? ((int)blockIdx.x % 8) * (nbx / 8) + (int)blockIdx.x / 8 : (int)blockIdx.x;
    const int e = bx * EPB + s;
    {
        const double* src = reinterpret_cast<const double*>(&Rarg);
        T* dst = reinterpret_cast<T*>(&R);
        for (int q = t; q < (int)(sizeof(Ref<N, double>) / sizeof(double)); q += OT) dst[q] = (T)src[q];
    }
    const bool node = s < EPB && e < ne;
    const long long estride = (long long)ne * N3;
    const int i = l % N, j = (l / N) % N, k = l / N2;
    const int pj = l / N2, fl = l - pj * N2;  // piece of the pass and its point / face node
    if (node) {
#pragma unroll
        for (int q = 0; q < RB; ++q)
            U[q][s][l] = live[q] ? u[(long long)(rhs0 + q) * estride + (long long)e * N3 + l] : T(0);
    }
    int p0 = 0, nconf = 0, np = 0;
    if (node) {
        p0 = fstart[2 * e];
        nconf = fstart[2 * e + 1] - p0;
        np = fstart[2 * e + 2] - p0;
    }
    if (node && l == 0) {
        npc[s] = np - nconf;
        ncc[s] = nconf;
    }
    if (!node && l == 0 && s < EPB) npc[s] = ncc[s] = 0;
    __syncthreads();
    T acc[RB];
    T Jx = T(1), Jy = T(1), Jz = T(1);
#pragma unroll
    for (int q = 0; q < RB; ++q) acc[q] = T(0);
    if (node) {
        Jx = (T)J[3 * e];
        Jy = (T)J[3 * e + 1];
        Jz = (T)J[3 * e + 2];
        const T sx = Jy * Jz / Jx * R.w[j] * R.w[k], sy = Jx * Jz / Jy * R.w[i] * R.w[k],
                     sz = Jx * Jy / Jz * R.w[i] * R.w[j];
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            T ax = T(0), ay = T(0), az = T(0);
#pragma unroll
            for (int a = 0; a < N; ++a) {
                ax += R.K1[i][a] * U[q][s][(k * N + j) * N + a];
                ay += R.K1[j][a] * U[q][s][(k * N + a) * N + i];
                az += R.K1[k][a] * U[q][s][(a * N + j) * N + i];
            }
            acc[q] = sx * ax + sy * ay + sz * az;
        }
    }
    int npmax = 0, ncmax = 0;
#pragma unroll
    for (int q = 0; q < EPB; ++q) {
        npmax = max(npmax, npc[q]);
        ncmax = max(ncmax, ncc[q]);
    }
    const int o = pj * N2;  // this piece's block of N^2 in the slot arrays
    // every node adds the pass's pieces (results in A2 / A3): v_s(m) FT[b][a] + sg d_s(m) / J_d FD[b][a]
#define OCT_GATHER(first, count)                                                                          \
    for (int q = 0; q < N && q < (count); ++q) {                                                          \
        const int fq = pcs[(first) + q].face;                                                             \
        const int dq = fq >> 1;                                                                           \
        const int m = dq == 0 ? i : (dq == 1 ? j : k);                                                    \
        const int a = dq == 0 ? j : i;                                                                    \
        const int b = dq == 2 ? j : k;                                                                    \
        const T vm = (fq & 1) ? R.eR[m] : R.eL[m];                                                   \
        const T dm = ((fq & 1) ? R.dR[m] : -R.dL[m]) / (dq == 0 ? Jx : (dq == 1 ? Jy : Jz));         \
        _Pragma("unroll") for (int c = 0; c < RB; ++c) acc[c] +=                                          \
            vm * A2[c][s][q * N2 + b * N + a] + dm * A3[c][s][q * N2 + b * N + a];                        \
    }
    // conforming pieces and boundary faces (every table entry the identity): the flux at the face
    // nodes directly, N pieces per pass
    for (int pass = 0; pass < ncmax; pass += N) {
        const int pi = pass + pj;
        if (node && pi < nconf) {
            const Piece P = pcs[p0 + pi];
            const bool inner = P.nb >= 0;
            const int fc = P.face, d = fc >> 1;
            const int sd = d == 0 ? 1 : (d == 1 ? N : N2);
            const int s1 = d == 0 ? N : 1;
            const int s2 = d == 2 ? N : N2;
            const int a = fl % N, b = fl / N;
            const T* vS = (fc & 1) ? R.eR : R.eL;
            const T* dS = (fc & 1) ? R.dR : R.dL;
            const T* vO = (fc & 1) ? R.eL : R.eR;
            const T* dO = (fc & 1) ? R.dL : R.dR;
            const T iJ = T(1) / (d == 0 ? Jx : (d == 1 ? Jy : Jz));
            const T iJn = (T)P.ijn;
            const T sg = (fc & 1) ? T(1) : -T(1);
            const T half = inner ? T(0.5) : T(1);
            const T W = R.w[a] * R.w[b] * (T)P.wsc;
            const int lo = a * s1 + b * s2;
#pragma unroll
            for (int c = 0; c < RB; ++c) {
                T tv = T(0), dv = T(0), tn = T(0), dn = T(0);
#pragma unroll
                for (int m = 0; m < N; ++m) {
                    const T x = U[c][s][m * sd + lo];
                    tv += vS[m] * x;
                    dv += dS[m] * x;
                }
                if (inner && live[c]) {
                    const T* un = u + (long long)(rhs0 + c) * estride + (long long)P.nb * N3;
#pragma unroll
                    for (int m = 0; m < N; ++m) {
                        const T x = un[m * sd + lo];
                        tn += vO[m] * x;
                        dn += dO[m] * x;
                    }
                }
                dv *= iJ;
                dn *= iJn;
                const T jmp = inner ? tv - tn : tv;
                const T davg = inner ? T(0.5) * (dv + dn) : dv;
                A2[c][s][o + fl] = W * ((T)P.sig * jmp - sg * davg);
                A3[c][s][o + fl] = W * (-half * jmp);
            }
        }
        __syncthreads();
        if (node) { OCT_GATHER(p0 + pass, nconf - pass) }
        __syncthreads();
    }
    // hanging pieces: interpolation to the piece's points and back
    p0 += nconf;
    np -= nconf;
    for (int pass = 0; pass < npmax; pass += N) {
        const int pi = pass + pj;
        const bool act = node && pi < np;
        Piece P;
        P.nb = -1;
        P.s1 = P.s2 = P.n1 = P.n2 = P.face = 0;
        P.sig = P.wsc = P.ijn = 0.0;
        if (act) P = pcs[p0 + pi];
        const bool inner = P.nb >= 0;
        const int fc = P.face, d = fc >> 1;
        // traces on the face nodes (a, b) = (fl % N, fl / N): own face, and the neighbour's opposite face
        if (act) {
            const int sd = d == 0 ? 1 : (d == 1 ? N : N2);
            const int s1 = d == 0 ? N : 1;
            const int s2 = d == 2 ? N : N2;
            const int a = fl % N, b = fl / N;
            const int lo = a * s1 + b * s2;
            const T* vS = (fc & 1) ? R.eR : R.eL;
            const T* dS = (fc & 1) ? R.dR : R.dL;
            const T* vO = (fc & 1) ? R.eL : R.eR;
            const T* dO = (fc & 1) ? R.dL : R.dR;
            const T iJ = T(1) / (d == 0 ? Jx : (d == 1 ? Jy : Jz));
            const T iJn = (T)P.ijn;
#pragma unroll
            for (int c = 0; c < RB; ++c) {
                T tv = T(0), dv = T(0), tn = T(0), dn = T(0);
#pragma unroll
                for (int m = 0; m < N; ++m) {
                    const T x = U[c][s][m * sd + lo];
                    tv += vS[m] * x;
                    dv += dS[m] * x;
                }
                if (inner && live[c]) {
                    const T* un = u + (long long)(rhs0 + c) * estride + (long long)P.nb * N3;
#pragma unroll
                    for (int m = 0; m < N; ++m) {
                        const T x = un[m * sd + lo];
                        tn += vO[m] * x;
                        dn += dO[m] * x;
                    }
                }
                A0[c][s][o + fl] = tv;
                A1[c][s][o + fl] = dv * iJ;
                A2[c][s][o + fl] = tn;
                A3[c][s][o + fl] = dn * iJn;
            }
        }
        __syncthreads();
        // interpolation along t1: X[b][q1] = sum_a I1[q1][a] F[b][a]
        if (act) {
            const int q1 = fl % N, b = fl / N;
            T Is[N], In[N];
#pragma unroll
            for (int a = 0; a < N; ++a) {
                Is[a] = tab[(long long)P.s1 * N2 + q1 * N + a];
                In[a] = tab[(long long)P.n1 * N2 + q1 * N + a];
            }
#pragma unroll
            for (int c = 0; c < RB; ++c) {
                T x0 = T(0), x1 = T(0), x2 = T(0), x3 = T(0);
#pragma unroll
                for (int a = 0; a < N; ++a) {
                    x0 += Is[a] * A0[c][s][o + b * N + a];
                    x1 += Is[a] * A1[c][s][o + b * N + a];
                    x2 += In[a] * A2[c][s][o + b * N + a];
                    x3 += In[a] * A3[c][s][o + b * N + a];
                }
                B0[c][s][o + fl] = x0;
                B1[c][s][o + fl] = x1;
                B2[c][s][o + fl] = x2;
                B3[c][s][o + fl] = x3;
            }
        }
        __syncthreads();
        // along t2, and the flux at the piece point (q2, q1); seen from this element (outward
        // normal sg e_d): [u] = u - u_nb, {d_n u} = sg {du/dx_d}
        if (act) {
            const int q1 = fl % N, q2 = fl / N;
            T Is[N], In[N];
#pragma unroll
            for (int b = 0; b < N; ++b) {
                Is[b] = tab[(long long)P.s2 * N2 + q2 * N + b];
                In[b] = tab[(long long)P.n2 * N2 + q2 * N + b];
            }
            const T sg = (fc & 1) ? T(1) : -T(1);
            const T half = inner ? T(0.5) : T(1);
            const T W = R.w[q1] * R.w[q2] * (T)P.wsc;
#pragma unroll
            for (int c = 0; c < RB; ++c) {
                T tr = T(0), dr = T(0), trn = T(0), drn = T(0);
#pragma unroll
                for (int b = 0; b < N; ++b) {
                    tr += Is[b] * B0[c][s][o + b * N + q1];
                    dr += Is[b] * B1[c][s][o + b * N + q1];
                    trn += In[b] * B2[c][s][o + b * N + q1];
                    drn += In[b] * B3[c][s][o + b * N + q1];
                }
                const T jmp = inner ? tr - trn : tr;
                const T davg = inner ? T(0.5) * (dr + drn) : dr;
                A0[c][s][o + fl] = W * ((T)P.sig * jmp - sg * davg);
                A1[c][s][o + fl] = W * (-half * jmp);
            }
        }
        __syncthreads();
        // back onto the face nodes: transpose along t2 ...
        if (act) {
            const int q1 = fl % N, b = fl / N;
            T I2[N];
#pragma unroll
            for (int q2 = 0; q2 < N; ++q2) I2[q2] = tab[(long long)P.s2 * N2 + q2 * N + b];
#pragma unroll
            for (int c = 0; c < RB; ++c) {
                T y0 = T(0), y1 = T(0);
#pragma unroll
                for (int q2 = 0; q2 < N; ++q2) {
                    y0 += I2[q2] * A0[c][s][o + q2 * N + q1];
                    y1 += I2[q2] * A1[c][s][o + q2 * N + q1];
                }
                B0[c][s][o + fl] = y0;
                B1[c][s][o + fl] = y1;
            }
        }
        __syncthreads();
        // ... and along t1
        if (act) {
            const int a = fl % N, b = fl / N;
            T I1[N];
#pragma unroll
            for (int q1 = 0; q1 < N; ++q1) I1[q1] = tab[(long long)P.s1 * N2 + q1 * N + a];
#pragma unroll
            for (int c = 0; c < RB; ++c) {
                T y0 = T(0), y1 = T(0);
#pragma unroll
                for (int q1 = 0; q1 < N; ++q1) {
                    y0 += I1[q1] * B0[c][s][o + b * N + q1];
                    y1 += I1[q1] * B1[c][s][o + b * N + q1];
                }
                A2[c][s][o + fl] = y0;
                A3[c][s][o + fl] = y1;
            }
        }
        __syncthreads();
        if (node) { OCT_GATHER(p0 + pass, np - pass) }
        __syncthreads();
    }
    if (!node) return;
#pragma unroll
    for (int c = 0; c < RB; ++c) {
        if (!live[c]) continue;
        const long long g = (long long)(rhs0 + c) * estride + (long long)e * N3 + l;
        if constexpr (MODE == OP_APPLY) {
            y[g] = acc[c];
        } else if constexpr (MODE == OP_RESID) {
            y[g] = f[g] - acc[c];
        } else {
            const T dv = U[c][s][l];
            z[g] += dv;
            const T rn = r[g] - acc[c];
            r[g] = rn;
            y[g] = c1 * dv + c2 * dinv[(long long)e * N3 + l] * rn;
        }
    }
#undef OCT_GATHER
}

// grid (chunks of 256, nrhs): per-node kernels over one level's fields
inline dim3 node_grid(long long ndof, int nrhs) { return dim3((unsigned)((ndof + 255) / 256), (unsigned)nrhs); }

// r = f, z = 0, d = c0 D^-1 f (smoothing from a zero start)
template <typename T>
__global__ __launch_bounds__(256) void k_oct_start0(long long ndof, const RhsState* __restrict__ st,
                                                    const T* __restrict__ f, T* __restrict__ r,
                                                    T* __restrict__ z, T* __restrict__ d,
                                                    const T* __restrict__ dinv, T c0) {
    const int rhs = blockIdx.y;
    if (st && !st[rhs].active) return;
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q >= ndof) return;
    const long long g = (long long)rhs * ndof + q;
    const T fv = f[g];
    r[g] = fv;
    z[g] = T(0);
    d[g] = c0 * dinv[q] * fv;
}

// d = c0 D^-1 r
template <typename T>
__global__ __launch_bounds__(256) void k_oct_dstart(long long ndof, const RhsState* __restrict__ st,
                                                    const T* __restrict__ r, T* __restrict__ d,
                                                    const T* __restrict__ dinv, T c0) {
    const int rhs = blockIdx.y;
    if (st && !st[rhs].active) return;
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q >= ndof) return;
    const long long g = (long long)rhs * ndof + q;
    d[g] = c0 * dinv[q] * r[g];
}

// z += d
template <typename T>
__global__ __launch_bounds__(256) void k_oct_add(long long ndof, const RhsState* __restrict__ st,
                                                 const T* __restrict__ d, T* __restrict__ z) {
    const int rhs = blockIdx.y;
    if (st && !st[rhs].active) return;
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q >= ndof) return;
    const long long g = (long long)rhs * ndof + q;
    z[g] += d[g];
}

// FP32 V-cycle under FP64 CG: the residual narrowed to FP32, the correction widened to FP64
__global__ __launch_bounds__(256) void k_oct_narrow(long long n, const RhsState* __restrict__ st, long long ndof,
                                                    const double* __restrict__ a, float* __restrict__ b) {
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    if (st && !st[q / ndof].active) return;
    b[q] = (float)a[q];
}
__global__ __launch_bounds__(256) void k_oct_widen(long long n, const RhsState* __restrict__ st, long long ndof,
                                                   const float* __restrict__ a, double* __restrict__ b) {
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    if (st && !st[q / ndof].active) return;
    b[q] = (double)a[q];
}

// PCG: p = z + beta p
__global__ __launch_bounds__(256) void k_oct_pdir(long long ndof, const RhsState* __restrict__ st,
                                                  const double* __restrict__ z, double* __restrict__ p) {
    const int rhs = blockIdx.y;
    if (!st[rhs].active) return;
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q >= ndof) return;
    const long long g = (long long)rhs * ndof + q;
    p[g] = z[g] + st[rhs].beta * p[g];
}

// PCG: x += alpha p, r -= alpha q
__global__ __launch_bounds__(256) void k_oct_xr(long long ndof, const RhsState* __restrict__ st,
                                                const double* __restrict__ p, const double* __restrict__ qv,
                                                double* __restrict__ x, double* __restrict__ r) {
    const int rhs = blockIdx.y;
    if (!st[rhs].active) return;
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q >= ndof) return;
    const long long g = (long long)rhs * ndof + q;
    const double a = st[rhs].alpha;
    x[g] += a * p[g];
    r[g] -= a * qv[g];
}

// y = x * sqrt(dinv) (Lanczos on D^-1/2 A D^-1/2), one vector
__global__ __launch_bounds__(256) void k_oct_dscale(long long ndof, const double* __restrict__ dinv,
                                                    const double* __restrict__ x, double* __restrict__ y) {
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q >= ndof) return;
    y[q] = x[q] * sqrt(dinv[q]);
}

// Degree transfers on the same elements: I[f][c] = coarse basis c at fine node f.
template <int NF, int NC, typename T>
struct DegI {
    T I[NF][NC];
};

// rc = P^T rf, one thread per coarse node
template <int NF, int NC, typename T>
__global__ __launch_bounds__(256) void k_oct_restrict_deg(DegI<NF, NC, T> Tm, int ne, const RhsState* __restrict__ st,
                                                          const T* __restrict__ rf, T* __restrict__ rc) {
    constexpr int F3 = NF * NF * NF, C3 = NC * NC * NC;
    const int rhs = blockIdx.y;
    if (st && !st[rhs].active) return;
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q >= (long long)ne * C3) return;
    const long long e = q / C3;
    const int l = (int)(q - e * C3);
    const int a = l % NC, b = (l / NC) % NC, c = l / (NC * NC);
    const T* src = rf + ((long long)rhs * ne + e) * F3;
    T acc = T(0);
    for (int kk = 0; kk < NF; ++kk) {
        T ay = T(0);
        for (int jj = 0; jj < NF; ++jj) {
            T ax = T(0);
#pragma unroll
            for (int ii = 0; ii < NF; ++ii) ax += Tm.I[ii][a] * src[(kk * NF + jj) * NF + ii];
            ay += Tm.I[jj][b] * ax;
        }
        acc += Tm.I[kk][c] * ay;
    }
    rc[(long long)rhs * ne * C3 + q] = acc;
}

// zf += P zc, one thread per fine node
template <int NF, int NC, typename T>
__global__ __launch_bounds__(256) void k_oct_prolong_deg(DegI<NF, NC, T> Tm, int ne, const RhsState* __restrict__ st,
                                                         const T* __restrict__ zc, T* __restrict__ zf) {
    constexpr int F3 = NF * NF * NF, C3 = NC * NC * NC;
    const int rhs = blockIdx.y;
    if (st && !st[rhs].active) return;
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q >= (long long)ne * F3) return;
    const long long e = q / F3;
    const int l = (int)(q - e * F3);
    const int ii = l % NF, jj = (l / NF) % NF, kk = l / (NF * NF);
    const T* src = zc + ((long long)rhs * ne + e) * C3;
    T acc = T(0);
    for (int c = 0; c < NC; ++c) {
        T ay = T(0);
        for (int b = 0; b < NC; ++b) {
            T ax = T(0);
#pragma unroll
            for (int a = 0; a < NC; ++a) ax += Tm.I[ii][a] * src[(c * NC + b) * NC + a];
            ay += Tm.I[jj][b] * ax;
        }
        acc += Tm.I[kk][c] * ay;
    }
    zf[(long long)rhs * ne * F3 + q] += acc;
}

// Mesh transfers at degree 1 (2 x 2 x 2 nodes).  Fine element e: parent element par[e] of the
// coarser mesh and per axis a table entry m[3e + d] (0 same extent, 1 lower half, 2 upper half).
template <typename T>
__global__ __launch_bounds__(256) void k_oct_prolong_mesh(int nef, int nec, const int* __restrict__ par,
                                                          const int* __restrict__ m, const T* __restrict__ tab,
                                                          const RhsState* __restrict__ st,
                                                          const T* __restrict__ zc, T* __restrict__ zf) {
    const int rhs = blockIdx.y;
    if (st && !st[rhs].active) return;
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q >= (long long)nef * 8) return;
    const int e = (int)(q >> 3), l = (int)(q & 7);
    const int ii = l & 1, jj = (l >> 1) & 1, kk = l >> 2;
    const T* Tx = tab + m[3 * e] * 4 + ii * 2;
    const T* Ty = tab + m[3 * e + 1] * 4 + jj * 2;
    const T* Tz = tab + m[3 * e + 2] * 4 + kk * 2;
    const T* src = zc + ((long long)rhs * nec + par[e]) * 8;
    T acc = T(0);
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) acc += Tz[c] * Ty[b] * Tx[a] * src[(c * 2 + b) * 2 + a];
    zf[(long long)rhs * nef * 8 + q] += acc;
}

// rc = P^T rf: coarse element c gathers its fine elements kids[kstart[c] .. kstart[c+1])
template <typename T>
__global__ __launch_bounds__(256) void k_oct_restrict_mesh(int nef, int nec, const int* __restrict__ kstart,
                                                           const int* __restrict__ kids, const int* __restrict__ m,
                                                           const T* __restrict__ tab,
                                                           const RhsState* __restrict__ st,
                                                           const T* __restrict__ rf, T* __restrict__ rc) {
    const int rhs = blockIdx.y;
    if (st && !st[rhs].active) return;
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q >= (long long)nec * 8) return;
    const int c = (int)(q >> 3), l = (int)(q & 7);
    const int a = l & 1, b = (l >> 1) & 1, cc = l >> 2;
    T acc = T(0);
    for (int t = kstart[c]; t < kstart[c + 1]; ++t) {
        const int e = kids[t];
        const T* Tx = tab + m[3 * e] * 4;
        const T* Ty = tab + m[3 * e + 1] * 4;
        const T* Tz = tab + m[3 * e + 2] * 4;
        const T* src = rf + ((long long)rhs * nef + e) * 8;
        for (int kk = 0; kk < 2; ++kk)
            for (int jj = 0; jj < 2; ++jj)
                for (int ii = 0; ii < 2; ++ii)
                    acc += Tz[kk * 2 + cc] * Ty[jj * 2 + b] * Tx[ii * 2 + a] * src[(kk * 2 + jj) * 2 + ii];
    }
    rc[(long long)rhs * nec * 8 + q] = acc;
}

// b = 4 pi M f + lift(g): the mass J_x J_y J_z w_i w_j w_k, and on each boundary face of the
// element (bstart[6e + face] = offset of its (q+1)^2 points in g, -1 if interior) the Nitsche lift
// (sigma v - d_n v) integrated against g with the face's own GL rule.
template <int N>
__global__ __launch_bounds__(256) void k_oct_rhs(Ref<N> R, int ne, long long nbp, double eps_sig_q,
                                                 const double* __restrict__ J, const int* __restrict__ bstart,
                                                 const double* __restrict__ f, const double* __restrict__ gb,
                                                 double* __restrict__ b) {
    constexpr int N2 = N * N, N3 = N * N * N;
    const int rhs = blockIdx.y;
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q >= (long long)ne * N3) return;
    const int e = (int)(q / N3), l = (int)(q - (long long)e * N3);
    const int i = l % N, j = (l / N) % N, k = l / N2;
    const double Jv[3] = {J[3 * e], J[3 * e + 1], J[3 * e + 2]};
    const long long g = (long long)rhs * ne * N3 + q;
    double acc = 4.0 * M_PI * Jv[0] * Jv[1] * Jv[2] * R.w[i] * R.w[j] * R.w[k] * f[g];
    for (int fc = 0; fc < 6; ++fc) {
        const int off = bstart[6 * e + fc];
        if (off < 0) continue;
        const int d = fc >> 1;
        const double sg = (fc & 1) ? 1.0 : -1.0;
        const int m = d == 0 ? i : (d == 1 ? j : k);
        const int a = d == 0 ? j : i;
        const int bb = d == 2 ? j : k;
        const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
        const double sig = eps_sig_q / (2.0 * Jv[d]);
        const double v = (fc & 1) ? R.eR[m] : R.eL[m];
        const double dn = ((fc & 1) ? R.dR[m] : R.dL[m]) / Jv[d];
        const double W = R.w[a] * R.w[bb] * Jv[t1] * Jv[t2];
        acc += (sig * v - sg * dn) * W * gb[(long long)rhs * nbp + off + bb * N + a];
    }
    b[g] = acc;
}

// Dirichlet data by quadrature (Sec. 6.3): g_s(r_p) = sum_q W_q f_s(x_q) / |r_p - x_q| over the
// finest level's nodes (GL nodes: none lies on the boundary, every term is finite).  Grid
// (point blocks, source blocks of BR, node parts): a thread owns one boundary point and BR
// sources; the part's nodes stream through LDS in tiles of BT (coordinates and BR weighted
// values); each part writes its partial sums, added in a fixed order by k_oct_bsum.
constexpr int BT = 256, BR = 12;

__global__ __launch_bounds__(BT) void k_oct_bdata(long long ndof, int nbp, int nsrc, int tiles_per_part,
                                                  const double* __restrict__ nx, const double* __restrict__ ny,
                                                  const double* __restrict__ nz, const double* __restrict__ nw,
                                                  const double* __restrict__ px, const double* __restrict__ py,
                                                  const double* __restrict__ pz, const double* __restrict__ f,
                                                  double* __restrict__ part) {
    __shared__ double X[BT], Y[BT], Z[BT], V[BR][BT];
    const int p = blockIdx.x * BT + threadIdx.x;
    const int s0 = blockIdx.y * BR;
    const int part_id = blockIdx.z;
    const double rx = p < nbp ? px[p] : 0.0, ry = p < nbp ? py[p] : 0.0, rz = p < nbp ? pz[p] : 0.0;
    double acc[BR];
#pragma unroll
    for (int r = 0; r < BR; ++r) acc[r] = 0.0;
    const long long t0 = (long long)part_id * tiles_per_part;
    for (long long t = t0; t < t0 + tiles_per_part; ++t) {
        const long long q0 = t * BT;
        if (q0 >= ndof) break;
        const long long q = q0 + threadIdx.x;
        const bool in = q < ndof;
        X[threadIdx.x] = in ? nx[q] : 0.0;
        Y[threadIdx.x] = in ? ny[q] : 0.0;
        Z[threadIdx.x] = in ? nz[q] : 1e30;  // padding far away: contributes 0 * tiny
        const double w = in ? nw[q] : 0.0;
#pragma unroll
        for (int r = 0; r < BR; ++r)
            V[r][threadIdx.x] = (in && s0 + r < nsrc) ? w * f[(long long)(s0 + r) * ndof + q] : 0.0;
        __syncthreads();
        const int cnt = (int)min((long long)BT, ndof - q0);
        for (int k = 0; k < cnt; ++k) {
            const double dx = rx - X[k], dy = ry - Y[k], dz = rz - Z[k];
            const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
            // hardware estimate of r2^(-1/2) (about 5e-8) refined by two terms of the series
            // (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + ..., e = 1 - r2 y^2: error O(e^3)
            double inv = __builtin_amdgcn_rsq(r2);
            const double e = fma(-(r2 * inv), inv, 1.0);
            inv = fma(inv * e, fma(0.375, e, 0.5), inv);
#pragma unroll
            for (int r = 0; r < BR; ++r) acc[r] += V[r][k] * inv;
        }
        __syncthreads();
    }
    if (p >= nbp) return;
#pragma unroll
    for (int r = 0; r < BR; ++r)
        if (s0 + r < nsrc) part[((long long)part_id * nsrc + s0 + r) * nbp + p] = acc[r];
}

__global__ __launch_bounds__(256) void k_oct_bsum(int nparts, int nsrc, int nbp, const double* __restrict__ part,
                                                  double* __restrict__ g) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= (long long)nsrc * nbp) return;
    double acc = 0.0;
    for (int k = 0; k < nparts; ++k) acc += part[(long long)k * nsrc * nbp + i];
    g[i] = acc;
}

// Exchange on the octree grid (Sec. 6.1): W_k = sum_s phi_s v_ks pointwise (v_ks = v_sk, row-major
// pair index of i <= j), and per pair k the partial sums of W_q rho_k v_k over chunks of 1024 nodes
// (rho_k = phi_i phi_j recomputed), added in a fixed order on the host.
__global__ __launch_bounds__(256) void k_oct_wk(long long ndof, int norb, const double* __restrict__ phi,
                                                const double* __restrict__ v, double* __restrict__ W) {
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    const int k = blockIdx.y;
    if (q >= ndof) return;
    double acc = 0.0;
    for (int s = 0; s < norb; ++s) {
        const int i = min(k, s), j = max(k, s);
        const int p = i * norb - i * (i - 1) / 2 + (j - i);
        acc += phi[(long long)s * ndof + q] * v[(long long)p * ndof + q];
    }
    W[(long long)k * ndof + q] = acc;
}

__global__ __launch_bounds__(256) void k_oct_kij(long long ndof, const int* __restrict__ pi, const int* __restrict__ pj,
                                                 const double* __restrict__ phi, const double* __restrict__ v,
                                                 const double* __restrict__ w, double* __restrict__ partial,
                                                 int nchunk) {
    __shared__ double red[256];
    const int p = blockIdx.y, c = blockIdx.x;
    const double* fi = phi + (long long)pi[p] * ndof;
    const double* fj = phi + (long long)pj[p] * ndof;
    const double* vp = v + (long long)p * ndof;
    double acc = 0.0;
    for (int u = 0; u < 4; ++u) {
        const long long q = (long long)c * 1024 + u * 256 + threadIdx.x;
        if (q < ndof) acc += w[q] * fi[q] * fj[q] * vp[q];
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(long long)p * nchunk + c] = red[0];
}

// ---------------------------------------------------------------------------------------------
// host side

struct TCell {
    int lv[3];
    long long ix[3];
    int gen;
    int parent;
    int child0 = -1, nchild = 0;
};

struct Level {
    int q = 1, n = 2;
    int ne = 0;
    long long ndof = 0;
    std::vector<int> cells;               // tree cell of each element
    std::vector<double> Jh;               // half-widths, 3 per element
    std::vector<int> fsh;                 // piece ranges: {first, first hanging} per element, + end
    std::vector<Piece> ph;
    std::vector<double> diag;
    double* J = nullptr;
    int* fstart = nullptr;
    Piece* pcs = nullptr;
    double* dinv = nullptr;
    float* dinv32 = nullptr;
    // transfer to the next coarser level
    int kind = 0;                         // 1 degree step, 2 mesh step
    std::vector<double> Ideg;             // n_f x n_c
    int* par = nullptr;                   // mesh step: parent per fine element
    int* msel = nullptr;                  // per fine element and axis: table entry
    int* kstart = nullptr;                // per coarse element: its fine elements
    int* kids = nullptr;
    // smoother
    double lam_lo = 0, lam_hi = 0, c0 = 0;
    std::vector<double> cp, cr;
    int degree = 0;
};

}  // namespace oct
}  // namespace dg

struct dg_octree {
    int device = 0;
    int E[3];
    double lo[3], hi[3], h[3];
    int q = 4;
    int rhs_per_block = 0;                // right-hand sides per operator work-group (1, 2, 4; 0 by degree)
    dg_opts opts;
    std::vector<dg::oct::TCell> tree;
    int max_gen = 0;
    std::vector<dg::oct::Level> lv;       // finest first; the last is the base mesh at degree 1
    std::vector<double> xi[9], wgl[9];    // GL nodes and weights per point count
    double* tab[9] = {};                  // interpolation tables per point count (device)
    float* tab32[9] = {};                 // the same in FP32
    bool fp32 = false;                    // FP32 V-cycle under FP64 CG (DG_PREC_FP32_PC)
    float *r32 = nullptr, *z32 = nullptr; // its finest-level input and output
    std::vector<double> tabh[9];
    int* bstart = nullptr;                // finest level: boundary offsets
    double* qnodes = nullptr;             // quadrature data: node x, y, z, weight (4 x n_dofs), then the
                                          // boundary points' x, y, z (3 x n_boundary), built on first use
    double* qpart = nullptr;              // its partial sums
    long long qpart_cap = 0;
    // exchange and quadrature-data work space, kept between calls (grows to the largest call)
    double *xrho = nullptr, *xb = nullptr, *xv = nullptr, *xpart = nullptr, *xg = nullptr;
    int *xpi = nullptr, *xpj = nullptr;
    long long xcap = 0, xpart_cap = 0, xg_cap = 0;
    int xnorb = 0;
    std::vector<int> bsh;
    long long nbp = 0;                    // boundary points
    dg::LevelHost base;                   // uniform base mesh at degree 1 (coarsest solve)
    dg::CoarseDev* cdev = nullptr;
    // work space (per right-hand-side capacity)
    int cap = 0;
    std::vector<double*> wf, wz, wr, wd0, wd1, wt;
    double* cscr = nullptr;
    double *px = nullptr, *pr = nullptr, *pz = nullptr, *pp = nullptr, *pq = nullptr;
    double* partial = nullptr;
    int pstride = 0;
    dg::RhsState* st = nullptr;
    int st_cap = 0;
};

namespace dg {
namespace oct {
namespace {

template <typename T>
T* oalloc(long long n) {
    void* p = nullptr;
    if (n <= 0) n = 1;
    OCHK(hipMalloc(&p, (size_t)n * sizeof(T)));
    return (T*)p;
}
template <typename T>
void ofree(T*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}
template <typename T>
T* upload(const std::vector<T>& v) {
    T* p = oalloc<T>((long long)v.size());
    if (!v.empty()) OCHK(hipMemcpy(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
    return p;
}

void cell_bounds(const dg_octree& O, const TCell& c, double a[3], double b[3]) {
    for (int d = 0; d < 3; ++d) {
        a[d] = O.lo[d] + O.h[d] * std::ldexp((double)c.ix[d], -c.lv[d]);
        b[d] = a[d] + std::ldexp(O.h[d], -c.lv[d]);
    }
}

// split axes of a cell (L_d >= L/2), children in (z, y, x) order of their half, x fastest
void children_of(const dg_octree& O, const TCell& c, std::vector<TCell>& kids) {
    double L[3], Lm = 0.0;
    for (int d = 0; d < 3; ++d) {
        L[d] = std::ldexp(O.h[d], -c.lv[d]);
        Lm = std::max(Lm, L[d]);
    }
    bool S[3];
    for (int d = 0; d < 3; ++d) S[d] = L[d] >= 0.5 * Lm;
    kids.clear();
    for (int oz = 0; oz < (S[2] ? 2 : 1); ++oz)
        for (int oy = 0; oy < (S[1] ? 2 : 1); ++oy)
            for (int ox = 0; ox < (S[0] ? 2 : 1); ++ox) {
                const int o[3] = {ox, oy, oz};
                TCell k;
                for (int d = 0; d < 3; ++d) {
                    k.lv[d] = c.lv[d] + (S[d] ? 1 : 0);
                    k.ix[d] = S[d] ? 2 * c.ix[d] + o[d] : c.ix[d];
                }
                k.gen = c.gen + 1;
                kids.push_back(k);
            }
}

// GL points ([k][j][i]) and physical weights of a cell, appended to x, y, z, w
void cell_points(const dg_octree& O, const TCell& c, std::vector<double>& x, std::vector<double>& y,
                 std::vector<double>& z, std::vector<double>& w) {
    const int n = O.q + 1;
    const std::vector<double>& xi = O.xi[n];
    const std::vector<double>& wr = O.wgl[n];
    double a[3], b[3];
    cell_bounds(O, c, a, b);
    double px[3][9], pw[3][9];
    for (int d = 0; d < 3; ++d)
        for (int m = 0; m < n; ++m) {
            px[d][m] = a[d] + 0.5 * (b[d] - a[d]) * (xi[m] + 1.0);
            pw[d][m] = 0.5 * (b[d] - a[d]) * wr[m];
        }
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                x.push_back(px[0][i]);
                y.push_back(px[1][j]);
                z.push_back(px[2][k]);
                w.push_back(pw[2][k] * pw[1][j] * pw[0][i]);
            }
}

void refine(dg_octree& O, dg_density_fn rho, void* user, double delta, int max_depth, long long max_elements) {
    O.tree.clear();
    for (int ez = 0; ez < O.E[2]; ++ez)
        for (int ey = 0; ey < O.E[1]; ++ey)
            for (int ex = 0; ex < O.E[0]; ++ex) {
                TCell c;
                c.lv[0] = c.lv[1] = c.lv[2] = 0;
                c.ix[0] = ex;
                c.ix[1] = ey;
                c.ix[2] = ez;
                c.gen = 0;
                c.parent = -1;
                O.tree.push_back(c);
            }
    long long leaves = (long long)O.tree.size();
    if (leaves > max_elements) throw std::invalid_argument("base mesh exceeds max_elements");
    std::vector<int> active(O.tree.size());
    for (size_t i = 0; i < active.size(); ++i) active[i] = (int)i;
    const int N3 = (O.q + 1) * (O.q + 1) * (O.q + 1);
    O.max_gen = 0;
    while (!active.empty() && rho) {
        std::vector<int> cand;
        for (int c : active)
            if (O.tree[c].gen < max_depth) cand.push_back(c);
        if (cand.empty()) break;
        std::vector<double> x, y, z, w;
        std::vector<std::vector<TCell>> kids(cand.size());
        for (size_t t = 0; t < cand.size(); ++t) {
            cell_points(O, O.tree[cand[t]], x, y, z, w);
            children_of(O, O.tree[cand[t]], kids[t]);
            for (const TCell& k : kids[t]) cell_points(O, k, x, y, z, w);
        }
        std::vector<double> v(x.size(), 0.0);
        rho((long long)x.size(), x.data(), y.data(), z.data(), v.data(), user);
        std::vector<int> next;
        size_t off = 0;
        for (size_t t = 0; t < cand.size(); ++t) {
            double I = 0.0;
            for (int m = 0; m < N3; ++m) I += v[off + m] * w[off + m];
            off += N3;
            double Ik = 0.0;
            for (size_t kk = 0; kk < kids[t].size(); ++kk) {
                double s = 0.0;
                for (int m = 0; m < N3; ++m) s += v[off + m] * w[off + m];
                off += N3;
                Ik += s;
            }
            if (!std::isfinite(I) || !std::isfinite(Ik)) throw std::invalid_argument("density is not finite");
            if (std::fabs(I - Ik) > delta) {
                const int c = cand[t];
                O.tree[c].child0 = (int)O.tree.size();
                O.tree[c].nchild = (int)kids[t].size();
                for (TCell k : kids[t]) {
                    k.parent = c;
                    next.push_back((int)O.tree.size());
                    O.tree.push_back(k);
                }
                leaves += (long long)kids[t].size() - 1;
                O.max_gen = std::max(O.max_gen, O.tree[c].gen + 1);
                if (leaves > max_elements) throw std::invalid_argument("refinement exceeds max_elements");
            }
        }
        active.swap(next);
    }
}

void collect(const dg_octree& O, int c, int gen_cut, std::vector<int>& out) {
    const TCell& t = O.tree[c];
    if (t.nchild == 0 || (gen_cut >= 0 && t.gen >= gen_cut)) {
        out.push_back(c);
        return;
    }
    for (int k = 0; k < t.nchild; ++k) collect(O, t.child0 + k, gen_cut, out);
}

int table_entry(int k, long long j) {
    if (k > KMAX) throw std::invalid_argument("level jump across a face beyond the interpolation tables");
    return (1 << k) - 1 + (int)j;
}

// Elements, pieces, diagonal of one level (cells and degree set).
void build_level(dg_octree& O, Level& L, bool finest) {
    const int n = L.n, N2 = n * n, N3 = n * n * n;
    L.ne = (int)L.cells.size();
    L.ndof = (long long)L.ne * N3;
    std::vector<double> A(3 * L.ne), B(3 * L.ne);
    int Lm[3] = {0, 0, 0};
    for (int e = 0; e < L.ne; ++e) {
        const TCell& c = O.tree[L.cells[e]];
        cell_bounds(O, c, &A[3 * e], &B[3 * e]);
        for (int d = 0; d < 3; ++d) Lm[d] = std::max(Lm[d], c.lv[d]);
    }
    L.Jh.resize(3 * L.ne);
    for (int i = 0; i < 3 * L.ne; ++i) L.Jh[i] = 0.5 * (B[i] - A[i]);
    std::vector<long long> lo(3 * L.ne), hi(3 * L.ne);
    for (int e = 0; e < L.ne; ++e) {
        const TCell& c = O.tree[L.cells[e]];
        for (int d = 0; d < 3; ++d) {
            lo[3 * e + d] = c.ix[d] << (Lm[d] - c.lv[d]);
            hi[3 * e + d] = (c.ix[d] + 1) << (Lm[d] - c.lv[d]);
        }
    }
    const long long top[3] = {(long long)O.E[0] << Lm[0], (long long)O.E[1] << Lm[1], (long long)O.E[2] << Lm[2]};
    std::vector<std::vector<Piece>> face(6 * (size_t)L.ne);
    std::vector<std::vector<int>> bpos(6 * (size_t)L.ne);  // (finest) boundary faces
    const double eps = O.opts.penalty_eps;
    const double pen = (double)(L.q + 1) * (L.q + 1) / eps;
    auto desc = [&](int e, int t, long long plo, long long plen) {
        const long long len = hi[3 * e + t] - lo[3 * e + t];
        int k = 0;
        while ((plen << k) < len) ++k;
        return table_entry(k, (plo - lo[3 * e + t]) / plen);
    };
    for (int d = 0; d < 3; ++d) {
        const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
        std::map<long long, std::vector<int>> by_lo;
        for (int e = 0; e < L.ne; ++e) by_lo[lo[3 * e + d]].push_back(e);
        for (int a = 0; a < L.ne; ++a) {
            auto it = by_lo.find(hi[3 * a + d]);
            if (it == by_lo.end()) continue;
            for (int b : it->second) {
                if (!(lo[3 * a + t1] < hi[3 * b + t1] && lo[3 * b + t1] < hi[3 * a + t1] && lo[3 * a + t2] < hi[3 * b + t2] &&
                      lo[3 * b + t2] < hi[3 * a + t2]))
                    continue;
                long long plo[2], plen[2];
                double half[2];
                int tt[2] = {t1, t2};
                for (int u = 0; u < 2; ++u) {
                    const int t = tt[u];
                    const bool aSmall = hi[3 * a + t] - lo[3 * a + t] <= hi[3 * b + t] - lo[3 * b + t];
                    const int S = aSmall ? a : b;
                    plo[u] = lo[3 * S + t];
                    plen[u] = hi[3 * S + t] - lo[3 * S + t];
                    half[u] = 0.5 * (B[3 * S + t] - A[3 * S + t]);
                }
                const double hF = std::min(B[3 * a + d] - A[3 * a + d], B[3 * b + d] - A[3 * b + d]);
                Piece pa, pb;
                pa.nb = b;
                pb.nb = a;
                pa.s1 = pb.n1 = desc(a, t1, plo[0], plen[0]);
                pa.s2 = pb.n2 = desc(a, t2, plo[1], plen[1]);
                pa.n1 = pb.s1 = desc(b, t1, plo[0], plen[0]);
                pa.n2 = pb.s2 = desc(b, t2, plo[1], plen[1]);
                pa.face = 2 * d + 1;
                pb.face = 2 * d;
                pa.sig = pb.sig = pen / hF;
                pa.wsc = pb.wsc = half[0] * half[1];
                pa.ijn = 1.0 / L.Jh[3 * b + d];
                pb.ijn = 1.0 / L.Jh[3 * a + d];
                face[6 * a + 2 * d + 1].push_back(pa);
                face[6 * b + 2 * d].push_back(pb);
            }
        }
    }
    std::vector<int> bs;
    long long nbp = 0;
    if (finest) bs.assign(6 * (size_t)L.ne, -1);
    for (int e = 0; e < L.ne; ++e)
        for (int d = 0; d < 3; ++d)
            for (int sgi = 0; sgi < 2; ++sgi) {
                const bool on = sgi == 0 ? lo[3 * e + d] == 0 : hi[3 * e + d] == top[d];
                if (!on) continue;
                const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
                Piece p;
                p.nb = -1;
                p.s1 = p.s2 = p.n1 = p.n2 = 0;
                p.face = 2 * d + sgi;
                p.sig = pen / (B[3 * e + d] - A[3 * e + d]);
                p.wsc = L.Jh[3 * e + t1] * L.Jh[3 * e + t2];
                p.ijn = 0.0;
                face[6 * e + 2 * d + sgi].push_back(p);
                if (finest) {
                    bs[6 * e + 2 * d + sgi] = (int)nbp;
                    nbp += N2;
                }
            }
    if (finest) {
        O.bsh = bs;
        O.nbp = nbp;
    }
    // per element: the conforming pieces and boundary faces, then the hanging pieces (each
    // group face by face, a face's pieces by neighbour); fsh = {first, first hanging} per element
    L.fsh.assign(2 * (size_t)L.ne + 1, 0);
    L.ph.clear();
    auto conforming = [](const Piece& p) { return p.s1 == 0 && p.s2 == 0 && p.n1 == 0 && p.n2 == 0; };
    for (int e = 0; e < L.ne; ++e) {
        for (int fc = 0; fc < 6; ++fc)
            std::sort(face[6 * e + fc].begin(), face[6 * e + fc].end(),
                      [](const Piece& x, const Piece& y) { return x.nb < y.nb; });
        L.fsh[2 * e] = (int)L.ph.size();
        for (int hang = 0; hang < 2; ++hang) {
            if (hang) L.fsh[2 * e + 1] = (int)L.ph.size();
            for (int fc = 0; fc < 6; ++fc)
                for (const Piece& p : face[6 * e + fc])
                    if (conforming(p) != (hang == 1)) L.ph.push_back(p);
        }
    }
    L.fsh[2 * (size_t)L.ne] = (int)L.ph.size();
    // diagonal: volume terms and, per piece, sum_q W T^2 sigma - kappa T d_n T (separable)
    std::vector<double> xi, w, D;
    node_rule(L.q, 1, xi, w, D);
    std::vector<double> K1d(n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int q = 0; q < n; ++q) K1d[i] += D[q * n + i] * w[q] * D[q * n + i];
    std::vector<double> eL, eR, dL, dR;
    lagrange_eval(xi, {-1.0}, eL);
    lagrange_eval(xi, {1.0}, eR);
    lagrange_deriv(xi, {-1.0}, dL);
    lagrange_deriv(xi, {1.0}, dR);
    const std::vector<double>& tab = O.tabh[n];
    L.diag.assign(L.ndof, 0.0);
    for (int e = 0; e < L.ne; ++e) {
        const double Jx = L.Jh[3 * e], Jy = L.Jh[3 * e + 1], Jz = L.Jh[3 * e + 2];
        const double Jv[3] = {Jx, Jy, Jz};
        double* De = &L.diag[(size_t)e * N3];
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i)
                    De[(k * n + j) * n + i] = Jy * Jz / Jx * w[k] * w[j] * K1d[i] + Jx * Jz / Jy * w[k] * K1d[j] * w[i] +
                                              Jx * Jy / Jz * K1d[k] * w[j] * w[i];
        for (int pi = L.fsh[2 * e]; pi < L.fsh[2 * e + 2]; ++pi) {
            const Piece& P = L.ph[pi];
            const int fc = P.face;
            const int d = fc >> 1;
            const double sg = (fc & 1) ? 1.0 : -1.0;
            const std::vector<double>& v = (fc & 1) ? eR : eL;
            const std::vector<double>& dv = (fc & 1) ? dR : dL;
            const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
            {
                const double kappa = P.nb < 0 ? 2.0 : 1.0;
                // piece half-widths along t1 and t2: this element's, shrunk by the table level
                double S1[9] = {0}, S2[9] = {0};
                auto level_of = [](int entry) {
                    int k = 0;
                    while (((2 << k) - 1) <= entry) ++k;
                    return k;
                };
                const double h1 = Jv[t1] / (double)(1 << level_of(P.s1));
                const double h2 = Jv[t2] / (double)(1 << level_of(P.s2));
                for (int a = 0; a < n; ++a)
                    for (int q = 0; q < n; ++q) {
                        const double I1 = tab[(size_t)P.s1 * N2 + q * n + a];
                        const double I2 = tab[(size_t)P.s2 * N2 + q * n + a];
                        S1[a] += h1 * w[q] * I1 * I1;
                        S2[a] += h2 * w[q] * I2 * I2;
                    }
                for (int m = 0; m < n; ++m) {
                    const double nrm = P.sig * v[m] * v[m] - kappa * v[m] * sg * dv[m] / Jv[d];
                    for (int b = 0; b < n; ++b)
                        for (int a = 0; a < n; ++a) {
                            int ii, jj, kk;
                            if (d == 0) { ii = m; jj = a; kk = b; }
                            else if (d == 1) { ii = a; jj = m; kk = b; }
                            else { ii = a; jj = b; kk = m; }
                            De[(kk * n + jj) * n + ii] += nrm * S1[a] * S2[b];
                        }
                }
            }
        }
    }
    std::vector<double> dinv(L.ndof);
    for (long long q = 0; q < L.ndof; ++q) dinv[q] = 1.0 / L.diag[q];
    L.J = upload(L.Jh);
    L.fstart = upload(L.fsh);
    L.pcs = upload(L.ph);
    L.dinv = upload(dinv);
    std::vector<float> dinv32(dinv.begin(), dinv.end());
    L.dinv32 = upload(dinv32);
}

template <int N>
Ref<N> make_ref(int q) {
    Ref<N> R;
    std::vector<double> xi, w, D, eL, eR, dL, dR;
    node_rule(q, 1, xi, w, D);
    lagrange_eval(xi, {-1.0}, eL);
    lagrange_eval(xi, {1.0}, eR);
    lagrange_deriv(xi, {-1.0}, dL);
    lagrange_deriv(xi, {1.0}, dR);
    for (int i = 0; i < N; ++i) {
        for (int a = 0; a < N; ++a) {
            double s = 0.0;
            for (int m = 0; m < N; ++m) s += D[m * N + i] * w[m] * D[m * N + a];
            R.K1[i][a] = s;
        }
        R.w[i] = w[i];
        R.eL[i] = eL[i];
        R.eR[i] = eR[i];
        R.dL[i] = dL[i];
        R.dR[i] = dR[i];
    }
    return R;
}

// the level's tables in the field type
template <typename T>
const T* tab_of(const dg_octree& O, int n);
template <>
const double* tab_of<double>(const dg_octree& O, int n) { return O.tab[n]; }
template <>
const float* tab_of<float>(const dg_octree& O, int n) { return O.tab32[n]; }
template <typename T>
const T* dinv_of(const Level& L);
template <>
const double* dinv_of<double>(const Level& L) { return L.dinv; }
template <>
const float* dinv_of<float>(const Level& L) { return L.dinv32; }

template <int N, int RB, typename T>
void op_launch_nb(const dg_octree& O, const Level& L, int mode, int nrhs, const RhsState* st, const T* u, T* y,
                  const T* f, T* r, T* z, double c1, double c2, hipStream_t s) {
    constexpr int EPB = OT / (N * N * N);
    static const Ref<N> R = make_ref<N>(N - 1);
    dim3 grid((L.ne + EPB - 1) / EPB, (nrhs + RB - 1) / RB);
    const T* tab = tab_of<T>(O, N);
    const T* dinv = dinv_of<T>(L);
    if (mode == OP_APPLY)
        hipLaunchKernelGGL((k_oct_op<N, OP_APPLY, RB, T>), grid, dim3(OT), 0, s, R, L.ne, nrhs, L.J, L.fstart, L.pcs,
                           tab, st, u, y, f, r, z, dinv, (T)c1, (T)c2);
    else if (mode == OP_RESID)
        hipLaunchKernelGGL((k_oct_op<N, OP_RESID, RB, T>), grid, dim3(OT), 0, s, R, L.ne, nrhs, L.J, L.fstart, L.pcs,
                           tab, st, u, y, f, r, z, dinv, (T)c1, (T)c2);
    else
        hipLaunchKernelGGL((k_oct_op<N, OP_CHEB, RB, T>), grid, dim3(OT), 0, s, R, L.ne, nrhs, L.J, L.fstart, L.pcs,
                           tab, st, u, y, f, r, z, dinv, (T)c1, (T)c2);
}

// right-hand sides per work-group: several share the element's geometry, pieces and tables and
// give each thread independent work between the barriers
template <int N, typename T>
void op_launch_n(const dg_octree& O, const Level& L, int mode, int nrhs, const RhsState* st, const T* u, T* y,
                 const T* f, T* r, T* z, double c1, double c2, hipStream_t s) {
    // 0: by type and degree, the fastest measured: four in FP32 and at degree 4 in FP64, else two
    const int rb = O.rhs_per_block > 0 ? O.rhs_per_block : (sizeof(T) == 4 || N == 5 ? 4 : 2);
    if (rb >= 4 && nrhs >= 4)
        op_launch_nb<N, 4, T>(O, L, mode, nrhs, st, u, y, f, r, z, c1, c2, s);
    else if (rb >= 2 && nrhs >= 2)
        op_launch_nb<N, 2, T>(O, L, mode, nrhs, st, u, y, f, r, z, c1, c2, s);
    else
        op_launch_nb<N, 1, T>(O, L, mode, nrhs, st, u, y, f, r, z, c1, c2, s);
}

template <typename T>
void op_launch(const dg_octree& O, const Level& L, int mode, int nrhs, const RhsState* st, const T* u, T* y,
               const T* f, T* r, T* z, double c1, double c2, hipStream_t s) {
    if (nrhs == 0 || L.ne == 0) return;
    switch (L.n) {
        case 2: op_launch_n<2, T>(O, L, mode, nrhs, st, u, y, f, r, z, c1, c2, s); break;
        case 3: op_launch_n<3, T>(O, L, mode, nrhs, st, u, y, f, r, z, c1, c2, s); break;
        case 4: op_launch_n<4, T>(O, L, mode, nrhs, st, u, y, f, r, z, c1, c2, s); break;
        case 5: op_launch_n<5, T>(O, L, mode, nrhs, st, u, y, f, r, z, c1, c2, s); break;
        default: throw std::invalid_argument("octree operator: degree 1 to 4");
    }
}

template <int NF, int NC, typename T>
void deg_transfer(const Level& F, bool restrict_, int nrhs, const RhsState* st, const T* a, T* b, hipStream_t s) {
    DegI<NF, NC, T> Tm;
    for (int f = 0; f < NF; ++f)
        for (int c = 0; c < NC; ++c) Tm.I[f][c] = (T)F.Ideg[f * NC + c];
    if (restrict_)
        hipLaunchKernelGGL((k_oct_restrict_deg<NF, NC, T>), node_grid((long long)F.ne * NC * NC * NC, nrhs), dim3(256),
                           0, s, Tm, F.ne, st, a, b);
    else
        hipLaunchKernelGGL((k_oct_prolong_deg<NF, NC, T>), node_grid((long long)F.ne * NF * NF * NF, nrhs), dim3(256),
                           0, s, Tm, F.ne, st, a, b);
}

// restrict (rc = R rf) or prolong-and-add (zf += P zc) between level l and l + 1
template <typename T>
void transfer(const dg_octree& O, int l, bool restrict_, int nrhs, const RhsState* st, const T* a, T* b,
              hipStream_t s) {
    const Level& F = O.lv[l];
    const Level& C = O.lv[l + 1];
    if (F.kind == 2) {
        if (restrict_)
            hipLaunchKernelGGL((k_oct_restrict_mesh<T>), node_grid((long long)C.ne * 8, nrhs), dim3(256), 0, s, F.ne,
                               C.ne, F.kstart, F.kids, F.msel, tab_of<T>(O, 2), st, a, b);
        else
            hipLaunchKernelGGL((k_oct_prolong_mesh<T>), node_grid((long long)F.ne * 8, nrhs), dim3(256), 0, s, F.ne,
                               C.ne, F.par, F.msel, tab_of<T>(O, 2), st, a, b);
        return;
    }
    const int key = F.n * 10 + C.n;
    switch (key) {
        case 53: deg_transfer<5, 3, T>(F, restrict_, nrhs, st, a, b, s); break;
        case 32: deg_transfer<3, 2, T>(F, restrict_, nrhs, st, a, b, s); break;
        case 42: deg_transfer<4, 2, T>(F, restrict_, nrhs, st, a, b, s); break;
        default: throw std::logic_error("octree: no degree transfer for this pair");
    }
}

void ensure_work(dg_octree& O, int nrhs) {
    if (nrhs <= O.cap) return;
    auto fr = [](std::vector<double*>& v) {
        for (auto& p : v) ofree(p);
        v.clear();
    };
    fr(O.wf);
    fr(O.wz);
    fr(O.wr);
    fr(O.wd0);
    fr(O.wd1);
    fr(O.wt);
    ofree(O.cscr);
    ofree(O.px);
    ofree(O.pr);
    ofree(O.pz);
    ofree(O.pp);
    ofree(O.pq);
    ofree(O.partial);
    for (const Level& L : O.lv) {
        const long long n = L.ndof * nrhs;
        O.wf.push_back(oalloc<double>(n));
        O.wz.push_back(oalloc<double>(n));
        O.wr.push_back(oalloc<double>(n));
        O.wd0.push_back(oalloc<double>(n));
        O.wd1.push_back(oalloc<double>(n));
        O.wt.push_back(oalloc<double>(n));
    }
    O.cscr = oalloc<double>(2LL * nrhs * O.lv.back().ndof);
    const long long n0 = O.lv[0].ndof * nrhs;
    O.px = oalloc<double>(n0);
    O.pr = oalloc<double>(n0);
    O.pz = oalloc<double>(n0);
    O.pp = oalloc<double>(n0);
    O.pq = oalloc<double>(n0);
    ofree(O.r32);
    ofree(O.z32);
    if (O.fp32) {
        O.r32 = oalloc<float>(n0);
        O.z32 = oalloc<float>(n0);
    }
    O.pstride = chunks_of(O.lv[0].ndof);
    O.partial = oalloc<double>((long long)nrhs * O.pstride);
    O.cap = nrhs;
}

void ensure_state(dg_octree& O, int nrhs) {
    if (nrhs <= O.st_cap) return;
    ofree(O.st);
    O.st = oalloc<RhsState>(nrhs);
    O.st_cap = nrhs;
}

// Chebyshev smoothing of level l on f from z (zero_start: z = 0), the work vectors of the level
// (the FP64 buffers hold FP32 values in their first half when T is float)
template <typename T>
void smooth(dg_octree& O, int l, int nrhs, const RhsState* st, const T* f, T* z, bool zero_start, hipStream_t s) {
    const Level& L = O.lv[l];
    T* r = reinterpret_cast<T*>(O.wr[l]);
    T* d0 = reinterpret_cast<T*>(O.wd0[l]);
    T* d1 = reinterpret_cast<T*>(O.wd1[l]);
    const T* dinv = dinv_of<T>(L);
    if (zero_start) {
        hipLaunchKernelGGL((k_oct_start0<T>), node_grid(L.ndof, nrhs), dim3(256), 0, s, L.ndof, st, f, r, z, d0, dinv,
                           (T)L.c0);
    } else {
        op_launch<T>(O, L, OP_RESID, nrhs, st, z, r, f, nullptr, nullptr, 0.0, 0.0, s);
        hipLaunchKernelGGL((k_oct_dstart<T>), node_grid(L.ndof, nrhs), dim3(256), 0, s, L.ndof, st, r, d0, dinv,
                           (T)L.c0);
    }
    for (int k = 1; k < L.degree; ++k) {
        op_launch<T>(O, L, OP_CHEB, nrhs, st, d0, d1, nullptr, r, z, L.cp[k - 1], L.cr[k - 1], s);
        std::swap(d0, d1);
    }
    hipLaunchKernelGGL((k_oct_add<T>), node_grid(L.ndof, nrhs), dim3(256), 0, s, L.ndof, st, d0, z);
}

// z = V f on level l (f is not modified)
template <typename T>
void vcycle(dg_octree& O, int l, int nrhs, const RhsState* st, const T* f, T* z, hipStream_t s) {
    const int nl = (int)O.lv.size();
    if (l == nl - 1) {
        launch_coarse<T>(O.cdev, O.base, nrhs, st, f, z, O.cscr, s);
        return;
    }
    const Level& L = O.lv[l];
    T* t = reinterpret_cast<T*>(O.wt[l]);
    T* fc = reinterpret_cast<T*>(O.wf[l + 1]);
    T* zc = reinterpret_cast<T*>(O.wz[l + 1]);
    smooth<T>(O, l, nrhs, st, f, z, true, s);
    op_launch<T>(O, L, OP_RESID, nrhs, st, z, t, f, nullptr, nullptr, 0.0, 0.0, s);
    transfer<T>(O, l, true, nrhs, st, t, fc, s);
    vcycle<T>(O, l + 1, nrhs, st, fc, zc, s);
    transfer<T>(O, l, false, nrhs, st, zc, z, s);
    smooth<T>(O, l, nrhs, st, f, z, false, s);
}

// the preconditioner z = V r at the finest level in the solve's V-cycle precision
void precondition(dg_octree& O, int nrhs, const RhsState* st, const double* r, double* z, hipStream_t s) {
    if (!O.fp32) {
        vcycle<double>(O, 0, nrhs, st, r, z, s);
        return;
    }
    const long long n = O.lv[0].ndof * nrhs;
    const dim3 g((unsigned)((n + 255) / 256));
    hipLaunchKernelGGL(k_oct_narrow, g, dim3(256), 0, s, n, st, O.lv[0].ndof, r, O.r32);
    vcycle<float>(O, 0, nrhs, st, O.r32, O.z32, s);
    hipLaunchKernelGGL(k_oct_widen, g, dim3(256), 0, s, n, st, O.lv[0].ndof, O.z32, z);
}

void lanczos_bounds(dg_octree& O, int l, hipStream_t s) {
    Level& L = O.lv[l];
    const long long n = L.ndof;
    std::vector<double> h(n);
    double nrm = 0.0;
    for (long long i = 0; i < n; ++i) {
        const uint32_t v = (uint32_t)((uint64_t)i * 2654435761ull + 12345ull);
        h[i] = (double)v / 4294967296.0 - 0.5;
        nrm += h[i] * h[i];
    }
    nrm = std::sqrt(nrm);
    for (auto& x : h) x /= nrm;
    double* v = upload(h);
    double *vp = oalloc<double>(n), *w = oalloc<double>(n), *tmp = oalloc<double>(n);
    const int nc = chunks_of(n);
    double* part = oalloc<double>(nc);
    launch_fill<double>(vp, 0.0, n, s);
    std::vector<double> alphas, betas, hp(nc);
    auto dot = [&](const double* a, const double* b) {
        launch_dot<double, double>(n, 1, nullptr, a, b, part, nc, s);
        OCHK(hipMemcpyAsync(hp.data(), part, sizeof(double) * nc, hipMemcpyDeviceToHost, s));
        OCHK(hipStreamSynchronize(s));
        double acc = 0.0;
        for (double x : hp) acc += x;
        return acc;
    };
    double beta = 0.0;
    const int steps = (int)std::min<long long>(O.opts.lanczos_steps, n);
    for (int k = 0; k < steps; ++k) {
        hipLaunchKernelGGL(k_oct_dscale, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, L.dinv, v, tmp);
        op_launch<double>(O, L, OP_APPLY, 1, nullptr, tmp, w, nullptr, nullptr, nullptr, 0.0, 0.0, s);
        hipLaunchKernelGGL(k_oct_dscale, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, L.dinv, w, w);
        launch_axpby(n, -beta, vp, 1.0, w, s);
        const double alpha = dot(w, v);
        launch_axpby(n, -alpha, v, 1.0, w, s);
        alphas.push_back(alpha);
        beta = std::sqrt(std::max(0.0, dot(w, w)));
        if (k == steps - 1 || beta == 0.0) break;
        betas.push_back(beta);
        std::swap(v, vp);
        launch_copy(w, v, n, s);
        launch_axpby(n, 0.0, w, 1.0 / beta, v, s);
    }
    OCHK(hipStreamSynchronize(s));
    OCHK(hipGetLastError());
    ofree(v);
    ofree(vp);
    ofree(w);
    ofree(tmp);
    ofree(part);
    betas.resize(alphas.size() > 0 ? alphas.size() - 1 : 0);
    const double lmax = tridiag_max_eig(alphas, betas);
    L.lam_hi = O.opts.cheb_safety * lmax;
    L.lam_lo = L.lam_hi / O.opts.cheb_ratio;
    const double theta = 0.5 * (L.lam_hi + L.lam_lo), delta = 0.5 * (L.lam_hi - L.lam_lo);
    const double sigma1 = theta / delta;
    L.c0 = 1.0 / theta;
    double rho = 1.0 / sigma1;
    L.degree = (l >= 1 && L.q == 1 && O.opts.cheb_degree_h > 0) ? O.opts.cheb_degree_h : O.opts.cheb_degree;
    L.cp.clear();
    L.cr.clear();
    for (int k = 1; k < L.degree; ++k) {
        const double rn = 1.0 / (2.0 * sigma1 - rho);
        L.cp.push_back(rn * rho);
        L.cr.push_back(2.0 * rn / delta);
        rho = rn;
    }
}

void build_tables(dg_octree& O, int n) {
    std::vector<double> xi, w, D;
    node_rule(n - 1, 1, xi, w, D);
    O.xi[n] = xi;
    O.wgl[n] = w;
    std::vector<double>& T = O.tabh[n];
    T.assign((size_t)NTAB * n * n, 0.0);
    for (int k = 0; k <= KMAX; ++k)
        for (long long j = 0; j < (1LL << k); ++j) {
            std::vector<double> x(n), Lm;
            for (int q = 0; q < n; ++q) x[q] = -1.0 + (2.0 * j + 1.0 + xi[q]) / (double)(1LL << k);
            lagrange_eval(xi, x, Lm);
            std::copy(Lm.begin(), Lm.end(), T.begin() + (size_t)table_entry(k, j) * n * n);
        }
    O.tab[n] = upload(T);
    std::vector<float> T32(T.begin(), T.end());
    O.tab32[n] = upload(T32);
}

}  // namespace

void destroy(dg_octree* O) {
    if (!O) return;
    (void)hipSetDevice(O->device);
    for (Level& L : O->lv) {
        ofree(L.J);
        ofree(L.fstart);
        ofree(L.pcs);
        ofree(L.dinv);
        ofree(L.dinv32);
        ofree(L.par);
        ofree(L.msel);
        ofree(L.kstart);
        ofree(L.kids);
    }
    for (auto& t : O->tab) ofree(t);
    for (auto& t : O->tab32) ofree(t);
    ofree(O->r32);
    ofree(O->z32);
    ofree(O->bstart);
    ofree(O->qnodes);
    ofree(O->qpart);
    ofree(O->xrho);
    ofree(O->xb);
    ofree(O->xv);
    ofree(O->xpart);
    ofree(O->xg);
    ofree(O->xpi);
    ofree(O->xpj);
    ofree(O->cdev);
    for (auto* v : {&O->wf, &O->wz, &O->wr, &O->wd0, &O->wd1, &O->wt})
        for (auto& p : *v) ofree(p);
    ofree(O->cscr);
    ofree(O->px);
    ofree(O->pr);
    ofree(O->pz);
    ofree(O->pp);
    ofree(O->pq);
    ofree(O->partial);
    ofree(O->st);
    delete O;
}

dg_octree* create(const dg_octree_desc& D, dg_density_fn rho, void* user, const dg_opts& opts) {
    for (int d = 0; d < 3; ++d)
        if (D.ne[d] < 1 || D.ne[d] > 8 || !(D.hi[d] > D.lo[d]))
            throw std::invalid_argument("octree base mesh: 1 to 8 elements per axis on a non-empty box");
    if (D.q < 1 || D.q > 4) throw std::invalid_argument("octree degree q: 1 to 4");
    if (D.max_depth < 0 || D.max_depth > KMAX) throw std::invalid_argument("octree max_depth: 0 to 8");
    if (!(D.delta_q > 0.0)) throw std::invalid_argument("octree delta_q must be positive");
    if (D.max_elements < 1) throw std::invalid_argument("octree max_elements must be positive");
    if (opts.precision != DG_PREC_FP64 && opts.precision != DG_PREC_FP32_PC)
        throw std::invalid_argument("octree solves: precision FP64 or FP32_PC");
    if (opts.cheb_degree < 1 || opts.cheb_degree_h < 0 || opts.cheb_ratio <= 1.0 || opts.cheb_safety < 1.0 ||
        opts.lanczos_steps < 2 || !(opts.penalty_eps > 0.0) || !(opts.rtol > 0.0) || opts.max_iter < 0)
        throw std::invalid_argument("invalid solver options");
    dg_octree* O = new dg_octree();
    try {
        OCHK(hipGetDevice(&O->device));
        for (int d = 0; d < 3; ++d) {
            O->E[d] = D.ne[d];
            O->lo[d] = D.lo[d];
            O->hi[d] = D.hi[d];
            O->h[d] = (D.hi[d] - D.lo[d]) / D.ne[d];
        }
        O->q = D.q;
        O->opts = opts;
        O->fp32 = opts.precision == DG_PREC_FP32_PC;
        for (int n = 2; n <= D.q + 1; ++n) build_tables(*O, n);
        refine(*O, rho, user, D.delta_q, D.max_depth, D.max_elements);
        // levels: degree steps on the leaves, then the tree cut at generation G-1 .. 0 at degree 1
        std::vector<std::pair<int, int>> specs;  // (gen_cut, q); gen_cut -1: the leaves
        int qq = D.q;
        specs.push_back({-1, qq});
        while (qq > 1) {
            qq /= 2;
            specs.push_back({-1, qq});
        }
        for (int g = O->max_gen - 1; g >= 0; --g) specs.push_back({g, 1});
        const int nroot = D.ne[0] * D.ne[1] * D.ne[2];
        O->lv.resize(specs.size());
        for (size_t l = 0; l < specs.size(); ++l) {
            Level& L = O->lv[l];
            L.q = specs[l].second;
            L.n = L.q + 1;
            for (int c = 0; c < nroot; ++c) collect(*O, c, specs[l].first, L.cells);
            build_level(*O, L, l == 0);
        }
        O->bstart = upload(O->bsh);
        // transfers
        for (size_t l = 0; l + 1 < O->lv.size(); ++l) {
            Level& F = O->lv[l];
            Level& C = O->lv[l + 1];
            if (F.q != C.q) {
                F.kind = 1;
                std::vector<double> Lm;
                lagrange_eval(O->xi[C.n], O->xi[F.n], Lm);
                F.Ideg = Lm;
                continue;
            }
            F.kind = 2;
            std::map<int, int> elem_of;  // tree cell -> coarse element
            for (int e = 0; e < C.ne; ++e) elem_of[C.cells[e]] = e;
            std::vector<int> par(F.ne), msel(3 * F.ne);
            std::vector<std::vector<int>> kl(C.ne);
            for (int e = 0; e < F.ne; ++e) {
                const int c = F.cells[e];
                auto it = elem_of.find(c);
                const int pc = it != elem_of.end() ? c : O->tree[c].parent;
                const int ce = elem_of.at(pc);
                par[e] = ce;
                kl[ce].push_back(e);
                for (int d = 0; d < 3; ++d) {
                    const int k = O->tree[c].lv[d] - O->tree[pc].lv[d];
                    msel[3 * e + d] = k == 0 ? 0 : 1 + (int)(O->tree[c].ix[d] & 1);
                }
            }
            std::vector<int> ks(C.ne + 1, 0), kids;
            for (int e = 0; e < C.ne; ++e) {
                ks[e] = (int)kids.size();
                kids.insert(kids.end(), kl[e].begin(), kl[e].end());
            }
            ks[C.ne] = (int)kids.size();
            F.par = upload(par);
            F.msel = upload(msel);
            F.kstart = upload(ks);
            F.kids = upload(kids);
        }
        // coarsest: the base mesh at degree 1, exact solve by fast diagonalisation
        LevelHost& B = O->base;
        for (int d = 0; d < 3; ++d) {
            B.E[d] = D.ne[d];
            B.lo[d] = D.lo[d];
            B.h[d] = O->h[d];
        }
        B.p = 1;
        B.n = 2;
        B.family = 1;
        B.ndof = (long long)nroot * 8;
        CoarseDev C;
        build_coarse(B, opts.penalty_eps, C);
        O->cdev = oalloc<CoarseDev>(1);
        OCHK(hipMemcpy(O->cdev, &C, sizeof(C), hipMemcpyHostToDevice));
        if (O->lv.back().ne != nroot || O->lv.back().q != 1) throw std::logic_error("octree: coarsest level");
        hipStream_t s = nullptr;
        for (size_t l = 0; l + 1 < O->lv.size(); ++l) lanczos_bounds(*O, (int)l, s);
        OCHK(hipDeviceSynchronize());
    } catch (...) {
        destroy(O);
        throw;
    }
    return O;
}

long long n_dofs(const dg_octree* O) { return O->lv[0].ndof; }

void node_coords(const dg_octree* O, double* x, double* y, double* z) {
    const Level& L = O->lv[0];
    const int n = L.n;
    const std::vector<double>& xi = O->xi[n];
    long long off = 0;
    for (int e = 0; e < L.ne; ++e) {
        double a[3], b[3];
        cell_bounds(*O, O->tree[L.cells[e]], a, b);
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i, ++off) {
                    x[off] = a[0] + 0.5 * (b[0] - a[0]) * (xi[i] + 1.0);
                    y[off] = a[1] + 0.5 * (b[1] - a[1]) * (xi[j] + 1.0);
                    z[off] = a[2] + 0.5 * (b[2] - a[2]) * (xi[k] + 1.0);
                }
    }
}

void boundary_coords(const dg_octree* O, double* x, double* y, double* z) {
    const Level& L = O->lv[0];
    const int n = L.n;
    const std::vector<double>& xi = O->xi[n];
    for (int e = 0; e < L.ne; ++e) {
        double a[3], b[3];
        cell_bounds(*O, O->tree[L.cells[e]], a, b);
        for (int fc = 0; fc < 6; ++fc) {
            const int off = O->bsh[6 * e + fc];
            if (off < 0) continue;
            const int d = fc >> 1;
            const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
            for (int bb = 0; bb < n; ++bb)
                for (int aa = 0; aa < n; ++aa) {
                    double P[3];
                    P[d] = (fc & 1) ? b[d] : a[d];
                    P[t1] = a[t1] + 0.5 * (b[t1] - a[t1]) * (xi[aa] + 1.0);
                    P[t2] = a[t2] + 0.5 * (b[t2] - a[t2]) * (xi[bb] + 1.0);
                    const long long o = off + bb * n + aa;
                    x[o] = P[0];
                    y[o] = P[1];
                    z[o] = P[2];
                }
        }
    }
}

void elements(const dg_octree* O, double* lohi, int* gen) {
    const Level& L = O->lv[0];
    for (int e = 0; e < L.ne; ++e) {
        double a[3], b[3];
        const TCell& c = O->tree[L.cells[e]];
        cell_bounds(*O, c, a, b);
        if (lohi)
            for (int d = 0; d < 3; ++d) {
                lohi[6 * e + d] = a[d];
                lohi[6 * e + 3 + d] = b[d];
            }
        if (gen) gen[e] = c.gen;
    }
}

void info(const dg_octree* O, long long* ne, long long* ndof, long long* nbp, int* nlev, int* max_gen) {
    if (ne) *ne = O->lv[0].ne;
    if (ndof) *ndof = O->lv[0].ndof;
    if (nbp) *nbp = O->nbp;
    if (nlev) *nlev = (int)O->lv.size();
    if (max_gen) *max_gen = O->max_gen;
}

void level_info(const dg_octree* O, int level, long long* ne, int* q, double* lam_lo, double* lam_hi) {
    if (level < 0 || level >= (int)O->lv.size()) throw std::invalid_argument("level out of range");
    const Level& L = O->lv[level];
    if (ne) *ne = L.ne;
    if (q) *q = L.q;
    if (lam_lo) *lam_lo = L.lam_lo;
    if (lam_hi) *lam_hi = L.lam_hi;
}

void boundary_data(dg_octree* O, int nsrc, const double* f, double* g, hipStream_t s);

void rhs(dg_octree* O, int nrhs, const double* f, const double* g, double* b, hipStream_t s) {
    const Level& L = O->lv[0];
    if (!g && O->nbp > 0) {  // Dirichlet data by quadrature of f
        const long long need = (long long)nrhs * O->nbp;
        if (need > O->xg_cap) {
            ofree(O->xg);
            O->xg = oalloc<double>(need);
            O->xg_cap = need;
        }
        boundary_data(O, nrhs, f, O->xg, s);
        g = O->xg;
    }
    const double pen = (double)(L.q + 1) * (L.q + 1) / O->opts.penalty_eps;
    const dim3 grid = node_grid(L.ndof, nrhs);
    switch (L.n) {
        case 2: hipLaunchKernelGGL(k_oct_rhs<2>, grid, dim3(256), 0, s, make_ref<2>(1), L.ne, O->nbp, pen, L.J, O->bstart, f, g, b); break;
        case 3: hipLaunchKernelGGL(k_oct_rhs<3>, grid, dim3(256), 0, s, make_ref<3>(2), L.ne, O->nbp, pen, L.J, O->bstart, f, g, b); break;
        case 4: hipLaunchKernelGGL(k_oct_rhs<4>, grid, dim3(256), 0, s, make_ref<4>(3), L.ne, O->nbp, pen, L.J, O->bstart, f, g, b); break;
        case 5: hipLaunchKernelGGL(k_oct_rhs<5>, grid, dim3(256), 0, s, make_ref<5>(4), L.ne, O->nbp, pen, L.J, O->bstart, f, g, b); break;
    }
    OCHK(hipGetLastError());
}

// node coordinates and GL weights of the finest level, then the Dirichlet points (device, once)
void ensure_qnodes(dg_octree* O) {
    const Level& L = O->lv[0];
    const long long nd = L.ndof, nb = O->nbp;
    if (O->qnodes) return;
    {
        std::vector<double> h(4 * nd + 3 * nb);
        node_coords(O, &h[0], &h[nd], &h[2 * nd]);
        const int n = L.n;
        const std::vector<double>& w = O->wgl[n];
        for (int e = 0; e < L.ne; ++e) {
            const double J3 = L.Jh[3 * e] * L.Jh[3 * e + 1] * L.Jh[3 * e + 2];
            for (int k = 0; k < n; ++k)
                for (int j = 0; j < n; ++j)
                    for (int i = 0; i < n; ++i)
                        h[3 * nd + (long long)e * n * n * n + (k * n + j) * n + i] = J3 * w[k] * w[j] * w[i];
        }
        if (nb > 0) boundary_coords(O, &h[4 * nd], &h[4 * nd + nb], &h[4 * nd + 2 * nb]);
        O->qnodes = upload(h);
    }
}

void boundary_data(dg_octree* O, int nsrc, const double* f, double* g, hipStream_t s) {
    const Level& L = O->lv[0];
    const long long nd = L.ndof, nb = O->nbp;
    if (nsrc == 0 || nb == 0) return;
    ensure_qnodes(O);
    const int pblocks = (int)((nb + BT - 1) / BT), sblocks = (nsrc + BR - 1) / BR;
    const long long tiles = (nd + BT - 1) / BT;
    // node parts: enough work-groups for several per compute unit
    long long parts = std::max<long long>(1, std::min<long long>(tiles, (4096 + pblocks * sblocks - 1) /
                                                                            ((long long)pblocks * sblocks)));
    parts = std::min<long long>(parts, 65535);
    const int tpp = (int)((tiles + parts - 1) / parts);
    parts = (tiles + tpp - 1) / tpp;
    const long long need = parts * nsrc * nb;
    if (need > O->qpart_cap) {
        ofree(O->qpart);
        O->qpart = oalloc<double>(need);
        O->qpart_cap = need;
    }
    const double* q = O->qnodes;
    hipLaunchKernelGGL(k_oct_bdata, dim3(pblocks, sblocks, (unsigned)parts), dim3(BT), 0, s, nd, (int)nb, nsrc, tpp,
                       q, q + nd, q + 2 * nd, q + 3 * nd, q + 4 * nd, q + 4 * nd + nb, q + 4 * nd + 2 * nb, f,
                       O->qpart);
    hipLaunchKernelGGL(k_oct_bsum, dim3((unsigned)((nsrc * nb + 255) / 256)), dim3(256), 0, s, (int)parts, nsrc,
                       (int)nb, O->qpart, g);
    OCHK(hipGetLastError());
}

void apply(dg_octree* O, int level, int nrhs, const double* u, double* y, hipStream_t s) {
    if (level < 0 || level >= (int)O->lv.size()) throw std::invalid_argument("level out of range");
    op_launch<double>(*O, O->lv[level], OP_APPLY, nrhs, nullptr, u, y, nullptr, nullptr, nullptr, 0.0, 0.0, s);
    OCHK(hipGetLastError());
}

void apply_f32(dg_octree* O, int level, int nrhs, const float* u, float* y, hipStream_t s) {
    if (level < 0 || level >= (int)O->lv.size()) throw std::invalid_argument("level out of range");
    op_launch<float>(*O, O->lv[level], OP_APPLY, nrhs, nullptr, u, y, nullptr, nullptr, nullptr, 0.0, 0.0, s);
    OCHK(hipGetLastError());
}

void vcycle_once(dg_octree* O, int nrhs, const double* r, double* z, hipStream_t s) {
    ensure_work(*O, nrhs);
    vcycle<double>(*O, 0, nrhs, nullptr, r, z, s);
    OCHK(hipGetLastError());
}

// FP64 MG-PCG on the finest level; returns the worst status over the right-hand sides
int solve(dg_octree* O, int nrhs, const double* b, double* x, dg_rhs_stats* stats, hipStream_t s) {
    ensure_work(*O, nrhs);
    ensure_state(*O, nrhs);
    const Level& L = O->lv[0];
    const long long n = L.ndof;
    const int nc = chunks_of(n);
    std::vector<RhsState> h(nrhs);
    for (auto& S : h) {
        std::memset(&S, 0, sizeof(S));
        S.tol2 = O->opts.rtol * O->opts.rtol;
        S.maxit = O->opts.max_iter;
        S.active = 1;
    }
    RhsState* st = O->st;
    OCHK(hipMemcpyAsync(st, h.data(), sizeof(RhsState) * nrhs, hipMemcpyHostToDevice, s));
    OCHK(hipMemcpyAsync(O->pr, b, sizeof(double) * n * nrhs, hipMemcpyDeviceToDevice, s));
    launch_fill<double>(x, 0.0, n * nrhs, s);
    launch_fill<double>(O->pp, 0.0, n * nrhs, s);
    launch_dot<double, double>(n, nrhs, nullptr, b, b, O->partial, O->pstride, s);
    launch_finalize(FIN_BB, nrhs, st, O->partial, O->pstride, nc, s);
    launch_dot<double, double>(n, nrhs, nullptr, O->pr, O->pr, O->partial, O->pstride, s);
    launch_finalize(FIN_RR0, nrhs, st, O->partial, O->pstride, nc, s);
    const int every = std::max(1, O->opts.check_every);
    for (int it = 0; it < O->opts.max_iter;) {
        for (int k = 0; k < every && it < O->opts.max_iter; ++k, ++it) {
            precondition(*O, nrhs, st, O->pr, O->pz, s);
            launch_dot<double, double>(n, nrhs, st, O->pr, O->pz, O->partial, O->pstride, s);
            launch_finalize(FIN_RZ, nrhs, st, O->partial, O->pstride, nc, s);
            hipLaunchKernelGGL(k_oct_pdir, node_grid(n, nrhs), dim3(256), 0, s, n, st, O->pz, O->pp);
            op_launch<double>(*O, L, OP_APPLY, nrhs, st, O->pp, O->pq, nullptr, nullptr, nullptr, 0.0, 0.0, s);
            launch_dot<double, double>(n, nrhs, st, O->pp, O->pq, O->partial, O->pstride, s);
            launch_finalize(FIN_PQ, nrhs, st, O->partial, O->pstride, nc, s);
            hipLaunchKernelGGL(k_oct_xr, node_grid(n, nrhs), dim3(256), 0, s, n, st, O->pp, O->pq, x, O->pr);
            launch_dot<double, double>(n, nrhs, st, O->pr, O->pr, O->partial, O->pstride, s);
            launch_finalize(FIN_RR, nrhs, st, O->partial, O->pstride, nc, s);
        }
        OCHK(hipMemcpyAsync(h.data(), st, sizeof(RhsState) * nrhs, hipMemcpyDeviceToHost, s));
        OCHK(hipStreamSynchronize(s));
        bool any = false;
        for (const auto& S : h) any = any || S.active;
        if (!any) break;
    }
    OCHK(hipGetLastError());
    // FP64 residual of the returned solution
    op_launch<double>(*O, L, OP_RESID, nrhs, nullptr, x, O->pr, b, nullptr, nullptr, 0.0, 0.0, s);
    launch_dot<double, double>(n, nrhs, nullptr, O->pr, O->pr, O->partial, O->pstride, s);
    std::vector<double> part((size_t)nrhs * O->pstride);
    OCHK(hipMemcpyAsync(part.data(), O->partial, sizeof(double) * part.size(), hipMemcpyDeviceToHost, s));
    OCHK(hipMemcpyAsync(h.data(), st, sizeof(RhsState) * nrhs, hipMemcpyDeviceToHost, s));
    OCHK(hipStreamSynchronize(s));
    int worst = DG_OK;
    for (int i = 0; i < nrhs; ++i) {
        double rr = 0.0;
        for (int c = 0; c < nc; ++c) rr += part[(size_t)i * O->pstride + c];
        const RhsState& S = h[i];
        const double rel = S.bb > 0.0 ? std::sqrt(rr / S.bb) : 0.0;
        int status = DG_OK;
        if (S.breakdown) status = DG_ERR_BREAKDOWN;
        else if (S.bb > 0.0 && S.rr > S.tol2 * S.bb) status = DG_WARN_NOT_CONVERGED;
        if (status == DG_ERR_BREAKDOWN || (status == DG_WARN_NOT_CONVERGED && worst == DG_OK)) worst = status;
        if (stats) {
            stats[i].iters = S.iters;
            stats[i].outer_iters = 1;
            stats[i].status = status;
            stats[i].guess_used = 0;
            stats[i].rel_residual = rel;
        }
    }
    return worst;
}

// Exchange: pair densities, their right-hand sides (data given or by quadrature), the solves,
// W_k and K_ij; returns the worst solve status.
int exchange(dg_octree* O, int norb, const double* phi, const double* g, double* v_out, double* W, double* K,
             double* ex, dg_rhs_stats* stats, hipStream_t s) {
    const long long nd = O->lv[0].ndof;
    const int np = norb * (norb + 1) / 2;
    std::vector<int> hi, hj;
    for (int i = 0; i < norb; ++i)
        for (int j = i; j < norb; ++j) {
            hi.push_back(i);
            hj.push_back(j);
        }
    if (norb != O->xnorb) {
        ofree(O->xpi);
        ofree(O->xpj);
        O->xpi = upload(hi);
        O->xpj = upload(hj);
        O->xnorb = norb;
    }
    if ((long long)np * nd > O->xcap) {
        ofree(O->xrho);
        ofree(O->xb);
        ofree(O->xv);
        O->xrho = oalloc<double>(np * nd);
        O->xb = oalloc<double>(np * nd);
        O->xv = oalloc<double>(np * nd);
        O->xcap = np * nd;
    }
    const int nchunk = chunks_of(nd);
    if ((long long)np * nchunk > O->xpart_cap) {
        ofree(O->xpart);
        O->xpart = oalloc<double>((long long)np * nchunk);
        O->xpart_cap = (long long)np * nchunk;
    }
    double* v = v_out ? v_out : O->xv;
    launch_pair_products(nd, np, phi, O->xpi, O->xpj, O->xrho, s);
    rhs(O, np, O->xrho, g, O->xb, s);
    const int worst = solve(O, np, O->xb, v, stats, s);
    if (W) hipLaunchKernelGGL(k_oct_wk, dim3((unsigned)((nd + 255) / 256), norb), dim3(256), 0, s, nd, norb, phi, v, W);
    ensure_qnodes(O);
    hipLaunchKernelGGL(k_oct_kij, dim3(nchunk, np), dim3(256), 0, s, nd, O->xpi, O->xpj, phi, v, O->qnodes + 3 * nd,
                       O->xpart, nchunk);
    std::vector<double> hp((size_t)np * nchunk);
    OCHK(hipMemcpyAsync(hp.data(), O->xpart, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, s));
    OCHK(hipStreamSynchronize(s));
    double e = 0.0;
    for (int p = 0; p < np; ++p) {
        double k = 0.0;
        for (int c = 0; c < nchunk; ++c) k += hp[(size_t)p * nchunk + c];
        if (K) K[p] = k;
        e += (hi[p] == hj[p] ? 1.0 : 2.0) * k;
    }
    if (ex) *ex = e;
    return worst;
}

}  // namespace oct
}  // namespace dg

// ---------------------------------------------------------------------------------------------
// C ABI

extern "C" {

dg_status dg_octree_create(const dg_octree_desc* desc, dg_density_fn rho, void* user, const dg_opts* opts,
                           dg_octree** out) {
    return dg::guarded([&] {
        if (!desc || !out) throw std::invalid_argument("null argument");
        *out = nullptr;
        dg_opts o;
        if (opts) o = *opts;
        else dg_opts_default(&o);
        *out = dg::oct::create(*desc, rho, user, o);
    });
}

dg_status dg_octree_info(const dg_octree* o, long long* n_elements, long long* n_dofs, long long* n_boundary,
                         int* n_levels, int* max_generation) {
    return dg::guarded([&] {
        if (!o) throw std::invalid_argument("null octree");
        dg::oct::info(o, n_elements, n_dofs, n_boundary, n_levels, max_generation);
    });
}

dg_status dg_octree_level_info(const dg_octree* o, int level, long long* n_elements, int* q, double* lam_lo,
                               double* lam_hi) {
    return dg::guarded([&] {
        if (!o) throw std::invalid_argument("null octree");
        dg::oct::level_info(o, level, n_elements, q, lam_lo, lam_hi);
    });
}

dg_status dg_octree_elements(const dg_octree* o, double* lohi, int* generation) {
    return dg::guarded([&] {
        if (!o) throw std::invalid_argument("null octree");
        dg::oct::elements(o, lohi, generation);
    });
}

dg_status dg_octree_nodes(const dg_octree* o, double* x, double* y, double* z) {
    return dg::guarded([&] {
        if (!o || !x || !y || !z) throw std::invalid_argument("null argument");
        dg::oct::node_coords(o, x, y, z);
    });
}

dg_status dg_octree_boundary_points(const dg_octree* o, double* x, double* y, double* z) {
    return dg::guarded([&] {
        if (!o || ((!x || !y || !z) && o->nbp > 0)) throw std::invalid_argument("null argument");
        dg::oct::boundary_coords(o, x, y, z);
    });
}

dg_status dg_octree_rhs(dg_octree* o, int nrhs, const double* f, const double* g, double* b, void* stream) {
    return dg::guarded([&] {
        if (!o || nrhs < 0) throw std::invalid_argument("bad arguments");
        if (nrhs == 0) return;
        if (!f || !b) throw std::invalid_argument("null argument");
        (void)hipSetDevice(o->device);
        dg::oct::rhs(o, nrhs, f, g, b, (hipStream_t)stream);
    });
}

dg_status dg_octree_boundary_data(dg_octree* o, int nsrc, const double* f, double* g, void* stream) {
    return dg::guarded([&] {
        if (!o || nsrc < 0) throw std::invalid_argument("bad arguments");
        if (nsrc == 0) return;
        if (!f || (!g && o->nbp > 0)) throw std::invalid_argument("null argument");
        (void)hipSetDevice(o->device);
        dg::oct::boundary_data(o, nsrc, f, g, (hipStream_t)stream);
    });
}

dg_status dg_octree_apply(dg_octree* o, int level, int nrhs, const double* u, double* y, void* stream) {
    return dg::guarded([&] {
        if (!o || nrhs < 0) throw std::invalid_argument("bad arguments");
        if (nrhs == 0) return;
        if (!u || !y) throw std::invalid_argument("null argument");
        (void)hipSetDevice(o->device);
        dg::oct::apply(o, level, nrhs, u, y, (hipStream_t)stream);
    });
}

dg_status dg_octree_apply_f32(dg_octree* o, int level, int nrhs, const float* u, float* y, void* stream) {
    return dg::guarded([&] {
        if (!o || nrhs < 0) throw std::invalid_argument("bad arguments");
        if (nrhs == 0) return;
        if (!u || !y) throw std::invalid_argument("null argument");
        (void)hipSetDevice(o->device);
        dg::oct::apply_f32(o, level, nrhs, u, y, (hipStream_t)stream);
    });
}

dg_status dg_octree_vcycle(dg_octree* o, int nrhs, const double* r, double* z, void* stream) {
    return dg::guarded([&] {
        if (!o || nrhs < 0) throw std::invalid_argument("bad arguments");
        if (nrhs == 0) return;
        if (!r || !z) throw std::invalid_argument("null argument");
        (void)hipSetDevice(o->device);
        dg::oct::vcycle_once(o, nrhs, r, z, (hipStream_t)stream);
    });
}

dg_status dg_octree_solve(dg_octree* o, int nrhs, const double* b, double* x, dg_rhs_stats* stats, void* stream) {
    int worst = DG_OK;
    const dg_status st = dg::guarded([&] {
        if (!o || nrhs < 0) throw std::invalid_argument("bad arguments");
        if (nrhs == 0) return;
        if (!b || !x) throw std::invalid_argument("null argument");
        (void)hipSetDevice(o->device);
        worst = dg::oct::solve(o, nrhs, b, x, stats, (hipStream_t)stream);
    });
    return st != DG_OK ? st : (dg_status)worst;
}

dg_status dg_octree_set_rhs_per_block(dg_octree* o, int rhs_per_block) {
    return dg::guarded([&] {
        if (!o || (rhs_per_block != 0 && rhs_per_block != 1 && rhs_per_block != 2 && rhs_per_block != 4))
            throw std::invalid_argument("rhs_per_block must be 0, 1, 2 or 4");
        o->rhs_per_block = rhs_per_block;
    });
}

dg_status dg_octree_exchange(dg_octree* o, int norb, const double* phi, const double* g_pairs, double* v_pairs,
                             double* W, double* K, double* e_x, dg_rhs_stats* stats, void* stream) {
    int worst = DG_OK;
    const dg_status st = dg::guarded([&] {
        if (!o || norb < 1 || norb > 64 || !phi) throw std::invalid_argument("bad arguments");
        (void)hipSetDevice(o->device);
        worst = dg::oct::exchange(o, norb, phi, g_pairs, v_pairs, W, K, e_x, stats, (hipStream_t)stream);
    });
    return st != DG_OK ? st : (dg_status)worst;
}

void dg_octree_destroy(dg_octree* o) { dg::oct::destroy(o); }

}  // extern "C"
