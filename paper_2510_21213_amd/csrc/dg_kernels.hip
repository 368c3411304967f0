// HIP kernels of the DG Poisson library for gfx950 (CDNA4, wave64).
//
// Operator.  On a uniform hexahedral mesh the SIPDG matrix of eq.
// (sip_bilinear) with GLL collocation is the Kronecker sum
//     A = A1x (x) My (x) Mz + Mx (x) A1y (x) Mz + Mx (x) My (x) A1z
// (the penalty acts along the face normal only).  Each 1D matrix A1 is
// block-tridiagonal: an element's diagonal block B_t (local stiffness plus
// the own-element parts of the face terms; t marks boundary elements, which
// carry the Nitsche terms) and a rank-2 coupling to each neighbour that needs
// only the neighbour's face value and face normal derivative.  For the right
// neighbour (value u0 and derivative d0 at its left end)
//     y_e += e_R (-d0/2 - sigma u0) + d_R (u0/2),
// and for the left neighbour (value up and derivative dp at its right end)
//     y_e += e_L ( dp/2 - sigma up) - d_L (up/2).
//
// Tiling.  The operator kernels of degrees 1, 2 and 4 (every level of the benchmark
// hierarchies) are slab kernels (k_slab): a work-group owns a TX x TY tile of elements in the
// x-y plane of one right-hand side and marches along z through a chunk of element layers; per
// layer it stages the tile and its ring of x/y neighbour elements in LDS, computes the x and y
// terms of element pairs in two thread halves at once and the z term of each node column in
// registers (the previous and next layers supply the z neighbours, so no z halo is read), and
// applies the step's epilogue (Chebyshev update, residual, search direction, restriction).  The
// other degrees (3, 5, 6, 7) use the earlier brick kernel (k_brick): a BE^3-element brick staged
// in LDS, neighbour lines outside it read from global memory.  Work-group indices are remapped
// so that each XCD receives a contiguous range of tiles.
//
// Reductions are deterministic: every work-group writes one partial sum to a
// fixed slot and a second kernel adds the slots in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <mutex>
#include <stdexcept>
#include <type_traits>

#include "dg_kernels.h"

namespace dg {

// ---------------------------------------------------------------------------
// helpers

// Work-group w of G is dispatched to XCD w % 8; give XCD x the contiguous
// logical range [start_x, start_x + count_x).
__device__ __forceinline__ int xcd_remap(int w, int G) {
    constexpr int NX = 8;
    if (G < NX) return w;
    const int x = w % NX, slot = w / NX;
    const int base = G / NX, rem = G % NX;
    return x * base + min(x, rem) + slot;
}

__device__ __forceinline__ int etype(int e, int E) { return (e == 0 ? 1 : 0) | (e == E - 1 ? 2 : 0); }

template <int WG>
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < WG / 64; ++i) s += red[i];
    }
    return s;  // valid in thread 0
}

constexpr int wg_of(int nt) { return ((nt + 63) / 64) * 64; }
// element layers per z chunk of the slab kernel, at most (its z loop is unrolled over them)
constexpr int slab_zmax(int n) { return n == 2 ? 2 : 4; }

template <int N>
constexpr int be_of() { return N <= 3 ? 4 : (N <= 6 ? 2 : 1); }

// One axis of the operator over a brick row of NB = BE*N values (elements
// e0 .. e0+BE-1).  hl*: face value / derivative of element e0-1 at its right
// end; hr*: of element e0+BE at its left end (only read when they exist).
// Face values are the end nodes on Gauss-Lobatto axes; on Gauss-Legendre axes
// (A.gl) they are the traces eR . line and eL . line, and the jump terms reach
// every node of the line through eL and eR.
template <typename T, int N, int BE>
__device__ __forceinline__ void axis_row(const AxisDev<T>& A, int e0, int E, const T* row, T hlu, T hld, T hru,
                                         T hrd, T* out) {
    const T sg = A.sigma;
    const T half = (T)0.5;
#pragma unroll
    for (int b = 0; b < BE; ++b) {
        const int e = e0 + b;
        if (e < E) {
            const int t = etype(e, E);
            T acc[N];
#pragma unroll
            for (int i = 0; i < N; ++i) {
                T s = 0;
#pragma unroll
                for (int l = 0; l < N; ++l) s += A.B[t][i][l] * row[b * N + l];
                acc[i] = s;
            }
            if (e > 0) {
                T up, dp;
                if (b > 0) {
                    dp = 0;
#pragma unroll
                    for (int l = 0; l < N; ++l) dp += A.dR[l] * row[(b - 1) * N + l];
                    if (A.gl) {
                        up = 0;
#pragma unroll
                        for (int l = 0; l < N; ++l) up += A.eR[l] * row[(b - 1) * N + l];
                    } else {
                        up = row[b * N - 1];
                    }
                } else {
                    up = hlu;
                    dp = hld;
                }
                if (A.gl) {
                    const T c = half * dp - sg * up;
#pragma unroll
                    for (int i = 0; i < N; ++i) acc[i] += A.eL[i] * c - half * A.dL[i] * up;
                } else {
                    acc[0] += half * dp - sg * up;
#pragma unroll
                    for (int i = 0; i < N; ++i) acc[i] -= half * A.dL[i] * up;
                }
            }
            if (e < E - 1) {
                T u0, d0;
                if (b < BE - 1) {
                    d0 = 0;
#pragma unroll
                    for (int l = 0; l < N; ++l) d0 += A.dL[l] * row[(b + 1) * N + l];
                    if (A.gl) {
                        u0 = 0;
#pragma unroll
                        for (int l = 0; l < N; ++l) u0 += A.eL[l] * row[(b + 1) * N + l];
                    } else {
                        u0 = row[(b + 1) * N];
                    }
                } else {
                    u0 = hru;
                    d0 = hrd;
                }
                if (A.gl) {
                    const T c = -half * d0 - sg * u0;
#pragma unroll
                    for (int i = 0; i < N; ++i) acc[i] += A.eR[i] * c + half * A.dR[i] * u0;
                } else {
                    acc[N - 1] += -half * d0 - sg * u0;
#pragma unroll
                    for (int i = 0; i < N; ++i) acc[i] += half * A.dR[i] * u0;
                }
            }
#pragma unroll
            for (int i = 0; i < N; ++i) out[b * N + i] = acc[i];
        } else {
#pragma unroll
            for (int i = 0; i < N; ++i) out[b * N + i] = 0;
        }
    }
}

// Element access through a uniform base pointer and a 32-bit element index
// (one right-hand side holds far fewer than 2^29 values), so that loads use
// the scalar-base + 32-bit-offset addressing form.
template <typename T>
__device__ __forceinline__ T ld32(const T* base, uint32_t idx) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + idx * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void st32(T* base, uint32_t idx, T v) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + idx * (uint32_t)sizeof(T)) = v;
}

// 1/x: hardware reciprocal, refined by Newton steps to full precision in FP64.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}

template <typename T>
struct BrickArgs {
    const LevelDev<T>* L;
    int E0, E1, E2;
    int nb0, nb1, nb2;
    int nrhs;
    long long ndof;
    const RhsState* st;  // per right-hand side (active flag, beta); may be null
    const T* u;
    const T* u2;
    const T* f;
    const T* zprev;
    T* out;
    T* out2;
    double* partial;
    int pstride;
    T cp, cr;
};

// Reads one input value (BM_PQ combines u + beta u2).
template <typename T, int MODE>
__device__ __forceinline__ T ldin(const T* u, const T* u2, uint32_t idx, T beta) {
    if constexpr (MODE == BM_PQ)
        return ld32(u, idx) + beta * ld32(u2, idx);
    else
        return ld32(u, idx);
}

// Inputs of the operator over one brick, held in registers: the thread's
// own column along Z (thread (X, Y)), and the neighbour lines of the three
// rows the thread owns in the face halo: its X row (thread (Yr, Zr)), its Y
// row (thread (Xr, Zr)) and its Z column.  All of them are loaded before the
// first barrier so that a work-group pays one round of memory latency.
template <typename T, int N, int BE>
struct BrickIn {
    static constexpr int NB = N * BE;
    T ucol[NB];
    T hxl[N], hxr[N], hyl[N], hyr[N], hzl[N], hzr[N];
};

// Element indices are clamped into the mesh so that every load is in bounds
// and needs no branch: values loaded for a row, column or halo line outside
// the mesh are never read by the operator (axis_row only touches elements
// below E and neighbours that exist), so they need no masking.
template <typename T, int N, int BE, int MODE>
__device__ __forceinline__ void brick_load(int E0, int E1, int E2, int ex0, int ey0, int ez0, const T* u,
                                           const T* u2, T beta, BrickIn<T, N, BE>& in) {
    constexpr int NB = N * BE, N2 = N * N, N3 = N * N * N;
    const int t = threadIdx.x;
    auto eoff = [&](int ex, int ey, int ez) -> uint32_t {
        ex = min(ex, E0 - 1);
        ey = min(ey, E1 - 1);
        ez = min(ez, E2 - 1);
        return (uint32_t)((ez * E1 + ey) * E0 + ex) * N3;
    };
    const int a0 = (t % NB), a1 = min(t / NB, NB - 1);  // (X, Y) column, (Y, Z) X row, (X, Z) Y row
    // own column and its Z halo: thread (X, Y) = (a0, a1)
    {
        const int ex = ex0 + a0 / N, i = a0 % N, ey = ey0 + a1 / N, j = a1 % N;
        const uint32_t loc = j * N + i;
#pragma unroll
        for (int b = 0; b < BE; ++b) {
            const uint32_t o = eoff(ex, ey, ez0 + b) + loc;
#pragma unroll
            for (int k = 0; k < N; ++k) in.ucol[b * N + k] = ldin<T, MODE>(u, u2, o + k * N2, beta);
        }
        const uint32_t ol = eoff(ex, ey, max(ez0 - 1, 0)) + loc, orr = eoff(ex, ey, ez0 + BE) + loc;
#pragma unroll
        for (int l = 0; l < N; ++l) {
            in.hzl[l] = ldin<T, MODE>(u, u2, ol + l * N2, beta);
            in.hzr[l] = ldin<T, MODE>(u, u2, orr + l * N2, beta);
        }
    }
    // X row (Yr, Zr) = (a0, a1): neighbour lines along x
    {
        const int ey = ey0 + a0 / N, j = a0 % N, ez = ez0 + a1 / N, k = a1 % N;
        const uint32_t loc = (k * N + j) * N;
        const uint32_t ol = eoff(max(ex0 - 1, 0), ey, ez) + loc, orr = eoff(ex0 + BE, ey, ez) + loc;
#pragma unroll
        for (int l = 0; l < N; ++l) {
            in.hxl[l] = ldin<T, MODE>(u, u2, ol + l, beta);
            in.hxr[l] = ldin<T, MODE>(u, u2, orr + l, beta);
        }
    }
    // Y row (Xr, Zr) = (a0, a1): neighbour lines along y
    {
        const int ex = ex0 + a0 / N, i = a0 % N, ez = ez0 + a1 / N, k = a1 % N;
        const uint32_t loc = k * N2 + i;
        const uint32_t ol = eoff(ex, max(ey0 - 1, 0), ez) + loc, orr = eoff(ex, ey0 + BE, ez) + loc;
#pragma unroll
        for (int l = 0; l < N; ++l) {
            in.hyl[l] = ldin<T, MODE>(u, u2, ol + l * N, beta);
            in.hyr[l] = ldin<T, MODE>(u, u2, orr + l * N, beta);
        }
    }
}

// Face value and normal derivative of the neighbour lines.
template <typename T, int N>
__device__ __forceinline__ void halo_reduce(const AxisDev<T>& A, const T* hl, const T* hr, T& hlu, T& hld, T& hru,
                                            T& hrd) {
    hld = 0;
    hrd = 0;
#pragma unroll
    for (int l = 0; l < N; ++l) {
        hld += A.dR[l] * hl[l];
        hrd += A.dL[l] * hr[l];
    }
    if (A.gl) {
        hlu = 0;
        hru = 0;
#pragma unroll
        for (int l = 0; l < N; ++l) {
            hlu += A.eR[l] * hl[l];
            hru += A.eL[l] * hr[l];
        }
    } else {
        hlu = hl[N - 1];
        hru = hr[0];
    }
}

// Computes y = A u over the brick from the loaded inputs.  On return, for
// column threads with a valid column, ycol[Z] holds (A u) along the column.
// The x and y terms accumulate in one LDS array (sx): the y phase adds to
// what the x phase wrote, after a barrier; each y row touches only its own
// entries, so the read-modify-write needs no atomics.
template <typename T, int N, int BE>
__device__ __forceinline__ void brick_compute(int E0, int E1, int E2, const LevelDev<T>& L, int ex0, int ey0,
                                              int ez0, const BrickIn<T, N, BE>& in, T* su, T* sx, T* ycol) {
    constexpr int NB = N * BE, NT = NB * NB, SY = NB + 1, SZ = NB * SY;
    const int t = threadIdx.x;
    const int a0 = t % NB, a1 = t / NB;
    if (t < NT) {
#pragma unroll
        for (int Z = 0; Z < NB; ++Z) su[Z * SZ + a1 * SY + a0] = in.ucol[Z];
    }
    __syncthreads();
    if (t < NT) {
        {  // x axis: thread (Yr, Zr) = (a0, a1)
            const int ey = ey0 + a0 / N, j = a0 % N, ez = ez0 + a1 / N, k = a1 % N;
            if (ey < E1 && ez < E2) {
                T row[NB], out[NB];
#pragma unroll
                for (int x = 0; x < NB; ++x) row[x] = su[a1 * SZ + a0 * SY + x];
                T hlu, hld, hru, hrd;
                halo_reduce<T, N>(L.ax[0], in.hxl, in.hxr, hlu, hld, hru, hrd);
                axis_row<T, N, BE>(L.ax[0], ex0, E0, row, hlu, hld, hru, hrd, out);
                const T sc = L.ax[1].m[j] * L.ax[2].m[k];
#pragma unroll
                for (int x = 0; x < NB; ++x) sx[a1 * SZ + a0 * SY + x] = out[x] * sc;
            }
        }
    }
    __syncthreads();
    if (t < NT) {
        {  // y axis: thread (Xr, Zr) = (a0, a1)
            const int ex = ex0 + a0 / N, i = a0 % N, ez = ez0 + a1 / N, k = a1 % N;
            if (ex < E0 && ez < E2) {
                T row[NB], out[NB];
#pragma unroll
                for (int y = 0; y < NB; ++y) row[y] = su[a1 * SZ + y * SY + a0];
                T hlu, hld, hru, hrd;
                halo_reduce<T, N>(L.ax[1], in.hyl, in.hyr, hlu, hld, hru, hrd);
                axis_row<T, N, BE>(L.ax[1], ey0, E1, row, hlu, hld, hru, hrd, out);
                const T sc = L.ax[0].m[i] * L.ax[2].m[k];
#pragma unroll
                for (int y = 0; y < NB; ++y) sx[a1 * SZ + y * SY + a0] += out[y] * sc;
            }
        }
    }
    __syncthreads();
    {  // z axis in registers: thread (X, Y) = (a0, a1)
        const int ex = ex0 + a0 / N, i = a0 % N, ey = ey0 + a1 / N, j = a1 % N;
        if (t < NT && ex < E0 && ey < E1) {
            T hlu, hld, hru, hrd, out[NB];
            halo_reduce<T, N>(L.ax[2], in.hzl, in.hzr, hlu, hld, hru, hrd);
            axis_row<T, N, BE>(L.ax[2], ez0, E2, in.ucol, hlu, hld, hru, hrd, out);
            const T sc = L.ax[0].m[i] * L.ax[1].m[j];
#pragma unroll
            for (int Z = 0; Z < NB; ++Z) ycol[Z] = out[Z] * sc + sx[Z * SZ + a1 * SY + a0];
        }
    }
}

template <typename T, int N, int BE, int MODE>
__global__ __launch_bounds__(wg_of(N* BE* N* BE), 2) void k_brick(BrickArgs<T> a) {
    constexpr int NB = N * BE, NT = NB * NB, SY = NB + 1, SZ = NB * SY, N3 = N * N * N;
    constexpr int WG = wg_of(NT);
    constexpr bool HAS_F = MODE == BM_RESID || MODE == BM_RESIDDOT || MODE == BM_CHEB || MODE == BM_CHEBDOT;
    constexpr bool IS_CHEB = MODE == BM_CHEB || MODE == BM_CHEBDOT;
    __shared__ T su[NB * SZ];
    __shared__ T sx[NB * SZ];
    __shared__ double red[WG / 64];

    const int nbr = a.nb0 * a.nb1 * a.nb2;
    const int w = xcd_remap(blockIdx.x, nbr * a.nrhs);
    const int rhs = w / nbr, br = w % nbr;
    if (a.st && !a.st[rhs].active) return;
    const int bx = br % a.nb0, by = (br / a.nb0) % a.nb1, bz = br / (a.nb0 * a.nb1);
    const int ex0 = bx * BE, ey0 = by * BE, ez0 = bz * BE;
    const int E0 = a.E0, E1 = a.E1, E2 = a.E2;
    const LevelDev<T>& L = *a.L;
    const long long base = (long long)rhs * a.ndof;
    const T* u = a.u + base;
    const T* u2 = (MODE == BM_PQ) ? a.u2 + base : nullptr;
    const T* fb = HAS_F ? a.f + base : nullptr;
    const T* zpb = (IS_CHEB && a.zprev) ? a.zprev + base : nullptr;
    T* ob = a.out + base;
    T* ob2 = (MODE == BM_PQ) ? a.out2 + base : nullptr;
    T beta = 0;
    if constexpr (MODE == BM_PQ) beta = (T)a.st[rhs].beta;

    const int t = threadIdx.x;
    const int X = t % NB, Y = t / NB;
    const int exX = ex0 + X / N, iX = X % N, eyY = ey0 + Y / N, jY = Y % N;
    const bool colok = t < NT && exX < E0 && eyY < E1;
    auto gidx = [&](int Z) -> uint32_t {
        return (uint32_t)(((ez0 + Z / N) * E1 + eyY) * E0 + exX) * N3 + ((Z % N) * N + jY) * N + iX;
    };
    // clamped index for loads of the thread's column (in bounds for every lane)
    auto cidx = [&](int Z) -> uint32_t {
        const int ez = min(ez0 + Z / N, E2 - 1), ey = min(eyY, E1 - 1), ex = min(exX, E0 - 1);
        return (uint32_t)((ez * E1 + ey) * E0 + ex) * N3 + ((Z % N) * N + jY) * N + iX;
    };

    BrickIn<T, N, BE> in;
    brick_load<T, N, BE, MODE>(E0, E1, E2, ex0, ey0, ez0, u, u2, beta, in);
    // The column's f and zprev are loaded after the operator: issued before
    // it they would hold registers through the three axis phases.
    T ycol[NB];
    brick_compute<T, N, BE>(E0, E1, E2, L, ex0, ey0, ez0, in, su, sx, ycol);
    T fcol[NB], zpcol[NB];
    if constexpr (HAS_F) {
#pragma unroll
        for (int Z = 0; Z < NB; ++Z) fcol[Z] = ld32(fb, cidx(Z));
    }
    if constexpr (IS_CHEB) {
        if (zpb) {
#pragma unroll
            for (int Z = 0; Z < NB; ++Z) zpcol[Z] = ld32(zpb, cidx(Z));
        } else {
#pragma unroll
            for (int Z = 0; Z < NB; ++Z) zpcol[Z] = (T)0;
        }
    }

    double dot = 0.0;
    if (colok) {
        const int tx = etype(exX, E0), ty = etype(eyY, E1);
        const T mx = L.ax[0].m[iX], my = L.ax[1].m[jY];
        const T dxm = L.ax[0].Bd[tx][iX] * my, mxdy = mx * L.ax[1].Bd[ty][jY], mxy = mx * my;
#pragma unroll
        for (int Z = 0; Z < NB; ++Z) {
            const int ez = ez0 + Z / N, k = Z % N;
            if (ez >= E2) continue;
            const uint32_t idx = gidx(Z);
            const T y = ycol[Z];
            if constexpr (MODE == BM_APPLY) {
                st32(ob, idx, y);
            } else if constexpr (MODE == BM_RESID || MODE == BM_RESIDDOT) {
                const T r = fcol[Z] - y;
                st32(ob, idx, r);
                if constexpr (MODE == BM_RESIDDOT) dot += (double)r * (double)r;
            } else if constexpr (IS_CHEB) {
                const int tz = etype(ez, E2);
                const T mz = L.ax[2].m[k];
                const T D = (dxm + mxdy) * mz + mxy * L.ax[2].Bd[tz][k];
                const T uz = in.ucol[Z];
                const T zn = uz + a.cp * (uz - zpcol[Z]) + a.cr * (fcol[Z] - y) * recip(D);
                st32(ob, idx, zn);
                if constexpr (MODE == BM_CHEBDOT) dot += (double)fcol[Z] * (double)zn;
            } else if constexpr (MODE == BM_PQ) {
                st32(ob2, idx, in.ucol[Z]);
                st32(ob, idx, y);
                dot += (double)in.ucol[Z] * (double)y;
            }
        }
    }
    if constexpr (MODE == BM_CHEBDOT || MODE == BM_PQ || MODE == BM_RESIDDOT) {
        const double s = block_sum<WG>(dot, red);
        if (t == 0) a.partial[(long long)rhs * a.pstride + br] = s;
    }
}

// ---------------------------------------------------------------------------
// Slab operator kernel (levels of degree 1, 2 and 4).
//
// A work-group owns a TX x TY tile of elements in the x-y plane of one
// right-hand side and marches along z through a chunk of element layers.  Per
// layer, the tile and the ring of x and y neighbour elements around it (the
// face halo) are staged in LDS.  Every thread keeps one node column of the
// layer in registers and computes its z term, with the previous and next
// layers as neighbours (already in registers, so no z halo is read).  Half of
// the threads compute the x terms of pairs of elements along x rows and the
// other half the y terms of pairs along y rows, at the same time, into two LDS
// arrays; each thread then adds the three terms of its column.  The loads of
// the next layers are issued before the current layer is computed.  Every
// element uses the interior block in reference units (RefDev); on a domain
// face the Nitsche terms follow from ghost face data (elem_op).

template <typename T>
struct SlabArgs {
    const LevelDev<T>* L;
    int E0, E1, E2;
    int nt0, nt1;   // tiles along x and y
    int zlen, nzc;  // element layers per chunk, chunks along z
    int nrhs;
    long long ndof;
    const RhsState* st;
    const T* u;
    const void* uf;   // BM_PQ32: the FP32 (or BF16) field that takes the place of u
    const T* u2;
    const T* f;
    const T* zprev;
    T* out;
    T* out2;
    double* partial;
    int pstride;
    T cp, cr;
    // BM_RESTRICT: coarse level (same elements, degree p/2) and its outputs
    const LevelDev<T>* Lc;
    const TransferDev* tr;
    T* fc;
    T* z1c;
    long long ndofc;
    T c0c;
    const T* dinvc;  // BM_RESTRICT: inverse diagonal of the coarse level (its first smoothing iterate)
};

// Coefficients of the interior block in the even/odd form of RefDev (symmetric
// and invariant under the reflection of the reference element; aR_l = -aL_{p-l}):
// 17 scalars for p = 4, held in scalar registers for the whole work-group.
template <typename T, int N>
struct SlabCoef {
    static constexpr int H = N / 2;
    T Pe[H][H], Po[H][H];
    T Bm[H + 1];
    T qe[H], qo[H], qm;
    T aL[N];
    T sig;
};

template <typename T, int N>
__device__ __forceinline__ void load_coef(SlabCoef<T, N>& c, const RefDev<T>& R) {
    constexpr int H = N / 2;
#pragma unroll
    for (int i = 0; i < H; ++i) {
#pragma unroll
        for (int l = 0; l < H; ++l) {
            c.Pe[i][l] = R.Pe[i][l];
            c.Po[i][l] = R.Po[i][l];
        }
        c.qe[i] = R.qe[i];
        c.qo[i] = R.qo[i];
    }
#pragma unroll
    for (int i = 0; i <= H; ++i) c.Bm[i] = (N & 1) ? R.Bm[i] : (T)0;
    c.qm = (N & 1) ? R.qm : (T)0;
#pragma unroll
    for (int i = 0; i < N; ++i) c.aL[i] = R.aL[i];
    c.sig = R.sig;
}

template <typename T, int N>
__device__ __forceinline__ T face_l(const SlabCoef<T, N>& c, const T* v) {
    T s = 0;
#pragma unroll
    for (int l = 0; l < N; ++l) s += c.aL[l] * v[l];
    return s;
}
template <typename T, int N>
__device__ __forceinline__ T face_r(const SlabCoef<T, N>& c, const T* v) {
    T s = 0;
#pragma unroll
    for (int l = 0; l < N; ++l) s -= c.aL[N - 1 - l] * v[l];
    return s;
}

// One element along one axis, reference units: acc = B A plus the coupling to
// the left neighbour (U its value at its right end, Dv = aR . its line) and to
// the right neighbour (U0 its value at its left end, D0 = aL . its line):
//   acc_i += (aR_i U0 - aL_i U) / 2,  acc_0 += Dv/2 - sig U,  acc_p -= D0/2 + sig U0.
// With the ghost data U = -A_0, Dv = aL.A - 2 sig A_0 on a left domain face and
// U0 = -A_p, D0 = aR.A + 2 sig A_p on a right one, the same formula gives the
// block of a boundary element (its Nitsche face terms).
//
// B is invariant under the reflection of the reference element and aR_i =
// -aL_{p-i}, so the rows i and p-i are computed together from the even and odd
// parts of A (ue = A_l + A_{p-l}, uo = A_l - A_{p-l}) and of the coupling
// (S = U0 + U, D = U0 - U): acc_i, acc_{p-i} = ev_i +- od_i (32 operations per
// element at p = 4 instead of 41).
template <typename T, int N>
__device__ __forceinline__ void elem_op(const SlabCoef<T, N>& c, const T* A, T U, T Dv, T U0, T D0, T* acc) {
    constexpr int H = N / 2;
    constexpr bool ODD = (N & 1) != 0;
    const T S = U0 + U, D = U0 - U;
    T ue[H + 1], uo[H];
#pragma unroll
    for (int l = 0; l < H; ++l) {
        ue[l] = A[l] + A[N - 1 - l];
        uo[l] = A[l] - A[N - 1 - l];
    }
    if constexpr (ODD) ue[H] = A[H];
#pragma unroll
    for (int i = 0; i < H; ++i) {
        T ev = c.qe[i] * S, od = c.qo[i] * D;
#pragma unroll
        for (int l = 0; l < H; ++l) {
            ev += c.Pe[i][l] * ue[l];
            od += c.Po[i][l] * uo[l];
        }
        if constexpr (ODD) ev += c.Bm[i] * ue[H];
        acc[i] = ev + od;
        acc[N - 1 - i] = ev - od;
    }
    if constexpr (ODD) {
        T m = c.qm * S;
#pragma unroll
        for (int l = 0; l <= H; ++l) m += c.Bm[l] * ue[l];
        acc[H] = m;
    }
    acc[0] += (T)0.5 * Dv - c.sig * U;
    acc[N - 1] -= (T)0.5 * D0 + c.sig * U0;
}

// x or y term of the element pair (e, e+1) of a row staged in LDS at su[pb +
// s PSTR]: s in [0, N) the left neighbour line, [N, 3N) the pair, [3N, 4N) the
// right neighbour line.  nE elements along the axis; neighbours that do not
// exist are replaced by ghost data and their lines are not used.  The
// results, times sc, go to so[ob + s OSTR], s in [0, 2N) (the second element
// only if it exists).
template <typename T, int N, int PSTR, int OSTR>
__device__ __forceinline__ void pair_row(const SlabCoef<T, N>& c, const T* su, int pb, T* so, int ob, int e, int nE,
                                         T sc) {
    T A[N], B[N], out[N];
#pragma unroll
    for (int l = 0; l < N; ++l) {
        A[l] = su[pb + (N + l) * PSTR];
        B[l] = su[pb + (2 * N + l) * PSTR];
    }
    const bool has2 = e + 1 < nE;
    const T fRA = face_r(c, A);
    T U, Dv, U0, D0;
    if (e > 0) {
        T nl[N];
#pragma unroll
        for (int l = 0; l < N; ++l) nl[l] = su[pb + l * PSTR];
        U = nl[N - 1];
        Dv = face_r(c, nl);
    } else {
        U = -A[0];
        Dv = face_l(c, A) - (T)2 * c.sig * A[0];
    }
    if (has2) {
        U0 = B[0];
        D0 = face_l(c, B);
    } else {
        U0 = -A[N - 1];
        D0 = fRA + (T)2 * c.sig * A[N - 1];
    }
    elem_op(c, A, U, Dv, U0, D0, out);
#pragma unroll
    for (int i = 0; i < N; ++i) so[ob + i * OSTR] = out[i] * sc;
    if (has2) {
        if (e + 2 < nE) {
            T nr[N];
#pragma unroll
            for (int l = 0; l < N; ++l) nr[l] = su[pb + (3 * N + l) * PSTR];
            U0 = nr[0];
            D0 = face_l(c, nr);
        } else {
            U0 = -B[N - 1];
            D0 = face_r(c, B) + (T)2 * c.sig * B[N - 1];
        }
        elem_op(c, B, A[N - 1], fRA, U0, D0, out);
#pragma unroll
        for (int i = 0; i < N; ++i) so[ob + (N + i) * OSTR] = out[i] * sc;
    }
}

typedef __amdgpu_buffer_rsrc_t brsrc;

// Raw buffer access (byte offsets; voff per lane, soff uniform).  Loads outside
// the buffer's size return 0 and such stores are dropped, so an indexing slip
// cannot reach other memory.
template <typename T>
__device__ __forceinline__ brsrc rsrc_of(const T* p, long long n) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)(n * (long long)sizeof(T)), 0x00020000);
}
__device__ __forceinline__ void bload(float& v, brsrc r, uint32_t voff, uint32_t soff) {
    v = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ void bload(double& v, brsrc r, uint32_t voff, uint32_t soff) {
    v = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void bstore(float v, brsrc r, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, 0);
}
__device__ __forceinline__ void bstore(double v, brsrc r, uint32_t voff, uint32_t soff) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
}
// Field element of storage type S as the compute type T: fields of the compute type as they are;
// BF16 fields widened on load (exact) and rounded to nearest even on store; FP32 fields of an FP64
// computation widened on load and rounded to nearest on store.
template <typename S, typename T>
__device__ __forceinline__ void fload(T& v, brsrc r, uint32_t voff, uint32_t soff) {
    if constexpr (std::is_same<S, __bf16>::value) {
        const unsigned short h = __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0);
        v = (T)__uint_as_float((uint32_t)h << 16);
    } else if constexpr (sizeof(S) != sizeof(T)) {
        S w;
        bload(w, r, voff, soff);
        v = (T)w;
    } else {
        bload(v, r, voff, soff);
    }
}
// (The FP32 -> BF16 conversion is the hardware's, v_cvt_pk_bf16_f32 on gfx950: round to nearest even.)
template <typename S, typename T>
__device__ __forceinline__ void fstore(T v, brsrc r, uint32_t voff, uint32_t soff) {
    if constexpr (std::is_same<S, __bf16>::value) {
        const __bf16 h = (__bf16)(float)v;
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, h), r, voff, soff, 0);
    } else if constexpr (sizeof(S) != sizeof(T)) {
        bstore((S)v, r, voff, soff);
    } else {
        bstore(v, r, voff, soff);
    }
}
__device__ __forceinline__ __bf16 to_bf16(float v) { return (__bf16)v; }
__device__ __forceinline__ float from_bf16(__bf16 h) {
    return __uint_as_float((uint32_t)__builtin_bit_cast(unsigned short, h) << 16);
}

// The N values of a node column of one element layer (stride N^2 values), fields of storage type
// S.  BM_PQ and BM_PQ32 read u + beta u2; in BM_PQ32 u is the V-cycle output, a field of type ZP
// (FP32 or BF16), addressed at sizeof(ZP) / sizeof(T) of the byte offsets of T = double, and u2
// the search direction, stored as SP (FP64, or FP32 when the direction is kept in single
// precision: the new direction is then rounded to SP here, before it is used, so that q = A p is
// the product of exactly the direction that is stored).
template <typename T, int N, int MODE, typename S = T, typename ZP = float, typename SP = S>
__device__ __forceinline__ void load_col(T* v, brsrc ru, brsrc ru2, uint32_t voff, uint32_t soff, T beta) {
    if constexpr (MODE == BM_PQ32) {
        static_assert(sizeof(T) == 8 && sizeof(S) == 8, "BM_PQ32 is an FP64 step");
        constexpr uint32_t R = sizeof(T) / sizeof(ZP);
#pragma unroll
        for (int k = 0; k < N; ++k) {
            float zf;
            fload<ZP>(zf, ru, voff / R, soff / R + k * N * N * (uint32_t)sizeof(ZP));
            v[k] = (T)zf;
        }
    } else {
#pragma unroll
        for (int k = 0; k < N; ++k) fload<S>(v[k], ru, voff, soff + k * N * N * (uint32_t)sizeof(S));
    }
    if constexpr (MODE == BM_PQ) {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            T w;
            fload<S>(w, ru2, voff, soff + k * N * N * (uint32_t)sizeof(S));
            v[k] += beta * w;
        }
    } else if constexpr (MODE == BM_PQ32) {
        constexpr uint32_t R2 = sizeof(T) / sizeof(SP);
#pragma unroll
        for (int k = 0; k < N; ++k) {
            T w;
            fload<SP>(w, ru2, voff / R2, soff / R2 + k * N * N * (uint32_t)sizeof(SP));
            v[k] += beta * w;
            if constexpr (sizeof(SP) == 4) v[k] = (T)(float)v[k];
        }
    }
}

// ---- x and y terms on the matrix cores (BF16 operands, FP32 accumulation) ----------------
// For one axis, the element line's N outputs are one matrix-vector product with the 15-vector of
// the line and its two neighbour lines along the axis: acc = [C_L | B | C_R] (left, own, right),
// the reference-element form of elem_op (C_L and C_R carry the face couplings, rank 2 each).
// Sixteen lines make the columns of one v_mfma_f32_16x16x16_bf16 (K = 16 >= 3N = 15); the same
// 16 x 16 matrix (rows >= N and column 15 zero) serves every line of the level and both axes.
// Lines next to a domain face read ghost neighbour lines (mf_ghosts) that reproduce the Nitsche
// terms through the same couplings.
typedef short mf_s4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ short mf_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

// Entry (i, k) of [C_L | B | C_R] in reference units.
template <int N>
__device__ __forceinline__ float mf_coef(const RefDev<float>& R, int i, int k) {
    if (i >= N || k >= 3 * N) return 0.f;
    const int blk = k / N, l = k - blk * N;
    const float aRi = -R.aL[N - 1 - i];
    if (blk == 1) return R.B[i][l];
    if (blk == 0) {  // left neighbour: U = its value at the right end, Dv = aR . its line
        const float aRl = -R.aL[N - 1 - l];
        float v = (l == N - 1) ? -0.5f * R.aL[i] : 0.f;
        if (i == 0) v += 0.5f * aRl - (l == N - 1 ? R.sig : 0.f);
        return v;
    }
    // right neighbour: U0 = its value at the left end, D0 = aL . its line
    float v = (l == 0) ? 0.5f * aRi : 0.f;
    if (i == N - 1) v -= 0.5f * R.aL[l] + (l == 0 ? R.sig : 0.f);
    return v;
}

// Ghost neighbour lines of the element lines next to a domain face, written into the staging
// rows: a line g with g at the far end and one more entry chosen so that the couplings of the
// line see the ghost value U and derivative D of the Nitsche form (elem_op's ghost data).
template <int N, int TX, int TY>
__device__ __forceinline__ void mf_ghosts(const SlabCoef<float, N>& c, float* su, int tx0, int ty0, int E0,
                                          int E1) {
    constexpr int NX = TX * N, NY = TY * N, RS = NX + 2 * N, PS = RS * (NY + 2 * N);
    const int nvx = min(TX, E0 - tx0), nvy = min(TY, E1 - ty0);  // valid elements of the tile per axis
    const bool lx = tx0 == 0, rx = tx0 + TX >= E0, ly = ty0 == 0, ry = ty0 + TY >= E1;
    const int t = threadIdx.x;
    // tasks: x rows (NY * N) and y columns (NX * N), each on its left and right side
    const int nx_tasks = 2 * NY * N, ny_tasks = 2 * NX * N;
    for (int q = t; q < nx_tasks + ny_tasks; q += blockDim.x) {
        int base, stride, first, side, ok;
        if (q < nx_tasks) {
            side = q & 1;
            const int row = q >> 1, Yr = row % NY, kr = row / NY;
            ok = (side ? rx : lx) && (Yr / N) < nvy;
            base = kr * PS + (Yr + N) * RS;
            stride = 1;
            first = side ? N + (nvx - 1) * N : N;  // the boundary element's line
        } else {
            const int q2 = q - nx_tasks;
            side = q2 & 1;
            const int col = q2 >> 1, Xc = col % NX, kr = col / NX;
            ok = (side ? ry : ly) && (Xc / N) < nvx;
            base = kr * PS + Xc + N;
            stride = RS;
            first = side ? N + (nvy - 1) * N : N;
        }
        if (!ok) continue;
        float A[N];
#pragma unroll
        for (int l = 0; l < N; ++l) A[l] = su[base + (first + l) * stride];
        float g[N];
#pragma unroll
        for (int l = 0; l < N; ++l) g[l] = 0.f;
        if (!side) {  // left ghost: U = -A_0, Dv = aL.A - 2 sig A_0; g = (g0, 0, ..., 0, U)
            const float U = -A[0], Dv = face_l(c, A) - 2.f * c.sig * A[0];
            g[N - 1] = U;
            g[0] = -(Dv + c.aL[0] * U) / c.aL[N - 1];
        } else {      // right ghost: U0 = -A_p, D0 = aR.A + 2 sig A_p; g = (U0, 0, ..., 0, gp)
            const float U0 = -A[N - 1], D0 = face_r(c, A) + 2.f * c.sig * A[N - 1];
            g[0] = U0;
            g[N - 1] = (D0 - c.aL[0] * U0) / c.aL[N - 1];
        }
        const int gpos = side ? first + N : first - N;
#pragma unroll
        for (int l = 0; l < N; ++l) su[base + (gpos + l) * stride] = g[l];
    }
}

// x and y terms of the layer staged in su into sxy (same layout as pair_row's output), on the
// matrix cores.  Lines of elements outside the mesh produce values nobody reads.
template <int N, int TX, int TY>
__device__ __forceinline__ void mf_xy_terms(const RefDev<float>& R, const mf_s4& Aop, const float* su, float* sxy) {
    constexpr int NX = TX * N, NY = TY * N, RS = NX + 2 * N, PS = RS * (NY + 2 * N), OR = NX, OP = OR * NY;
    constexpr int NLX = NY * N * TX, NLY = NX * N * TY;       // element lines per axis in the layer
    constexpr int NBX = (NLX + 15) / 16, NBY = (NLY + 15) / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    const int n = lane & 15, kq = (lane >> 4) * 4;           // column of B, first of its 4 K rows
    for (int blk = wave; blk < NBX + NBY; blk += nwaves) {
        const bool xa = blk < NBX;
        const int lam = (xa ? blk : blk - NBX) * 16 + n;    // this lane's line
        const int nlines = xa ? NLX : NLY;
        const bool lv = lam < nlines;
        int base = 0, stride = 1, obase = 0, ostride = 1;
        float sc = 0.f;
        if (lv) {
            if (xa) {  // x line: row (Yr, kr), element e
                const int row = lam / TX, e = lam % TX, Yr = row % NY, kr = row / NY;
                base = kr * PS + (Yr + N) * RS + e * N;
                stride = 1;
                obase = kr * OP + Yr * OR + e * N;
                ostride = 1;
                sc = R.scale[0] * R.w[Yr % N] * R.w[kr];
            } else {   // y line: column (Xc, kr), element e
                const int col = lam / TY, e = lam % TY, Xc = col % NX, kr = col / NX;
                base = kr * PS + e * N * RS + Xc + N;
                stride = RS;
                obase = N * OP + kr * OP + e * N * OR + Xc;
                ostride = OR;
                sc = R.scale[1] * R.w[Xc % N] * R.w[kr];
            }
        }
        mf_s4 b;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = kq + j;
            b[j] = (lv && k < 3 * N) ? mf_bf16(su[base + k * stride]) : (short)0;
        }
        mf_f4 d = {0.f, 0.f, 0.f, 0.f};
        d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(Aop, b, d, 0, 0, 0);
        // d[j] = output node kq + j of line n: lines are this lane's column, so swap the roles:
        // lane (n, kq) holds rows kq..kq+3 of column n
        if (lv) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int i = kq + j;
                if (i < N) sxy[obase + i * ostride] = d[j] * sc;
            }
        }
    }
}

// S: storage type of the fields u, u2, f, zprev, out, out2 (T, or BF16 for FP32 arithmetic; the
// pointers of SlabArgs<T> then address BF16 data); ZP: type of the BM_PQ32 input uf; SP: storage
// type of the BM_PQ32 search direction (u2 in, out2 out); SC: storage type of the BM_RESTRICT
// outputs fc and z1c (the coarse level's source and first smoothing iterate).
template <typename T, int N, int TX, int TY, int MODE, bool MF = false, typename S = T, typename ZP = float,
          typename SP = S, typename SC = T>
__global__ __launch_bounds__(wg_of(TX* TY* N* N)) void k_slab(SlabArgs<T> a) {
    constexpr int NX = TX * N, NY = TY * N, NT = NX * NY, N2 = N * N, N3 = N2 * N;
    constexpr int WG = wg_of(NT);
    constexpr int RS = NX + 2 * N, PS = RS * (NY + 2 * N);  // LDS staging: row and plane strides
    constexpr int OR = NX, OP = OR * NY;                     // LDS x / y terms: row and plane strides
    constexpr int NP = NT / 2;                               // element pairs per axis and layer
    // first thread of the y pairs: the next wave boundary when the work-group still holds all
    // y pairs from there, so that no wave computes both an x and a y pair row
    constexpr int YB = ((NP + 63) / 64) * 64 + NP <= WG ? ((NP + 63) / 64) * 64 : NP;
    constexpr int NH = 2 * (TX + TY);                        // halo elements per layer
    constexpr int HS = (NH + TX * TY - 1) / (TX * TY);       // halo columns per thread
    constexpr uint32_t SZ = sizeof(S);
    static_assert(TX % 2 == 0 && TY % 2 == 0, "tiles hold whole element pairs");
    constexpr bool HAS_F = MODE == BM_RESID || MODE == BM_RESIDDOT || MODE == BM_CHEB || MODE == BM_CHEBDOT ||
                           MODE == BM_RESTRICT;
    constexpr bool IS_CHEB = MODE == BM_CHEB || MODE == BM_CHEBDOT;
    constexpr bool IS_PQ = MODE == BM_PQ || MODE == BM_PQ32;
    constexpr bool DOT = MODE == BM_CHEBDOT || IS_PQ || MODE == BM_RESIDDOT;
    constexpr int NC = (N - 1) / 2 + 1, NC3 = NC * NC * NC;  // BM_RESTRICT: coarse nodes per edge (degree p/2)
    __shared__ T su[N * PS];
    __shared__ T sr[MODE == BM_RESTRICT ? NC * OP : 1];  // BM_RESTRICT: residual contracted along z
    __shared__ T sxy[2 * N * OP];
    __shared__ double red[WG / 64];

    const int per_rhs = a.nt0 * a.nt1 * a.nzc;
    const int w = xcd_remap(blockIdx.x, per_rhs * a.nrhs);
    const int rhs = w / per_rhs, slot = w % per_rhs;
    if (a.st && !a.st[rhs].active) return;
    const int chunk = slot / (a.nt0 * a.nt1), tile = slot % (a.nt0 * a.nt1);
    const int tx0 = (tile % a.nt0) * TX, ty0 = (tile / a.nt0) * TY;
    const int E0 = a.E0, E1 = a.E1, E2 = a.E2;
    const int ezb = chunk * a.zlen, eze = min(E2, ezb + a.zlen);
    const uint32_t lstride = (uint32_t)(E0 * E1 * N3) * SZ;  // bytes per element layer

    const long long base = (long long)rhs * a.ndof;
    const S* const uS = reinterpret_cast<const S*>(a.u);
    brsrc ru;
    if constexpr (MODE == BM_PQ32)
        ru = rsrc_of(reinterpret_cast<const ZP*>(a.uf) + base, a.ndof);
    else
        ru = rsrc_of(uS + base, a.ndof);
    brsrc ru2;
    if constexpr (MODE == BM_PQ32)
        ru2 = rsrc_of(reinterpret_cast<const SP*>(a.u2) + base, a.ndof);
    else
        ru2 = rsrc_of(IS_PQ ? reinterpret_cast<const S*>(a.u2) + base : uS + base, a.ndof);
    const brsrc rf = rsrc_of(HAS_F ? reinterpret_cast<const S*>(a.f) + base : uS + base, a.ndof);
    const brsrc rzp = rsrc_of(IS_CHEB && a.zprev ? reinterpret_cast<const S*>(a.zprev) + base : uS + base, a.ndof);
    // BM_RESTRICT stores no fine field
    S* const obase = MODE == BM_RESTRICT ? const_cast<S*>(uS) : reinterpret_cast<S*>(a.out);
    const brsrc ro = rsrc_of(obase + base, a.ndof);
    brsrc ro2;
    if constexpr (MODE == BM_PQ32)
        ro2 = rsrc_of(reinterpret_cast<SP*>(a.out2) + base, a.ndof);
    else
        ro2 = rsrc_of(IS_PQ ? reinterpret_cast<S*>(a.out2) + base : obase + base, a.ndof);
    T beta = 0;
    if constexpr (IS_PQ) beta = (T)a.st[rhs].beta;
    const bool has_zp = IS_CHEB && a.zprev;

    const RefDev<T>& R = a.L->ref;
    SlabCoef<T, N> c;
    load_coef(c, R);
    mf_s4 mfA = {0, 0, 0, 0};
    if constexpr (MF) {
        static_assert(sizeof(T) == 4 && 3 * N <= 16, "matrix-core x/y terms: FP32 fields, at most 5 nodes per edge");
        const int lane = threadIdx.x & 63;
#pragma unroll
        for (int j = 0; j < 4; ++j) mfA[j] = mf_bf16(mf_coef<N>(R, lane & 15, (lane >> 4) * 4 + j));
    }

    const int t = threadIdx.x;
    const bool tact = t < NT;
    // column role: thread -> (element el of the tile, node (i, j) of its face)
    const int tc = min(t, NT - 1);
    const int el = tc / N2, i = tc % N, j = (tc / N) % N;
    const int exl = el % TX, eyl = el / TX;
    const int X = exl * N + i, Y = eyl * N + j;
    const int ex = tx0 + exl, ey = ty0 + eyl;
    const bool colok = tact && ex < E0 && ey < E1;
    const uint32_t coff = ((uint32_t)((min(ey, E1 - 1) * E0 + min(ex, E0 - 1)) * N3 + j * N + i)) * SZ;
    const int su_own = (Y + N) * RS + X + N;
    const int so_own = Y * OR + X;
    const T wi = R.w[i], wj = R.w[j];
    const T P2 = R.scale[2] * wi * wj;  // z-term scale, and the z part of the diagonal per reference entry
    T P1 = 0;                           // x and y parts of the diagonal (times w_k)
    if constexpr (IS_CHEB) {
        T bdx = R.B[i][i], bdy = R.B[j][j];
        if (ex == 0 && i == 0) bdx += R.aL[0];
        if (ex == E0 - 1 && i == N - 1) bdx -= R.aR[N - 1];
        if (ey == 0 && j == 0) bdy += R.aL[0];
        if (ey == E1 - 1 && j == N - 1) bdy -= R.aR[N - 1];
        P1 = R.scale[0] * bdx * wj + R.scale[1] * wi * bdy;
    }
    // halo role: the same node (i, j) of halo element he = el + s TX TY
    uint32_t hoff[HS];
    int hsu[HS];
    bool hok[HS];
#pragma unroll
    for (int s = 0; s < HS; ++s) {
        const int he = el + s * TX * TY;
        hok[s] = tact && he < NH;
        const int hq = min(he, NH - 1);
        int hx, hy, Xe, Ye;
        if (hq < 2 * TY) {  // x sides
            const int q = hq % TY, side = hq / TY;
            hx = side ? tx0 + TX : tx0 - 1;
            hy = ty0 + q;
            Xe = side ? NX + N + i : i;
            Ye = q * N + j + N;
        } else {  // y sides
            const int q = (hq - 2 * TY) % TX, side = (hq - 2 * TY) / TX;
            hx = tx0 + q;
            hy = side ? ty0 + TY : ty0 - 1;
            Xe = q * N + i + N;
            Ye = side ? NY + N + j : j;
        }
        hx = max(0, min(hx, E0 - 1));
        hy = max(0, min(hy, E1 - 1));
        hoff[s] = ((uint32_t)((hy * E0 + hx) * N3 + j * N + i)) * SZ;
        hsu[s] = Ye * RS + Xe;
    }
    // pair role: x pairs for t < NP, y pairs for YB <= t < YB + NP
    const bool isx = t < NP, isy = t >= YB && t < YB + NP;
    int pb, ob, pe;
    bool pok;
    T psc;
    if (isx) {
        const int pa = t % (TX / 2), row = t / (TX / 2), Yr = row % NY, kr = row / NY;
        pe = tx0 + 2 * pa;
        pok = pe < E0 && ty0 + Yr / N < E1;
        pb = kr * PS + (Yr + N) * RS + 2 * pa * N;
        ob = kr * OP + Yr * OR + 2 * pa * N;
        psc = R.scale[0] * R.w[Yr % N] * R.w[kr];
    } else {
        const int q = min(max(t - YB, 0), NP - 1), pa = q % (TY / 2), col = q / (TY / 2), Xc = col % NX, kr = col / NX;
        pe = ty0 + 2 * pa;
        pok = isy && pe < E1 && tx0 + Xc / N < E0;
        pb = kr * PS + 2 * pa * N * RS + Xc + N;
        ob = N * OP + kr * OP + 2 * pa * N * OR + Xc;
        psc = R.scale[1] * R.w[Xc % N] * R.w[kr];
    }

    // prologue: face data of the layer below the chunk, this layer's column and halo, the next column
    T cur[N], nxt[N], nx2[N], hal[HS][N];
    T prevU = 0, prevD = 0;
    if (ezb > 0) {
        load_col<T, N, MODE, S, ZP, SP>(nx2, ru, ru2, coff, (uint32_t)(ezb - 1) * lstride, beta);
        prevU = nx2[N - 1];
        prevD = face_r(c, nx2);
    }
    load_col<T, N, MODE, S, ZP, SP>(cur, ru, ru2, coff, (uint32_t)ezb * lstride, beta);
#pragma unroll
    for (int s = 0; s < HS; ++s) load_col<T, N, MODE, S, ZP, SP>(hal[s], ru, ru2, hoff[s], (uint32_t)ezb * lstride, beta);
    if (ezb + 1 < E2) load_col<T, N, MODE, S, ZP, SP>(nxt, ru, ru2, coff, (uint32_t)(ezb + 1) * lstride, beta);
    // cr / D for the nodes of an interior layer, and for the bottom / top node of a boundary layer
    T crD[N], crD0 = 0, crDN = 0;
    if constexpr (IS_CHEB) {
#pragma unroll
        for (int k = 0; k < N; ++k) crD[k] = a.cr * recip(P1 * R.w[k] + P2 * R.B[k][k]);
        crD0 = a.cr * recip(P1 * R.w[0] + P2 * (R.B[0][0] + R.aL[0]));
        crDN = a.cr * recip(P1 * R.w[N - 1] + P2 * (R.B[N - 1][N - 1] - R.aR[N - 1]));
    }

    double dot = 0.0;
    constexpr int ZMAX = slab_zmax(N);  // longest chunk (tile_compiled)
#pragma unroll
    for (int zq = 0; zq < ZMAX; ++zq) {
        const int ez = ezb + zq;
        if (ez >= eze) break;
        const uint32_t soff = (uint32_t)ez * lstride;
        // stage this layer
        if (tact) {
#pragma unroll
            for (int k = 0; k < N; ++k) su[k * PS + su_own] = cur[k];
        }
#pragma unroll
        for (int s = 0; s < HS; ++s) {
            if (hok[s]) {
#pragma unroll
                for (int k = 0; k < N; ++k) su[k * PS + hsu[s]] = hal[s][k];
            }
        }
        // loads for later layers and for this layer's epilogue
        if (ez + 1 < eze) {
#pragma unroll
            for (int s = 0; s < HS; ++s) load_col<T, N, MODE, S, ZP, SP>(hal[s], ru, ru2, hoff[s], soff + lstride, beta);
        }
        if (ez + 1 < eze && ez + 2 < E2) load_col<T, N, MODE, S, ZP, SP>(nx2, ru, ru2, coff, soff + 2 * lstride, beta);
        T fcol[N], zpcol[N];
        if constexpr (HAS_F) {
#pragma unroll
            for (int k = 0; k < N; ++k) fload<S>(fcol[k], rf, coff, soff + k * N2 * SZ);
        }
        if constexpr (IS_CHEB) {
            if (has_zp) {
#pragma unroll
                for (int k = 0; k < N; ++k) fload<S>(zpcol[k], rzp, coff, soff + k * N2 * SZ);
            } else {
#pragma unroll
                for (int k = 0; k < N; ++k) zpcol[k] = 0;
            }
        }
        __syncthreads();
        // x and y terms of element pairs (MF: of element lines, on the matrix cores)
        if constexpr (MF) {
            if (tx0 == 0 || ty0 == 0 || tx0 + TX >= E0 || ty0 + TY >= E1) {  // uniform in the work-group
                mf_ghosts<N, TX, TY>(c, su, tx0, ty0, E0, E1);
                __syncthreads();
            }
            mf_xy_terms<N, TX, TY>(R, mfA, su, sxy);
        } else {
            if (pok) {
                if (isx)
                    pair_row<T, N, 1, 1>(c, su, pb, sxy, ob, pe, E0, psc);
                else
                    pair_row<T, N, RS, OR>(c, su, pb, sxy, ob, pe, E1, psc);
            }
        }
        // z term of the column
        T zacc[N];
        {
            T U, Dv, U0, D0;
            if (ez > 0) {
                U = prevU;
                Dv = prevD;
            } else {
                U = -cur[0];
                Dv = face_l(c, cur) - (T)2 * c.sig * cur[0];
            }
            const T fRc = face_r(c, cur);
            if (ez + 1 < E2) {
                U0 = nxt[0];
                D0 = face_l(c, nxt);
            } else {
                U0 = -cur[N - 1];
                D0 = fRc + (T)2 * c.sig * cur[N - 1];
            }
            elem_op(c, cur, U, Dv, U0, D0, zacc);
            prevU = cur[N - 1];
            prevD = fRc;
        }
        __syncthreads();
        T rr[N];  // BM_RESTRICT: the column's residual (0 outside the mesh)
        if constexpr (MODE == BM_RESTRICT) {
#pragma unroll
            for (int k = 0; k < N; ++k) rr[k] = 0;
        }
        if (colok) {
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const T y = zacc[k] * P2 + sxy[k * OP + so_own] + sxy[N * OP + k * OP + so_own];
                const uint32_t so = soff + k * N2 * SZ;
                if constexpr (MODE == BM_APPLY) {
                    fstore<S>(y, ro, coff, so);
                } else if constexpr (MODE == BM_RESID || MODE == BM_RESIDDOT) {
                    const T r = fcol[k] - y;
                    fstore<S>(r, ro, coff, so);
                    if constexpr (MODE == BM_RESIDDOT) dot += (double)r * (double)r;
                } else if constexpr (IS_CHEB) {
                    T cd = crD[k];
                    if (k == 0 && ez == 0) cd = crD0;
                    if (k == N - 1 && ez == E2 - 1) cd = crDN;
                    const T uz = cur[k];
                    const T zn = uz + a.cp * (uz - zpcol[k]) + cd * (fcol[k] - y);
                    fstore<S>(zn, ro, coff, so);
                    if constexpr (MODE == BM_CHEBDOT) dot += (double)fcol[k] * (double)zn;
                } else if constexpr (MODE == BM_PQ32) {
                    constexpr uint32_t R2 = sizeof(T) / sizeof(SP);
                    fstore<SP>(cur[k], ro2, coff / R2, so / R2);
                    fstore<S>(y, ro, coff, so);
                    dot += (double)cur[k] * (double)y;
                } else if constexpr (IS_PQ) {
                    fstore<S>(cur[k], ro2, coff, so);
                    fstore<S>(y, ro, coff, so);
                    dot += (double)cur[k] * (double)y;
                } else if constexpr (MODE == BM_RESTRICT) {
                    rr[k] = fcol[k] - y;
                }
            }
        }
        if constexpr (MODE == BM_RESTRICT) {
            // fc = (P x P x P)^T r per element: along z in registers, then along y and x
            // from LDS; one thread per coarse node of the tile's elements in this layer
            const TransferDev& tr = *a.tr;
            auto Pm = [&](int i, int c) -> T {
                if constexpr (sizeof(T) == 8)
                    return tr.P[i][c];
                else
                    return tr.Pf[i][c];
            };
            if (tact) {
#pragma unroll
                for (int cc = 0; cc < NC; ++cc) {
                    T s = 0;
#pragma unroll
                    for (int k = 0; k < N; ++k) s += Pm(k, cc) * rr[k];
                    sr[cc * OP + so_own] = s;
                }
            }
            __syncthreads();
            for (int o = t; o < TX * TY * NC3; o += WG) {
                const int el2 = o / NC3, loc = o % NC3;
                const int ca = loc % NC, cb = (loc / NC) % NC, cz = loc / (NC * NC);
                const int exl2 = el2 % TX, eyl2 = el2 / TX, exo = tx0 + exl2, eyo = ty0 + eyl2;
                if (exo >= E0 || eyo >= E1) continue;
                T pa[N], s = 0;
#pragma unroll
                for (int i = 0; i < N; ++i) pa[i] = Pm(i, ca);
#pragma unroll
                for (int jj = 0; jj < N; ++jj) {
                    T u = 0;
#pragma unroll
                    for (int i = 0; i < N; ++i) u += pa[i] * sr[cz * OP + (eyl2 * N + jj) * OR + exl2 * N + i];
                    s += Pm(jj, cb) * u;
                }
                const long long idx =
                    (long long)rhs * a.ndofc + ((long long)(ez * E1 + eyo) * E0 + exo) * NC3 + loc;
                if constexpr (std::is_same<SC, __bf16>::value) {
                    static_assert(sizeof(T) == 4, "BF16 coarse fields: FP32 arithmetic only");
                    reinterpret_cast<__bf16*>(a.fc)[idx] = to_bf16(s);
                    if (a.z1c)
                        reinterpret_cast<__bf16*>(a.z1c)[idx] =
                            to_bf16(a.c0c * s * a.dinvc[idx - (long long)rhs * a.ndofc]);
                } else {
                    a.fc[idx] = s;
                    if (a.z1c) a.z1c[idx] = a.c0c * s * a.dinvc[idx - (long long)rhs * a.ndofc];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < N; ++k) {
            cur[k] = nxt[k];
            nxt[k] = nx2[k];
        }
    }
    if constexpr (DOT) {
        const double s = block_sum<WG>(dot, red);
        if (t == 0) a.partial[(long long)rhs * a.pstride + slot] = s;
    }
}

template <typename T, int N, int BE>
static void brick_dispatch(int mode, const BrickArgs<T>& a, int grid, hipStream_t s) {
    constexpr int WG = wg_of(N * BE * N * BE);
    switch (mode) {
        case BM_APPLY: hipLaunchKernelGGL((k_brick<T, N, BE, BM_APPLY>), dim3(grid), dim3(WG), 0, s, a); break;
        case BM_RESID: hipLaunchKernelGGL((k_brick<T, N, BE, BM_RESID>), dim3(grid), dim3(WG), 0, s, a); break;
        case BM_CHEB: hipLaunchKernelGGL((k_brick<T, N, BE, BM_CHEB>), dim3(grid), dim3(WG), 0, s, a); break;
        case BM_CHEBDOT: hipLaunchKernelGGL((k_brick<T, N, BE, BM_CHEBDOT>), dim3(grid), dim3(WG), 0, s, a); break;
        case BM_PQ: hipLaunchKernelGGL((k_brick<T, N, BE, BM_PQ>), dim3(grid), dim3(WG), 0, s, a); break;
        case BM_RESIDDOT: hipLaunchKernelGGL((k_brick<T, N, BE, BM_RESIDDOT>), dim3(grid), dim3(WG), 0, s, a); break;
    }
}

// Tile of the slab kernel for (precision, nodes per edge): TX x TY elements,
// or {0, 0} where the brick kernel is used.  Layers per z chunk: enough
// chunks for a few thousand work-groups at typical batch sizes.  These are the
// built-in defaults; tile_set overrides them for levels set up afterwards.
static void default_tile(int fp64, int n, int mode, int& tx, int& ty, int& zlen) {
    tx = ty = 0;
    zlen = 4;
    switch (n) {
        case 2: tx = ty = 8; zlen = 2; break;
        case 3: tx = ty = 4; zlen = 4; break;
        case 5:
            // FP64 holds twice the registers: 2x2 tiles pack best.  FP32 smoothing steps and
            // the residual-restriction run fastest on 4x2 tiles, the step with two inputs per
            // node (PQ) on 4x4 (measured)
            if (fp64) {
                tx = ty = 2;
            } else {
                tx = 4;
                ty = (mode == BM_CHEB || mode == BM_CHEBDOT || mode == BM_RESTRICT) ? 2 : 4;
            }
            zlen = 4;
            break;
        default: break;
    }
}

// The shapes launch_slab has kernels for.
static bool tile_compiled(int n, int tx, int ty, int zlen) {
    if (zlen < 1 || zlen > slab_zmax(n)) return false;
    switch (n) {
        case 2: return tx == 8 && ty == 8;
        case 3: return tx == 4 && ty == 4;
        case 5: return (tx == 4 && ty == 2) || (tx == 4 && ty == 4) || (tx == 2 && ty == 2);
        default: return false;
    }
}

namespace {
struct TileTable {
    std::mutex mu;
    bool set[2][8][7] = {};
    int v[2][8][7][3] = {};
};
TileTable& tile_table() {
    static TileTable t;
    return t;
}
}  // namespace

bool tile_set(int fp_bytes, int n, int mode, int tx, int ty, int zlen) {
    if ((fp_bytes != 4 && fp_bytes != 8) || n < 2 || n > 8 || mode < 0 || mode > BM_RESTRICT) return false;
    if (!tile_compiled(n, tx, ty, zlen)) return false;
    auto& t = tile_table();
    std::lock_guard<std::mutex> lock(t.mu);
    const int f = fp_bytes == 8;
    t.set[f][n - 1][mode] = true;
    t.v[f][n - 1][mode][0] = tx;
    t.v[f][n - 1][mode][1] = ty;
    t.v[f][n - 1][mode][2] = zlen;
    return true;
}

bool tile_get(int fp_bytes, int n, int mode, int* tx, int* ty, int* zlen) {
    if ((fp_bytes != 4 && fp_bytes != 8) || n < 2 || n > 8 || mode < 0 || mode > BM_RESTRICT) return false;
    auto& t = tile_table();
    std::lock_guard<std::mutex> lock(t.mu);
    const int f = fp_bytes == 8;
    int x, y, z;
    if (t.set[f][n - 1][mode]) {
        x = t.v[f][n - 1][mode][0]; y = t.v[f][n - 1][mode][1]; z = t.v[f][n - 1][mode][2];
    } else {
        default_tile(f, n, mode, x, y, z);
    }
    if (tx) *tx = x;
    if (ty) *ty = y;
    if (zlen) *zlen = z;
    return true;
}

void assign_tiles(LevelHost& L) {
    for (int f = 0; f < 2; ++f)
        for (int m = 0; m <= BM_RESTRICT; ++m) {
            int* t = L.tile[f][m];
            if (L.n < 2 || L.n > 8 || !tile_get(f ? 8 : 4, L.n, m, &t[0], &t[1], &t[2])) t[0] = t[1] = 0, t[2] = 4;
        }
}

struct SlabGeom {
    int tx, ty, nt0, nt1, zlen, nzc;
};

template <typename T>
static SlabGeom slab_geom(const LevelHost& L, int mode) {
    SlabGeom g;
    const int* t = L.tile[sizeof(T) == 8][mode == BM_PQ32 ? BM_PQ : mode];
    g.tx = t[0];
    g.ty = t[1];
    g.zlen = t[2];
    if (!g.tx) return g;
    g.nt0 = (L.E[0] + g.tx - 1) / g.tx;
    g.nt1 = (L.E[1] + g.ty - 1) / g.ty;
    g.zlen = std::min(g.zlen, L.E[2]);
    g.nzc = (L.E[2] + g.zlen - 1) / g.zlen;
    return g;
}

template <typename T>
int op_blocks(const LevelHost& L, int mode) {
    const SlabGeom g = slab_geom<T>(L, mode);
    return g.tx ? g.nt0 * g.nt1 * g.nzc : bricks_of(L);
}
template int op_blocks<float>(const LevelHost&, int);
template int op_blocks<double>(const LevelHost&, int);

template <typename T, int N, int TX, int TY>
static void slab_dispatch(int mode, const SlabArgs<T>& a, int grid, hipStream_t s) {
    constexpr int WG = wg_of(TX * TY * N * N);
    switch (mode) {
        case BM_APPLY: hipLaunchKernelGGL((k_slab<T, N, TX, TY, BM_APPLY>), dim3(grid), dim3(WG), 0, s, a); break;
        case BM_RESID: hipLaunchKernelGGL((k_slab<T, N, TX, TY, BM_RESID>), dim3(grid), dim3(WG), 0, s, a); break;
        case BM_CHEB: hipLaunchKernelGGL((k_slab<T, N, TX, TY, BM_CHEB>), dim3(grid), dim3(WG), 0, s, a); break;
        case BM_CHEBDOT: hipLaunchKernelGGL((k_slab<T, N, TX, TY, BM_CHEBDOT>), dim3(grid), dim3(WG), 0, s, a); break;
        case BM_PQ: hipLaunchKernelGGL((k_slab<T, N, TX, TY, BM_PQ>), dim3(grid), dim3(WG), 0, s, a); break;
        case BM_RESIDDOT: hipLaunchKernelGGL((k_slab<T, N, TX, TY, BM_RESIDDOT>), dim3(grid), dim3(WG), 0, s, a); break;
        case BM_RESTRICT:
            if constexpr (N == 3 || N == 5)
                hipLaunchKernelGGL((k_slab<T, N, TX, TY, BM_RESTRICT>), dim3(grid), dim3(WG), 0, s, a);
            break;
        case BM_PQ32:
            if constexpr (sizeof(T) == 8)
                hipLaunchKernelGGL((k_slab<T, N, TX, TY, BM_PQ32>), dim3(grid), dim3(WG), 0, s, a);
            break;
    }
}

// The BF16-field forms: FP32 arithmetic on BF16 fields (smoothing, smoothing with f.z, restriction,
// whose coarse outputs are BF16 too when lpc), or the FP64 search-direction step reading a BF16
// V-cycle output.  Degree 4 has every form; degree 2 (the level below a degree-4 finest level)
// smoothing and a restriction into FP32 coarse fields.
template <typename T, int N, int TX, int TY>
static void slab_dispatch_lp(int mode, const SlabArgs<T>& a, int grid, hipStream_t s, bool lpc) {
    constexpr int WG = wg_of(TX * TY * N * N);
    if constexpr (sizeof(T) == 4) {
        switch (mode) {
            case BM_CHEB:
                hipLaunchKernelGGL((k_slab<T, N, TX, TY, BM_CHEB, false, __bf16>), dim3(grid), dim3(WG), 0, s, a);
                break;
            case BM_CHEBDOT:
                if constexpr (N == 5)
                    hipLaunchKernelGGL((k_slab<T, N, TX, TY, BM_CHEBDOT, false, __bf16>), dim3(grid), dim3(WG), 0, s,
                                       a);
                break;
            case BM_RESTRICT:
                if constexpr (N == 5) {
                    if (lpc)
                        hipLaunchKernelGGL((k_slab<T, N, TX, TY, BM_RESTRICT, false, __bf16, float, __bf16, __bf16>),
                                           dim3(grid), dim3(WG), 0, s, a);
                    else
                        hipLaunchKernelGGL((k_slab<T, N, TX, TY, BM_RESTRICT, false, __bf16>), dim3(grid), dim3(WG), 0,
                                           s, a);
                } else {
                    hipLaunchKernelGGL((k_slab<T, N, TX, TY, BM_RESTRICT, false, __bf16>), dim3(grid), dim3(WG), 0, s,
                                       a);
                }
                break;
        }
    } else {
        if (mode == BM_PQ32)
            hipLaunchKernelGGL((k_slab<T, N, TX, TY, BM_PQ32, false, T, __bf16, float>), dim3(grid), dim3(WG), 0, s, a);
    }
}

template <typename T>
static bool launch_slab(int mode, const LevelHost& L, const LevelDev<T>* dev, int nrhs, const RhsState* st,
                        const T* u, const T* u2, const T* f, const T* zprev, T* out, T* out2, double* partial,
                        int pstride, double cp, double cr, hipStream_t s, const LevelHost* Lc = nullptr,
                        const LevelDev<T>* devc = nullptr, T* fc = nullptr, T* z1c = nullptr, double c0c = 0,
                        const void* uf = nullptr, bool mf = false, bool lp = false, bool lpc = false) {
    SlabGeom g = slab_geom<T>(L, mode);
    if (mf && mode == BM_APPLY && L.n == 5) {  // no partial sums: the smoothing steps' 4 x 2 tile, 4 layers
        g.tx = 4;
        g.ty = 2;
        g.nt0 = (L.E[0] + 3) / 4;
        g.nt1 = (L.E[1] + 1) / 2;
        g.zlen = std::min(4, L.E[2]);
        g.nzc = (L.E[2] + g.zlen - 1) / g.zlen;
    }
    if (!g.tx) return false;
    // the matrix-core form exists for FP32 fields of degree 4 on 4 x 2 tiles
    if (mf && !(sizeof(T) == 4 && L.n == 5 && g.tx == 4 && g.ty == 2 &&
                (mode == BM_APPLY || mode == BM_CHEB || mode == BM_CHEBDOT)))
        return false;
    if (mode == BM_RESTRICT && L.n != 3 && L.n != 5) return false;
    SlabArgs<T> a;
    a.Lc = devc;
    a.tr = L.devtr;
    a.fc = fc;
    a.z1c = z1c;
    a.ndofc = Lc ? Lc->ndof : 0;
    if constexpr (sizeof(T) == 8)
        a.dinvc = Lc ? Lc->dinv64 : nullptr;
    else
        a.dinvc = Lc ? Lc->dinv32 : nullptr;
    a.c0c = (T)c0c;
    a.L = dev;
    a.E0 = L.E[0]; a.E1 = L.E[1]; a.E2 = L.E[2];
    a.nt0 = g.nt0; a.nt1 = g.nt1; a.zlen = g.zlen; a.nzc = g.nzc;
    a.nrhs = nrhs;
    a.ndof = L.ndof;
    a.st = st;
    a.u = u; a.uf = uf; a.u2 = u2; a.f = f; a.zprev = zprev; a.out = out; a.out2 = out2;
    a.partial = partial;
    a.pstride = pstride;
    a.cp = (T)cp;
    a.cr = (T)cr;
    const int grid = g.nt0 * g.nt1 * g.nzc * nrhs;
    if (grid == 0) return true;
    // the kernel unrolls its z loop over at most slab_zmax(n) layers
    if (g.zlen > slab_zmax(L.n)) throw std::logic_error("slab chunk longer than the kernel's z loop");
    if constexpr (sizeof(T) == 4) {
        if (mf) {
            constexpr int WG = wg_of(4 * 2 * 5 * 5);
            switch (mode) {
                case BM_APPLY: hipLaunchKernelGGL((k_slab<float, 5, 4, 2, BM_APPLY, true>), dim3(grid), dim3(WG), 0, s, a); break;
                case BM_CHEB: hipLaunchKernelGGL((k_slab<float, 5, 4, 2, BM_CHEB, true>), dim3(grid), dim3(WG), 0, s, a); break;
                case BM_CHEBDOT: hipLaunchKernelGGL((k_slab<float, 5, 4, 2, BM_CHEBDOT, true>), dim3(grid), dim3(WG), 0, s, a); break;
            }
            return true;
        }
    }
    if (lp) {  // BF16 fields: FP32 smoothing and restriction steps (degree 4 and 2), or the FP64 BM_PQ32 step
        if constexpr (sizeof(T) == 4) {
            if (L.n == 5) {
                if (mode != BM_CHEB && mode != BM_CHEBDOT && mode != BM_RESTRICT) return false;
            } else if (L.n == 3) {
                if (mode != BM_CHEB && !(mode == BM_RESTRICT && !lpc)) return false;
            } else {
                return false;
            }
        } else {
            if (mode != BM_PQ32 || L.n != 5) return false;
        }
        if (L.n == 3) {
            if (g.tx == 4 && g.ty == 4) slab_dispatch_lp<T, 3, 4, 4>(mode, a, grid, s, lpc);
            else return false;
            return true;
        }
        if (g.tx == 4 && g.ty == 2) slab_dispatch_lp<T, 5, 4, 2>(mode, a, grid, s, lpc);
        else if (g.tx == 4 && g.ty == 4) slab_dispatch_lp<T, 5, 4, 4>(mode, a, grid, s, lpc);
        else if (g.tx == 2 && g.ty == 2) slab_dispatch_lp<T, 5, 2, 2>(mode, a, grid, s, lpc);
        else return false;
        return true;
    }
    if (g.tx == 8 && g.ty == 8 && L.n == 2) slab_dispatch<T, 2, 8, 8>(mode, a, grid, s);
    else if (g.tx == 4 && g.ty == 4 && L.n == 3) slab_dispatch<T, 3, 4, 4>(mode, a, grid, s);
    else if (g.tx == 4 && g.ty == 2 && L.n == 5) slab_dispatch<T, 5, 4, 2>(mode, a, grid, s);
    else if (g.tx == 4 && g.ty == 4 && L.n == 5) slab_dispatch<T, 5, 4, 4>(mode, a, grid, s);
    else if (g.tx == 2 && g.ty == 2 && L.n == 5) slab_dispatch<T, 5, 2, 2>(mode, a, grid, s);
    else return false;
    return true;
}

template <typename T>
void launch_brick(int mode, const LevelHost& L, const LevelDev<T>* dev, int nrhs, const RhsState* st, const T* u,
                  const T* u2, const T* f, const T* zprev, T* out, T* out2, double* partial, int pstride, double cp,
                  double cr, hipStream_t s) {
    if (launch_slab<T>(mode, L, dev, nrhs, st, u, u2, f, zprev, out, out2, partial, pstride, cp, cr, s)) return;
    BrickArgs<T> a;
    a.L = dev;
    a.E0 = L.E[0]; a.E1 = L.E[1]; a.E2 = L.E[2];
    a.nb0 = L.nbr[0]; a.nb1 = L.nbr[1]; a.nb2 = L.nbr[2];
    a.nrhs = nrhs;
    a.ndof = L.ndof;
    a.st = st;
    a.u = u; a.u2 = u2; a.f = f; a.zprev = zprev; a.out = out; a.out2 = out2;
    a.partial = partial;
    a.pstride = pstride;
    a.cp = (T)cp;
    a.cr = (T)cr;
    const int grid = bricks_of(L) * nrhs;
    if (grid == 0) return;
    switch (L.n) {
        case 2: brick_dispatch<T, 2, be_of<2>()>(mode, a, grid, s); break;
        case 3: brick_dispatch<T, 3, be_of<3>()>(mode, a, grid, s); break;
        case 4: brick_dispatch<T, 4, be_of<4>()>(mode, a, grid, s); break;
        case 5: brick_dispatch<T, 5, be_of<5>()>(mode, a, grid, s); break;
        case 6: brick_dispatch<T, 6, be_of<6>()>(mode, a, grid, s); break;
        case 7: brick_dispatch<T, 7, be_of<7>()>(mode, a, grid, s); break;
        case 8: brick_dispatch<T, 8, be_of<8>()>(mode, a, grid, s); break;
    }
}

bool launch_brick_mf(int mode, const LevelHost& L, const LevelDev<float>* dev, int nrhs, const RhsState* st,
                     const float* u, const float* f, const float* zprev, float* out, double* partial, int pstride,
                     double cp, double cr, hipStream_t s) {
    return launch_slab<float>(mode, L, dev, nrhs, st, u, nullptr, f, zprev, out, nullptr, partial, pstride, cp, cr, s,
                              nullptr, nullptr, nullptr, nullptr, 0.0, nullptr, true);
}

bool launch_brick_lp(int mode, const LevelHost& L, const LevelDev<float>* dev, int nrhs, const RhsState* st,
                     const float* u, const float* f, const float* zprev, float* out, double* partial, int pstride,
                     double cp, double cr, hipStream_t s) {
    return launch_slab<float>(mode, L, dev, nrhs, st, u, nullptr, f, zprev, out, nullptr, partial, pstride, cp, cr, s,
                              nullptr, nullptr, nullptr, nullptr, 0.0, nullptr, false, true);
}

bool launch_restrict_lp(const LevelHost& Lf, const LevelDev<float>* devf, const LevelHost& Lc,
                        const LevelDev<float>* devc, int nrhs, const RhsState* st, const float* z, const float* f,
                        float* fc, float* z1c, double c0c, hipStream_t s, bool coarse_bf16) {
    if (!z || Lf.hcoarse || Lc.n != (Lf.n - 1) / 2 + 1) return false;
    return launch_slab<float>(BM_RESTRICT, Lf, devf, nrhs, st, z, nullptr, f, nullptr, nullptr, nullptr, nullptr, 0,
                              0, 0, s, &Lc, devc, fc, z1c, c0c, nullptr, false, true, coarse_bf16);
}

__global__ __launch_bounds__(256) void k_widen(const float* __restrict__ a, double* __restrict__ b, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) b[i] = (double)a[i];
}

bool has_pq_mixed(const LevelHost& L) { return slab_geom<double>(L, BM_PQ).tx != 0; }

void launch_pq_mixed(const LevelHost& L, const LevelDev<double>* dev, int nrhs, const RhsState* st, const float* z,
                     const double* pold, double* q, double* pnew, double* tmp, double* partial, int pstride,
                     hipStream_t s, bool zbf16) {
    if (nrhs == 0) return;
    if (zbf16) {  // z holds BF16 values
        if (!launch_slab<double>(BM_PQ32, L, dev, nrhs, st, q, pold, nullptr, nullptr, q, pnew, partial, pstride, 0.0,
                                 0.0, s, nullptr, nullptr, nullptr, nullptr, 0.0, z, false, true))
            throw std::logic_error("launch_pq_mixed: no BF16-input kernel for this level");
        return;
    }
    // u is never read in BM_PQ32 (uf takes its place); q keeps the resource base valid
    if (launch_slab<double>(BM_PQ32, L, dev, nrhs, st, q, pold, nullptr, nullptr, q, pnew, partial, pstride, 0.0,
                            0.0, s, nullptr, nullptr, nullptr, nullptr, 0.0, z))
        return;
    if (!tmp) throw std::logic_error("launch_pq_mixed: no slab kernel for this degree and no widening buffer");
    const long long n = L.ndof * nrhs;
    hipLaunchKernelGGL(k_widen, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, z, tmp, n);
    launch_brick<double>(BM_PQ, L, dev, nrhs, st, tmp, pold, nullptr, nullptr, q, pnew, partial, pstride, 0.0, 0.0, s);
}

template void launch_brick<double>(int, const LevelHost&, const LevelDev<double>*, int, const RhsState*,
                                   const double*, const double*, const double*, const double*, double*, double*,
                                   double*, int, double, double, hipStream_t);
template void launch_brick<float>(int, const LevelHost&, const LevelDev<float>*, int, const RhsState*, const float*,
                                  const float*, const float*, const float*, float*, float*, double*, int, double,
                                  double, hipStream_t);

// ---------------------------------------------------------------------------
// restriction: fc = P^T (f - A z) over a fine brick

template <typename T>
struct TransferArgs {
    const LevelDev<T>* Lf;
    const LevelDev<T>* Lc;
    const TransferDev* tr;
    int E0, E1, E2;        // fine elements
    int nb0, nb1, nb2;     // fine bricks
    int Ec0, Ec1, Ec2;     // coarse elements
    int nrhs;
    long long ndof, ndofc;
    const RhsState* st;
    const T* z;            // restriction: fine iterate (may be null); prolongation: coarse correction
    const T* f;            // fine right-hand side
    T* fc;                 // restriction output
    T* z1c;                // optional c0c Dc^-1 fc
    T* zf;                 // prolongation target
    T c0c;
};

template <typename T>
__device__ __forceinline__ T trP(const TransferDev& tr, int a, int b) {
    if constexpr (sizeof(T) == 8)
        return tr.P[a][b];
    else
        return tr.Pf[a][b];
}

template <typename T, int NF, int BE, int NC, bool HC, bool HASZ>
__global__ __launch_bounds__(wg_of(NF* BE* NF* BE), 2) void k_restrict(TransferArgs<T> a) {
    constexpr int NB = NF * BE, NT = NB * NB, SY = NB + 1, SZ = NB * SY, N3 = NF * NF * NF;
    constexpr int CBE = HC ? BE / 2 : BE;  // coarse elements per brick edge
    constexpr int NCB = CBE * NC;          // coarse nodes per brick edge
    constexpr int NC3 = NC * NC * NC;
    constexpr int WG = wg_of(NT);
    static_assert(!HC || BE % 2 == 0, "mesh coarsening needs an even brick edge");
    __shared__ T su[NB * SZ];
    __shared__ T sx[NB * SZ];

    const int nbr = a.nb0 * a.nb1 * a.nb2;
    const int w = xcd_remap(blockIdx.x, nbr * a.nrhs);
    const int rhs = w / nbr, br = w % nbr;
    if (a.st && !a.st[rhs].active) return;
    const int bx = br % a.nb0, by = (br / a.nb0) % a.nb1, bz = br / (a.nb0 * a.nb1);
    const int ex0 = bx * BE, ey0 = by * BE, ez0 = bz * BE;
    const long long base = (long long)rhs * a.ndof;
    const T* f = a.f + base;
    const int t = threadIdx.x;
    const int X = t % NB, Y = t / NB;
    const int exX = ex0 + X / NF, iX = X % NF, eyY = ey0 + Y / NF, jY = Y % NF;
    const bool colok = t < NT && exX < a.E0 && eyY < a.E1;
    const int E0 = a.E0, E1 = a.E1, E2 = a.E2;

    T rcol[NB], fcol[NB];
    BrickIn<T, NF, BE> in;
    if constexpr (HASZ) {
        brick_load<T, NF, BE, BM_APPLY>(E0, E1, E2, ex0, ey0, ez0, a.z + base, nullptr, (T)0, in);
        brick_compute<T, NF, BE>(E0, E1, E2, *a.Lf, ex0, ey0, ez0, in, su, sx, rcol);
    }
#pragma unroll
    for (int Z = 0; Z < NB; ++Z) {
        const int ez = ez0 + Z / NF, k = Z % NF;
        fcol[Z] = (colok && ez < E2) ? ld32(f, (uint32_t)((ez * E1 + eyY) * E0 + exX) * N3 + (k * NF + jY) * NF + iX) : (T)0;
    }
#pragma unroll
    for (int Z = 0; Z < NB; ++Z) {
        const int ez = ez0 + Z / NF;
        T r = 0;
        if (colok && ez < E2) {
            if constexpr (HASZ)
                r = fcol[Z] - rcol[Z];
            else
                r = fcol[Z];
        }
        rcol[Z] = r;
    }
    __syncthreads();  // LDS of the apply is free again
    const TransferDev& tr = *a.tr;
    // along Z in registers -> su[Zc][Y][X]
    if (t < NT) {
#pragma unroll
        for (int Zc = 0; Zc < NCB; ++Zc) {
            T s = 0;
#pragma unroll
            for (int Z = 0; Z < NB; ++Z) s += trP<T>(tr, Z, Zc) * rcol[Z];
            su[Zc * SZ + Y * SY + X] = s;
        }
    }
    __syncthreads();
    // along Y: thread (X, Zc) -> sx[Zc][Yc][X]
    if (t < NB * NCB) {
        const int Xr = t % NB, Zc = t / NB;
        T col[NB];
#pragma unroll
        for (int y = 0; y < NB; ++y) col[y] = su[Zc * SZ + y * SY + Xr];
#pragma unroll
        for (int Yc = 0; Yc < NCB; ++Yc) {
            T s = 0;
#pragma unroll
            for (int y = 0; y < NB; ++y) s += trP<T>(tr, y, Yc) * col[y];
            sx[Zc * SZ + Yc * SY + Xr] = s;
        }
    }
    __syncthreads();
    // along X: thread (Yc, Zc) -> coarse output
    if (t < NCB * NCB) {
        const int Yc = t % NCB, Zc = t / NCB;
        const int ecx0 = HC ? ex0 / 2 : ex0, ecy0 = HC ? ey0 / 2 : ey0, ecz0 = HC ? ez0 / 2 : ez0;
        const int ecy = ecy0 + Yc / NC, jc = Yc % NC, ecz = ecz0 + Zc / NC, kc = Zc % NC;
        if (ecy < a.Ec1 && ecz < a.Ec2) {
            T col[NB];
#pragma unroll
            for (int x = 0; x < NB; ++x) col[x] = sx[Zc * SZ + Yc * SY + x];
            const long long cbase = (long long)rhs * a.ndofc;
#pragma unroll
            for (int Xc = 0; Xc < NCB; ++Xc) {
                const int ecx = ecx0 + Xc / NC, ic = Xc % NC;
                if (ecx >= a.Ec0) continue;
                T s = 0;
#pragma unroll
                for (int x = 0; x < NB; ++x) s += trP<T>(tr, x, Xc) * col[x];
                const long long idx = cbase + ((long long)(ecz * a.Ec1 + ecy) * a.Ec0 + ecx) * NC3 + (kc * NC + jc) * NC + ic;
                a.fc[idx] = s;
                if (a.z1c) {
                    const LevelDev<T>& Lc = *a.Lc;
                    const int tx = etype(ecx, a.Ec0), ty = etype(ecy, a.Ec1), tz = etype(ecz, a.Ec2);
                    const T mx = Lc.ax[0].m[ic], my = Lc.ax[1].m[jc], mz = Lc.ax[2].m[kc];
                    const T D = Lc.ax[0].Bd[tx][ic] * my * mz + mx * Lc.ax[1].Bd[ty][jc] * mz + mx * my * Lc.ax[2].Bd[tz][kc];
                    a.z1c[idx] = a.c0c * s / D;
                }
            }
        }
    }
}

// prolongation and correction: zf += P zc over a fine brick
template <typename T, int NF, int BE, int NC, bool HC>
__global__ __launch_bounds__(wg_of(NF* BE* NF* BE)) void k_prolong(TransferArgs<T> a) {
    constexpr int NB = NF * BE, NT = NB * NB, N3 = NF * NF * NF;
    constexpr int CBE = HC ? BE / 2 : BE;
    constexpr int NCB = CBE * NC;
    constexpr int NC3 = NC * NC * NC;
    __shared__ T sc[NCB * NCB * NCB];
    __shared__ T s1[NCB * NCB * NB];
    __shared__ T s2[NCB * NB * NB];

    const int nbr = a.nb0 * a.nb1 * a.nb2;
    const int w = xcd_remap(blockIdx.x, nbr * a.nrhs);
    const int rhs = w / nbr, br = w % nbr;
    if (a.st && !a.st[rhs].active) return;
    const int bx = br % a.nb0, by = (br / a.nb0) % a.nb1, bz = br / (a.nb0 * a.nb1);
    const int ex0 = bx * BE, ey0 = by * BE, ez0 = bz * BE;
    const int ecx0 = HC ? ex0 / 2 : ex0, ecy0 = HC ? ey0 / 2 : ey0, ecz0 = HC ? ez0 / 2 : ez0;
    const int t = threadIdx.x;
    const T* zc = a.z + (long long)rhs * a.ndofc;
    for (int q = t; q < NCB * NCB * NCB; q += blockDim.x) {
        const int Xc = q % NCB, Yc = (q / NCB) % NCB, Zc = q / (NCB * NCB);
        const int ecx = ecx0 + Xc / NC, ecy = ecy0 + Yc / NC, ecz = ecz0 + Zc / NC;
        T v = 0;
        if (ecx < a.Ec0 && ecy < a.Ec1 && ecz < a.Ec2)
            v = zc[((long long)(ecz * a.Ec1 + ecy) * a.Ec0 + ecx) * NC3 + ((Zc % NC) * NC + (Yc % NC)) * NC + (Xc % NC)];
        sc[q] = v;
    }
    __syncthreads();
    const TransferDev& tr = *a.tr;
    if (t < NCB * NCB) {  // along X: thread (Yc, Zc)
        const int Yc = t % NCB, Zc = t / NCB;
        T c[NCB];
#pragma unroll
        for (int x = 0; x < NCB; ++x) c[x] = sc[(Zc * NCB + Yc) * NCB + x];
#pragma unroll
        for (int X = 0; X < NB; ++X) {
            T s = 0;
#pragma unroll
            for (int x = 0; x < NCB; ++x) s += trP<T>(tr, X, x) * c[x];
            s1[(Zc * NCB + Yc) * NB + X] = s;
        }
    }
    __syncthreads();
    if (t < NB * NCB) {  // along Y: thread (X, Zc)
        const int X = t % NB, Zc = t / NB;
        T c[NCB];
#pragma unroll
        for (int y = 0; y < NCB; ++y) c[y] = s1[(Zc * NCB + y) * NB + X];
#pragma unroll
        for (int Y = 0; Y < NB; ++Y) {
            T s = 0;
#pragma unroll
            for (int y = 0; y < NCB; ++y) s += trP<T>(tr, Y, y) * c[y];
            s2[(Zc * NB + Y) * NB + X] = s;
        }
    }
    __syncthreads();
    if (t < NT) {  // along Z: thread (X, Y), add into the fine field
        const int X = t % NB, Y = t / NB;
        const int exX = ex0 + X / NF, iX = X % NF, eyY = ey0 + Y / NF, jY = Y % NF;
        if (exX < a.E0 && eyY < a.E1) {
            T c[NCB];
#pragma unroll
            for (int z = 0; z < NCB; ++z) c[z] = s2[(z * NB + Y) * NB + X];
            T* zf = a.zf + (long long)rhs * a.ndof;
#pragma unroll
            for (int Z = 0; Z < NB; ++Z) {
                const int ez = ez0 + Z / NF, k = Z % NF;
                if (ez >= a.E2) continue;
                T s = 0;
#pragma unroll
                for (int z = 0; z < NCB; ++z) s += trP<T>(tr, Z, z) * c[z];
                const long long idx = ((long long)(ez * a.E1 + eyY) * a.E0 + exX) * N3 + (k * NF + jY) * NF + iX;
                zf[idx] += s;
            }
        }
    }
}

template <typename T>
static TransferArgs<T> transfer_args(const LevelHost& Lf, const LevelHost& Lc, int nrhs, const RhsState* st) {
    TransferArgs<T> a;
    a.tr = Lf.devtr;
    a.E0 = Lf.E[0]; a.E1 = Lf.E[1]; a.E2 = Lf.E[2];
    a.nb0 = Lf.nbr[0]; a.nb1 = Lf.nbr[1]; a.nb2 = Lf.nbr[2];
    a.Ec0 = Lc.E[0]; a.Ec1 = Lc.E[1]; a.Ec2 = Lc.E[2];
    a.nrhs = nrhs;
    a.ndof = Lf.ndof;
    a.ndofc = Lc.ndof;
    a.st = st;
    a.z = nullptr; a.f = nullptr; a.fc = nullptr; a.z1c = nullptr; a.zf = nullptr;
    a.Lf = nullptr; a.Lc = nullptr;
    a.c0c = 0;
    return a;
}

#define DG_TRANSFER_CASES(MACRO) \
    MACRO(8, 4, false)           \
    MACRO(7, 4, false)           \
    MACRO(6, 3, false)           \
    MACRO(5, 3, false)           \
    MACRO(4, 2, false)           \
    MACRO(3, 2, false)           \
    MACRO(2, 2, true)

template <typename T>
void launch_restrict(const LevelHost& Lf, const LevelDev<T>* devf, const LevelHost& Lc, const LevelDev<T>* devc,
                     int nrhs, const RhsState* st, const T* z, const T* f, T* fc, T* z1c, double c0c,
                     hipStream_t s) {
    // degree steps with an iterate: the slab kernel with the restriction in its epilogue
    if (z && !Lf.hcoarse && Lc.n == (Lf.n - 1) / 2 + 1 &&
        launch_slab<T>(BM_RESTRICT, Lf, devf, nrhs, st, z, nullptr, f, nullptr, nullptr, nullptr, nullptr, 0, 0, 0, s,
                       &Lc, devc, fc, z1c, c0c))
        return;
    TransferArgs<T> a = transfer_args<T>(Lf, Lc, nrhs, st);
    a.Lf = devf; a.Lc = devc; a.z = z; a.f = f; a.fc = fc; a.z1c = z1c; a.c0c = (T)c0c;
    const int grid = bricks_of(Lf) * nrhs;
    if (grid == 0) return;
    const bool hc = Lf.hcoarse;
#define DG_R(NF, NC, HC)                                                                                         \
    if (Lf.n == NF && Lc.n == NC && hc == HC) {                                                                 \
        constexpr int BE = be_of<NF>();                                                                         \
        constexpr int WG = wg_of(NF * BE * NF * BE);                                                            \
        if (z)                                                                                                  \
            hipLaunchKernelGGL((k_restrict<T, NF, BE, NC, HC, true>), dim3(grid), dim3(WG), 0, s, a);           \
        else                                                                                                    \
            hipLaunchKernelGGL((k_restrict<T, NF, BE, NC, HC, false>), dim3(grid), dim3(WG), 0, s, a);          \
        return;                                                                                                 \
    }
    DG_TRANSFER_CASES(DG_R)
#undef DG_R
    fprintf(stderr, "dg: no restriction kernel for %d -> %d\n", Lf.n, Lc.n);
}

// Prolongation and correction of a degree step, zf += (P x P x P) zc element by
// element (the coarse and fine levels share the elements).  A work-group
// takes EPW consecutive elements (of the packed right-hand sides): their coarse
// values are staged in LDS with coalesced loads, then one thread per fine node
// column (i, j) of an element contracts along x and y (NC^2 coarse values per
// coarse z node) and then along z in registers, and updates its NF nodes.
// SET: zf = scale[rhs] * P zc (every fine node written once) instead of zf += P zc.
// SF: storage type of zf (T, or BF16 under FP32 arithmetic: read, add, round to nearest even); SZ:
// storage type of zc (T, or BF16 widened on load).
template <typename T, int NF, int NC, bool SET = false, typename SF = T, typename SZ = T>
__global__ __launch_bounds__(256) void k_prolong_deg(const TransferDev* __restrict__ trp, long long nelem_rhs,
                                                     long long nelem, const RhsState* st, const SZ* __restrict__ zc,
                                                     SF* __restrict__ zf, const double* __restrict__ scale = nullptr) {
    constexpr int NF2 = NF * NF, NF3 = NF2 * NF, NC3 = NC * NC * NC;
    constexpr int EPW = 256 / NF2;
    __shared__ T sc[EPW * NC3];
    const TransferDev& tr = *trp;
    auto Pm = [&](int i, int c) -> T {
        if constexpr (sizeof(T) == 8)
            return tr.P[i][c];
        else
            return tr.Pf[i][c];
    };
    const long long e0 = (long long)blockIdx.x * EPW;
    const int ne = (int)min((long long)EPW, nelem - e0);
    for (int q = threadIdx.x; q < ne * NC3; q += 256) {
        if constexpr (std::is_same<SZ, __bf16>::value)
            sc[q] = from_bf16(zc[e0 * NC3 + q]);
        else
            sc[q] = zc[e0 * NC3 + q];
    }
    __syncthreads();
    const int el = threadIdx.x / NF2, col = threadIdx.x % NF2;
    if (el >= ne) return;
    const long long e = e0 + el;
    if (st && !st[e / nelem_rhs].active) return;
    const int i = col % NF, j = col / NF;
    T pi[NC], pj[NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) {
        pi[a] = Pm(i, a);
        pj[a] = Pm(j, a);
    }
    T t[NC];
    const T* c = sc + el * NC3;
#pragma unroll
    for (int cz = 0; cz < NC; ++cz) {
        T acc = 0;
#pragma unroll
        for (int b = 0; b < NC; ++b) {
            T u = 0;
#pragma unroll
            for (int a = 0; a < NC; ++a) u += pi[a] * c[(cz * NC + b) * NC + a];
            acc += pj[b] * u;
        }
        t[cz] = acc;
    }
    SF* out = zf + e * NF3 + col;
    const T sc_rhs = SET ? (T)scale[e / nelem_rhs] : (T)0;
#pragma unroll
    for (int k = 0; k < NF; ++k) {
        T v = 0;
#pragma unroll
        for (int cz = 0; cz < NC; ++cz) v += Pm(k, cz) * t[cz];
        if constexpr (std::is_same<SF, __bf16>::value) {
            static_assert(!SET && sizeof(T) == 4, "BF16 fine fields: FP32 correction only");
            out[k * NF2] = to_bf16(from_bf16(out[k * NF2]) + v);
        } else if constexpr (SET) {
            out[k * NF2] = v * sc_rhs;
        } else {
            out[k * NF2] += v;
        }
    }
}

bool launch_prolong_set(const LevelHost& Lf, const LevelHost& Lc, int nrhs, const double* zc, double* zf,
                        const double* scale, hipStream_t s) {
    if (Lf.hcoarse || Lf.E[0] != Lc.E[0] || Lf.E[1] != Lc.E[1] || Lf.E[2] != Lc.E[2]) return false;
    const long long nel = (long long)Lf.E[0] * Lf.E[1] * Lf.E[2];
    const long long tot = nel * nrhs;
    if (tot == 0) return true;
#define DG_PS(NF, NC)                                                                                          \
    if (Lf.n == NF && Lc.n == NC) {                                                                            \
        constexpr int EPW = 256 / (NF * NF);                                                                   \
        hipLaunchKernelGGL((k_prolong_deg<double, NF, NC, true>), dim3((unsigned)((tot + EPW - 1) / EPW)),     \
                           dim3(256), 0, s, Lf.devtr, nel, tot, nullptr, zc, zf, scale);                       \
        return true;                                                                                           \
    }
    DG_PS(5, 3)
    DG_PS(3, 2)
#undef DG_PS
    return false;
}

bool launch_prolong_lp(const LevelHost& Lf, const LevelHost& Lc, int nrhs, const RhsState* st, const float* zc,
                       float* zf, hipStream_t s, bool coarse_bf16) {
    if (Lf.hcoarse || Lf.E[0] != Lc.E[0] || Lf.E[1] != Lc.E[1] || Lf.E[2] != Lc.E[2]) return false;
    const bool d42 = Lf.n == 5 && Lc.n == 3, d21 = Lf.n == 3 && Lc.n == 2 && !coarse_bf16;
    if (!d42 && !d21) return false;
    const long long nel = (long long)Lf.E[0] * Lf.E[1] * Lf.E[2];
    const long long tot = nel * nrhs;
    if (tot == 0) return true;
    __bf16* zfb = reinterpret_cast<__bf16*>(zf);
    if (d21) {
        constexpr int EPW = 256 / 9;
        hipLaunchKernelGGL((k_prolong_deg<float, 3, 2, false, __bf16>), dim3((unsigned)((tot + EPW - 1) / EPW)),
                           dim3(256), 0, s, Lf.devtr, nel, tot, st, zc, zfb, nullptr);
        return true;
    }
    constexpr int EPW = 256 / 25;
    const unsigned grid = (unsigned)((tot + EPW - 1) / EPW);
    if (coarse_bf16)
        hipLaunchKernelGGL((k_prolong_deg<float, 5, 3, false, __bf16, __bf16>), dim3(grid), dim3(256), 0, s, Lf.devtr,
                           nel, tot, st, reinterpret_cast<const __bf16*>(zc), zfb, nullptr);
    else
        hipLaunchKernelGGL((k_prolong_deg<float, 5, 3, false, __bf16>), dim3(grid), dim3(256), 0, s, Lf.devtr, nel,
                           tot, st, zc, zfb, nullptr);
    return true;
}

template <typename T>
void launch_prolong(const LevelHost& Lf, const LevelHost& Lc, int nrhs, const RhsState* st, const T* zc, T* zf,
                    hipStream_t s) {
    if (!Lf.hcoarse && Lf.E[0] == Lc.E[0] && Lf.E[1] == Lc.E[1] && Lf.E[2] == Lc.E[2]) {
        const long long nel = (long long)Lf.E[0] * Lf.E[1] * Lf.E[2];
        const long long tot = nel * nrhs;
        if (tot == 0) return;
#define DG_PD(NF, NC)                                                                                          \
        if (Lf.n == NF && Lc.n == NC) {                                                                        \
            constexpr int EPW = 256 / (NF * NF);                                                               \
            hipLaunchKernelGGL((k_prolong_deg<T, NF, NC>), dim3((unsigned)((tot + EPW - 1) / EPW)), dim3(256), \
                               0, s, Lf.devtr, nel, tot, st, zc, zf);                                          \
            return;                                                                                            \
        }
        DG_PD(5, 3)
        DG_PD(3, 2)
#undef DG_PD
    }
    TransferArgs<T> a = transfer_args<T>(Lf, Lc, nrhs, st);
    a.z = zc; a.zf = zf;
    const int grid = bricks_of(Lf) * nrhs;
    if (grid == 0) return;
    const bool hc = Lf.hcoarse;
#define DG_P(NF, NC, HC)                                                                                \
    if (Lf.n == NF && Lc.n == NC && hc == HC) {                                                        \
        constexpr int BE = be_of<NF>();                                                                \
        constexpr int WG = wg_of(NF * BE * NF * BE);                                                   \
        hipLaunchKernelGGL((k_prolong<T, NF, BE, NC, HC>), dim3(grid), dim3(WG), 0, s, a);             \
        return;                                                                                        \
    }
    DG_TRANSFER_CASES(DG_P)
#undef DG_P
    fprintf(stderr, "dg: no prolongation kernel for %d -> %d\n", Lf.n, Lc.n);
}

template void launch_restrict<double>(const LevelHost&, const LevelDev<double>*, const LevelHost&,
                                      const LevelDev<double>*, int, const RhsState*, const double*, const double*,
                                      double*, double*, double, hipStream_t);
template void launch_restrict<float>(const LevelHost&, const LevelDev<float>*, const LevelHost&,
                                     const LevelDev<float>*, int, const RhsState*, const float*, const float*, float*,
                                     float*, double, hipStream_t);
template void launch_prolong<double>(const LevelHost&, const LevelHost&, int, const RhsState*, const double*, double*,
                                     hipStream_t);
template void launch_prolong<float>(const LevelHost&, const LevelHost&, int, const RhsState*, const float*, float*,
                                    hipStream_t);

// ---------------------------------------------------------------------------
// coarsest level: exact solve by fast diagonalisation, one work-group per RHS

// Padded LDS strides of the coarsest-level array g[Z][Y][X] (at most CMAX per
// axis): odd row stride and a plane stride that spreads the Z lines over the
// banks.
constexpr int CSY = CMAX + 1;
constexpr int CSZ = CMAX * CSY + 2;

// Exact coarsest-level solve of one right-hand side by a work-group of 1024 / LPT threads: rr and
// zz are its fields (element-major, ndof values), g (CMAX * CSZ doubles) and Qs (3 CMAX^2) LDS.
template <typename T, int LPT = 1>
__device__ __forceinline__ void coarse_wg(const CoarseDev* __restrict__ C, long long ndof, const T* __restrict__ rr,
                                          T* __restrict__ zz, double* g, double (*Qs)[CMAX][CMAX]) {
    const int nx = C->n[0], ny = C->n[1], nz = C->n[2], N = C->N;
    const int E0 = C->E[0], E1 = C->E[1];
    const int N3 = N * N * N;
    const int t = threadIdx.x;
    const int nd = (int)ndof;
    for (int q = t; q < 3 * CMAX * CMAX; q += blockDim.x) (&Qs[0][0][0])[q] = (&C->Q[0][0][0])[q];
    for (int q = t; q < nd; q += blockDim.x) {
        const int e = q / N3, l = q - e * N3;
        const int ex = e % E0, ey = (e / E0) % E1, ez = e / (E0 * E1);
        const int i = l % N, j = (l / N) % N, k = l / (N * N);
        const int Xg = ex * N + i, Yg = ey * N + j, Zg = ez * N + k;
        g[Zg * CSZ + Yg * CSY + Xg] = (double)rr[q] * C->s[0][Xg] * C->s[1][Yg] * C->s[2][Zg];
    }
    __syncthreads();
    // three contractions with Q^T, the eigenvalue scaling, three with Q.  A
    // line of n values is shared by 4 threads, each producing a quarter of
    // the outputs; a work-group of fewer than 1024 threads takes LPT lines
    // per thread group.
    for (int pass = 0; pass < 6; ++pass) {
        const int axis = pass % 3;
        const bool fwd = pass < 3;
        const int n = C->n[axis];
        const int nl = (nx * ny * nz) / n;
        const int part = t & 3;
        double w[LPT][CMAX / 4];
        int o[LPT], stride[LPT];
        bool act[LPT];
#pragma unroll
        for (int m = 0; m < LPT; ++m) {
            const int line = (t >> 2) + m * ((int)blockDim.x >> 2);
            act[m] = line < nl;
            o[m] = 0;
            stride[m] = 1;
            if (act[m]) {
                if (axis == 0) { const int Zg = line / ny, Yg = line % ny; o[m] = Zg * CSZ + Yg * CSY; stride[m] = 1; }
                else if (axis == 1) { const int Zg = line / nx, Xg = line % nx; o[m] = Zg * CSZ + Xg; stride[m] = CSY; }
                else { const int Yg = line / nx, Xg = line % nx; o[m] = Yg * CSY + Xg; stride[m] = CSZ; }
                double v[CMAX];
#pragma unroll
                for (int b = 0; b < CMAX; ++b) v[b] = b < n ? g[o[m] + b * stride[m]] : 0.0;
#pragma unroll
                for (int a4 = 0; a4 < CMAX / 4; ++a4) {
                    const int a2 = part + 4 * a4;
                    double s = 0.0;
#pragma unroll
                    for (int b = 0; b < CMAX; ++b)
                        if (a2 < n && b < n) s += (fwd ? Qs[axis][b][a2] : Qs[axis][a2][b]) * v[b];
                    w[m][a4] = s;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < LPT; ++m) {
            if (act[m]) {
#pragma unroll
                for (int a4 = 0; a4 < CMAX / 4; ++a4) {
                    const int a2 = part + 4 * a4;
                    if (a2 < n) g[o[m] + a2 * stride[m]] = w[m][a4];
                }
            }
        }
        __syncthreads();
        if (pass == 2) {
            for (int q = t; q < nx * ny * nz; q += blockDim.x) {
                const int Xg = q % nx, Yg = (q / nx) % ny, Zg = q / (nx * ny);
                g[Zg * CSZ + Yg * CSY + Xg] /= (C->lam[0][Xg] + C->lam[1][Yg] + C->lam[2][Zg]);
            }
            __syncthreads();
        }
    }
    for (int q = t; q < nd; q += blockDim.x) {
        const int e = q / N3, l = q - e * N3;
        const int ex = e % E0, ey = (e / E0) % E1, ez = e / (E0 * E1);
        const int i = l % N, j = (l / N) % N, k = l / (N * N);
        const int Xg = ex * N + i, Yg = ey * N + j, Zg = ez * N + k;
        zz[q] = (T)(g[Zg * CSZ + Yg * CSY + Xg] * C->s[0][Xg] * C->s[1][Yg] * C->s[2][Zg]);
    }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_coarse(const CoarseDev* __restrict__ C, int nrhs, long long ndof,
                                                 const RhsState* st, const T* __restrict__ r, T* __restrict__ z) {
    __shared__ double g[CMAX * CSZ];
    __shared__ double Qs[3][CMAX][CMAX];
    const int rhs = blockIdx.x;
    if (st && !st[rhs].active) return;
    coarse_wg<T>(C, ndof, r + (long long)rhs * ndof, z + (long long)rhs * ndof, g, Qs);
}

// The same exact solve spread over many work-groups, in three launches (each a barrier-free
// phase): per z plane the x and y contractions with Q^T of S r; per group of 16 z lines the z
// contraction with Q^T, the division by the eigenvalue sums and the z contraction with Q; per z
// plane the x and y contractions with Q and the scaling by S back into element order.  g1, g2:
// FP64 scratch, nrhs lexicographic fields of the level (X fastest).  At most CMAX nodes per axis,
// so a z plane (at most 256 nodes) is one work-group.
__device__ __forceinline__ int coarse_em(const CoarseDev& C, int X, int Y, int Z) {
    const int N = C.N;
    const int ex = X / N, i = X - ex * N, ey = Y / N, j = Y - ey * N, ez = Z / N, k = Z - ez * N;
    return ((ez * C.E[1] + ey) * C.E[0] + ex) * N * N * N + (k * N + j) * N + i;
}

template <typename T>
__global__ __launch_bounds__(256) void k_coarse_xy_fwd(const CoarseDev* __restrict__ Cp, long long ndof,
                                                       const RhsState* st, const T* __restrict__ r,
                                                       double* __restrict__ g1) {
    __shared__ double sp[CMAX * CMAX], tp[CMAX * CMAX];
    const int rhs = blockIdx.y, Z = blockIdx.x, t = threadIdx.x;
    if (st && !st[rhs].active) return;
    const CoarseDev& C = *Cp;
    const int nx = C.n[0], ny = C.n[1], nxy = nx * ny;
    const T* rr = r + (long long)rhs * ndof;
    if (t < nxy) {
        const int X = t % nx, Y = t / nx;
        sp[t] = (double)rr[coarse_em(C, X, Y, Z)] * C.s[0][X] * C.s[1][Y];
    }
    __syncthreads();
    if (t < nxy) {  // (Y, Xo): along x
        const int Xo = t % nx, Y = t / nx;
        double a = 0.0;
        for (int X = 0; X < nx; ++X) a += C.Q[0][X][Xo] * sp[Y * nx + X];
        tp[t] = a;
    }
    __syncthreads();
    if (t < nxy) {  // (Yo, Xo): along y
        const int Xo = t % nx, Yo = t / nx;
        double a = 0.0;
        for (int Y = 0; Y < ny; ++Y) a += C.Q[1][Y][Yo] * tp[Y * nx + Xo];
        g1[(long long)rhs * ndof + (long long)Z * nxy + t] = a * C.s[2][Z];
    }
}

__global__ __launch_bounds__(256) void k_coarse_z(const CoarseDev* __restrict__ Cp, long long ndof, const RhsState* st,
                                                  const double* __restrict__ g1, double* __restrict__ g2) {
    __shared__ double sv[16][CMAX + 1];
    const int rhs = blockIdx.y, t = threadIdx.x;
    if (st && !st[rhs].active) return;
    const CoarseDev& C = *Cp;
    const int nx = C.n[0], nxy = nx * C.n[1], nz = C.n[2];
    const int ln = t / 16, k = t % 16, line = blockIdx.x * 16 + ln;  // 16 z lines of 16 entries
    const bool ok = line < nxy && k < nz;
    const double* a1 = g1 + (long long)rhs * ndof;
    double v = 0.0;
    if (ok) {
        for (int Z = 0; Z < nz; ++Z) v += C.Q[2][Z][k] * a1[(long long)Z * nxy + line];
        v /= (C.lam[0][line % nx] + C.lam[1][line / nx] + C.lam[2][k]);
    }
    sv[ln][k] = v;
    __syncthreads();
    if (ok) {
        double w = 0.0;
        for (int c = 0; c < nz; ++c) w += C.Q[2][k][c] * sv[ln][c];
        g2[(long long)rhs * ndof + (long long)k * nxy + line] = w;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_coarse_xy_back(const CoarseDev* __restrict__ Cp, long long ndof,
                                                        const RhsState* st, const double* __restrict__ g2,
                                                        T* __restrict__ z) {
    __shared__ double sp[CMAX * CMAX], tp[CMAX * CMAX];
    const int rhs = blockIdx.y, Z = blockIdx.x, t = threadIdx.x;
    if (st && !st[rhs].active) return;
    const CoarseDev& C = *Cp;
    const int nx = C.n[0], ny = C.n[1], nxy = nx * ny;
    if (t < nxy) sp[t] = g2[(long long)rhs * ndof + (long long)Z * nxy + t];
    __syncthreads();
    if (t < nxy) {  // (Yo, X): along x
        const int X = t % nx, Yo = t / nx;
        double a = 0.0;
        for (int Xo = 0; Xo < nx; ++Xo) a += C.Q[0][X][Xo] * sp[Yo * nx + Xo];
        tp[t] = a;
    }
    __syncthreads();
    if (t < nxy) {  // (Y, X): along y, scaled, into element order
        const int X = t % nx, Y = t / nx;
        double a = 0.0;
        for (int Yo = 0; Yo < ny; ++Yo) a += C.Q[1][Y][Yo] * tp[Yo * nx + X];
        z[(long long)rhs * ndof + coarse_em(C, X, Y, Z)] = (T)(a * C.s[0][X] * C.s[1][Y] * C.s[2][Z]);
    }
}

template <typename T>
void launch_coarse(const CoarseDev* C, const LevelHost& L, int nrhs, const RhsState* st, const T* r, T* z,
                   double* scratch, hipStream_t s) {
    if (nrhs == 0) return;
    const int nx = L.E[0] * L.n, ny = L.E[1] * L.n, nz = L.E[2] * L.n;
    if (!scratch || nx > CMAX || ny > CMAX || nz > CMAX) {  // one work-group per right-hand side
        hipLaunchKernelGGL((k_coarse<T>), dim3(nrhs), dim3(1024), 0, s, C, nrhs, L.ndof, st, r, z);
        return;
    }
    double* g1 = scratch;
    double* g2 = scratch + (long long)nrhs * L.ndof;
    hipLaunchKernelGGL((k_coarse_xy_fwd<T>), dim3(nz, nrhs), dim3(256), 0, s, C, L.ndof, st, r, g1);
    hipLaunchKernelGGL(k_coarse_z, dim3((nx * ny + 15) / 16, nrhs), dim3(256), 0, s, C, L.ndof, st, g1, g2);
    hipLaunchKernelGGL((k_coarse_xy_back<T>), dim3(nz, nrhs), dim3(256), 0, s, C, L.ndof, st, g2, z);
}
template void launch_coarse<double>(const CoarseDev*, const LevelHost&, int, const RhsState*, const double*, double*,
                                    double*, hipStream_t);
template void launch_coarse<float>(const CoarseDev*, const LevelHost&, int, const RhsState*, const float*, float*,
                                   double*, hipStream_t);

// ---------------------------------------------------------------------------
// pointwise kernels: grid (chunks, nrhs), 256 threads x 4 values per chunk

template <typename T, int N>
__device__ __forceinline__ T diag_at(const LevelDev<T>& L, int E0, int E1, int E2, long long q64) {
    constexpr int N3 = N * N * N;
    const int q = (int)q64;  // index within one right-hand side (< 2^31)
    const int e = q / N3, l = q - e * N3;
    const int ex = e % E0, ey = (e / E0) % E1, ez = e / (E0 * E1);
    const int i = l % N, j = (l / N) % N, k = l / (N * N);
    const int tx = etype(ex, E0), ty = etype(ey, E1), tz = etype(ez, E2);
    const T mx = L.ax[0].m[i], my = L.ax[1].m[j], mz = L.ax[2].m[k];
    return L.ax[0].Bd[tx][i] * my * mz + mx * L.ax[1].Bd[ty][j] * mz + mx * my * L.ax[2].Bd[tz][k];
}

// Inverse diagonal of a level's operator, one value per node (shared by every right-hand side).
template <int N>
__global__ __launch_bounds__(256) void k_dinv(const LevelDev<double>* __restrict__ L, int E0, int E1, int E2,
                                              long long ndof, double* __restrict__ d64, float* __restrict__ d32) {
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q >= ndof) return;
    const double d = 1.0 / diag_at<double, N>(*L, E0, E1, E2, q);
    d64[q] = d;
    d32[q] = (float)d;
}

void launch_dinv(const LevelHost& L, hipStream_t s) {
    const long long n = L.ndof;
    const dim3 grid((unsigned)((n + 255) / 256));
#define DG_DI(NN) \
    case NN: hipLaunchKernelGGL((k_dinv<NN>), grid, dim3(256), 0, s, L.dev64, L.E[0], L.E[1], L.E[2], n, L.dinv64, L.dinv32); break;
    switch (L.n) { DG_DI(2) DG_DI(3) DG_DI(4) DG_DI(5) DG_DI(6) DG_DI(7) DG_DI(8) }
#undef DG_DI
}

// The pointwise kernels below run on a grid (right-hand side, chunk of 1024 nodes) with the
// right-hand side fastest, so that the work-groups of one chunk follow each other and share
// its slice of the inverse-diagonal table in L2.
template <typename T>
const T* dinv_of(const LevelHost& L);
template <>
const double* dinv_of<double>(const LevelHost& L) { return L.dinv64; }
template <>
const float* dinv_of<float>(const LevelHost& L) { return L.dinv32; }

inline dim3 rhs_chunk_grid(long long ndof, int nrhs) {
    const int nc = chunks_of(ndof);
    if (nc > 65535) throw std::logic_error("field too large for the pointwise kernels' grid");
    return dim3((unsigned)nrhs, (unsigned)nc);
}

template <typename T>
__global__ __launch_bounds__(256) void k_cheb0(const T* __restrict__ dinv, long long ndof, const RhsState* st,
                                               const T* __restrict__ f, T* __restrict__ z, T c0) {
    const int rhs = blockIdx.x;
    if (st && !st[rhs].active) return;
    const long long base = (long long)rhs * ndof;
    const long long q0 = (long long)blockIdx.y * 1024 + threadIdx.x;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const long long q = q0 + v * 256;
        if (q < ndof) z[base + q] = c0 * f[base + q] * dinv[q];
    }
}

template <typename T>
void launch_cheb0(const LevelHost& L, const LevelDev<T>* dev, int nrhs, const RhsState* st, const T* f, T* z,
                  double c0, hipStream_t s) {
    (void)dev;
    if (nrhs == 0) return;
    hipLaunchKernelGGL((k_cheb0<T>), rhs_chunk_grid(L.ndof, nrhs), dim3(256), 0, s, dinv_of<T>(L), L.ndof, st, f, z,
                       (T)c0);
}
template void launch_cheb0<double>(const LevelHost&, const LevelDev<double>*, int, const RhsState*, const double*,
                                   double*, double, hipStream_t);
template void launch_cheb0<float>(const LevelHost&, const LevelDev<float>*, int, const RhsState*, const float*,
                                  float*, double, hipStream_t);

template <typename T>
__global__ __launch_bounds__(256) void k_update(const T* __restrict__ dinv, long long ndof, const RhsState* st,
                                                T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p,
                                                const T* __restrict__ q_, T* __restrict__ z1, T c0,
                                                double* __restrict__ partial, int pstride) {
    __shared__ double red[4];
    const int rhs = blockIdx.x;
    if (!st[rhs].active) return;
    const T alpha = (T)st[rhs].alpha;
    const long long base = (long long)rhs * ndof;
    const long long q0 = (long long)blockIdx.y * 1024 + threadIdx.x;
    double acc = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const long long q = q0 + v * 256;
        if (q < ndof) {
            const long long g = base + q;
            x[g] += alpha * p[g];
            const T rn = r[g] - alpha * q_[g];
            r[g] = rn;
            acc += (double)rn * (double)rn;
            if (z1) z1[g] = c0 * rn * dinv[q];
        }
    }
    const double s = block_sum<256>(acc, red);
    if (threadIdx.x == 0) partial[(long long)rhs * pstride + blockIdx.y] = s;
}

template <typename T>
void launch_update(const LevelHost& L, const LevelDev<T>* dev, int nrhs, const RhsState* st, T* x, T* r, const T* p,
                   const T* q, T* z1, double c0, double* partial, int pstride, hipStream_t s) {
    (void)dev;
    if (nrhs == 0) return;
    hipLaunchKernelGGL((k_update<T>), rhs_chunk_grid(L.ndof, nrhs), dim3(256), 0, s, dinv_of<T>(L), L.ndof, st, x, r,
                       p, q, z1, (T)c0, partial, pstride);
}
template void launch_update<double>(const LevelHost&, const LevelDev<double>*, int, const RhsState*, double*, double*,
                                    const double*, const double*, double*, double, double*, int, hipStream_t);
template void launch_update<float>(const LevelHost&, const LevelDev<float>*, int, const RhsState*, float*, float*,
                                   const float*, const float*, float*, double, double*, int, hipStream_t);

template <typename TO, typename TP>
__global__ __launch_bounds__(256) void k_update_pc(const double* __restrict__ dinv, long long ndof, const RhsState* st,
                                                   double* __restrict__ x, double* __restrict__ r,
                                                   const TP* __restrict__ p, const double* __restrict__ q_,
                                                   TO* __restrict__ r32, TO* __restrict__ z1, double c0,
                                                   double* __restrict__ partial, int pstride) {
    __shared__ double red[4];
    const int rhs = blockIdx.x;
    if (!st[rhs].active) return;
    const double alpha = st[rhs].alpha;
    const long long base = (long long)rhs * ndof;
    const long long q0 = (long long)blockIdx.y * 1024 + threadIdx.x;
    double acc = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const long long q = q0 + v * 256;
        if (q < ndof) {
            const long long g = base + q;
            x[g] += alpha * (double)p[g];
            const double rn = r[g] - alpha * q_[g];
            r[g] = rn;
            acc += rn * rn;
            if constexpr (std::is_same<TO, __bf16>::value) {
                r32[g] = to_bf16((float)rn);
                z1[g] = to_bf16((float)(c0 * rn * dinv[q]));
            } else {
                r32[g] = (float)rn;
                z1[g] = (float)(c0 * rn * dinv[q]);
            }
        }
    }
    const double s = block_sum<256>(acc, red);
    if (threadIdx.x == 0) partial[(long long)rhs * pstride + blockIdx.y] = s;
}

template <typename TO>
__global__ __launch_bounds__(256) void k_to32_cheb0(const double* __restrict__ dinv, long long ndof,
                                                    const RhsState* st, const double* __restrict__ r,
                                                    TO* __restrict__ r32, TO* __restrict__ z1, double c0) {
    const int rhs = blockIdx.x;
    if (st && !st[rhs].active) return;
    const long long base = (long long)rhs * ndof;
    const long long q0 = (long long)blockIdx.y * 1024 + threadIdx.x;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const long long q = q0 + v * 256;
        if (q < ndof) {
            const double rv = r[base + q];
            if constexpr (std::is_same<TO, __bf16>::value) {
                r32[base + q] = to_bf16((float)rv);
                z1[base + q] = to_bf16((float)(c0 * rv * dinv[q]));
            } else {
                r32[base + q] = (float)rv;
                z1[base + q] = (float)(c0 * rv * dinv[q]);
            }
        }
    }
}

void launch_update_pc(const LevelHost& L, const LevelDev<double>* dev, int nrhs, const RhsState* st, double* x,
                      double* r, const double* p, const double* q, float* r32, float* z1, double c0, double* partial,
                      int pstride, hipStream_t s, bool bf16) {
    (void)dev;
    if (nrhs == 0) return;
    if (bf16)  // BF16 fields; the search direction is stored in FP32 (the BF16-input BM_PQ32 step writes it)
        hipLaunchKernelGGL((k_update_pc<__bf16, float>), rhs_chunk_grid(L.ndof, nrhs), dim3(256), 0, s, L.dinv64, L.ndof,
                           st, x, r, reinterpret_cast<const float*>(p), q, reinterpret_cast<__bf16*>(r32),
                           reinterpret_cast<__bf16*>(z1), c0, partial, pstride);
    else
        hipLaunchKernelGGL((k_update_pc<float, double>), rhs_chunk_grid(L.ndof, nrhs), dim3(256), 0, s, L.dinv64, L.ndof,
                           st, x, r, p, q, r32, z1, c0, partial, pstride);
}

void launch_to32_cheb0(const LevelHost& L, const LevelDev<double>* dev, int nrhs, const RhsState* st, const double* r,
                       float* r32, float* z1, double c0, hipStream_t s, bool bf16) {
    (void)dev;
    if (nrhs == 0) return;
    if (bf16)
        hipLaunchKernelGGL(k_to32_cheb0<__bf16>, rhs_chunk_grid(L.ndof, nrhs), dim3(256), 0, s, L.dinv64, L.ndof, st,
                           r, reinterpret_cast<__bf16*>(r32), reinterpret_cast<__bf16*>(z1), c0);
    else
        hipLaunchKernelGGL(k_to32_cheb0<float>, rhs_chunk_grid(L.ndof, nrhs), dim3(256), 0, s, L.dinv64, L.ndof, st,
                           r, r32, z1, c0);
}

template <typename TA, typename TB>
__global__ __launch_bounds__(256) void k_dot(long long ndof, const RhsState* st, const TA* __restrict__ a,
                                             const TB* __restrict__ b, double* __restrict__ partial, int pstride) {
    __shared__ double red[4];
    const int rhs = blockIdx.y;
    if (st && !st[rhs].active) return;
    const long long base = (long long)rhs * ndof;
    const long long q0 = (long long)blockIdx.x * 1024 + threadIdx.x;
    double acc = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const long long q = q0 + v * 256;
        if (q < ndof) acc += (double)a[base + q] * (double)b[base + q];
    }
    const double s = block_sum<256>(acc, red);
    if (threadIdx.x == 0) partial[(long long)rhs * pstride + blockIdx.x] = s;
}

template <typename TA, typename TB>
void launch_dot(long long ndof, int nrhs, const RhsState* st, const TA* a, const TB* b, double* partial, int pstride,
                hipStream_t s) {
    if (nrhs == 0) return;
    dim3 grid(chunks_of(ndof), nrhs);
    hipLaunchKernelGGL((k_dot<TA, TB>), grid, dim3(256), 0, s, ndof, st, a, b, partial, pstride);
}
template void launch_dot<double, double>(long long, int, const RhsState*, const double*, const double*, double*, int,
                                         hipStream_t);
template void launch_dot<float, float>(long long, int, const RhsState*, const float*, const float*, double*, int,
                                       hipStream_t);

__global__ __launch_bounds__(256) void k_finalize(int what, RhsState* st, const double* __restrict__ partial,
                                                  int pstride, int nblk) {
    __shared__ double red[256];
    const int rhs = blockIdx.x;
    RhsState& S = st[rhs];
    const bool gated = (what == FIN_RZ || what == FIN_PQ || what == FIN_RR || what == FIN_FLEX || what == FIN_RZ0 ||
                        what == FIN_CR || what == FIN_CAC);
    if (gated && !S.active) return;
    double acc = 0.0;
    const double* p = partial + (long long)rhs * pstride;
    for (int i = threadIdx.x; i < nblk; i += 256) acc += p[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double s = red[0];
    switch (what) {
        case FIN_BB: S.bb = s; break;
        case FIN_RR0:
            S.rr = s;
            S.iters = 0;
            S.breakdown = 0;
            S.active = (s > S.tol2 * S.bb) && S.maxit > 0 ? 1 : 0;
            break;
        case FIN_RZ:
            S.beta = (S.iters == 0) ? 0.0 : s / S.rz_old;
            S.rz_prev = S.rz_old;
            S.rz = s;
            S.rz_old = s;
            break;
        case FIN_FLEX:
            S.beta = (S.iters == 0) ? 0.0 : (S.rz - s) / S.rz_prev;
            break;
        case FIN_RZ0:
            S.beta = 0.0;
            S.rz_prev = S.rz_old;
            S.rz = s;
            S.rz_old = s;
            break;
        case FIN_CR: S.cr = s; break;
        case FIN_CAC: S.cac = s; break;
        case FIN_PQ:
            S.pq = s;
            if (!(s > 0.0) || !(S.rz > 0.0)) {
                S.breakdown = 1;
                S.active = 0;
            } else {
                S.alpha = S.rz / s;
            }
            break;
        case FIN_RR:
            S.rr = s;
            S.iters += 1;
            S.active = (s > S.tol2 * S.bb && S.iters < S.maxit) ? 1 : 0;
            break;
        case FIN_TRUE: S.rr = s; break;
        case FIN_OUTER:
            S.rr = s;
            S.scale = sqrt(s);
            S.active = (s > S.tol2 * S.bb) ? 1 : 0;
            break;
    }
}

__global__ __launch_bounds__(256) void k_guard_state(int nrhs, RhsState* st, int outer, int drop_all) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nrhs) return;
    RhsState& S = st[i];
    S.guess = (!drop_all && S.bb > 0.0 && S.rr < S.bb) ? 1 : 0;
    if (S.guess) return;
    S.rr = S.bb;
    if (outer) {
        S.scale = sqrt(S.bb);
        S.active = (S.bb > S.tol2 * S.bb) ? 1 : 0;
    }
}

__global__ __launch_bounds__(256) void k_guard_fields(long long n, const RhsState* st, const double* __restrict__ b,
                                                      double* __restrict__ x, double* __restrict__ r) {
    const int rhs = blockIdx.y;
    if (st[rhs].guess) return;
    const long long base = (long long)rhs * n;
    const long long q0 = (long long)blockIdx.x * 1024 + threadIdx.x;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const long long q = q0 + v * 256;
        if (q < n) {
            x[base + q] = 0.0;
            r[base + q] = b[base + q];
        }
    }
}

void launch_guard(int nrhs, long long n, RhsState* st, const double* b, double* x, double* r, bool outer,
                  bool drop_all, hipStream_t s) {
    if (nrhs == 0) return;
    hipLaunchKernelGGL(k_guard_state, dim3((nrhs + 255) / 256), dim3(256), 0, s, nrhs, st, outer ? 1 : 0,
                       drop_all ? 1 : 0);
    hipLaunchKernelGGL(k_guard_fields, dim3(chunks_of(n), nrhs), dim3(256), 0, s, n, st, b, x, r);
}

void launch_finalize(int what, int nrhs, RhsState* st, const double* partial, int pstride, int nblk, hipStream_t s) {
    if (nrhs == 0) return;
    hipLaunchKernelGGL(k_finalize, dim3(nrhs), dim3(256), 0, s, what, st, partial, pstride, nblk);
}

__global__ __launch_bounds__(256) void k_gate(int nrhs, RhsState* st, const RhsState* gate) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < nrhs && !gate[i].active) st[i].active = 0;
}

void launch_gate(int nrhs, RhsState* st, const RhsState* gate, hipStream_t s) {
    if (nrhs == 0) return;
    hipLaunchKernelGGL(k_gate, dim3((nrhs + 255) / 256), dim3(256), 0, s, nrhs, st, gate);
}

__global__ __launch_bounds__(256) void k_inner_init(int nrhs, const RhsState* outer, RhsState* inner, double rtol,
                                                    double inner_rtol, int maxit) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nrhs) return;
    const RhsState O = outer[i];
    const double need = O.rr > 0 ? 0.9 * rtol * sqrt(O.bb / O.rr) : 1.0;
    const double tin = fmin(0.5, fmax(inner_rtol, need));
    RhsState S{};
    S.tol2 = tin * tin;
    S.maxit = maxit;
    S.active = O.active;
    S.bb = 1.0;
    S.scale = 1.0;
    inner[i] = S;
}

void launch_inner_init(int nrhs, const RhsState* outer, RhsState* inner, double rtol, double inner_rtol, int maxit,
                       hipStream_t s) {
    if (nrhs == 0) return;
    hipLaunchKernelGGL(k_inner_init, dim3((nrhs + 255) / 256), dim3(256), 0, s, nrhs, outer, inner, rtol, inner_rtol,
                       maxit);
}

// ---------------------------------------------------------------------------
// right-hand side: b = 4 pi M rho + lift(g)

template <int N>
__global__ __launch_bounds__(256) void k_rhs(const LevelDev<double>* __restrict__ L, int E0, int E1, int E2,
                                             long long ndof, const double* __restrict__ rho,
                                             const double* __restrict__ phi, const int* __restrict__ pi,
                                             const int* __restrict__ pj, const double* __restrict__ g, long long nface,
                                             double* __restrict__ b) {
    constexpr int N3 = N * N * N;
    const int rhs = blockIdx.y;
    const long long base = (long long)rhs * ndof;
    const int NX = E0 * N, NY = E1 * N, NZ = E2 * N;
    const long long ox = 0, oxp = (long long)NZ * NY, oy = 2LL * NZ * NY, oyp = oy + (long long)NZ * NX,
                    oz = oy + 2LL * NZ * NX, ozp = oz + (long long)NY * NX;
    const double* gg = g + (long long)rhs * nface;
    const long long q0 = (long long)blockIdx.x * 1024 + threadIdx.x;
    const double* ph_i = phi ? phi + (long long)pi[rhs] * ndof : nullptr;
    const double* ph_j = phi ? phi + (long long)pj[rhs] * ndof : nullptr;
    const AxisDev<double>& ax = L->ax[0];
    const AxisDev<double>& ay = L->ax[1];
    const AxisDev<double>& az = L->ax[2];
    for (int v = 0; v < 4; ++v) {
        const long long q = q0 + v * 256;
        if (q >= ndof) break;
        const int qi = (int)q;
        const int e = qi / N3, l = qi - e * N3;
        const int ex = e % E0, ey = (e / E0) % E1, ez = e / (E0 * E1);
        const int i = l % N, j = (l / N) % N, k = l / (N * N);
        const int X = ex * N + i, Y = ey * N + j, Z = ez * N + k;
        const double src = phi ? ph_i[q] * ph_j[q] : rho[base + q];
        const double mx = ax.m[i], my = ay.m[j], mz = az.m[k];
        double val = 4.0 * M_PI * mx * my * mz * src;
        if (ex == 0) val += ax.liftL[i] * my * mz * gg[ox + (long long)Z * NY + Y];
        if (ex == E0 - 1) val += ax.liftR[i] * my * mz * gg[oxp + (long long)Z * NY + Y];
        if (ey == 0) val += ay.liftL[j] * mx * mz * gg[oy + (long long)Z * NX + X];
        if (ey == E1 - 1) val += ay.liftR[j] * mx * mz * gg[oyp + (long long)Z * NX + X];
        if (ez == 0) val += az.liftL[k] * mx * my * gg[oz + (long long)Y * NX + X];
        if (ez == E2 - 1) val += az.liftR[k] * mx * my * gg[ozp + (long long)Y * NX + X];
        b[base + q] = val;
    }
}

void launch_rhs(const LevelHost& L, const LevelDev<double>* dev, int nrhs, const double* rho, const double* phi,
                const int* pi, const int* pj, const double* g, long long nface, double* b, hipStream_t s) {
    if (nrhs == 0) return;
    dim3 grid(chunks_of(L.ndof), nrhs);
#define DG_RHS(NN)                                                                                               \
    case NN:                                                                                                     \
        hipLaunchKernelGGL((k_rhs<NN>), grid, dim3(256), 0, s, dev, L.E[0], L.E[1], L.E[2], L.ndof, rho, phi, pi, \
                           pj, g, nface, b);                                                                     \
        break;
    switch (L.n) { DG_RHS(2) DG_RHS(3) DG_RHS(4) DG_RHS(5) DG_RHS(6) DG_RHS(7) DG_RHS(8) }
#undef DG_RHS
}

// ---------------------------------------------------------------------------
// iterative refinement conversions and helpers

__global__ __launch_bounds__(256) void k_to_inner(long long ndof, const RhsState* st, const double* __restrict__ r64,
                                                  float* __restrict__ r32) {
    const int rhs = blockIdx.y;
    if (!st[rhs].active) return;
    const double inv = 1.0 / st[rhs].scale;
    const long long base = (long long)rhs * ndof;
    const long long q0 = (long long)blockIdx.x * 1024 + threadIdx.x;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const long long q = q0 + v * 256;
        if (q < ndof) r32[base + q] = (float)(r64[base + q] * inv);
    }
}

__global__ __launch_bounds__(256) void k_correct(long long ndof, const RhsState* st, const float* __restrict__ d32,
                                                 double* __restrict__ x64) {
    const int rhs = blockIdx.y;
    if (!st[rhs].active) return;
    const double sc = st[rhs].scale;
    const long long base = (long long)rhs * ndof;
    const long long q0 = (long long)blockIdx.x * 1024 + threadIdx.x;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const long long q = q0 + v * 256;
        if (q < ndof) x64[base + q] += sc * (double)d32[base + q];
    }
}

void launch_to_inner(long long ndof, int nrhs, const RhsState* st, const double* r64, float* r32, hipStream_t s) {
    if (nrhs == 0) return;
    hipLaunchKernelGGL(k_to_inner, dim3(chunks_of(ndof), nrhs), dim3(256), 0, s, ndof, st, r64, r32);
}
void launch_correct(long long ndof, int nrhs, const RhsState* st, const float* d32, double* x64, hipStream_t s) {
    if (nrhs == 0) return;
    hipLaunchKernelGGL(k_correct, dim3(chunks_of(ndof), nrhs), dim3(256), 0, s, ndof, st, d32, x64);
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill(T* x, T v, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) x[i] = v;
}
template <typename T>
void launch_fill(T* x, T v, long long n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL((k_fill<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, v, n);
}
template void launch_fill<double>(double*, double, long long, hipStream_t);
template void launch_fill<float>(float*, float, long long, hipStream_t);
template void launch_fill<unsigned>(unsigned*, unsigned, long long, hipStream_t);

__global__ __launch_bounds__(256) void k_segcopy(const double* __restrict__ src, const long long* __restrict__ soff,
                                                  double* __restrict__ dst, const long long* __restrict__ doff,
                                                  long long len) {
    const double* a = src + soff[blockIdx.y];
    double* b = dst + doff[blockIdx.y];
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < len; i += (long long)gridDim.x * 256) b[i] = a[i];
}

void launch_segcopy(const double* src, const long long* soff, double* dst, const long long* doff, long long len,
                    int nseg, hipStream_t s) {
    if (nseg <= 0 || len <= 0) return;
    const int gx = (int)std::min<long long>((len + 255) / 256, 256);
    hipLaunchKernelGGL(k_segcopy, dim3(gx, nseg), dim3(256), 0, s, src, soff, dst, doff, len);
}

__global__ __launch_bounds__(256) void k_copy(const double* __restrict__ a, double* __restrict__ b, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) b[i] = a[i];
}
void launch_copy(const double* a, double* b, long long n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, b, n);
}

template <int N>
__global__ __launch_bounds__(256) void k_dscale(const LevelDev<double>* __restrict__ L, int E0, int E1, int E2,
                                                long long ndof, const double* __restrict__ x, double* __restrict__ y) {
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q < ndof) y[q] = x[q] / sqrt(diag_at<double, N>(*L, E0, E1, E2, q));
}
void launch_dscale(const LevelHost& L, const LevelDev<double>* dev, const double* x, double* y, hipStream_t s) {
    const unsigned grid = (unsigned)((L.ndof + 255) / 256);
#define DG_DS(NN) \
    case NN: hipLaunchKernelGGL((k_dscale<NN>), dim3(grid), dim3(256), 0, s, dev, L.E[0], L.E[1], L.E[2], L.ndof, x, y); break;
    switch (L.n) { DG_DS(2) DG_DS(3) DG_DS(4) DG_DS(5) DG_DS(6) DG_DS(7) DG_DS(8) }
#undef DG_DS
}

__global__ __launch_bounds__(256) void k_axpby(long long n, double a, const double* __restrict__ x, double b,
                                               double* __restrict__ y) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) y[i] = a * x[i] + b * y[i];
}
void launch_axpby(long long n, double a, const double* x, double b, double* y, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_axpby, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, a, x, b, y);
}

template <int N>
__global__ __launch_bounds__(256) void k_source_of(const LevelDev<double>* __restrict__ L, long long ndof, long long n,
                                                   const double* __restrict__ r, double* __restrict__ rho) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int l = (int)((i % ndof) % (N * N * N));  // node within its element (the mass is element-local)
    const double m = L->ax[0].m[l % N] * L->ax[1].m[(l / N) % N] * L->ax[2].m[l / (N * N)];
    rho[i] = r[i] / (4.0 * M_PI * m);
}
__global__ __launch_bounds__(256) void k_lcgc_scale(long long ndof, const RhsState* st, const double* __restrict__ r,
                                                    double* __restrict__ c, double* __restrict__ q) {
    const int rhs = blockIdx.x;
    if (!st[rhs].active) return;
    const double cac = st[rhs].cac;
    const double g = cac > 0.0 ? st[rhs].cr / cac : 0.0;
    const long long base = (long long)rhs * ndof;
    const long long q0 = (long long)blockIdx.y * 1024 + threadIdx.x;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const long long i = q0 + v * 256;
        if (i < ndof) {
            c[base + i] *= g;
            q[base + i] = r[base + i] - g * q[base + i];
        }
    }
}
void launch_lcgc_scale(long long ndof, int nrhs, const RhsState* st, const double* r, double* c, double* q,
                       hipStream_t s) {
    if (nrhs == 0) return;
    hipLaunchKernelGGL(k_lcgc_scale, rhs_chunk_grid(ndof, nrhs), dim3(256), 0, s, ndof, st, r, c, q);
}

void launch_source_of(const LevelHost& L, const LevelDev<double>* dev, int nrhs, const double* r, double* rho,
                      hipStream_t s) {
    const long long n = L.ndof * nrhs;
    if (n <= 0) return;
    const unsigned grid = (unsigned)((n + 255) / 256);
#define DG_SO(NN) \
    case NN: hipLaunchKernelGGL((k_source_of<NN>), dim3(grid), dim3(256), 0, s, dev, L.ndof, n, r, rho); break;
    switch (L.n) { DG_SO(2) DG_SO(3) DG_SO(4) DG_SO(5) DG_SO(6) DG_SO(7) DG_SO(8) }
#undef DG_SO
}

// ---------------------------------------------------------------------------
// exchange: W_k = sum_s phi_s v_ks and partial sums of w_node rho_ij v_ij

constexpr int XMAX_ORB = 32;

template <int N>
__global__ __launch_bounds__(256) void k_exchange(const LevelDev<double>* __restrict__ L, int E0, int E1, int E2,
                                                  long long ndof, int norb, const double* __restrict__ phi,
                                                  const double* __restrict__ v, double* __restrict__ W,
                                                  double* __restrict__ partial, int pstride) {
    constexpr int N3 = N * N * N;
    __shared__ double red[4];
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    const bool ok = q < ndof;
    double ph[XMAX_ORB], w[XMAX_ORB];
    double wq = 0.0;
    if (ok) {
        const int l = (int)q % N3;
        const int i = l % N, j = (l / N) % N, k = l / (N * N);
        wq = L->ax[0].m[i] * L->ax[1].m[j] * L->ax[2].m[k];
    }
    for (int a = 0; a < norb; ++a) {
        ph[a] = ok ? phi[(long long)a * ndof + q] : 0.0;
        w[a] = 0.0;
    }
    int pidx = 0;
    for (int a = 0; a < norb; ++a) {
        for (int b = a; b < norb; ++b, ++pidx) {
            const double vv = ok ? v[(long long)pidx * ndof + q] : 0.0;
            w[a] += ph[b] * vv;
            if (b != a) w[b] += ph[a] * vv;
            const double s = block_sum<256>(wq * ph[a] * ph[b] * vv, red);
            if (threadIdx.x == 0) partial[(long long)pidx * pstride + blockIdx.x] = s;
            __syncthreads();
        }
    }
    if (ok)
        for (int a = 0; a < norb; ++a) W[(long long)a * ndof + q] = w[a];
}

// The same for a compile-time orbital count: orbital values and W sums in registers (the
// run-time count above keeps them in scratch memory), one wave reduction per pair and a
// single barrier per work-group for all pair partial sums.  Used for 8 orbitals at p = 4;
// 16 orbitals would need more registers than a lane has.
template <int N, int NORB>
__global__ __launch_bounds__(256) void k_exchange_n(const LevelDev<double>* __restrict__ L, long long ndof,
                                                    const double* __restrict__ phi, const double* __restrict__ v,
                                                    double* __restrict__ W, double* __restrict__ partial,
                                                    int pstride) {
    constexpr int N3 = N * N * N, NPAIR = NORB * (NORB + 1) / 2;
    __shared__ double red[4][NPAIR];
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    const bool ok = q < ndof;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double ph[NORB], w[NORB];
    double wq = 0.0;
    if (ok) {
        const int l = (int)(q % N3);
        const int i = l % N, j = (l / N) % N, k = l / (N * N);
        wq = L->ax[0].m[i] * L->ax[1].m[j] * L->ax[2].m[k];
    }
#pragma unroll
    for (int a = 0; a < NORB; ++a) {
        ph[a] = ok ? phi[(long long)a * ndof + q] : 0.0;
        w[a] = 0.0;
    }
#pragma unroll
    for (int a = 0; a < NORB; ++a) {
#pragma unroll
        for (int b = a; b < NORB; ++b) {
            const int pidx = a * NORB - a * (a - 1) / 2 + (b - a);
            const double vv = ok ? v[(long long)pidx * ndof + q] : 0.0;
            w[a] += ph[b] * vv;
            if (b != a) w[b] += ph[a] * vv;
            double kv = wq * ph[a] * ph[b] * vv;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) kv += __shfl_xor(kv, off, 64);
            if (lane == 0) red[wave][pidx] = kv;
        }
    }
    __syncthreads();
    for (int p = threadIdx.x; p < NPAIR; p += 256)
        partial[(long long)p * pstride + blockIdx.x] = (red[0][p] + red[1][p]) + (red[2][p] + red[3][p]);
    if (ok) {
#pragma unroll
        for (int a = 0; a < NORB; ++a) W[(long long)a * ndof + q] = w[a];
    }
}

void launch_exchange(const LevelHost& L, const LevelDev<double>* dev, int norb, const double* phi, const double* v,
                     double* W, double* partial, int pstride, hipStream_t s) {
    const unsigned grid = (unsigned)((L.ndof + 255) / 256);
    if (L.n == 5 && norb == 8) {
        hipLaunchKernelGGL((k_exchange_n<5, 8>), dim3(grid), dim3(256), 0, s, dev, L.ndof, phi, v, W, partial,
                           pstride);
        return;
    }

#define DG_X(NN)                                                                                                   \
    case NN:                                                                                                       \
        hipLaunchKernelGGL((k_exchange<NN>), dim3(grid), dim3(256), 0, s, dev, L.E[0], L.E[1], L.E[2], L.ndof, norb, \
                           phi, v, W, partial, pstride);                                                           \
        break;
    switch (L.n) { DG_X(2) DG_X(3) DG_X(4) DG_X(5) DG_X(6) DG_X(7) DG_X(8) }
#undef DG_X
}

__global__ __launch_bounds__(256) void k_pair_products(long long ndof, const double* __restrict__ phi,
                                                       const int* __restrict__ pi, const int* __restrict__ pj,
                                                       double* __restrict__ rho) {
    const int q = blockIdx.y;
    const double* a = phi + (long long)pi[q] * ndof;
    const double* b = phi + (long long)pj[q] * ndof;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < ndof; i += (long long)gridDim.x * 256)
        rho[(long long)q * ndof + i] = a[i] * b[i];
}
void launch_pair_products(long long ndof, int npairs, const double* phi, const int* pi, const int* pj, double* rho,
                          hipStream_t s) {
    if (npairs == 0) return;
    hipLaunchKernelGGL(k_pair_products, dim3(256, npairs), dim3(256), 0, s, ndof, phi, pi, pj, rho);
}

// rho[q - first] = phi_i phi_j for the pairs q = first .. first + count - 1 of norb orbitals, pair q = (i, j),
// i <= j, in row-major order: q = i norb - i (i - 1) / 2 + (j - i).
__global__ __launch_bounds__(256) void k_pair_densities(long long ndof, int norb, int first,
                                                        const double* __restrict__ phi, double* __restrict__ rho) {
    const int qo = blockIdx.y;
    int q = first + qo, i = 0;
    while (q >= norb - i) {  // row i holds the norb - i pairs (i, i..norb-1)
        q -= norb - i;
        ++i;
    }
    const int j = i + q;
    const double* a = phi + (long long)i * ndof;
    const double* b = phi + (long long)j * ndof;
    double* out = rho + (long long)qo * ndof;
    for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < ndof; k += (long long)gridDim.x * 256)
        out[k] = a[k] * b[k];
}
void launch_pair_densities(long long ndof, int norb, int first, int count, const double* phi, double* rho,
                           hipStream_t s) {
    if (count <= 0 || ndof <= 0) return;
    const long long blocks = std::min<long long>(1024, (ndof + 255) / 256);
    hipLaunchKernelGGL(k_pair_densities, dim3((unsigned)blocks, count), dim3(256), 0, s, ndof, norb, first, phi, rho);
}

__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ partial, int pstride, int nblk,
                                                      double* __restrict__ K) {
    __shared__ double red[256];
    const int qd = blockIdx.x;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nblk; i += 256) acc += partial[(long long)qd * pstride + i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) K[qd] = red[0];
}
void launch_sum_partials(int nq, const double* partial, int pstride, int nblk, double* K, hipStream_t s) {
    if (nq == 0) return;
    hipLaunchKernelGGL(k_sum_partials, dim3(nq), dim3(256), 0, s, partial, pstride, nblk, K);
}

// ---------------------------------------------------------------------------
// Fused solve of small meshes: one work-group per right-hand side runs the whole PCG and its
// V-cycle.  Level fields live in the right-hand side's work space (global memory, L2-resident
// at these sizes); the operand of every operator application and the intermediate arrays of the
// transfers are staged in two LDS arrays of FUSED_MAX_DOF doubles.  Work-group barriers separate
// the phases; there is no grid-wide synchronisation, so right-hand sides of different sizes and
// iteration counts need nothing from each other.

namespace {

// The work-group's view of its LDS: in resident mode every level field lives in LDS for the whole
// solve (offsets FusedLevel::lf/lza/lzb); otherwise the fields live in the right-hand side's
// work space and the operand of each operator application is staged into su.  sy receives the
// operator's output; g and Qs are the coarsest solve's scratch; red the reduction slots.
struct WgCtx {
    double* lds;
    double* su;
    double* sy;
    double* g;
    double* Qs;
    double* red;
    bool resident;
};

// Sum over the work-group, the same value (added in a fixed order) in every thread.
__device__ __forceinline__ double wg_sum(double v, double* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();  // red may still be read by the previous sum
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < FUSED_THREADS / 64; ++i) s += red[i];
    return s;
}

__device__ __forceinline__ void wg_copy(const double* __restrict__ src, double* __restrict__ dst, int n) {
#pragma unroll 8
    for (int q = threadIdx.x; q < n; q += FUSED_THREADS) dst[q] = src[q];
    __syncthreads();
}

// A field as an operator operand in LDS: itself in resident mode, else staged into su.
__device__ __forceinline__ const double* wg_operand(const WgCtx& w, const double* g, int n) {
    if (w.resident) return g;
    wg_copy(g, w.su, n);
    return w.su;
}

// Element-major index of the level node with global indices (X, Y, Z).
__device__ __forceinline__ int em_index(const FusedLevel& F, int X, int Y, int Z) {
    const int n = F.n;
    const int ex = X / n, i = X - ex * n, ey = Y / n, j = Y - ey * n, ez = Z / n, k = Z - ez * n;
    return ((ez * F.E[1] + ey) * F.E[0] + ex) * n * n * n + (k * n + j) * n + i;
}

// sy = A su on level F (element-major), axis by axis: one thread per element line computes the
// line's N outputs with the reference-element block shared by every element and axis (the slab
// kernel's elem_op): the neighbours along the axis supply their face value and normal
// derivative, and a domain face supplies ghost data that reproduces its Nitsche terms.  The
// output is scaled by the axis factor and the two tangential GLL weights.
template <int N>
__device__ void wg_apply_n(const FusedLevel& F, const double* su, double* sy) {
    constexpr int N2 = N * N, N3 = N2 * N;
    const RefDev<double>& R = F.L->ref;
    SlabCoef<double, N> c;
    load_coef(c, R);
    const int E0 = F.E[0], E1 = F.E[1];
    const int nlines = F.ndof / N;
#pragma unroll 1
    for (int axis = 0; axis < 3; ++axis) {
        const int Ed = F.E[axis];
        const int s_in = axis == 0 ? 1 : (axis == 1 ? N : N2);
        const int s_el = axis == 0 ? N3 : (axis == 1 ? E0 * N3 : E0 * E1 * N3);
        const double sca = R.scale[axis];
        for (int t = threadIdx.x; t < nlines; t += FUSED_THREADS) {
            const int e = t / N2, ln = t - e * N2;
            const int a = ln % N, b = ln / N;  // the other two local indices, lower axis first
            int off, ed;
            if (axis == 0) {
                off = a * N + b * N2;
                ed = e % E0;
            } else if (axis == 1) {
                off = a + b * N2;
                ed = (e / E0) % E1;
            } else {
                off = a + b * N;
                ed = e / (E0 * E1);
            }
            const int base = e * N3 + off;
            double A[N], nb[N], acc[N];
#pragma unroll
            for (int l = 0; l < N; ++l) A[l] = su[base + l * s_in];
            double U, Dv, U0, D0;
            if (ed > 0) {
#pragma unroll
                for (int l = 0; l < N; ++l) nb[l] = su[base - s_el + l * s_in];
                U = nb[N - 1];
                Dv = face_r(c, nb);
            } else {
                U = -A[0];
                Dv = face_l(c, A) - 2.0 * c.sig * A[0];
            }
            if (ed < Ed - 1) {
#pragma unroll
                for (int l = 0; l < N; ++l) nb[l] = su[base + s_el + l * s_in];
                U0 = nb[0];
                D0 = face_l(c, nb);
            } else {
                U0 = -A[N - 1];
                D0 = face_r(c, A) + 2.0 * c.sig * A[N - 1];
            }
            elem_op(c, A, U, Dv, U0, D0, acc);
            const double sc = sca * R.w[a] * R.w[b];
#pragma unroll
            for (int i = 0; i < N; ++i) {
                if (axis == 0)
                    sy[base + i * s_in] = acc[i] * sc;
                else
                    sy[base + i * s_in] += acc[i] * sc;
            }
        }
        __syncthreads();
    }
}

__device__ void wg_apply(const FusedLevel& F, const double* su, double* sy) {
    switch (F.n) {
        case 2: wg_apply_n<2>(F, su, sy); break;
        case 3: wg_apply_n<3>(F, su, sy); break;
        case 4: wg_apply_n<4>(F, su, sy); break;
        case 5: wg_apply_n<5>(F, su, sy); break;
    }
}

// One Chebyshev step on level F: out = z + cp (z - zp) + cr D^-1 (f - A z); zp null: the previous
// iterate is zero (the second pre-smoothing step, whose recurrence starts from z = 0).
__device__ void wg_cheb(const WgCtx& w, const FusedLevel& F, const double* __restrict__ f, const double* z,
                        const double* __restrict__ zp, double* __restrict__ out, double cp, double cr) {
    const double* zin = wg_operand(w, z, F.ndof);
    wg_apply(F, zin, w.sy);
#pragma unroll 8
    for (int q = threadIdx.x; q < F.ndof; q += FUSED_THREADS) {
        const double zq = zin[q];
        out[q] = zq + cp * (zq - (zp ? zp[q] : 0.0)) + cr * F.dinv[q] * (f[q] - w.sy[q]);
    }
    __syncthreads();
}

// fc = P^T r from the fine level F to the coarse level C; r in w.sy (element-major), t1 a free
// array of F.ndof values.  With z1c, also z1c = C.c0 D_C^-1 fc (the coarse level's first iterate).
__device__ void wg_restrict(const WgCtx& w, const FusedLevel& F, const FusedLevel& C, double* t1, double* fc,
                            double* z1c) {
    const int NXf = F.N[0], NYf = F.N[1], NZf = F.N[2];
    const int NXc = C.N[0], NYc = C.N[1], NZc = C.N[2];
    const double *P0 = F.P[0], *P1 = F.P[1], *P2 = F.P[2];
    double* sy = w.sy;
    for (int o = threadIdx.x; o < NXc * NYf * NZf; o += FUSED_THREADS) {  // along x: (Xc, Yf, Zf)
        const int Xc = o % NXc, Yf = (o / NXc) % NYf, Zf = o / (NXc * NYf);
        const int lo = F.rlo[0][Xc], cnt = F.rcnt[0][Xc];
        double s = 0.0;
        for (int c = 0; c < cnt; ++c) s += P0[(lo + c) * NXc + Xc] * sy[em_index(F, lo + c, Yf, Zf)];
        t1[o] = s;
    }
    __syncthreads();
    for (int o = threadIdx.x; o < NXc * NYc * NZf; o += FUSED_THREADS) {  // along y: (Xc, Yc, Zf)
        const int Xc = o % NXc, Yc = (o / NXc) % NYc, Zf = o / (NXc * NYc);
        const int lo = F.rlo[1][Yc], cnt = F.rcnt[1][Yc];
        double s = 0.0;
        for (int c = 0; c < cnt; ++c) s += P1[(lo + c) * NYc + Yc] * t1[(Zf * NYf + lo + c) * NXc + Xc];
        sy[o] = s;
    }
    __syncthreads();
    const int n = C.n, n3 = n * n * n;
    for (int o = threadIdx.x; o < C.ndof; o += FUSED_THREADS) {  // along z, into the coarse field
        const int e = o / n3, l = o - e * n3;
        const int Xc = (e % C.E[0]) * n + l % n, Yc = ((e / C.E[0]) % C.E[1]) * n + (l / n) % n,
                  Zc = (e / (C.E[0] * C.E[1])) * n + l / (n * n);
        const int lo = F.rlo[2][Zc], cnt = F.rcnt[2][Zc];
        double s = 0.0;
        for (int c = 0; c < cnt; ++c) s += P2[(lo + c) * NZc + Zc] * sy[((lo + c) * NYc + Yc) * NXc + Xc];
        fc[o] = s;
        if (z1c) z1c[o] = C.c0 * C.dinv[o] * s;
    }
    __syncthreads();
}

// zf += P zc from the coarse level C to the fine level F (element-major); t1 a free array of F.ndof.
__device__ void wg_prolong_add(const WgCtx& w, const FusedLevel& F, const FusedLevel& C, const double* zc,
                               double* zf, double* t1) {
    const int NXf = F.N[0], NYf = F.N[1];
    const int NXc = C.N[0], NYc = C.N[1], NZc = C.N[2];
    const double *P0 = F.P[0], *P1 = F.P[1], *P2 = F.P[2];
    double* sy = w.sy;
    for (int o = threadIdx.x; o < NXf * NYc * NZc; o += FUSED_THREADS) {  // along x: (Xf, Yc, Zc)
        const int Xf = o % NXf, Yc = (o / NXf) % NYc, Zc = o / (NXf * NYc);
        const int lo = F.plo[0][Xf], cnt = F.pcnt[0][Xf];
        double s = 0.0;
        for (int c = 0; c < cnt; ++c) s += P0[Xf * NXc + lo + c] * zc[em_index(C, lo + c, Yc, Zc)];
        t1[o] = s;
    }
    __syncthreads();
    for (int o = threadIdx.x; o < NXf * NYf * NZc; o += FUSED_THREADS) {  // along y: (Xf, Yf, Zc)
        const int Xf = o % NXf, Yf = (o / NXf) % NYf, Zc = o / (NXf * NYf);
        const int lo = F.plo[1][Yf], cnt = F.pcnt[1][Yf];
        double s = 0.0;
        for (int c = 0; c < cnt; ++c) s += P1[Yf * NYc + lo + c] * t1[(Zc * NYc + lo + c) * NXf + Xf];
        sy[o] = s;
    }
    __syncthreads();
    const int n = F.n, n3 = n * n * n;
    for (int o = threadIdx.x; o < F.ndof; o += FUSED_THREADS) {  // along z, added to the fine field
        const int e = o / n3, l = o - e * n3;
        const int Xf = (e % F.E[0]) * n + l % n, Yf = ((e / F.E[0]) % F.E[1]) * n + (l / n) % n,
                  Zf = (e / (F.E[0] * F.E[1])) * n + l / (n * n);
        const int lo = F.plo[2][Zf], cnt = F.pcnt[2][Zf];
        double s = 0.0;
        for (int c = 0; c < cnt; ++c) s += P2[Zf * NZc + lo + c] * sy[((lo + c) * NYf + Yf) * NXf + Xf];
        zf[o] += s;
    }
    __syncthreads();
}

// Fields of a level: in LDS (resident) or in the right-hand side's work space.
__device__ __forceinline__ double* lvf(const WgCtx& w, double* ws, const FusedLevel& F, int which) {
    if (w.resident) return w.lds + (which == 0 ? F.lf : which == 1 ? F.lza : F.lzb);
    return ws + (which == 0 ? F.off_f : which == 1 ? F.off_za : F.off_zb);
}

// z = B r, one V-cycle from level 0 (r: the level-0 source, lvf(level 0, 0)); returns the field
// that holds z (one of the level-0 smoother fields).
__device__ double* wg_vcycle(const WgCtx& w, const FusedMeshDev& M, double* ws) {
    const int nl = M.nl;
    double* zcur[FUSED_MAX_LEVELS];
    double* zoth[FUSED_MAX_LEVELS];
    for (int l = 0; l + 1 < nl; ++l) {
        const FusedLevel& F = M.lv[l];
        const double* f = lvf(w, ws, F, 0);
        double* cur = lvf(w, ws, F, 1);
        double* prev = lvf(w, ws, F, 2);
        if (l == 0) {  // lower levels receive their first iterate from the restriction
#pragma unroll 8
            for (int q = threadIdx.x; q < F.ndof; q += FUSED_THREADS) cur[q] = F.c0 * F.dinv[q] * f[q];
            __syncthreads();
        }
        for (int k = 1; k < F.deg; ++k) {
            wg_cheb(w, F, f, cur, k == 1 ? nullptr : prev, prev, F.cp[k - 1], F.cr[k - 1]);
            double* t = cur; cur = prev; prev = t;
        }
        // residual into sy, restricted to the next level
        const double* zin = wg_operand(w, cur, F.ndof);
        wg_apply(F, zin, w.sy);
#pragma unroll 8
        for (int q = threadIdx.x; q < F.ndof; q += FUSED_THREADS) w.sy[q] = f[q] - w.sy[q];
        __syncthreads();
        const FusedLevel& C = M.lv[l + 1];
        wg_restrict(w, F, C, w.resident ? prev : w.su, lvf(w, ws, C, 0), l + 2 < nl ? lvf(w, ws, C, 1) : nullptr);
        zcur[l] = cur;
        zoth[l] = prev;
    }
    const FusedLevel& Lc = M.lv[nl - 1];
    double* zc = lvf(w, ws, Lc, 1);
    coarse_wg<double, 1024 / FUSED_THREADS>(M.coarse, Lc.ndof, lvf(w, ws, Lc, 0), zc, w.g,
                                            reinterpret_cast<double(*)[CMAX][CMAX]>(w.Qs));
    __syncthreads();
    for (int l = nl - 2; l >= 0; --l) {
        const FusedLevel& F = M.lv[l];
        const double* f = lvf(w, ws, F, 0);
        double* cur = zcur[l];
        double* prev = zoth[l];
        wg_prolong_add(w, F, M.lv[l + 1], zc, cur, w.resident ? prev : w.su);
        for (int k = 0; k < F.deg; ++k) {
            wg_cheb(w, F, f, cur, k == 0 ? nullptr : prev, prev, k == 0 ? 0.0 : F.cp[k - 1],
                    k == 0 ? F.c0 : F.cr[k - 1]);
            double* t = cur; cur = prev; prev = t;
        }
        zc = cur;
    }
    return zc;
}

__global__ __launch_bounds__(FUSED_THREADS) void k_fused_pcg(const FusedMeshDev* __restrict__ Mp, int nrhs,
                                                            const double* __restrict__ b_all,
                                                            double* __restrict__ x_all, RhsState* st,
                                                            double* __restrict__ ws_all, int has_x0, int guard) {
    __shared__ double lds[FUSED_LDS_DOUBLES];
    const FusedMeshDev& M = *Mp;
    WgCtx w;
    w.lds = lds;
    w.resident = M.resident != 0;
    w.red = lds + FUSED_LDS_DOUBLES - FUSED_THREADS / 64;
    if (w.resident) {
        w.su = nullptr;
        w.sy = lds + M.lsy;
        w.g = lds + M.lsy;
    } else {
        w.su = lds;
        w.sy = lds + FUSED_MAX_DOF;
        w.g = lds;
    }
    w.Qs = w.g + CMAX * CSZ;
    const int rhs = blockIdx.x;
    const FusedLevel& F0 = M.lv[0];
    const int nd = F0.ndof;
    const double* __restrict__ b = b_all + (long long)rhs * nd;
    double* __restrict__ x = x_all + (long long)rhs * nd;
    double* ws = ws_all + (long long)rhs * M.ws_per_rhs;
    double* r = lvf(w, ws, F0, 0);
    double* p = ws + M.off_p;
    const double tol2 = st[rhs].tol2;
    const int maxit = st[rhs].maxit;
    const int T = threadIdx.x;
    double acc = 0.0;
#pragma unroll 8
    for (int q = T; q < nd; q += FUSED_THREADS) acc += b[q] * b[q];
    const double bb = wg_sum(acc, w.red);
    // r = b - A x of the current x (its operand staged in the level-0 smoother field, free here)
    auto residual = [&]() -> double {
        double* xs = w.resident ? lvf(w, ws, F0, 1) : w.su;
        wg_copy(x, xs, nd);
        wg_apply(F0, xs, w.sy);
        double a = 0.0;
#pragma unroll 8
        for (int q = T; q < nd; q += FUSED_THREADS) {
            const double rq = b[q] - w.sy[q];
            r[q] = rq;
            a += rq * rq;
        }
        return wg_sum(a, w.red);
    };
    // start: r = b - A x0, or x = 0 and r = b; a guarded guess is kept only if its residual is below ||b||
    double rr = 0.0;
    int guess = 0;
    if (has_x0) {
        rr = residual();
        guess = (!guard || rr < bb) ? 1 : 0;
    }
    if (!guess) {
#pragma unroll 8
        for (int q = T; q < nd; q += FUSED_THREADS) {
            x[q] = 0.0;
            r[q] = b[q];
        }
        rr = bb;
        __syncthreads();
    }
    int iters = 0, breakdown = 0;
    for (int pass = 0; pass < 4; ++pass) {  // the first PCG pass and up to three restarts
        breakdown = 0;
        if (rr > tol2 * bb && iters < maxit) {
            double* z = wg_vcycle(w, M, ws);
            acc = 0.0;
#pragma unroll 8
            for (int q = T; q < nd; q += FUSED_THREADS) {
                acc += r[q] * z[q];
                p[q] = z[q];
            }
            double rz = wg_sum(acc, w.red);
            while (true) {
                // q = A p, with the LDS copy of p (resident: z's field now holds p)
                const double* pl = w.resident ? z : wg_operand(w, p, nd);
                wg_apply(F0, pl, w.sy);
                acc = 0.0;
#pragma unroll 8
                for (int q = T; q < nd; q += FUSED_THREADS) acc += pl[q] * w.sy[q];
                const double pq = wg_sum(acc, w.red);
                if (!(pq > 0.0) || !(rz > 0.0)) {
                    breakdown = 1;
                    break;
                }
                const double alpha = rz / pq;
                acc = 0.0;
#pragma unroll 8
                for (int q = T; q < nd; q += FUSED_THREADS) {
                    x[q] += alpha * pl[q];
                    const double rq = r[q] - alpha * w.sy[q];
                    r[q] = rq;
                    acc += rq * rq;
                }
                rr = wg_sum(acc, w.red);
                ++iters;
                if (!(rr > tol2 * bb) || iters >= maxit) break;
                z = wg_vcycle(w, M, ws);
                acc = 0.0;
#pragma unroll 8
                for (int q = T; q < nd; q += FUSED_THREADS) acc += r[q] * z[q];
                const double rzn = wg_sum(acc, w.red);
                const double beta = rzn / rz;
                rz = rzn;
#pragma unroll 8
                for (int q = T; q < nd; q += FUSED_THREADS) {
                    const double pn = z[q] + beta * p[q];
                    p[q] = pn;
                    z[q] = pn;
                }
                __syncthreads();
            }
        }
        rr = residual();  // of the current iterate, recomputed
        const bool miss = bb > 0.0 && rr > tol2 * bb * 1.0201;  // (1.01 rtol)^2
        if (!(miss && iters < maxit && !breakdown)) break;
    }
    if (T == 0) {
        RhsState& S = st[rhs];
        S.bb = bb;
        S.rr = rr;
        S.iters = iters;
        S.breakdown = breakdown;
        S.guess = guess;
        S.active = 0;
    }
}

}  // namespace

void launch_fused_pcg(const FusedMeshDev* M, int nrhs, const double* b, double* x, RhsState* st, double* ws,
                      bool has_x0, bool guard, hipStream_t s) {
    if (nrhs == 0) return;
    hipLaunchKernelGGL(k_fused_pcg, dim3(nrhs), dim3(FUSED_THREADS), 0, s, M, nrhs, b, x, st, ws, has_x0 ? 1 : 0,
                       guard ? 1 : 0);
}

// ---------------------------------------------------------------------------
// Group-persistent fused solve.  A group of K work-groups owns one right-hand side for the whole
// FP64 PCG: every phase (a smoothing step, a residual, a transfer, a step of the coarsest solve, a
// PCG vector update) is spread over the group's K * GROUP_THREADS threads, and a group barrier
// separates the phases.  Level fields live in the right-hand side's work space (global memory;
// small meshes stay in L2).  The operator is evaluated per node: the node's three element lines
// and the face value (and, on the line's end nodes, the face derivative) of the neighbouring
// elements along each axis.  Groups need nothing from each other, so the launch has no
// grid-wide barrier, and right-hand sides of one launch converge independently.
//
// Group barrier: thread 0 of each work-group adds one arrival to the right-hand side's counter
// (release at agent scope) and polls it until all K work-groups of the group have arrived at
// this barrier (counter >= barriers passed * K), then acquires.  The poll is bounded: past
// `spin` polls, or when another work-group of the group has given up, it sets the group's
// give-up flag and the work-groups leave the kernel (every wave ends); the right-hand side
// reports GROUP_SYNC_FAILED.  Measured on gfx950, a barrier over 8 work-groups costs about
// 1.3 us and one over 256 about 8 us (arrivals at one counter are serialised), against about
// 1.8 us between two kernels replayed from a graph: small groups are what pays.

namespace {

struct GroupArgs {
    const FusedMeshDev* M;
    int nrhs, K;
    const double* b;
    double* x;
    RhsState* st;
    double* ws;
    unsigned* sync;
    int has_x0, guard;
    long long spin;
};

struct GCtx {
    int gi, gs;          // this thread's index within the group, threads in the group
    int rank, K;
    unsigned* cnt;       // the group's arrival counter
    unsigned* fail;      // the group's give-up flag
    unsigned passed;     // barriers passed (thread 0)
    long long spin;
    int nsum;            // group sums taken (alternates the two slot sets)
    double* slots;       // 2 * K doubles of the right-hand side's work space
    double* red;         // LDS: one value per wave
    double* lds;         // LDS: GROUP_LDS_DOUBLES, the staged operand of an operator phase
    int* ok;             // LDS: the barrier's outcome for the work-group
};

__device__ bool g_bar(GCtx& c) {
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(c.cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned target = ++c.passed * (unsigned)c.K;
        long long n = 0;
        while (__hip_atomic_load(c.cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++n > c.spin || __hip_atomic_load(c.fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                __hip_atomic_store(c.fail, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *c.ok = ok;
    }
    __syncthreads();
    return *c.ok != 0;
}

// Sum of v over the group, taken at a barrier: the work-group's sum goes to its slot, and after
// the barrier every thread adds the K slots in slot order (the same value in every thread of the
// group).  Two slot sets alternate, so a work-group that runs ahead cannot overwrite slots that
// another still reads (a barrier separates any two sums that share a set).
__device__ bool g_sum(GCtx& c, double v, double& out) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    double* set = c.slots + (c.nsum & 1) * c.K;
    ++c.nsum;
    if ((threadIdx.x & 63) == 0) c.red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < GROUP_THREADS / 64; ++w) s += c.red[w];
        set[c.rank] = s;
    }
    if (!g_bar(c)) return false;
    double s = 0.0;
    for (int r = 0; r < c.K; ++r) s += set[r];
    out = s;
    return true;
}

// (A u) at node q of level F: the sum over the three axes of the node's row of the element-line
// form (interior block B, the coupling to the neighbours' face values U and U0 and, on the line's
// first and last node, to their face derivatives; ghost data on a domain face, as elem_op), times
// the axis scale and the GLL weights of the other two local indices.
template <int N>
__device__ __forceinline__ double g_apply_node(const FusedLevel& F, const RefDev<double>& R,
                                               const double* __restrict__ u, int q) {
    constexpr int N2 = N * N, N3 = N2 * N;
    const int e = q / N3, loc = q - e * N3;
    const int li[3] = {loc % N, (loc / N) % N, loc / N2};
    const int E0 = F.E[0], E1 = F.E[1];
    const int ei[3] = {e % E0, (e / E0) % E1, e / (E0 * E1)};
    const int s_in[3] = {1, N, N2};
    const int s_el[3] = {N3, E0 * N3, E0 * E1 * N3};
    double sum = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int i = li[d];
        const int base = q - i * s_in[d];
        double A[N];
#pragma unroll
        for (int l = 0; l < N; ++l) A[l] = u[base + l * s_in[d]];
        double acc = 0.0;
#pragma unroll
        for (int l = 0; l < N; ++l) acc += R.B[i][l] * A[l];
        double U, U0;
        if (ei[d] > 0) {
            const int nb = base - s_el[d];
            U = u[nb + (N - 1) * s_in[d]];
            if (i == 0) {
                double Dv = 0.0;
#pragma unroll
                for (int l = 0; l < N; ++l) Dv += R.aR[l] * u[nb + l * s_in[d]];
                acc += 0.5 * Dv - R.sig * U;
            }
        } else {
            U = -A[0];
            if (i == 0) {
                double Dv = -2.0 * R.sig * A[0];
#pragma unroll
                for (int l = 0; l < N; ++l) Dv += R.aL[l] * A[l];
                acc += 0.5 * Dv - R.sig * U;
            }
        }
        if (ei[d] < F.E[d] - 1) {
            const int nb = base + s_el[d];
            U0 = u[nb];
            if (i == N - 1) {
                double D0 = 0.0;
#pragma unroll
                for (int l = 0; l < N; ++l) D0 += R.aL[l] * u[nb + l * s_in[d]];
                acc -= 0.5 * D0 + R.sig * U0;
            }
        } else {
            U0 = -A[N - 1];
            if (i == N - 1) {
                double D0 = 2.0 * R.sig * A[N - 1];
#pragma unroll
                for (int l = 0; l < N; ++l) D0 += R.aR[l] * A[l];
                acc -= 0.5 * D0 + R.sig * U0;
            }
        }
        acc += 0.5 * (R.aR[i] * U0 - R.aL[i] * U);
        const int a = d == 0 ? li[1] : li[0], b2 = d == 2 ? li[1] : li[2];
        sum += acc * R.scale[d] * R.w[a] * R.w[b2];
    }
    return sum;
}

// The operand of an operator phase: copied whole into the work-group's LDS when the level fits
// (each work-group reads the field once, coalesced, instead of every node gathering its lines
// from L2), else read in place.  The caller's group barrier orders the copy against the next
// phase's.
constexpr int GROUP_LDS_DOUBLES = 8192;
__device__ __forceinline__ const double* g_stage(const double* __restrict__ u, int n, double* lds) {
    if (n > GROUP_LDS_DOUBLES) return u;
#pragma unroll 4
    for (int q = threadIdx.x; q < n; q += GROUP_THREADS) lds[q] = u[q];
    __syncthreads();
    return lds;
}

// out = z + cp (z - zp) + cr D^-1 (f - A z) on the nodes of this thread (zp null: zero).
// Returns this thread's part of dotv . out when dotv is given.
template <int N>
__device__ __noinline__ double g_cheb(int gi, int gs, const FusedLevel& F, const RefDev<double>& R, const double* __restrict__ f,
                         const double* __restrict__ z, const double* __restrict__ zp, double* __restrict__ out,
                         double cp, double cr, const double* __restrict__ dotv, double* lds) {
    const double* zs = g_stage(z, F.ndof, lds);
    double acc = 0.0;
    for (int q = gi; q < F.ndof; q += gs) {
        const double zq = zs[q];
        const double o = zq + cp * (zq - (zp ? zp[q] : 0.0)) + cr * F.dinv[q] * (f[q] - g_apply_node<N>(F, R, zs, q));
        out[q] = o;
        if (dotv) acc += dotv[q] * o;
    }
    return acc;
}

// out = f - A u; optionally z1 = c0 D^-1 out.  Returns this thread's part of out . out.
template <int N>
__device__ __noinline__ double g_resid(int gi, int gs, const FusedLevel& F, const RefDev<double>& R, const double* __restrict__ f,
                          const double* __restrict__ u, double* __restrict__ out, double* __restrict__ z1,
                          double* lds) {
    const double* us = g_stage(u, F.ndof, lds);
    double acc = 0.0;
    for (int q = gi; q < F.ndof; q += gs) {
        const double rq = f[q] - g_apply_node<N>(F, R, us, q);
        out[q] = rq;
        if (z1) z1[q] = F.c0 * F.dinv[q] * rq;
        acc += rq * rq;
    }
    return acc;
}

// out = A u.  Returns this thread's part of u . out.
template <int N>
__device__ __noinline__ double g_apply(int gi, int gs, const FusedLevel& F, const RefDev<double>& R, const double* __restrict__ u,
                          double* __restrict__ out, double* lds) {
    const double* us = g_stage(u, F.ndof, lds);
    double acc = 0.0;
    for (int q = gi; q < F.ndof; q += gs) {
        const double y = g_apply_node<N>(F, R, us, q);
        out[q] = y;
        acc += us[q] * y;
    }
    return acc;
}

#define DG_GN(F, CALL)                 \
    switch ((F).n) {                   \
        case 2: { constexpr int NN = 2; CALL; } break; \
        case 3: { constexpr int NN = 3; CALL; } break; \
        case 4: { constexpr int NN = 4; CALL; } break; \
        default: { constexpr int NN = 5; CALL; } break; \
    }

// fc = P^T t from level F to level C (each coarse node gathers the fine nodes of its element, or of
// its two children per axis, with the tensor product of the 1D weights); optionally
// z1c = C.c0 D_C^-1 fc.
__device__ __noinline__ void g_restrict(int gi, int gs, const FusedLevel& F, const FusedLevel& C, const double* __restrict__ t,
                           double* __restrict__ fc, double* __restrict__ z1c) {
    const int n = C.n, n3 = n * n * n;
    const int NXc = C.N[0], NYc = C.N[1], NZc = C.N[2];
    for (int o = gi; o < C.ndof; o += gs) {
        const int e = o / n3, l = o - e * n3;
        const int Xc = (e % C.E[0]) * n + l % n, Yc = ((e / C.E[0]) % C.E[1]) * n + (l / n) % n,
                  Zc = (e / (C.E[0] * C.E[1])) * n + l / (n * n);
        const int x0 = F.rlo[0][Xc], xn = F.rcnt[0][Xc];
        const int y0 = F.rlo[1][Yc], yn = F.rcnt[1][Yc];
        const int z0 = F.rlo[2][Zc], zn = F.rcnt[2][Zc];
        double s = 0.0;
        for (int cz = 0; cz < zn; ++cz) {
            const double wz = F.P[2][(z0 + cz) * NZc + Zc];
            for (int cy = 0; cy < yn; ++cy) {
                const double wyz = wz * F.P[1][(y0 + cy) * NYc + Yc];
                double sx = 0.0;
                for (int cx = 0; cx < xn; ++cx)
                    sx += F.P[0][(x0 + cx) * NXc + Xc] * t[em_index(F, x0 + cx, y0 + cy, z0 + cz)];
                s += wyz * sx;
            }
        }
        fc[o] = s;
        if (z1c) z1c[o] = C.c0 * C.dinv[o] * s;
    }
}

// zf += P zc from level C to level F (each fine node gathers the coarse nodes of its (parent) element).
__device__ __noinline__ void g_prolong_add(int gi, int gs, const FusedLevel& F, const FusedLevel& C, const double* __restrict__ zc,
                              double* __restrict__ zf) {
    const int n = F.n, n3 = n * n * n;
    const int NXc = C.N[0], NYc = C.N[1], NZc = C.N[2];
    for (int q = gi; q < F.ndof; q += gs) {
        const int e = q / n3, l = q - e * n3;
        const int Xf = (e % F.E[0]) * n + l % n, Yf = ((e / F.E[0]) % F.E[1]) * n + (l / n) % n,
                  Zf = (e / (F.E[0] * F.E[1])) * n + l / (n * n);
        const int x0 = F.plo[0][Xf], xn = F.pcnt[0][Xf];
        const int y0 = F.plo[1][Yf], yn = F.pcnt[1][Yf];
        const int z0 = F.plo[2][Zf], zn = F.pcnt[2][Zf];
        double s = 0.0;
        for (int cz = 0; cz < zn; ++cz) {
            const double wz = F.P[2][Zf * NZc + z0 + cz];
            for (int cy = 0; cy < yn; ++cy) {
                const double wyz = wz * F.P[1][Yf * NYc + y0 + cy];
                double sx = 0.0;
                for (int cx = 0; cx < xn; ++cx) sx += F.P[0][Xf * NXc + x0 + cx] * zc[em_index(C, x0 + cx, y0 + cy, z0 + cz)];
                s += wyz * sx;
            }
        }
        zf[q] += s;
    }
}

// The coarsest solve's eigendata staged in LDS once per work-group.
struct GCoarse {
    double Q[3][CMAX][CMAX];
    double lam[3][CMAX];
    double s[3][CMAX];
};

// Exact solve on the coarsest level C in three group phases: g1 = (Q^T (x) Q^T along x and y) S r,
// then per z line the contraction with Q^T, the division by the eigenvalue sums and the
// contraction with Q, then z = S (Q (x) Q along x and y) g2 (element-major).  g1, g2: lexicographic
// scratch, X fastest.
__device__ __noinline__ void g_coarse_fwd(int gi, int gs, const FusedLevel& C, const GCoarse& Cs,
                                          const double* __restrict__ r, double* __restrict__ g1) {
    const int nx = C.N[0], ny = C.N[1], nz = C.N[2];
    const int nxy = nx * ny, nall = nxy * nz;
    for (int o = gi; o < nall; o += gs) {
        const int Xo = o % nx, Yo = (o / nx) % ny, Z = o / nxy;
        double s = 0.0;
        for (int Y = 0; Y < ny; ++Y) {
            double sx = 0.0;
            for (int X = 0; X < nx; ++X) sx += Cs.Q[0][X][Xo] * Cs.s[0][X] * r[em_index(C, X, Y, Z)];
            s += Cs.Q[1][Y][Yo] * Cs.s[1][Y] * sx;
        }
        g1[o] = s * Cs.s[2][Z];
    }
}

__device__ __noinline__ void g_coarse_z(int gi, int gs, const FusedLevel& C, const GCoarse& Cs,
                                        const double* __restrict__ g1, double* __restrict__ g2) {
    const int nx = C.N[0], ny = C.N[1], nz = C.N[2];
    const int nxy = nx * ny;
    for (int o = gi; o < nxy; o += gs) {
        const int Xo = o % nx, Yo = o / nx;
        double v[CMAX];
#pragma unroll
        for (int k = 0; k < CMAX; ++k) {
            double s = 0.0;
            if (k < nz) {
                for (int Z = 0; Z < nz; ++Z) s += Cs.Q[2][Z][k] * g1[Z * nxy + o];
                s /= (Cs.lam[0][Xo] + Cs.lam[1][Yo] + Cs.lam[2][k]);
            }
            v[k] = s;
        }
        for (int Z = 0; Z < nz; ++Z) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < CMAX; ++k)
                if (k < nz) s += Cs.Q[2][Z][k] * v[k];
            g2[Z * nxy + o] = s;
        }
    }
}

__device__ __noinline__ void g_coarse_back(int gi, int gs, const FusedLevel& C, const GCoarse& Cs,
                                           const double* __restrict__ g2, double* __restrict__ z) {
    const int nx = C.N[0], ny = C.N[1], nz = C.N[2];
    const int nxy = nx * ny, nall = nxy * nz;
    for (int o = gi; o < nall; o += gs) {
        const int X = o % nx, Y = (o / nx) % ny, Z = o / nxy;
        double s = 0.0;
        for (int Yo = 0; Yo < ny; ++Yo) {
            double sx = 0.0;
            for (int Xo = 0; Xo < nx; ++Xo) sx += Cs.Q[0][X][Xo] * g2[Z * nxy + Yo * nx + Xo];
            s += Cs.Q[1][Y][Yo] * sx;
        }
        z[em_index(C, X, Y, Z)] = s * Cs.s[0][X] * Cs.s[1][Y] * Cs.s[2][Z];
    }
}

// Exact solve on the coarsest level C in three group phases: g1 = (Q^T (x) Q^T along x and y) S r,
// then per z line the contraction with Q^T, the division by the eigenvalue sums and the
// contraction with Q, then z = S (Q (x) Q along x and y) g2 (element-major).  g1, g2: lexicographic
// scratch, X fastest.
__device__ bool g_coarse(GCtx& c, const FusedLevel& C, const GCoarse& Cs, const double* __restrict__ r,
                         double* __restrict__ z, double* __restrict__ g1, double* __restrict__ g2) {
    g_coarse_fwd(c.gi, c.gs, C, Cs, r, g1);
    if (!g_bar(c)) return false;
    g_coarse_z(c.gi, c.gs, C, Cs, g1, g2);
    if (!g_bar(c)) return false;
    g_coarse_back(c.gi, c.gs, C, Cs, g2, z);
    return g_bar(c);
}

__device__ __forceinline__ double* g_field(double* ws, const FusedLevel& F, int which) {
    return ws + (which == 0 ? F.off_f : which == 1 ? F.off_za : F.off_zb);
}

// z = B r, one V-cycle from level 0 whose first smoothing iterate is already in lv[0]'s za; the
// last smoothing step also sums r . z (rz).  Returns the field that holds z, or null when a
// barrier gave up.
__device__ double* g_vcycle(GCtx& c, const FusedMeshDev& M, const RefDev<double>* Rs, const GCoarse& Cs, double* ws,
                            const double* r, double& rz) {
    const int nl = M.nl;
    double* t = ws + M.off_t;
    for (int l = 0; l + 1 < nl; ++l) {
        const FusedLevel& F = M.lv[l];
        const double* f = l == 0 ? r : g_field(ws, F, 0);
        double* cur = g_field(ws, F, 1);
        double* prev = g_field(ws, F, 2);
        for (int k = 1; k < F.deg; ++k) {
            DG_GN(F, g_cheb<NN>(c.gi, c.gs, F, Rs[l], f, cur, k == 1 ? nullptr : prev, prev, F.cp[k - 1], F.cr[k - 1],
                                nullptr, c.lds))
            if (!g_bar(c)) return nullptr;
            double* sw = cur; cur = prev; prev = sw;
        }
        DG_GN(F, g_resid<NN>(c.gi, c.gs, F, Rs[l], f, cur, t, nullptr, c.lds))
        if (!g_bar(c)) return nullptr;
        const FusedLevel& C = M.lv[l + 1];
        g_restrict(c.gi, c.gs, F, C, t, g_field(ws, C, 0), l + 2 < nl ? g_field(ws, C, 1) : nullptr);
        if (!g_bar(c)) return nullptr;
    }
    const FusedLevel& Lc = M.lv[nl - 1];
    double* zc = g_field(ws, Lc, 1);
    if (!g_coarse(c, Lc, Cs, g_field(ws, Lc, 0), zc, ws + M.off_g1, ws + M.off_g2)) return nullptr;
    if (nl == 1) {  // a single level: the exact solve is the preconditioner (its source is r)
        double part = 0.0;
        for (int q = c.gi; q < Lc.ndof; q += c.gs) part += r[q] * zc[q];
        if (!g_sum(c, part, rz)) return nullptr;
        return zc;
    }
    for (int l = nl - 2; l >= 0; --l) {
        const FusedLevel& F = M.lv[l];
        const double* f = l == 0 ? r : g_field(ws, F, 0);
        // the pre-smoothing left its iterate in za after an even number of swaps, else in zb
        const bool odd = ((F.deg - 1) & 1) != 0;
        double* cur = g_field(ws, F, odd ? 2 : 1);
        double* prev = g_field(ws, F, odd ? 1 : 2);
        g_prolong_add(c.gi, c.gs, F, M.lv[l + 1], zc, cur);
        if (!g_bar(c)) return nullptr;
        for (int k = 0; k < F.deg; ++k) {
            const bool last = l == 0 && k == F.deg - 1;
            double part = 0.0;
            DG_GN(F, part = g_cheb<NN>(c.gi, c.gs, F, Rs[l], f, cur, k == 0 ? nullptr : prev, prev,
                                        k == 0 ? 0.0 : F.cp[k - 1], k == 0 ? F.c0 : F.cr[k - 1], last ? r : nullptr, c.lds))
            if (last) {
                if (!g_sum(c, part, rz)) return nullptr;
            } else if (!g_bar(c)) {
                return nullptr;
            }
            double* sw = cur; cur = prev; prev = sw;
        }
        zc = cur;
    }
    return zc;
}

__global__ __launch_bounds__(GROUP_THREADS) void k_group_pcg(GroupArgs a) {
    __shared__ double red[GROUP_THREADS / 64];
    __shared__ int ok;
    __shared__ GCoarse Cs;
    __shared__ RefDev<double> Rs[FUSED_MAX_LEVELS];  // reference-element tables of every level
    __shared__ double ulds[GROUP_LDS_DOUBLES];
    const int b = blockIdx.x, xcd = b % 8, j = b / 8;
    const int rank = j % a.K, rhs = (j / a.K) * 8 + xcd;  // the group's work-groups share one XCD
    if (rhs >= a.nrhs) return;
    const FusedMeshDev& M = *a.M;
    GCtx c;
    c.rank = rank;
    c.K = a.K;
    c.gi = rank * GROUP_THREADS + (int)threadIdx.x;
    c.gs = a.K * GROUP_THREADS;
    c.cnt = a.sync + 2 * rhs;
    c.fail = a.sync + 2 * rhs + 1;
    c.passed = 0;
    c.spin = a.spin;
    c.nsum = 0;
    c.red = red;
    c.lds = ulds;
    c.ok = &ok;
    double* ws = a.ws + (long long)rhs * M.ws_group;
    c.slots = ws + M.off_red;
    {
        const CoarseDev& CD = *M.coarse;
        for (int q = threadIdx.x; q < 3 * CMAX * CMAX; q += GROUP_THREADS) (&Cs.Q[0][0][0])[q] = (&CD.Q[0][0][0])[q];
        for (int q = threadIdx.x; q < 3 * CMAX; q += GROUP_THREADS) {
            (&Cs.lam[0][0])[q] = (&CD.lam[0][0])[q];
            (&Cs.s[0][0])[q] = (&CD.s[0][0])[q];
        }
        constexpr int RW = (int)(sizeof(RefDev<double>) / sizeof(double));
        static_assert(sizeof(RefDev<double>) % sizeof(double) == 0, "RefDev<double> is a table of doubles");
        for (int q = threadIdx.x; q < M.nl * RW; q += GROUP_THREADS)
            reinterpret_cast<double*>(&Rs[q / RW])[q % RW] = reinterpret_cast<const double*>(&M.lv[q / RW].L->ref)[q % RW];
    }
    const FusedLevel& F0 = M.lv[0];
    const int nd = F0.ndof;
    const double* __restrict__ bv = a.b + (long long)rhs * nd;
    double* __restrict__ x = a.x + (long long)rhs * nd;
    double* r = g_field(ws, F0, 0);  // the level-0 source slot holds the residual
    double* p = ws + M.off_p;
    double* q = ws + M.off_q;
    double* z1 = g_field(ws, F0, 1);
    const double tol2 = a.st[rhs].tol2;
    const int maxit = a.st[rhs].maxit;
    bool live = true;
    int iters = 0, breakdown = 0, guess = 0;
    double bb = 0.0, rr = 0.0;
    do {  // one pass; `break` leaves it when a barrier gave up (live = false)
        double acc = 0.0;
        for (int i = c.gi; i < nd; i += c.gs) acc += bv[i] * bv[i];
        if (!(live = g_sum(c, acc, bb))) break;
        if (a.has_x0) {
            DG_GN(F0, acc = g_resid<NN>(c.gi, c.gs, F0, Rs[0], bv, x, r, z1, c.lds))
            if (!(live = g_sum(c, acc, rr))) break;
            guess = (!a.guard || rr < bb) ? 1 : 0;
        }
        if (!guess) {
            for (int i = c.gi; i < nd; i += c.gs) {
                x[i] = 0.0;
                r[i] = bv[i];
                z1[i] = F0.c0 * F0.dinv[i] * bv[i];
            }
            if (!(live = g_bar(c))) break;
            rr = bb;
        }
        for (int pass = 0; pass < 4 && live; ++pass) {  // the first PCG pass and up to three restarts
            breakdown = 0;
            if (rr > tol2 * bb && iters < maxit) {
                double rz = 0.0;
                double* z = g_vcycle(c, M, Rs, Cs, ws, r, rz);
                if (!(live = z != nullptr)) break;
                for (int i = c.gi; i < nd; i += c.gs) p[i] = z[i];
                if (!(live = g_bar(c))) break;
                while (true) {
                    double pq = 0.0;
                    DG_GN(F0, acc = g_apply<NN>(c.gi, c.gs, F0, Rs[0], p, q, c.lds))
                    if (!(live = g_sum(c, acc, pq))) break;
                    if (!(pq > 0.0) || !(rz > 0.0)) {
                        breakdown = 1;
                        break;
                    }
                    const double alpha = rz / pq;
                    acc = 0.0;
                    for (int i = c.gi; i < nd; i += c.gs) {
                        x[i] += alpha * p[i];
                        const double ri = r[i] - alpha * q[i];
                        r[i] = ri;
                        z1[i] = F0.c0 * F0.dinv[i] * ri;
                        acc += ri * ri;
                    }
                    if (!(live = g_sum(c, acc, rr))) break;
                    ++iters;
                    if (!(rr > tol2 * bb) || iters >= maxit) break;
                    double rzn = 0.0;
                    z = g_vcycle(c, M, Rs, Cs, ws, r, rzn);
                    if (!(live = z != nullptr)) break;
                    const double beta = rzn / rz;
                    rz = rzn;
                    for (int i = c.gi; i < nd; i += c.gs) p[i] = z[i] + beta * p[i];
                    if (!(live = g_bar(c))) break;
                }
                if (!live) break;
            }
            // residual of the current iterate, recomputed (and the next pass's first smoothing iterate)
            DG_GN(F0, acc = g_resid<NN>(c.gi, c.gs, F0, Rs[0], bv, x, r, z1, c.lds))
            if (!(live = g_sum(c, acc, rr))) break;
            const bool miss = bb > 0.0 && rr > tol2 * bb * 1.0201;  // (1.01 rtol)^2
            if (!(miss && iters < maxit && !breakdown)) break;
        }
    } while (false);
    if (threadIdx.x == 0 && (rank == 0 || !live)) {
        RhsState& S = a.st[rhs];
        S.active = 0;
        if (!live) {
            S.breakdown = GROUP_SYNC_FAILED;
        } else {
            S.bb = bb;
            S.rr = rr;
            S.iters = iters;
            S.breakdown = breakdown;
            S.guess = guess;
        }
    }
}

#undef DG_GN

}  // namespace

void launch_group_pcg(const FusedMeshDev* M, int K, int nrhs, const double* b, double* x, RhsState* st, double* ws,
                      unsigned* sync, bool has_x0, bool guard, long long spin, hipStream_t s) {
    if (nrhs == 0) return;
    if (K < 1 || K > GROUP_MAX_K) throw std::runtime_error("group-persistent solve: bad work-group count");
    launch_fill<unsigned>(sync, 0u, 2LL * nrhs, s);
    GroupArgs a{M, nrhs, K, b, x, st, ws, sync, has_x0 ? 1 : 0, guard ? 1 : 0, spin};
    const dim3 grid((unsigned)(((nrhs + 7) / 8) * 8 * K));
    hipLaunchKernelGGL(k_group_pcg, grid, dim3(GROUP_THREADS), 0, s, a);
}

}  // namespace dg
