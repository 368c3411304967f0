// Learned initial guess: a 3D U-Net on the element grid, with hand-written
// HIP forward, backward and Adam kernels, and its use as the PCG initial
// guess.
//
// Tensors are channels-last [batch][z][y][x][channel]: FP32 in training, BF16
// between the layers of the inference forward (the guess).  One channel per
// node of an element, so an element-major field of the library is the
// network's input or output tensor as it is.  Architecture, parameter order
// and loss are fixed in include/dg_poisson.h (dg_net_*).
//
// Kernels: forward convolutions on the matrix cores (implicit GEMM with BF16
// operands and FP32 accumulation; the 3x3x3 stride-1 layers stage their input
// box in LDS) and a direct FP32 form (weights read by uniform loads), both with
// fused bias and ReLU; gradient with respect to the input by the
// loop over the taps that touch an input voxel; gradient with respect to the
// weights by LDS-tiled partial sums over voxel chunks followed by a
// fixed-order reduction (deterministic).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <functional>
#include <stdexcept>
#include <string>
#include <vector>

#include "dg_internal.h"
#include "dg_kernels.h"

namespace {

struct NetError : std::runtime_error {
    using std::runtime_error::runtime_error;
};

#define NCHK(x)                                                                                              \
    do {                                                                                                     \
        hipError_t e_ = (x);                                                                                 \
        if (e_ != hipSuccess)                                                                                \
            throw NetError(std::string(#x) + ": " + hipGetErrorString(e_) + " at line " + std::to_string(__LINE__)); \
    } while (0)

constexpr int CO_GROUP = 8;   // output channels per thread in the convolution kernels

// ---------------------------------------------------------------------------
// kernels

// y[b][o][co] = act(bias[co] + sum_t sum_ci x[b][in(o,t)][ci] W[t][ci][co])
template <int KS, int STRIDE>
__global__ __launch_bounds__(256) void k_conv_fwd(const float* __restrict__ x, const float* __restrict__ W,
                                                  const float* __restrict__ bias, float* __restrict__ y, int D, int H,
                                                  int Wd, int Ci, int Do, int Ho, int Wo, int Co, int relu) {
    const int nvo = Do * Ho * Wo;
    const int o = blockIdx.x * 256 + threadIdx.x;
    const int co0 = blockIdx.y * CO_GROUP;
    const int b = blockIdx.z;
    if (o >= nvo) return;
    const int ox = o % Wo, oy = (o / Wo) % Ho, oz = o / (Wo * Ho);
    constexpr int PAD = (KS - 1) / 2;
    float acc[CO_GROUP];
#pragma unroll
    for (int c = 0; c < CO_GROUP; ++c) acc[c] = (co0 + c < Co) ? bias[co0 + c] : 0.f;
    const float* xb = x + (long long)b * D * H * Wd * Ci;
    for (int t = 0; t < KS * KS * KS; ++t) {
        const int dz = t / (KS * KS), dy = (t / KS) % KS, dx = t % KS;
        const int iz = oz * STRIDE - PAD + dz, iy = oy * STRIDE - PAD + dy, ix = ox * STRIDE - PAD + dx;
        if (iz < 0 || iz >= D || iy < 0 || iy >= H || ix < 0 || ix >= Wd) continue;
        const float* xv = xb + ((long long)(iz * H + iy) * Wd + ix) * Ci;
        const float* wt = W + ((long long)t * Ci) * Co + co0;
        for (int ci = 0; ci < Ci; ++ci) {
            const float v = xv[ci];
            const float* w = wt + (long long)ci * Co;
#pragma unroll
            for (int c = 0; c < CO_GROUP; ++c)
                if (co0 + c < Co) acc[c] += v * w[c];
        }
    }
    float* yo = y + ((long long)b * nvo + o) * Co + co0;
#pragma unroll
    for (int c = 0; c < CO_GROUP; ++c)
        if (co0 + c < Co) yo[c] = relu ? fmaxf(acc[c], 0.f) : acc[c];
}

// Same convolution as an implicit GEMM on the matrix cores: BF16 operands,
// FP32 accumulation (v_mfma_f32_16x16x32_bf16).  A wave computes 16 output
// voxels x 16*NB output channels; per tap and chunk of 32 input channels the
// A operand is 8 channels of one input voxel per lane (lane = voxel m + 16 kb,
// channels 8 kb .. 8 kb + 7) and the B operand 8 input channels of one output
// channel from the transposed BF16 weights Wt[tap][co][ci] (zero padded to
// CoP = 16 NB and CiP = multiple of 32).  The 16x16 result of a block holds
// D[4 kb + r][m] in lane m + 16 kb, register r.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Eight consecutive channels of one voxel as BF16 operands (RNE conversion of FP32 activations;
// BF16 activations as they are).  p is 16-byte aligned.
__device__ __forceinline__ bf16x8 load8_bf16(const float* p) {
    const float4 v0 = *reinterpret_cast<const float4*>(p);
    const float4 v1 = *reinterpret_cast<const float4*>(p + 4);
    bf16x8 a;
    a[0] = (__bf16)v0.x; a[1] = (__bf16)v0.y; a[2] = (__bf16)v0.z; a[3] = (__bf16)v0.w;
    a[4] = (__bf16)v1.x; a[5] = (__bf16)v1.y; a[6] = (__bf16)v1.z; a[7] = (__bf16)v1.w;
    return a;
}
__device__ __forceinline__ bf16x8 load8_bf16(const __bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }

template <int KS, int STRIDE, int NB, typename TX = float, typename TY = float>
__global__ __launch_bounds__(256) void k_conv_mfma(const TX* __restrict__ x, const __bf16* __restrict__ Wt,
                                                   const float* __restrict__ bias, TY* __restrict__ y, int D, int H,
                                                   int Wd, int Ci, int CiP, int Do, int Ho, int Wo, int Co,
                                                   int relu) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nvo = Do * Ho * Wo;
    const int vox0 = (blockIdx.x * 4 + wave) * 16;
    const int b = blockIdx.y;
    if (vox0 >= nvo) return;  // uniform per wave; the kernel has no barrier
    const int m = lane & 15, kb = lane >> 4;
    const int o = vox0 + m;
    const bool ov = o < nvo;
    const int ox = o % Wo, oy = (o / Wo) % Ho, oz = o / (Wo * Ho);
    constexpr int PAD = (KS - 1) / 2;
    f32x4 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    const TX* xb = x + (long long)b * D * H * Wd * Ci;
    const bool vec = (Ci % 8) == 0;
    for (int t = 0; t < KS * KS * KS; ++t) {
        const int dz = t / (KS * KS), dy = (t / KS) % KS, dx = t % KS;
        const int iz = oz * STRIDE - PAD + dz, iy = oy * STRIDE - PAD + dy, ix = ox * STRIDE - PAD + dx;
        const bool valid = ov && iz >= 0 && iz < D && iy >= 0 && iy < H && ix >= 0 && ix < Wd;
        const TX* xv = xb + (long long)((valid ? (iz * H + iy) * Wd + ix : 0)) * Ci;
        for (int cc = 0; cc < CiP; cc += 32) {
            const int ci0 = cc + 8 * kb;
            bf16x8 a;
            if (vec && valid && ci0 + 8 <= Ci) {
                a = load8_bf16(xv + ci0);
            } else if (valid && ci0 + 8 <= Ci) {  // whole chunk in range, rows not 16-byte aligned
#pragma unroll
                for (int q = 0; q < 8; ++q) a[q] = (__bf16)xv[ci0 + q];
            } else {
#pragma unroll
                for (int q = 0; q < 8; ++q) a[q] = (valid && ci0 + q < Ci) ? (__bf16)xv[ci0 + q] : (__bf16)0.f;
            }
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const bf16x8 w = *reinterpret_cast<const bf16x8*>(Wt + ((long long)(t * NB * 16 + nb * 16 + m) * CiP + ci0));
                acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, w, acc[nb], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int co = nb * 16 + m;
        if (co >= Co) continue;
        const float bco = bias[co];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o2 = vox0 + 4 * kb + r;
            if (o2 < nvo) {
                const float v = acc[nb][r] + bco;
                y[((long long)b * nvo + o2) * Co + co] = (TY)(relu ? fmaxf(v, 0.f) : v);
            }
        }
    }
}

// 3x3x3 stride-1 convolution on the matrix cores with the input staged in
// LDS.  A work-group of four waves owns CV_VPW consecutive output voxels of
// one sample; the box of input voxels they read (their z planes and rows,
// plus one voxel of padding on each side, zeros outside the grid) is staged
// once per chunk of 32 input channels as BF16, [voxel][32 channels], so each
// input value is converted once instead of once per tap.  Each wave computes
// CV_MB blocks of 16 voxels x 16 NB output channels: per tap it reads its A
// operands from LDS (16 bytes per lane, the 8 channels 8 kb .. 8 kb + 7 of
// voxel m = lane % 16) and NB B operands from the transposed weights, and
// issues CV_MB x NB MFMAs, so every weight load feeds CV_MB of them.
constexpr int CV_MB = 2;                 // voxel blocks per wave
constexpr int CV_VPW = 4 * 16 * CV_MB;  // voxels per work-group

// Box of input voxels staged for the output voxels [v0, v1) of a D x H x W grid.
struct ConvBox {
    int z0, y0, bz, by, bx;  // first plane and row (may be -1), extents
};
__host__ __device__ inline ConvBox conv_box(int v0, int v1, int H, int W) {
    const int HW = H * W;
    const int zlo = v0 / HW, zhi = (v1 - 1) / HW;
    int ylo = 0, yhi = H - 1;
    if (zlo == zhi) {
        ylo = (v0 % HW) / W;
        yhi = ((v1 - 1) % HW) / W;
    }
    ConvBox b;
    b.z0 = zlo - 1;
    b.y0 = ylo - 1;
    b.bz = zhi - zlo + 3;
    b.by = yhi - ylo + 3;
    b.bx = W + 2;
    return b;
}

template <int NB, typename TX = float, typename TY = float>
__global__ __launch_bounds__(256) void k_conv3_lds(const TX* __restrict__ x, const __bf16* __restrict__ Wt,
                                                   const float* __restrict__ bias, TY* __restrict__ y, int D, int H,
                                                   int Wd, int Ci, int CiP, int Co, int relu) {
    extern __shared__ __attribute__((aligned(16))) unsigned char conv_lds[];
    bf16x8* sx = reinterpret_cast<bf16x8*>(conv_lds);  // [box voxel][4 groups of 8 channels]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nvo = D * H * Wd;
    const int v0 = blockIdx.x * CV_VPW, v1 = min(nvo, v0 + CV_VPW);
    const int b = blockIdx.y;
    const ConvBox bx = conv_box(v0, v1, H, Wd);
    const int nbox = bx.bz * bx.by * bx.bx;
    const int m = lane & 15, kb = lane >> 4;
    // LDS voxel index of each block's voxel (centre tap), clamped to the grid
    int cen[CV_MB];
#pragma unroll
    for (int q = 0; q < CV_MB; ++q) {
        const int o = min(v0 + (wave * CV_MB + q) * 16 + m, nvo - 1);
        const int ox = o % Wd, oy = (o / Wd) % H, oz = o / (Wd * H);
        cen[q] = ((oz - bx.z0) * bx.by + (oy - bx.y0)) * bx.bx + ox + 1;
    }
    f32x4 acc[CV_MB][NB];
#pragma unroll
    for (int q = 0; q < CV_MB; ++q)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[q][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    const TX* xb = x + (long long)b * nvo * Ci;
    const bool vec = (Ci % 8) == 0;
    for (int cc = 0; cc < CiP; cc += 32) {
        if (cc) __syncthreads();  // the previous chunk's reads are done
        for (int e = threadIdx.x; e < nbox * 4; e += 256) {
            const int bv = e >> 2, g = e & 3;
            const int ix = bv % bx.bx - 1, iy = (bv / bx.bx) % bx.by + bx.y0, iz = bv / (bx.bx * bx.by) + bx.z0;
            const int ci0 = cc + 8 * g;
            bf16x8 a;
            const bool inside = ix >= 0 && ix < Wd && iy >= 0 && iy < H && iz >= 0 && iz < D;
            const TX* xv = xb + (long long)((inside ? (iz * H + iy) * Wd + ix : 0)) * Ci;
            if (inside && vec && ci0 + 8 <= Ci) {
                a = load8_bf16(xv + ci0);
            } else {
#pragma unroll
                for (int q = 0; q < 8; ++q) a[q] = (inside && ci0 + q < Ci) ? (__bf16)xv[ci0 + q] : (__bf16)0.f;
            }
            sx[e] = a;
        }
        __syncthreads();
#pragma unroll 3
        for (int t = 0; t < 27; ++t) {
            const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
            const int toff = ((dz - 1) * bx.by + (dy - 1)) * bx.bx + (dx - 1);
            bf16x8 w[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
                w[nb] = *reinterpret_cast<const bf16x8*>(Wt + ((long long)(t * NB * 16 + nb * 16 + m) * CiP + cc + 8 * kb));
#pragma unroll
            for (int q = 0; q < CV_MB; ++q) {
                const bf16x8 a = sx[(cen[q] + toff) * 4 + kb];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) acc[q][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, w[nb], acc[q][nb], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < CV_MB; ++q) {
        const int vb = v0 + (wave * CV_MB + q) * 16;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int co = nb * 16 + m;
            if (co >= Co) continue;
            const float bco = bias[co];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int o2 = vb + 4 * kb + r;
                if (o2 < v1) {
                    const float v = acc[q][nb][r] + bco;
                    y[((long long)b * nvo + o2) * Co + co] = (TY)(relu ? fmaxf(v, 0.f) : v);
                }
            }
        }
    }
}

// Wt[t][co][ci] = bf16(W[t][ci][co]), zero padded to [taps][CoP][CiP].
__global__ __launch_bounds__(256) void k_weights_bf16(const float* __restrict__ W, __bf16* __restrict__ Wt, int taps,
                                                      int Ci, int Co, int CiP, int CoP) {
    const long long n = (long long)taps * CoP * CiP;
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int ci = (int)(i % CiP), co = (int)((i / CiP) % CoP), t = (int)(i / ((long long)CiP * CoP));
    const float v = (ci < Ci && co < Co) ? W[((long long)t * Ci + ci) * Co + co] : 0.f;
    Wt[i] = (__bf16)v;
}

// dx[b][i][ci] = sum over (o, t) with in(o,t) = i of sum_co dy[b][o][co] W[t][ci][co]
template <int KS, int STRIDE>
__global__ __launch_bounds__(256) void k_conv_bwd_data(const float* __restrict__ dy, const float* __restrict__ W,
                                                       float* __restrict__ dx, int D, int H, int Wd, int Ci, int Do,
                                                       int Ho, int Wo, int Co) {
    const int nvi = D * H * Wd;
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int ci0 = blockIdx.y * CO_GROUP;
    const int b = blockIdx.z;
    if (i >= nvi) return;
    const int ix = i % Wd, iy = (i / Wd) % H, iz = i / (Wd * H);
    constexpr int PAD = (KS - 1) / 2;
    float acc[CO_GROUP] = {};
    const float* dyb = dy + (long long)b * Do * Ho * Wo * Co;
    for (int t = 0; t < KS * KS * KS; ++t) {
        const int dz = t / (KS * KS), dyy = (t / KS) % KS, dxx = t % KS;
        const int nz = iz + PAD - dz, ny = iy + PAD - dyy, nx = ix + PAD - dxx;
        if (nz < 0 || ny < 0 || nx < 0) continue;
        if (nz % STRIDE || ny % STRIDE || nx % STRIDE) continue;
        const int oz = nz / STRIDE, oy = ny / STRIDE, ox = nx / STRIDE;
        if (oz >= Do || oy >= Ho || ox >= Wo) continue;
        const float* g = dyb + ((long long)(oz * Ho + oy) * Wo + ox) * Co;
        const float* wt = W + (long long)t * Ci * Co + (long long)ci0 * Co;
        for (int co = 0; co < Co; ++co) {
            const float v = g[co];
#pragma unroll
            for (int c = 0; c < CO_GROUP; ++c)
                if (ci0 + c < Ci) acc[c] += v * wt[(long long)c * Co + co];
        }
    }
    float* out = dx + ((long long)b * nvi + i) * Ci + ci0;
#pragma unroll
    for (int c = 0; c < CO_GROUP; ++c)
        if (ci0 + c < Ci) out[c] = acc[c];
}

// Partial weight gradients: block (tap, ci tile of 16, co tile of 16, chunk s)
// sums x[b][in(o,t)][ci] dy[b][o][co] over its share of the (b, o) pairs.
constexpr int WG_TILE = 16;
constexpr int WG_CHUNK = 64;

template <int KS, int STRIDE>
__global__ __launch_bounds__(256) void k_conv_bwd_weight(const float* __restrict__ x, const float* __restrict__ dy,
                                                         float* __restrict__ part, int B, int D, int H, int Wd,
                                                         int Ci, int Do, int Ho, int Wo, int Co, int nsplit) {
    __shared__ float sx[WG_CHUNK][WG_TILE + 1];
    __shared__ float sg[WG_CHUNK][WG_TILE + 1];
    constexpr int PAD = (KS - 1) / 2;
    const int ntci = (Ci + WG_TILE - 1) / WG_TILE, ntco = (Co + WG_TILE - 1) / WG_TILE;
    int bid = blockIdx.x;
    const int split = bid % nsplit;
    bid /= nsplit;
    const int tco = bid % ntco;
    bid /= ntco;
    const int tci = bid % ntci;
    const int t = bid / ntci;
    const int dz = t / (KS * KS), dyy = (t / KS) % KS, dxx = t % KS;
    const int tid = threadIdx.x;
    const int lci = tid / WG_TILE, lco = tid % WG_TILE;
    const int nvo = Do * Ho * Wo;
    const long long total = (long long)B * nvo;
    const long long per = (total + nsplit - 1) / nsplit;
    const long long beg = split * per, end = min(total, beg + per);
    float acc = 0.f;
    for (long long c0 = beg; c0 < end; c0 += WG_CHUNK) {
        // stage WG_CHUNK output voxels: their input voxel for this tap, and dy
        for (int q = tid; q < WG_CHUNK * WG_TILE; q += 256) {
            const int r = q / WG_TILE, c = q % WG_TILE;
            const long long bo = c0 + r;
            float vx = 0.f, vg = 0.f;
            if (bo < end) {
                const int b = (int)(bo / nvo), o = (int)(bo % nvo);
                const int ox = o % Wo, oy = (o / Wo) % Ho, oz = o / (Wo * Ho);
                const int iz = oz * STRIDE - PAD + dz, iy = oy * STRIDE - PAD + dyy, ix = ox * STRIDE - PAD + dxx;
                const int ci = tci * WG_TILE + c, co = tco * WG_TILE + c;
                if (ci < Ci && iz >= 0 && iz < D && iy >= 0 && iy < H && ix >= 0 && ix < Wd)
                    vx = x[(((long long)b * D + iz) * H + iy) * Wd * (long long)Ci + (long long)ix * Ci + ci];
                if (co < Co) vg = dy[((long long)b * nvo + o) * Co + co];
            }
            sx[r][c] = vx;
            sg[r][c] = vg;
        }
        __syncthreads();
#pragma unroll 8
        for (int r = 0; r < WG_CHUNK; ++r) acc += sx[r][lci] * sg[r][lco];
        __syncthreads();
    }
    const int ci = tci * WG_TILE + lci, co = tco * WG_TILE + lco;
    if (ci < Ci && co < Co) part[((long long)split * KS * KS * KS * Ci + (long long)t * Ci + ci) * Co + co] = acc;
}

// out[j] = sum_s part[s][j]  (fixed order)
__global__ __launch_bounds__(256) void k_reduce_splits(const float* __restrict__ part, float* __restrict__ out,
                                                       long long n, int nsplit) {
    const long long j = (long long)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    float s = 0.f;
    for (int k = 0; k < nsplit; ++k) s += part[(long long)k * n + j];
    out[j] = s;
}

// db[co] = sum over (b, o) of dy[b][o][co]   (one block per co, fixed order)
__global__ __launch_bounds__(256) void k_bias_grad(const float* __restrict__ dy, float* __restrict__ db,
                                                   long long nbo, int Co) {
    __shared__ float red[256];
    const int co = blockIdx.x;
    float s = 0.f;
    for (long long q = threadIdx.x; q < nbo; q += 256) s += dy[q * Co + co];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) db[co] = red[0];
}

// g *= (y > 0)
__global__ __launch_bounds__(256) void k_relu_mask(float* __restrict__ g, const float* __restrict__ y, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n && !(y[i] > 0.f)) g[i] = 0.f;
}

// nearest x2 upsampling of [B][d][h][w][C] to [B][D][H][W][C] (D <= 2d ...)
template <typename T>
__global__ __launch_bounds__(256) void k_upsample(const T* __restrict__ s, T* __restrict__ u, int B, int d,
                                                  int h, int w, int D, int H, int W, int C) {
    const long long n = (long long)B * D * H * W * C;
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int c = (int)(i % C);
    long long v = i / C;
    const int x = (int)(v % W), y = (int)((v / W) % H), z = (int)((v / (W * H)) % D), b = (int)(v / ((long long)W * H * D));
    u[i] = s[((((long long)b * d + z / 2) * h + y / 2) * w + x / 2) * C + c];
}

__global__ __launch_bounds__(256) void k_upsample_bwd(const float* __restrict__ gu, float* __restrict__ gs, int B,
                                                      int d, int h, int w, int D, int H, int W, int C) {
    const long long n = (long long)B * d * h * w * C;
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int c = (int)(i % C);
    long long v = i / C;
    const int x = (int)(v % w), y = (int)((v / w) % h), z = (int)((v / (w * h)) % d), b = (int)(v / ((long long)w * h * d));
    float s = 0.f;
    for (int a = 0; a < 2; ++a)
        for (int e = 0; e < 2; ++e)
            for (int f = 0; f < 2; ++f) {
                const int Z = 2 * z + a, Y = 2 * y + e, X = 2 * x + f;
                if (Z < D && Y < H && X < W) s += gu[((((long long)b * D + Z) * H + Y) * W + X) * C + c];
            }
    gs[i] = s;
}

// cat[v][0:C1] = a[v], cat[v][C1:C1+C2] = b[v]  and the reverse split (add into ga, gb when acc)
template <typename T>
__global__ __launch_bounds__(256) void k_concat(const T* __restrict__ a, const T* __restrict__ b,
                                                T* __restrict__ cat, long long nv, int C1, int C2) {
    const int C = C1 + C2;
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= nv * C) return;
    const long long v = i / C;
    const int c = (int)(i % C);
    cat[i] = c < C1 ? a[v * C1 + c] : b[v * C2 + c - C1];
}
__global__ __launch_bounds__(256) void k_split(const float* __restrict__ gcat, float* __restrict__ ga,
                                               float* __restrict__ gb, long long nv, int C1, int C2, int acc_b) {
    const int C = C1 + C2;
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= nv * C) return;
    const long long v = i / C;
    const int c = (int)(i % C);
    if (c < C1)
        ga[v * C1 + c] = gcat[i];
    else if (acc_b)
        gb[v * C2 + c - C1] += gcat[i];
    else
        gb[v * C2 + c - C1] = gcat[i];
}

__global__ __launch_bounds__(256) void k_add(float* __restrict__ a, const float* __restrict__ b, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) a[i] += b[i];
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, long long n, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Per-sample scale and input: s = sqrt(mean(rho^2)); x = rho / s (FP32).
__global__ __launch_bounds__(256) void k_sumsq(const double* __restrict__ a, double* __restrict__ part, long long n) {
    __shared__ double red[256];
    const int b = blockIdx.y;
    double s = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const double v = a[(long long)b * n + i];
        s += v * v;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(long long)b * gridDim.x + blockIdx.x] = red[0];
}
__global__ void k_scale_of(const double* __restrict__ part, int nblk, long long n, double* __restrict__ scale) {
    const int b = blockIdx.x;
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < nblk; ++i) s += part[(long long)b * nblk + i];
    const double r = sqrt(s / (double)n);
    scale[b] = r > 0.0 ? r : 1.0;
}
template <typename T>
__global__ __launch_bounds__(256) void k_to_input(const double* __restrict__ a, const double* __restrict__ scale,
                                                  T* __restrict__ x, long long n) {
    const int b = blockIdx.y;
    const double inv = 1.0 / scale[b];
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        x[(long long)b * n + i] = (T)(float)(a[(long long)b * n + i] * inv);
}
__global__ __launch_bounds__(256) void k_f2bf(const float* __restrict__ a, __bf16* __restrict__ b, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) b[i] = (__bf16)a[i];
}
__global__ __launch_bounds__(256) void k_from_output(const float* __restrict__ y, const double* __restrict__ scale,
                                                     double* __restrict__ v, long long n) {
    const int b = blockIdx.y;
    const double s = scale[b];
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        v[(long long)b * n + i] = s * (double)y[(long long)b * n + i];
}

// Loss pieces: e = y - t (FP64), and after Ae is known: per sample sum e.Ae, and
// dy = 2 Ae / tAt.
__global__ __launch_bounds__(256) void k_err(const float* __restrict__ y, const double* __restrict__ t,
                                             double* __restrict__ e, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) e[i] = (double)y[i] - t[i];
}
__global__ __launch_bounds__(256) void k_loss_grad(const double* __restrict__ Ae, const double* __restrict__ tAt,
                                                   float* __restrict__ dy, long long n) {
    const int b = blockIdx.y;
    const double c = 2.0 / tAt[b];
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        dy[(long long)b * n + i] = (float)(c * Ae[(long long)b * n + i]);
}
__global__ __launch_bounds__(256) void k_err_d(const double* __restrict__ y, const double* __restrict__ t,
                                               double* __restrict__ e, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) e[i] = y[i] - t[i];
}
__global__ __launch_bounds__(256) void k_loss_grad_d(const double* __restrict__ src, const double* __restrict__ den,
                                                     double* __restrict__ g, long long n) {
    const int b = blockIdx.y;
    const double c = 2.0 / den[b];
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        g[(long long)b * n + i] = c * src[(long long)b * n + i];
}
__global__ __launch_bounds__(256) void k_dot_part(const double* __restrict__ a, const double* __restrict__ b,
                                                  double* __restrict__ part, long long n) {
    __shared__ double red[256];
    const int s = blockIdx.y;
    double acc = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        acc += a[(long long)s * n + i] * b[(long long)s * n + i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(long long)s * gridDim.x + blockIdx.x] = red[0];
}

// Continuous projection of a DG field (element-major, N nodes per element
// edge): every node shared by neighbouring elements (faces, edges, corners)
// is replaced by the average of its copies, gathered in a fixed order.
template <int N>
__global__ __launch_bounds__(256) void k_continuize(const double* __restrict__ u, double* __restrict__ w, int E0,
                                                    int E1, int E2, long long ndof) {
    constexpr int N3 = N * N * N;
    const int b = blockIdx.y;
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q >= ndof) return;
    const int qi = (int)q;
    const int e = qi / N3, l = qi - e * N3;
    const int ex = e % E0, ey = (e / E0) % E1, ez = e / (E0 * E1);
    const int i = l % N, j = (l / N) % N, k = l / (N * N);
    // per axis: own copy, plus the neighbour's copy when the node is on a shared face
    int nex = 1, ney = 1, nez = 1;
    int xe[2] = {ex, 0}, xi[2] = {i, 0}, ye[2] = {ey, 0}, yj[2] = {j, 0}, ze[2] = {ez, 0}, zk[2] = {k, 0};
    if (i == 0 && ex > 0) { xe[1] = ex - 1; xi[1] = N - 1; nex = 2; }
    if (i == N - 1 && ex < E0 - 1) { xe[1] = ex + 1; xi[1] = 0; nex = 2; }
    if (j == 0 && ey > 0) { ye[1] = ey - 1; yj[1] = N - 1; ney = 2; }
    if (j == N - 1 && ey < E1 - 1) { ye[1] = ey + 1; yj[1] = 0; ney = 2; }
    if (k == 0 && ez > 0) { ze[1] = ez - 1; zk[1] = N - 1; nez = 2; }
    if (k == N - 1 && ez < E2 - 1) { ze[1] = ez + 1; zk[1] = 0; nez = 2; }
    const double* ub = u + (long long)b * ndof;
    double s = 0.0;
    for (int c = 0; c < nez; ++c)
        for (int bb = 0; bb < ney; ++bb)
            for (int a = 0; a < nex; ++a)
                s += ub[(long long)((ze[c] * E1 + ye[bb]) * E0 + xe[a]) * N3 + (zk[c] * N + yj[bb]) * N + xi[a]];
    w[(long long)b * ndof + q] = s / (double)(nex * ney * nez);
}

__global__ __launch_bounds__(256) void k_f2d(const float* __restrict__ a, double* __restrict__ b, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) b[i] = (double)a[i];
}
__global__ __launch_bounds__(256) void k_d2f(const double* __restrict__ a, float* __restrict__ b, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}
__global__ __launch_bounds__(256) void k_scale_samples(double* __restrict__ v, const double* __restrict__ scale,
                                                       long long n) {
    const int b = blockIdx.y;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        v[(long long)b * n + i] *= scale[b];
}

inline unsigned nblocks(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

// ---------------------------------------------------------------------------
// network object

struct dg_net {
    dg_net_config cfg;
    struct Layer {
        std::string name;
        int k, s, ci, co;
        long long woff, boff;  // offsets of W and bias in the parameter vector
    };
    std::vector<Layer> layers;
    long long nparams = 0;
    bool bf16 = true;          // forward convolutions on the matrix cores (BF16 operands)
    bool wt_dirty = true;      // BF16 weight copies out of date
    __bf16* wt = nullptr;      // BF16 transposed weights, per layer at wtoff
    std::vector<long long> wtoff;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr, *part = nullptr;
    long long part_cap = 0;
    int t = 0;  // Adam steps taken
    // activations for the current batch and grid
    int B = 0, E[3] = {0, 0, 0};
    struct Buf {
        float* d = nullptr;
        long long n = 0;
    };
    std::vector<Buf> act;   // per layer output
    // inference with BF16 activations (the guess): per layer output and decoder inputs, and the
    // input; allocated with the FP32 set, on first use
    struct Buf16 {
        __bf16* d = nullptr;
        long long n = 0;
    };
    std::vector<Buf16> act16, aux16;
    Buf16 xin16;
    std::vector<Buf> aux;   // upsampled / concatenated inputs
    std::vector<Buf> grd;   // gradient work buffers
    std::vector<std::array<int, 3>> dims;  // spatial dims per level
    Buf xin;                               // copy of the last forward input
    double *e = nullptr, *Ae = nullptr, *tAt = nullptr, *dpart = nullptr, *scale = nullptr, *vtmp = nullptr;
    double *w1 = nullptr, *w2 = nullptr, *x0 = nullptr;
    float *xbuf = nullptr, *ybuf = nullptr, *dybuf = nullptr;
    long long cap_field = 0;
};

namespace {

thread_local std::string g_net_err;

dg_status net_guard(const std::function<void()>& fn) {
    try {
        fn();
        return DG_OK;
    } catch (const NetError& e) {
        g_net_err = e.what();
        return std::string(e.what()).find("hip") != std::string::npos ? DG_ERR_HIP : DG_ERR_ARG;
    } catch (const std::exception& e) {
        g_net_err = e.what();
        return DG_ERR_ARG;
    }
}

template <typename T>
T* nalloc(long long n) {
    void* p = nullptr;
    NCHK(hipMalloc(&p, (size_t)std::max(1LL, n) * sizeof(T)));
    return (T*)p;
}
template <typename T>
void nfree(T*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

int layer_index(const dg_net* net, const std::string& name) {
    for (size_t i = 0; i < net->layers.size(); ++i)
        if (net->layers[i].name == name) return (int)i;
    throw NetError("no layer " + name);
}

inline int pad_to(int v, int m) { return (v + m - 1) / m * m; }

void refresh_bf16(dg_net* net, hipStream_t s) {
    if (!net->wt) {
        long long tot = 0;
        net->wtoff.clear();
        for (const auto& L : net->layers) {
            net->wtoff.push_back(tot);
            tot += (long long)L.k * L.k * L.k * pad_to(L.co, 16) * pad_to(L.ci, 32);
        }
        net->wt = nalloc<__bf16>(tot);
    }
    for (size_t i = 0; i < net->layers.size(); ++i) {
        const auto& L = net->layers[i];
        const int taps = L.k * L.k * L.k, CiP = pad_to(L.ci, 32), CoP = pad_to(L.co, 16);
        const long long n = (long long)taps * CoP * CiP;
        hipLaunchKernelGGL(k_weights_bf16, dim3(nblocks(n)), dim3(256), 0, s, net->p + L.woff, net->wt + net->wtoff[i],
                           taps, L.ci, L.co, CiP, CoP);
    }
    net->wt_dirty = false;
}

template <typename TX, typename TY>
void conv_forward_mfma(const dg_net* net, int li, const TX* x, TY* y, int B, const int* din, const int* dout,
                       int relu, hipStream_t s) {
    const auto& L = net->layers[li];
    const int CiP = pad_to(L.ci, 32), NB = pad_to(L.co, 16) / 16;
    const int nvo = dout[0] * dout[1] * dout[2];
    dim3 grid((nvo + 63) / 64, B);
    const __bf16* Wt = net->wt + net->wtoff[li];
    const float* b = net->p + L.boff;
#define CM(KS, ST, NBV) hipLaunchKernelGGL((k_conv_mfma<KS, ST, NBV, TX, TY>), grid, dim3(256), 0, s, x, Wt, b, y, din[0], din[1], din[2], L.ci, CiP, dout[0], dout[1], dout[2], L.co, relu)
#define CMN(KS, ST) switch (NB) { case 1: CM(KS, ST, 1); break; case 2: CM(KS, ST, 2); break; case 4: CM(KS, ST, 4); break; default: throw NetError("unsupported channel count for the matrix-core path"); }
    if (L.k == 1) { CMN(1, 1) }
    else if (L.s == 1) {
        // LDS-staged kernel; the largest input box over the work-groups sizes its LDS
        int maxbox = 0;
        for (int v0 = 0; v0 < nvo; v0 += CV_VPW) {
            const ConvBox bx = conv_box(v0, std::min(nvo, v0 + CV_VPW), dout[1], dout[2]);
            maxbox = std::max(maxbox, bx.bz * bx.by * bx.bx);
        }
        const size_t lds = (size_t)maxbox * 64;
        if (lds > 64 * 1024) throw NetError("convolution input box too large for LDS");
        dim3 g3((nvo + CV_VPW - 1) / CV_VPW, B);
#define C3(NBV) hipLaunchKernelGGL((k_conv3_lds<NBV, TX, TY>), g3, dim3(256), lds, s, x, Wt, b, y, din[0], din[1], din[2], L.ci, CiP, L.co, relu)
        switch (NB) {
            case 1: C3(1); break;
            case 2: C3(2); break;
            case 4: C3(4); break;
            default: throw NetError("unsupported channel count for the matrix-core path");
        }
#undef C3
    }
    else { CMN(3, 2) }
#undef CMN
#undef CM
}

void conv_forward(const dg_net::Layer& L, const float* P, const float* x, float* y, int B, const int* din,
                  const int* dout, int relu, hipStream_t s) {
    dim3 grid(nblocks((long long)dout[0] * dout[1] * dout[2]), (L.co + CO_GROUP - 1) / CO_GROUP, B);
    const float* W = P + L.woff;
    const float* b = P + L.boff;
#define CF(KS, ST) hipLaunchKernelGGL((k_conv_fwd<KS, ST>), grid, dim3(256), 0, s, x, W, b, y, din[0], din[1], din[2], L.ci, dout[0], dout[1], dout[2], L.co, relu)
    if (L.k == 1) CF(1, 1);
    else if (L.s == 1) CF(3, 1);
    else CF(3, 2);
#undef CF
}

// Gradients of a convolution: dx (may be null), dW and db into net->g.
void conv_backward(dg_net* net, const dg_net::Layer& L, const float* x, const float* dy, float* dx, int B,
                   const int* din, const int* dout, hipStream_t s) {
    const float* W = net->p + L.woff;
    if (dx) {
        dim3 grid(nblocks((long long)din[0] * din[1] * din[2]), (L.ci + CO_GROUP - 1) / CO_GROUP, B);
#define CB(KS, ST) hipLaunchKernelGGL((k_conv_bwd_data<KS, ST>), grid, dim3(256), 0, s, dy, W, dx, din[0], din[1], din[2], L.ci, dout[0], dout[1], dout[2], L.co)
        if (L.k == 1) CB(1, 1);
        else if (L.s == 1) CB(3, 1);
        else CB(3, 2);
#undef CB
    }
    const int taps = L.k * L.k * L.k;
    const long long nw = (long long)taps * L.ci * L.co;
    const long long nbo = (long long)B * dout[0] * dout[1] * dout[2];
    const int nsplit = (int)std::max(1LL, std::min(64LL, nbo / 512));
    if (net->part_cap < nw * nsplit) throw NetError("internal: gradient work space too small");
    const int ntci = (L.ci + WG_TILE - 1) / WG_TILE, ntco = (L.co + WG_TILE - 1) / WG_TILE;
    const unsigned blocks = (unsigned)(taps * ntci * ntco * nsplit);
#define CW(KS, ST) hipLaunchKernelGGL((k_conv_bwd_weight<KS, ST>), dim3(blocks), dim3(256), 0, s, x, dy, net->part, B, din[0], din[1], din[2], L.ci, dout[0], dout[1], dout[2], L.co, nsplit)
    if (L.k == 1) CW(1, 1);
    else if (L.s == 1) CW(3, 1);
    else CW(3, 2);
#undef CW
    hipLaunchKernelGGL(k_reduce_splits, dim3(nblocks(nw)), dim3(256), 0, s, net->part, net->g + L.woff, nw, nsplit);
    hipLaunchKernelGGL(k_bias_grad, dim3(L.co), dim3(256), 0, s, dy, net->g + L.boff, nbo, L.co);
}

void ensure_buffers(dg_net* net, int B, const int* E) {
    if (net->B == B && net->E[0] == E[0] && net->E[1] == E[1] && net->E[2] == E[2]) return;
    NCHK(hipDeviceSynchronize());  // buffers may still be in use by queued kernels
    for (auto& b : net->act) nfree(b.d);
    for (auto& b : net->aux) nfree(b.d);
    for (auto& b : net->grd) nfree(b.d);
    for (auto& b : net->act16) nfree(b.d);
    for (auto& b : net->aux16) nfree(b.d);
    net->act16.clear();
    net->aux16.clear();
    nfree(net->xin16.d);
    net->xin16.n = 0;  // input16 allocates it again for the new grid
    const int Lv = net->cfg.levels, C = net->cfg.channels;
    net->dims.assign(Lv, {0, 0, 0});
    net->dims[0] = {E[2], E[1], E[0]};  // z, y, x
    for (int l = 1; l < Lv; ++l)
        for (int d = 0; d < 3; ++d) net->dims[l][d] = (net->dims[l - 1][d] + 1) / 2;
    auto vox = [&](int l) { return (long long)net->dims[l][0] * net->dims[l][1] * net->dims[l][2]; };
    net->act.assign(net->layers.size(), {});
    for (size_t i = 0; i < net->layers.size(); ++i) {
        const auto& L = net->layers[i];
        int lev = 0;
        if (L.name.rfind("enc", 0) == 0) lev = L.name[3] - '0';
        else if (L.name.rfind("down", 0) == 0) lev = L.name[4] - '0' + 1;
        else if (L.name.rfind("up", 0) == 0) lev = L.name[2] - '0';
        else if (L.name.rfind("merge", 0) == 0) lev = L.name[5] - '0';
        net->act[i].n = (long long)B * vox(lev) * L.co;
        net->act[i].d = nalloc<float>(net->act[i].n);
    }
    // aux: per decoder level l: upsampled input [vox(l)][C], concat [vox(l)][2C]
    net->aux.assign(2 * Lv, {});
    net->grd.assign(4, {});
    long long mx = 0;
    for (int l = 0; l < Lv; ++l) {
        net->aux[2 * l].n = (long long)B * vox(l) * C;
        net->aux[2 * l + 1].n = (long long)B * vox(l) * 2 * C;
        net->aux[2 * l].d = nalloc<float>(net->aux[2 * l].n);
        net->aux[2 * l + 1].d = nalloc<float>(net->aux[2 * l + 1].n);
        mx = std::max(mx, (long long)B * vox(l) * 2 * C);
    }
    mx = std::max(mx, (long long)B * vox(0) * std::max(net->cfg.in_channels, net->cfg.out_channels));
    for (auto& b : net->grd) {
        b.n = mx;
        b.d = nalloc<float>(mx);
    }
    nfree(net->xin.d);
    net->xin.n = (long long)B * vox(0) * net->cfg.in_channels;
    net->xin.d = nalloc<float>(net->xin.n);
    // weight-gradient partial sums: sized once for the largest layer, so that the
    // buffer is never replaced while kernels that use it are queued
    long long need = 0;
    for (const auto& L : net->layers) {
        int lev = 0;
        if (L.name.rfind("enc", 0) == 0) lev = L.name[3] - '0';
        else if (L.name.rfind("down", 0) == 0) lev = L.name[4] - '0' + 1;
        else if (L.name.rfind("up", 0) == 0) lev = L.name[2] - '0';
        else if (L.name.rfind("merge", 0) == 0) lev = L.name[5] - '0';
        const long long nbo = (long long)B * vox(lev);
        const long long nsplit = std::max(1LL, std::min(64LL, nbo / 512));
        need = std::max(need, (long long)L.k * L.k * L.k * L.ci * L.co * nsplit);
    }
    if (net->part_cap < need) {
        NCHK(hipDeviceSynchronize());
        nfree(net->part);
        net->part = nalloc<float>(need);
        net->part_cap = need;
    }
    net->B = B;
    net->E[0] = E[0]; net->E[1] = E[1]; net->E[2] = E[2];
}

// Forward pass on x [B][Ez][Ey][Ex][Cin]; the output is the activation of "out".
const float* forward(dg_net* net, int B, const int* E, const float* x, hipStream_t s) {
    ensure_buffers(net, B, E);
    // the input is kept for the backward pass (a caller may have written it there already)
    if (x != net->xin.d) NCHK(hipMemcpyAsync(net->xin.d, x, sizeof(float) * net->xin.n, hipMemcpyDeviceToDevice, s));
    x = net->xin.d;
    const int Lv = net->cfg.levels, C = net->cfg.channels;
    auto A = [&](const std::string& n) { return net->act[layer_index(net, n)].d; };
    auto D = [&](int l) { return net->dims[l].data(); };
    if (net->bf16 && net->wt_dirty) refresh_bf16(net, s);
    // conv_forward by layer name, on the matrix cores when enabled
    auto run = [&](const std::string& n, const float* in, float* out, const int* din, const int* dout, int relu) {
        const int li = layer_index(net, n);
        if (net->bf16)
            conv_forward_mfma(net, li, in, out, B, din, dout, relu, s);
        else
            conv_forward(net->layers[li], net->p, in, out, B, din, dout, relu, s);
    };
    run("in", x, A("in"), D(0), D(0), 1);
    const float* h = A("in");
    for (int l = 0; l < Lv; ++l) {
        const std::string a = "enc" + std::to_string(l) + "a", b = "enc" + std::to_string(l) + "b";
        run(a, h, A(a), D(l), D(l), 1);
        run(b, A(a), A(b), D(l), D(l), 1);
        if (l < Lv - 1) {
            const std::string dn = "down" + std::to_string(l);
            run(dn, A(b), A(dn), D(l), D(l + 1), 1);
            h = A(dn);
        }
    }
    const float* d = A("enc" + std::to_string(Lv - 1) + "b");
    for (int l = Lv - 2; l >= 0; --l) {
        const std::string up = "up" + std::to_string(l), mg = "merge" + std::to_string(l);
        const long long nu = net->aux[2 * l].n;
        hipLaunchKernelGGL(k_upsample<float>, dim3(nblocks(nu)), dim3(256), 0, s, d, net->aux[2 * l].d, B, D(l + 1)[0],
                           D(l + 1)[1], D(l + 1)[2], D(l)[0], D(l)[1], D(l)[2], C);
        run(up, net->aux[2 * l].d, A(up), D(l), D(l), 1);
        const long long nv = (long long)B * D(l)[0] * D(l)[1] * D(l)[2];
        hipLaunchKernelGGL(k_concat<float>, dim3(nblocks(nv * 2 * C)), dim3(256), 0, s, A(up),
                           A("enc" + std::to_string(l) + "b"), net->aux[2 * l + 1].d, nv, C, C);
        run(mg, net->aux[2 * l + 1].d, A(mg), D(l), D(l), 1);
        d = A(mg);
    }
    run("out", d, A("out"), D(0), D(0), 0);
    return A("out");
}

// Inference forward on the matrix cores with BF16 activations: every layer reads and writes BF16
// (the convolutions accumulate in FP32 and round their output to nearest even), except the last,
// whose FP32 output is the activation of "out".  The input x16 is BF16 (net->xin16).  The FP32
// activations of the training forward are not touched, so a backward pass still needs forward().
const float* forward16(dg_net* net, int B, const int* E, const __bf16* x16, hipStream_t s) {
    ensure_buffers(net, B, E);
    const int Lv = net->cfg.levels, C = net->cfg.channels;
    if (net->act16.empty()) {
        net->act16.assign(net->layers.size(), {});
        for (size_t i = 0; i < net->layers.size(); ++i) {
            net->act16[i].n = net->act[i].n;
            net->act16[i].d = nalloc<__bf16>(net->act16[i].n);
        }
        net->aux16.assign(net->aux.size(), {});
        for (size_t i = 0; i < net->aux.size(); ++i) {
            net->aux16[i].n = net->aux[i].n;
            net->aux16[i].d = nalloc<__bf16>(net->aux16[i].n);
        }
    }
    if (net->wt_dirty) refresh_bf16(net, s);
    auto A = [&](const std::string& n) { return net->act16[layer_index(net, n)].d; };
    auto D = [&](int l) { return net->dims[l].data(); };
    auto run = [&](const std::string& n, const __bf16* in, __bf16* out, const int* din, const int* dout, int relu) {
        conv_forward_mfma<__bf16, __bf16>(net, layer_index(net, n), in, out, B, din, dout, relu, s);
    };
    run("in", x16, A("in"), D(0), D(0), 1);
    const __bf16* h = A("in");
    for (int l = 0; l < Lv; ++l) {
        const std::string a = "enc" + std::to_string(l) + "a", b = "enc" + std::to_string(l) + "b";
        run(a, h, A(a), D(l), D(l), 1);
        run(b, A(a), A(b), D(l), D(l), 1);
        if (l < Lv - 1) {
            const std::string dn = "down" + std::to_string(l);
            run(dn, A(b), A(dn), D(l), D(l + 1), 1);
            h = A(dn);
        }
    }
    const __bf16* d = A("enc" + std::to_string(Lv - 1) + "b");
    for (int l = Lv - 2; l >= 0; --l) {
        const std::string up = "up" + std::to_string(l), mg = "merge" + std::to_string(l);
        const long long nu = net->aux16[2 * l].n;
        hipLaunchKernelGGL(k_upsample<__bf16>, dim3(nblocks(nu)), dim3(256), 0, s, d, net->aux16[2 * l].d, B,
                           D(l + 1)[0], D(l + 1)[1], D(l + 1)[2], D(l)[0], D(l)[1], D(l)[2], C);
        run(up, net->aux16[2 * l].d, A(up), D(l), D(l), 1);
        const long long nv = (long long)B * D(l)[0] * D(l)[1] * D(l)[2];
        hipLaunchKernelGGL(k_concat<__bf16>, dim3(nblocks(nv * 2 * C)), dim3(256), 0, s, A(up),
                           A("enc" + std::to_string(l) + "b"), net->aux16[2 * l + 1].d, nv, C, C);
        run(mg, net->aux16[2 * l + 1].d, A(mg), D(l), D(l), 1);
        d = A(mg);
    }
    float* out = net->act[layer_index(net, "out")].d;
    conv_forward_mfma<__bf16, float>(net, layer_index(net, "out"), d, out, B, D(0), D(0), 0, s);
    return out;
}

__bf16* input16(dg_net* net, long long n) {
    if (!net->xin16.d || net->xin16.n < n) {
        NCHK(hipDeviceSynchronize());
        nfree(net->xin16.d);
        net->xin16.d = nalloc<__bf16>(n);
        net->xin16.n = n;
    }
    return net->xin16.d;
}

// Backward pass for upstream gradient dy of the output; fills net->g.
void backward(dg_net* net, const float* dy, hipStream_t s) {
    const int B = net->B, Lv = net->cfg.levels, C = net->cfg.channels;
    auto A = [&](const std::string& n) { return net->act[layer_index(net, n)].d; };
    auto Ly = [&](const std::string& n) -> const dg_net::Layer& { return net->layers[layer_index(net, n)]; };
    auto D = [&](int l) { return net->dims[l].data(); };
    auto nv = [&](int l) { return (long long)B * D(l)[0] * D(l)[1] * D(l)[2]; };
    float *g0 = net->grd[0].d, *g1 = net->grd[1].d, *g2 = net->grd[2].d, *g3 = net->grd[3].d;
    // encoder skip gradients are kept in the aux buffers of the upsampled inputs (free after forward)
    const float* dout = (Lv >= 2) ? A("merge0") : A("enc0b");
    conv_backward(net, Ly("out"), dout, dy, g0, B, D(0), D(0), s);  // g0 = grad of d_0
    for (int l = 0; l < Lv - 1; ++l) {
        const std::string up = "up" + std::to_string(l), mg = "merge" + std::to_string(l);
        // through the ReLU of merge_l
        hipLaunchKernelGGL(k_relu_mask, dim3(nblocks(nv(l) * C)), dim3(256), 0, s, g0, A(mg), nv(l) * C);
        conv_backward(net, Ly(mg), net->aux[2 * l + 1].d, g0, g1, B, D(l), D(l), s);  // g1 = grad of concat
        // split: u part -> g2, skip part -> aux[2l] (reused as the skip gradient of e_l)
        hipLaunchKernelGGL(k_split, dim3(nblocks(nv(l) * 2 * C)), dim3(256), 0, s, g1, g2, net->aux[2 * l].d,
                           nv(l), C, C, 0);
        hipLaunchKernelGGL(k_relu_mask, dim3(nblocks(nv(l) * C)), dim3(256), 0, s, g2, A(up), nv(l) * C);
        // input of up_l is upsample(d_{l+1}); recompute it into g3 for the weight gradient
        const float* dsrc = (l + 1 == Lv - 1) ? A("enc" + std::to_string(l + 1) + "b") : A("merge" + std::to_string(l + 1));
        hipLaunchKernelGGL(k_upsample<float>, dim3(nblocks(nv(l) * C)), dim3(256), 0, s, dsrc, g3, B, D(l + 1)[0],
                           D(l + 1)[1], D(l + 1)[2], D(l)[0], D(l)[1], D(l)[2], C);
        conv_backward(net, Ly(up), g3, g2, g1, B, D(l), D(l), s);  // g1 = grad of the upsampled tensor
        hipLaunchKernelGGL(k_upsample_bwd, dim3(nblocks(nv(l + 1) * C)), dim3(256), 0, s, g1, g0, B, D(l + 1)[0],
                           D(l + 1)[1], D(l + 1)[2], D(l)[0], D(l)[1], D(l)[2], C);  // g0 = grad of d_{l+1}
    }
    // encoder, from the bottom level up; g0 holds the gradient of e_{L-1}
    for (int l = Lv - 1; l >= 0; --l) {
        const std::string a = "enc" + std::to_string(l) + "a", b = "enc" + std::to_string(l) + "b";
        if (l < Lv - 1) {
            // total gradient of e_l = skip part (aux[2l]) + down path (g0)
            hipLaunchKernelGGL(k_add, dim3(nblocks(nv(l) * C)), dim3(256), 0, s, g0, net->aux[2 * l].d, nv(l) * C);
        }
        hipLaunchKernelGGL(k_relu_mask, dim3(nblocks(nv(l) * C)), dim3(256), 0, s, g0, A(b), nv(l) * C);
        conv_backward(net, Ly(b), A(a), g0, g1, B, D(l), D(l), s);  // g1 = grad of a
        hipLaunchKernelGGL(k_relu_mask, dim3(nblocks(nv(l) * C)), dim3(256), 0, s, g1, A(a), nv(l) * C);
        const float* hin = (l == 0) ? A("in") : A("down" + std::to_string(l - 1));
        conv_backward(net, Ly(a), hin, g1, g0, B, D(l), D(l), s);  // g0 = grad of h_l
        hipLaunchKernelGGL(k_relu_mask, dim3(nblocks(nv(l) * C)), dim3(256), 0, s, g0, hin, nv(l) * C);
        if (l > 0) {
            const std::string dn = "down" + std::to_string(l - 1);
            conv_backward(net, Ly(dn), A("enc" + std::to_string(l - 1) + "b"), g0, g1, B, D(l - 1), D(l), s);
            std::swap(g0, g1);  // g0 = down-path gradient of e_{l-1}
        }
    }
    conv_backward(net, Ly("in"), net->xin.d, g0, nullptr, B, D(0), D(0), s);
}

}  // namespace

extern "C" {

const char* dg_net_last_error(void) { return g_net_err.c_str(); }

dg_status dg_net_create(const dg_net_config* cfg, dg_net** out) {
    return net_guard([&] {
        if (!cfg || !out) throw NetError("null argument");
        if (cfg->levels < 1 || cfg->levels > 6 || cfg->channels < 1 || cfg->channels > 256 || cfg->in_channels < 1 ||
            cfg->out_channels < 1)
            throw NetError("invalid network configuration");
        auto* net = new dg_net();
        net->cfg = *cfg;
        const int Lv = cfg->levels, C = cfg->channels;
        auto add = [&](const std::string& n, int k, int s, int ci, int co) {
            dg_net::Layer L{n, k, s, ci, co, 0, 0};
            L.woff = net->nparams;
            net->nparams += (long long)k * k * k * ci * co;
            L.boff = net->nparams;
            net->nparams += co;
            net->layers.push_back(L);
        };
        add("in", 1, 1, cfg->in_channels, C);
        for (int l = 0; l < Lv; ++l) {
            add("enc" + std::to_string(l) + "a", 3, 1, C, C);
            add("enc" + std::to_string(l) + "b", 3, 1, C, C);
            if (l < Lv - 1) add("down" + std::to_string(l), 3, 2, C, C);
        }
        for (int l = Lv - 2; l >= 0; --l) {
            add("up" + std::to_string(l), 3, 1, C, C);
            add("merge" + std::to_string(l), 3, 1, 2 * C, C);
        }
        add("out", 1, 1, C, cfg->out_channels);
        net->p = nalloc<float>(net->nparams);
        net->g = nalloc<float>(net->nparams);
        net->m = nalloc<float>(net->nparams);
        net->v = nalloc<float>(net->nparams);
        NCHK(hipMemset(net->p, 0, sizeof(float) * net->nparams));
        NCHK(hipMemset(net->m, 0, sizeof(float) * net->nparams));
        NCHK(hipMemset(net->v, 0, sizeof(float) * net->nparams));
        *out = net;
    });
}

void dg_net_destroy(dg_net* net) {
    if (!net) return;
    (void)hipDeviceSynchronize();
    for (auto& b : net->act) nfree(b.d);
    for (auto& b : net->aux) nfree(b.d);
    for (auto& b : net->grd) nfree(b.d);
    for (auto& b : net->act16) nfree(b.d);
    for (auto& b : net->aux16) nfree(b.d);
    nfree(net->xin16.d);
    nfree(net->xin.d);
    nfree(net->wt);
    nfree(net->p); nfree(net->g); nfree(net->m); nfree(net->v); nfree(net->part);
    nfree(net->e); nfree(net->Ae); nfree(net->tAt); nfree(net->dpart); nfree(net->scale); nfree(net->vtmp);
    nfree(net->xbuf); nfree(net->ybuf); nfree(net->dybuf); nfree(net->w1); nfree(net->w2); nfree(net->x0);
    delete net;
}

long long dg_net_num_params(const dg_net* net) { return net ? net->nparams : -1; }

dg_status dg_net_set_params(dg_net* net, const float* params, long long n) {
    return net_guard([&] {
        if (!net || !params || n != net->nparams) throw NetError("parameter count mismatch");
        NCHK(hipMemcpy(net->p, params, sizeof(float) * n, hipMemcpyHostToDevice));
        NCHK(hipMemset(net->m, 0, sizeof(float) * n));
        NCHK(hipMemset(net->v, 0, sizeof(float) * n));
        net->t = 0;
        net->wt_dirty = true;
    });
}

dg_status dg_net_get_params(const dg_net* net, float* params, long long n) {
    return net_guard([&] {
        if (!net || !params || n != net->nparams) throw NetError("parameter count mismatch");
        NCHK(hipMemcpy(params, net->p, sizeof(float) * n, hipMemcpyDeviceToHost));
    });
}

dg_status dg_net_forward(dg_net* net, int batch, const int* ne, const float* x, float* y, hipStream_t stream) {
    return net_guard([&] {
        if (!net || !ne || !x || !y || batch < 1) throw NetError("bad arguments");
        const float* out = forward(net, batch, ne, x, stream);
        const long long n = (long long)batch * ne[0] * ne[1] * ne[2] * net->cfg.out_channels;
        NCHK(hipMemcpyAsync(y, out, sizeof(float) * n, hipMemcpyDeviceToDevice, stream));
        NCHK(hipGetLastError());
    });
}

dg_status dg_net_infer(dg_net* net, int batch, const int* ne, const float* x, float* y, hipStream_t stream) {
    return net_guard([&] {
        if (!net || !ne || !x || !y || batch < 1 || ne[0] < 1 || ne[1] < 1 || ne[2] < 1) throw NetError("bad arguments");
        const long long nx = (long long)batch * ne[0] * ne[1] * ne[2] * net->cfg.in_channels;
        ensure_buffers(net, batch, ne);  // first: a new grid frees the BF16 input buffer
        __bf16* x16 = input16(net, nx);
        hipLaunchKernelGGL(k_f2bf, dim3(nblocks(nx)), dim3(256), 0, stream, x, x16, nx);
        const float* out = forward16(net, batch, ne, x16, stream);
        const long long ny = (long long)batch * ne[0] * ne[1] * ne[2] * net->cfg.out_channels;
        NCHK(hipMemcpyAsync(y, out, sizeof(float) * ny, hipMemcpyDeviceToDevice, stream));
        NCHK(hipGetLastError());
    });
}

dg_status dg_net_backward(dg_net* net, const float* dy, float* grad, hipStream_t stream) {
    return net_guard([&] {
        if (!net || !dy || net->B == 0) throw NetError("call dg_net_forward first");
        backward(net, dy, stream);
        if (grad) NCHK(hipMemcpyAsync(grad, net->g, sizeof(float) * net->nparams, hipMemcpyDeviceToDevice, stream));
        NCHK(hipGetLastError());
    });
}

dg_status dg_net_adam(dg_net* net, float lr, float b1, float b2, float eps, hipStream_t stream) {
    return net_guard([&] {
        if (!net) throw NetError("null net");
        net->t += 1;
        const float c1 = 1.f - std::pow(b1, (float)net->t), c2 = 1.f - std::pow(b2, (float)net->t);
        hipLaunchKernelGGL(k_adam, dim3(nblocks(net->nparams)), dim3(256), 0, stream, net->p, net->g, net->m, net->v,
                           net->nparams, lr, b1, b2, eps, c1, c2);
        net->wt_dirty = true;
        NCHK(hipGetLastError());
    });
}

dg_status dg_net_set_bf16(dg_net* net, int enable) {
    return net_guard([&] {
        if (!net) throw NetError("null net");
        net->bf16 = enable != 0;
        net->wt_dirty = true;
    });
}

dg_status dg_net_save(const dg_net* net, const char* path) {
    return net_guard([&] {
        if (!net || !path) throw NetError("bad arguments");
        std::vector<float> h(net->nparams);
        NCHK(hipMemcpy(h.data(), net->p, sizeof(float) * net->nparams, hipMemcpyDeviceToHost));
        std::ofstream f(path, std::ios::binary);
        if (!f) throw NetError(std::string("cannot write ") + path);
        const char magic[8] = {'D', 'G', 'N', 'E', 'T', '0', '0', '1'};
        f.write(magic, 8);
        const int hdr[4] = {net->cfg.levels, net->cfg.channels, net->cfg.in_channels, net->cfg.out_channels};
        f.write((const char*)hdr, sizeof(hdr));
        const long long n = net->nparams;
        f.write((const char*)&n, sizeof(n));
        f.write((const char*)h.data(), sizeof(float) * n);
    });
}

dg_status dg_net_load(dg_net* net, const char* path) {
    return net_guard([&] {
        if (!net || !path) throw NetError("bad arguments");
        std::ifstream f(path, std::ios::binary);
        if (!f) throw NetError(std::string("cannot read ") + path);
        char magic[8];
        f.read(magic, 8);
        if (std::memcmp(magic, "DGNET001", 8) != 0) throw NetError("not a network file");
        int hdr[4];
        f.read((char*)hdr, sizeof(hdr));
        if (hdr[0] != net->cfg.levels || hdr[1] != net->cfg.channels || hdr[2] != net->cfg.in_channels ||
            hdr[3] != net->cfg.out_channels)
            throw NetError("network file has a different configuration");
        long long n = 0;
        f.read((char*)&n, sizeof(n));
        if (n != net->nparams) throw NetError("network file has a different size");
        std::vector<float> h(n);
        f.read((char*)h.data(), sizeof(float) * n);
        if (!f) throw NetError("truncated network file");
        NCHK(hipMemcpy(net->p, h.data(), sizeof(float) * n, hipMemcpyHostToDevice));
        NCHK(hipMemset(net->m, 0, sizeof(float) * n));
        NCHK(hipMemset(net->v, 0, sizeof(float) * n));
        net->t = 0;
        net->wt_dirty = true;
    });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// training step and guess, using the solver context (dg_api.hip)

namespace dg {
// Provided by dg_api.hip.
const LevelHost& ctx_fine_level(const dg_ctx* ctx, int mesh_id);
const LevelHost& ctx_level(const dg_ctx* ctx, int mesh_id, int level);
}

namespace {

void launch_continuize(const dg::LevelHost& L, int batch, const double* u, double* w, hipStream_t s) {
    dim3 grid(nblocks(L.ndof), batch);
#define KC(NN) case NN: hipLaunchKernelGGL((k_continuize<NN>), grid, dim3(256), 0, s, u, w, L.E[0], L.E[1], L.E[2], L.ndof); break;
    switch (L.n) { KC(2) KC(3) KC(4) KC(5) KC(6) KC(7) KC(8) default: throw NetError("unsupported degree"); }
#undef KC
}

// The network's output is a field on multigrid level 1 (nodal, element-major,
// one channel per node).  Its guess on the finest level is P C y: C makes it
// continuous, P interpolates it to the finest degree.  y: FP32 [B][ndof1];
// out: FP64 [B][ndof0].  tmp1, tmp2: FP64 [B][ndof1] work space.
void output_map(const dg::LevelHost& L0, const dg::LevelHost& L1, int B, const float* y, double* out, double* tmp1,
                double* tmp2, hipStream_t s) {
    const long long n1 = L1.ndof * B;
    hipLaunchKernelGGL(k_f2d, dim3(nblocks(n1)), dim3(256), 0, s, y, tmp1, n1);
    launch_continuize(L1, B, tmp1, tmp2, s);
    dg::launch_fill<double>(out, 0.0, L0.ndof * B, s);
    dg::launch_prolong<double>(L0, L1, B, nullptr, tmp2, out, s);
}

// The guess: scale[b] * output_map(y) for sample b, the scale applied by the prolongation
// itself where the step from level 1 to level 0 is a degree step (one write of the fine field).
void output_map_scaled(const dg::LevelHost& L0, const dg::LevelHost& L1, int B, const float* y, double* out,
                       double* tmp1, double* tmp2, const double* scale, hipStream_t s) {
    const long long n1 = L1.ndof * B;
    hipLaunchKernelGGL(k_f2d, dim3(nblocks(n1)), dim3(256), 0, s, y, tmp1, n1);
    launch_continuize(L1, B, tmp1, tmp2, s);
    if (dg::launch_prolong_set(L0, L1, B, tmp2, out, scale, s)) return;
    dg::launch_fill<double>(out, 0.0, L0.ndof * B, s);
    dg::launch_prolong<double>(L0, L1, B, nullptr, tmp2, out, s);
    hipLaunchKernelGGL(k_scale_samples, dim3(64, B), dim3(256), 0, s, out, scale, L0.ndof);
}

// Transpose of output_map: gy = C P^T g (C is symmetric).  g: FP64 [B][ndof0].
void output_map_transpose(const dg::LevelHost& L0, const dg::LevelHost& L1, int B, const double* g, float* gy,
                          double* tmp1, double* tmp2, hipStream_t s) {
    dg::launch_restrict<double>(L0, L0.dev64, L1, L1.dev64, B, nullptr, nullptr, g, tmp1, nullptr, 0.0, s);
    launch_continuize(L1, B, tmp1, tmp2, s);
    const long long n1 = L1.ndof * B;
    hipLaunchKernelGGL(k_d2f, dim3(nblocks(n1)), dim3(256), 0, s, tmp2, gy, n1);
}

}  // namespace

namespace {

void ensure_field(dg_net* net, long long n, int B) {
    if (net->cap_field >= n) return;
    NCHK(hipDeviceSynchronize());
    nfree(net->e); nfree(net->Ae); nfree(net->tAt); nfree(net->dpart); nfree(net->scale); nfree(net->vtmp);
    nfree(net->xbuf); nfree(net->ybuf); nfree(net->dybuf); nfree(net->w1); nfree(net->w2); nfree(net->x0);
    net->w1 = nalloc<double>(n);
    net->w2 = nalloc<double>(n);
    net->x0 = nalloc<double>(n);
    net->e = nalloc<double>(n);
    net->Ae = nalloc<double>(n);
    net->vtmp = nalloc<double>(n);
    net->tAt = nalloc<double>(B * 4 + 4);
    net->scale = nalloc<double>(B * 4 + 4);
    net->dpart = nalloc<double>((long long)(B * 4 + 4) * 64);
    net->xbuf = nalloc<float>(n);
    net->ybuf = nalloc<float>(n);
    net->dybuf = nalloc<float>(n);
    net->cap_field = n;
}

// per-sample dot products a.b over n values, B samples -> host
std::vector<double> sample_dots(dg_net* net, const double* a, const double* b, long long n, int B, hipStream_t s) {
    const int nb = 64;
    hipLaunchKernelGGL(k_dot_part, dim3(nb, B), dim3(256), 0, s, a, b, net->dpart, n);
    std::vector<double> h((size_t)B * nb), out(B, 0.0);
    NCHK(hipMemcpyAsync(h.data(), net->dpart, sizeof(double) * B * nb, hipMemcpyDeviceToHost, s));
    NCHK(hipStreamSynchronize(s));
    for (int b2 = 0; b2 < B; ++b2)
        for (int i = 0; i < nb; ++i) out[b2] += h[(size_t)b2 * nb + i];
    return out;
}

}  // namespace

extern "C" {

// Scaled input x = rho / s with s = rms(rho) per sample (FP32 out), s to scale (device [B]).
dg_status dg_net_prepare_input(dg_net* net, int batch, long long n_dofs, const double* rho, float* x, double* scale,
                               hipStream_t stream) {
    return net_guard([&] {
        if (!net || !rho || !x || !scale || batch < 1 || n_dofs < 1) throw NetError("bad arguments");
        ensure_field(net, n_dofs * batch, batch);
        const int nb = 64;
        hipLaunchKernelGGL(k_sumsq, dim3(nb, batch), dim3(256), 0, stream, rho, net->dpart, n_dofs);
        hipLaunchKernelGGL(k_scale_of, dim3(batch), dim3(64), 0, stream, net->dpart, nb, n_dofs, scale);
        hipLaunchKernelGGL(k_to_input<float>, dim3(nb, batch), dim3(256), 0, stream, rho, scale, x, n_dofs);
        NCHK(hipGetLastError());
    });
}

// One training step on a batch: forward on x, relative A-norm loss against the
// scaled targets t (FP64, field order), backward, Adam.  Returns the mean loss.
dg_status dg_net_train_step(dg_net* net, dg_ctx* ctx, int mesh_id, int batch, const float* x, const double* t,
                            float lr, int mode, double* loss, hipStream_t stream) {
    return net_guard([&] {
        if (!net || !ctx || !x || !t || batch < 1) throw NetError("bad arguments");
        const dg::LevelHost& L0 = dg::ctx_fine_level(ctx, mesh_id);
        const dg::LevelHost& L1 = dg::ctx_level(ctx, mesh_id, 1);
        const int ne[3] = {L0.E[0], L0.E[1], L0.E[2]};
        const long long nd = L0.ndof;
        if (net->cfg.in_channels != L0.n * L0.n * L0.n || net->cfg.out_channels != L1.n * L1.n * L1.n ||
            L1.E[0] != L0.E[0] || L1.E[1] != L0.E[1] || L1.E[2] != L0.E[2])
            throw NetError("network channels must equal the nodes per element of levels 0 (input) and 1 (output)");
        ensure_field(net, nd * batch, batch);
        const float* y = forward(net, batch, ne, x, stream);
        const long long n = nd * batch;
        output_map(L0, L1, batch, y, net->x0, net->w1, net->w2, stream);
        hipLaunchKernelGGL(k_err_d, dim3(nblocks(n)), dim3(256), 0, stream, net->x0, t, net->e, n);
        dg::launch_brick<double>(dg::BM_APPLY, L0, L0.dev64, batch, nullptr, net->e, nullptr, nullptr, nullptr,
                                 net->Ae, nullptr, nullptr, 0, 0, 0, stream);
        dg::launch_brick<double>(dg::BM_APPLY, L0, L0.dev64, batch, nullptr, t, nullptr, nullptr, nullptr, net->vtmp,
                                 nullptr, nullptr, 0, 0, 0, stream);
        std::vector<double> eAe = sample_dots(net, net->e, net->Ae, nd, batch, stream);
        std::vector<double> tAt = sample_dots(net, t, net->vtmp, nd, batch, stream);
        double L = 0.0;
        for (int b = 0; b < batch; ++b) L += eAe[b] / tAt[b];
        if (loss) *loss = L / batch;
        // output gradient: mode 0: 2 A e / (tAt B), the A-norm gradient;
        // mode 1: 2 e / (t.t B), relative nodal L2; mode 2: 2 B_mg A e / (tAt B),
        // the A-norm gradient preconditioned by one V-cycle (B_mg A e ~ e).
        std::vector<double> scaled(batch);
        const double* gsrc = net->Ae;
        if (mode == 1) {
            std::vector<double> tt = sample_dots(net, t, t, nd, batch, stream);
            for (int b = 0; b < batch; ++b) scaled[b] = tt[b] * batch;
            gsrc = net->e;
        } else {
            for (int b = 0; b < batch; ++b) scaled[b] = tAt[b] * batch;
            if (mode == 2) {
                if (dg_vcycle_apply(ctx, mesh_id, 0, batch, net->Ae, net->vtmp, stream) != DG_OK)
                    throw NetError(std::string("V-cycle failed: ") + dg_last_error());
                gsrc = net->vtmp;
            }
        }
        NCHK(hipMemcpyAsync(net->tAt, scaled.data(), sizeof(double) * batch, hipMemcpyHostToDevice, stream));
        // gradient with respect to the fine-level guess, then through P^T and C to the network output
        double* gx = const_cast<double*>(gsrc);  // a work buffer of the network: scaled in place
        hipLaunchKernelGGL(k_loss_grad_d, dim3(64, batch), dim3(256), 0, stream, gsrc, net->tAt, gx, nd);
        output_map_transpose(L0, L1, batch, gx, net->dybuf, net->w1, net->w2, stream);
        backward(net, net->dybuf, stream);
        net->t += 1;
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        const float c1 = 1.f - std::pow(b1, (float)net->t), c2 = 1.f - std::pow(b2, (float)net->t);
        hipLaunchKernelGGL(k_adam, dim3(nblocks(net->nparams)), dim3(256), 0, stream, net->p, net->g, net->m, net->v,
                           net->nparams, lr, b1, b2, eps, c1, c2);
        net->wt_dirty = true;
        NCHK(hipGetLastError());
    });
}

// Initial guesses v0 = s * net(rho / s) for a batch of fields (FP64 in and out).
dg_status dg_net_guess(dg_net* net, const dg_ctx* ctx, int mesh_id, int batch, const double* rho, double* v0,
                       hipStream_t stream) {
    return net_guard([&] {
        if (!net || !ctx || !rho || !v0 || batch < 1) throw NetError("bad arguments");
        const dg::LevelHost& L0 = dg::ctx_fine_level(ctx, mesh_id);
        const dg::LevelHost& L1 = dg::ctx_level(ctx, mesh_id, 1);
        if (net->cfg.in_channels != L0.n * L0.n * L0.n || net->cfg.out_channels != L1.n * L1.n * L1.n)
            throw NetError("network channels do not match the mesh levels 0 and 1");
        const int ne[3] = {L0.E[0], L0.E[1], L0.E[2]};
        const long long n_dofs = L0.ndof;
        ensure_field(net, n_dofs * batch, batch);
        ensure_buffers(net, batch, ne);
        if (net->xin.n != n_dofs * batch) throw NetError("internal: input buffer size");
        const int nb = 64;
        hipLaunchKernelGGL(k_sumsq, dim3(nb, batch), dim3(256), 0, stream, rho, net->dpart, n_dofs);
        hipLaunchKernelGGL(k_scale_of, dim3(batch), dim3(64), 0, stream, net->dpart, nb, n_dofs, net->scale);
        const float* y;
        if (net->bf16) {  // matrix cores with BF16 activations
            __bf16* x16 = input16(net, n_dofs * batch);
            hipLaunchKernelGGL(k_to_input<__bf16>, dim3(nb, batch), dim3(256), 0, stream, rho, net->scale, x16, n_dofs);
            y = forward16(net, batch, ne, x16, stream);
        } else {          // FP32 vector path
            hipLaunchKernelGGL(k_to_input<float>, dim3(nb, batch), dim3(256), 0, stream, rho, net->scale, net->xin.d,
                               n_dofs);
            y = forward(net, batch, ne, net->xin.d, stream);
        }
        output_map_scaled(L0, L1, batch, y, v0, net->w1, net->w2, net->scale, stream);
        NCHK(hipGetLastError());
    });
}

}  // extern "C"
