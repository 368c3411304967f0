// Dirichlet data of the auxiliary-mesh Poisson problem by quadrature (Sec. 6.3).
//
// The full-space problem -Lap u = 4 pi f is restated on the mesh domain with
// Dirichlet data equal to the Coulomb potential of f on the boundary, and that
// integral is evaluated with the quadrature rule of the mesh's own nodal grid
// (here the GLL grid, whose weights are the lumped mass W_q):
//
//     g(r) = sum_q W_q f(x_q) / |r - x_q|      for every boundary node r.
//
// Every boundary node is itself a grid node (and, on an element face, also the
// node of the neighbouring element at the same place), where the integrand is
// singular; the method has f vanish there, so terms closer than a millionth of
// the smallest element width are left out.
//
// Work per source: n_face * n_dofs pair terms, a dense FP64 boundary-by-volume
// sum bound by FP64 vector issue.  The kernels are laid out for that:
//  * k_quad_pack writes, for a tile of R sources, the records W_q f_s(x_q)
//    (s in the tile) in lattice order of the grid nodes [Z][Y][X];
//  * in k_quad each lane owns one boundary node and the R sums of the tile;
//    all lanes visit the grid nodes in the same order, so the node's x
//    coordinate and its R weighted values are wave-uniform and are read with
//    scalar loads into SGPR operands of the FMAs;
//  * the squared distance is built per lattice row: dy^2 + dz^2 once, then one
//    FMA per node; 1/|r| is the hardware reciprocal square root refined by the
//    first two terms of its error series;
//  * only rows on the boundary surface of the lattice (and the first and last
//    node of the other rows) can hold a coincident node, so only those terms
//    pay for the distance test;
//  * the Z planes are split into parts so that a launch holds several rounds of
//    resident waves; the parts' partial sums are added in a fixed order by
//    k_quad_sum.  Work-groups are ordered so that each XCD takes the boundary
//    tiles of one part at a time: they stream the same records through its L2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <stdexcept>

#include "dg_internal.h"
#include "dg_kernels.h"

namespace dg {

namespace {

constexpr int QUAD_RMAX = 48;      // sources per tile (accumulators per lane)
// waves a launch aims for: 32 per SIMD, several rounds of the waves that fit at once (the loop
// waits on scalar loads, so waves queued behind the resident ones keep the SIMDs fed; measured
// on the 36 pair densities of 16^3 elements, p = 4: 8 per SIMD 44.3 ms, 16 38.2, 32 36.9, 64 38.4)
constexpr int QUAD_WAVES = 32768;
constexpr int QUAD_BLOCK = 256;    // threads per workgroup (its waves read the same records)
constexpr int QUAD_NB = 1;         // boundary nodes per lane (each scalar-loaded value feeds QUAD_NB FMAs)

__global__ __launch_bounds__(256) void k_quad_pack(const LevelDev<double>* __restrict__ dev, int Ex, int Ey, int n,
                                                   long long ndof, int NX, int NY, int nsrc, int r0, int R,
                                                   const double* __restrict__ f, const double* __restrict__ phi,
                                                   const int* __restrict__ pi, const int* __restrict__ pj,
                                                   double* __restrict__ rec) {
    const long long q = blockIdx.x * 256LL + threadIdx.x;
    if (q >= ndof) return;
    const int n3 = n * n * n;
    const long long e = q / n3;
    const int l = (int)(q - e * n3);
    const int i = l % n, j = (l / n) % n, k = l / (n * n);
    const int ex = (int)(e % Ex), ey = (int)((e / Ex) % Ey), ez = (int)(e / ((long long)Ex * Ey));
    const double w = dev->ax[0].m[i] * dev->ax[1].m[j] * dev->ax[2].m[k];
    const long long G = (ex * n + i) + (long long)NX * ((ey * n + j) + (long long)NY * (ez * n + k));
    double* out = rec + G * R;
    for (int r = 0; r < R; ++r) {
        const int s = r0 + r;
        double v = 0.0;
        if (s < nsrc)
            v = w * (f ? f[(long long)s * ndof + q] : phi[(long long)pi[s] * ndof + q] * phi[(long long)pj[s] * ndof + q]);
        out[r] = v;
    }
}

// 1/|r - x_q| for the lane's boundary node at squared distance d2 + (bx - xq)^2; with MASK,
// 0 for a node at the boundary node itself.
template <bool MASK>
__device__ __forceinline__ double inv_dist(double bx, double d2, double xq, double drop2) {
    const double dx = bx - xq;
    const double r2 = fma(dx, dx, d2);
    // the hardware estimate is good to about 5e-8; with e = 1 - r2 y^2 the exact value is
    // y (1 - e)^(-1/2) = y (1 + e/2 + 3e^2/8 + ...), so two terms of the series leave O(e^3)
    double y = __builtin_amdgcn_rsq(r2);
    const double e = fma(-(r2 * y), y, 1.0);
    y = fma(y * e, fma(0.375, e, 0.5), y);
    if (MASK) y = r2 > drop2 ? y : 0.0;
    return y;
}

// acc += sum over the row's nodes x0 <= xq < x1 of (W f)_xq / |r - x_q| for the lane's NB
// boundary nodes.  The inverse distances of U nodes are formed together (independent chains,
// one scalar load of their coordinates), then their R weighted values are read as
// wave-uniform operands.  U = 8 for wide tiles (36 sources of 16^3 elements, p = 4: U = 4
// 36.4 ms, 6 34.4, 8 33.6, 16 47.5 with 3 waves per SIMD); narrow tiles keep 4, and so does
// the widest (48 accumulators: with U = 8 it would drop to 3 waves per SIMD).
template <int R, int NB, bool MASK>
__device__ __forceinline__ void quad_run(const double (&bx)[NB], const double (&d2)[NB],
                                         const double* __restrict__ xs, const double* __restrict__ row, int x0,
                                         int x1, double drop2, double (&acc)[NB][R]) {
    constexpr int U = NB == 1 ? (R >= 24 && R <= 40 ? 8 : 4) : 2;
    int xq = x0;
    for (; xq + U <= x1; xq += U) {
        double y[U][NB];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < NB; ++k) y[u][k] = inv_dist<MASK>(bx[k], d2[k], xs[xq + u], drop2);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double* wf = row + (long long)(xq + u) * R;
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int k = 0; k < NB; ++k) acc[k][r] = fma(wf[r], y[u][k], acc[k][r]);
        }
    }
    for (; xq < x1; ++xq) {
        double y[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) y[k] = inv_dist<MASK>(bx[k], d2[k], xs[xq], drop2);
        const double* wf = row + (long long)xq * R;
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < NB; ++k) acc[k][r] = fma(wf[r], y[k], acc[k][r]);
    }
}

// Work-groups are dispatched to the eight XCDs round robin (w % 8).  Give XCD x a contiguous
// range of the logical work-group order, in which consecutive work-groups are the boundary
// tiles of one part of the lattice: the tiles in flight on an XCD then stream the same
// records through its L2.
__device__ __forceinline__ int quad_xcd_remap(int w, int G) {
    constexpr int NXCD = 8;
    if (G < NXCD) return w;
    const int x = w % NXCD, slot = w / NXCD;
    const int base = G / NXCD, rem = G % NXCD;
    return x * base + min(x, rem) + slot;
}

// boundary node -> lattice indices (face order x-, x+ [Z][Y]; y-, y+ [Z][X]; z-, z+ [Y][X])
__device__ __forceinline__ void face_node(int bb, int NX, int NY, int NZ, int& X, int& Y, int& Z) {
    const int fx = NZ * NY, fy = NZ * NX, fz = NY * NX;
    if (bb < 2 * fx) {
        const int side = bb >= fx, rem = bb - side * fx;
        Z = rem / NY; Y = rem % NY; X = side ? NX - 1 : 0;
    } else if (bb < 2 * fx + 2 * fy) {
        const int t = bb - 2 * fx, side = t >= fy, rem = t - side * fy;
        Z = rem / NX; X = rem % NX; Y = side ? NY - 1 : 0;
    } else {
        const int t = bb - 2 * fx - 2 * fy, side = t >= fz, rem = t - side * fz;
        Y = rem / NX; X = rem % NX; Z = side ? NZ - 1 : 0;
    }
}

template <int R>
__global__ __launch_bounds__(QUAD_BLOCK) void k_quad(const double* __restrict__ xs, const double* __restrict__ ys,
                                              const double* __restrict__ zs, int NX, int NY, int NZ, int nface,
                                              int zper, int ntb, double drop2, const double* __restrict__ rec,
                                              double* __restrict__ out, int nsrc, int r0, int direct) {
    constexpr int NB = QUAD_NB;
    // logical work-group: boundary tile (fastest) and part of the lattice
    const int w = quad_xcd_remap(blockIdx.x, gridDim.x);
    const int tile = w % ntb, part = w / ntb;
    int bnode[NB];
    double bx[NB], by[NB], bz[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        bnode[k] = tile * (QUAD_BLOCK * NB) + k * QUAD_BLOCK + threadIdx.x;
        int X, Y, Z;
        face_node(bnode[k] < nface ? bnode[k] : nface - 1, NX, NY, NZ, X, Y, Z);
        bx[k] = xs[X]; by[k] = ys[Y]; bz[k] = zs[Z];
    }
    double acc[NB][R];
#pragma unroll
    for (int k = 0; k < NB; ++k)
#pragma unroll
        for (int r = 0; r < R; ++r) acc[k][r] = 0.0;
    const int z0 = part * zper, z1 = min(NZ, z0 + zper);
    for (int zq = z0; zq < z1; ++zq) {
        double dz2[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            const double dz = bz[k] - zs[zq];
            dz2[k] = dz * dz;
        }
        const bool zedge = zq == 0 || zq == NZ - 1;
        for (int yq = 0; yq < NY; ++yq) {
            double d2[NB];
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                const double dy = by[k] - ys[yq];
                d2[k] = fma(dy, dy, dz2[k]);
            }
            const double* row = rec + ((long long)zq * NY + yq) * NX * R;
            // a row on the lattice's boundary surface is tested node by node; any other row
            // only at its two end nodes (x faces).  Three consecutive ranges, no branches,
            // so that one set of accumulators serves all of them.
            const bool edge = zedge || yq == 0 || yq == NY - 1;
            const int m1 = edge ? NX : 1, u1 = edge ? NX : NX - 1;
            quad_run<R, NB, true>(bx, d2, xs, row, 0, m1, drop2, acc);
            quad_run<R, NB, false>(bx, d2, xs, row, m1, u1, drop2, acc);
            quad_run<R, NB, true>(bx, d2, xs, row, u1, NX, drop2, acc);
        }
    }
    // direct: out is g [nsrc][nface]; else the split's partial sums [split][R][nface]
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        if (bnode[k] >= nface) continue;
        double* o = direct ? out + (long long)r0 * nface + bnode[k] : out + (long long)part * R * nface + bnode[k];
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (r0 + r < nsrc) o[(long long)r * nface] = acc[k][r];
    }
}

__global__ __launch_bounds__(256) void k_quad_sum(const double* __restrict__ part, int S, int R, int nface,
                                                  int nsrc, int r0, double* __restrict__ g) {
    const long long t = blockIdx.x * 256LL + threadIdx.x;
    const int nr = min(R, nsrc - r0);
    if (t >= (long long)nr * nface) return;
    double acc = 0.0;
    for (int s = 0; s < S; ++s) acc += part[(long long)s * R * nface + t];
    g[(long long)r0 * nface + t] = acc;
}

template <int R>
void launch_quad_r(int ntb, int S, const double* nodes, int NX, int NY, int NZ, int nface, int zper, double drop2,
                   const double* rec, double* out, int nsrc, int r0, int direct, hipStream_t s) {
    hipLaunchKernelGGL(k_quad<R>, dim3((unsigned)(ntb * S)), dim3(QUAD_BLOCK), 0, s, nodes, nodes + NX,
                       nodes + NX + NY, NX, NY, NZ, nface, zper, ntb, drop2, rec, out, nsrc, r0, direct);
}

}  // namespace

// Work space of the entry point that allocates nothing (dg_boundary_data_noalloc): the packed
// records and the split partial sums live in this array, one copy per GPU, kept until the
// process ends.  Host code never uses its name as an address: quad_scratch_init looks up each
// device's copy once and quad_scratch returns it.  Every call on a GPU shares that GPU's copy.
constexpr long long QUAD_SCRATCH_DOUBLES = 8LL << 20;  // 64 MiB
static __device__ __align__(256) double scratch[QUAD_SCRATCH_DOUBLES];

namespace {
constexpr int QUAD_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch[QUAD_MAX_DEVICES] = {};
}  // namespace

hipError_t quad_scratch_init(int device) {
    if (device < 0 || device >= QUAD_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[device] = static_cast<double*>(p);
    return hipSuccess;
}

double* quad_scratch(int device, long long* capacity) {
    if (capacity) *capacity = QUAD_SCRATCH_DOUBLES;
    if (device < 0 || device >= QUAD_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch[device];
}

QuadPlan quad_plan(const LevelHost& L, int nsrc) {
    QuadPlan P{};
    const long long NX = (long long)L.E[0] * L.n, NY = (long long)L.E[1] * L.n, NZ = (long long)L.E[2] * L.n;
    P.nface = 2 * (NZ * NY + NZ * NX + NY * NX);
    P.ntile = std::max(1, (nsrc + QUAD_RMAX - 1) / QUAD_RMAX);
    const int per = (nsrc + P.ntile - 1) / P.ntile;
    P.R = per < 4 ? per : (per + 3) / 4 * 4;  // 1-3 sources (a single density) unpadded
    const long long wpb = QUAD_BLOCK / 64, blocks = (P.nface + QUAD_BLOCK * QUAD_NB - 1) / (QUAD_BLOCK * QUAD_NB);
    const long long want = (QUAD_WAVES + wpb * blocks - 1) / (wpb * blocks);
    const int S0 = (int)std::max(1LL, std::min(NZ, want));
    P.zper = (int)((NZ + S0 - 1) / S0);
    P.S = (int)((NZ + P.zper - 1) / P.zper);
    P.rec_len = L.ndof * P.R;
    P.part_len = P.S > 1 ? (long long)P.S * P.R * P.nface : 0;
    return P;
}

// A plan whose records and partial sums fit in `capacity` doubles: the widest source tile that
// still leaves room for enough split parts to give the launch about a thousand work-groups (or
// the most it can), narrower tiles meaning more passes over the grid.  R = 0: the mesh does not
// fit even with one source per pass and no split.
QuadPlan quad_plan_bounded(const LevelHost& L, int nsrc, long long capacity) {
    const QuadPlan full = quad_plan(L, nsrc);
    if (nsrc <= 0 || full.rec_len + full.part_len <= capacity) return full;
    static const int tiles[] = {48, 44, 40, 36, 32, 28, 24, 20, 16, 12, 8, 4, 3, 2, 1};
    const long long NZ = (long long)L.E[2] * L.n;
    const long long ntb = (full.nface + QUAD_BLOCK * QUAD_NB - 1) / (QUAD_BLOCK * QUAD_NB);
    QuadPlan best{};
    long long best_wg = -1;
    for (int R : tiles) {
        if (R > full.R) continue;
        const long long rec = L.ndof * R;
        if (rec > capacity) continue;
        const long long smax = std::min<long long>(full.S, (capacity - rec) / ((long long)R * full.nface));
        const int S0 = (int)std::max(1LL, std::min(NZ, smax));
        QuadPlan P = full;
        P.R = R;
        P.ntile = (nsrc + R - 1) / R;
        P.zper = (int)((NZ + S0 - 1) / S0);
        P.S = (int)((NZ + P.zper - 1) / P.zper);
        P.rec_len = rec;
        P.part_len = P.S > 1 ? (long long)P.S * R * P.nface : 0;
        if (P.rec_len + P.part_len > capacity) continue;
        const long long wg = ntb * P.S;
        if (wg > best_wg) {
            best = P;
            best_wg = wg;
        }
        if (wg >= std::min<long long>(1024, ntb * full.S)) return P;
    }
    return best;  // R = 0 when nothing fits
}

void launch_quad_data(const LevelHost& L, const LevelDev<double>* dev, const double* nodes, const QuadPlan& P,
                      int nsrc, const double* f, const double* phi, const int* pi, const int* pj, double* rec,
                      double* part, double* g, hipStream_t s) {
    if (nsrc <= 0) return;
    const int NX = L.E[0] * L.n, NY = L.E[1] * L.n, NZ = L.E[2] * L.n;
    if (P.nface != 2 * ((long long)NZ * NY + (long long)NZ * NX + (long long)NY * NX) || P.nface > (1LL << 30) ||
        P.R < 1 || P.R > QUAD_RMAX || (P.R > 3 && P.R % 4) || (P.S > 1 && !part) || (long long)P.S * P.zper < NZ)
        throw std::logic_error("quadrature plan does not fit the mesh");
    const double hmin = std::min({L.h[0], L.h[1], L.h[2]});
    const double drop2 = (1e-6 * hmin) * (1e-6 * hmin);
    const int nface = (int)P.nface;
    const int ntb = (nface + QUAD_BLOCK * QUAD_NB - 1) / (QUAD_BLOCK * QUAD_NB);
    if ((long long)ntb * P.S >= (1LL << 31)) throw std::logic_error("quadrature grid too large");
    for (int r0 = 0; r0 < nsrc; r0 += P.R) {
        hipLaunchKernelGGL(k_quad_pack, dim3((unsigned)((L.ndof + 255) / 256)), dim3(256), 0, s, dev, L.E[0], L.E[1],
                           L.n, L.ndof, NX, NY, nsrc, r0, P.R, f, phi, pi, pj, rec);
        const int direct = P.S == 1;
        double* out = direct ? g : part;
        switch (P.R) {
#define QUAD_CASE(RR) \
    case RR: launch_quad_r<RR>(ntb, P.S, nodes, NX, NY, NZ, nface, P.zper, drop2, rec, out, nsrc, r0, direct, s); break;
            QUAD_CASE(1) QUAD_CASE(2) QUAD_CASE(3) QUAD_CASE(4) QUAD_CASE(8) QUAD_CASE(12) QUAD_CASE(16) QUAD_CASE(20) QUAD_CASE(24)
            QUAD_CASE(28) QUAD_CASE(32) QUAD_CASE(36) QUAD_CASE(40) QUAD_CASE(44) QUAD_CASE(48)
#undef QUAD_CASE
            default: throw std::logic_error("no quadrature kernel for this tile");
        }
        if (!direct) {
            const long long cnt = (long long)std::min(P.R, nsrc - r0) * nface;
            hipLaunchKernelGGL(k_quad_sum, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, part, P.S, P.R,
                               nface, nsrc, r0, g);
        }
    }
}

}  // namespace dg
