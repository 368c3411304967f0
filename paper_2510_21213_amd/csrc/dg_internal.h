// Internal declarations shared by the host set-up code, the kernels and the
// C ABI of the DG Poisson library.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/dg_poisson.h"

namespace dg {

constexpr int NMAX = 8;        // nodes per element edge (p <= 7)
constexpr int NBMAX = 16;      // nodes per brick edge
constexpr int CMAX = 16;       // coarsest level: nodes per axis

// One coordinate direction of one multigrid level, in the precision T of the
// kernels that read it.  Element blocks are indexed by the position type
// t = (left boundary ? 1 : 0) | (right boundary ? 2 : 0).
template <typename T>
struct AxisDev {
    T B[4][NMAX][NMAX];  // diagonal 1D block of an element (volume + own-face terms)
    T Bd[4][NMAX];       // diagonal of B
    T dL[NMAX];          // u -> u'(left end of the element)
    T dR[NMAX];          // u -> u'(right end of the element)
    T eL[NMAX];          // u -> u(left end of the element): the first node for GLL
    T eR[NMAX];          // u -> u(right end of the element): the last node for GLL
    T m[NMAX];           // mass at the nodes J*w (lumped for GLL, exact for GL)
    T liftL[NMAX];       // boundary lift of the left boundary element
    T liftR[NMAX];       // boundary lift of the right boundary element
    T sigma;             // penalty of this level along this axis
    int E;               // elements along this axis
    int gl;              // 1: Gauss-Legendre nodes (face values by eL / eR), 0: Gauss-Lobatto
};

// Reference-element form of a level's interior 1D block, shared by the three
// axes.  On an axis of element half-width J the interior block is B/J, the
// face-derivative rows aL/J and aR/J, the penalty sig/J and the lumped mass
// J w; so the x term of the operator is (J_y J_z / J_x) B (x) w (x) w, and
// scale[d] holds that factor for axis d.  Elements on a domain face use the
// same block: the Nitsche terms follow from ghost face data (see elem_op).
template <typename T>
struct RefDev {
    T B[NMAX][NMAX];
    T aL[NMAX], aR[NMAX];
    T w[NMAX];
    T sig;
    T scale[3];
    // Even/odd form of the block and of the face coupling (H = n/2 mirrored pairs
    // (i, p-i)): Pe/Po = (B_il +- B_i,p-l)/2, Bm[i] = B_iH (odd n, i <= H),
    // qe/qo = (aR_i -+ aL_i)/4, qm = aR_H/2.
    T Pe[NMAX / 2][NMAX / 2], Po[NMAX / 2][NMAX / 2];
    T Bm[NMAX / 2 + 1];
    T qe[NMAX / 2], qo[NMAX / 2], qm;
};

template <typename T>
struct LevelDev {
    AxisDev<T> ax[3];
    RefDev<T> ref;
};

// Brick-level 1D transfer between a level and the next coarser one:
// P[a][b] maps coarse brick node b to fine brick node a.
struct TransferDev {
    double P[NBMAX][NBMAX];
    float Pf[NBMAX][NBMAX];
};

// Coarsest level exact solve: S = M^{-1/2}, S A1 S = Q diag(lam) Q^T per axis.
struct CoarseDev {
    double Q[3][CMAX][CMAX];
    double lam[3][CMAX];
    double s[3][CMAX];
    int n[3];      // nodes per axis
    int E[3];      // elements per axis
    int N;         // nodes per element edge
    int pad;
};

// Per right-hand-side iteration state (device).
struct RhsState {
    double bb;      // ||b||^2
    double rz;      // r.z of this iteration
    double rz_old;  // r.z of the previous iteration
    double rz_prev; // flexible CG: r.z of the iteration before (the denominator of Polak-Ribiere beta)
    double pq;      // p.Ap
    double rr;      // r.r
    double alpha, beta;
    double tol2;    // (rtol)^2
    double scale;   // iterative refinement: ||r_outer||
    double cr, cac; // learned coarse-grid correction: c.r and c.Ac of the network's correction c
    int active;     // 1 while iterating
    int iters;      // completed iterations
    int maxit;
    int breakdown;
    int guess;      // 1 when a supplied initial guess passed the guard (its residual is below ||b||)
};

// Host description of one level.
struct LevelHost {
    int E[3];
    int p, n;
    int family = 0;  // node family (dg_opts.node_family)
    double h[3], lo[3];
    long long ndof;
    double lam_lo = 0, lam_hi = 0;
    LevelDev<double> d64;
    LevelDev<float> d32;
    LevelDev<double>* dev64 = nullptr;  // device copies
    LevelDev<float>* dev32 = nullptr;
    double* dinv64 = nullptr;  // inverse diagonal of the level's operator, one value per node (device)
    float* dinv32 = nullptr;
    // transfer to the next coarser level (unused on the coarsest)
    bool hcoarse = false;
    TransferDev tr;
    TransferDev* devtr = nullptr;
    int nbr[3];      // bricks per axis
    int be;          // elements per brick edge
    // slab-kernel tile per arithmetic (0 FP32, 1 FP64) and operator step (BrickMode):
    // {tx, ty, zlen}; tx = 0 selects the brick kernel.  Fixed when the level is set up.
    int tile[2][7][3];
};

// Host-side numerics (dg_setup.cpp).
void gll(int p, std::vector<double>& xi, std::vector<double>& w, std::vector<double>& D);
void gl(int p, std::vector<double>& xi, std::vector<double>& w, std::vector<double>& D);
// the nodes, weights and derivative matrix of a node family (0 GLL, 1 GL)
void node_rule(int p, int family, std::vector<double>& xi, std::vector<double>& w, std::vector<double>& D);
void lagrange_eval(const std::vector<double>& nodes, const std::vector<double>& x, std::vector<double>& L);
void lagrange_deriv(const std::vector<double>& nodes, const std::vector<double>& x, std::vector<double>& G);
void jacobi_eigen(int n, std::vector<double>& A, std::vector<double>& lam, std::vector<double>& V);
void build_axis(int E, int p, double lo, double hi, double eps, AxisDev<double>& ax, std::vector<double>* dense,
                std::vector<double>* nodes, int family = 0);
void build_ref(int p, double eps, const double h[3], RefDev<double>& r);
int brick_edge(int n);
std::vector<std::pair<std::array<int, 3>, int>> hierarchy(const int E[3], int p, int n_levels);
void build_transfer(const LevelHost& fine, const LevelHost& coarse, TransferDev& tr);
void build_coarse(const LevelHost& L, double eps, CoarseDev& c);
double tridiag_max_eig(const std::vector<double>& a, const std::vector<double>& b);

// C ABI error handling shared by the library's modules (dg_api.hip): run fn, map its exceptions to
// a status and the message of dg_last_error(); hip_fail throws the HIP error kind.
dg_status guarded(const std::function<void()>& fn);
[[noreturn]] void hip_fail(const std::string& what);

}  // namespace dg
