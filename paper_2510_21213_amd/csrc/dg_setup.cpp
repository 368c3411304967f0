// Host-side numerics of the DG Poisson library: reference element, 1D SIPDG
// element blocks, multigrid hierarchy and transfers, and the eigendata of the
// coarsest-level exact solve.  Everything here runs once per mesh at set-up.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <stdexcept>

#include "dg_internal.h"

namespace dg {

// Legendre P_p(x) and P_p'(x) by the three-term recurrence.
static void legendre(int p, double x, double& P, double& dP) {
    double pm = 1.0, pc = x;
    if (p == 0) { P = 1.0; dP = 0.0; return; }
    for (int k = 1; k < p; ++k) {
        double pn = ((2.0 * k + 1.0) * x * pc - k * pm) / (k + 1.0);
        pm = pc;
        pc = pn;
    }
    P = pc;
    // (1 - x^2) P_p' = p (P_{p-1} - x P_p)
    dP = (std::fabs(1.0 - x * x) > 0.0) ? p * (pm - x * pc) / (1.0 - x * x) : 0.5 * p * (p + 1) * std::pow(x, p + 1);
}

// Gauss-Lobatto-Legendre nodes (end points and the roots of P_p'), weights
// 2/(p(p+1) P_p(x_i)^2) and the derivative matrix D[i][j] = l_j'(x_i).
void gll(int p, std::vector<double>& xi, std::vector<double>& w, std::vector<double>& D) {
    const int n = p + 1;
    xi.assign(n, 0.0);
    w.assign(n, 0.0);
    D.assign(n * n, 0.0);
    xi[0] = -1.0;
    xi[p] = 1.0;
    for (int i = 1; i < p; ++i) {
        double x = -std::cos(M_PI * i / p);  // Chebyshev-Lobatto start
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre(p, x, P, dP);
            // q = P_p', q' = P_p'' from (1-x^2) P'' = 2x P' - p(p+1) P
            double ddP = (2.0 * x * dP - p * (p + 1.0) * P) / (1.0 - x * x);
            double dx = dP / ddP;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        xi[i] = x;
    }
    std::sort(xi.begin(), xi.end());
    std::vector<double> Pv(n);
    for (int i = 0; i < n; ++i) {
        double P, dP;
        legendre(p, xi[i], P, dP);
        Pv[i] = P;
        w[i] = 2.0 / (p * (p + 1.0) * P * P);
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            if (i != j) D[i * n + j] = Pv[i] / (Pv[j] * (xi[i] - xi[j]));
    D[0] = -p * (p + 1.0) / 4.0;
    D[p * n + p] = p * (p + 1.0) / 4.0;
}

// Gauss-Legendre nodes (the roots of P_{p+1}, by Newton's method from the usual cosine
// estimates), weights 2 / ((1 - x^2) P_{p+1}'(x)^2) and the derivative matrix D[i][j] = l_j'(x_i).
void gl(int p, std::vector<double>& xi, std::vector<double>& w, std::vector<double>& D) {
    const int n = p + 1;
    xi.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double x = -std::cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre(n, x, P, dP);
            const double dx = P / dP;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        xi[i] = x;
    }
    std::sort(xi.begin(), xi.end());
    for (int i = 0; i < n; ++i) {
        double P, dP;
        legendre(n, xi[i], P, dP);
        w[i] = 2.0 / ((1.0 - xi[i] * xi[i]) * dP * dP);
    }
    std::vector<double> G;
    lagrange_deriv(xi, xi, G);
    D = G;
}

void node_rule(int p, int family, std::vector<double>& xi, std::vector<double>& w, std::vector<double>& D) {
    if (family == 1)
        gl(p, xi, w, D);
    else
        gll(p, xi, w, D);
}

// G[a*n + j] = l_j'(x_a): the product rule on the product formula of the Lagrange basis.
void lagrange_deriv(const std::vector<double>& nodes, const std::vector<double>& x, std::vector<double>& G) {
    const int n = (int)nodes.size(), m = (int)x.size();
    G.assign((size_t)m * n, 0.0);
    for (int a = 0; a < m; ++a)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                if (k == j) continue;
                double term = 1.0 / (nodes[j] - nodes[k]);
                for (int q = 0; q < n; ++q)
                    if (q != j && q != k) term *= (x[a] - nodes[q]) / (nodes[j] - nodes[q]);
                G[a * n + j] += term;
            }
}

// L[a*n + j] = l_j(x_a), Lagrange basis on `nodes`, product formula.
void lagrange_eval(const std::vector<double>& nodes, const std::vector<double>& x, std::vector<double>& L) {
    const int n = (int)nodes.size(), m = (int)x.size();
    L.assign((size_t)m * n, 1.0);
    for (int a = 0; a < m; ++a)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k)
                if (k != j) L[a * n + j] *= (x[a] - nodes[k]) / (nodes[j] - nodes[k]);
}

// Cyclic Jacobi eigenvalue iteration for a symmetric n x n matrix (row-major).
// On exit lam is ascending and column k of V (V[i*n+k]) its eigenvector.
void jacobi_eigen(int n, std::vector<double>& A, std::vector<double>& lam, std::vector<double>& V) {
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += A[i * n + j] * A[i * n + j];
                if (i != j) off += A[i * n + j] * A[i * n + j];
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = A[p * n + q];
                if (apq == 0.0) continue;
                double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {  // A <- A J (columns p, q)
                    double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // A <- J^T A (rows p, q)
                    double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    double vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = c * vkp - s * vkq;
                    V[k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    std::vector<int> ord(n);
    for (int i = 0; i < n; ++i) ord[i] = i;
    std::sort(ord.begin(), ord.end(), [&](int a, int b) { return A[a * n + a] < A[b * n + b]; });
    std::vector<double> V2((size_t)n * n);
    lam.assign(n, 0.0);
    for (int k = 0; k < n; ++k) {
        lam[k] = A[ord[k] * n + ord[k]];
        for (int i = 0; i < n; ++i) V2[i * n + k] = V[i * n + ord[k]];
    }
    V.swap(V2);
}

double tridiag_max_eig(const std::vector<double>& a, const std::vector<double>& b) {
    const int n = (int)a.size();
    std::vector<double> T((size_t)n * n, 0.0), lam, V;
    for (int i = 0; i < n; ++i) {
        T[i * n + i] = a[i];
        if (i + 1 < n) T[i * n + i + 1] = T[(i + 1) * n + i] = b[i];
    }
    jacobi_eigen(n, T, lam, V);
    return lam[n - 1];
}

// One axis of one level: E uniform elements of degree p on [lo, hi].
// Element block for position type t (bit 0: left boundary, bit 1: right
// boundary): local stiffness plus the own-element parts of the face terms of
// eq. (sip_bilinear); boundary faces carry the symmetric Nitsche terms.
// Optionally returns the dense 1D matrix and the node coordinates.  The face terms use the
// element's traces: eL, eR (the values at its ends) and dL, dR (the derivatives there); for GLL
// eL and eR pick the end nodes, for GL they are the Lagrange basis evaluated at -1 and +1.
void build_axis(int E, int p, double lo, double hi, double eps, AxisDev<double>& ax, std::vector<double>* dense,
                std::vector<double>* nodes, int family) {
    const int n = p + 1;
    std::vector<double> xi, w, D;
    node_rule(p, family, xi, w, D);
    const double h = (hi - lo) / E, J = 0.5 * h;
    const double sigma = (p + 1.0) * (p + 1.0) / (eps * h);
    std::memset(&ax, 0, sizeof(ax));
    ax.E = E;
    ax.sigma = sigma;
    double K[NMAX][NMAX] = {};
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int q = 0; q < n; ++q) s += D[q * n + i] * w[q] * D[q * n + j];
            K[i][j] = s / J;
        }
    ax.gl = family == 1;
    if (family == 1) {
        std::vector<double> ends = {-1.0, 1.0}, Le, Ge;
        lagrange_eval(xi, ends, Le);
        lagrange_deriv(xi, ends, Ge);
        for (int l = 0; l < n; ++l) {
            ax.eL[l] = Le[l];
            ax.eR[l] = Le[n + l];
            ax.dL[l] = Ge[l] / J;
            ax.dR[l] = Ge[n + l] / J;
        }
    } else {
        for (int l = 0; l < n; ++l) {
            ax.eL[l] = (l == 0);
            ax.eR[l] = (l == p);
            ax.dL[l] = D[0 * n + l] / J;
            ax.dR[l] = D[p * n + l] / J;
        }
    }
    for (int l = 0; l < n; ++l) ax.m[l] = J * w[l];
    for (int t = 0; t < 4; ++t) {
        const bool lb = t & 1, rb = t & 2;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double v = K[i][j];
                const double eLi = ax.eL[i], eLj = ax.eL[j], eRi = ax.eR[i], eRj = ax.eR[j];
                if (lb)  // Nitsche, left boundary: j = e_L, g = -d_L
                    v += eLi * ax.dL[j] + ax.dL[i] * eLj + sigma * eLi * eLj;
                else     // interior face on the left, this element on its plus side
                    v += 0.5 * (eLi * ax.dL[j] + ax.dL[i] * eLj) + sigma * eLi * eLj;
                if (rb)  // Nitsche, right boundary: j = e_R, g = +d_R
                    v += -(eRi * ax.dR[j] + ax.dR[i] * eRj) + sigma * eRi * eRj;
                else     // interior face on the right, this element on its minus side
                    v += -0.5 * (eRi * ax.dR[j] + ax.dR[i] * eRj) + sigma * eRi * eRj;
                ax.B[t][i][j] = v;
            }
        for (int i = 0; i < n; ++i) ax.Bd[t][i] = ax.B[t][i][i];
    }
    for (int i = 0; i < n; ++i) {
        ax.liftL[i] = sigma * ax.eL[i] + ax.dL[i];
        ax.liftR[i] = sigma * ax.eR[i] - ax.dR[i];
    }
    if (dense) {
        const int N = E * n;
        dense->assign((size_t)N * N, 0.0);
        auto& A = *dense;
        for (int e = 0; e < E; ++e) {
            int t = (e == 0 ? 1 : 0) | (e == E - 1 ? 2 : 0);
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) A[(size_t)(e * n + i) * N + e * n + j] += ax.B[t][i][j];
            if (e + 1 < E) {  // coupling to the right neighbour: -1/2 e_R d_L^T + 1/2 d_R e_L^T - sigma e_R e_L^T
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < n; ++j) {
                        double v = -0.5 * ax.eR[i] * ax.dL[j] + 0.5 * ax.dR[i] * ax.eL[j] - sigma * ax.eR[i] * ax.eL[j];
                        A[(size_t)(e * n + i) * N + (e + 1) * n + j] += v;
                        A[(size_t)((e + 1) * n + j) * N + e * n + i] += v;
                    }
            }
        }
    }
    if (nodes) {
        nodes->resize((size_t)E * n);
        for (int e = 0; e < E; ++e)
            for (int i = 0; i < n; ++i) (*nodes)[e * n + i] = lo + e * h + J * (xi[i] + 1.0);
    }
}

// Interior block in reference units (J = 1): stiffness D^T diag(w) D plus the
// own-element halves of both interior faces; the penalty sigma J =
// (p+1)^2 / (2 eps) follows from sigma = (p+1)^2 / (eps h) with h = 2J.
void build_ref(int p, double eps, const double h[3], RefDev<double>& r) {
    const int n = p + 1;
    std::vector<double> xi, w, D;
    gll(p, xi, w, D);
    std::memset(&r, 0, sizeof(r));
    const double sig = (p + 1.0) * (p + 1.0) / (2.0 * eps);
    r.sig = sig;
    for (int l = 0; l < n; ++l) {
        r.aL[l] = D[0 * n + l];
        r.aR[l] = D[p * n + l];
        r.w[l] = w[l];
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double v = 0.0;
            for (int q = 0; q < n; ++q) v += D[q * n + i] * w[q] * D[q * n + j];
            const double eLi = (i == 0), eLj = (j == 0), eRi = (i == p), eRj = (j == p);
            v += 0.5 * (eLi * r.aL[j] + r.aL[i] * eLj) + sig * eLi * eLj;
            v += -0.5 * (eRi * r.aR[j] + r.aR[i] * eRj) + sig * eRi * eRj;
            r.B[i][j] = v;
        }
    const int H = n / 2;
    for (int i = 0; i < H; ++i) {
        for (int l = 0; l < H; ++l) {
            r.Pe[i][l] = 0.5 * (r.B[i][l] + r.B[i][n - 1 - l]);
            r.Po[i][l] = 0.5 * (r.B[i][l] - r.B[i][n - 1 - l]);
        }
        r.qe[i] = 0.25 * (r.aR[i] - r.aL[i]);
        r.qo[i] = 0.25 * (r.aR[i] + r.aL[i]);
    }
    if (n & 1) {
        for (int i = 0; i <= H; ++i) r.Bm[i] = r.B[i][H];
        r.qm = 0.5 * r.aR[H];
    }
    const double J[3] = {0.5 * h[0], 0.5 * h[1], 0.5 * h[2]};
    r.scale[0] = J[1] * J[2] / J[0];
    r.scale[1] = J[0] * J[2] / J[1];
    r.scale[2] = J[0] * J[1] / J[2];
}

int brick_edge(int n) { return n <= 3 ? 4 : (n <= 6 ? 2 : 1); }

// Levels from fine to coarse: degree p -> p/2 -> ... -> 1, then halve the
// element counts while all are even, until `n_levels` levels exist or (when
// n_levels is 0) the coarsest level has at most CMAX nodes per axis.
std::vector<std::pair<std::array<int, 3>, int>> hierarchy(const int E[3], int p, int n_levels) {
    std::vector<std::pair<std::array<int, 3>, int>> lv;
    lv.push_back({{E[0], E[1], E[2]}, p});
    while (true) {
        auto [Ec, pc] = lv.back();
        if (n_levels > 0 && (int)lv.size() >= n_levels) break;
        if (pc > 1) { lv.push_back({Ec, pc / 2}); continue; }
        int mx = std::max(Ec[0], std::max(Ec[1], Ec[2]));
        if (n_levels == 0 && mx * (pc + 1) <= CMAX) break;
        if ((Ec[0] | Ec[1] | Ec[2]) & 1) {
            if (n_levels > 0) throw std::runtime_error("cannot build the requested number of levels");
            break;
        }
        lv.push_back({{Ec[0] / 2, Ec[1] / 2, Ec[2] / 2}, 1});
    }
    return lv;
}

// Brick-level interpolation from the coarse level to the fine one.  Degree
// step: same elements, I[i][j] = l^c_j(xi^f_i) block-diagonally.  Mesh step:
// fine element b takes its parent b/2 and child position c = b%2, with
// I_c[i][j] = l^c_j((xi^f_i + 2c - 1)/2).
void build_transfer(const LevelHost& fine, const LevelHost& coarse, TransferDev& tr) {
    std::memset(&tr, 0, sizeof(tr));
    std::vector<double> xf, wf, Df, xc, wc, Dc;
    node_rule(fine.p, fine.family, xf, wf, Df);
    node_rule(coarse.p, coarse.family, xc, wc, Dc);
    const int nf = fine.n, nc = coarse.n, be = fine.be;
    const bool hc = fine.E[0] != coarse.E[0];
    for (int b = 0; b < be; ++b) {
        std::vector<double> pts(nf), L;
        int cb;
        if (!hc) {
            pts = xf;
            cb = b;
        } else {
            for (int i = 0; i < nf; ++i) pts[i] = (xf[i] + 2.0 * (b % 2) - 1.0) / 2.0;
            cb = b / 2;
        }
        lagrange_eval(xc, pts, L);
        for (int i = 0; i < nf; ++i)
            for (int j = 0; j < nc; ++j) {
                tr.P[b * nf + i][cb * nc + j] = L[i * nc + j];
                tr.Pf[b * nf + i][cb * nc + j] = (float)L[i * nc + j];
            }
    }
}

void build_coarse(const LevelHost& L, double eps, CoarseDev& c) {
    std::memset(&c, 0, sizeof(c));
    c.N = L.n;
    for (int d = 0; d < 3; ++d) {
        AxisDev<double> ax;
        std::vector<double> A;
        build_axis(L.E[d], L.p, L.lo[d], L.lo[d] + L.h[d] * L.E[d], eps, ax, &A, nullptr, L.family);
        const int n = L.E[d] * L.n;
        if (n > CMAX) throw std::runtime_error("coarsest level too large for the exact solve");
        c.n[d] = n;
        c.E[d] = L.E[d];
        std::vector<double> s(n);
        for (int e = 0; e < L.E[d]; ++e)
            for (int i = 0; i < L.n; ++i) s[e * L.n + i] = 1.0 / std::sqrt(ax.m[i]);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) A[(size_t)i * n + j] *= s[i] * s[j];
        std::vector<double> lam, V;
        jacobi_eigen(n, A, lam, V);
        for (int i = 0; i < n; ++i) {
            c.s[d][i] = s[i];
            c.lam[d][i] = lam[i];
            for (int k = 0; k < n; ++k) c.Q[d][i][k] = V[i * n + k];
        }
    }
}

}  // namespace dg
