// Host-side 1D reference data of the method, in FP64.
//
// * Gauss-Lobatto points of [0,1] and the Lagrange basis on them.
// * Exact mass matrix M_hat (Gauss-Legendre quadrature with n+1 points, exact
//   for the degree-2p integrand) and stiffness K_hat = D^T M_hat D, where D is
//   the nodal differentiation matrix (l_j' is interpolated exactly by its
//   nodal values).  Sec. 3.1, eq. (eval_pipeline) needs only these two.
// * A_hat = K_hat + own-side SIPG face blocks of both faces, eq. (face_coupling)
//   and eq. (cell_block), penalty sigma_hat = C p (p+1) (Sec. 6.2).
// * Generalized symmetric eigen-decomposition P_hat S = M_hat S Lambda by
//   Cholesky reduction and cyclic Jacobi rotations (Golub & Van Loan,
//   "Matrix Computations", Sec. 8.5), giving the fast-diagonalization factors
//   of Sec. 5.2.
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace tpfdm {

namespace {

// Legendre P_k(x) and P_k'(x) by the three-term recurrence.
void legendre(int k, double x, double* P, double* dP) {
    double p0 = 1.0, p1 = x;
    if (k == 0) { *P = 1.0; *dP = 0.0; return; }
    for (int m = 1; m < k; ++m) {
        double p2 = ((2 * m + 1) * x * p1 - m * p0) / (m + 1);
        p0 = p1;
        p1 = p2;
    }
    *P = p1;
    // (1 - x^2) P_k' = k (P_{k-1} - x P_k)
    *dP = k * (p0 - x * p1) / (1.0 - x * x);
}

}  // namespace

// n Gauss-Lobatto points on [0,1]: the endpoints and the roots of P_{n-1}'
// found by Newton's method from Chebyshev-Gauss-Lobatto guesses.
void gll_points(int n, double* x) {
    const int p = n - 1;
    x[0] = 0.0;
    x[p] = 1.0;
    for (int k = 1; k < p; ++k) {
        double xi = -std::cos(M_PI * k / p);
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre(p, xi, &P, &dP);
            // Legendre ODE: (1 - x^2) P'' = 2 x P' - p(p+1) P
            double d2P = (2.0 * xi * dP - p * (p + 1) * P) / (1.0 - xi * xi);
            double step = dP / d2P;
            xi -= step;
            if (std::fabs(step) < 1e-17) break;
        }
        x[k] = 0.5 * (1.0 + xi);
    }
}

// nq Gauss-Legendre points and weights on [0,1] (Newton on P_nq).
void gauss_points(int nq, double* x, double* w) {
    for (int k = 0; k < nq; ++k) {
        double xi = -std::cos(M_PI * (k + 0.75) / (nq + 0.5));
        double P = 0, dP = 1;
        for (int it = 0; it < 100; ++it) {
            legendre(nq, xi, &P, &dP);
            double step = P / dP;
            xi -= step;
            if (std::fabs(step) < 1e-17) break;
        }
        legendre(nq, xi, &P, &dP);
        x[k] = 0.5 * (1.0 + xi);
        w[k] = 1.0 / ((1.0 - xi * xi) * dP * dP);  // 2/((1-xi^2)P'^2), halved for [0,1]
    }
}

void reference_matrices(int n, double C, double* M, double* K, double* A) {
    std::vector<double> x(n), bw(n), D(n * n), Mm(n * n, 0.0), Km(n * n, 0.0);
    gll_points(n, x.data());
    for (int j = 0; j < n; ++j) {
        double prod = 1.0;
        for (int k = 0; k < n; ++k)
            if (k != j) prod *= (x[j] - x[k]);
        bw[j] = 1.0 / prod;  // barycentric weights
    }
    // differentiation matrix D[i][j] = l_j'(x_i)
    for (int i = 0; i < n; ++i) {
        double diag = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            D[i * n + j] = (bw[j] / bw[i]) / (x[i] - x[j]);
            diag -= D[i * n + j];
        }
        D[i * n + i] = diag;
    }
    // mass matrix by Gauss-Legendre quadrature, Lagrange values by the
    // second (true) barycentric formula
    const int nq = n + 1;
    std::vector<double> xq(nq), wq(nq), L(n);
    gauss_points(nq, xq.data(), wq.data());
    for (int q = 0; q < nq; ++q) {
        int hit = -1;
        for (int j = 0; j < n; ++j)
            if (xq[q] == x[j]) hit = j;
        if (hit >= 0) {
            for (int j = 0; j < n; ++j) L[j] = (j == hit) ? 1.0 : 0.0;
        } else {
            double den = 0.0;
            for (int j = 0; j < n; ++j) den += bw[j] / (xq[q] - x[j]);
            for (int j = 0; j < n; ++j) L[j] = (bw[j] / (xq[q] - x[j])) / den;
        }
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) Mm[i * n + j] += wq[q] * L[i] * L[j];
    }
    // K = D^T M D
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            double s = 0.0;
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) s += D[i * n + a] * Mm[i * n + j] * D[j * n + b];
            Km[a * n + b] = s;
        }
    // symmetrize against rounding
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < a; ++b) {
            double m = 0.5 * (Mm[a * n + b] + Mm[b * n + a]);
            Mm[a * n + b] = Mm[b * n + a] = m;
            double k = 0.5 * (Km[a * n + b] + Km[b * n + a]);
            Km[a * n + b] = Km[b * n + a] = k;
        }
    if (M) std::copy(Mm.begin(), Mm.end(), M);
    if (K) std::copy(Km.begin(), Km.end(), K);
    if (A) {
        // own-side face blocks: right face (cell is K^-, endpoint 1) and left
        // face (cell is K^+, endpoint 0); value vectors are unit vectors for
        // the GLL basis, derivative vectors are rows of D.
        const double sigma = C * (n - 1) * n;
        std::copy(Km.begin(), Km.end(), A);
        const int r = n - 1;
        A[r * n + r] += sigma;
        A[0] += sigma;
        for (int j = 0; j < n; ++j) {
            const double g1 = D[r * n + j], g0 = D[0 * n + j];
            A[r * n + j] -= 0.5 * g1;
            A[j * n + r] -= 0.5 * g1;
            A[0 * n + j] += 0.5 * g0;
            A[j * n + 0] += 0.5 * g0;
        }
    }
}

// Endpoint derivatives of the n Lagrange functions on [0, 1]: g0[j] =
// l_j'(0), g1[j] = l_j'(1) (the vectors g of eq. (face_coupling) on the
// reference interval), rows 0 and n-1 of the nodal differentiation matrix.
void endpoint_derivatives(int n, double* g0, double* g1) {
    std::vector<double> x(n), bw(n);
    gll_points(n, x.data());
    for (int j = 0; j < n; ++j) {
        double prod = 1.0;
        for (int k = 0; k < n; ++k)
            if (k != j) prod *= (x[j] - x[k]);
        bw[j] = 1.0 / prod;
    }
    for (int r = 0; r < 2; ++r) {
        const int i = r == 0 ? 0 : n - 1;
        double* g = r == 0 ? g0 : g1;
        double diag = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            g[j] = (bw[j] / bw[i]) / (x[i] - x[j]);
            diag -= g[j];
        }
        g[i] = diag;
    }
}

// Embedding of a coarse cell's polynomial into its two children along one
// axis: P_c[i][j] = l_j((x_i + c) / 2), coarse Lagrange function j at node i
// of child c (left c = 0, right c = 1) in the parent's coordinates
// (barycentric evaluation; a node that coincides with a coarse node gives a
// unit row).
void prolongation_1d(int n, double* P0, double* P1) {
    std::vector<double> x(n), bw(n);
    gll_points(n, x.data());
    for (int j = 0; j < n; ++j) {
        double prod = 1.0;
        for (int k = 0; k < n; ++k)
            if (k != j) prod *= (x[j] - x[k]);
        bw[j] = 1.0 / prod;
    }
    for (int c = 0; c < 2; ++c) {
        double* P = c == 0 ? P0 : P1;
        for (int i = 0; i < n; ++i) {
            const double t = 0.5 * (x[i] + c);
            int hit = -1;
            for (int j = 0; j < n; ++j)
                if (t == x[j]) hit = j;
            if (hit >= 0) {
                for (int j = 0; j < n; ++j) P[i * n + j] = j == hit ? 1.0 : 0.0;
                continue;
            }
            double den = 0.0;
            for (int j = 0; j < n; ++j) den += bw[j] / (t - x[j]);
            for (int j = 0; j < n; ++j) P[i * n + j] = (bw[j] / (t - x[j])) / den;
        }
    }
}

// The Hermite-type basis of Sec. 3.1 (eq. (hermite_conditions)) for n >= 4
// points (degree p = n - 1 >= 3): psi_0, psi_1 carry the value and the
// derivative at 0, psi_{p-1}, psi_p the derivative and the value at 1, each
// the cubic Hermite polynomial with that endpoint datum; the p - 3 interior
// functions are Lagrange polynomials on the interior Gauss-Lobatto nodes of
// the (n-2)-point rule times the bubble x^2 (1-x)^2, so they have no value
// and no derivative at either end.  T[i * n + j] = psi_j(x_i) at the n
// Gauss-Lobatto nodes: nodal (Lagrange) coefficients = T * Hermite ones.
void hermite_transform(int n, double* T) {
    std::vector<double> x(n), z(std::max(n - 2, 2));
    gll_points(n, x.data());
    gll_points(std::max(n - 2, 2), z.data());
    const int nint = n - 4;   // interior functions, nodes z[1 .. n-4]
    for (int i = 0; i < n; ++i) {
        const double t = x[i], t2 = t * t, t3 = t2 * t;
        double* row = T + i * n;
        row[0] = 1.0 - 3.0 * t2 + 2.0 * t3;
        row[1] = t - 2.0 * t2 + t3;
        row[n - 2] = t3 - t2;
        row[n - 1] = 3.0 * t2 - 2.0 * t3;
        const double bubble = t2 * (1.0 - t) * (1.0 - t);
        for (int k = 0; k < nint; ++k) {
            double l = 1.0;
            for (int m = 0; m < nint; ++m)
                if (m != k) l *= (t - z[1 + m]) / (z[1 + k] - z[1 + m]);
            row[2 + k] = l * bubble;
        }
    }
}

// Inverse of a small dense matrix (row-major) by Gauss-Jordan elimination
// with partial pivoting; false when a pivot vanishes.
bool invert_small(int n, const double* A, double* Ai) {
    std::vector<double> W(static_cast<size_t>(n) * 2 * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < 2 * n; ++j) W[i * 2 * n + j] = j < n ? A[i * n + j] : (j - n == i ? 1.0 : 0.0);
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(W[r * 2 * n + c]) > std::fabs(W[piv * 2 * n + c])) piv = r;
        if (!(std::fabs(W[piv * 2 * n + c]) > 0.0)) return false;
        if (piv != c)
            for (int j = 0; j < 2 * n; ++j) std::swap(W[c * 2 * n + j], W[piv * 2 * n + j]);
        const double d = 1.0 / W[c * 2 * n + c];
        for (int j = 0; j < 2 * n; ++j) W[c * 2 * n + j] *= d;
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double f = W[r * 2 * n + c];
            if (f == 0.0) continue;
            for (int j = 0; j < 2 * n; ++j) W[r * 2 * n + j] -= f * W[c * 2 * n + j];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Ai[i * n + j] = W[i * 2 * n + n + j];
    return true;
}

// X <- T^T X T for a symmetric bilinear-form matrix X (row-major n x n).
void congruence(int n, const double* T, double* X) {
    std::vector<double> Y(static_cast<size_t>(n) * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += X[i * n + k] * T[k * n + j];
            Y[i * n + j] = s;
        }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += T[k * n + i] * Y[k * n + j];
            X[i * n + j] = s;
        }
}

// A vertex patch along one direction: two adjacent cells of nc points
// (degree nc - 1, the same length), n = 2 nc DoFs, cell 0's first.  Mass
// and stiffness are block-diagonal (one cell each); the patch operator has
// the cell block A_hat (the interior stencil: stiffness plus the own-side
// blocks of both faces) on each cell and, off the diagonal, the coupling of
// the face between them (eq. (face_coupling) with cell 0 on the '-' side):
//   N^{-+}[i][j] = -sigma e1_i e0_j - 1/2 e1_i g0_j + 1/2 g1_i e0_j,
// e0, e1 the unit vectors of the first and last point, g0, g1 the endpoint
// derivatives, sigma = C p (p+1); N^{+-} is its transpose.
void patch_reference(int nc, double C, double* M, double* K, double* A) {
    const int n = 2 * nc;
    double Mc[kMaxN * kMaxN], Kc[kMaxN * kMaxN], Ac[kMaxN * kMaxN], g0[kMaxN], g1[kMaxN];
    reference_matrices(nc, C, Mc, Kc, Ac);
    endpoint_derivatives(nc, g0, g1);
    const double sigma = C * (nc - 1) * nc;
    for (int i = 0; i < n * n; ++i) M[i] = K[i] = A[i] = 0.0;
    for (int b = 0; b < 2; ++b)
        for (int i = 0; i < nc; ++i)
            for (int j = 0; j < nc; ++j) {
                const int o = (b * nc + i) * n + b * nc + j;
                M[o] = Mc[i * nc + j];
                K[o] = Kc[i * nc + j];
                A[o] = Ac[i * nc + j];
            }
    for (int i = 0; i < nc; ++i)
        for (int j = 0; j < nc; ++j) {
            double v = 0.0;
            if (i == nc - 1 && j == 0) v -= sigma;
            if (i == nc - 1) v -= 0.5 * g0[j];
            if (j == 0) v += 0.5 * g1[i];
            A[i * n + nc + j] = v;
            A[(nc + j) * n + i] = v;
        }
}

// Generalized symmetric-definite eigenproblem P S = M S diag(lam).
// Returns 0 on success, -1 when M is not SPD.
int gen_eigen(int n, const double* M, const double* P, double* S, double* lam) {
    std::vector<double> L(n * n, 0.0);
    for (int j = 0; j < n; ++j) {
        double d = M[j * n + j];
        for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
        if (!(d > 0.0)) return -1;
        L[j * n + j] = std::sqrt(d);
        for (int i = j + 1; i < n; ++i) {
            double s = M[i * n + j];
            for (int k = 0; k < j; ++k) s -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = s / L[j * n + j];
        }
    }
    // Y = L^{-1} P  (forward substitution on each column)
    std::vector<double> Y(n * n), Cm(n * n);
    for (int c = 0; c < n; ++c)
        for (int i = 0; i < n; ++i) {
            double s = P[i * n + c];
            for (int k = 0; k < i; ++k) s -= L[i * n + k] * Y[k * n + c];
            Y[i * n + c] = s / L[i * n + i];
        }
    // C = L^{-1} Y^T  (= L^{-1} P L^{-T}, symmetric)
    for (int c = 0; c < n; ++c)
        for (int i = 0; i < n; ++i) {
            double s = Y[c * n + i];
            for (int k = 0; k < i; ++k) s -= L[i * n + k] * Cm[k * n + c];
            Cm[i * n + c] = s / L[i * n + i];
        }
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < a; ++b) {
            double m = 0.5 * (Cm[a * n + b] + Cm[b * n + a]);
            Cm[a * n + b] = Cm[b * n + a] = m;
        }
    // cyclic Jacobi
    std::vector<double> V(n * n, 0.0);
    for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += Cm[i * n + j] * Cm[i * n + j];
                if (i != j) off += Cm[i * n + j] * Cm[i * n + j];
            }
        if (off <= 1e-32 * tot) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = Cm[p * n + q];
                if (apq == 0.0) continue;
                const double tau = (Cm[q * n + q] - Cm[p * n + p]) / (2.0 * apq);
                const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                for (int k = 0; k < n; ++k) {  // C <- C J (columns p, q)
                    const double ckp = Cm[k * n + p], ckq = Cm[k * n + q];
                    Cm[k * n + p] = c * ckp - s * ckq;
                    Cm[k * n + q] = s * ckp + c * ckq;
                }
                for (int k = 0; k < n; ++k) {  // C <- J^T C (rows p, q)
                    const double cpk = Cm[p * n + k], cqk = Cm[q * n + k];
                    Cm[p * n + k] = c * cpk - s * cqk;
                    Cm[q * n + k] = s * cpk + c * cqk;
                }
                for (int k = 0; k < n; ++k) {  // V <- V J
                    const double vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = c * vkp - s * vkq;
                    V[k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    // S = L^{-T} V (back substitution on each column)
    std::vector<double> Sm(n * n);
    for (int c = 0; c < n; ++c)
        for (int i = n - 1; i >= 0; --i) {
            double s = V[i * n + c];
            for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * Sm[k * n + c];
            Sm[i * n + c] = s / L[i * n + i];
        }
    // sort ascending, fix signs
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::sort(order.begin(), order.end(),
              [&](int a, int b) { return Cm[a * n + a] < Cm[b * n + b]; });
    for (int jj = 0; jj < n; ++jj) {
        const int j = order[jj];
        lam[jj] = Cm[j * n + j];
        int imax = 0;
        for (int i = 1; i < n; ++i)
            if (std::fabs(Sm[i * n + j]) > std::fabs(Sm[imax * n + j])) imax = i;
        const double sg = Sm[imax * n + j] < 0 ? -1.0 : 1.0;
        for (int i = 0; i < n; ++i) S[i * n + jj] = sg * Sm[i * n + j];
    }
    return 0;
}

bool build_eo_apply(int n, const double* M, const double* P, double* out) {
    const int h = n / 2, hc = (n + 1) / 2;
    double scale = 0.0;
    for (int i = 0; i < n * n; ++i) scale = std::max(scale, std::max(std::fabs(M[i]), std::fabs(P[i])));
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const int a = i * n + j, b = (n - 1 - i) * n + (n - 1 - j);
            if (std::fabs(M[a] - M[b]) > 1e-12 * scale || std::fabs(P[a] - P[b]) > 1e-12 * scale) return false;
        }
    const double* mats[2] = {M, P};
    double* o = out;
    for (int m = 0; m < 2; ++m) {
        const double* A = mats[m];
        for (int i = 0; i < hc; ++i)
            for (int j = 0; j < hc; ++j)
                *o++ = (j < h) ? 0.5 * (A[i * n + j] + A[i * n + (n - 1 - j)]) : A[i * n + j];
        for (int i = 0; i < h; ++i)
            for (int j = 0; j < h; ++j) *o++ = 0.5 * (A[i * n + j] - A[i * n + (n - 1 - j)]);
    }
    return true;
}

bool build_eo_inverse(int n, const double* S, const double* lam, double* out) {
    const int h = n / 2, hc = (n + 1) / 2;
    std::vector<int> sym, anti;
    std::vector<double> Sp(n * n);
    for (int c = 0; c < n; ++c) {
        double dot = 0.0, nrm = 0.0;
        for (int k = 0; k < n; ++k) {
            dot += S[k * n + c] * S[(n - 1 - k) * n + c];
            nrm += S[k * n + c] * S[k * n + c];
        }
        const double sg = dot >= 0.0 ? 1.0 : -1.0;
        if (std::fabs(std::fabs(dot) - nrm) > 1e-8 * nrm) return false;
        for (int k = 0; k < n; ++k) Sp[k * n + c] = 0.5 * (S[k * n + c] + sg * S[(n - 1 - k) * n + c]);
        (sg > 0 ? sym : anti).push_back(c);
    }
    if (static_cast<int>(sym.size()) != hc || static_cast<int>(anti.size()) != h) return false;
    double* o = out;
    for (int k = 0; k < hc; ++k)
        for (int c = 0; c < hc; ++c) *o++ = Sp[k * n + sym[c]];
    for (int k = 0; k < h; ++k)
        for (int c = 0; c < h; ++c) *o++ = Sp[k * n + anti[c]];
    for (int c = 0; c < hc; ++c) *o++ = lam[sym[c]];
    for (int c = 0; c < h; ++c) *o++ = lam[anti[c]];
    return true;
}

}  // namespace tpfdm
