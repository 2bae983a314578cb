// Host construction of the 1D reference operators on LGL nodes.
//
// Paper: Sec. 2.2 (nodal tensor-product basis, SBP property, Eq. SBP),
// Sec. 3.2 (ESFR correction operator, Eq. Km: in 1D on LGL nodes every row of
// D^p is d = p! lambda, lambda the barycentric weights, so K = 2 c d d^T),
// Sec. 4 (FR projection Pi~ = (W + K)^-1 W, Eq. Fr projection, which for a
// rank-one K is I - alpha W^-1 d d^T with alpha = 2c / (1 + 2c d^T W^-1 d)).
#include "nsfr_host.h"

#include <cmath>
#include <cstring>
#include <utility>

namespace nsfr {

static void legendre_pair(int p, double x, double& Pp, double& Pm) {
    double P0 = 1.0, P1 = x;
    if (p == 0) { Pp = 1.0; Pm = 0.0; return; }
    for (int k = 2; k <= p; ++k) {
        double P2 = ((2.0 * k - 1.0) * x * P1 - (k - 1.0) * P0) / k;
        P0 = P1;
        P1 = P2;
    }
    Pp = P1;
    Pm = P0;
}

void build_ops(int p, double c, Ops& ops, HostOps& h) {
    const int n = p + 1;
    h.p = p;
    h.n = n;
    // LGL nodes: Newton on (1 - x^2) P_p'(x) = p (P_{p-1} - x P_p)
    for (int i = 0; i < n; ++i) h.x[i] = -std::cos(M_PI * i / p);
    for (int i = 1; i < p; ++i) {
        double x = h.x[i];
        for (int it = 0; it < 100; ++it) {
            double Pp, Pm;
            legendre_pair(p, x, Pp, Pm);
            double dx = (x * Pp - Pm) / ((p + 1) * Pp);
            x -= dx;
            if (std::fabs(dx) < 1e-17) break;
        }
        h.x[i] = x;
    }
    h.x[0] = -1.0;
    h.x[p] = 1.0;
    for (int i = 0; i <= p / 2; ++i) {   // exact symmetry about 0
        double s = 0.5 * (h.x[p - i] - h.x[i]);
        h.x[i] = -s;
        h.x[p - i] = s;
    }
    if (p % 2 == 0) h.x[p / 2] = 0.0;
    for (int i = 0; i < n; ++i) {
        double Pp, Pm;
        legendre_pair(p, h.x[i], Pp, Pm);
        h.w[i] = 2.0 / (p * (p + 1.0) * Pp * Pp);
    }
    // barycentric weights and the differentiation matrix
    double lam[MAXN];
    for (int j = 0; j < n; ++j) {
        double prod = 1.0;
        for (int k = 0; k < n; ++k)
            if (k != j) prod *= (h.x[j] - h.x[k]);
        lam[j] = 1.0 / prod;
    }
    for (int i = 0; i < n; ++i) {
        double diag = 0.0;
        for (int j = 0; j < n; ++j) {
            if (i == j) continue;
            h.D[i][j] = (lam[j] / lam[i]) / (h.x[i] - h.x[j]);
            diag -= h.D[i][j];
        }
        h.D[i][i] = diag;
    }
    // skew volume operator S1 = W D - D^T W, made exactly antisymmetric (the
    // kernels rely on S1[b][a] = -S1[a][b] bitwise for discrete conservation)
    for (int i = 0; i < n; ++i) {
        h.S1[i][i] = 0.0;
        for (int j = i + 1; j < n; ++j) {
            const double wd = h.w[i] * h.D[i][j];
            const double dw = h.D[j][i] * h.w[j];
            h.S1[i][j] = wd - dw;
            h.S1[j][i] = -h.S1[i][j];
        }
    }
    // d = p! lambda; FR projection in rank-one form
    double fact = 1.0;
    for (int k = 2; k <= p; ++k) fact *= k;
    double mu = 0.0;
    for (int j = 0; j < n; ++j) {
        h.d[j] = fact * lam[j];
        mu += h.d[j] * h.d[j] / h.w[j];
    }
    double alpha = 2.0 * c / (1.0 + 2.0 * c * mu);
    for (int j = 0; j < n; ++j) {
        h.pia[j] = alpha * h.d[j] / h.w[j];
        h.pib[j] = h.d[j];
    }
    h.mu = mu;
    h.alpha = alpha;
    // pack the device copy
    for (int i = 0; i < MAXN; ++i) {
        ops.w[i] = i < n ? h.w[i] : 0.0;
        ops.x[i] = i < n ? h.x[i] : 0.0;
        ops.pia[i] = i < n ? h.pia[i] : 0.0;
        ops.pib[i] = i < n ? h.pib[i] : 0.0;
        for (int j = 0; j < MAXN; ++j) {
            bool in = i < n && j < n;
            ops.S1h[i][j] = in ? 0.5 * h.S1[i][j] : 0.0;
            ops.D[i][j] = in ? h.D[i][j] : 0.0;
        }
    }
}

// ---- Gauss-Legendre operators (uncollocated quadrature; Sec. 3.3, Sec. 4
// Eq. Fr projection with the basis evaluated at the quadrature points)

static void solve_small(int n, double* A, double* B, int m) {
    // B <- A^-1 B for an n x n matrix A and an n x m right-hand side
    // (Gauss-Jordan elimination with partial pivoting; row-major).
    for (int k = 0; k < n; ++k) {
        int piv = k;
        for (int i = k + 1; i < n; ++i)
            if (std::fabs(A[i * n + k]) > std::fabs(A[piv * n + k])) piv = i;
        if (piv != k) {
            for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[piv * n + j]);
            for (int j = 0; j < m; ++j) std::swap(B[k * m + j], B[piv * m + j]);
        }
        const double r = A[k * n + k];
        for (int j = 0; j < n; ++j) A[k * n + j] /= r;
        for (int j = 0; j < m; ++j) B[k * m + j] /= r;
        for (int i = 0; i < n; ++i) {
            if (i == k) continue;
            const double f = A[i * n + k];
            if (f == 0.0) continue;
            for (int j = 0; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
            for (int j = 0; j < m; ++j) B[i * m + j] -= f * B[k * m + j];
        }
    }
}

static double lagrange(const double* x, int n, int j, double t) {
    double v = 1.0;
    for (int k = 0; k < n; ++k)
        if (k != j) v *= (t - x[k]) / (x[j] - x[k]);
    return v;
}

static double lagrange_d(const double* x, int n, int j, double t) {
    double s = 0.0;
    for (int m = 0; m < n; ++m) {
        if (m == j) continue;
        double v = 1.0 / (x[j] - x[m]);
        for (int k = 0; k < n; ++k)
            if (k != j && k != m) v *= (t - x[k]) / (x[j] - x[k]);
        s += v;
    }
    return s;
}

void build_gl_ops(int p, int q, double c, const HostOps& h, GLOps& g) {
    const int n = p + 1;
    std::memset(&g, 0, sizeof(g));
    g.p = p;
    g.n = n;
    g.q = q;
    // Gauss-Legendre nodes: roots of P_q by Newton from Chebyshev guesses;
    // weights 2 / ((1 - x^2) P_q'(x)^2), P_q' = q (x P_q - P_{q-1}) / (x^2 - 1)
    for (int i = 0; i < q; ++i) {
        double x = -std::cos(M_PI * (i + 0.75) / (q + 0.5));
        for (int it = 0; it < 100; ++it) {
            double Pq, Pm;
            legendre_pair(q, x, Pq, Pm);
            const double dP = q * (x * Pq - Pm) / (x * x - 1.0);
            const double dx = Pq / dP;
            x -= dx;
            if (std::fabs(dx) < 1e-17) break;
        }
        g.xq[i] = x;
    }
    for (int i = 0; i < q / 2; ++i) {   // exact symmetry about 0
        const double sx = 0.5 * (g.xq[q - 1 - i] - g.xq[i]);
        g.xq[i] = -sx;
        g.xq[q - 1 - i] = sx;
    }
    if (q % 2) g.xq[q / 2] = 0.0;
    for (int i = 0; i < q; ++i) {
        double Pq, Pm;
        legendre_pair(q, g.xq[i], Pq, Pm);
        const double dP = q * (g.xq[i] * Pq - Pm) / (g.xq[i] * g.xq[i] - 1.0);
        g.wq[i] = 2.0 / ((1.0 - g.xq[i] * g.xq[i]) * dP * dP);
    }
    for (int i = 0; i < q / 2; ++i) {
        const double w = 0.5 * (g.wq[i] + g.wq[q - 1 - i]);
        g.wq[i] = g.wq[q - 1 - i] = w;
    }
    // basis at the quadrature points and its derivative
    for (int i = 0; i < q; ++i)
        for (int a = 0; a < n; ++a) {
            g.chi[i * n + a] = lagrange(h.x, n, a, g.xq[i]);
            g.chid[i * n + a] = lagrange_d(h.x, n, a, g.xq[i]);
        }
    // M = chi^T Wq chi; K = c (D^p)^T M D^p; projections
    double M[MAXN * MAXN], K[MAXN * MAXN], Dp[MAXN * MAXN], T[MAXN * MAXN], R[MAXN * MAXQ];
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            double v = 0.0;
            for (int i = 0; i < q; ++i) v += g.chi[i * n + a] * g.wq[i] * g.chi[i * n + b];
            M[a * n + b] = v;
        }
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) Dp[a * n + b] = (a == b) ? 1.0 : 0.0;
    for (int k = 0; k < p; ++k) {
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) {
                double v = 0.0;
                for (int m = 0; m < n; ++m) v += Dp[a * n + m] * h.D[m][b];
                T[a * n + b] = v;
            }
        std::memcpy(Dp, T, sizeof(double) * n * n);
    }
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            double v = 0.0;
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) v += Dp[i * n + a] * M[i * n + j] * Dp[j * n + b];
            K[a * n + b] = c * v;
        }
    for (int pass = 0; pass < 2; ++pass) {
        double A[MAXN * MAXN];
        for (int k = 0; k < n * n; ++k) A[k] = M[k] + (pass ? K[k] : 0.0);
        for (int a = 0; a < n; ++a)
            for (int i = 0; i < q; ++i) R[a * q + i] = g.chi[i * n + a] * g.wq[i];
        solve_small(n, A, R, q);
        double* out = pass ? g.pit : g.pi;
        for (int k = 0; k < n * q; ++k) out[k] = R[k];
    }
    // flux basis: differentiation on the quadrature points and end values
    // (diagonal = minus the off-diagonal row sum, so that Dq 1 = 0 to rounding)
    double* Dq = g.dq;
    for (int i = 0; i < q; ++i) {
        double rs = 0.0;
        for (int j = 0; j < q; ++j)
            if (j != i) {
                Dq[i * q + j] = lagrange_d(g.xq, q, j, g.xq[i]);
                rs += Dq[i * q + j];
            }
        Dq[i * q + i] = -rs;
    }
    for (int i = 0; i < q; ++i) {
        g.sqh[i * q + i] = 0.0;
        for (int j = i + 1; j < q; ++j) {
            const double v = 0.5 * (g.wq[i] * Dq[i * q + j] - Dq[j * q + i] * g.wq[j]);
            g.sqh[i * q + j] = v;
            g.sqh[j * q + i] = -v;
        }
        g.tl[i] = lagrange(g.xq, q, i, -1.0);
        g.tr[i] = lagrange(g.xq, q, i, 1.0);
    }
}

double c_hu(int p) {
    Ops ops;
    HostOps h;
    build_ops(p, 0.0, ops, h);
    double q = 0.0;
    for (int i = 0; i <= p; ++i) q += h.w[i] * std::pow(h.x[i], 2 * p);
    double Ep = q - 2.0 / (2.0 * p + 1.0);
    double fact = 1.0;
    for (int k = 2; k <= p; ++k) fact *= k;
    return Ep / (2.0 * fact * fact);
}

}  // namespace nsfr

extern "C" nsfr_status nsfr_c_hu(int32_t p, double* out) {
    if (!out || p < 2 || p > 5) {
        nsfr::set_error("nsfr_c_hu: p must be in 2..5 and out non-null");
        return NSFR_EINVAL;
    }
    *out = nsfr::c_hu(p);
    return NSFR_OK;
}
