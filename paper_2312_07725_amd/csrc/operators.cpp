// Host construction of the 1D reference operators on LGL nodes.
//
// Paper: Sec. 2.2 (nodal tensor-product basis, SBP property, Eq. SBP),
// Sec. 3.2 (ESFR correction operator, Eq. Km: in 1D on LGL nodes every row of
// D^p is d = p! lambda, lambda the barycentric weights, so K = 2 c d d^T),
// Sec. 4 (FR projection Pi~ = (W + K)^-1 W, Eq. Fr projection, which for a
// rank-one K is I - alpha W^-1 d d^T with alpha = 2c / (1 + 2c d^T W^-1 d)).
#include "nsfr_host.h"

#include <cmath>

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
