// Small node-parallel kernels: wave-speed maximum, CFL step, diagnostics,
// state checks and RK helpers. All reductions are two-pass with a fixed
// combination order, so results are bitwise reproducible.
//
// Paper: Sec. 7 opening paragraph (adaptive step from the maximum wave
// speed, CFL 0.1), Sec. 6.2 / 6.3
// (global conservation and entropy conservation: sum_i R_i and
// sum v . R vanish on a periodic mesh), Sec. 2.1 (entropy variables
// v = [(gamma - s)/(gamma - 1) - beta |u|^2, 2 beta u, -2 beta],
// s = ln p - gamma ln rho).
#include "nsfr_host.h"

namespace nsfr {

constexpr int RB = 256;   // threads per reduction block

template <typename Op>
__device__ double block_reduce(double v, Op op, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = RB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = op(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

struct OpMax { __device__ double operator()(double a, double b) const { return fmax(a, b); } };
struct OpSum { __device__ double operator()(double a, double b) const { return a + b; } };

__global__ __launch_bounds__(RB) void wavespeed_partial(int64_t nn, const double* U, double gamma, double* part) {
    __shared__ double sh[RB];
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < nn; i += (int64_t)gridDim.x * RB) {
        double r = U[i], ir = 1.0 / r;
        double u = U[nn + i] * ir, v = U[2 * nn + i] * ir, w = U[3 * nn + i] * ir;
        double p = (gamma - 1.0) * (U[4 * nn + i] - 0.5 * r * (u * u + v * v + w * w));
        m = fmax(m, sqrt(u * u + v * v + w * w) + sqrt(gamma * p * ir));
    }
    double r = block_reduce(m, OpMax(), sh);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
}

__global__ __launch_bounds__(RB) void max_final(int n, const double* part, double* out) {
    __shared__ double sh[RB];
    double m = 0.0;
    for (int i = threadIdx.x; i < n; i += RB) m = fmax(m, part[i]);
    double r = block_reduce(m, OpMax(), sh);
    if (threadIdx.x == 0) out[0] = r;
}

__global__ void cfl_kernel(const double* lam, double cfl, double dx, double* dt) {
    if (threadIdx.x == 0 && blockIdx.x == 0) dt[0] = cfl * dx / lam[0];
}

__global__ void advance_time_kernel(double* t, const double* dt) {
    if (threadIdx.x == 0 && blockIdx.x == 0) t[0] = t[0] + dt[0];
}

// 8 partial sums per block: [v.R, |v.R|, R0..R4, max|R|]
__global__ __launch_bounds__(RB) void diag_partial(int64_t nn, const double* U, const double* V, const double* R,
                                                   double gamma, double* part) {
    __shared__ double sh[RB];
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < nn; i += (int64_t)gridDim.x * RB) {
        double r = U[i], ir = 1.0 / r;
        double u = U[nn + i] * ir, v = U[2 * nn + i] * ir, w = U[3 * nn + i] * ir;
        double q2 = u * u + v * v + w * w;
        double p = (gamma - 1.0) * (U[4 * nn + i] - 0.5 * r * q2);
        double beta = 0.5 * r / p;
        double s = log(p) - gamma * log(r);
        double ev[5] = {(gamma - s) / (gamma - 1.0) - beta * q2, 2 * beta * u, 2 * beta * v, 2 * beta * w, -2 * beta};
        if (V)
            for (int k = 0; k < 5; ++k) ev[k] = V[k * nn + i];
        for (int k = 0; k < 5; ++k) {
            double Rk = R[k * nn + i];
            double vr = ev[k] * Rk;
            acc[0] += vr;
            acc[1] += fabs(vr);
            acc[2 + k] += Rk;
            acc[7] = fmax(acc[7], fabs(Rk));
        }
    }
    for (int k = 0; k < 8; ++k) {
        double r = (k == 7) ? block_reduce(acc[k], OpMax(), sh) : block_reduce(acc[k], OpSum(), sh);
        if (threadIdx.x == 0) part[k * gridDim.x + blockIdx.x] = r;
    }
}

__global__ __launch_bounds__(RB) void diag_final(int n, const double* part, double* out) {
    __shared__ double sh[RB];
    for (int k = 0; k < 8; ++k) {
        double a = 0.0;
        for (int i = threadIdx.x; i < n; i += RB) a = (k == 7) ? fmax(a, part[k * n + i]) : a + part[k * n + i];
        double r = (k == 7) ? block_reduce(a, OpMax(), sh) : block_reduce(a, OpSum(), sh);
        if (threadIdx.x == 0) out[k] = r;
    }
}

__global__ __launch_bounds__(RB) void check_kernel(int64_t nn, const double* U, double gamma, int32_t* count) {
    __shared__ double sh[RB];
    double bad = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < nn; i += (int64_t)gridDim.x * RB) {
        double r = U[i];
        double m1 = U[nn + i], m2 = U[2 * nn + i], m3 = U[3 * nn + i], E = U[4 * nn + i];
        double p = (gamma - 1.0) * (E - 0.5 * (m1 * m1 + m2 * m2 + m3 * m3) / r);
        bool ok = (r > 0.0) && (p > 0.0) && (m1 == m1) && (m2 == m2) && (m3 == m3) && (E == E);
        bad += ok ? 0.0 : 1.0;
    }
    double r = block_reduce(bad, OpSum(), sh);
    if (threadIdx.x == 0) count[blockIdx.x] = (int32_t)r;
}

__global__ __launch_bounds__(RB) void ke_partial(int64_t nn, const double* U, const double* invWJ, double* part,
                                                 double* grad) {
    __shared__ double sh[RB];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < nn; i += (int64_t)gridDim.x * RB) {
        double wj = 1.0 / invWJ[i];
        double r = U[i], ir = 1.0 / r;
        double u = U[nn + i] * ir, v = U[2 * nn + i] * ir, w = U[3 * nn + i] * ir;
        double q2 = u * u + v * v + w * w;
        acc += wj * 0.5 * r * q2;
        if (grad) {
            grad[i] = -0.5 * wj * q2;
            grad[nn + i] = wj * u;
            grad[2 * nn + i] = wj * v;
            grad[3 * nn + i] = wj * w;
            grad[4 * nn + i] = 0.0;
        }
    }
    double r = block_reduce(acc, OpSum(), sh);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
}

__global__ __launch_bounds__(RB) void sum_final(int n, const double* part, double* out) {
    __shared__ double sh[RB];
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += RB) a += part[i];
    double r = block_reduce(a, OpSum(), sh);
    if (threadIdx.x == 0) out[0] = r;
}

// out = (ca + cb h) z + (da + db h) x (+ out if accumulate); h = *dt or 0
__global__ void lincomb_kernel(int64_t n, double* out, const double* z, double ca, double cb, const double* x,
                               double da, double db, const double* dt, int accumulate) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double h = dt ? dt[0] : 0.0;
    double v = 0.0;
    if (z) v += (ca + cb * h) * z[i];
    if (x) v += (da + db * h) * x[i];
    if (accumulate) v += out[i];
    out[i] = v;
}

hipError_t launch_lincomb(int64_t n, double* out, const double* z, double ca, double cb, const double* x, double da,
                          double db, const double* dt, int accumulate, hipStream_t s) {
    lincomb_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, out, z, ca, cb, x, da, db, dt, accumulate);
    return hipGetLastError();
}

static int nblocks(int64_t nn) {
    int64_t b = (nn + RB - 1) / RB;
    return (int)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}

hipError_t launch_max_wavespeed(int64_t nn, const double* U, double gamma, double* partial, int nblk, double* lam,
                                hipStream_t s) {
    int nb = nblocks(nn);
    if (nb > nblk) nb = nblk;
    wavespeed_partial<<<nb, RB, 0, s>>>(nn, U, gamma, partial);
    max_final<<<1, RB, 0, s>>>(nb, partial, lam);
    return hipGetLastError();
}

hipError_t launch_cfl_dt(const double* lam, double cfl, double dx, double* dt, hipStream_t s) {
    cfl_kernel<<<1, 64, 0, s>>>(lam, cfl, dx, dt);
    return hipGetLastError();
}

hipError_t launch_advance_time(double* t, const double* dt, hipStream_t s) {
    advance_time_kernel<<<1, 64, 0, s>>>(t, dt);
    return hipGetLastError();
}

hipError_t launch_diagnostics(int64_t nn, const double* U, const double* V, const double* R, double gamma,
                              double* partial, int nblk, double* out, hipStream_t s) {
    int nb = nblocks(nn);
    if (nb > nblk / 8) nb = nblk / 8;
    diag_partial<<<nb, RB, 0, s>>>(nn, U, V, R, gamma, partial);
    diag_final<<<1, RB, 0, s>>>(nb, partial, out);
    return hipGetLastError();
}

hipError_t launch_kinetic_energy(int64_t nn, const double* U, const double* invWJ, double* partial, int nblk,
                                 double* ke, double* grad, hipStream_t s) {
    int nb = nblocks(nn);
    if (nb > nblk) nb = nblk;
    ke_partial<<<nb, RB, 0, s>>>(nn, U, invWJ, partial, grad);
    sum_final<<<1, RB, 0, s>>>(nb, partial, ke);
    return hipGetLastError();
}

hipError_t launch_check_state(int64_t nn, const double* U, double gamma, int32_t* count, hipStream_t s) {
    check_kernel<<<64, RB, 0, s>>>(nn, U, gamma, count);
    return hipGetLastError();
}


}  // namespace nsfr
