// Exact inverse of the FR-modified mass (the `mass = 1` option of a
// collocated context): an independent check of the weight-adjusted inverse,
// not part of the fast path.
//
// Paper: Sec. 3.2, Eq. Km. On the collocated LGL basis M_m = diag(W J) and
// K_m = sum over (s, v, w) in {0, p}^3 without (0, 0, 0) of
// c^((s + v + w) / p) D_svw^T M_m D_svw, D_svw = D_z^w (x) D_y^v (x) D_x^s
// with D^0 = I. The p-th derivative matrix D^p maps every row to the same
// vector d = p! lambda (barycentric weights), so for the set S of directions
// with exponent p the entry (a, b) of D_svw^T M_m D_svw is
//   [a_k = b_k for k not in S] prod_{k in S} d(a_k) d(b_k)
//     * sum of W J over the nodes that agree with a outside S,
// a sum over at most 7 direction subsets per entry. The dense matrix of each
// element (m = n^3 rows) is factorised once at context creation (Cholesky,
// in place, one workgroup per element) and applied per right-hand side by a
// forward and a backward substitution (one wave per element and state).
#include "nsfr_host.h"

namespace nsfr {

constexpr int EXACT_BUILD_BLOCK = 256;
constexpr int EXACT_FACTOR_BLOCK = 256;

// d = p! lambda, the common row of D^p (kernel argument by value)
struct DVec {
    double d[MAXN];
};

// Lower triangle (with the diagonal) of M_m + K_m of every element into
// L [E][m][m] (row-major; the upper triangle is not written).
template <int N>
__global__ __launch_bounds__(EXACT_BUILD_BLOCK) void exact_mass_build_kernel(int64_t E, const double* __restrict__ invWJ,
                                                                            DVec dv, double c, double* __restrict__ L) {
    constexpr int N2 = N * N, M = N2 * N;
    __shared__ double wj[M];
    __shared__ double sx[N2], sy[N2], sz[N2];   // sums over one direction: sx[j + N k], sy[i + N k], sz[i + N j]
    __shared__ double sxy[N], sxz[N], syz[N], sxyz;
    const int64_t e = blockIdx.x;
    const int tid = threadIdx.x, nth = blockDim.x;
    for (int a = tid; a < M; a += nth) wj[a] = 1.0 / invWJ[e * M + a];
    __syncthreads();
    for (int t = tid; t < N2; t += nth) {
        const int u = t % N, v = t / N;
        double a = 0.0, b = 0.0, g = 0.0;
        for (int r = 0; r < N; ++r) {
            a += wj[r + N * u + N2 * v];   // over i at (j, k) = (u, v)
            b += wj[u + N * r + N2 * v];   // over j at (i, k) = (u, v)
            g += wj[u + N * v + N2 * r];   // over k at (i, j) = (u, v)
        }
        sx[t] = a;
        sy[t] = b;
        sz[t] = g;
    }
    __syncthreads();
    for (int t = tid; t < N; t += nth) {
        double a = 0.0, b = 0.0, g = 0.0;
        for (int r = 0; r < N; ++r) {
            a += sx[r + N * t];   // over i, j at k = t
            b += sx[t + N * r];   // over i, k at j = t
            g += sy[t + N * r];   // over j, k at i = t
        }
        sxy[t] = a;
        sxz[t] = b;
        syz[t] = g;
    }
    if (tid == 0) {
        double a = 0.0;
        for (int r = 0; r < M; ++r) a += wj[r];
        sxyz = a;
    }
    __syncthreads();
    const double c2 = c * c, c3 = c2 * c;
    double* Le = L + e * (int64_t)M * M;
    for (int idx = tid; idx < M * M; idx += nth) {
        const int ra = idx / M, rb = idx - ra * M;
        if (rb > ra) continue;
        const int ai = ra % N, aj = (ra / N) % N, ak = ra / N2;
        const int bi = rb % N, bj = (rb / N) % N, bk = rb / N2;
        const double dx = dv.d[ai] * dv.d[bi], dy = dv.d[aj] * dv.d[bj], dz = dv.d[ak] * dv.d[bk];
        const bool ei = ai == bi, ej = aj == bj, ek = ak == bk;
        double v = (ra == rb) ? wj[ra] : 0.0;
        if (ej && ek) v += c * dx * sx[aj + N * ak];        // S = {x}
        if (ei && ek) v += c * dy * sy[ai + N * ak];        // S = {y}
        if (ei && ej) v += c * dz * sz[ai + N * aj];        // S = {z}
        if (ek) v += c2 * dx * dy * sxy[ak];                // S = {x, y}
        if (ej) v += c2 * dx * dz * sxz[aj];                // S = {x, z}
        if (ei) v += c2 * dy * dz * syz[ai];                // S = {y, z}
        v += c3 * dx * dy * dz * sxyz;                      // S = {x, y, z}
        Le[(int64_t)ra * M + rb] = v;
    }
}

// In-place Cholesky factorisation of the lower triangle of each element's
// m x m block, column by column (one workgroup per element). A non-positive
// pivot sets *fail and is replaced by 1 so that the factorisation finishes.
__global__ __launch_bounds__(EXACT_FACTOR_BLOCK) void exact_mass_factor_kernel(int m, double* __restrict__ L,
                                                                              int* __restrict__ fail) {
    __shared__ double piv;
    double* A = L + (int64_t)blockIdx.x * m * m;
    const int tid = threadIdx.x, nth = blockDim.x;
    for (int j = 0; j < m; ++j) {
        if (tid == 0) {
            double s = A[(int64_t)j * m + j];
            for (int k = 0; k < j; ++k) s -= A[(int64_t)j * m + k] * A[(int64_t)j * m + k];
            if (!(s > 0.0)) {
                atomicOr(fail, 1);
                s = 1.0;
            }
            piv = sqrt(s);
            A[(int64_t)j * m + j] = piv;
        }
        __syncthreads();
        const double dj = piv;
        for (int i = j + 1 + tid; i < m; i += nth) {
            double s = A[(int64_t)i * m + j];
            for (int k = 0; k < j; ++k) s -= A[(int64_t)i * m + k] * A[(int64_t)j * m + k];
            A[(int64_t)i * m + j] = s / dj;
        }
        __syncthreads();
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// out = -(M_m + K_m)^-1 R for every element and state: wave s of workgroup e
// solves L y = R, then L^T x = y, with the vector spread over the lanes
// (entry k held by lane k mod 64 in its chunk k / 64).
template <int N>
__global__ __launch_bounds__(320) void exact_mass_solve_kernel(int64_t E, const double* __restrict__ L,
                                                               const double* __restrict__ R, double* __restrict__ out) {
    constexpr int M = N * N * N, NC = (M + 63) / 64;
    const int64_t e = blockIdx.x;
    const int s = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int64_t SE = E * M;
    const double* Le = L + e * (int64_t)M * M;
    const double* r = R + s * SE + e * M;
    double y[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) y[c] = 0.0;
    // forward: y_i = (r_i - sum_{k < i} L_ik y_k) / L_ii
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        for (int i = 64 * c; i < 64 * c + 64 && i < M; ++i) {
            double part = 0.0;
#pragma unroll
            for (int cc = 0; cc <= c; ++cc) {
                const int k = lane + 64 * cc;
                if (k < i) part += Le[(int64_t)i * M + k] * y[cc];
            }
            const double yi = (r[i] - wave_sum(part)) / Le[(int64_t)i * M + i];
            if (lane == i - 64 * c) y[c] = yi;
        }
    }
    // backward: x_i = (y_i - sum_{k > i} L_ki x_k) / L_ii
#pragma unroll
    for (int c = NC - 1; c >= 0; --c) {
        for (int i = (64 * c + 63 < M - 1 ? 64 * c + 63 : M - 1); i >= 64 * c; --i) {
            double part = 0.0;
#pragma unroll
            for (int cc = c; cc < NC; ++cc) {
                const int k = lane + 64 * cc;
                if (k > i && k < M) part += Le[(int64_t)k * M + i] * y[cc];
            }
            const double sum = wave_sum(part);
            const double yi = __shfl(y[c], i - 64 * c, 64);
            const double xi = (yi - sum) / Le[(int64_t)i * M + i];
            if (lane == i - 64 * c) y[c] = xi;
        }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const int k = lane + 64 * c;
        if (k < M) out[s * SE + e * M + k] = -y[c];
    }
}

size_t exact_mass_doubles(int p, int64_t E) {
    const int64_t m = (int64_t)(p + 1) * (p + 1) * (p + 1);
    return (size_t)(E * m * m);
}

template <int N>
static hipError_t exact_factor_t(int64_t E, const double* invWJ, const DVec& dv, double c, double* L, int* fail,
                                 hipStream_t s) {
    exact_mass_build_kernel<N><<<(unsigned)E, EXACT_BUILD_BLOCK, 0, s>>>(E, invWJ, dv, c, L);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    exact_mass_factor_kernel<<<(unsigned)E, EXACT_FACTOR_BLOCK, 0, s>>>(N * N * N, L, fail);
    return hipGetLastError();
}

hipError_t launch_exact_mass_factor(int p, int64_t E, const double* invWJ, const double* d, double c, double* L,
                                    int* fail, hipStream_t s) {
    DVec dv;
    for (int i = 0; i < MAXN; ++i) dv.d[i] = i <= p ? d[i] : 0.0;
    switch (p) {
        case 2: return exact_factor_t<3>(E, invWJ, dv, c, L, fail, s);
        case 3: return exact_factor_t<4>(E, invWJ, dv, c, L, fail, s);
        case 4: return exact_factor_t<5>(E, invWJ, dv, c, L, fail, s);
        case 5: return exact_factor_t<6>(E, invWJ, dv, c, L, fail, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_exact_mass_solve(int p, int64_t E, const double* L, const double* R, double* out, hipStream_t s) {
    switch (p) {
        case 2: exact_mass_solve_kernel<3><<<(unsigned)E, 320, 0, s>>>(E, L, R, out); break;
        case 3: exact_mass_solve_kernel<4><<<(unsigned)E, 320, 0, s>>>(E, L, R, out); break;
        case 4: exact_mass_solve_kernel<5><<<(unsigned)E, 320, 0, s>>>(E, L, R, out); break;
        case 5: exact_mass_solve_kernel<6><<<(unsigned)E, 320, 0, s>>>(E, L, R, out); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace nsfr
