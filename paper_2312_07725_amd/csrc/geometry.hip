// Mesh and metric setup kernel (untimed; runs once per context).
//
// Paper: Sec. 7 (opening paragraph), Eq. warped grid (nonsymmetric periodic warp of a uniform
// hexahedral grid), Sec. 2.2 (covariant basis a_j, Jacobian J, cofactor matrix
// C with C^T = J (J^Omega)^-1, built with the conservative curl form so that
// the discrete GCL of Eq. GCL holds to round-off).
//
// The grid is of the solution degree: node coordinates are the warp evaluated
// at the LGL nodes. For each (n, m, l) cyclic, with V_j = (X_l - X_centre,l)
// dX_m/dxi_j, C[n][i] = -(curl_xi V)_i, every derivative taken with the 1D
// LGL derivative matrix along its direction.
#include "nsfr_host.h"

namespace nsfr {

template <int P>
__global__ __launch_bounds__(256) void geometry_kernel(Ops ops, int nx, int ny, int nz, double lo, double hi,
                                                       double beta, double l, double* X, double* Cline,
                                                       double* invWJ, double* Jout) {
    constexpr int N = P + 1, N2 = N * N, N3 = N2 * N;
    __shared__ double sX[3][N3], sXl[3][N3], sG[3][3][N3], sV[3][N3];
    const int64_t E = (int64_t)nx * ny * nz;
    const int64_t e = blockIdx.x;
    const int ex = (int)(e % nx), ey = (int)((e / nx) % ny), ez = (int)(e / ((int64_t)nx * ny));
    const double hx = (hi - lo) / nx, hy = (hi - lo) / ny, hz = (hi - lo) / nz;
    const double ctr[3] = {lo + hx * (ex + 0.5), lo + hy * (ey + 0.5), lo + hz * (ez + 0.5)};
    const int t = threadIdx.x;
    const int a = t % N, b = (t / N) % N, c = t / N2;
    const bool on = t < N3;
    double J = 0.0;
    if (on) {
        double A = lo + hx * (ex + 0.5 * (ops.x[a] + 1.0));
        double B = lo + hy * (ey + 0.5 * (ops.x[b] + 1.0));
        double Cc = lo + hz * (ez + 0.5 * (ops.x[c] + 1.0));
        double xyz[3];
        xyz[0] = A + beta * sin(A / l) * sin(B / l) * sin(2.0 * Cc / l);
        xyz[1] = B + beta * sin(4.0 * A / l) * sin(B / l) * sin(3.0 * Cc / l);
        xyz[2] = Cc + beta * sin(2.0 * A / l) * sin(5.0 * B / l) * sin(Cc / l);
        for (int m = 0; m < 3; ++m) {
            sX[m][t] = xyz[m];
            sXl[m][t] = xyz[m] - ctr[m];
            X[(m * E + e) * N3 + t] = xyz[m];
        }
    }
    __syncthreads();
    if (on) {
        for (int m = 0; m < 3; ++m) {
            double g0 = 0.0, g1 = 0.0, g2 = 0.0;
            for (int q = 0; q < N; ++q) {
                g0 += ops.D[a][q] * sX[m][q + N * b + N2 * c];
                g1 += ops.D[b][q] * sX[m][a + N * q + N2 * c];
                g2 += ops.D[c][q] * sX[m][a + N * b + N2 * q];
            }
            sG[m][0][t] = g0;
            sG[m][1][t] = g1;
            sG[m][2][t] = g2;
        }
        double(*G)[3][N3] = sG;
        J = G[0][0][t] * (G[1][1][t] * G[2][2][t] - G[1][2][t] * G[2][1][t]) -
            G[0][1][t] * (G[1][0][t] * G[2][2][t] - G[1][2][t] * G[2][0][t]) +
            G[0][2][t] * (G[1][0][t] * G[2][1][t] - G[1][1][t] * G[2][0][t]);
        Jout[e * N3 + t] = J;
        invWJ[e * N3 + t] = 1.0 / (ops.w[a] * ops.w[b] * ops.w[c] * J);
    }
    // line positions and line indices of this node for the three directions
    const int pos[3] = {a, b, c};
    const int lin[3] = {b + N * c, a + N * c, a + N * b};
    for (int nn = 0; nn < 3; ++nn) {
        const int mm = (nn + 1) % 3, ll = (nn + 2) % 3;
        __syncthreads();
        if (on)
            for (int j = 0; j < 3; ++j) sV[j][t] = sXl[ll][t] * sG[mm][j][t];
        __syncthreads();
        if (on) {
            double dV[3][3];   // dV[j][i] = d V_j / d xi_i
            for (int j = 0; j < 3; ++j) {
                double d0 = 0.0, d1 = 0.0, d2 = 0.0;
                for (int q = 0; q < N; ++q) {
                    d0 += ops.D[a][q] * sV[j][q + N * b + N2 * c];
                    d1 += ops.D[b][q] * sV[j][a + N * q + N2 * c];
                    d2 += ops.D[c][q] * sV[j][a + N * b + N2 * q];
                }
                dV[j][0] = d0;
                dV[j][1] = d1;
                dV[j][2] = d2;
            }
            double Cn[3];
            Cn[0] = -(dV[2][1] - dV[1][2]);
            Cn[1] = -(dV[0][2] - dV[2][0]);
            Cn[2] = -(dV[1][0] - dV[0][1]);
            for (int i = 0; i < 3; ++i)
                Cline[((int64_t)(i * 3 + nn) * E + e) * N3 + pos[i] * N2 + lin[i]] = Cn[i];
        }
    }
}

template <int P>
__global__ void geometry_export_kernel(int64_t E, const double* Cline, double* C) {
    constexpr int N = P + 1, N2 = N * N, N3 = N2 * N;
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= E * N3) return;
    int64_t e = idx / N3;
    int node = (int)(idx - e * N3);
    int a = node % N, b = (node / N) % N, c = node / N2;
    const int pos[3] = {a, b, c};
    const int lin[3] = {b + N * c, a + N * c, a + N * b};
    for (int n = 0; n < 3; ++n)
        for (int i = 0; i < 3; ++i)
            C[((int64_t)(n * 3 + i) * E + e) * N3 + node] =
                Cline[((int64_t)(i * 3 + n) * E + e) * N3 + pos[i] * N2 + lin[i]];
}

hipError_t launch_geometry(int p, const Ops& ops, int nx, int ny, int nz, double lo, double hi, double beta,
                           double l, double* X, double* Cline, double* invWJ, double* J, hipStream_t s) {
    int64_t E = (int64_t)nx * ny * nz;
    dim3 grid((unsigned)E), block(256);
    switch (p) {
        case 2: geometry_kernel<2><<<grid, block, 0, s>>>(ops, nx, ny, nz, lo, hi, beta, l, X, Cline, invWJ, J); break;
        case 3: geometry_kernel<3><<<grid, block, 0, s>>>(ops, nx, ny, nz, lo, hi, beta, l, X, Cline, invWJ, J); break;
        case 4: geometry_kernel<4><<<grid, block, 0, s>>>(ops, nx, ny, nz, lo, hi, beta, l, X, Cline, invWJ, J); break;
        case 5: geometry_kernel<5><<<grid, block, 0, s>>>(ops, nx, ny, nz, lo, hi, beta, l, X, Cline, invWJ, J); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_geometry_export(int p, int64_t E, const double* Cline, double* C, hipStream_t s) {
    int n3 = (p + 1) * (p + 1) * (p + 1);
    int64_t tot = E * n3;
    dim3 grid((unsigned)((tot + 255) / 256)), block(256);
    switch (p) {
        case 2: geometry_export_kernel<2><<<grid, block, 0, s>>>(E, Cline, C); break;
        case 3: geometry_export_kernel<3><<<grid, block, 0, s>>>(E, Cline, C); break;
        case 4: geometry_export_kernel<4><<<grid, block, 0, s>>>(E, Cline, C); break;
        case 5: geometry_export_kernel<5><<<grid, block, 0, s>>>(E, Cline, C); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace nsfr
