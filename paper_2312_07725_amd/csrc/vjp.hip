// Discrete adjoint of the NSFR right-hand side: g = (d(dU/dt)/dU)^T lam.
//
// With dU/dt = -A R(U) + (source independent of U) and A the weight-adjusted
// inverse (symmetric), g = -(dR/dU)^T mu with mu = A lam. R is a sum of
// two-point-flux terms: for a volume pair (a, b) on a line the scalar
// mu . R collects w_perp S1[a][b] (mu_a - mu_b) . f_s(U_a, U_b), and for a face
// node pair (own o, neighbour n) it collects W_f (mu_o - mu_n) . f*(U_o, U_n).
// Each thread owns one line as in the forward kernel, differentiates those
// scalars in reverse mode with respect to the primitive variables of its own
// nodes (face pairs: only the own node; the neighbouring element's thread
// produces the other half), the three directions are summed in LDS in a fixed
// order, and the primitive cotangents are mapped to conservative ones.
//
// Paper: Eq. NSFR, Eq. weight-adj ESFR mass, Sec. 3.3 (two-point flux). The
// adjoint itself has no counterpart in the paper.
#include "nsfr_host.h"

namespace nsfr {

constexpr int VJP_BLOCK_MAX = 512;

// Closed-form branches of the two derivative helpers below, kept out of line
// so that their logarithms are only evaluated for the rare pairs that need them.
__device__ __noinline__ void ln_mean_grad_closed(double a, double b, double& La, double& Lb, double& L) {
    double la = log(a), lb = log(b);
    double il = 1.0 / (la - lb);
    L = (a - b) * il;
    La = (1.0 - L / a) * il;
    Lb = (L / b - 1.0) * il;
}

__device__ __noinline__ void inv_ln_mean_grad_closed(double a, double b, double& Ia, double& Ib, double& I) {
    double la = log(a), lb = log(b);
    double L = (a - b) / (la - lb);
    I = 1.0 / L;
    double il = 1.0 / (la - lb);
    double La = (1.0 - L / a) * il, Lb = (L / b - 1.0) * il;
    Ia = -I * I * La;
    Ib = -I * I * Lb;
}

// d/da and d/db of the logarithmic mean L(a, b) (homogeneous of degree one):
// with s = a + b, f = (a - b)/s and G(f) = f / atanh(f),
// dL/da = (G + G' (1 - f)) / 2, dL/db = (G - G' (1 + f)) / 2.
__device__ __forceinline__ void ln_mean_grad(double a, double b, double& La, double& Lb, double& L) {
    double s = a + b, d = a - b;
    double f = d * rcp_pos(s);
    double u = f * f;
    if (u < LN_SWITCH) {
        double G = __builtin_fma(u, __builtin_fma(u, __builtin_fma(u, -44.0 / 945.0, -4.0 / 45.0), -1.0 / 3.0), 1.0);
        double Gp = f * __builtin_fma(u, __builtin_fma(u, __builtin_fma(u, -3424.0 / 14175.0, -264.0 / 945.0),
                                                       -16.0 / 45.0), -2.0 / 3.0);
        L = 0.5 * s * G;
        La = 0.5 * (G + Gp * (1.0 - f));
        Lb = 0.5 * (G - Gp * (1.0 + f));
    } else {
        ln_mean_grad_closed(a, b, La, Lb, L);
    }
}

// d/da, d/db of IL = 1 / L(a, b): with H(f) = atanh(f) / f, IL = (2/s) H,
// dIL/da = (2/s^2)(-H + H' (1 - f)), dIL/db = (2/s^2)(-H - H' (1 + f)).
__device__ __forceinline__ void inv_ln_mean_grad(double a, double b, double rs, double& Ia, double& Ib, double& I) {
    double d = a - b;
    double f = d * rs;
    double u = f * f;
    if (u < LN_SWITCH) {
        double H = __builtin_fma(u, __builtin_fma(u, __builtin_fma(u, 1.0 / 7.0, 1.0 / 5.0), 1.0 / 3.0), 1.0);
        double Hp = f * __builtin_fma(u, __builtin_fma(u, __builtin_fma(u, 8.0 / 9.0, 6.0 / 7.0), 4.0 / 5.0), 2.0 / 3.0);
        I = 2.0 * rs * H;
        double k = 2.0 * rs * rs;
        Ia = k * (-H + Hp * (1.0 - f));
        Ib = k * (-H - Hp * (1.0 + f));
    } else {
        inv_ln_mean_grad_closed(a, b, Ia, Ib, I);
    }
}

// Accumulate the primitive cotangents (rho, u, v, w, p, beta) of
// dl . f_s(A, B; N) into gA and gB.
template <int VARIANT>
__device__ __forceinline__ void ec_flux_vjp(const Prim& A, const Prim& B, double nx, double ny, double nz, double c1,
                                            const double dl[5], double gA[6], double gB[6]) {
    const double una = A.u * nx + A.v * ny + A.w * nz;
    const double unb = B.u * nx + B.v * ny + B.w * nz;
    const double un = 0.5 * (una + unb);
    double rho_ln, Lra, Lrb;
    ln_mean_grad(A.rho, B.rho, Lra, Lrb, rho_ln);
    const double rsb = rcp_pos(A.beta + B.beta);
    double ibl, Iba, Ibb;
    inv_ln_mean_grad(A.beta, B.beta, rsb, Iba, Ibb, ibl);
    const double frho = rho_ln * un;
    const double um = 0.5 * (A.u + B.u), vm = 0.5 * (A.v + B.v), wm = 0.5 * (A.w + B.w);
    const double dE = dl[4];
    double gfrho, gum, gvm, gwm, gun, guna = 0.0, gunb = 0.0, gibl;
    double gua = 0.0, gva = 0.0, gwa = 0.0, gub = 0.0, gvb = 0.0, gwb = 0.0;
    double gpa = 0.0, gpb = 0.0, gra = 0.0, grb = 0.0, gba = 0.0, gbb = 0.0;
    if (VARIANT == 0) {
        const double pm = 0.5 * (A.p + B.p);
        const double uab = A.u * B.u + A.v * B.v + A.w * B.w;
        const double X = c1 * ibl + 0.5 * uab;
        gfrho = dl[0] + dl[1] * um + dl[2] * vm + dl[3] * wm + dE * X;
        gum = dl[1] * frho;
        gvm = dl[2] * frho;
        gwm = dl[3] * frho;
        const double gpm = dl[1] * nx + dl[2] * ny + dl[3] * nz + dE * un;
        gpa += 0.5 * gpm;
        gpb += 0.5 * gpm;
        gibl = dE * frho * c1;
        const double guab = 0.5 * dE * frho;
        gua += guab * B.u; gva += guab * B.v; gwa += guab * B.w;
        gub += guab * A.u; gvb += guab * A.v; gwb += guab * A.w;
        // pe = pm un - (pa - pb)(una - unb) / 4
        gun = gfrho * rho_ln + dE * pm;
        const double gdp = -0.25 * dE * (una - unb);
        const double gdun = -0.25 * dE * (A.p - B.p);
        gpa += gdp;
        gpb -= gdp;
        guna += gdun;
        gunb -= gdun;
    } else {
        const double ph = 0.5 * (A.rho + B.rho) * rsb;
        const double qa = A.u * A.u + A.v * A.v + A.w * A.w;
        const double qb = B.u * B.u + B.v * B.v + B.w * B.w;
        const double X = c1 * ibl - 0.25 * (qa + qb);
        const double Fm1 = um * frho + ph * nx, Fm2 = vm * frho + ph * ny, Fm3 = wm * frho + ph * nz;
        const double g1 = dl[1] + dE * um, g2 = dl[2] + dE * vm, g3 = dl[3] + dE * wm;
        gfrho = dl[0] + g1 * um + g2 * vm + g3 * wm + dE * X;
        gum = g1 * frho + dE * Fm1;
        gvm = g2 * frho + dE * Fm2;
        gwm = g3 * frho + dE * Fm3;
        const double gph = g1 * nx + g2 * ny + g3 * nz;
        gra += 0.5 * rsb * gph;
        grb += 0.5 * rsb * gph;
        gba -= ph * rsb * gph;
        gbb -= ph * rsb * gph;
        const double gX = dE * frho;
        gibl = gX * c1;
        const double gq = -0.25 * gX;
        gua += 2.0 * gq * A.u; gva += 2.0 * gq * A.v; gwa += 2.0 * gq * A.w;
        gub += 2.0 * gq * B.u; gvb += 2.0 * gq * B.v; gwb += 2.0 * gq * B.w;
        gun = gfrho * rho_ln;
    }
    // frho = rho_ln * un
    const double grl = gfrho * un;
    gra += grl * Lra;
    grb += grl * Lrb;
    gba += gibl * Iba;
    gbb += gibl * Ibb;
    // un = (una + unb) / 2, una = u_a . N
    guna += 0.5 * gun;
    gunb += 0.5 * gun;
    gua += guna * nx + 0.5 * gum; gva += guna * ny + 0.5 * gvm; gwa += guna * nz + 0.5 * gwm;
    gub += gunb * nx + 0.5 * gum; gvb += gunb * ny + 0.5 * gvm; gwb += gunb * nz + 0.5 * gwm;
    gA[0] += gra; gA[1] += gua; gA[2] += gva; gA[3] += gwa; gA[4] += gpa; gA[5] += gba;
    gB[0] += grb; gB[1] += gub; gB[2] += gvb; gB[3] += gwb; gB[4] += gpb; gB[5] += gbb;
}

// mu = A lam (c != 0): Pi~^T, (W J)^-1, Pi~ along the three directions.
template <int P>
__global__ __launch_bounds__(VJP_BLOCK_MAX) void mass_apply_kernel(StageArgs A, const double* lam, double* mu) {
    constexpr int N = P + 1, N2 = N * N, N3 = N2 * N;
    extern __shared__ double lds[];
    const int tid = threadIdx.x, nth = blockDim.x;
    const int epb = A.epb;
    const int64_t E = A.geo.E, e0 = (int64_t)blockIdx.x * epb, SE = E * N3;
    for (int idx = tid; idx < epb * N3; idx += nth) {
        int el = idx / N3, node = idx - el * N3;
        int64_t e = e0 + el;
#pragma unroll
        for (int s = 0; s < 5; ++s) lds[(el * 5 + s) * N3 + node] = (e < E) ? lam[s * SE + e * N3 + node] : 0.0;
    }
    __syncthreads();
    for (int d = 0; d < 3; ++d) {
        for (int it = tid; it < epb * 5 * N2; it += nth) {
            int l = it % N2, sl = it / N2;
            int t1 = l % N, t2 = l / N;
            int base = d == 0 ? N * t1 + N2 * t2 : (d == 1 ? t1 + N2 * t2 : t1 + N * t2);
            int stride = d == 0 ? 1 : (d == 1 ? N : N2);
            double* x = lds + sl * N3 + base;
            double v[N], t = 0.0;
#pragma unroll
            for (int a = 0; a < N; ++a) { v[a] = x[a * stride]; t += A.ops.pia[a] * v[a]; }
#pragma unroll
            for (int a = 0; a < N; ++a) x[a * stride] = v[a] - A.ops.pib[a] * t;
        }
        __syncthreads();
    }
    for (int idx = tid; idx < epb * N3; idx += nth) {
        int el = idx / N3, node = idx - el * N3;
        int64_t e = e0 + el;
        double iw = (e < E) ? A.geo.invWJ[e * N3 + node] : 0.0;
#pragma unroll
        for (int s = 0; s < 5; ++s) lds[(el * 5 + s) * N3 + node] *= iw;
    }
    __syncthreads();
    for (int d = 0; d < 3; ++d) {
        for (int it = tid; it < epb * 5 * N2; it += nth) {
            int l = it % N2, sl = it / N2;
            int t1 = l % N, t2 = l / N;
            int base = d == 0 ? N * t1 + N2 * t2 : (d == 1 ? t1 + N2 * t2 : t1 + N * t2);
            int stride = d == 0 ? 1 : (d == 1 ? N : N2);
            double* x = lds + sl * N3 + base;
            double v[N], t = 0.0;
#pragma unroll
            for (int a = 0; a < N; ++a) { v[a] = x[a * stride]; t += A.ops.pib[a] * v[a]; }
#pragma unroll
            for (int a = 0; a < N; ++a) x[a * stride] = v[a] - A.ops.pia[a] * t;
        }
        __syncthreads();
    }
    for (int idx = tid; idx < epb * N3; idx += nth) {
        int el = idx / N3, node = idx - el * N3;
        int64_t e = e0 + el;
        if (e < E) {
#pragma unroll
            for (int s = 0; s < 5; ++s) mu[s * SE + e * N3 + node] = lds[(el * 5 + s) * N3 + node];
        }
    }
}

__device__ __forceinline__ int64_t nbr_elem(int64_t e, int dir, int side, int nx, int ny, int nz) {
    int ex = (int)(e % nx);
    int64_t r = e / nx;
    int ey = (int)(r % ny);
    int ez = (int)(r / ny);
    if (dir == 0) ex = (ex + side + nx) % nx;
    else if (dir == 1) ey = (ey + side + ny) % ny;
    else ez = (ez + side + nz) % nz;
    return ex + (int64_t)nx * (ey + (int64_t)ny * ez);
}

// Reverse sweep. mu_given: mu is read from `mu` (c != 0); otherwise
// mu = lam / (W J) is formed on the fly (c = 0, A diagonal).
template <int P, int VARIANT>
__global__ __launch_bounds__(VJP_BLOCK_MAX) void vjp_kernel(StageArgs A, const double* lam, const double* mu,
                                                            int mu_given, double* g) {
    constexpr int N = P + 1, N2 = N * N, N3 = N2 * N, LINES = 3 * N2;
    extern __shared__ double lds[];
    const int tid = threadIdx.x, nth = blockDim.x;
    const int epb = A.epb;
    const int64_t E = A.geo.E, e0 = (int64_t)blockIdx.x * epb, SE = E * N3;
    const double gm1 = A.gamma - 1.0, c1 = A.c1;
    double* lp = lds;                      // [epb][6][N3] primitives, later cotangents
    double* lm = lds + epb * 6 * N3;       // [epb][5][N3] mu

    for (int idx = tid; idx < epb * N3; idx += nth) {
        int el = idx / N3, node = idx - el * N3;
        int64_t e = e0 + el;
        if (e < E) {
            const double* U = A.Uin + e * N3 + node;
            Prim q = primitives(U[0], U[SE], U[2 * SE], U[3 * SE], U[4 * SE], gm1);
            double* L = lp + el * 6 * N3 + node;
            L[0] = q.rho; L[N3] = q.u; L[2 * N3] = q.v; L[3 * N3] = q.w; L[4 * N3] = q.p; L[5 * N3] = q.beta;
            const double iw = mu_given ? 1.0 : A.geo.invWJ[e * N3 + node];
            const double* src = (mu_given ? mu : lam) + e * N3 + node;
#pragma unroll
            for (int s = 0; s < 5; ++s) lm[(el * 5 + s) * N3 + node] = src[s * SE] * iw;
        }
    }
    __syncthreads();

    const bool lt = tid < epb * LINES;
    const int el = lt ? tid / LINES : 0;
    const int rem = tid - el * LINES;
    const int dir = rem / N2;
    const int l = rem - dir * N2;
    const int64_t e = e0 + el;
    const bool active = lt && (e < E);
    const int t1 = l % N, t2 = l / N;
    const int base = dir == 0 ? N * t1 + N2 * t2 : (dir == 1 ? t1 + N2 * t2 : t1 + N * t2);
    const int stride = dir == 0 ? 1 : (dir == 1 ? N : N2);

    Prim q[N];
    double cx[N], cy[N], cz[N];
    if (active) {
        const double* L = lp + el * 6 * N3;
#pragma unroll
        for (int a = 0; a < N; ++a) {
            int node = base + a * stride;
            q[a].rho = L[node]; q[a].u = L[N3 + node]; q[a].v = L[2 * N3 + node];
            q[a].w = L[3 * N3 + node]; q[a].p = L[4 * N3 + node]; q[a].beta = L[5 * N3 + node];
        }
        const double* Cl = A.geo.Cline + ((int64_t)(dir * 3) * E + e) * N3 + l;
#pragma unroll
        for (int a = 0; a < N; ++a) {
            cx[a] = Cl[a * N2];
            cy[a] = Cl[SE + a * N2];
            cz[a] = Cl[2 * SE + a * N2];
        }
    }
    __syncthreads();   // primitive block dead; mu block stays

    double G[N][6];
#pragma unroll
    for (int a = 0; a < N; ++a)
#pragma unroll
        for (int k = 0; k < 6; ++k) G[a][k] = 0.0;
    if (active) {
        const double* M = lm + el * 5 * N3 + base;
#pragma unroll
        for (int a = 0; a < N - 1; ++a) {
#pragma unroll
            for (int b = a + 1; b < N; ++b) {
                const double sab = A.ops.S1h[a][b];
                double dl[5];
#pragma unroll
                for (int s = 0; s < 5; ++s) dl[s] = sab * (M[s * N3 + a * stride] - M[s * N3 + b * stride]);
                ec_flux_vjp<VARIANT>(q[a], q[b], cx[a] + cx[b], cy[a] + cy[b], cz[a] + cz[b], c1, dl, G[a], G[b]);
            }
        }
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int aown = side ? N - 1 : 0;
            const int anbr = side ? 0 : N - 1;
            const double sg = side ? 0.5 : -0.5;
            const int64_t en = nbr_elem(e, dir, side ? 1 : -1, A.geo.nx, A.geo.ny, A.geo.nz);
            const double* Cn = A.geo.Cline + ((int64_t)(dir * 3) * E + en) * N3 + anbr * N2 + l;
            const int64_t gn = en * N3 + base + anbr * stride;
            const double* Ub = A.Uin + gn;
            Prim qn = primitives(Ub[0], Ub[SE], Ub[2 * SE], Ub[3 * SE], Ub[4 * SE], gm1);
            const double iwn = mu_given ? 1.0 : A.geo.invWJ[gn];
            const double* src = (mu_given ? mu : lam) + gn;
            double dl[5];
#pragma unroll
            for (int s = 0; s < 5; ++s) dl[s] = M[s * N3 + aown * stride] - src[s * SE] * iwn;
            double nx = sg * (cx[aown] + Cn[0]), ny = sg * (cy[aown] + Cn[SE]), nz = sg * (cz[aown] + Cn[2 * SE]);
            double gdummy[6] = {0, 0, 0, 0, 0, 0};
            ec_flux_vjp<VARIANT>(q[aown], qn, nx, ny, nz, c1, dl, G[aown], gdummy);
        }
    }
    __syncthreads();   // mu reads done before the cotangent block is written

    const double wperp = A.ops.w[t1] * A.ops.w[t2];
    for (int ph = 0; ph < 3; ++ph) {
        if (active && dir == ph) {
            double* x = lp + el * 6 * N3 + base;
#pragma unroll
            for (int k = 0; k < 6; ++k)
#pragma unroll
                for (int a = 0; a < N; ++a) {
                    double v = G[a][k] * wperp;
                    if (ph == 0) x[k * N3 + a * stride] = v;
                    else x[k * N3 + a * stride] += v;
                }
        }
        __syncthreads();
    }

    // primitive cotangents -> conservative cotangents, g = -(dR/dU)^T mu
    for (int idx = tid; idx < epb * N3; idx += nth) {
        int eli = idx / N3, node = idx - eli * N3;
        int64_t ee = e0 + eli;
        if (ee >= E) continue;
        const int64_t gi = ee * N3 + node;
        const double* U = A.Uin + gi;
        const double r = U[0];
        const double ir = 1.0 / r;
        const double u = U[SE] * ir, v = U[2 * SE] * ir, w = U[3 * SE] * ir;
        const double p = gm1 * (U[4 * SE] - 0.5 * r * (u * u + v * v + w * w));
        const double beta = 0.5 * r / p;
        const double* x = lp + eli * 6 * N3 + node;
        double gr = x[0], gu = x[N3], gv = x[2 * N3], gw = x[3 * N3], gp = x[4 * N3], gb = x[5 * N3];
        // beta = rho / (2 p)
        gr += gb * 0.5 / p;
        gp -= gb * beta / p;
        // p = (gamma-1)(E - |m|^2 / (2 rho)), u = m / rho
        const double gE = gm1 * gp;
        const double gm1x = gu * ir - gm1 * u * gp;
        const double gm2 = gv * ir - gm1 * v * gp;
        const double gm3 = gw * ir - gm1 * w * gp;
        const double grho = gr - (gu * u + gv * v + gw * w) * ir + gm1 * 0.5 * (u * u + v * v + w * w) * gp;
        g[gi] = -grho;
        g[SE + gi] = -gm1x;
        g[2 * SE + gi] = -gm2;
        g[3 * SE + gi] = -gm3;
        g[4 * SE + gi] = -gE;
    }
}

template <int P>
static hipError_t vjp_p(bool cwa, int variant, const StageArgs& a, const double* lam, double* g, double* mu_ws,
                        hipStream_t s) {
    constexpr int N = P + 1, N3 = N * N * N, LINES = 3 * N * N;
    int threads = ((a.epb * LINES + 63) / 64) * 64;
    unsigned blocks = (unsigned)((a.geo.E + a.epb - 1) / a.epb);
    if (cwa) {
        mass_apply_kernel<P><<<blocks, threads, (size_t)a.epb * 5 * N3 * sizeof(double), s>>>(a, lam, mu_ws);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    size_t lds = (size_t)a.epb * 11 * N3 * sizeof(double);
    if (variant)
        vjp_kernel<P, 1><<<blocks, threads, lds, s>>>(a, lam, mu_ws, cwa ? 1 : 0, g);
    else
        vjp_kernel<P, 0><<<blocks, threads, lds, s>>>(a, lam, mu_ws, cwa ? 1 : 0, g);
    return hipGetLastError();
}

hipError_t launch_vjp(int p, bool cwa, int variant, const StageArgs& a0, const double* lam, double* g, double* mu_ws,
                      hipStream_t s) {
    // the reverse sweep keeps 11 doubles per node in LDS; stay within 64 KiB
    StageArgs a = a0;
    const int n3 = (p + 1) * (p + 1) * (p + 1);
    const int lds_cap = (int)(65536 / (11 * n3 * sizeof(double)));
    if (a.epb > lds_cap) a.epb = lds_cap;
    if (a.epb < 1 || a.epb * 3 * (p + 1) * (p + 1) > VJP_BLOCK_MAX) return hipErrorInvalidValue;
    switch (p) {
        case 2: return vjp_p<2>(cwa, variant, a, lam, g, mu_ws, s);
        case 3: return vjp_p<3>(cwa, variant, a, lam, g, mu_ws, s);
        case 4: return vjp_p<4>(cwa, variant, a, lam, g, mu_ws, s);
        case 5: return vjp_p<5>(cwa, variant, a, lam, g, mu_ws, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace nsfr
