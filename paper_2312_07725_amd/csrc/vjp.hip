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

// A logarithmic mean (or its reciprocal) and its two partial derivatives.
struct MeanGrad {
    double v, da, db;
};

// Closed-form branches of the two derivative helpers below, kept out of line
// so that their logarithms are only evaluated for the rare pairs that need
// them; results are returned by value (in registers).
__device__ __noinline__ MeanGrad ln_mean_grad_closed(double a, double b) {
    const double la = log(a), lb = log(b);
    const double il = 1.0 / (la - lb);
    MeanGrad r;
    r.v = (a - b) * il;
    r.da = (1.0 - r.v / a) * il;
    r.db = (r.v / b - 1.0) * il;
    return r;
}

__device__ __noinline__ MeanGrad inv_ln_mean_grad_closed(double a, double b) {
    const double la = log(a), lb = log(b);
    const double L = (a - b) / (la - lb);
    const double il = 1.0 / (la - lb);
    const double La = (1.0 - L / a) * il, Lb = (L / b - 1.0) * il;
    MeanGrad r;
    r.v = 1.0 / L;
    r.da = -r.v * r.v * La;
    r.db = -r.v * r.v * Lb;
    return r;
}

// The logarithmic mean L(a, b) and its partial derivatives (L is homogeneous
// of degree one): with s = a + b, f = (a - b)/s and G(f) = f / atanh(f),
// dL/da = (G + G' (1 - f)) / 2, dL/db = (G - G' (1 + f)) / 2.
__device__ __forceinline__ MeanGrad ln_mean_grad(double a, double b) {
    const double s = a + b, d = a - b;
    const double f = d * rcp_pos(s);
    const double u = f * f;
    MeanGrad r;
    const double G = __builtin_fma(u, __builtin_fma(u, __builtin_fma(u, -44.0 / 945.0, -4.0 / 45.0), -1.0 / 3.0), 1.0);
    const double Gp = f * __builtin_fma(u, __builtin_fma(u, __builtin_fma(u, -3424.0 / 14175.0, -264.0 / 945.0),
                                                         -16.0 / 45.0), -2.0 / 3.0);
    r.v = 0.5 * s * G;
    r.da = 0.5 * (G + Gp * (1.0 - f));
    r.db = 0.5 * (G - Gp * (1.0 + f));
    if (u >= LN_SWITCH) r = ln_mean_grad_closed(a, b);
    return r;
}

// IL = 1 / L(a, b) and its partial derivatives: with H(f) = atanh(f) / f,
// IL = (2/s) H, dIL/da = (2/s^2)(-H + H' (1 - f)), dIL/db = (2/s^2)(-H - H' (1 + f)).
__device__ __forceinline__ MeanGrad inv_ln_mean_grad(double a, double b, double rs) {
    const double d = a - b;
    const double f = d * rs;
    const double u = f * f;
    MeanGrad r;
    const double H = __builtin_fma(u, __builtin_fma(u, __builtin_fma(u, 1.0 / 7.0, 1.0 / 5.0), 1.0 / 3.0), 1.0);
    const double Hp = f * __builtin_fma(u, __builtin_fma(u, __builtin_fma(u, 8.0 / 9.0, 6.0 / 7.0), 4.0 / 5.0), 2.0 / 3.0);
    const double k = 2.0 * rs * rs;
    r.v = 2.0 * rs * H;
    r.da = k * (-H + Hp * (1.0 - f));
    r.db = k * (-H - Hp * (1.0 + f));
    if (u >= LN_SWITCH) r = inv_ln_mean_grad_closed(a, b);
    return r;
}

// One-sided adjoint: accumulate only the primitive cotangents of A in
// dl . f_s(A, B; N). Used by the node-centric reverse sweep, where each node
// of a line differentiates its own side of every pair it belongs to.
template <int VARIANT>
__device__ __forceinline__ void ec_flux_vjp_a(const Prim& A, const Prim& B, double nx, double ny, double nz,
                                              double c1, const double dl[5], double gA[6]) {
    const double una = A.u * nx + A.v * ny + A.w * nz;
    const double unb = B.u * nx + B.v * ny + B.w * nz;
    const double un = 0.5 * (una + unb);
    const MeanGrad lr = ln_mean_grad(A.rho, B.rho);
    const double rsb = rcp_pos(A.beta + B.beta);
    const MeanGrad lb = inv_ln_mean_grad(A.beta, B.beta, rsb);
    const double frho = lr.v * un;
    const double um = 0.5 * (A.u + B.u), vm = 0.5 * (A.v + B.v), wm = 0.5 * (A.w + B.w);
    const double dE = dl[4];
    double gra, gua, gva, gwa, gpa, gba, gun, guna;
    if (VARIANT == 0) {
        const double pm = 0.5 * (A.p + B.p);
        const double uab = A.u * B.u + A.v * B.v + A.w * B.w;
        const double X = c1 * lb.v + 0.5 * uab;
        const double gfrho = dl[0] + dl[1] * um + dl[2] * vm + dl[3] * wm + dE * X;
        const double guab = 0.5 * dE * frho;
        gun = gfrho * lr.v + dE * pm;
        guna = 0.5 * gun - 0.25 * dE * (A.p - B.p);
        gua = guab * B.u + 0.5 * dl[1] * frho;
        gva = guab * B.v + 0.5 * dl[2] * frho;
        gwa = guab * B.w + 0.5 * dl[3] * frho;
        gpa = 0.5 * (dl[1] * nx + dl[2] * ny + dl[3] * nz + dE * un) - 0.25 * dE * (una - unb);
        gra = gfrho * un * lr.da;
        gba = dE * frho * c1 * lb.da;
    } else {
        const double ph = 0.5 * (A.rho + B.rho) * rsb;
        const double qa = A.u * A.u + A.v * A.v + A.w * A.w;
        const double qb = B.u * B.u + B.v * B.v + B.w * B.w;
        const double X = c1 * lb.v - 0.25 * (qa + qb);
        const double Fm1 = um * frho + ph * nx, Fm2 = vm * frho + ph * ny, Fm3 = wm * frho + ph * nz;
        const double g1 = dl[1] + dE * um, g2 = dl[2] + dE * vm, g3 = dl[3] + dE * wm;
        const double gfrho = dl[0] + g1 * um + g2 * vm + g3 * wm + dE * X;
        const double gph = g1 * nx + g2 * ny + g3 * nz;
        const double gX = dE * frho;
        const double gq2 = -0.5 * gX;   // 2 * (-1/4) gX
        gun = gfrho * lr.v;
        guna = 0.5 * gun;
        gua = gq2 * A.u + 0.5 * (g1 * frho + dE * Fm1);
        gva = gq2 * A.v + 0.5 * (g2 * frho + dE * Fm2);
        gwa = gq2 * A.w + 0.5 * (g3 * frho + dE * Fm3);
        gpa = 0.0;
        gra = 0.5 * rsb * gph + gfrho * un * lr.da;
        gba = -ph * rsb * gph + gX * c1 * lb.da;
    }
    gA[0] += gra;
    gA[1] += gua + guna * nx;
    gA[2] += gva + guna * ny;
    gA[3] += gwa + guna * nz;
    gA[4] += gpa;
    gA[5] += gba;
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

// LDS doubles per element of the reverse sweep: primitives [6][PN3], metric
// columns [9][N3] (line-major), mu [5][PN3].
__host__ __device__ constexpr int vjp_lds_doubles(int n) {
    return 11 * (n * n * n + n * n) + 9 * n * n * n;
}

// Reverse sweep, node-centric. mu_given: mu is read from `mu` (c != 0);
// otherwise mu = lam / (W J) is formed on the fly (c = 0, A diagonal).
// One thread per node. For each of the three line directions in turn it
// differentiates its own side of the pairs its node forms along that line,
// and its own side of the face pair if the node is a line end. Every pair is
// thus evaluated twice, once per side, which keeps the per-thread state to
// one node: the loop over partners stays rolled, the cotangent of the node
// accumulates in registers in a fixed order (deterministic), and no
// cross-thread reduction is needed.
template <int P, int VARIANT>
__global__ __launch_bounds__(VJP_BLOCK_MAX) void vjp_kernel(StageArgs A, const double* lam, const double* mu,
                                                            int mu_given, double* g) {
    constexpr int N = P + 1, N2 = N * N, N3 = N2 * N;
    constexpr int PN3 = padded_block<N>();
    constexpr int LDSE = vjp_lds_doubles(N);
    extern __shared__ double lds[];
    __shared__ double sS1h[N][N];
    const int tid = threadIdx.x, nth = blockDim.x;
    const int epb = A.epb;
    const int64_t E = A.geo.E, SE = E * N3;
    const int64_t e0 = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * epb;
    const double gm1 = A.gamma - 1.0, c1 = A.c1;

    if (tid < N * N) sS1h[tid / N][tid % N] = A.ops.S1h[tid / N][tid % N];
    for (int idx = tid; idx < epb * N3; idx += nth) {
        const int el = idx / N3, node = idx - el * N3;
        const int64_t e = e0 + el;
        if (e < E) {
            const double* U = A.Uin + e * N3 + node;
            const Prim q = primitives(U[0], U[SE], U[2 * SE], U[3 * SE], U[4 * SE], gm1);
            double* L = lds + el * LDSE + pad_node<N>(node);
            L[0] = q.rho; L[PN3] = q.u; L[2 * PN3] = q.v; L[3 * PN3] = q.w; L[4 * PN3] = q.p; L[5 * PN3] = q.beta;
            const double iw = mu_given ? 1.0 : A.geo.invWJ[e * N3 + node];
            const double* src = (mu_given ? mu : lam) + e * N3 + node;
            double* Lm = lds + el * LDSE + 6 * PN3 + 9 * N3 + pad_node<N>(node);
#pragma unroll
            for (int s = 0; s < 5; ++s) Lm[s * PN3] = src[s * SE] * iw;
            const double* Cg = A.geo.Cline + e * N3 + node;
            double* Lc0 = lds + el * LDSE + 6 * PN3 + node;
#pragma unroll
            for (int k = 0; k < 9; ++k) Lc0[k * N3] = Cg[k * SE];
        }
    }
    __syncthreads();

    const int el = tid / N3;
    const int node = tid - el * N3;
    const int64_t e = e0 + el;
    if (el >= epb || e >= E) return;   // no barrier follows
    const int i = node % N, j = (node / N) % N, k = node / N2;
    const double* Lp = lds + el * LDSE;
    const double* Lm = lds + el * LDSE + 6 * PN3 + 9 * N3;
    const int pa = pad_node<N>(node);
    const Prim qa = lds_prim<PN3>(Lp, pa);
    double ma[5];
#pragma unroll
    for (int s = 0; s < 5; ++s) ma[s] = Lm[s * PN3 + pa];

    double G[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll 1
    for (int dir = 0; dir < 3; ++dir) {
        // position of the node on its line, the line index and its stride
        const int a = dir == 0 ? i : (dir == 1 ? j : k);
        const int l = dir == 0 ? j + N * k : (dir == 1 ? i + N * k : i + N * j);
        const int stride = dir == 0 ? 1 : (dir == 1 ? N : N2);
        const int base = node - a * stride;
        const int pbase = pad_node<N>(base), pstride = padded_stride<N>(dir);   // the line in the LDS node index
        const double* Lc = Lp + 6 * PN3 + 3 * dir * N3 + l;
        const double cax = Lc[a * N2], cay = Lc[N3 + a * N2], caz = Lc[2 * N3 + a * N2];
        double Gd[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll 1
        for (int b = 0; b < N; ++b) {
            if (b == a) continue;
            const int pb = pbase + b * pstride;
            const Prim qb = lds_prim<PN3>(Lp, pb);
            const double sab = sS1h[a][b];
            double dl[5];
#pragma unroll
            for (int s = 0; s < 5; ++s) dl[s] = sab * (ma[s] - Lm[s * PN3 + pb]);
            ec_flux_vjp_a<VARIANT>(qa, qb, cax + Lc[b * N2], cay + Lc[N3 + b * N2], caz + Lc[2 * N3 + b * N2], c1,
                                   dl, Gd);
        }
        if (a == 0 || a == N - 1) {
            const int side = (a == N - 1) ? 1 : 0;
            const int anbr = side ? 0 : N - 1;
            const double sg = side ? 0.5 : -0.5;
            const int64_t en = neighbour(e, dir, side ? 1 : -1, A.geo.nx, A.geo.ny, A.geo.nz);
            const double* Cn = A.geo.Cline + ((int64_t)(dir * 3) * E + en) * N3 + anbr * N2 + l;
            const int64_t gn = en * N3 + base + anbr * stride;
            const double* Ub = A.Uin + gn;
            const Prim qn = primitives(Ub[0], Ub[SE], Ub[2 * SE], Ub[3 * SE], Ub[4 * SE], gm1);
            const double iwn = mu_given ? 1.0 : A.geo.invWJ[gn];
            const double* src = (mu_given ? mu : lam) + gn;
            double dl[5];
#pragma unroll
            for (int s = 0; s < 5; ++s) dl[s] = ma[s] - src[s * SE] * iwn;
            ec_flux_vjp_a<VARIANT>(qa, qn, sg * (cax + Cn[0]), sg * (cay + Cn[SE]), sg * (caz + Cn[2 * SE]), c1, dl,
                                   Gd);
        }
        const double wperp = A.ops.w[l % N] * A.ops.w[l / N];
#pragma unroll
        for (int s = 0; s < 6; ++s) G[s] = __builtin_fma(wperp, Gd[s], G[s]);
    }

    // primitive cotangents -> conservative cotangents, g = -(dR/dU)^T mu
    const int64_t gi = e * N3 + node;
    const double ir = rcp_pos(qa.rho);
    const double u = qa.u, v = qa.v, w = qa.w, pp = qa.p;
    const double ip = rcp_pos(pp);
    double gr = G[0], gp = G[4];
    // beta = rho / (2 p)
    gr += G[5] * 0.5 * ip;
    gp -= G[5] * qa.beta * ip;
    // p = (gamma-1)(E - |m|^2 / (2 rho)), u = m / rho
    const double gE = gm1 * gp;
    const double gm1x = G[1] * ir - gm1 * u * gp;
    const double gm2 = G[2] * ir - gm1 * v * gp;
    const double gm3 = G[3] * ir - gm1 * w * gp;
    const double grho = gr - (G[1] * u + G[2] * v + G[3] * w) * ir + gm1 * 0.5 * (u * u + v * v + w * w) * gp;
    g[gi] = -grho;
    g[SE + gi] = -gm1x;
    g[2 * SE + gi] = -gm2;
    g[3 * SE + gi] = -gm3;
    g[4 * SE + gi] = -gE;
}

template <int P>
static hipError_t vjp_p(bool cwa, int variant, const StageArgs& a, const double* lam, double* g, double* mu_ws,
                        hipStream_t s) {
    constexpr int N = P + 1, N3 = N * N * N, LINES = 3 * N * N;
    int threads = ((a.epb * LINES + 63) / 64) * 64;            // mass kernel: one thread per line
    int vthreads = ((a.epb * N3 + 63) / 64) * 64;              // reverse sweep: one per node
    unsigned blocks = (unsigned)((a.geo.E + a.epb - 1) / a.epb);
    if (cwa) {
        mass_apply_kernel<P><<<blocks, threads, (size_t)a.epb * 5 * N3 * sizeof(double), s>>>(a, lam, mu_ws);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    size_t lds = (size_t)a.epb * vjp_lds_doubles(N) * sizeof(double);
    if (variant)
        vjp_kernel<P, 1><<<blocks, vthreads, lds, s>>>(a, lam, mu_ws, cwa ? 1 : 0, g);
    else
        vjp_kernel<P, 0><<<blocks, vthreads, lds, s>>>(a, lam, mu_ws, cwa ? 1 : 0, g);
    return hipGetLastError();
}

hipError_t launch_vjp(int p, bool cwa, int variant, const StageArgs& a0, const double* lam, double* g, double* mu_ws,
                      hipStream_t s) {
    // as many elements per workgroup as 64 KiB of LDS and the block size allow
    StageArgs a = a0;
    const int n = p + 1;
    const int lds_cap = (int)(65536 / (vjp_lds_doubles(n) * sizeof(double)));
    const int thr_cap = VJP_BLOCK_MAX / (n * n * n);
    a.epb = lds_cap < thr_cap ? lds_cap : thr_cap;
    if (a.epb < 1 || a.epb * 3 * n * n > VJP_BLOCK_MAX) return hipErrorInvalidValue;
    switch (p) {
        case 2: return vjp_p<2>(cwa, variant, a, lam, g, mu_ws, s);
        case 3: return vjp_p<3>(cwa, variant, a, lam, g, mu_ws, s);
        case 4: return vjp_p<4>(cwa, variant, a, lam, g, mu_ws, s);
        case 5: return vjp_p<5>(cwa, variant, a, lam, g, mu_ws, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace nsfr
