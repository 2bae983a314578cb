// Device building blocks shared by the NSFR kernels (gfx950, FP64).
//
// Paper references: Sec. 2.1 (Euler system, entropy variables, Tadmor's
// condition Eq. EC flux), Sec. 3.3 (entropy-conserving two-point flux of
// Chandrashekar in the variables rho, u, beta = rho / (2p); the experiments of
// Sec. 7 use Ranocha's pressure fix, stated in the opening paragraph of
// Sec. 7), Sec. 6.1 (free-stream preservation).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nsfr {

constexpr int MAXN = 6;   // p <= 5

// 1D operators of degree p, passed to kernels by value (kernel-argument
// memory, read through the scalar cache).
struct Ops {
    double w[MAXN];            // LGL weights
    double S1h[MAXN][MAXN];    // (W D - D^T W) / 2: volume block of (Q~ - Q~^T), halved
    double D[MAXN][MAXN];      // strong derivative D_ij = l_j'(x_i)
    double pia[MAXN];          // FR projection Pi~ = I - pia pib^T (rank one)
    double pib[MAXN];
    double x[MAXN];            // LGL nodes
};

// Per-node primitive variables used by the two-point flux.
struct Prim {
    double rho, u, v, w, p, beta;
};

// 1/x for x > 0 normal: hardware reciprocal estimate refined by two Newton
// steps (error well below one ulp of the products that use it).
__device__ __forceinline__ double rcp_pos(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}

__device__ __forceinline__ Prim primitives(double r, double m1, double m2, double m3, double E, double gm1) {
    Prim q;
    double ir = rcp_pos(r);
    q.rho = r;
    q.u = m1 * ir;
    q.v = m2 * ir;
    q.w = m3 * ir;
    double kin = 0.5 * (m1 * q.u + m2 * q.v + m3 * q.w);
    q.p = gm1 * (E - kin);
    q.beta = 0.5 * r * rcp_pos(q.p);
    return q;
}

// Primitive variables of the forward kernels. The pressure is carried as its
// difference pd = p - pref from a reference pressure pref that is constant over
// the mesh for one evaluation.
//
// Why: in low-Mach flows p is a large constant plus a small variation (the
// Mach-0.1 vortex has p ~ 71 varying by ~0.3), and the momentum residual is the
// derivative of the variation. The constant part pref of the momentum flux
// pref N sums to exactly zero at every node in exact arithmetic: its volume
// and surface contributions are the free-stream residual of a constant state,
// which vanishes by the discrete GCL and the single-valued face metric
// (Sec. 6.1). Evaluated in FP64 it leaves round-off of order eps pref |C|,
// which is most of the momentum residual's round-off. The forward kernels
// therefore drop pref N from the momentum flux (keeping it in the energy
// flux, where pref un does not cancel) and need pd accurate to eps |pd|, not
// eps p: E - kin is formed with its exact rounding remainder (Fast2Sum, valid
// since E >= kin when p > 0) and the product with gamma - 1 with its FMA
// remainder, so that pd = (p_hi - pref) + p_lo loses nothing to the
// cancellation of p_hi against pref.
struct PrimR {
    double rho, u, v, w, pd, beta;
};

// Every operation is rounded as written (no FMA contraction): the kernels
// evaluate this at several sites (staging, face traces) and rely on getting
// the same bits for the same state, and the Fast2Sum of E - kin is exact only
// when kin is the same rounded value in both of its uses.
__device__ __forceinline__ PrimR primitives_ref(double r, double m1, double m2, double m3, double E, double gm1,
                                                double pref) {
#pragma clang fp contract(off)
    PrimR q;
    double ir = rcp_pos(r);
    q.rho = r;
    q.u = m1 * ir;
    q.v = m2 * ir;
    q.w = m3 * ir;
    double kin = 0.5 * (m1 * q.u + m2 * q.v + m3 * q.w);
    double s = E - kin;
    double es = (E - s) - kin;                        // E - kin = s + es exactly
    double ph = gm1 * s;
    double pl = __builtin_fma(gm1, s, -ph) + gm1 * es; // gm1 (E - kin) = ph + pl
    q.pd = (ph - pref) + pl;
    q.beta = 0.5 * r * rcp_pos(ph);
    return q;
}

// Reference pressure of one evaluation: the pressure at the first node of the
// state array (plain FP64; every workgroup computes the identical value).
__device__ __forceinline__ double reference_pressure(const double* U, int64_t SE, double gm1) {
    const double r = U[0], m1 = U[SE], m2 = U[2 * SE], m3 = U[3 * SE], E = U[4 * SE];
    return gm1 * (E - 0.5 * (m1 * m1 + m2 * m2 + m3 * m3) / r);
}

// Threshold on the squared relative jump below which the logarithmic mean
// uses its series: at u < 1e-4 the first omitted term of either series is
// below u^4 / 9 < 1.2e-17 relative, under half an FP64 ulp.
constexpr double LN_SWITCH = 1e-4;

// Closed forms of the logarithmic mean and of its reciprocal, for the rare
// pairs whose squared relative jump exceeds the series switch. Kept out of
// line: inlined, the compiler hoists and shares the logarithms of the node
// values across all pairs of a line and evaluates them unconditionally.
__device__ __noinline__ double ln_mean_closed(double a, double b) { return (a - b) / (log(a) - log(b)); }
__device__ __noinline__ double inv_ln_mean_closed(double a, double b) { return (log(a) - log(b)) / (a - b); }

// Logarithmic mean (a - b) / (ln a - ln b). Series branch:
// s / 2 * f / atanh(f) with f = (a - b) / s, u = f^2, and
// f / atanh(f) = 1 - u/3 - 4u^2/45 - 44u^3/945 - ..., truncated after u^3
// (relative truncation below 3e-18 for u < 1e-4). Exactly symmetric in (a, b).
__device__ __forceinline__ double ln_mean(double a, double b) {
    double s = a + b, d = a - b;
    double f = d * rcp_pos(s);
    double u = f * f;
    if (u < LN_SWITCH) {
        double q = __builtin_fma(u, __builtin_fma(u, __builtin_fma(u, -44.0 / 945.0, -4.0 / 45.0), -1.0 / 3.0), 1.0);
        return 0.5 * s * q;
    }
    return ln_mean_closed(a, b);
}

// Reciprocal of the logarithmic mean, (ln a - ln b) / (a - b); series branch
// 2 / s * atanh(f) / f with atanh(f) / f = 1 + u/3 + u^2/5 + u^3/7 + ...
__device__ __forceinline__ double inv_ln_mean(double a, double b, double rs) {
    double d = a - b;
    double f = d * rs;
    double u = f * f;
    if (u < LN_SWITCH) {
        double q = __builtin_fma(u, __builtin_fma(u, __builtin_fma(u, 1.0 / 7.0, 1.0 / 5.0), 1.0 / 3.0), 1.0);
        return 2.0 * rs * q;
    }
    return inv_ln_mean_closed(a, b);
}

// Entropy-conserving, kinetic-energy-preserving two-point flux f_s(A, B) . N
// for the (unnormalised) direction N (Sec. 3.3; Tadmor's condition, Eq. EC
// flux), with the constant pref N left out of the momentum flux (see PrimR).
// VARIANT 0: momentum pressure is the arithmetic mean of p, energy flux
// completed by Tadmor's condition (Ranocha's pressure fix); VARIANT 1: plain
// Chandrashekar, pressure rho_avg / (2 beta_avg), whose difference from pref
// is the beta-weighted mean (beta_a pd_a + beta_b pd_b) / (beta_a + beta_b).
//
// Every expression is written so that swapping A and B leaves each rounded
// operand unchanged or negates both factors of a product, so the result is
// bitwise symmetric in (A, B) and odd in N even under FMA contraction.
template <int VARIANT>
__device__ __forceinline__ void ec_flux(const PrimR& A, const PrimR& B, double nx, double ny, double nz,
                                        double c1, double pref, double F[5]) {
    double una = A.u * nx + A.v * ny + A.w * nz;
    double unb = B.u * nx + B.v * ny + B.w * nz;
    double un = 0.5 * (una + unb);
    double rho_ln = ln_mean(A.rho, B.rho);
    double rsb = rcp_pos(A.beta + B.beta);
    double ibl = inv_ln_mean(A.beta, B.beta, rsb);
    double frho = rho_ln * un;
    double um = 0.5 * (A.u + B.u), vm = 0.5 * (A.v + B.v), wm = 0.5 * (A.w + B.w);
    F[0] = frho;
    if (VARIANT == 0) {
        double pm = 0.5 * (A.pd + B.pd);
        F[1] = um * frho + pm * nx;
        F[2] = vm * frho + pm * ny;
        F[3] = wm * frho + pm * nz;
        double uab = A.u * B.u + A.v * B.v + A.w * B.w;
        double pe = (pm + pref) * un - 0.25 * (A.pd - B.pd) * (una - unb);   // = (pa unb + pb una) / 2
        F[4] = frho * (c1 * ibl + 0.5 * uab) + pe;
    } else {
        double ph = (__dmul_rn(A.beta, A.pd) + __dmul_rn(B.beta, B.pd)) * rsb;
        F[1] = um * frho + ph * nx;
        F[2] = vm * frho + ph * ny;
        F[3] = wm * frho + ph * nz;
        double qa = A.u * A.u + A.v * A.v + A.w * A.w;
        double qb = B.u * B.u + B.v * B.v + B.w * B.w;
        F[4] = frho * (c1 * ibl - 0.25 * (qa + qb)) + (um * F[1] + vm * F[2] + wm * F[3]) + pref * un;
    }
}

// Local Lax-Friedrichs term -|N| lambda_max (UB - UA) / 2 added to the
// surface flux of the manufactured-solution runs (the upwind dissipation of
// Sec. 7.1, read as local Lax-Friedrichs on the conservative jumps).
__device__ __forceinline__ void llf_add(const PrimR& A, const PrimR& B, const double UA[5], const double UB[5],
                                        double nx, double ny, double nz, double gamma, double pref, double F[5]) {
    double nn = sqrt(nx * nx + ny * ny + nz * nz);
    double inn = 1.0 / nn;
    double una = fabs((A.u * nx + A.v * ny + A.w * nz) * inn);
    double unb = fabs((B.u * nx + B.v * ny + B.w * nz) * inn);
    double ca = sqrt(gamma * (pref + A.pd) / A.rho), cb = sqrt(gamma * (pref + B.pd) / B.rho);
    double lam = fmax(una + ca, unb + cb);
    double k = 0.5 * lam * nn;
    for (int s = 0; s < 5; ++s) F[s] -= k * (UB[s] - UA[s]);
}

// Entropy-stable Roe-type matrix dissipation on the jump of the entropy
// variables, F -= |N| R |Lambda| T R^T [v] / 2 (Sec. 6.3: Roe's dissipation
// recast with entropy-variable jumps dissipates entropy; Sec. 7.1: the
// manufactured-solution runs add Roe dissipation to the EC flux). R, Lambda
// and Barth's scaling T (R T R^T = du/dv) are those of the flux Jacobian in
// the direction n = N / |N| at the averaged state (logarithmic-mean density,
// mean velocity, p = mean(rho) / (2 mean(beta))): two acoustic waves, the
// entropy wave, and the shear block p |u.n| (I - n n^T) acting on
// w = [v]_m + u [v]_E. The entropy jump uses log1p of the relative jumps, so
// that near-equal states keep their relative accuracy.
__device__ __forceinline__ void roe_add(const PrimR& A, const PrimR& B, double nx, double ny, double nz,
                                        double gamma, double pref, double F[5]) {
    const double gm1 = gamma - 1.0;
    const double pa = pref + A.pd, pb = pref + B.pd;
    // jump of the entropy variables [v] = v(B) - v(A)
    const double ds = log1p((B.pd - A.pd) / pa) - gamma * log1p((B.rho - A.rho) / A.rho);
    const double qa = A.u * A.u + A.v * A.v + A.w * A.w, qb = B.u * B.u + B.v * B.v + B.w * B.w;
    double dv[5];
    dv[0] = -ds / gm1 - (B.beta * qb - A.beta * qa);
    dv[1] = 2.0 * (B.beta * B.u - A.beta * A.u);
    dv[2] = 2.0 * (B.beta * B.v - A.beta * A.v);
    dv[3] = 2.0 * (B.beta * B.w - A.beta * A.w);
    dv[4] = -2.0 * (B.beta - A.beta);
    (void)pb;
    // averaged state
    const double rho = ln_mean(A.rho, B.rho);
    const double u = 0.5 * (A.u + B.u), v = 0.5 * (A.v + B.v), w = 0.5 * (A.w + B.w);
    const double p = 0.5 * (A.rho + B.rho) / (A.beta + B.beta);
    const double nn = sqrt(nx * nx + ny * ny + nz * nz);
    const double inn = 1.0 / nn;
    const double n0 = nx * inn, n1 = ny * inn, n2 = nz * inn;
    const double a = sqrt(gamma * p / rho);
    const double q2 = u * u + v * v + w * w;
    const double h = a * a / gm1 + 0.5 * q2;
    const double un = u * n0 + v * n1 + w * n2;
    double D[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 2; ++k) {   // acoustic waves u.n -+ a
        const double sg = k ? 1.0 : -1.0;
        const double r1 = u + sg * a * n0, r2 = v + sg * a * n1, r3 = w + sg * a * n2, r4 = h + sg * a * un;
        const double c = (dv[0] + r1 * dv[1] + r2 * dv[2] + r3 * dv[3] + r4 * dv[4]) * fabs(un + sg * a) * rho /
                         (2.0 * gamma);
        D[0] += c;
        D[1] += c * r1;
        D[2] += c * r2;
        D[3] += c * r3;
        D[4] += c * r4;
    }
    {   // entropy wave u.n
        const double c = (dv[0] + u * dv[1] + v * dv[2] + w * dv[3] + 0.5 * q2 * dv[4]) * fabs(un) * gm1 * rho / gamma;
        D[0] += c;
        D[1] += c * u;
        D[2] += c * v;
        D[3] += c * w;
        D[4] += c * 0.5 * q2;
    }
    {   // shear waves u.n
        const double w0 = dv[1] + u * dv[4], w1 = dv[2] + v * dv[4], w2 = dv[3] + w * dv[4];
        const double wn = w0 * n0 + w1 * n1 + w2 * n2;
        const double P0 = w0 - wn * n0, P1 = w1 - wn * n1, P2 = w2 - wn * n2;
        const double c = fabs(un) * p;
        D[1] += c * P0;
        D[2] += c * P1;
        D[3] += c * P2;
        D[4] += c * (u * P0 + v * P1 + w * P2);
    }
    const double k2 = 0.5 * nn;
#pragma unroll
    for (int s = 0; s < 5; ++s) F[s] -= k2 * D[s];
}

// Manufactured-solution source q(x, t) of Sec. 7.1.
__device__ __forceinline__ void mms_source(double x, double y, double z, double t, double gamma, double q[5]) {
    const double pi = 3.141592653589793238462643383279502884;
    double c1 = pi / 10.0;
    double c2 = -pi / 5.0 + pi / 20.0 * (1.0 + 5.0 * gamma);
    double c3 = pi / 100.0 * (gamma - 1.0);
    double c4 = pi / 20.0 * (-7.0 + 15.0 * gamma);
    double c5 = pi / 100.0 * (3.0 * gamma - 2.0);
    double s = x + y + z - 2.0 * t;
    double cs = cos(pi * s), s2 = sin(2.0 * pi * s);
    q[0] = c1 * cs;
    q[1] = q[2] = q[3] = c2 * cs + c3 * s2;
    q[4] = c4 * cs + c5 * s2;
}


// ---- indexing helpers shared by the element kernels

// Periodic neighbour of element e across the face (dir, side = +-1); 32-bit
// arithmetic (the library limits meshes to fewer than 2^31 elements).
__device__ __forceinline__ int neighbour(int e, int dir, int side, int nx, int ny, int nz) {
    const unsigned ue = (unsigned)e;
    int ex = (int)(ue % (unsigned)nx);
    const unsigned r = ue / (unsigned)nx;
    int ey = (int)(r % (unsigned)ny);
    int ez = (int)(r / (unsigned)ny);
    if (dir == 0) ex = ex + side < 0 ? nx - 1 : (ex + side >= nx ? 0 : ex + side);
    else if (dir == 1) ey = ey + side < 0 ? ny - 1 : (ey + side >= ny ? 0 : ey + side);
    else ez = ez + side < 0 ? nz - 1 : (ez + side >= nz ? 0 : ez + side);
    return ex + nx * (ey + ny * ez);
}

// Node index of position 0 and the node stride along line l of direction dir
// (line index l = t1 + N t2 over the two tangential indices).
template <int N>
__device__ __forceinline__ void line_geometry(int dir, int l, int& base, int& stride) {
    const int t1 = l % N, t2 = l / N;
    if (dir == 0) { base = N * t1 + N * N * t2; stride = 1; }
    else if (dir == 1) { base = t1 + N * N * t2; stride = N; }
    else { base = t1 + N * t2; stride = N * N; }
}

// LDS index of a node in a padded node block. For even N one pad slot
// follows every xi-row, so that the lanes of a wave, which own consecutive
// lines and read the same position along them, spread over the LDS banks (a
// row stride of an even number of doubles would fold them onto a fraction of
// the banks); an odd N already spreads them and is not padded (measured: the
// pad cost 7% at p = 2 and 4). A padded block holds N^3 + N^2 doubles for
// every N.
template <int N>
__device__ __forceinline__ int pad_node(int node) {   // node >= 0
    if constexpr (N % 2 == 1) return node;
    else return node + (int)((unsigned)node / N);
}
// Length of a padded xi-row.
template <int N>
constexpr int padded_row() {
    return N % 2 == 1 ? N : N + 1;
}
// Padded-index step along a line of direction dir (xi, eta, zeta): a row's pad
// slot is passed at every eta or zeta step and at no xi step, so the padded
// index of node a of the line base + a stride is pad_node(base) + a times this.
template <int N>
__device__ __forceinline__ int padded_stride(int dir) {
    return dir == 0 ? 1 : (dir == 1 ? padded_row<N>() : padded_row<N>() * N);
}
template <int N>
constexpr int padded_block() {
    return N * N * N + N * N;
}

// Primitive variables of a node from the LDS block [6][PN3] (padded index):
// lds_prim for the adjoint (component 4 = p), lds_primr for the forward
// kernels (component 4 = p - pref).
template <int PN3>
__device__ __forceinline__ Prim lds_prim(const double* L, int pn) {
    Prim q;
    q.rho = L[pn];
    q.u = L[PN3 + pn];
    q.v = L[2 * PN3 + pn];
    q.w = L[3 * PN3 + pn];
    q.p = L[4 * PN3 + pn];
    q.beta = L[5 * PN3 + pn];
    return q;
}
template <int PN3>
__device__ __forceinline__ PrimR lds_primr(const double* L, int pn) {
    PrimR q;
    q.rho = L[pn];
    q.u = L[PN3 + pn];
    q.v = L[2 * PN3 + pn];
    q.w = L[3 * PN3 + pn];
    q.pd = L[4 * PN3 + pn];
    q.beta = L[5 * PN3 + pn];
    return q;
}

// Workgroups are dispatched to the 8 XCDs round-robin; remap the workgroup
// index so that each XCD processes one contiguous range of elements, which
// keeps most face-neighbour reads inside that XCD's L2.
__device__ __forceinline__ int xcd_remap(int g, int nb) {
    constexpr int NX = 8;
    const int q = nb / NX, r = nb % NX;
    const int x = g % NX, k = g / NX;
    return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

}  // namespace nsfr
