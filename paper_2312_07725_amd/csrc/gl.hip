// NSFR on Gauss-Legendre (uncollocated) quadrature, with overintegration:
// metric terms at the quadrature points, the entropy projection, and the
// fused right-hand-side / RK-stage kernel.
//
// Paper: Sec. 3.3 (Eq. NSFR with the hybridised operator of Eq. skew-symm
// qtilde oper: the volume-volume block Wq Dq - Dq^T Wq per direction and the
// surface-volume blocks phi_f^T W_f n_f; the two-point fluxes take the
// entropy-projected conservative variables u~ = u(chi v^), v^ = Pi v(chi u^)),
// Sec. 4 (Eq. weight-adj ESFR mass and Eq. Fr projection with the solution
// basis evaluated at the quadrature points), Sec. 5 (sum factorisation,
// Eq. sum-factorization: every dense 1D operator is applied one direction at a
// time), Sec. 7 (opening paragraph: Gauss-Legendre quadrature, solution
// coefficients on the LGL nodes, overintegration = extra quadrature points).
//
// The solution coefficients are the nodal values on the n^3 LGL nodes; the
// volume rule has q^3 Gauss points (q = n + overintegration) and each face q^2
// points. Per right-hand side two kernels run:
//   * gl_project_kernel: interpolate u to the volume points, form the entropy
//     variables, project them onto the solution basis (v^), and evaluate v^ at
//     the face points of every face (the neighbours read these);
//   * gl_stage_kernel: entropy-projected states at the volume and face points,
//     the hybrid Hadamard sum (one thread per line: the pairs along the line,
//     the pairs of each volume point with the two face points at the line's
//     ends, and the surface numerical flux at those ends), the transpose
//     interpolation of the volume and face residuals to the coefficients, the
//     weight-adjusted inverse, and the RK combination.
//
// The conservative DG scheme the paper compares against (Sec. 3.1 Eq. cons
// DG strong, Sec. 7.4: same rule, Roe's surface flux, an overintegrated
// variant) runs on the same operators and metric terms with two kernels of
// its own: gl_project_kernel<.., DG = true> writes the interpolated
// conservative states at the face points, and dg_stage_kernel evaluates the
// strong-form volume term chi^T W Dphi_k f^r_k, the surface term
// chi_f^T W_f [N . f* - n . phi_f f^r] and the same mass inverse and RK
// combination.
#include "nsfr_host.h"

namespace nsfr {

constexpr int GL_BLOCK = 256;   // projection kernels; NSFR stage (3 q^2 <= 243 line threads)
constexpr int DG_BLOCK = 512;   // DG stage (3 q^2 <= 432 line threads at q = 12)

// ---- sum-factorised 1D operator in LDS: dst = M applied along axis AX of
// src (dims S0 x S1 x S2, x fastest) for `ns` contiguous blocks; M is
// OUT x IN row-major, or its transpose stored IN x OUT when TR. One thread
// per (block, line): the line's IN inputs are read once into registers and
// its OUT outputs written once, so the index arithmetic is paid per line.
template <int S0, int S1, int S2, int AX, int OUT, bool TR, int SP = S0, int DP = (AX == 0 ? OUT : S0)>
__device__ __forceinline__ void lds_pass(const double* __restrict__ src, double* __restrict__ dst,
                                         const double* __restrict__ M, int ns) {
    // SP, DP: pitch of an x-row in src and dst (>= the row length; a padded
    // pitch spreads the lanes of the x- and y-passes over the LDS banks)
    constexpr int IN = AX == 0 ? S0 : (AX == 1 ? S1 : S2);
    constexpr int D1 = AX == 1 ? OUT : S1, D2 = AX == 2 ? OUT : S2;
    constexpr int SRC = SP * S1 * S2, NL = S0 * S1 * S2 / IN, DST = DP * D1 * D2;
    constexpr int SST = AX == 0 ? 1 : (AX == 1 ? SP : SP * S1);   // stride along the axis in src
    constexpr int DSS = AX == 0 ? 1 : (AX == 1 ? DP : DP * D1);   // and in dst
    for (int it = threadIdx.x; it < ns * NL; it += blockDim.x) {
        const int b = it / NL, ln = it - b * NL;
        int sb, db;
        if (AX == 0) {          // ln = i1 + S1 i2
            sb = ln * SP;
            db = ln * DP;
        } else if (AX == 1) {   // ln = i0 + S0 i2
            const int i0 = ln % S0, i2 = ln / S0;
            sb = i0 + SP * S1 * i2;
            db = i0 + DP * OUT * i2;
        } else {                // ln = i0 + S0 i1
            const int i0 = ln % S0, i1 = ln / S0;
            sb = i0 + SP * i1;
            db = i0 + DP * i1;
        }
        const double* x = src + b * SRC + sb;
        double v[IN];
#pragma unroll
        for (int m = 0; m < IN; ++m) v[m] = x[m * SST];
        double* y = dst + b * DST + db;
#pragma unroll
        for (int o = 0; o < OUT; ++o) {
            double acc = 0.0;
#pragma unroll
            for (int m = 0; m < IN; ++m) acc = __builtin_fma(TR ? M[m * OUT + o] : M[o * IN + m], v[m], acc);
            y[o * DSS] = acc;
        }
    }
}

// x-row pitch for rows of n doubles: a length that is a multiple of 4 puts
// the 16 lanes of an x-pass, which step through consecutive rows, on a
// quarter of the LDS bank pairs or fewer, so such rows get one pad slot;
// other lengths at most halve them and are left unpadded (the pad's index
// arithmetic then costs more than it saves).
__host__ __device__ constexpr int bank_pitch(int n) { return n % 4 == 0 ? n + 1 : n; }

// LDS doubles of the DG stage kernel for epb elements with volume row pitch
// xq, and the pitch it uses: padded unless that would not fit one element in
// gfx950's 160 KiB of LDS per workgroup (p = 5 with 12 points).
__host__ __device__ constexpr int dg_stage_doubles(int n, int q, int xq, int epb) {
    return 2 * q * n + q * q + 3 * q + epb * (5 * xq * q * q + 5 * xq * q * n + 30 * q * q + 30 * q * n);
}
__host__ __device__ constexpr int dg_row_pitch(int n, int q) {
    return dg_stage_doubles(n, q, bank_pitch(q), 1) * 8 <= 160 * 1024 ? bank_pitch(q) : q;
}

// Face slabs of a coefficient array X [nb][5][n^3] (nb element blocks): copy
// the six end slabs into SL [nb][6][5][n^2] (tangential indices in increasing
// direction order, first fastest).
template <int N, int XP = N, int SLP = N>
__device__ __forceinline__ void gather_slabs(const double* __restrict__ X, double* __restrict__ SL, int nb) {
    // XP: x-row pitch of X's blocks; SLP: pitch of a slab's first tangential row
    constexpr int N2 = N * N;
    for (int it = threadIdx.x; it < nb * 30 * N2; it += blockDim.x) {
        const int el = it / (30 * N2), r = it - el * 30 * N2;
        const int f = r / (5 * N2), r2 = r - f * 5 * N2;
        const int s = r2 / N2, t = r2 - s * N2;
        const int d = f / 2, end = (f % 2) ? N - 1 : 0;
        const int u1 = t % N, u2 = t / N;
        const int a = d == 0 ? end : u1, b = d == 0 ? u1 : (d == 1 ? end : u2), c = d == 2 ? end : u2;
        SL[(el * 30 + f * 5 + s) * (SLP * N) + u1 + SLP * u2] = X[(el * 5 + s) * (XP * N2) + a + XP * (b + N * c)];
    }
}

// Add the six face slabs FS [nb][6][5][n^2] onto the coefficient array X
// [nb][5][n^3] (node-parallel: each node adds the slabs of the faces it lies on).
template <int N, int XP = N, int SLP = N>
__device__ __forceinline__ void scatter_add_slabs(double* __restrict__ X, const double* __restrict__ FS, int nb) {
    // XP: x-row pitch of X's blocks; SLP: pitch of a slab's first tangential row
    constexpr int N2 = N * N, N3 = N2 * N, SB = SLP * N;
    for (int it = threadIdx.x; it < nb * 5 * N3; it += blockDim.x) {
        const int el = it / (5 * N3), r = it - el * 5 * N3;
        const int s = r / N3, nd = r - s * N3;
        const int a = nd % N, b = (nd / N) % N, c = nd / N2;
        const double* fs = FS + (el * 30 + s) * SB;
        double* x = X + (el * 5 + s) * (XP * N2) + a + XP * (b + N * c);
        double acc = *x;
        if (a == 0) acc += fs[0 * 5 * SB + b + SLP * c];
        if (a == N - 1) acc += fs[1 * 5 * SB + b + SLP * c];
        if (b == 0) acc += fs[2 * 5 * SB + a + SLP * c];
        if (b == N - 1) acc += fs[3 * 5 * SB + a + SLP * c];
        if (c == 0) acc += fs[4 * 5 * SB + a + SLP * b];
        if (c == N - 1) acc += fs[5 * 5 * SB + a + SLP * b];
        *x = acc;
    }
}

// entropy variables v(u) of Sec. 2.1 (U = -rho s / (gamma - 1))
__device__ __forceinline__ void entropy_vars(const double u[5], double gm1, double gamma, double v[5]) {
    const double r = u[0], ir = 1.0 / r;
    const double a = u[1] * ir, b = u[2] * ir, c = u[3] * ir;
    const double q2 = a * a + b * b + c * c;
    const double p = gm1 * (u[4] - 0.5 * r * q2);
    const double beta = 0.5 * r / p;
    const double s = log(p) - gamma * log(r);
    v[0] = (gamma - s) / gm1 - beta * q2;
    v[1] = 2.0 * beta * a;
    v[2] = 2.0 * beta * b;
    v[3] = 2.0 * beta * c;
    v[4] = -2.0 * beta;
}

// primitives of u(v) (the inverse entropy map): beta = -v5 / 2,
// u = v_m / (2 beta), s = gamma - (gamma - 1)(v1 + beta |u|^2),
// ln p = (s + gamma ln(2 beta)) / (1 - gamma), rho = 2 beta p
__device__ __forceinline__ PrimR prims_from_entropy(const double v[5], double gm1, double gamma, double pref) {
    PrimR q;
    const double beta = -0.5 * v[4];
    const double ib = 0.5 / beta;
    q.u = v[1] * ib;
    q.v = v[2] * ib;
    q.w = v[3] * ib;
    const double s = gamma - gm1 * (v[0] + beta * (q.u * q.u + q.v * q.v + q.w * q.w));
    const double p = exp((s + gamma * log(2.0 * beta)) / (-gm1));
    q.rho = 2.0 * beta * p;
    q.pd = p - pref;
    q.beta = beta;
    return q;
}

// ---- metric terms at the quadrature points (once per context). The
// cofactors are the conservative-curl cofactors of the LGL grid (degree p)
// evaluated as polynomials, J the determinant of the grid polynomial's
// derivative; one thread per (element, volume point) and per (element,
// face point). Cline is the line-major cofactor array of the collocated
// geometry: column d, component m of node (a, b, c) at
// [((d * 3 + m) * E + e) * n^3 + pos_d * n^2 + line_d] with pos = (a, b, c)
// and line = (b + n c, a + n c, a + n b).
template <int N>
__device__ __forceinline__ int64_t cline_index(int d, int m, int64_t E, int64_t e, int a, int b, int c) {
    constexpr int N2 = N * N;
    const int pos = d == 0 ? a : (d == 1 ? b : c);
    const int lin = d == 0 ? b + N * c : (d == 1 ? a + N * c : a + N * b);
    return ((int64_t)(d * 3 + m) * E + e) * (N2 * N) + pos * N2 + lin;
}

template <int N, int Q>
__global__ void gl_geometry_kernel(const GLOps* __restrict__ ops, int64_t E, const double* __restrict__ X,
                                   const double* __restrict__ Cline, double* Cq, double* invWJ, double* Xq) {
    constexpr int N3 = N * N * N, Q2 = Q * Q, Q3 = Q2 * Q;
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gid >= E * Q3) return;
    const int64_t e = gid / Q3;
    const int t = (int)(gid - e * Q3);
    const int i = t % Q, j = (t / Q) % Q, k = t / Q2;
    const double* chi = ops->chi;
    const double* chid = ops->chid;
    double x[3] = {0.0, 0.0, 0.0}, G[3][3] = {}, Cv[3][3] = {};
    for (int c = 0; c < N; ++c)
        for (int b = 0; b < N; ++b)
            for (int a = 0; a < N; ++a) {
                const int nd = a + N * (b + N * c);
                const double wi = chi[i * N + a], wj = chi[j * N + b], wk = chi[k * N + c];
                const double w = wi * wj * wk;
                const double w0 = chid[i * N + a] * wj * wk, w1 = wi * chid[j * N + b] * wk,
                             w2 = wi * wj * chid[k * N + c];
                for (int m = 0; m < 3; ++m) {
                    const double xv = X[(m * E + e) * N3 + nd];
                    x[m] += w * xv;
                    G[m][0] += w0 * xv;
                    G[m][1] += w1 * xv;
                    G[m][2] += w2 * xv;
                    for (int d = 0; d < 3; ++d) Cv[m][d] += w * Cline[cline_index<N>(d, m, E, e, a, b, c)];
                }
            }
    const double J = G[0][0] * (G[1][1] * G[2][2] - G[1][2] * G[2][1]) -
                     G[0][1] * (G[1][0] * G[2][2] - G[1][2] * G[2][0]) +
                     G[0][2] * (G[1][0] * G[2][1] - G[1][1] * G[2][0]);
    invWJ[e * Q3 + t] = 1.0 / (ops->wq[i] * ops->wq[j] * ops->wq[k] * J);
    for (int m = 0; m < 3; ++m) Xq[(m * E + e) * Q3 + t] = x[m];
    const int pos[3] = {i, j, k};
    const int lin[3] = {j + Q * k, i + Q * k, i + Q * j};
    for (int d = 0; d < 3; ++d)
        for (int m = 0; m < 3; ++m) Cq[((int64_t)(d * 3 + m) * E + e) * Q3 + pos[d] * Q2 + lin[d]] = Cv[m][d];
}

template <int N, int Q>
__global__ void gl_face_geometry_kernel(const GLOps* __restrict__ ops, int64_t E, const double* __restrict__ Cline,
                                        double* Cf) {
    constexpr int Q2 = Q * Q;
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gid >= E * 6 * Q2) return;
    const int64_t e = gid / (6 * Q2);
    const int r = (int)(gid - e * 6 * Q2);
    const int f = r / Q2, t = r - f * Q2;
    const int d = f / 2, side = f % 2;
    const int t1 = t % Q, t2 = t / Q;
    const int end = side ? N - 1 : 0;
    const double* chi = ops->chi;
    for (int m = 0; m < 3; ++m) {
        double acc = 0.0;
        for (int c = 0; c < N; ++c)
            for (int b = 0; b < N; ++b) {
                // tangential LGL indices (b, c) in increasing direction order
                const int64_t ix = d == 0 ? cline_index<N>(d, m, E, e, end, b, c)
                                          : (d == 1 ? cline_index<N>(d, m, E, e, b, end, c)
                                                    : cline_index<N>(d, m, E, e, b, c, end));
                acc += chi[t1 * N + b] * chi[t2 * N + c] * Cline[ix];
            }
        Cf[((int64_t)(f * 3 + m) * E + e) * Q2 + t] = acc;
    }
}

// ---- entropy projection: v^ = Pi v(chi u^) and v^ at every face point
template <int N, int Q, bool DG>
__global__ __launch_bounds__(GL_BLOCK) void gl_project_kernel(const GLOps* __restrict__ ops, int64_t E,
                                                              const double* __restrict__ U, double gamma,
                                                              double* vhat, double* ft) {
    constexpr int N2 = N * N, N3 = N2 * N, Q2 = Q * Q, Q3 = Q2 * Q;
    // x-row pitches of the LDS arrays (padded for the NSFR projection, so that
    // the lanes of the x- and y-passes fall on different LDS banks)
    constexpr int XN = DG ? N : bank_pitch(N), XQ = DG ? Q : bank_pitch(Q);
    constexpr int BN = XN * N2, BQ = XQ * Q2;   // block sizes of an n^3 and a q^3 array
    auto pn = [](int nd) {   // node -> padded index (the identity without padding)
        if constexpr (XN == N) return nd;
        else return nd % N + XN * (nd / N);
    };
    auto pq = [](int t) {    // volume or face point (rows of q) -> padded index
        if constexpr (XQ == Q) return t;
        else return t % Q + XQ * (t / Q);
    };
    extern __shared__ double lds[];
    constexpr int AS = DG ? 5 * N3 : 5 * BQ, BS = DG ? 0 : 5 * BQ;
    double* mchi = lds;              // Q x N
    double* mpi = mchi + Q * N;      // N x Q
    double* A = mpi + N * Q;         // AS
    double* B = A + AS;              // BS
    double* SL = B + BS;             // [6][5][N^2] end slabs (row pitch XN)
    double* T = SL + 30 * XN * N;    // [6][5][Q N] (row pitch XQ)
    double* SF = T + 30 * XQ * N;    // [6][5][Q^2] (row pitch XQ)
    const int tid = threadIdx.x;
    const int64_t e = blockIdx.x;
    const int64_t SE = E * N3;
    const double gm1 = gamma - 1.0;
    for (int i = tid; i < Q * N; i += blockDim.x) {
        mchi[i] = ops->chi[i];
        mpi[i] = ops->pi[i];
    }
    for (int i = tid; i < 5 * N3; i += blockDim.x) {
        const int s = i / N3, nd = i - s * N3;
        A[s * BN + pn(nd)] = U[s * SE + e * N3 + nd];
    }
    __syncthreads();
    if constexpr (!DG) {
        lds_pass<N, N, N, 0, Q, false, XN, XQ>(A, B, mchi, 5);
        __syncthreads();
        lds_pass<Q, N, N, 1, Q, false, XQ, XQ>(B, A, mchi, 5);
        __syncthreads();
        lds_pass<Q, Q, N, 2, Q, false, XQ, XQ>(A, B, mchi, 5);
        __syncthreads();
        for (int t = tid; t < Q3; t += blockDim.x) {
            const int pt = pq(t);
            double u[5], v[5];
#pragma unroll
            for (int s = 0; s < 5; ++s) u[s] = B[s * BQ + pt];
            entropy_vars(u, gm1, gamma, v);
#pragma unroll
            for (int s = 0; s < 5; ++s) B[s * BQ + pt] = v[s];
        }
        __syncthreads();
        lds_pass<Q, Q, Q, 2, N, false, XQ, XQ>(B, A, mpi, 5);
        __syncthreads();
        lds_pass<Q, Q, N, 1, N, false, XQ, XQ>(A, B, mpi, 5);
        __syncthreads();
        lds_pass<Q, N, N, 0, N, false, XQ, XN>(B, A, mpi, 5);
        __syncthreads();
        for (int i = tid; i < 5 * N3; i += blockDim.x) {
            const int s = i / N3, nd = i - s * N3;
            vhat[s * SE + e * N3 + nd] = A[s * BN + pn(nd)];
        }
    }
    // v^ (DG: u) at the face points: the end slab of the coefficients,
    // interpolated along the first and then the second tangential direction
    gather_slabs<N, XN, XN>(A, SL, 1);
    __syncthreads();
    lds_pass<N, N, 1, 0, Q, false, XN, XQ>(SL, T, mchi, 30);
    __syncthreads();
    lds_pass<Q, N, 1, 1, Q, false, XQ, XQ>(T, SF, mchi, 30);
    __syncthreads();
    for (int it = tid; it < 30 * Q2; it += blockDim.x) {
        const int fs = it / Q2, t = it - fs * Q2;
        ft[((int64_t)fs * E + e) * Q2 + t] = SF[fs * (XQ * Q) + pq(t)];
    }
}

// Minimum waves per SIMD the register allocation of the NSFR stage must
// allow: at q = 5 a cap of 256 registers (2 waves, 128 B of spill) is faster
// than the uncapped allocation (1 wave); from q = 6 the cap spills 0.25-1.7 KB
// per lane and is slower, and up to q = 4 the kernel fits 2 waves without it.
__host__ __device__ constexpr int gl_stage_min_waves(int q) { return q == 5 ? 2 : 1; }

// ---- the stage: one element per workgroup
template <int N, int Q, int VARIANT>
__global__ __launch_bounds__(GL_BLOCK) __attribute__((amdgpu_waves_per_eu(gl_stage_min_waves(Q))))
void gl_stage_kernel(StageArgs A, GLArgs G) {
    constexpr int N2 = N * N, N3 = N2 * N, Q2 = Q * Q, Q3 = Q2 * Q;
    // x-row pitches of the LDS arrays, so that lanes stepping through rows of
    // n or q values fall on different LDS banks; block sizes of an n^3 and a
    // q^3 array
    constexpr int XN = bank_pitch(N), XQ = bank_pitch(Q), BN = XN * N2, BQ = XQ * Q2;
    auto pn = [](int nd) {   // node -> padded index (the identity without padding)
        if constexpr (XN == N) return nd;
        else return nd % N + XN * (nd / N);
    };
    auto pq = [](int t) {    // volume point -> padded index
        if constexpr (XQ == Q) return t;
        else return t % Q + XQ * (t / Q);
    };
    extern __shared__ double lds[];
    double* mchi = lds;               // Q x N
    double* mpit = mchi + Q * N;      // N x Q
    double* msq = mpit + N * Q;       // Q x Q (halved skew operator)
    double* mtl = msq + Q2;           // Q
    double* mtr = mtl + Q;            // Q
    double* mw = mtr + Q;             // Q
    double* BA = mw + Q;              // 6 BQ: pass buffer, then the volume primitives
    double* BB = BA + 6 * BQ;         // 5 BQ: pass buffer, then the volume residual
    double* FP = BB + 5 * BQ;         // [6 faces][6][Q^2]: primitives at the own face points
    double* RF = FP + 36 * Q2;        // [6 faces][5][Q^2]: face-point residuals (unpadded: the
                                      // padded face arrays would cost the eighth workgroup per CU)
    double* TF = RF + 30 * Q2;        // [6 faces][5][Q N]: their first tangential contraction
    const int tid = threadIdx.x, nth = blockDim.x;
    const int64_t e = blockIdx.x;
    const int64_t E = A.geo.E;
    const int64_t SE = E * N3;
    const double gamma = A.gamma, gm1 = gamma - 1.0, c1 = A.c1;
    const double pref = reference_pressure(A.Uin, SE, gm1);
    const GLOps* ops = G.ops;
    for (int i = tid; i < Q * N; i += nth) {
        mchi[i] = ops->chi[i];
        mpit[i] = ops->pit[i];
    }
    for (int i = tid; i < Q2; i += nth) msq[i] = ops->sqh[i];
    for (int i = tid; i < Q; i += nth) {
        mtl[i] = ops->tl[i];
        mtr[i] = ops->tr[i];
        mw[i] = ops->wq[i];
    }
    // 1. v^ of this element -> volume points; own face points from the face traces
    for (int i = tid; i < 5 * N3; i += nth) {
        const int s = i / N3, nd = i - s * N3;
        BA[s * BN + pn(nd)] = G.vhat[s * SE + e * N3 + nd];
    }
    for (int it = tid; it < 6 * Q2; it += nth) {
        const int f = it / Q2, t = it - f * Q2;
        double v[5];
#pragma unroll
        for (int s = 0; s < 5; ++s) v[s] = G.ft[((int64_t)(f * 5 + s) * E + e) * Q2 + t];
        const PrimR q = prims_from_entropy(v, gm1, gamma, pref);
        double* L = FP + f * 6 * Q2 + t;
        L[0] = q.rho;
        L[Q2] = q.u;
        L[2 * Q2] = q.v;
        L[3 * Q2] = q.w;
        L[4 * Q2] = q.pd;
        L[5 * Q2] = q.beta;
    }
    __syncthreads();
    lds_pass<N, N, N, 0, Q, false, XN, XQ>(BA, BB, mchi, 5);
    __syncthreads();
    lds_pass<Q, N, N, 1, Q, false, XQ, XQ>(BB, BA, mchi, 5);
    __syncthreads();
    lds_pass<Q, Q, N, 2, Q, false, XQ, XQ>(BA, BB, mchi, 5);
    __syncthreads();
    for (int t = tid; t < Q3; t += nth) {
        const int pt = pq(t);
        double v[5];
#pragma unroll
        for (int s = 0; s < 5; ++s) v[s] = BB[s * BQ + pt];
        const PrimR q = prims_from_entropy(v, gm1, gamma, pref);
        BA[pt] = q.rho;
        BA[BQ + pt] = q.u;
        BA[2 * BQ + pt] = q.v;
        BA[3 * BQ + pt] = q.w;
        BA[4 * BQ + pt] = q.pd;
        BA[5 * BQ + pt] = q.beta;
    }
    __syncthreads();

    // 2. one thread per line, in two passes whose register footprints do not
    //    add up: (a) the volume pairs along the line, accumulated into BB in a
    //    fixed direction order; (b) the pairs of every volume point with the two
    //    end face points (weights t_L, t_R) and the surface numerical flux at
    //    both ends, added into BB in the same order, face residuals into RF
    //    (each face point belongs to one line)
    const int lt = tid;
    const bool active = lt < 3 * Q2;
    const int dir = active ? lt / Q2 : 0;
    const int l = active ? lt - dir * Q2 : 0;
    const int t1 = l % Q, t2 = l / Q;
    // the line's first point and point stride in the padded volume arrays
    const int base = dir == 0 ? XQ * (t1 + Q * t2) : (dir == 1 ? t1 + XQ * Q * t2 : t1 + XQ * t2);
    const int stride = dir == 0 ? 1 : (dir == 1 ? XQ : XQ * Q);
    const double wperp = mw[t1] * mw[t2];
    const double* Cl = G.geo.Cq + (int64_t)(3 * dir) * E * Q3 + e * Q3 + l;   // [comp][pos Q^2]
    const int64_t CS = E * Q3;
    const int64_t FS = E * Q2;
    auto volp = [&](int a) {
        const int t = base + a * stride;
        return PrimR{BA[t], BA[BQ + t], BA[2 * BQ + t], BA[3 * BQ + t], BA[4 * BQ + t], BA[5 * BQ + t]};
    };
    // the line's volume residual into BB: phase ph stores (first pass) or adds
    auto accumulate = [&](double (&Rv)[5][Q], bool first) {
        for (int ph = 0; ph < 3; ++ph) {
            if (active && dir == ph) {
#pragma unroll
                for (int s = 0; s < 5; ++s)
#pragma unroll
                    for (int a = 0; a < Q; ++a) {
                        const double v = Rv[s][a] * wperp;
                        double* x = BB + s * BQ + base + a * stride;
                        if (first && ph == 0) *x = v;
                        else *x += v;
                    }
            }
            __syncthreads();
        }
    };
    {   // (a) volume-volume pairs (S/2 folded into msq, direction C(a) + C(b))
        double Rv[5][Q];
#pragma unroll
        for (int s = 0; s < 5; ++s)
#pragma unroll
            for (int a = 0; a < Q; ++a) Rv[s][a] = 0.0;
        if (active) {
#pragma unroll
            for (int a = 0; a < Q - 1; ++a) {
                const PrimR qa = volp(a);
                const double cax = Cl[a * Q2], cay = Cl[CS + a * Q2], caz = Cl[2 * CS + a * Q2];
#pragma unroll
                for (int b = a + 1; b < Q; ++b) {
                    const PrimR qb = volp(b);
                    double F[5];
                    ec_flux<VARIANT>(qa, qb, cax + Cl[b * Q2], cay + Cl[CS + b * Q2], caz + Cl[2 * CS + b * Q2], c1,
                                     pref, F);
                    const double sab = msq[a * Q + b];
#pragma unroll
                    for (int s = 0; s < 5; ++s) {
                        Rv[s][a] = __builtin_fma(sab, F[s], Rv[s][a]);
                        Rv[s][b] = __builtin_fma(-sab, F[s], Rv[s][b]);
                    }
                }
            }
        }
        accumulate(Rv, true);
    }
    {   // (b) the two ends of the line
        double Rv[5][Q];
#pragma unroll
        for (int s = 0; s < 5; ++s)
#pragma unroll
            for (int a = 0; a < Q; ++a) Rv[s][a] = 0.0;
        if (active) {
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const int f = 2 * dir + side;
                const double sg = side ? 1.0 : -1.0;
                const double* tw = side ? mtr : mtl;
                const double* Fp = FP + f * 6 * Q2 + l;
                const PrimR qf = PrimR{Fp[0], Fp[Q2], Fp[2 * Q2], Fp[3 * Q2], Fp[4 * Q2], Fp[5 * Q2]};
                const double* Cfo = G.geo.Cf + ((int64_t)(f * 3) * E + e) * Q2 + l;
                const double cfx = Cfo[0], cfy = Cfo[FS], cfz = Cfo[2 * FS];
                double rf[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
                // volume-face pairs: +/- t[a] W_perp F(u~_a, u~_f; (C_a + C_f)/2) on the
                // volume point, the opposite on the face point
#pragma unroll
                for (int a = 0; a < Q; ++a) {
                    const PrimR qa = volp(a);
                    double F[5];
                    ec_flux<VARIANT>(qa, qf, Cl[a * Q2] + cfx, Cl[CS + a * Q2] + cfy, Cl[2 * CS + a * Q2] + cfz, c1,
                                     pref, F);
                    const double wgt = 0.5 * sg * tw[a];
#pragma unroll
                    for (int s = 0; s < 5; ++s) {
                        Rv[s][a] = __builtin_fma(wgt, F[s], Rv[s][a]);
                        rf[s] = __builtin_fma(-wgt, F[s], rf[s]);
                    }
                }
                // surface numerical flux with the neighbour's face point
                const int en = A.geo.nbr[(int64_t)f * E + e];
                const int fn = 2 * dir + (1 - side);
                double vn[5];
#pragma unroll
                for (int s = 0; s < 5; ++s) vn[s] = G.ft[((int64_t)(fn * 5 + s) * E + en) * Q2 + l];
                const PrimR qn = prims_from_entropy(vn, gm1, gamma, pref);
                const double* Cfn = G.geo.Cf + ((int64_t)(fn * 3) * E + en) * Q2 + l;
                const double nx = 0.5 * sg * (cfx + Cfn[0]), ny = 0.5 * sg * (cfy + Cfn[FS]),
                             nz = 0.5 * sg * (cfz + Cfn[2 * FS]);
                double F[5];
                ec_flux<VARIANT>(qf, qn, nx, ny, nz, c1, pref, F);
                if (A.diss == 1) {
                    auto cons = [&](const PrimR& q, double out[5]) {
                        out[0] = q.rho;
                        out[1] = q.rho * q.u;
                        out[2] = q.rho * q.v;
                        out[3] = q.rho * q.w;
                        out[4] = (pref + q.pd) / gm1 + 0.5 * q.rho * (q.u * q.u + q.v * q.v + q.w * q.w);
                    };
                    double Uo[5], Un[5];
                    cons(qf, Uo);
                    cons(qn, Un);
                    llf_add(qf, qn, Uo, Un, nx, ny, nz, gamma, pref, F);
                } else if (A.diss == 2) {
                    roe_add(qf, qn, nx, ny, nz, gamma, pref, F);
                }
#pragma unroll
                for (int s = 0; s < 5; ++s) RF[(f * 5 + s) * Q2 + l] = (rf[s] + F[s]) * wperp;
            }
        }
        accumulate(Rv, false);
    }
    // manufactured source at the volume points: R -= W J q
    const int mode = A.mode;
    double dt = 0.0, cstage = 0.0;
    if (mode >= MODE_RK1) {
        dt = *A.dt;
        cstage = (mode == MODE_RK1) ? 0.0 : (mode == MODE_RK4 ? 1.0 : 0.5);
    }
    if (A.source) {
        const double t = (A.tdev ? *A.tdev : A.t) + cstage * dt;
        const int64_t EQ = E * Q3;
        for (int p = tid; p < Q3; p += nth) {
            double qs[5];
            const double* X = G.geo.Xq + e * Q3 + p;
            mms_source(X[0], X[EQ], X[2 * EQ], t, gamma, qs);
            const double wj = 1.0 / G.geo.invWJ[e * Q3 + p];
#pragma unroll
            for (int s = 0; s < 5; ++s) BB[s * BQ + pq(p)] -= wj * qs[s];
        }
    }
    __syncthreads();

    // 3. to the coefficients: chi^T along z, y, x of the volume residual, then
    //    the face residuals through the tangential chi^T onto the end slabs
    //    (the face residuals go through the tangential chi^T, RF -> TF -> RF as
    //    [6][5][N^2], alongside the first two volume passes)
    lds_pass<Q, Q, Q, 2, N, true, XQ, XQ>(BB, BA, mchi, 5);
    lds_pass<Q, Q, 1, 0, N, true>(RF, TF, mchi, 30);
    __syncthreads();
    lds_pass<Q, Q, N, 1, N, true, XQ, XQ>(BA, BB, mchi, 5);
    lds_pass<N, Q, 1, 1, N, true>(TF, RF, mchi, 30);
    __syncthreads();
    lds_pass<Q, N, N, 0, N, true, XQ, XN>(BB, BA, mchi, 5);
    __syncthreads();
    scatter_add_slabs<N, XN, N>(BA, RF, 1);
    __syncthreads();
    if (mode == MODE_RESIDUAL) {
        for (int it = tid; it < 5 * N3; it += nth) {
            const int s = it / N3, nd = it - s * N3;
            A.out[s * SE + e * N3 + nd] = BA[s * BN + pn(nd)];
        }
        return;
    }
    // 4. weight-adjusted inverse: Pi~^T (coefficients -> points), (W J)^-1, Pi~
    lds_pass<N, N, N, 0, Q, true, XN, XQ>(BA, BB, mpit, 5);
    __syncthreads();
    lds_pass<Q, N, N, 1, Q, true, XQ, XQ>(BB, BA, mpit, 5);
    __syncthreads();
    lds_pass<Q, Q, N, 2, Q, true, XQ, XQ>(BA, BB, mpit, 5);
    __syncthreads();
    for (int it = tid; it < 5 * Q3; it += nth) {
        if constexpr (XQ == Q) {
            BB[it] *= G.geo.invWJ[e * Q3 + it % Q3];
        } else {
            const int s = it / Q3, t = it - s * Q3;
            BB[s * BQ + pq(t)] *= G.geo.invWJ[e * Q3 + t];
        }
    }
    __syncthreads();
    lds_pass<Q, Q, Q, 2, N, false, XQ, XQ>(BB, BA, mpit, 5);
    __syncthreads();
    lds_pass<Q, Q, N, 1, N, false, XQ, XQ>(BA, BB, mpit, 5);
    __syncthreads();
    lds_pass<Q, N, N, 0, N, false, XQ, XN>(BB, BA, mpit, 5);
    __syncthreads();
    // 5. RK combination
    for (int it = tid; it < 5 * N3; it += nth) {
        const int s = it / N3, nd = it - s * N3;
        const int64_t gi = s * SE + e * N3 + nd;
        const double k = -BA[s * BN + pn(nd)];
        switch (mode) {
            case MODE_RHS: A.out[gi] = k; break;
            case MODE_RK1: {
                const double u = A.Uin[gi];
                A.acc[gi] = __builtin_fma(dt / 6.0, k, u);
                A.out[gi] = __builtin_fma(0.5 * dt, k, u);
            } break;
            case MODE_RK2:
                A.acc[gi] = __builtin_fma(dt / 3.0, k, A.acc[gi]);
                A.out[gi] = __builtin_fma(0.5 * dt, k, A.Un[gi]);
                break;
            case MODE_RK3:
                A.acc[gi] = __builtin_fma(dt / 3.0, k, A.acc[gi]);
                A.out[gi] = __builtin_fma(dt, k, A.Un[gi]);
                break;
            default: A.out[gi] = __builtin_fma(dt / 6.0, k, A.acc[gi]); break;
        }
    }
}

// ---- conservative DG (Sec. 3.1 Eq. cons DG strong)

// Roe's flux N . f* = (f(A) + f(B)) . N / 2 - |N| |A^| (B - A) / 2 at Roe's
// average (sqrt(rho)-weighted velocity and total enthalpy, rho^ =
// sqrt(rho_A rho_B)); |A^| dU as the sum over the two acoustic waves, the
// entropy wave and the shear waves (Roe 1981; Sec. 7.4 uses it for DG). The
// momentum flux carries p - p_ref (the constant p_ref N terms cancel in the
// residual by the discrete GCL, as in the NSFR kernels).
__device__ __forceinline__ void roe_flux_dev(const double A[5], const double B[5], double nx, double ny, double nz,
                                             double gamma, double pref, double F[5]) {
    const double gm1 = gamma - 1.0;
    const double ra = A[0], rb = B[0];
    const double ira = 1.0 / ra, irb = 1.0 / rb;
    const double ua = A[1] * ira, va = A[2] * ira, wa = A[3] * ira;
    const double ub = B[1] * irb, vb = B[2] * irb, wb = B[3] * irb;
    const double pa = gm1 * (A[4] - 0.5 * (A[1] * ua + A[2] * va + A[3] * wa));
    const double pb = gm1 * (B[4] - 0.5 * (B[1] * ub + B[2] * vb + B[3] * wb));
    const double una = ua * nx + va * ny + wa * nz, unb = ub * nx + vb * ny + wb * nz;
    // central part (momentum with p - p_ref)
    const double pda = pa - pref, pdb = pb - pref;
    F[0] = 0.5 * (A[0] * una + B[0] * unb);
    F[1] = 0.5 * (A[1] * una + B[1] * unb + (pda + pdb) * nx);
    F[2] = 0.5 * (A[2] * una + B[2] * unb + (pda + pdb) * ny);
    F[3] = 0.5 * (A[3] * una + B[3] * unb + (pda + pdb) * nz);
    F[4] = 0.5 * ((A[4] + pa) * una + (B[4] + pb) * unb);
    // Roe average
    const double nn = sqrt(nx * nx + ny * ny + nz * nz);
    const double inn = 1.0 / nn;
    const double ex = nx * inn, ey = ny * inn, ez = nz * inn;
    const double sa = sqrt(ra), sb = sqrt(rb);
    const double iw = 1.0 / (sa + sb);
    const double u = (sa * ua + sb * ub) * iw, v = (sa * va + sb * vb) * iw, w = (sa * wa + sb * wb) * iw;
    const double H = (sa * (A[4] + pa) * ira + sb * (B[4] + pb) * irb) * iw;
    const double q2 = u * u + v * v + w * w;
    const double c2 = gm1 * (H - 0.5 * q2);
    const double c = sqrt(c2), ic2 = 1.0 / c2;
    const double rho = sa * sb;
    const double un = u * ex + v * ey + w * ez;
    const double du = ub - ua, dv = vb - va, dw = wb - wa;
    const double dun = du * ex + dv * ey + dw * ez;
    const double dp = pdb - pda;
    double D[5];
    {   // entropy wave
        const double a = (rb - ra - dp * ic2) * fabs(un);
        D[0] = a;
        D[1] = a * u;
        D[2] = a * v;
        D[3] = a * w;
        D[4] = a * 0.5 * q2;
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {   // acoustic waves u.n -+ c
        const double sg = k ? 1.0 : -1.0;
        const double a = (dp + sg * rho * c * dun) * (0.5 * ic2) * fabs(un + sg * c);
        D[0] += a;
        D[1] += a * (u + sg * c * ex);
        D[2] += a * (v + sg * c * ey);
        D[3] += a * (w + sg * c * ez);
        D[4] += a * (H + sg * c * un);
    }
    {   // shear waves
        const double b = rho * fabs(un);
        const double sx = du - dun * ex, sy = dv - dun * ey, sz = dw - dun * ez;
        D[1] += b * sx;
        D[2] += b * sy;
        D[3] += b * sz;
        D[4] += b * (u * du + v * dv + w * dw - un * dun);
    }
    const double k = 0.5 * nn;
#pragma unroll
    for (int s = 0; s < 5; ++s) F[s] -= k * D[s];
}

// epb elements per workgroup (A.epb), one thread per (element, line). LDS:
// the 1D operators, VA [epb][5][q^3] (states at the volume points, then the
// volume residual, then ping-pong), VB [epb][5][q^2 n] (ping-pong), RF
// [epb][6][5][q^2] (face-point residuals). Every sum-factorised pass treats the
// epb x 5 state blocks of a buffer as one contiguous array.
template <int N, int Q>
__global__ __launch_bounds__(DG_BLOCK) void dg_stage_kernel(StageArgs A, GLArgs G) {
    constexpr int N2 = N * N, N3 = N2 * N, Q2 = Q * Q, Q3 = Q2 * Q, L3 = 3 * Q2;
    // x-row pitches of the volume arrays (bank spread, as in the NSFR kernels)
    // and the block sizes of an n^3 and a q^3 array
    constexpr int XQ = dg_row_pitch(N, Q), XN = XQ == Q ? N : bank_pitch(N), BN = XN * N2, BQ = XQ * Q2;
    auto pn = [](int nd) {   // node -> padded index (the identity without padding)
        if constexpr (XN == N) return nd;
        else return nd % N + XN * (nd / N);
    };
    auto pq = [](int t) {    // volume point -> padded index
        if constexpr (XQ == Q) return t;
        else return t % Q + XQ * (t / Q);
    };
    extern __shared__ double lds[];
    const int epb = A.epb;
    double* mchi = lds;               // Q x N
    double* mpit = mchi + Q * N;      // N x Q
    double* mdq = mpit + N * Q;       // Q x Q
    double* mtl = mdq + Q2;           // Q
    double* mtr = mtl + Q;            // Q
    double* mw = mtr + Q;             // Q
    double* VA = mw + Q;              // epb 5 BQ
    double* VB = VA + epb * 5 * BQ;   // epb 5 XQ Q N
    double* RF = VB + epb * 5 * XQ * Q * N;   // epb [6][5][Q^2]
    double* TF = RF + epb * 30 * Q2;      // epb [6][5][Q N]
    const int tid = threadIdx.x, nth = blockDim.x;
    const int64_t E = A.geo.E;
    const int64_t e0 = (int64_t)blockIdx.x * epb;
    const int nel = (int)(E - e0 < epb ? E - e0 : epb);   // elements of this block that exist
    const int64_t SE = E * N3;
    const double gamma = A.gamma, gm1 = gamma - 1.0;
    const double pref = reference_pressure(A.Uin, SE, gm1);
    const GLOps* ops = G.ops;
    for (int i = tid; i < Q * N; i += nth) {
        mchi[i] = ops->chi[i];
        mpit[i] = ops->pit[i];
    }
    for (int i = tid; i < Q2; i += nth) mdq[i] = ops->dq[i];
    for (int i = tid; i < Q; i += nth) {
        mtl[i] = ops->tl[i];
        mtr[i] = ops->tr[i];
        mw[i] = ops->wq[i];
    }
    // 1. u at the volume points: chi along x, y, z (VB -> VA -> VB -> VA);
    //    missing elements of a ragged last block are zero-filled
    for (int i = tid; i < epb * 5 * N3; i += nth) {
        const int el = i / (5 * N3), r = i - el * 5 * N3;
        const int s = r / N3, nd = r - s * N3;
        VB[(el * 5 + s) * BN + pn(nd)] = el < nel ? A.Uin[s * SE + (e0 + el) * N3 + nd] : 0.0;
    }
    __syncthreads();
    lds_pass<N, N, N, 0, Q, false, XN, XQ>(VB, VA, mchi, 5 * epb);
    __syncthreads();
    lds_pass<Q, N, N, 1, Q, false, XQ, XQ>(VA, VB, mchi, 5 * epb);
    __syncthreads();
    lds_pass<Q, Q, N, 2, Q, false, XQ, XQ>(VB, VA, mchi, 5 * epb);
    __syncthreads();

    // 2. one thread per (element, line): the contravariant flux f^r_k at the
    //    line's points, its flux-basis derivative (R_v[a] = w_a W_perp
    //    sum_b Dq[a][b] f^r_k(b)), its values at the two ends, and Roe's flux
    //    with the neighbour there
    const int el = tid / L3;
    const bool active = el < nel;
    const int lt = active ? tid - el * L3 : 0;
    const int dir = lt / Q2;
    const int l = lt - dir * Q2;
    const int64_t e = e0 + (active ? el : 0);
    const int t1 = l % Q, t2 = l / Q;
    // the line's first point and point stride in the padded volume arrays
    const int base = dir == 0 ? XQ * (t1 + Q * t2) : (dir == 1 ? t1 + XQ * Q * t2 : t1 + XQ * t2);
    const int stride = dir == 0 ? 1 : (dir == 1 ? XQ : XQ * Q);
    double* va = VA + (active ? el : 0) * 5 * BQ;
    const double wperp = mw[t1] * mw[t2];
    // (a) the flux-basis derivative along the line and the line's end values of
    //     f^r_k; the volume part into VA in a fixed direction order
    double Rf[2][5];
    {
        double Rv[5][Q];
#pragma unroll
        for (int s = 0; s < 5; ++s) {
#pragma unroll
            for (int a = 0; a < Q; ++a) Rv[s][a] = 0.0;
            Rf[0][s] = Rf[1][s] = 0.0;
        }
        if (active) {
            const double* Cl = G.geo.Cq + (int64_t)(3 * dir) * E * Q3 + e * Q3 + l;
            const int64_t CS = E * Q3;
#pragma unroll
            for (int b = 0; b < Q; ++b) {
                const int t = base + b * stride;
                const double r = va[t], m1 = va[BQ + t], m2 = va[2 * BQ + t], m3 = va[3 * BQ + t],
                             en = va[4 * BQ + t];
                const double cx = Cl[b * Q2], cy = Cl[CS + b * Q2], cz = Cl[2 * CS + b * Q2];
                const double ir = 1.0 / r;
                const double unb = (m1 * cx + m2 * cy + m3 * cz) * ir;
                const double p = gm1 * (en - 0.5 * (m1 * m1 + m2 * m2 + m3 * m3) * ir);
                const double pd = p - pref;
                const double fr[5] = {r * unb, m1 * unb + pd * cx, m2 * unb + pd * cy, m3 * unb + pd * cz,
                                      (en + p) * unb};
#pragma unroll
                for (int s = 0; s < 5; ++s) {
#pragma unroll
                    for (int a = 0; a < Q; ++a) Rv[s][a] = __builtin_fma(mdq[a * Q + b], fr[s], Rv[s][a]);
                    Rf[0][s] = __builtin_fma(mtl[b], fr[s], Rf[0][s]);
                    Rf[1][s] = __builtin_fma(mtr[b], fr[s], Rf[1][s]);
                }
            }
        }
        __syncthreads();   // the volume states (VA) are no longer read
        for (int ph = 0; ph < 3; ++ph) {
            if (active && dir == ph) {
#pragma unroll
                for (int s = 0; s < 5; ++s)
#pragma unroll
                    for (int a = 0; a < Q; ++a) {
                        const double v = Rv[s][a] * (mw[a] * wperp);
                        double* x = va + s * BQ + base + a * stride;
                        if (ph == 0) *x = v;
                        else *x += v;
                    }
            }
            __syncthreads();
        }
    }
    // (b) the face terms at both ends, N . f* - s t . f^r (s = -1 left, +1
    //     right), with Roe's flux against the neighbour's face state
    if (active) {
        const int64_t FS = E * Q2;
        double* rf = RF + el * 30 * Q2;
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int f = 2 * dir + side;
            const double sg = side ? 1.0 : -1.0;
            const double* Cfo = G.geo.Cf + ((int64_t)(f * 3) * E + e) * Q2 + l;
            const int en = A.geo.nbr[(int64_t)f * E + e];
            const int fn = 2 * dir + (1 - side);
            const double* Cfn = G.geo.Cf + ((int64_t)(fn * 3) * E + en) * Q2 + l;
            const double nx = 0.5 * sg * (Cfo[0] + Cfn[0]), ny = 0.5 * sg * (Cfo[FS] + Cfn[FS]),
                         nz = 0.5 * sg * (Cfo[2 * FS] + Cfn[2 * FS]);
            double uo[5], un[5], F[5];
#pragma unroll
            for (int s = 0; s < 5; ++s) {
                uo[s] = G.ft[((int64_t)(f * 5 + s) * E + e) * Q2 + l];
                un[s] = G.ft[((int64_t)(fn * 5 + s) * E + en) * Q2 + l];
            }
            roe_flux_dev(uo, un, nx, ny, nz, gamma, pref, F);
#pragma unroll
            for (int s = 0; s < 5; ++s) rf[(f * 5 + s) * Q2 + l] = (F[s] - sg * Rf[side][s]) * wperp;
        }
    }
    const int mode = A.mode;
    double dt = 0.0, cstage = 0.0;
    if (mode >= MODE_RK1) {
        dt = *A.dt;
        cstage = (mode == MODE_RK1) ? 0.0 : (mode == MODE_RK4 ? 1.0 : 0.5);
    }
    if (A.source) {
        const double t = (A.tdev ? *A.tdev : A.t) + cstage * dt;
        const int64_t EQ = E * Q3;
        for (int i = tid; i < nel * Q3; i += nth) {
            const int ei = i / Q3, p = i - ei * Q3;
            double qs[5];
            const double* X = G.geo.Xq + (e0 + ei) * Q3 + p;
            mms_source(X[0], X[EQ], X[2 * EQ], t, gamma, qs);
            const double wj = 1.0 / G.geo.invWJ[(e0 + ei) * Q3 + p];
#pragma unroll
            for (int s = 0; s < 5; ++s) VA[(ei * 5 + s) * BQ + pq(p)] -= wj * qs[s];
        }
    }
    __syncthreads();
    // 3. chi^T along z, y, x (VA -> VB -> VA -> VB), face residuals onto the end slabs
    lds_pass<Q, Q, Q, 2, N, true, XQ, XQ>(VA, VB, mchi, 5 * epb);
    lds_pass<Q, Q, 1, 0, N, true>(RF, TF, mchi, 30 * epb);
    __syncthreads();
    lds_pass<Q, Q, N, 1, N, true, XQ, XQ>(VB, VA, mchi, 5 * epb);
    lds_pass<N, Q, 1, 1, N, true>(TF, RF, mchi, 30 * epb);
    __syncthreads();
    lds_pass<Q, N, N, 0, N, true, XQ, XN>(VA, VB, mchi, 5 * epb);
    __syncthreads();
    scatter_add_slabs<N, XN, N>(VB, RF, epb);
    __syncthreads();
    if (mode == MODE_RESIDUAL) {
        for (int it = tid; it < nel * 5 * N3; it += nth) {
            const int ei = it / (5 * N3), r0 = it - ei * 5 * N3;
            const int s = r0 / N3, nd = r0 - s * N3;
            A.out[s * SE + (e0 + ei) * N3 + nd] = VB[(ei * 5 + s) * BN + pn(nd)];
        }
        return;
    }
    // 4. weight-adjusted inverse: Pi~^T (VB -> VA -> VB -> VA), 1 / (W J), Pi~ (VA -> VB -> VA -> VB)
    lds_pass<N, N, N, 0, Q, true, XN, XQ>(VB, VA, mpit, 5 * epb);
    __syncthreads();
    lds_pass<Q, N, N, 1, Q, true, XQ, XQ>(VA, VB, mpit, 5 * epb);
    __syncthreads();
    lds_pass<Q, Q, N, 2, Q, true, XQ, XQ>(VB, VA, mpit, 5 * epb);
    __syncthreads();
    for (int it = tid; it < nel * 5 * Q3; it += nth) {
        const int ei = it / (5 * Q3), t = it % Q3;
        if constexpr (XQ == Q) VA[it] *= G.geo.invWJ[(e0 + ei) * Q3 + t];
        else VA[(it / Q3) * BQ + pq(t)] *= G.geo.invWJ[(e0 + ei) * Q3 + t];
    }
    __syncthreads();
    lds_pass<Q, Q, Q, 2, N, false, XQ, XQ>(VA, VB, mpit, 5 * epb);
    __syncthreads();
    lds_pass<Q, Q, N, 1, N, false, XQ, XQ>(VB, VA, mpit, 5 * epb);
    __syncthreads();
    lds_pass<Q, N, N, 0, N, false, XQ, XN>(VA, VB, mpit, 5 * epb);
    __syncthreads();
    // 5. RK combination
    for (int it = tid; it < nel * 5 * N3; it += nth) {
        const int ei = it / (5 * N3), r0 = it - ei * 5 * N3;
        const int s = r0 / N3, nd = r0 - s * N3;
        const int64_t gi = s * SE + (e0 + ei) * N3 + nd;
        const double k = -VB[(ei * 5 + s) * BN + pn(nd)];
        switch (mode) {
            case MODE_RHS: A.out[gi] = k; break;
            case MODE_RK1: {
                const double u = A.Uin[gi];
                A.acc[gi] = __builtin_fma(dt / 6.0, k, u);
                A.out[gi] = __builtin_fma(0.5 * dt, k, u);
            } break;
            case MODE_RK2:
                A.acc[gi] = __builtin_fma(dt / 3.0, k, A.acc[gi]);
                A.out[gi] = __builtin_fma(0.5 * dt, k, A.Un[gi]);
                break;
            case MODE_RK3:
                A.acc[gi] = __builtin_fma(dt / 3.0, k, A.acc[gi]);
                A.out[gi] = __builtin_fma(dt, k, A.Un[gi]);
                break;
            default: A.out[gi] = __builtin_fma(dt / 6.0, k, A.acc[gi]); break;
        }
    }
}

static size_t dg_stage_lds(int p, int q, int epb) {
    const int n = p + 1;
    return (size_t)dg_stage_doubles(n, q, dg_row_pitch(n, q), epb) * sizeof(double);
}

// the projection kernels: operators, state buffers, and the face-slab
// buffers [6][5] x (n^2, q n, q^2)
static size_t slab_lds(int n, int q) { return (size_t)30 * (n * n + q * n + q * q); }

static size_t dg_project_lds(int p, int q) {
    const int n = p + 1;
    return (2 * q * n + 5 * n * n * n + slab_lds(n, q)) * sizeof(double);
}

static size_t gl_stage_lds(int p, int q) {
    const int n = p + 1, xn = bank_pitch(n), xq = bank_pitch(q);   // row pitches of the kernel's LDS arrays
    (void)xn;
    return (size_t)(2 * q * n + q * q + 3 * q + 11 * xq * q * q + 66 * q * q + 30 * q * n) * sizeof(double);
}

static size_t gl_project_lds(int p, int q) {
    const int n = p + 1, xn = bank_pitch(n), xq = bank_pitch(q);   // row pitches of the kernel's LDS arrays
    return (2 * q * n + 10 * (size_t)xq * q * q + 30 * (xn * n + xq * n + xq * q)) * sizeof(double);
}

size_t gl_lds_bytes(bool dg, int p, int q, int epb) {
    const size_t a = dg ? dg_stage_lds(p, q, epb) : gl_stage_lds(p, q);
    const size_t b = dg ? dg_project_lds(p, q) : gl_project_lds(p, q);
    return a > b ? a : b;
}

int gl_max_epb(bool dg, int p, int q, size_t lds_max) {
    if (!dg) return 1;
    int m = DG_BLOCK / (3 * q * q);
    while (m > 0 && gl_lds_bytes(dg, p, q, m) > lds_max) --m;
    return m;
}

int gl_default_epb(bool dg, int p, int q, int64_t E) {
    if (!dg) return 1;
    // about 256 threads per workgroup, but at least 2048 workgroups when the
    // mesh has them (8 per CU)
    int epb = 256 / (3 * q * q);
    while (epb > 1 && (E + epb - 1) / epb < 2048) --epb;
    return epb < 1 ? 1 : epb;
}

template <int N, int Q>
static hipError_t gl_geometry_nq(const GLOps* ops, int64_t E, const double* X, const double* Cline, double* Cq,
                                 double* Cf, double* invWJ, double* Xq, hipStream_t s) {
    const int64_t nv = E * Q * Q * Q, nf = E * 6 * Q * Q;
    gl_geometry_kernel<N, Q><<<(unsigned)((nv + 127) / 128), 128, 0, s>>>(ops, E, X, Cline, Cq, invWJ, Xq);
    gl_face_geometry_kernel<N, Q><<<(unsigned)((nf + 127) / 128), 128, 0, s>>>(ops, E, Cline, Cf);
    return hipGetLastError();
}

template <int N, int Q>
static hipError_t gl_stage_nq(int variant, const StageArgs& a, const GLArgs& g, hipStream_t s) {
    static_assert(3 * Q * Q <= GL_BLOCK, "one thread per line");
    const size_t lp = gl_project_lds(N - 1, Q), ls = gl_stage_lds(N - 1, Q);
    const unsigned blocks = (unsigned)a.geo.E;
    const int threads = ((3 * Q * Q + 63) / 64) * 64;
    gl_project_kernel<N, Q, false><<<blocks, GL_BLOCK, lp, s>>>(g.ops, a.geo.E, a.Uin, a.gamma, g.vhat, g.ft);
    if (variant) gl_stage_kernel<N, Q, 1><<<blocks, threads, ls, s>>>(a, g);
    else gl_stage_kernel<N, Q, 0><<<blocks, threads, ls, s>>>(a, g);
    return hipGetLastError();
}

template <int N, int Q>
static hipError_t dg_stage_nq(const StageArgs& a, const GLArgs& g, hipStream_t s) {
    static_assert(3 * Q * Q <= DG_BLOCK, "one thread per line");
    const int epb = a.epb;
    if (epb < 1 || epb * 3 * Q * Q > DG_BLOCK) return hipErrorInvalidConfiguration;
    const size_t lp = dg_project_lds(N - 1, Q), ls = dg_stage_lds(N - 1, Q, epb);
    const int threads = ((epb * 3 * Q * Q + 63) / 64) * 64;
    gl_project_kernel<N, Q, true><<<(unsigned)a.geo.E, GL_BLOCK, lp, s>>>(g.ops, a.geo.E, a.Uin, a.gamma, g.vhat,
                                                                          g.ft);
    dg_stage_kernel<N, Q><<<(unsigned)((a.geo.E + epb - 1) / epb), threads, ls, s>>>(a, g);
    return hipGetLastError();
}

// configure every kernel of an (N, Q) pair for its dynamic LDS (needed when a
// workgroup uses more than the default 64 KB)
static hipError_t set_lds(const void* f, size_t bytes) {
    return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int N, int Q>
static hipError_t gl_set_lds(size_t bytes) {
    hipError_t e = set_lds((const void*)gl_project_kernel<N, Q, false>, bytes);
    if (e == hipSuccess) e = set_lds((const void*)gl_stage_kernel<N, Q, 0>, bytes);
    if (e == hipSuccess) e = set_lds((const void*)gl_stage_kernel<N, Q, 1>, bytes);
    return e;
}

template <int N, int Q>
static hipError_t dg_set_lds(size_t bytes) {
    hipError_t e = set_lds((const void*)gl_project_kernel<N, Q, true>, bytes);
    if (e == hipSuccess) e = set_lds((const void*)dg_stage_kernel<N, Q>, bytes);
    return e;
}

// (n, q) pairs: NSFR with up to 3 extra points per direction, conservative DG
// with up to n extra (a rule of 2 (p + 1) points); the geometry serves both
#define NSFR_GL_TABLE(X)                                                                                     \
    X(3, 3) X(3, 4) X(3, 5) X(3, 6) X(4, 4) X(4, 5) X(4, 6) X(4, 7) X(5, 5) X(5, 6) X(5, 7) X(5, 8) X(6, 6) \
        X(6, 7) X(6, 8) X(6, 9)
#define NSFR_DG_TABLE(X)                                                                                     \
    X(3, 3) X(3, 4) X(3, 5) X(3, 6) X(4, 4) X(4, 5) X(4, 6) X(4, 7) X(4, 8) X(5, 5) X(5, 6) X(5, 7) X(5, 8) \
        X(5, 9) X(5, 10) X(6, 6) X(6, 7) X(6, 8) X(6, 9) X(6, 10) X(6, 11) X(6, 12)

hipError_t launch_gl_geometry(int p, int q, const GLOps* ops, int64_t E, const double* X, const double* Cline,
                              double* Cq, double* Cf, double* invWJ, double* Xq, hipStream_t s) {
#define NSFR_GEO(NN, QQ) \
    if (p + 1 == NN && q == QQ) return gl_geometry_nq<NN, QQ>(ops, E, X, Cline, Cq, Cf, invWJ, Xq, s);
    NSFR_DG_TABLE(NSFR_GEO)
#undef NSFR_GEO
    return hipErrorInvalidValue;
}

hipError_t launch_gl_stage(bool dg, int p, int q, int variant, const StageArgs& a, const GLArgs& g, hipStream_t s) {
#define NSFR_STG(NN, QQ) \
    if (p + 1 == NN && q == QQ) return gl_stage_nq<NN, QQ>(variant, a, g, s);
#define NSFR_DGS(NN, QQ) \
    if (p + 1 == NN && q == QQ) return dg_stage_nq<NN, QQ>(a, g, s);
    if (dg) {
        NSFR_DG_TABLE(NSFR_DGS)
    } else {
        NSFR_GL_TABLE(NSFR_STG)
    }
#undef NSFR_STG
#undef NSFR_DGS
    return hipErrorInvalidValue;
}

hipError_t gl_prepare(bool dg, int p, int q, size_t bytes) {
#define NSFR_LDS(NN, QQ) \
    if (p + 1 == NN && q == QQ) return gl_set_lds<NN, QQ>(bytes);
#define NSFR_DGL(NN, QQ) \
    if (p + 1 == NN && q == QQ) return dg_set_lds<NN, QQ>(bytes);
    if (dg) {
        NSFR_DG_TABLE(NSFR_DGL)
    } else {
        NSFR_GL_TABLE(NSFR_LDS)
    }
#undef NSFR_LDS
#undef NSFR_DGL
    return hipErrorInvalidValue;
}

}  // namespace nsfr
