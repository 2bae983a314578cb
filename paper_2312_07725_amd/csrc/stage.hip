// Fused NSFR right-hand-side / RK4-stage kernel for gfx950.
//
// Paper: Eq. NSFR (volume Hadamard term with the hybridised skew-symmetric
// operator, surface numerical flux), Sec. 5 (sum-factorised Hadamard product:
// on the tensor-product LGL element the volume-volume block of (Q~ - Q~^T) in
// direction k is S1 (x) W (x) W, nonzero only between nodes of one k-line;
// the surface-volume blocks cancel on collocated LGL nodes), Eq. weight-adj
// ESFR mass (A = Pi~ (W J)^-1 Pi~^T, Pi~ a tensor product of rank-one
// corrections of the identity), Sec. 7 opening paragraph (four-stage,
// fourth-order RK: read as classical RK4).
//
// Work decomposition: a workgroup owns `epb` elements. Every element has
// 3 (p+1)^2 lines (p+1)^2 per direction; one thread owns one line. Its line's
// residual lives in registers, the primitives (and at p = 3 the metric
// columns) in LDS, all
// (p+1) p / 2 node pairs are evaluated once each (pair symmetry), and the two
// endpoint face fluxes of the line are computed by the same thread, so every
// face node's surface term belongs to exactly one thread (no atomics; the
// kernel is deterministic). The partial residuals of the three directions go
// to three LDS slots and are summed in a fixed order by the first pass of the
// weight-adjusted inverse (plane and zeta-line passes); the RK combination
// runs node-parallel.
#include "nsfr_host.h"

namespace nsfr {

constexpr int STAGE_BLOCK_MAX = 512;

// Accumulator layout after the line sweep: per element three slots (one per
// line direction) of [5][SPN] (padded node index; SPN = slot_stride(N)),
// EBLK = acc_elem_stride(N) >= 3 SLOT doubles per element.
//
// The weight-adjusted inverse Pi~ (W J)^-1 Pi~^T with Pi~ = P (x) P (x) P,
// P = I - pia pib^T applied along a line as x <- x - pia (pib . x) (and P^T
// as x <- x - pib (pia . x)). The three 1D factors act on different indices
// and commute, so the operator is applied as P_xi P_eta [P_zeta (W J)^-1
// P_zeta^T] P_xi^T P_eta^T: a plane pass, a zeta-line pass that also scales,
// and a plane pass (three barriers instead of seven).

// Rank-one operator along xi and along eta on every (element, state,
// zeta-plane) of the workgroup: w <- w - vec (coef . w) on each xi-row, then
// on each eta-column. With SUM the input is the sum of the three direction
// slots (fixed order) and the result goes to slot 0.
template <int N, int SPN, int EBLK, bool SUM>
__device__ __forceinline__ void plane_pass(double* lr, int epb, const double* coef, const double* vec) {
    constexpr int N2 = N * N, SLOT = 5 * SPN;
    for (int it = threadIdx.x; it < epb * 5 * N; it += blockDim.x) {
        const int k = it % N, sl = it / N;   // zeta plane; element * 5 + state
        const int eli = sl / 5, st = sl - eli * 5;
        double* x = lr + eli * EBLK + st * SPN + pad_node<N>(N2 * k);   // the plane's first node
        constexpr int R = padded_row<N>();
        double w[N][N];   // [eta][xi]
#pragma unroll
        for (int j = 0; j < N; ++j)
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int pn = i + R * j;
                w[j][i] = SUM ? (x[pn] + x[SLOT + pn]) + x[2 * SLOT + pn] : x[pn];
            }
#pragma unroll
        for (int j = 0; j < N; ++j) {
            double t = 0.0;
#pragma unroll
            for (int i = 0; i < N; ++i) t += coef[i] * w[j][i];
#pragma unroll
            for (int i = 0; i < N; ++i) w[j][i] = w[j][i] - vec[i] * t;
        }
#pragma unroll
        for (int i = 0; i < N; ++i) {
            double t = 0.0;
#pragma unroll
            for (int j = 0; j < N; ++j) t += coef[j] * w[j][i];
#pragma unroll
            for (int j = 0; j < N; ++j) w[j][i] = w[j][i] - vec[j] * t;
        }
#pragma unroll
        for (int j = 0; j < N; ++j)
#pragma unroll
            for (int i = 0; i < N; ++i) x[i + R * j] = w[j][i];
    }
}

// P^T, the scaling by 1/(W J) at the line's nodes and P along zeta-lines,
// in slot 0. The epb * 5 * N^2 (element, state, line) items go to the
// threads as item tid + j * nth, j < 2 (nth >= epb * 3 N^2 covers them in
// two rounds); iw[j] holds 1/(W J) at item j's nodes, prefetched by the
// caller.
template <int N, int SPN, int EBLK>
__device__ __forceinline__ void zeta_pass(double* lr, int epb, const double (&iw)[2][N], const double* pia,
                                          const double* pib) {
    constexpr int N2 = N * N;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int it = threadIdx.x + j * blockDim.x;
        if (it >= epb * 5 * N2) break;
        const int l = it % N2, sl = it / N2;   // zeta line (base l, stride N^2); element * 5 + state
        const int eli = sl / 5, st = sl - eli * 5;
        double* x = lr + eli * EBLK + st * SPN + pad_node<N>(l);   // the line's first node
        constexpr int RN = padded_row<N>() * N;                         // padded zeta step
        double v[N];
        double t = 0.0;
#pragma unroll
        for (int a = 0; a < N; ++a) {
            v[a] = x[a * RN];
            t += pia[a] * v[a];
        }
#pragma unroll
        for (int a = 0; a < N; ++a) v[a] = (v[a] - pib[a] * t) * iw[j][a];
        t = 0.0;
#pragma unroll
        for (int a = 0; a < N; ++a) t += pib[a] * v[a];
#pragma unroll
        for (int a = 0; a < N; ++a) x[a * RN] = v[a] - pia[a] * t;
    }
}

// The whole stage for the `epb` elements starting at e0 (one workgroup).
//
// Where a line thread reads its line's metric column (3 N values): at p = 3
// from LDS (all nine columns staged line-major, [dir][comp][position][line],
// 9 N3 doubles per element), elsewhere from registers loaded straight from
// the line-major array. Under the 3-waves-per-SIMD register cap of p = 3 the
// LDS copy can be re-read instead of spilled; at p = 4, 5 (no cap) holding
// the column in registers measured slightly faster.
__host__ __device__ constexpr bool metric_in_lds(int p) { return p == 3; }

// State stride (doubles) of an accumulator slot. The lanes of a plane pass
// read the same node of consecutive (zeta plane, state) blocks, at LDS
// addresses N^2 k + SPN s (N^2 padded to N^2 + N for even N). In a model of
// the LDS as 32 four-byte banks serving a 64-bit access 16 lanes at a time
// (it reproduces the bank-conflict counts measured on gfx950 within 15%),
// such a group is conflict-free when its addresses differ mod 16. One more
// than the padded block (N^3 + N^2 + 1) achieves that for N = 3, 4; for
// N = 5 it (151) folds the lanes onto 8 bank pairs and 141 spreads them (the
// unpadded N = 5 block needs 125); for N = 6 the padded plane step (42, even)
// leaves conflicts that no stride removes, and 253 is as good as any.
__host__ __device__ constexpr int slot_stride(int n) { return n == 5 ? 141 : n * n * n + n * n + 1; }

// Element stride (doubles) of the accumulator: the three slots, plus a pad
// where the 5 N items of an element's plane pass (not a multiple of 16) let a
// 16-lane group straddle two elements: 2 doubles at N = 4 and 14 at N = 5 put
// the second element's blocks on the bank pairs the first leaves free (the
// tile limits stay 6 and 3).
__host__ __device__ constexpr int acc_elem_stride(int n) { return 15 * slot_stride(n) + (n == 4 ? 2 : n == 5 ? 14 : 0); }

// LDS per element (doubles): during the sweep the primitives [6][PN3]
// (padded) and at p = 3 the metric columns [9][N3]; afterwards the three
// direction slots [3][5][slot_stride] of the accumulator.
__host__ __device__ constexpr int stage_lds_per_elem(int n) {
    const int sweep = 6 * (n * n * n + n * n) + (metric_in_lds(n - 1) ? 9 * n * n * n : 0);
    const int acc = acc_elem_stride(n);
    return sweep > acc ? sweep : acc;
}

// A line thread keeps its residual in registers and reads the primitives
// from LDS inside the pair loop; after the sweep the LDS holds the direction
// slots of the accumulator.
template <int P, bool CWA, int VARIANT, int DISS>
__device__ __forceinline__ void stage_body(const StageArgs& A, const int64_t e0, double* lds) {
    constexpr int N = P + 1, N2 = N * N, N3 = N2 * N, LINES = 3 * N2;
    constexpr int PN3 = padded_block<N>();          // padded stride of a primitive component
    constexpr bool MLDS = metric_in_lds(P);
    constexpr int SPN = slot_stride(N);              // state stride of an accumulator slot
    static_assert(SPN >= (N % 2 ? N3 : PN3), "a slot state must hold the (padded) node block");
    constexpr int SLOT = 5 * SPN, EBLK = acc_elem_stride(N);   // direction slots of the accumulator
    constexpr int LDSE = stage_lds_per_elem(N);         // LDS doubles per element
    const int tid = threadIdx.x, nth = blockDim.x;
    const int epb = A.epb;
    const int64_t E = A.geo.E;
    const int64_t SE = E * N3;   // state stride
    // The workgroup's elements are consecutive (the last workgroup may hold
    // fewer than epb): its nodes are g0 + idx, idx < nwg, so node-parallel
    // work indexes global memory by a uniform base and a 32-bit lane offset.
    const int nel = (int)(E - e0 < epb ? E - e0 : epb);
    const int nwg = nel * N3;
    const int64_t g0 = e0 * N3;
    const double gm1 = A.gamma - 1.0;
    const double c1 = A.c1;
    const double pref = reference_pressure(A.Uin, SE, gm1);

    // ---- line ownership (one thread per line)
    const bool lt = tid < epb * LINES;
    const int el = lt ? tid / LINES : 0;
    const int rem = lt ? tid - el * LINES : 0;   // threads past the last line take line 0 (and stay idle)
    const int dir = rem / N2;
    const int l = rem - dir * N2;
    const int64_t e = e0 + el;
    const bool active = lt && (e < E);
    // metric column of the line in registers, straight from the line-major
    // array (coalesced across the lines of a direction; the loads overlap the
    // staging below)
    double cl[3][N];
    if (!MLDS && active) {
        const double* Cg = A.geo.Cline + ((int64_t)(3 * dir) * E + (active ? e : 0)) * N3 + l;
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int a = 0; a < N; ++a) cl[m][a] = Cg[(int64_t)m * SE + a * N2];
    }

    // ---- 1. stage the workgroup's elements: thread tid takes the nodes
    //         tid + j * nth, j < KS (nth >= epb * 3 N^2, so KS = ceil(N / 3)
    //         covers epb N^3). All state (and at p = 3 metric) loads are
    //         issued first, then the face traces below, then the primitives
    //         are formed, so that the staging's own data is not queued behind
    //         the traces.
    constexpr int KS = (N + 2) / 3;
    constexpr int NCS = MLDS ? 9 : 1;
    double su[KS][5], sc[KS][NCS];
#pragma unroll
    for (int j = 0; j < KS; ++j) {
        const int idx = tid + j * nth;
        if (idx < nwg) {
            const double* U = A.Uin + g0 + idx;
#pragma unroll
            for (int s = 0; s < 5; ++s) su[j][s] = U[s * SE];
            if (MLDS) {
                const double* Cg = A.geo.Cline + g0 + idx;   // same offset in line-major order
#pragma unroll
                for (int k = 0; k < NCS; ++k) sc[j][k] = Cg[k * SE];
            }
        }
    }

    // line geometry, and the traces of the two face neighbours across the
    // line's ends (periodic box): conserved state and metric column at the
    // neighbour's end node (and, with local Lax-Friedrichs, the own conserved
    // state). Requested before the primitives are formed, so that their latency
    // overlaps the staging.
    // A neighbour inside the workgroup's own element range (the workgroup's
    // elements are consecutive, so most xi-neighbours are) has its primitives
    // staged in LDS: its state is not loaded (fin = its local index). The
    // staged primitives are the ones computed from the loaded state, so the
    // flux is the same bit for bit; local Lax-Friedrichs needs the conserved
    // jump and always loads.
    int base, stride;
    line_geometry<N>(dir, l, base, stride);
    const int pbase = pad_node<N>(base), pstride = padded_stride<N>(dir);   // the line in the LDS node index
    double fU[2][5], fC[2][3], oU[2][5];
    int fin[2] = {-1, -1};
    if (active) {
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int anbr = side ? 0 : N - 1;
            const int64_t en = neighbour((int)e, dir, side ? 1 : -1, A.geo.nx, A.geo.ny, A.geo.nz);
            const double* Cn = A.geo.Cline + ((int64_t)(dir * 3) * E + en) * N3 + anbr * N2 + l;
            const double* Ub = A.Uin + en * N3 + base + anbr * stride;
            const int64_t loc = en - e0;
            if (DISS != 1 && loc >= 0 && loc < epb) fin[side] = (int)loc;
#pragma unroll
            for (int s = 0; s < 5; ++s) fU[side][s] = fin[side] < 0 ? Ub[s * SE] : 0.0;
#pragma unroll
            for (int m = 0; m < 3; ++m) fC[side][m] = Cn[m * SE];
            if (DISS == 1) {
                const double* Uo = A.Uin + e * N3 + base + (side ? N - 1 : 0) * stride;
#pragma unroll
                for (int s = 0; s < 5; ++s) oU[side][s] = Uo[s * SE];
            }
        }
    }

    // primitives (and at p = 3 the metric columns) -> LDS
#pragma unroll
    for (int j = 0; j < KS; ++j) {
        const int idx = tid + j * nth;
        const int eli = idx / N3, node = idx - eli * N3;
        if (idx < nwg) {
            const PrimR q = primitives_ref(su[j][0], su[j][1], su[j][2], su[j][3], su[j][4], gm1, pref);
            double* L = lds + eli * LDSE + pad_node<N>(node);
            L[0] = q.rho;
            L[PN3] = q.u;
            L[2 * PN3] = q.v;
            L[3 * PN3] = q.w;
            L[4 * PN3] = q.pd;
            L[5 * PN3] = q.beta;
            if (MLDS) {
                double* Lc0 = lds + eli * LDSE + 6 * PN3 + node;
#pragma unroll
                for (int k = 0; k < NCS; ++k) Lc0[k * N3] = sc[j][k];
            }
        }
    }
    __syncthreads();

    // ---- 2. the line's views of LDS
    const double* Lp = lds + el * LDSE;                             // primitives
    const double* Lc = lds + el * LDSE + 6 * PN3 + 3 * dir * N3 + l;   // [comp][position][line] (p = 3)
    auto cmet = [&](int m, int a) { return MLDS ? Lc[m * N3 + a * N2] : cl[m][a]; };

    // ---- 3. line residual: the two endpoint face fluxes, then the volume pairs
    double R[5][N];
#pragma unroll
    for (int s = 0; s < 5; ++s)
#pragma unroll
        for (int a = 0; a < N; ++a) R[s][a] = 0.0;
    if (active) {
        // the two endpoint face fluxes (own trace against the neighbour's)
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int aown = side ? N - 1 : 0;
            const double sg = side ? 0.5 : -0.5;   // outward reference normal / 2
            const int anbr = side ? 0 : N - 1;
            const PrimR qn = fin[side] >= 0
                                 ? lds_primr<PN3>(lds + fin[side] * LDSE, pbase + anbr * pstride)
                                 : primitives_ref(fU[side][0], fU[side][1], fU[side][2], fU[side][3], fU[side][4], gm1, pref);
            const PrimR qo = lds_primr<PN3>(Lp, pbase + aown * pstride);
            const double nx = sg * (cmet(0, aown) + fC[side][0]), ny = sg * (cmet(1, aown) + fC[side][1]),
                         nz = sg * (cmet(2, aown) + fC[side][2]);
            double F[5];
            ec_flux<VARIANT>(qo, qn, nx, ny, nz, c1, pref, F);
            if (DISS == 1) llf_add(qo, qn, oU[side], fU[side], nx, ny, nz, A.gamma, pref, F);
            else if (DISS == 2) roe_add(qo, qn, nx, ny, nz, A.gamma, pref, F);
#pragma unroll
            for (int s = 0; s < 5; ++s) R[s][aown] += F[s];
        }
        // volume pairs of the line
#pragma unroll
        for (int a = 0; a < N - 1; ++a) {
            const PrimR qa = lds_primr<PN3>(Lp, pbase + a * pstride);
            const double cax = cmet(0, a), cay = cmet(1, a), caz = cmet(2, a);
#pragma unroll
            for (int b = a + 1; b < N; ++b) {
                const PrimR qb = lds_primr<PN3>(Lp, pbase + b * pstride);
                const double cbx = cmet(0, b), cby = cmet(1, b), cbz = cmet(2, b);
                double F[5];
                // direction C(a) + C(b) = 2 N; the 1/2 is folded into S1h
                ec_flux<VARIANT>(qa, qb, cax + cbx, cay + cby, caz + cbz, c1, pref, F);
                const double sab = A.ops.S1h[a][b];
#pragma unroll
                for (int s = 0; s < 5; ++s) {
                    R[s][a] = __builtin_fma(sab, F[s], R[s][a]);
                    R[s][b] = __builtin_fma(-sab, F[s], R[s][b]);
                }
            }
        }
    }
    // The node-parallel epilogue gives thread tid the nodes tid + j * nth,
    // j < KP (nth >= epb * 3 N^2); with the weight-adjusted inverse it also
    // scales the zeta-line items of zeta_pass. Request their global operands
    // now, so that the latency overlaps the LDS passes.
    constexpr int KP = (N + 2) / 3;
    const int mode = A.mode;
    double pf_iw[KP], pf_a[KP][5], pf_b[KP][5], zw[2][N];
    auto fetch_epilogue = [&]() {
#pragma unroll
        for (int j = 0; j < KP; ++j) {
            const int idx = tid + j * nth;
            pf_iw[j] = 0.0;
#pragma unroll
            for (int s = 0; s < 5; ++s) pf_a[j][s] = pf_b[j][s] = 0.0;
            if (idx < nwg && mode != MODE_RESIDUAL) {
                const int64_t g = g0 + idx;
                if (!CWA) pf_iw[j] = A.geo.invWJ[g];
                const double* pa = mode == MODE_RK1 ? A.Uin : A.acc;
#pragma unroll
                for (int s = 0; s < 5; ++s) {
                    if (mode >= MODE_RK1) pf_a[j][s] = pa[s * SE + g];
                    if (mode == MODE_RK2 || mode == MODE_RK3) pf_b[j][s] = A.Un[s * SE + g];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int it = tid + j * nth;
            const int zl = it % N2, eli = it / N2 / 5;
#pragma unroll
            for (int a = 0; a < N; ++a) zw[j][a] = 0.0;
            if (CWA && mode != MODE_RESIDUAL && it < nel * 5 * N2) {
                const double* iw = A.geo.invWJ + g0 + (eli * N3 + zl);
#pragma unroll
                for (int a = 0; a < N; ++a) zw[j][a] = iw[a * N2];
            }
        }
    };
    fetch_epilogue();
    __syncthreads();   // all LDS line reads are done; the LDS becomes the accumulator

    // ---- 4. every line thread stores its residual, weighted by the
    //         tangential quadrature weights, in its direction's slot (one
    //         store per value, no read-modify-write)
    double* lr = lds;
    if (active) {
        const double wperp = A.ops.w[l % N] * A.ops.w[l / N];
        double* x = lr + el * EBLK + dir * SLOT;
#pragma unroll
        for (int s = 0; s < 5; ++s)
#pragma unroll
            for (int a = 0; a < N; ++a) x[s * SPN + pbase + a * pstride] = R[s][a] * wperp;
    }
    __syncthreads();
    // residual of (element, state, node): the three directions summed in a fixed order
    auto rsum = [&](int eli, int s, int node) {
        const double* x = lr + eli * EBLK + s * SPN + pad_node<N>(node);
        return (x[0] + x[SLOT]) + x[2 * SLOT];
    };

    // ---- 5. source, mass inverse, RK combination (node-parallel)
    double dt = 0.0, cstage = 0.0;
    if (mode >= MODE_RK1) {
        dt = *A.dt;
        cstage = (mode == MODE_RK1) ? 0.0 : (mode == MODE_RK4 ? 1.0 : 0.5);
    }
    if (A.source) {
        const double t = (A.tdev ? *A.tdev : A.t) + cstage * dt;
        for (int idx = tid; idx < nwg; idx += nth) {
            const int eli = idx / N3, node = idx - eli * N3;
            double qs[5];
            const double* X = A.geo.X + g0 + idx;
            mms_source(X[0], X[SE], X[2 * SE], t, A.gamma, qs);
            const double wj = 1.0 / A.geo.invWJ[g0 + idx];
            double* x = lr + eli * EBLK + pad_node<N>(node);   // slot 0
#pragma unroll
            for (int s = 0; s < 5; ++s) x[s * SPN] -= wj * qs[s];
        }
        __syncthreads();
    }
    if (mode == MODE_RESIDUAL) {
        for (int idx = tid; idx < nwg; idx += nth) {
            const int eli = idx / N3, node = idx - eli * N3;
#pragma unroll
            for (int s = 0; s < 5; ++s) A.out[s * SE + g0 + idx] = rsum(eli, s, node);
        }
        return;
    }
    if (CWA) {
        plane_pass<N, SPN, EBLK, true>(lr, epb, A.ops.pia, A.ops.pib);   // sum of the slots, P^T along xi, eta
        __syncthreads();
        zeta_pass<N, SPN, EBLK>(lr, epb, zw, A.ops.pia, A.ops.pib);   // P^T, 1/(W J), P along zeta
        __syncthreads();
        plane_pass<N, SPN, EBLK, false>(lr, epb, A.ops.pib, A.ops.pia);   // P along xi, eta
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < KP; ++j) {
        const int idx = tid + j * nth;
        const int eli = idx / N3, node = idx - eli * N3;
        if (idx >= nwg) continue;
        const int64_t g = g0 + idx;
#pragma unroll
        for (int s = 0; s < 5; ++s) {
            const double k = CWA ? -lr[eli * EBLK + s * SPN + pad_node<N>(node)] : -(rsum(eli, s, node) * pf_iw[j]);
            const int64_t gi = s * SE + g;
            switch (mode) {
                case MODE_RHS: A.out[gi] = k; break;
                case MODE_RK1: {
                    const double u = pf_a[j][s];
                    A.acc[gi] = __builtin_fma(dt / 6.0, k, u);
                    A.out[gi] = __builtin_fma(0.5 * dt, k, u);
                } break;
                case MODE_RK2: {
                    A.acc[gi] = __builtin_fma(dt / 3.0, k, pf_a[j][s]);
                    A.out[gi] = __builtin_fma(0.5 * dt, k, pf_b[j][s]);
                } break;
                case MODE_RK3: {
                    A.acc[gi] = __builtin_fma(dt / 3.0, k, pf_a[j][s]);
                    A.out[gi] = __builtin_fma(dt, k, pf_b[j][s]);
                } break;
                default: A.out[gi] = __builtin_fma(dt / 6.0, k, pf_a[j][s]); break;
            }
        }
    }
}

// threads per element of the stage kernel: one per line
__host__ __device__ constexpr int stage_threads_per_elem(int n) { return 3 * n * n; }

// Minimum waves per SIMD the register allocation must allow: at p = 3 the
// cap of 168 VGPRs (3 waves) holds the kernel without spill and is faster
// than the uncapped allocation (2 waves); at p = 4, 5 the same cap spills
// (192 B per lane at p = 4) and is about 1.5x slower.
__host__ __device__ constexpr int stage_min_waves(int p) { return p == 3 ? 3 : 1; }

template <int P, bool CWA, int VARIANT, int DISS>
__global__ __launch_bounds__(STAGE_BLOCK_MAX) __attribute__((amdgpu_waves_per_eu(stage_min_waves(P))))
void stage_kernel(StageArgs A) {
    extern __shared__ double lds[];
    const int g = xcd_remap(blockIdx.x, gridDim.x);
    stage_body<P, CWA, VARIANT, DISS>(A, (int64_t)g * A.epb, lds);
}

// Ensemble launch for one kind of flow (degree, c != 0, flux variant): one
// workgroup per work item (flow, first element) of the kind's slice of the
// work list, the flow's StageArgs read from the device table. The kernel is
// specialised like the single-flow one (block size, LDS and register budget
// of its own degree), so an ensemble step is one launch per kind present.
template <int P, bool CWA, int VARIANT>
__global__ __launch_bounds__(STAGE_BLOCK_MAX) __attribute__((amdgpu_waves_per_eu(stage_min_waves(P))))
void ensemble_kind_kernel(const StageArgs* __restrict__ table, const int2* __restrict__ items) {
    extern __shared__ double lds[];
    const int2 w = items[blockIdx.x];
    const int f = __builtin_amdgcn_readfirstlane(w.x);
    const int64_t e0 = __builtin_amdgcn_readfirstlane(w.y);
    stage_body<P, CWA, VARIANT, 0>(table[f], e0, lds);
}

template <int P, bool CWA, int V>
static hipError_t launch_kind_t(const StageArgs* table, const int2* items, int nitems, int epb, hipStream_t s) {
    constexpr int N = P + 1;
    const int threads = ((epb * stage_threads_per_elem(N) + 63) / 64) * 64;
    ensemble_kind_kernel<P, CWA, V><<<nitems, threads, stage_lds_bytes(P, epb), s>>>(table, items);
    return hipGetLastError();
}

static int stage_lds_doubles(int n) { return stage_lds_per_elem(n); }

size_t stage_lds_bytes(int p, int epb) { return (size_t)epb * stage_lds_doubles(p + 1) * sizeof(double); }

int max_epb(int p) {
    const int n = p + 1;
    const int by_threads = STAGE_BLOCK_MAX / stage_threads_per_elem(n);
    const int by_lds = (int)(65536 / (stage_lds_doubles(n) * sizeof(double)));
    return by_threads < by_lds ? by_threads : by_lds;
}

// Elements per workgroup when the configuration leaves the tile to the
// library: the fastest measured on the 16^3 and 32^3 warped TGV, never above
// max_epb.
int default_epb(int p) {
    int d;
    switch (p) {
        case 2: d = 2; break;
        case 3: d = 4; break;
        case 4: d = 3; break;
        default: d = 2; break;
    }
    const int m = max_epb(p);
    return d < m ? d : m;
}

template <int P, bool CWA, int V, int DISS>
static hipError_t launch_t(const StageArgs& a, hipStream_t s) {
    constexpr int N = P + 1;
    int threads = ((a.epb * stage_threads_per_elem(N) + 63) / 64) * 64;
    size_t lds = stage_lds_bytes(P, a.epb);
    unsigned blocks = (unsigned)((a.geo.E + a.epb - 1) / a.epb);
    stage_kernel<P, CWA, V, DISS><<<blocks, threads, lds, s>>>(a);
    return hipGetLastError();
}

// surface dissipation as a template parameter: the kernels without it keep
// the register budget of the pure entropy-conserving flux
template <int P, bool CWA, int V>
static hipError_t launch_d(const StageArgs& a, hipStream_t s) {
    switch (a.diss) {
        case 0: return launch_t<P, CWA, V, 0>(a, s);
        case 1: return launch_t<P, CWA, V, 1>(a, s);
        case 2: return launch_t<P, CWA, V, 2>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <int P>
static hipError_t launch_p(bool cwa, int v, const StageArgs& a, hipStream_t s) {
    if (cwa) return v ? launch_d<P, true, 1>(a, s) : launch_d<P, true, 0>(a, s);
    return v ? launch_d<P, false, 1>(a, s) : launch_d<P, false, 0>(a, s);
}

hipError_t launch_ensemble_kind(int kind, const StageArgs* table, const int2* items, int nitems, int epb,
                                hipStream_t s) {
    const int p = kind / 4 + 2;
    if (nitems < 1 || epb < 1 || epb > max_epb(p)) return hipErrorInvalidValue;
    switch (kind) {
#define NSFR_KIND(P, C, V) \
    case kind_code(P, C, V): return launch_kind_t<P, C, V>(table, items, nitems, epb, s);
        NSFR_KIND(2, false, 0) NSFR_KIND(2, false, 1) NSFR_KIND(2, true, 0) NSFR_KIND(2, true, 1)
        NSFR_KIND(3, false, 0) NSFR_KIND(3, false, 1) NSFR_KIND(3, true, 0) NSFR_KIND(3, true, 1)
        NSFR_KIND(4, false, 0) NSFR_KIND(4, false, 1) NSFR_KIND(4, true, 0) NSFR_KIND(4, true, 1)
        NSFR_KIND(5, false, 0) NSFR_KIND(5, false, 1) NSFR_KIND(5, true, 0) NSFR_KIND(5, true, 1)
#undef NSFR_KIND
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_stage(int p, bool cwa, int variant, const StageArgs& a, hipStream_t s) {
    if (a.epb < 1 || a.epb > max_epb(p)) return hipErrorInvalidValue;
    switch (p) {
        case 2: return launch_p<2>(cwa, variant, a, s);
        case 3: return launch_p<3>(cwa, variant, a, s);
        case 4: return launch_p<4>(cwa, variant, a, s);
        case 5: return launch_p<5>(cwa, variant, a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace nsfr
