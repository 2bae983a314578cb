/*
 * nsfr.h -- C ABI of libnsfr, the MI355X (gfx950) implementation of the
 * right-hand side of the nonlinearly stable flux reconstruction (NSFR) scheme
 * for 3D compressible Euler on curvilinear hexahedra (Cicchino & Nadarajah,
 * arXiv 2312.07725).
 *
 * Discretisation (all FP64):
 *   - solution, volume and surface quadrature on the p+1 Legendre-Gauss-Lobatto
 *     (LGL) nodes per direction, nodal Lagrange basis (Sec. 2.2; Sec. 7 opening
 *     paragraph);
 *   - volume term: entropy-conserving two-point flux differencing, the
 *     Hadamard product of the hybridised skew-symmetric operator with the
 *     metric-split reference two-point flux (Eq. NSFR), evaluated line by
 *     line (Sec. 5, sum-factorised Hadamard product);
 *   - surface term: the same two-point flux (optionally plus local
 *     Lax-Friedrichs or entropy-stable Roe-type matrix dissipation) at shared
 *     face nodes, lifted by the
 *     FR-modified mass (Eq. NSFR, last term; Sec. 3.2);
 *   - mass: weight-adjusted inverse Pi~ (W J)^-1 Pi~^T of the FR-modified mass
 *     (Eq. weight-adj ESFR mass, Eq. Fr projection); optionally (config mass
 *     = 1, nsfr_rhs only) the exact inverse of M_m + K_m (Eq. Km), factorised
 *     per element at nsfr_create, for checking the weight-adjusted one;
 *   - time: four-stage fourth-order RK, read as classical RK4 (Sec. 7, opening
 *     paragraph).
 *
 * Data layout. Every state-sized array is contiguous FP64 device memory of
 * 5 * E * (p+1)^3 doubles in the order [state][element][k][j][i], i (xi)
 * fastest; state = (rho, rho u, rho v, rho w, rho e); element
 * e = ex + nx * (ey + ny * ez). Arrays must be 8-byte aligned.
 *
 * Ownership. The caller allocates and owns every array passed in. The library
 * owns what it allocates in nsfr_create (operators, metrics, a residual-sized
 * workspace; with mass = 1 the per-element mass factors) and frees it in
 * nsfr_destroy. nsfr_rhs, nsfr_residual,
 * nsfr_rk4_step, nsfr_rk4_run and nsfr_rhs_vjp allocate nothing.
 *
 * Streams. All work is enqueued asynchronously on the context's HIP stream
 * (nsfr_create / nsfr_set_stream); only nsfr_check_state and the ensemble
 * constructors synchronise. A context is used by one host thread at a time.
 *
 * Errors. Every call returns an nsfr_status; no exception crosses the ABI.
 * Arguments are validated before any launch. nsfr_last_error() returns a
 * thread-local description of the most recent failure.
 */
#ifndef NSFR_H
#define NSFR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NSFR_OK = 0,
    NSFR_EINVAL = -1,        /* bad argument or configuration                 */
    NSFR_ENOMEM = -2,        /* device allocation failed                      */
    NSFR_EHIP = -3,          /* a HIP runtime call or kernel launch failed    */
    NSFR_EUNPHYSICAL = -4,   /* non-positive density or pressure, or NaN      */
    NSFR_ENOTSUP = -5        /* valid request the library does not implement  */
} nsfr_status;

typedef struct {
    int32_t p;            /* polynomial degree, 2..5 (n = p+1 LGL nodes per direction)   */
    int32_t ne[3];        /* elements per direction of the periodic box, each >= 1       */
    double lo, hi;        /* box [lo, hi]^3 (TGV: [0, 2 pi]; MMS: [-1, 1])               */
    double warp_beta;     /* amplitude of the nonsymmetric warp, Eq. warped grid         */
    double warp_l;        /* warp length l; <= 0 selects (hi - lo) / (2 pi)              */
    double gamma;         /* ratio of specific heats (1.4)                               */
    double c_fr;          /* FR parameter c in the convention of Eq. Km (1D K = 2c d d^T) */
    int32_t flux;         /* 0: Chandrashekar flux with Ranocha's pressure fix (arithmetic
                             mean pressure); 1: plain Chandrashekar flux                 */
    int32_t surface_diss; /* 0: entropy-conserving surface flux; 1: plus local
                             Lax-Friedrichs dissipation on the conservative jump; 2: plus
                             the entropy-stable Roe-type matrix dissipation on the jump
                             of the entropy variables (Sec. 6.3, Sec. 7.1)               */
    int32_t source;       /* 0: none; 1: manufactured-solution source of Sec. 7.1        */
    int32_t tile;         /* elements per workgroup of the stage kernel, 3 (p+1)^2 threads
                             (one per line) each, within 512 threads and 64 KB of LDS
                             (p = 2..5: at most 14, 6, 3, 2); 0 = tuned default. Must be
                             0 with quad = 1                                            */
    int32_t quad;         /* volume and surface quadrature (Sec. 3.3, Sec. 7 opening
                             paragraph): 0 = the LGL nodes themselves (collocated NSFR);
                             1 = Gauss-Legendre with p + 1 + overint points per direction,
                             the solution still stored as values at the LGL nodes, with the
                             entropy projection u~ = u(chi Pi v(chi u)) feeding the
                             two-point fluxes of the hybridised operator                 */
    int32_t overint;      /* extra quadrature points per direction (overintegration):
                             0..3 for NSFR, 0..p+1 for DG (p + 1 extra points give the
                             2 (p + 1)-point rule of the paper's overintegrated DG);
                             must be 0 with quad = 0                                     */
    int32_t scheme;       /* 0: NSFR (Eq. NSFR); 1: conservative DG in strong form (Sec.
                             3.1 Eq. cons DG strong) with Roe's surface flux, the
                             baseline of Sec. 7.4: u interpolated to the points (no
                             entropy projection), the contravariant flux C^T f(u)
                             differentiated in the flux basis, N . f* - n . phi_f f^r on
                             the faces, the same weight-adjusted inverse. Needs quad = 1
                             and surface_diss = 0; flux is ignored                       */
    int32_t mass;         /* inverse of the FR-modified mass M_m + K_m (Eq. Km): 0 = the
                             weight-adjusted approximation of Sec. 4 (Eq. weight-adj ESFR
                             mass; the fast path); 1 = the exact inverse, for checking
                             the approximation: the dense (p+1)^3 x (p+1)^3 matrix of
                             every element is assembled and Cholesky-factorised at
                             nsfr_create ((p+1)^6 doubles per element of device memory;
                             NSFR_ENOMEM if that does not fit, NSFR_EUNPHYSICAL if a
                             matrix is not positive definite) and nsfr_rhs applies it by
                             two triangular solves. Needs quad = 0; nsfr_rk4_step,
                             nsfr_rk4_step_static, nsfr_rk4_run, nsfr_rhs_vjp,
                             nsfr_rk4_step_vjp and ensembles return NSFR_ENOTSUP       */
} nsfr_config;

typedef struct nsfr_ctx nsfr_ctx;

/* Create a context on the current HIP device: builds the 1D LGL operators on
 * the host, the warped mesh, conservative-curl metric terms (Sec. 2.2, Eq. GCL)
 * and 1/(W J) on the device, and allocates the workspace. With quad = 1 it
 * also builds the Gauss-Legendre operators (basis at the points, L2 and ESFR
 * projections, flux-basis operator and end values) and evaluates the
 * cofactors, x and 1/(W J) at the volume points and the cofactors at the face
 * points (the LGL-grid polynomials, so the discrete GCL holds there too).
 * hip_stream may be NULL (default stream). Errors: NSFR_EINVAL (p outside
 * 2..5, ne < 1, hi <= lo, gamma <= 1, flux/surface_diss/source/quad/overint/
 * scheme out of range, negative tile, tile with quad = 1, overint with
 * quad = 0, DG with quad = 0 or surface_diss != 0),
 * NSFR_ENOTSUP if the Gauss-Legendre kernels need more LDS per workgroup than
 * the device allows, NSFR_ENOMEM, NSFR_EHIP, NSFR_EUNPHYSICAL if some node or
 * quadrature point has J <= 0. */
nsfr_status nsfr_create(const nsfr_config* cfg, void* hip_stream, nsfr_ctx** out);
nsfr_status nsfr_destroy(nsfr_ctx* ctx);
nsfr_status nsfr_set_stream(nsfr_ctx* ctx, void* hip_stream);

/* Number of elements and nodes per element ((p+1)^3). Host pointers. */
nsfr_status nsfr_sizes(const nsfr_ctx* ctx, int64_t* n_elem, int64_t* n_node_per_elem);

/* Physical node coordinates, device array [3][E][(p+1)^3] (Eq. warped grid at
 * the LGL nodes). */
nsfr_status nsfr_node_coords(nsfr_ctx* ctx, double* xyz);

/* Metric cofactor matrix and Jacobian at the nodes (Sec. 2.2): C is a device
 * array [3][3][E][(p+1)^3] with C[n][i] = (J a^i)_n, J is [E][(p+1)^3]. */
nsfr_status nsfr_geometry(nsfr_ctx* ctx, double* C, double* J);

/* Pre-mass residual R = R_vol + R_surf - W J q(t) of Eq. NSFR, so that
 * (M_m + K_m) dU/dt = -R. U and R are state-sized device arrays (R may not
 * alias U). t is used only by the manufactured source. */
nsfr_status nsfr_residual(nsfr_ctx* ctx, const double* U, double* R, double t);

/* dU/dt = -Pi~ (W J)^-1 Pi~^T R(U, t) (Eq. weight-adj ESFR mass). dUdt may not
 * alias U. */
nsfr_status nsfr_rhs(nsfr_ctx* ctx, const double* U, double* dUdt, double t);

/* One classical RK4 step, in place on U, with the step size read from device
 * memory dt_dev (one double) so that the launch sequence is static. work is a
 * caller-owned device array of 3 state-sized arrays (15 * E * (p+1)^3
 * doubles). t is the time at the start of the step (source only). */
nsfr_status nsfr_rk4_step(nsfr_ctx* ctx, double* U, const double* dt_dev, double t, double* work);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the RK4
 * step of nsfr_rk4_step without the work argument. Its three stage arrays
 * live in a workspace compiled into the library, NSFR_STATIC_MAX_NODES nodes
 * (120 MiB) per GPU, held by each GPU the library runs on until the process
 * ends; meshes with more than NSFR_STATIC_MAX_NODES nodes (E (p+1)^3) are
 * rejected with NSFR_EINVAL before any launch. The call allocates nothing.
 * Every call on one GPU shares that workspace: calls that overlap on one GPU
 * (other streams, other contexts, other threads) race and must be ordered by
 * the caller. Nothing in the workspace needs to start at zero (each stage
 * writes every value it later reads). */
#define NSFR_STATIC_MAX_NODES (1 << 20)
nsfr_status nsfr_rk4_step_static(nsfr_ctx* ctx, double* U, const double* dt_dev, double t);

/* nsteps RK4 steps replayed from a HIP graph of one step (the four stage
 * kernels). The time is read from and advanced in device memory t_dev (one
 * double) by dt each step; t_dev may be NULL when the configuration has no
 * source term (then the graph holds the stage kernels only). The graph is
 * built on first use for a given (U, dt_dev, t_dev, work) and kept in the
 * context. */
nsfr_status nsfr_rk4_run(nsfr_ctx* ctx, double* U, const double* dt_dev, double* t_dev,
                         int32_t nsteps, double* work);

/* lam_dev[0] = max over nodes of |u| + sqrt(gamma p / rho): the maximum wave
 * speed on which Sec. 7 (opening paragraph) bases its adaptive time step.
 * U is a state-sized device array; lam_dev is one device double. */
nsfr_status nsfr_max_wavespeed(nsfr_ctx* ctx, const double* U, double* lam_dev);

/* dt_dev[0] = cfl * (hi - lo) / (ne[0] (p+1)) / (max wave speed): the adaptive
 * step of Sec. 7 (opening paragraph), CFL = cfl, dx the mean node spacing. */
nsfr_status nsfr_cfl_dt(nsfr_ctx* ctx, const double* U, double cfl, double* dt_dev);

/* Vector-Jacobian product g = (d(dU/dt)/dU)^T lam of nsfr_rhs at (U, t),
 * including the Jacobians of the two-point volume and surface fluxes. The
 * weight-adjusted inverse is symmetric, so g = -(dR/dU)^T (A lam). g may not
 * alias U or lam. Collocated scheme with the EC surface flux only
 * (quad = 0, surface_diss = 0), else NSFR_ENOTSUP; the same for
 * nsfr_rk4_step_vjp. */
nsfr_status nsfr_rhs_vjp(nsfr_ctx* ctx, const double* U, const double* lam, double* g, double t);

/* Discrete adjoint of one RK4 step: given U^n, the step size and
 * lam_next = dJ/dU^{n+1}, writes lam = dJ/dU^n (may alias lam_next). work is
 * a caller-owned device array of 6 state-sized arrays. */
nsfr_status nsfr_rk4_step_vjp(nsfr_ctx* ctx, const double* U, const double* dt_dev, double t,
                              const double* lam_next, double* lam, double* work);

/* Diagnostics of R(U, t) (Sec. 6.2, 6.3, 7.3) into device array out (8 doubles):
 * [sum v.R, sum |v.R|, sum R_rho, sum R_mx, sum R_my, sum R_mz, sum R_E, max |R|],
 * v the entropy variables at the nodes (quad = 0) or the projected entropy
 * variables v^ = Pi v(chi u) (quad = 1, the variables whose product with R
 * vanishes, Sec. 6.3). Uses the library workspace. */
nsfr_status nsfr_diagnostics(nsfr_ctx* ctx, const double* U, double t, double* out);

/* Kinetic energy J_KE = sum over nodes of W J rho |u|^2 / 2 into ke_dev[0]
 * (device), and, if grad is not NULL, its gradient dJ_KE/dU (state-sized
 * device array): W J [-|u|^2/2, u, v, w, 0]. The objective of the
 * time-integrated sensitivity. Collocated scheme only (quad = 0, else
 * NSFR_ENOTSUP). */
nsfr_status nsfr_kinetic_energy(nsfr_ctx* ctx, const double* U, double* ke_dev, double* grad);

/* Synchronising state check: *bad_host = number of nodes with rho <= 0,
 * p <= 0 or a NaN; returns NSFR_EUNPHYSICAL if that number is positive. */
nsfr_status nsfr_check_state(nsfr_ctx* ctx, const double* U, int32_t* bad_host);

/* ---- ensembles of independent flows: per RK stage one launch per kind of
 * flow present (degree, c != 0, flux variant), each specialised like the
 * single-flow stage kernel --------------------------------------------- */
typedef struct nsfr_ens nsfr_ens;

/* n_flows configurations (any mix of p, ne, c and flux; surface_diss,
 * source and quad must be 0, else NSFR_ENOTSUP). The packed state is the
 * concatenation of the flows' state arrays; offsets (in doubles) are
 * returned by nsfr_ens_offsets (n_flows + 1 entries, host). */
nsfr_status nsfr_ens_create(const nsfr_config* cfgs, int32_t n_flows, void* hip_stream, nsfr_ens** out);
nsfr_status nsfr_ens_destroy(nsfr_ens* ens);
/* Stream (a hipStream_t, or null for the default stream) on which the
 * ensemble's later calls enqueue their work. */
nsfr_status nsfr_ens_set_stream(nsfr_ens* ens, void* hip_stream);
nsfr_status nsfr_ens_offsets(const nsfr_ens* ens, int64_t* offsets_host);
/* Right-hand side of every flow at time t (one launch per kind). */
nsfr_status nsfr_ens_rhs(nsfr_ens* ens, const double* U, double* dUdt, double t);
/* One RK4 step of every flow, in place; dt_dev holds one step size per flow;
 * work holds 3 packed-state-sized arrays. Four stages, each one launch per
 * kind. */
nsfr_status nsfr_ens_rk4_step(nsfr_ens* ens, double* U, const double* dt_dev, double t, double* work);
/* nsteps steps replayed from a HIP graph of one ensemble step. */
nsfr_status nsfr_ens_rk4_run(nsfr_ens* ens, double* U, const double* dt_dev, double t,
                             int32_t nsteps, double* work);
/* Elements per work item for degree p (2..5) used by the ensemble kernels
 * (the same bounds as the config's tile); epb = 0 restores the default. */
nsfr_status nsfr_ens_set_tile(nsfr_ens* ens, int32_t p, int32_t epb);

/* FR parameter c_HU (convention of Eq. Km) for degree p (2..5): the value for
 * which the FR-modified 1D mass of the exactly integrated Lagrange basis on
 * LGL nodes equals the collocated LGL mass (Sec. 7.2). c_HU = E_p / (2 (p!)^2)
 * with E_p the LGL quadrature error of x^(2p). Host output. */
nsfr_status nsfr_c_hu(int32_t p, double* c_out);

const char* nsfr_status_string(nsfr_status s);
const char* nsfr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* NSFR_H */
