// Host-side internals of libnsfr: context, operator tables, kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/nsfr.h"
#include "nsfr_device.h"

namespace nsfr {

struct HostOps {
    int p, n;
    double x[MAXN], w[MAXN], D[MAXN][MAXN], S1[MAXN][MAXN], d[MAXN];
    double pia[MAXN], pib[MAXN];
    double mu, alpha;
};

void build_ops(int p, double c, Ops& ops, HostOps& h);

// ---- uncollocated (Gauss-Legendre) quadrature
constexpr int MAXQ = 12;          // n + overintegration: NSFR up to n + 3, conservative DG up to 2 n
constexpr int MAX_OVERINT = 3;    // NSFR

// 1D operators of the Gauss-Legendre variant (row-major; n solution nodes on
// LGL, q quadrature points), copied to device memory once per context.
struct GLOps {
    int p, n, q;
    double xq[MAXQ], wq[MAXQ];
    double chi[MAXQ * MAXN];    // q x n: LGL Lagrange basis at the quadrature points
    double chid[MAXQ * MAXN];   // q x n: its derivative there
    double pi[MAXN * MAXQ];     // n x q: L2 projection M^-1 chi^T Wq
    double pit[MAXN * MAXQ];    // n x q: ESFR projection (M + K)^-1 chi^T Wq (Eq. Fr projection)
    double sqh[MAXQ * MAXQ];    // q x q: (Wq Dq - Dq^T Wq) / 2, exactly antisymmetric
    double tl[MAXQ], tr[MAXQ];  // flux basis (Lagrange on the quadrature points) at -1, +1
    double dq[MAXQ * MAXQ];     // q x q: derivative of the flux basis at the quadrature points
};

void build_gl_ops(int p, int q, double c, const HostOps& h, GLOps& g);

// Metric terms at the quadrature points.
struct GLGeo {
    const double* Cq;     // [3 dir][3 comp][E][pos * q^2 + line]: column dir of C, line-major
    const double* Cf;     // [3 dir][2 side][3 comp][E][q^2]: column dir of C on the faces normal to dir
                          // (face point t1 + q t2, tangential directions in increasing order)
    const double* invWJ;  // [E][q^3]
    const double* Xq;     // [3][E][q^3]
};

struct GLArgs {
    const GLOps* ops;     // device copy
    GLGeo geo;
    double* vhat;         // [5][E][n^3]: projected entropy variables (written by the projection kernel)
    double* ft;           // [3 dir][2 side][5][E][q^2]: their values at the face points
};


// Geometry of one mesh as the kernels see it.
struct Geo {
    int nx, ny, nz;
    int64_t E;
    const double* Cline;   // [3 dir][3 comp][E][n (position along line)][n^2 (line)]
    const double* invWJ;   // [E][n^3]
    const double* X;       // [3][E][n^3]
    const int* nbr;        // [6][E]: periodic neighbour across face (dir, side), at dir * 2 + (side > 0)
};

enum StageMode : int {
    MODE_RESIDUAL = 0,   // out = R
    MODE_RHS = 1,        // out = -A R
    MODE_RK1 = 2,        // acc = Uin + dt/6 k, out = Uin + dt/2 k
    MODE_RK2 = 3,        // acc += dt/3 k,      out = Un + dt/2 k
    MODE_RK3 = 4,        // acc += dt/3 k,      out = Un + dt k
    MODE_RK4 = 5         // out = acc + dt/6 k
};

struct StageArgs {
    const double* Uin;
    const double* Un;
    double* acc;
    double* out;
    const double* dt;      // device scalar (RK modes)
    const double* tdev;    // device time, or null to use t
    double t;
    Geo geo;
    Ops ops;
    double gamma, c1;      // c1 = 1 / (2 (gamma - 1))
    int epb;               // elements per workgroup
    int mode;
    int diss, source;
};

struct FlowDesc;   // ensemble (ensemble.hip)

// launchers (each returns hipSuccess or the launch error)
hipError_t launch_geometry(int p, const Ops& ops, int nx, int ny, int nz, double lo, double hi, double beta,
                           double l, double* X, double* Cline, double* invWJ, double* J, hipStream_t s);
hipError_t launch_stage(int p, bool cwa, int variant, const StageArgs& a, hipStream_t s);
// exact inverse of the FR-modified mass (exact_mass.hip): L [E][n^3][n^3]
size_t exact_mass_doubles(int p, int64_t E);
hipError_t launch_exact_mass_factor(int p, int64_t E, const double* invWJ, const double* d, double c, double* L,
                                    int* fail, hipStream_t s);
hipError_t launch_exact_mass_solve(int p, int64_t E, const double* L, const double* R, double* out, hipStream_t s);
int default_epb(int p);
size_t stage_lds_bytes(int p, int epb);
int max_epb(int p);
hipError_t launch_geometry_export(int p, int64_t E, const double* Cline, double* C, hipStream_t s);
hipError_t launch_max_wavespeed(int64_t nnodes, const double* U, double gamma, double* partial, int nblk,
                                double* lam, hipStream_t s);
hipError_t launch_cfl_dt(const double* lam, double cfl, double dx, double* dt, hipStream_t s);
// V: entropy variables to pair with R, or null to evaluate v(U) at the nodes
hipError_t launch_diagnostics(int64_t nnodes, const double* U, const double* V, const double* R, double gamma,
                              double* partial, int nblk, double* out, hipStream_t s);
hipError_t launch_kinetic_energy(int64_t nn, const double* U, const double* invWJ, double* partial, int nblk,
                                 double* ke, double* grad, hipStream_t s);
hipError_t launch_check_state(int64_t nnodes, const double* U, double gamma, int32_t* count, hipStream_t s);
hipError_t launch_advance_time(double* t, const double* dt, hipStream_t s);
hipError_t launch_vjp(int p, bool cwa, int variant, const StageArgs& a, const double* lam, double* g,
                      double* mu_ws, hipStream_t s);

hipError_t launch_lincomb(int64_t n, double* out, const double* z, double ca, double cb, const double* x, double da,
                          double db, const double* dt, int accumulate, hipStream_t s);

void set_error(const std::string& msg);

// kernel variant code used by the ensemble dispatcher
constexpr int kind_code(int p, bool cwa, int variant) { return (p - 2) * 4 + (cwa ? 2 : 0) + variant; }
StageArgs ctx_stage_args(const nsfr_ctx* c);
int ctx_kind(const nsfr_ctx* c);
int64_t ctx_state_size(const nsfr_ctx* c);
// one stage of every ensemble flow of one kind: one workgroup per work item
hipError_t launch_ensemble_kind(int kind, const StageArgs* table, const int2* items, int nitems, int epb,
                                hipStream_t s);

// Gauss-Legendre variant (gl.hip): p = 2..5 with q = p + 1 .. p + 4 points
// (NSFR) or q = p + 1 .. 2 (p + 1) points (conservative DG, dg = true)
hipError_t launch_gl_geometry(int p, int q, const GLOps* ops, int64_t E, const double* X, const double* Cline,
                              double* Cq, double* Cf, double* invWJ, double* Xq, hipStream_t s);
// the projection (NSFR) or face-trace (DG) kernel, then the stage kernel
// (one element per workgroup)
// (one element per workgroup for NSFR, a.epb elements for DG)
hipError_t launch_gl_stage(bool dg, int p, int q, int variant, const StageArgs& a, const GLArgs& g, hipStream_t s);
size_t gl_lds_bytes(bool dg, int p, int q, int epb);   // dynamic LDS of the larger of the two kernels
int gl_max_epb(bool dg, int p, int q, size_t lds_max);  // largest elements per workgroup (0: none fits)
int gl_default_epb(bool dg, int p, int q, int64_t E);
hipError_t gl_prepare(bool dg, int p, int q, size_t bytes);  // allow that much dynamic LDS (current device)

}  // namespace nsfr
