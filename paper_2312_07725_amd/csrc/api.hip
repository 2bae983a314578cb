// C ABI of libnsfr: argument validation, context lifetime, launch sequences.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "nsfr_host.h"

using namespace nsfr;

namespace nsfr {
static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
}  // namespace nsfr

struct nsfr_ctx {
    nsfr_config cfg;
    int dev = 0;
    hipStream_t stream = nullptr;
    int p = 0, n = 0, n3 = 0;
    int64_t E = 0;
    HostOps hops;
    Ops ops;
    double* X = nullptr;       // [3][E][n3]
    double* Cline = nullptr;   // [3][3][E][n3] line-major per direction
    int* nbr = nullptr;        // [6][E] face neighbours
    double* invWJ = nullptr;   // [E][n3]
    double* J = nullptr;       // [E][n3]
    double* wsR = nullptr;     // state-sized workspace
    double* wsR2 = nullptr;    // state-sized workspace (adjoint)
    double* red = nullptr;     // reduction partials
    int nred = 0;
    int32_t* cnt = nullptr;    // check_state counters (64)
    int epb = 0;
    // Gauss-Legendre variant (cfg.quad = 1): q points per direction
    int q = 0;
    GLOps* glops = nullptr;    // device copy of the 1D operators
    double* Cq = nullptr;      // [3][3][E][q^3] cofactors at the volume points, line-major
    double* Cf = nullptr;      // [6][3][E][q^2] cofactor column at the face points
    double* invWJq = nullptr;  // [E][q^3]
    double* Xq = nullptr;      // [3][E][q^3]
    double* vhat = nullptr;    // [5][E][n^3] projected entropy variables of the last stage's input
    double* ft = nullptr;      // [6][5][E][q^2] their face values
    // exact mass inverse (cfg.mass = 1): Cholesky factor of M_m + K_m per element
    double* Lmass = nullptr;   // [E][n^3][n^3], lower triangle
    // graph cache for nsfr_rk4_run
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    const void* gkey[4] = {nullptr, nullptr, nullptr, nullptr};
};

#define HIP_TRY(call)                                                                         \
    do {                                                                                      \
        hipError_t _e = (call);                                                               \
        if (_e != hipSuccess) {                                                               \
            set_error(std::string(#call) + ": " + hipGetErrorString(_e));                     \
            return NSFR_EHIP;                                                                 \
        }                                                                                     \
    } while (0)

static nsfr_status bad(const std::string& msg) {
    set_error(msg);
    return NSFR_EINVAL;
}

static nsfr_status validate(const nsfr_config* c) {
    if (!c) return bad("null config");
    if (c->p < 2 || c->p > 5) return bad("p must be in 2..5");
    for (int i = 0; i < 3; ++i)
        if (c->ne[i] < 1) return bad("ne must be >= 1 in every direction");
    if ((int64_t)c->ne[0] * c->ne[1] * c->ne[2] > (int64_t)1 << 31) return bad("too many elements");
    if (!(c->hi > c->lo)) return bad("hi must exceed lo");
    if (!(c->gamma > 1.0)) return bad("gamma must exceed 1");
    if (!(c->c_fr >= 0.0) || !std::isfinite(c->c_fr)) return bad("c_fr must be finite and >= 0");
    if (!std::isfinite(c->warp_beta)) return bad("warp_beta must be finite");
    if (c->flux < 0 || c->flux > 1) return bad("flux must be 0 or 1");
    if (c->surface_diss < 0 || c->surface_diss > 2) return bad("surface_diss must be 0, 1 or 2");
    if (c->source < 0 || c->source > 1) return bad("source must be 0 or 1");
    if (c->tile < 0 || (c->quad == 0 && c->tile > max_epb(c->p))) return bad("tile out of range for this p");
    if (c->quad < 0 || c->quad > 1) return bad("quad must be 0 (LGL collocated) or 1 (Gauss-Legendre)");
    if (c->scheme < 0 || c->scheme > 1) return bad("scheme must be 0 (NSFR) or 1 (conservative DG)");
    if (c->scheme == 1 && c->quad != 1) return bad("conservative DG runs on the Gauss-Legendre rule (quad = 1)");
    if (c->scheme == 1 && c->surface_diss != 0)
        return bad("conservative DG uses Roe's surface flux; surface_diss must be 0");
    const int omax = c->scheme == 1 ? c->p + 1 : MAX_OVERINT;
    if (c->overint < 0 || c->overint > omax)
        return bad("overint must be in 0.." + std::to_string(omax) + (c->scheme == 1 ? " for DG" : " for NSFR"));
    if (c->quad == 0 && c->overint != 0) return bad("overintegration needs the Gauss-Legendre rule (quad = 1)");
    if (c->quad == 1 && c->scheme == 0 && c->tile > 1)
        return bad("the NSFR Gauss-Legendre kernel runs one element per workgroup (tile must be 0 or 1)");
    if (c->mass < 0 || c->mass > 1) return bad("mass must be 0 (weight-adjusted) or 1 (exact inverse)");
    if (c->mass == 1 && c->quad != 0) return bad("the exact mass inverse is built for the collocated scheme (quad = 0)");
    return NSFR_OK;
}

static nsfr_status use_device(const nsfr_ctx* c) {
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != c->dev) HIP_TRY(hipSetDevice(c->dev));
    return NSFR_OK;
}

static bool aligned(const void* p) { return p && ((uintptr_t)p % 8 == 0); }

static void free_ctx(nsfr_ctx* c) {
    if (!c) return;
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    double* bufs[] = {c->X, c->Cline, c->invWJ, c->J, c->wsR, c->wsR2, c->red,
                      c->Cq, c->Cf, c->invWJq, c->Xq, c->vhat, c->ft, c->Lmass};
    for (double* b : bufs)
        if (b) (void)hipFree(b);
    if (c->cnt) (void)hipFree(c->cnt);
    if (c->nbr) (void)hipFree(c->nbr);
    if (c->glops) (void)hipFree(c->glops);
    delete c;
}

static StageArgs base_args(const nsfr_ctx* c) {
    StageArgs a;
    std::memset(&a, 0, sizeof(a));
    a.geo.nx = c->cfg.ne[0];
    a.geo.ny = c->cfg.ne[1];
    a.geo.nz = c->cfg.ne[2];
    a.geo.E = c->E;
    a.geo.Cline = c->Cline;
    a.geo.invWJ = c->invWJ;
    a.geo.X = c->X;
    a.geo.nbr = c->nbr;
    a.ops = c->ops;
    a.gamma = c->cfg.gamma;
    a.c1 = 1.0 / (2.0 * (c->cfg.gamma - 1.0));
    a.epb = c->epb;
    a.diss = c->cfg.surface_diss;
    a.source = c->cfg.source;
    return a;
}

static GLArgs gl_args(const nsfr_ctx* c) {
    GLArgs g;
    g.ops = c->glops;
    g.geo.Cq = c->Cq;
    g.geo.Cf = c->Cf;
    g.geo.invWJ = c->invWJq;
    g.geo.Xq = c->Xq;
    g.vhat = c->vhat;
    g.ft = c->ft;
    return g;
}

static nsfr_status stage(nsfr_ctx* c, StageArgs& a) {
    hipError_t e = c->cfg.quad ? launch_gl_stage(c->cfg.scheme == 1, c->p, c->q, c->cfg.flux, a, gl_args(c), c->stream)
                               : launch_stage(c->p, c->cfg.c_fr != 0.0, c->cfg.flux, a, c->stream);
    if (e != hipSuccess) {
        set_error(std::string("stage kernel launch: ") + hipGetErrorString(e));
        return NSFR_EHIP;
    }
    return NSFR_OK;
}

// Workspace of nsfr_rk4_step_static: three state-sized arrays of up to
// NSFR_STATIC_MAX_NODES nodes, one copy per GPU (device global). Host code
// never uses the symbol itself: its device address is looked up once per
// device (with that device current) and kept in g_static_ws.
static __device__ __align__(256) double scratch[(size_t)15 * NSFR_STATIC_MAX_NODES];

static std::mutex g_static_mu;
static double* g_static_ws[64] = {};

static nsfr_status static_workspace(int dev, double** out) {
    if (dev < 0 || dev >= 64) return bad("device index out of range for the static workspace");
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ws[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string("hipGetSymbolAddress(static workspace): ") + hipGetErrorString(e));
            return NSFR_EHIP;
        }
        g_static_ws[dev] = static_cast<double*>(p);
    }
    *out = g_static_ws[dev];
    return NSFR_OK;
}

extern "C" {

const char* nsfr_status_string(nsfr_status s) {
    switch (s) {
        case NSFR_OK: return "ok";
        case NSFR_EINVAL: return "invalid argument";
        case NSFR_ENOMEM: return "out of device memory";
        case NSFR_EHIP: return "HIP runtime error";
        case NSFR_EUNPHYSICAL: return "unphysical state";
        case NSFR_ENOTSUP: return "not supported";
    }
    return "unknown status";
}

const char* nsfr_last_error(void) { return g_last_error.c_str(); }

// Gauss-Legendre operators, metric terms at the quadrature points and the
// projection buffers (the context's LGL geometry is already built).
// Dense M_m + K_m of every element and its Cholesky factor (cfg.mass = 1).
static nsfr_status exact_mass_setup(nsfr_ctx* c) {
    const size_t nd = exact_mass_doubles(c->p, c->E);
    if (hipMalloc((void**)&c->Lmass, nd * sizeof(double)) != hipSuccess) {
        set_error("hipMalloc failed for the exact mass factors (" + std::to_string(nd * sizeof(double)) + " bytes)");
        return NSFR_ENOMEM;
    }
    HIP_TRY(hipMemsetAsync(c->cnt, 0, sizeof(int32_t), c->stream));
    HIP_TRY(launch_exact_mass_factor(c->p, c->E, c->invWJ, c->hops.d, c->cfg.c_fr, c->Lmass, c->cnt, c->stream));
    int32_t fail = 0;
    HIP_TRY(hipMemcpyAsync(&fail, c->cnt, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (fail) {
        set_error("the FR-modified mass of an element is not positive definite");
        return NSFR_EUNPHYSICAL;
    }
    return NSFR_OK;
}

static nsfr_status exact_mass_unsupported(const nsfr_ctx* c, const char* what) {
    if (!c->cfg.mass) return NSFR_OK;
    set_error(std::string(what) + ": the exact mass inverse (mass = 1) is offered by nsfr_rhs only");
    return NSFR_ENOTSUP;
}

static nsfr_status gl_setup(nsfr_ctx* c) {
    const int q = c->n + c->cfg.overint;
    c->q = q;
    const bool dg = c->cfg.scheme == 1;
    int lds_max = 0;
    HIP_TRY(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, c->dev));
    const int emax = gl_max_epb(dg, c->p, q, (size_t)lds_max);
    if (c->cfg.tile > emax && emax > 0) {
        set_error("tile " + std::to_string(c->cfg.tile) + " exceeds the " + std::to_string(emax) +
                  " elements per workgroup that fit this device for this p and rule");
        return NSFR_EINVAL;
    }
    c->epb = c->cfg.tile ? c->cfg.tile : gl_default_epb(dg, c->p, q, c->E);
    const size_t need = gl_lds_bytes(dg, c->p, q, c->epb);
    if (need > (size_t)lds_max) {
        set_error(std::string(dg ? "DG" : "NSFR") + " Gauss-Legendre kernels for p = " + std::to_string(c->p) + ", " + std::to_string(q) +
                  " points need " + std::to_string(need) + " bytes of LDS per workgroup; the device allows " +
                  std::to_string(lds_max));
        return NSFR_ENOTSUP;
    }
    HIP_TRY(gl_prepare(dg, c->p, q, need));
    GLOps h;
    build_gl_ops(c->p, q, c->cfg.c_fr, c->hops, h);
    const size_t E = (size_t)c->E, q2 = (size_t)q * q, q3 = q2 * q;
    struct A { double** p; size_t n; } allocs[] = {
        {&c->Cq, 9 * E * q3}, {&c->Cf, 18 * E * q2}, {&c->invWJq, E * q3}, {&c->Xq, 3 * E * q3},
        {&c->vhat, 5 * E * c->n3}, {&c->ft, 30 * E * q2}};
    for (auto& al : allocs)
        if (hipMalloc((void**)al.p, al.n * sizeof(double)) != hipSuccess) {
            set_error("hipMalloc failed for the Gauss-Legendre arrays");
            return NSFR_ENOMEM;
        }
    if (hipMalloc((void**)&c->glops, sizeof(GLOps)) != hipSuccess) {
        set_error("hipMalloc failed for the Gauss-Legendre operators");
        return NSFR_ENOMEM;
    }
    HIP_TRY(hipMemcpy(c->glops, &h, sizeof(GLOps), hipMemcpyHostToDevice));
    HIP_TRY(launch_gl_geometry(c->p, q, c->glops, c->E, c->X, c->Cline, c->Cq, c->Cf, c->invWJq, c->Xq, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    std::vector<double> iw(E * q3);
    HIP_TRY(hipMemcpy(iw.data(), c->invWJq, iw.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (double v : iw)
        if (!(v > 0.0)) {
            set_error("the warped mesh has a quadrature point with J <= 0");
            return NSFR_EUNPHYSICAL;
        }
    return NSFR_OK;
}

nsfr_status nsfr_create(const nsfr_config* cfg, void* hip_stream, nsfr_ctx** out) {
    if (!out) return bad("null output pointer");
    *out = nullptr;
    nsfr_status st = validate(cfg);
    if (st != NSFR_OK) return st;
    nsfr_ctx* c = new nsfr_ctx();
    c->cfg = *cfg;
    c->stream = (hipStream_t)hip_stream;
    c->p = cfg->p;
    c->n = cfg->p + 1;
    c->n3 = c->n * c->n * c->n;
    c->E = (int64_t)cfg->ne[0] * cfg->ne[1] * cfg->ne[2];
    c->epb = cfg->tile ? cfg->tile : default_epb(cfg->p);
    build_ops(c->p, cfg->c_fr, c->ops, c->hops);
    hipError_t he = hipGetDevice(&c->dev);
    if (he != hipSuccess) {
        set_error(std::string("hipGetDevice: ") + hipGetErrorString(he));
        free_ctx(c);
        return NSFR_EHIP;
    }
    const size_t nodes = (size_t)c->E * c->n3;
    c->nred = 8 * 1024;
    struct A { double** p; size_t n; } allocs[] = {
        {&c->X, 3 * nodes}, {&c->Cline, 9 * nodes}, {&c->invWJ, nodes}, {&c->J, nodes},
        {&c->wsR, 5 * nodes}, {&c->wsR2, 5 * nodes}, {&c->red, (size_t)c->nred}};
    for (auto& al : allocs) {
        if (hipMalloc((void**)al.p, al.n * sizeof(double)) != hipSuccess) {
            set_error("hipMalloc failed for the context's device arrays");
            free_ctx(c);
            return NSFR_ENOMEM;
        }
    }
    {   // face-neighbour table of the structured periodic box
        const int nx = cfg->ne[0], ny = cfg->ne[1], nz = cfg->ne[2];
        std::vector<int> nb((size_t)6 * c->E);
        for (int ez = 0; ez < nz; ++ez)
            for (int ey = 0; ey < ny; ++ey)
                for (int ex = 0; ex < nx; ++ex) {
                    const size_t e = ex + (size_t)nx * (ey + (size_t)ny * ez);
                    const int xm = (ex + nx - 1) % nx, xp = (ex + 1) % nx;
                    const int ym = (ey + ny - 1) % ny, yp = (ey + 1) % ny;
                    const int zm = (ez + nz - 1) % nz, zp = (ez + 1) % nz;
                    nb[0 * c->E + e] = xm + nx * (ey + ny * ez);
                    nb[1 * c->E + e] = xp + nx * (ey + ny * ez);
                    nb[2 * c->E + e] = ex + nx * (ym + ny * ez);
                    nb[3 * c->E + e] = ex + nx * (yp + ny * ez);
                    nb[4 * c->E + e] = ex + nx * (ey + ny * zm);
                    nb[5 * c->E + e] = ex + nx * (ey + ny * zp);
                }
        if (hipMalloc((void**)&c->nbr, nb.size() * sizeof(int)) != hipSuccess ||
            hipMemcpy(c->nbr, nb.data(), nb.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
            set_error("allocation or copy of the face-neighbour table failed");
            free_ctx(c);
            return NSFR_ENOMEM;
        }
    }
    if (hipMalloc((void**)&c->cnt, 64 * sizeof(int32_t)) != hipSuccess) {
        set_error("hipMalloc failed for the state-check counters");
        free_ctx(c);
        return NSFR_ENOMEM;
    }
    double l = cfg->warp_l > 0 ? cfg->warp_l : (cfg->hi - cfg->lo) / (2.0 * M_PI);
    he = launch_geometry(c->p, c->ops, cfg->ne[0], cfg->ne[1], cfg->ne[2], cfg->lo, cfg->hi, cfg->warp_beta, l, c->X,
                         c->Cline, c->invWJ, c->J, c->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
    if (he != hipSuccess) {
        set_error(std::string("geometry setup: ") + hipGetErrorString(he));
        free_ctx(c);
        return NSFR_EHIP;
    }
    // every node must have a positive Jacobian
    std::vector<double> J(nodes);
    he = hipMemcpy(J.data(), c->J, nodes * sizeof(double), hipMemcpyDeviceToHost);
    if (he != hipSuccess) {
        set_error(std::string("geometry copy: ") + hipGetErrorString(he));
        free_ctx(c);
        return NSFR_EHIP;
    }
    for (double v : J)
        if (!(v > 0.0)) {
            set_error("the warped mesh has a node with J <= 0");
            free_ctx(c);
            return NSFR_EUNPHYSICAL;
        }
    if (cfg->mass) {
        st = exact_mass_setup(c);
        if (st != NSFR_OK) {
            free_ctx(c);
            return st;
        }
    }
    if (cfg->quad) {
        st = gl_setup(c);
        if (st != NSFR_OK) {
            free_ctx(c);
            return st;
        }
    }
    *out = c;
    return NSFR_OK;
}

nsfr_status nsfr_destroy(nsfr_ctx* c) {
    if (!c) return bad("null context");
    (void)use_device(c);
    free_ctx(c);
    return NSFR_OK;
}

nsfr_status nsfr_set_stream(nsfr_ctx* c, void* s) {
    if (!c) return bad("null context");
    c->stream = (hipStream_t)s;
    return NSFR_OK;
}

nsfr_status nsfr_sizes(const nsfr_ctx* c, int64_t* ne, int64_t* nn) {
    if (!c || !ne || !nn) return bad("null argument");
    *ne = c->E;
    *nn = c->n3;
    return NSFR_OK;
}

nsfr_status nsfr_node_coords(nsfr_ctx* c, double* xyz) {
    if (!c || !aligned(xyz)) return bad("null or misaligned argument");
    nsfr_status st = use_device(c);
    if (st) return st;
    HIP_TRY(hipMemcpyAsync(xyz, c->X, 3 * (size_t)c->E * c->n3 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    return NSFR_OK;
}

nsfr_status nsfr_geometry(nsfr_ctx* c, double* C, double* J) {
    if (!c || !aligned(C) || !aligned(J)) return bad("null or misaligned argument");
    nsfr_status st = use_device(c);
    if (st) return st;
    HIP_TRY(launch_geometry_export(c->p, c->E, c->Cline, C, c->stream));
    HIP_TRY(hipMemcpyAsync(J, c->J, (size_t)c->E * c->n3 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    return NSFR_OK;
}

nsfr_status nsfr_residual(nsfr_ctx* c, const double* U, double* R, double t) {
    if (!c || !aligned(U) || !aligned(R) || U == R) return bad("null, misaligned or aliased argument");
    nsfr_status st = use_device(c);
    if (st) return st;
    StageArgs a = base_args(c);
    a.Uin = U;
    a.out = R;
    a.t = t;
    a.mode = MODE_RESIDUAL;
    return stage(c, a);
}

nsfr_status nsfr_rhs(nsfr_ctx* c, const double* U, double* dUdt, double t) {
    if (!c || !aligned(U) || !aligned(dUdt) || U == dUdt) return bad("null, misaligned or aliased argument");
    nsfr_status st = use_device(c);
    if (st) return st;
    StageArgs a = base_args(c);
    a.Uin = U;
    a.out = dUdt;
    a.t = t;
    if (c->cfg.mass) {   // residual, then -(M_m + K_m)^-1 R
        a.out = c->wsR;
        a.mode = MODE_RESIDUAL;
        if ((st = stage(c, a))) return st;
        HIP_TRY(launch_exact_mass_solve(c->p, c->E, c->Lmass, c->wsR, dUdt, c->stream));
        return NSFR_OK;
    }
    a.mode = MODE_RHS;
    return stage(c, a);
}

static nsfr_status rk4_enqueue(nsfr_ctx* c, double* U, const double* dt, double t, const double* tdev, double* work) {
    const size_t ns = 5 * (size_t)c->E * c->n3;
    double* acc = work;
    double* Ya = work + ns;
    double* Yb = work + 2 * ns;
    StageArgs a = base_args(c);
    a.dt = dt;
    a.t = t;
    a.tdev = tdev;
    a.Un = U;
    a.acc = acc;
    nsfr_status st;
    a.mode = MODE_RK1; a.Uin = U;  a.out = Ya; if ((st = stage(c, a))) return st;
    a.mode = MODE_RK2; a.Uin = Ya; a.out = Yb; if ((st = stage(c, a))) return st;
    a.mode = MODE_RK3; a.Uin = Yb; a.out = Ya; if ((st = stage(c, a))) return st;
    a.mode = MODE_RK4; a.Uin = Ya; a.out = U;  return stage(c, a);
}

nsfr_status nsfr_rk4_step(nsfr_ctx* c, double* U, const double* dt, double t, double* work) {
    if (!c || !aligned(U) || !aligned(dt) || !aligned(work)) return bad("null or misaligned argument");
    if (exact_mass_unsupported(c, "nsfr_rk4_step")) return NSFR_ENOTSUP;
    nsfr_status st = use_device(c);
    if (st) return st;
    return rk4_enqueue(c, U, dt, t, nullptr, work);
}

nsfr_status nsfr_rk4_step_static(nsfr_ctx* c, double* U, const double* dt, double t) {
    if (!c || !aligned(U) || !aligned(dt)) return bad("null or misaligned argument");
    if (exact_mass_unsupported(c, "nsfr_rk4_step_static")) return NSFR_ENOTSUP;
    const int64_t nodes = c->E * (int64_t)c->n3;
    if (nodes > NSFR_STATIC_MAX_NODES)
        return bad("nsfr_rk4_step_static: the mesh has " + std::to_string(nodes) +
                   " nodes; the static workspace holds at most " + std::to_string(NSFR_STATIC_MAX_NODES));
    nsfr_status st = use_device(c);
    if (st) return st;
    double* ws = nullptr;
    if ((st = static_workspace(c->dev, &ws))) return st;
    return rk4_enqueue(c, U, dt, t, nullptr, ws);
}

nsfr_status nsfr_rk4_run(nsfr_ctx* c, double* U, const double* dt, double* tdev, int32_t nsteps, double* work) {
    if (!c || !aligned(U) || !aligned(dt) || (tdev && !aligned(tdev)) || !aligned(work) || nsteps < 0)
        return bad("null, misaligned or negative argument");
    if (!tdev && c->cfg.source) return bad("t_dev is required when the source term is enabled");
    if (exact_mass_unsupported(c, "nsfr_rk4_run")) return NSFR_ENOTSUP;
    nsfr_status st = use_device(c);
    if (st) return st;
    if (nsteps == 0) return NSFR_OK;
    const void* key[4] = {U, dt, tdev, work};
    if (!c->gexec || std::memcmp(key, c->gkey, sizeof(key)) != 0) {
        if (c->gexec) { (void)hipGraphExecDestroy(c->gexec); c->gexec = nullptr; }
        if (c->graph) { (void)hipGraphDestroy(c->graph); c->graph = nullptr; }
        hipStream_t cap;
        HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipStream_t saved = c->stream;
        c->stream = cap;
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        nsfr_status s2 = NSFR_OK;
        if (e == hipSuccess) {
            s2 = rk4_enqueue(c, U, dt, 0.0, tdev, work);
            if (s2 == NSFR_OK && tdev) {
                hipError_t e2 = launch_advance_time(tdev, dt, cap);
                if (e2 != hipSuccess) s2 = NSFR_EHIP;
            }
            hipError_t e3 = hipStreamEndCapture(cap, &c->graph);
            if (e3 != hipSuccess && s2 == NSFR_OK) e = e3;
        }
        c->stream = saved;
        (void)hipStreamDestroy(cap);
        if (e != hipSuccess || s2 != NSFR_OK) {
            set_error(std::string("graph capture failed: ") + hipGetErrorString(e));
            return NSFR_EHIP;
        }
        HIP_TRY(hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
        std::memcpy(c->gkey, key, sizeof(key));
    }
    for (int i = 0; i < nsteps; ++i) HIP_TRY(hipGraphLaunch(c->gexec, c->stream));
    return NSFR_OK;
}

nsfr_status nsfr_max_wavespeed(nsfr_ctx* c, const double* U, double* lam) {
    if (!c || !aligned(U) || !aligned(lam)) return bad("null or misaligned argument");
    nsfr_status st = use_device(c);
    if (st) return st;
    HIP_TRY(launch_max_wavespeed((int64_t)c->E * c->n3, U, c->cfg.gamma, c->red, c->nred, lam, c->stream));
    return NSFR_OK;
}

nsfr_status nsfr_cfl_dt(nsfr_ctx* c, const double* U, double cfl, double* dt) {
    if (!c || !aligned(U) || !aligned(dt) || !(cfl > 0)) return bad("null, misaligned or non-positive argument");
    nsfr_status st = nsfr_max_wavespeed(c, U, c->red + c->nred - 1);
    if (st) return st;
    double dx = (c->cfg.hi - c->cfg.lo) / (c->cfg.ne[0] * (double)c->n);
    HIP_TRY(launch_cfl_dt(c->red + c->nred - 1, cfl, dx, dt, c->stream));
    return NSFR_OK;
}

nsfr_status nsfr_diagnostics(nsfr_ctx* c, const double* U, double t, double* out) {
    if (!c || !aligned(U) || !aligned(out)) return bad("null or misaligned argument");
    nsfr_status st = nsfr_residual(c, U, c->wsR, t);
    if (st) return st;
    // NSFR on the Gauss-Legendre rule: the entropy rate pairs R with the
    // projected entropy variables that the residual evaluation left in vhat
    const bool proj = c->cfg.quad && c->cfg.scheme == 0;
    HIP_TRY(launch_diagnostics((int64_t)c->E * c->n3, U, proj ? c->vhat : nullptr, c->wsR, c->cfg.gamma, c->red,
                               c->nred, out, c->stream));
    return NSFR_OK;
}

nsfr_status nsfr_kinetic_energy(nsfr_ctx* c, const double* U, double* ke, double* grad) {
    if (!c || !aligned(U) || !aligned(ke) || (grad && !aligned(grad)) || (const double*)grad == U)
        return bad("null, misaligned or aliased argument");
    if (c->cfg.quad) {
        set_error("kinetic_energy is built for the collocated LGL scheme (quad = 0)");
        return NSFR_ENOTSUP;
    }
    nsfr_status st = use_device(c);
    if (st) return st;
    HIP_TRY(launch_kinetic_energy((int64_t)c->E * c->n3, U, c->invWJ, c->red, c->nred, ke, grad, c->stream));
    return NSFR_OK;
}

nsfr_status nsfr_check_state(nsfr_ctx* c, const double* U, int32_t* bad_host) {
    if (!c || !aligned(U) || !bad_host) return bad("null or misaligned argument");
    nsfr_status st = use_device(c);
    if (st) return st;
    HIP_TRY(launch_check_state((int64_t)c->E * c->n3, U, c->cfg.gamma, c->cnt, c->stream));
    int32_t h[64];
    HIP_TRY(hipMemcpyAsync(h, c->cnt, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    int32_t tot = 0;
    for (int i = 0; i < 64; ++i) tot += h[i];
    *bad_host = tot;
    if (tot > 0) {
        set_error("state has nodes with rho <= 0, p <= 0 or NaN");
        return NSFR_EUNPHYSICAL;
    }
    return NSFR_OK;
}

nsfr_status nsfr_rhs_vjp(nsfr_ctx* c, const double* U, const double* lam, double* g, double t) {
    (void)t;   // the source term does not depend on U
    if (!c || !aligned(U) || !aligned(lam) || !aligned(g) || g == U || g == lam)
        return bad("null, misaligned or aliased argument");
    if (exact_mass_unsupported(c, "nsfr_rhs_vjp")) return NSFR_ENOTSUP;
    if (c->cfg.surface_diss || c->cfg.quad) {
        set_error("rhs_vjp supports the collocated scheme with the entropy-conserving surface flux only "
                  "(surface_diss = 0, quad = 0)");
        return NSFR_ENOTSUP;
    }
    nsfr_status st = use_device(c);
    if (st) return st;
    StageArgs a = base_args(c);
    a.Uin = U;
    hipError_t e = launch_vjp(c->p, c->cfg.c_fr != 0.0, c->cfg.flux, a, lam, g, c->wsR2, c->stream);
    if (e != hipSuccess) {
        set_error(std::string("vjp kernel launch: ") + hipGetErrorString(e));
        return NSFR_EHIP;
    }
    return NSFR_OK;
}

nsfr_status nsfr_rk4_step_vjp(nsfr_ctx* c, const double* U, const double* dt, double t, const double* lam_next,
                              double* lam, double* work) {
    if (!c || !aligned(U) || !aligned(dt) || !aligned(lam_next) || !aligned(lam) || !aligned(work) || lam == U)
        return bad("null, misaligned or aliased argument");
    if (exact_mass_unsupported(c, "nsfr_rk4_step_vjp")) return NSFR_ENOTSUP;
    if (c->cfg.surface_diss || c->cfg.quad) {
        set_error("rk4_step_vjp supports the collocated scheme with the entropy-conserving surface flux only "
                  "(surface_diss = 0, quad = 0)");
        return NSFR_ENOTSUP;
    }
    nsfr_status st = use_device(c);
    if (st) return st;
    const int64_t ns = 5 * c->E * (int64_t)c->n3;
    double* w0 = work;            // copy of lam_next
    double* Y2 = work + ns;
    double* Y3 = work + 2 * ns;
    double* Y4 = work + 3 * ns;
    double* kap = work + 4 * ns;  // stage derivative, then stage cotangent
    double* gs = work + 5 * ns;   // VJP of a stage
    hipStream_t s = c->stream;
    StageArgs a = base_args(c);
    // forward recomputation of the stage states (time enters only the source)
    auto f = [&](const double* Y, double tt, double* out) -> nsfr_status {
        StageArgs b = a;
        b.Uin = Y;
        b.out = out;
        b.t = tt;
        b.tdev = nullptr;
        b.mode = MODE_RHS;
        return stage(c, b);
    };
    auto vjp = [&](const double* Y, const double* k, double* out) -> nsfr_status {
        StageArgs b = a;
        b.Uin = Y;
        hipError_t e = launch_vjp(c->p, c->cfg.c_fr != 0.0, c->cfg.flux, b, k, out, c->wsR2, s);
        if (e != hipSuccess) {
            set_error(std::string("vjp kernel launch: ") + hipGetErrorString(e));
            return NSFR_EHIP;
        }
        return NSFR_OK;
    };
    // stage times need dt on the host only for the source term
    double hdt = 0.0;
    if (c->cfg.source) {
        HIP_TRY(hipMemcpyAsync(&hdt, dt, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    if ((st = f(U, t, kap))) return st;
    HIP_TRY(launch_lincomb(ns, Y2, U, 1.0, 0.0, kap, 0.0, 0.5, dt, 0, s));
    if ((st = f(Y2, t + 0.5 * hdt, kap))) return st;
    HIP_TRY(launch_lincomb(ns, Y3, U, 1.0, 0.0, kap, 0.0, 0.5, dt, 0, s));
    if ((st = f(Y3, t + 0.5 * hdt, kap))) return st;
    HIP_TRY(launch_lincomb(ns, Y4, U, 1.0, 0.0, kap, 0.0, 1.0, dt, 0, s));
    // reverse sweep: kappa_s = dJ/dk_s, g_s = f'(Y_s)^T kappa_s, lam = lam' + sum g_s
    HIP_TRY(launch_lincomb(ns, w0, lam_next, 1.0, 0.0, nullptr, 0.0, 0.0, nullptr, 0, s));
    HIP_TRY(launch_lincomb(ns, kap, w0, 0.0, 1.0 / 6.0, nullptr, 0.0, 0.0, dt, 0, s));
    if ((st = vjp(Y4, kap, gs))) return st;
    HIP_TRY(launch_lincomb(ns, lam, w0, 1.0, 0.0, gs, 1.0, 0.0, nullptr, 0, s));
    HIP_TRY(launch_lincomb(ns, kap, w0, 0.0, 1.0 / 3.0, gs, 0.0, 1.0, dt, 0, s));
    if ((st = vjp(Y3, kap, gs))) return st;
    HIP_TRY(launch_lincomb(ns, lam, nullptr, 0.0, 0.0, gs, 1.0, 0.0, nullptr, 1, s));
    HIP_TRY(launch_lincomb(ns, kap, w0, 0.0, 1.0 / 3.0, gs, 0.0, 0.5, dt, 0, s));
    if ((st = vjp(Y2, kap, gs))) return st;
    HIP_TRY(launch_lincomb(ns, lam, nullptr, 0.0, 0.0, gs, 1.0, 0.0, nullptr, 1, s));
    HIP_TRY(launch_lincomb(ns, kap, w0, 0.0, 1.0 / 6.0, gs, 0.0, 0.5, dt, 0, s));
    if ((st = vjp(U, kap, gs))) return st;
    HIP_TRY(launch_lincomb(ns, lam, nullptr, 0.0, 0.0, gs, 1.0, 0.0, nullptr, 1, s));
    return NSFR_OK;
}

}  // extern "C"

// exposed to the other translation units of the library (ensembles)
namespace nsfr {
StageArgs ctx_stage_args(const nsfr_ctx* c) { return base_args(c); }
int ctx_kind(const nsfr_ctx* c) { return kind_code(c->p, c->cfg.c_fr != 0.0, c->cfg.flux); }
int64_t ctx_state_size(const nsfr_ctx* c) { return 5 * c->E * (int64_t)c->n3; }
}  // namespace nsfr
