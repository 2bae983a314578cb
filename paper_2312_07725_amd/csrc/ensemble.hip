// Ensembles of independent flows: each RK stage of every flow, whatever its
// degree and mesh size, in one launch per kind of flow present (degree,
// c != 0, flux variant).
//
// Each flow owns an ordinary context (operators, warped mesh, metrics). The
// packed state is the concatenation of the flows' state arrays. A device table
// holds one StageArgs per (stage, flow) and a work list holds (flow, first
// element) items, grouped by kind and within a kind sorted by decreasing
// cost; a kind's launch runs one workgroup per item of its slice with the
// kernel specialised for that kind. Tiles (elements per item) are per degree
// and can be set from an autotuned table.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "nsfr_host.h"

using namespace nsfr;

namespace {
constexpr int NMODES = 5;   // RK1..RK4, RHS

int mode_slot(int mode) { return mode == MODE_RHS ? 4 : mode - MODE_RK1; }

int default_ens_epb(int p) { return default_epb(p); }
constexpr int NKINDS = 16;
}  // namespace

struct nsfr_ens {
    int nf = 0;
    int dev = 0;
    hipStream_t stream = nullptr;
    std::vector<nsfr_ctx*> flows;
    std::vector<nsfr_config> cfgs;
    std::vector<int64_t> offs;     // state offsets in doubles (nf + 1)
    std::vector<int> kinds;
    int epb[4] = {0, 0, 0, 0};     // per p = 2..5
    StageArgs* dtab = nullptr;     // [NMODES][nf]
    int2* ditems = nullptr;        // work list, grouped by kind
    int nitems = 0;
    int kbeg[NKINDS] = {}, kcnt[NKINDS] = {};   // each kind's slice of the work list
    bool items_ok = false;
    const void* key[NMODES][4] = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    const void* gkey[3] = {nullptr, nullptr, nullptr};
};

#define HIP_TRY(call)                                                                 \
    do {                                                                              \
        hipError_t _e = (call);                                                       \
        if (_e != hipSuccess) {                                                       \
            set_error(std::string(#call) + ": " + hipGetErrorString(_e));             \
            return NSFR_EHIP;                                                         \
        }                                                                             \
    } while (0)

static void ens_free(nsfr_ens* s) {
    if (!s) return;
    if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    if (s->dtab) (void)hipFree(s->dtab);
    if (s->ditems) (void)hipFree(s->ditems);
    for (auto* c : s->flows)
        if (c) nsfr_destroy(c);
    delete s;
}

// (re)build the sorted work list for the current tiles
static nsfr_status build_items(nsfr_ens* s) {
    struct Item { int f; int e0; int kind; double cost; };
    std::vector<Item> items;
    for (int f = 0; f < s->nf; ++f) {
        const nsfr_config& c = s->cfgs[f];
        const int n = c.p + 1, n3 = n * n * n;
        const int epb = s->epb[c.p - 2];
        const int64_t E = (int64_t)c.ne[0] * c.ne[1] * c.ne[2];
        const double per_node_pairs = 1.5 * (n - 1) + 6.0 / n;
        for (int64_t e0 = 0; e0 < E; e0 += epb) {
            int cnt = (int)std::min<int64_t>(epb, E - e0);
            items.push_back({f, (int)e0, s->kinds[f], cnt * n3 * per_node_pairs});
        }
    }
    std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) {
        return a.kind != b.kind ? a.kind < b.kind : a.cost > b.cost;
    });
    std::fill(s->kbeg, s->kbeg + NKINDS, 0);
    std::fill(s->kcnt, s->kcnt + NKINDS, 0);
    for (size_t i = 0; i < items.size(); ++i) {
        const int k = items[i].kind;
        if (s->kcnt[k] == 0) s->kbeg[k] = (int)i;
        ++s->kcnt[k];
    }
    std::vector<int2> h(items.size());
    for (size_t i = 0; i < items.size(); ++i) h[i] = make_int2(items[i].f, items[i].e0);
    if (s->ditems) (void)hipFree(s->ditems);
    s->ditems = nullptr;
    HIP_TRY(hipMalloc((void**)&s->ditems, std::max<size_t>(1, h.size()) * sizeof(int2)));
    HIP_TRY(hipMemcpy(s->ditems, h.data(), h.size() * sizeof(int2), hipMemcpyHostToDevice));
    s->nitems = (int)h.size();
    s->items_ok = true;
    std::memset(s->key, 0, sizeof(s->key));   // tables carry epb: rebuild them
    return NSFR_OK;
}

// StageArgs of every flow for one stage, for the given packed buffers
static nsfr_status build_table(nsfr_ens* s, int mode, const double* Uin, const double* Un, double* acc, double* out,
                               const double* dt, double t) {
    const int slot = mode_slot(mode);
    const void* k[4] = {Uin, out, acc, dt};
    if (std::memcmp(k, s->key[slot], sizeof(k)) == 0) return NSFR_OK;
    std::vector<StageArgs> tab(s->nf);
    for (int f = 0; f < s->nf; ++f) {
        StageArgs a = ctx_stage_args(s->flows[f]);
        const int64_t o = s->offs[f];
        a.Uin = Uin + o;
        a.Un = Un ? Un + o : nullptr;
        a.acc = acc ? acc + o : nullptr;
        a.out = out + o;
        a.dt = dt ? dt + f : nullptr;
        a.t = t;
        a.tdev = nullptr;
        a.mode = mode;
        a.epb = s->epb[s->cfgs[f].p - 2];
        tab[f] = a;
    }
    HIP_TRY(hipMemcpy(s->dtab + (size_t)slot * s->nf, tab.data(), tab.size() * sizeof(StageArgs),
                      hipMemcpyHostToDevice));
    std::memcpy(s->key[slot], k, sizeof(k));
    return NSFR_OK;
}

static nsfr_status launch(nsfr_ens* s, int mode, hipStream_t st) {
    const StageArgs* tab = s->dtab + (size_t)mode_slot(mode) * s->nf;
    for (int k = 0; k < NKINDS; ++k) {
        if (s->kcnt[k] == 0) continue;
        const int p = k / 4 + 2;
        hipError_t e = launch_ensemble_kind(k, tab, s->ditems + s->kbeg[k], s->kcnt[k], s->epb[p - 2], st);
        if (e != hipSuccess) {
            set_error(std::string("ensemble kernel launch: ") + hipGetErrorString(e));
            return NSFR_EHIP;
        }
    }
    return NSFR_OK;
}

static nsfr_status prepare_rk4(nsfr_ens* s, double* U, const double* dt, double t, double* work) {
    const int64_t tot = s->offs[s->nf];
    double* acc = work;
    double* Ya = work + tot;
    double* Yb = work + 2 * tot;
    nsfr_status st;
    if (!s->items_ok && (st = build_items(s))) return st;
    if ((st = build_table(s, MODE_RK1, U, U, acc, Ya, dt, t))) return st;
    if ((st = build_table(s, MODE_RK2, Ya, U, acc, Yb, dt, t))) return st;
    if ((st = build_table(s, MODE_RK3, Yb, U, acc, Ya, dt, t))) return st;
    return build_table(s, MODE_RK4, Ya, U, acc, U, dt, t);
}

static nsfr_status enqueue_rk4(nsfr_ens* s, hipStream_t st) {
    nsfr_status r;
    for (int m = MODE_RK1; m <= MODE_RK4; ++m)
        if ((r = launch(s, m, st))) return r;
    return NSFR_OK;
}

static bool al8(const void* p) { return p && ((uintptr_t)p % 8 == 0); }

extern "C" {

nsfr_status nsfr_ens_create(const nsfr_config* cfgs, int32_t n, void* stream, nsfr_ens** out) {
    if (!out) {
        set_error("null output pointer");
        return NSFR_EINVAL;
    }
    *out = nullptr;
    if (!cfgs || n < 1) {
        set_error("need at least one flow");
        return NSFR_EINVAL;
    }
    nsfr_ens* s = new nsfr_ens();
    s->nf = n;
    s->stream = (hipStream_t)stream;
    (void)hipGetDevice(&s->dev);
    for (int p = 2; p <= 5; ++p) s->epb[p - 2] = default_ens_epb(p);
    s->offs.push_back(0);
    for (int f = 0; f < n; ++f) {
        nsfr_config c = cfgs[f];
        if (c.source || c.surface_diss || c.quad || c.mass) {
            set_error("ensemble flows take the collocated LGL scheme with the entropy-conserving surface flux, "
                      "no source term and the weight-adjusted mass inverse");
            ens_free(s);
            return NSFR_ENOTSUP;
        }
        nsfr_ctx* ctx = nullptr;
        nsfr_status st = nsfr_create(&c, stream, &ctx);
        if (st != NSFR_OK) {
            ens_free(s);
            return st;
        }
        s->flows.push_back(ctx);
        s->cfgs.push_back(c);
        s->kinds.push_back(ctx_kind(ctx));
        s->offs.push_back(s->offs.back() + ctx_state_size(ctx));
    }
    if (hipMalloc((void**)&s->dtab, (size_t)NMODES * n * sizeof(StageArgs)) != hipSuccess) {
        set_error("hipMalloc failed for the ensemble tables");
        ens_free(s);
        return NSFR_ENOMEM;
    }
    nsfr_status st = build_items(s);
    if (st != NSFR_OK) {
        ens_free(s);
        return st;
    }
    *out = s;
    return NSFR_OK;
}

nsfr_status nsfr_ens_destroy(nsfr_ens* s) {
    if (!s) {
        set_error("null ensemble");
        return NSFR_EINVAL;
    }
    ens_free(s);
    return NSFR_OK;
}

nsfr_status nsfr_ens_set_stream(nsfr_ens* s, void* stream) {
    if (!s) {
        set_error("null ensemble");
        return NSFR_EINVAL;
    }
    s->stream = (hipStream_t)stream;
    return NSFR_OK;
}

nsfr_status nsfr_ens_offsets(const nsfr_ens* s, int64_t* offs) {
    if (!s || !offs) {
        set_error("null argument");
        return NSFR_EINVAL;
    }
    for (int f = 0; f <= s->nf; ++f) offs[f] = s->offs[f];
    return NSFR_OK;
}

nsfr_status nsfr_ens_set_tile(nsfr_ens* s, int32_t p, int32_t epb) {
    if (!s || p < 2 || p > 5) {
        set_error("null ensemble or p outside 2..5");
        return NSFR_EINVAL;
    }
    if (epb == 0) epb = default_ens_epb(p);
    if (epb < 1 || epb > max_epb(p)) {
        set_error("tile does not fit the stage workgroup (512 threads) or the LDS budget");
        return NSFR_EINVAL;
    }
    s->epb[p - 2] = epb;
    s->items_ok = false;
    if (s->gexec) { (void)hipGraphExecDestroy(s->gexec); s->gexec = nullptr; }
    if (s->graph) { (void)hipGraphDestroy(s->graph); s->graph = nullptr; }
    return NSFR_OK;
}

nsfr_status nsfr_ens_rhs(nsfr_ens* s, const double* U, double* dUdt, double t) {
    if (!s || !al8(U) || !al8(dUdt) || U == dUdt) {
        set_error("null, misaligned or aliased argument");
        return NSFR_EINVAL;
    }
    nsfr_status st;
    if (!s->items_ok && (st = build_items(s))) return st;
    if ((st = build_table(s, MODE_RHS, U, nullptr, nullptr, dUdt, nullptr, t))) return st;
    return launch(s, MODE_RHS, s->stream);
}

nsfr_status nsfr_ens_rk4_step(nsfr_ens* s, double* U, const double* dt, double t, double* work) {
    if (!s || !al8(U) || !al8(dt) || !al8(work)) {
        set_error("null or misaligned argument");
        return NSFR_EINVAL;
    }
    nsfr_status st = prepare_rk4(s, U, dt, t, work);
    if (st) return st;
    return enqueue_rk4(s, s->stream);
}

nsfr_status nsfr_ens_rk4_run(nsfr_ens* s, double* U, const double* dt, double t, int32_t nsteps, double* work) {
    if (!s || !al8(U) || !al8(dt) || !al8(work) || nsteps < 0) {
        set_error("null, misaligned or negative argument");
        return NSFR_EINVAL;
    }
    if (nsteps == 0) return NSFR_OK;
    nsfr_status st = prepare_rk4(s, U, dt, t, work);
    if (st) return st;
    const void* k[3] = {U, dt, work};
    if (!s->gexec || std::memcmp(k, s->gkey, sizeof(k)) != 0) {
        if (s->gexec) { (void)hipGraphExecDestroy(s->gexec); s->gexec = nullptr; }
        if (s->graph) { (void)hipGraphDestroy(s->graph); s->graph = nullptr; }
        hipStream_t cap;
        HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        nsfr_status r = NSFR_OK;
        if (e == hipSuccess) {
            r = enqueue_rk4(s, cap);
            hipError_t e2 = hipStreamEndCapture(cap, &s->graph);
            if (e2 != hipSuccess && r == NSFR_OK) e = e2;
        }
        (void)hipStreamDestroy(cap);
        if (e != hipSuccess || r != NSFR_OK) {
            set_error(std::string("ensemble graph capture failed: ") + hipGetErrorString(e));
            return NSFR_EHIP;
        }
        HIP_TRY(hipGraphInstantiate(&s->gexec, s->graph, nullptr, nullptr, 0));
        std::memcpy(s->gkey, k, sizeof(k));
    }
    for (int i = 0; i < nsteps; ++i) HIP_TRY(hipGraphLaunch(s->gexec, s->stream));
    return NSFR_OK;
}

}  // extern "C"
