// Ensembles of independent flows (placeholder entry points).
#include "nsfr_host.h"

using namespace nsfr;

extern "C" {
nsfr_status nsfr_ens_create(const nsfr_config*, int32_t, void*, nsfr_ens** out) {
    if (out) *out = nullptr;
    set_error("ensembles are not implemented in this build");
    return NSFR_ENOTSUP;
}
nsfr_status nsfr_ens_destroy(nsfr_ens*) { return NSFR_ENOTSUP; }
nsfr_status nsfr_ens_offsets(const nsfr_ens*, int64_t*) { return NSFR_ENOTSUP; }
nsfr_status nsfr_ens_rhs(nsfr_ens*, const double*, double*, double) { return NSFR_ENOTSUP; }
nsfr_status nsfr_ens_rk4_step(nsfr_ens*, double*, const double*, double, double*) { return NSFR_ENOTSUP; }
nsfr_status nsfr_ens_rk4_run(nsfr_ens*, double*, const double*, double, int32_t, double*) { return NSFR_ENOTSUP; }
nsfr_status nsfr_ens_set_tile(nsfr_ens*, int32_t, int32_t) { return NSFR_ENOTSUP; }
}
