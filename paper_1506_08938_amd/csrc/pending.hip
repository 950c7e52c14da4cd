// Entry points whose kernels are not written yet: they report
// NMF_E_UNSUPPORTED rather than computing anything.
#include "nmf_internal.h"

using namespace nmfi;

extern "C" int nmf_gram(const float *, int64_t, int32_t, float, int32_t, float *, void *) {
    return fail(NMF_E_UNSUPPORTED, "nmf_gram: not available yet");
}
extern "C" int nmf_product(const nmf_matrix *, int32_t, int32_t, const float *, int32_t, float *, void *) {
    return fail(NMF_E_UNSUPPORTED, "nmf_product: not available yet");
}
extern "C" int nmf_plan_create(const nmf_matrix *, int32_t, const nmf_reg *, const nmf_opts *, nmf_plan **, void *) {
    return fail(NMF_E_UNSUPPORTED, "nmf_plan_create: not available yet");
}
extern "C" int nmf_plan_run(nmf_plan *, float *, float *, int32_t, double *, nmf_stats *, void *) {
    return fail(NMF_E_UNSUPPORTED, "nmf_plan_run: not available yet");
}
extern "C" void nmf_plan_destroy(nmf_plan *) {}
extern "C" int nmf_fit(const nmf_matrix *, int32_t, const nmf_reg *, const nmf_opts *, float *, float *, double *, nmf_stats *, void *) {
    return fail(NMF_E_UNSUPPORTED, "nmf_fit: not available yet");
}
extern "C" int nmf_objective(const nmf_matrix *, int32_t, const nmf_reg *, const float *, const float *, double *, double *, void *) {
    return fail(NMF_E_UNSUPPORTED, "nmf_objective: not available yet");
}
extern "C" int nmf_basis_create(const float *, int64_t, int32_t, float, float, const nmf_opts *, nmf_basis **, void *) {
    return fail(NMF_E_UNSUPPORTED, "nmf_basis_create: not available yet");
}
extern "C" int nmf_foldin(const nmf_basis *, const nmf_matrix *, float *, int32_t *, void *) {
    return fail(NMF_E_UNSUPPORTED, "nmf_foldin: not available yet");
}
extern "C" void nmf_basis_destroy(nmf_basis *) {}
