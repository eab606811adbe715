// Batched integration of many independent patches (placeholder: per-patch launches).
#include <hip/hip_runtime.h>

#include <new>
#include <vector>

#include "batch.h"
#include "launch.h"

using namespace igaf;

struct igaf_batch {
    std::vector<igaf_plan*> plans;
};

extern "C" {

igaf_status igaf_batch_create(const igaf_patch_desc* descs, int32_t npatch, igaf_batch** out)
{
    if (!out) return set_error(IGAF_EINVAL, "out is NULL");
    *out = nullptr;
    if (!descs || npatch < 1) return set_error(IGAF_EINVAL, "descs NULL or npatch < 1");
    igaf_batch* B = new (std::nothrow) igaf_batch();
    if (!B) return set_error(IGAF_ENOMEM, "host allocation failed");
    for (int i = 0; i < npatch; ++i) {
        igaf_plan* p = nullptr;
        igaf_status st = igaf_plan_create(&descs[i], &p);
        if (st) {
            igaf_batch_destroy(B);
            return st;
        }
        B->plans.push_back(p);
        if (!plan_hot_supported(p)) {
            igaf_batch_destroy(B);
            return set_error(IGAF_EUNSUPPORTED, "batch patches need nquad = degree+1");
        }
    }
    *out = B;
    return IGAF_OK;
}

void igaf_batch_destroy(igaf_batch* B)
{
    if (!B) return;
    for (auto* p : B->plans) igaf_plan_destroy(p);
    delete B;
}

const igaf_plan* igaf_batch_plan(const igaf_batch* B, int32_t i)
{
    if (!B || i < 0 || i >= (int)B->plans.size()) return nullptr;
    return B->plans[i];
}

igaf_status igaf_batch_integrate_assemble_separate(igaf_batch* B, const double* const* kappa,
                                                   double* const* Mval, double* const* Kval,
                                                   void* stream)
{
    if (!B || !kappa || (!Mval && !Kval)) return set_error(IGAF_EINVAL, "NULL argument");
    for (size_t i = 0; i < B->plans.size(); ++i) {
        igaf_status st = igaf_integrate_assemble(B->plans[i], IGAF_SUMFACT, kappa[i], nullptr,
                                                 nullptr, Mval ? Mval[i] : nullptr,
                                                 Kval ? Kval[i] : nullptr, stream);
        if (st) return st;
    }
    return IGAF_OK;
}

igaf_status igaf_batch_integrate_assemble(igaf_batch* B, const double* const* kappa,
                                          double* const* Mval, double* const* Kval, void* stream)
{
    return igaf_batch_integrate_assemble_separate(B, kappa, Mval, Kval, stream);
}

}  // extern "C"
