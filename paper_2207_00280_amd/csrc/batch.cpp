// Batched integration + assembly of many independent patches (the paper's
// first concurrency level: parts of the mesh computed concurrently) in ONE
// launch.  Host side: per-patch plans, the device patch table and the work
// list of (patch, tile) items, sorted longest first so that the hardware's
// in-order workgroup dispatch balances the launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "batch.h"
#include "launch.h"

using namespace igaf;

namespace {

// Every tile of every patch, longest first; stable, so that the tiles of one
// patch stay in order (neighbouring tiles share kappa and tables in cache).
std::vector<int2> build_items(const std::vector<igaf_plan*>& plans)
{
    struct C {
        double cost;
        int2 it;
    };
    std::vector<C> all;
    for (size_t i = 0; i < plans.size(); ++i) {
        const PatchDev& pd = plan_dev(plans[i]);
        int n = 0;
        double c = 0.0;
        if (rows_tile_info(pd.p, pd.d[1].N, pd.d[2].N, pd.d[0].K, &n, &c) != 0) continue;
        for (int k = 0; k < n; ++k) all.push_back({c, make_int2((int)i, k)});
    }
    std::stable_sort(all.begin(), all.end(), [](const C& a, const C& b) { return a.cost > b.cost; });
    std::vector<int2> items;
    items.reserve(all.size());
    for (auto& c : all) items.push_back(c.it);
    return items;
}

}  // namespace

struct igaf_batch {
    std::vector<igaf_plan*> plans;
    int device = 0;
    int nitems = 0;
    BatchPatch* d_patches = nullptr;
    BatchPatch* h_patches = nullptr;   // pinned staging of the device table
    int2* d_items = nullptr;
    bool uploaded = false;
};

static void batch_free(igaf_batch* B)
{
    if (!B) return;
    if (B->d_patches) (void)hipFree(B->d_patches);
    if (B->h_patches) (void)hipHostFree(B->h_patches);
    if (B->d_items) (void)hipFree(B->d_items);
    for (auto* p : B->plans) igaf_plan_destroy(p);
    delete B;
}

static BatchPatch make_patch(const igaf_plan* p)
{
    BatchPatch b;
    std::memset(&b, 0, sizeof b);
    b.pd = plan_dev(p);
    b.rm = make_rowmap(b.pd);
    return b;
}

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
            batch_free(B);
            return st;
        }
        B->plans.push_back(p);
        if (!plan_hot_supported(p)) {
            batch_free(B);
            return set_error(IGAF_EUNSUPPORTED, "batch patches need nquad = degree+1");
        }
    }
    if (hipGetDevice(&B->device) != hipSuccess) {
        batch_free(B);
        return set_error(IGAF_EDEVICE, "hipGetDevice failed");
    }
    std::vector<int2> items = build_items(B->plans);
    B->nitems = (int)items.size();
    bool ok = hipMalloc(&B->d_items, sizeof(int2) * std::max<size_t>(1, items.size())) == hipSuccess &&
              hipMemcpy(B->d_items, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice) ==
                  hipSuccess &&
              hipMalloc(&B->d_patches, sizeof(BatchPatch) * npatch) == hipSuccess &&
              hipHostMalloc(&B->h_patches, sizeof(BatchPatch) * npatch, hipHostMallocDefault) == hipSuccess &&
              hipDeviceSynchronize() == hipSuccess;
    if (!ok) {
        batch_free(B);
        return set_error(IGAF_ENOMEM, "batch device allocation failed");
    }
    for (int i = 0; i < npatch; ++i) B->h_patches[i] = make_patch(B->plans[i]);
    *out = B;
    return IGAF_OK;
}

void igaf_batch_destroy(igaf_batch* B)
{
    if (!B) return;
    (void)hipDeviceSynchronize();
    batch_free(B);
}

const igaf_plan* igaf_batch_plan(const igaf_batch* B, int32_t i)
{
    if (!B || i < 0 || i >= (int)B->plans.size()) return nullptr;
    return B->plans[i];
}

igaf_status igaf_batch_info(const igaf_batch* B, int32_t* family, int32_t* grid, int32_t* nitems)
{
    if (!B) return set_error(IGAF_EINVAL, "batch is NULL");
    if (family) *family = 0;   // work items are tiles of row pencils
    if (grid) *grid = rows_batch_grid(B->nitems);
    if (nitems) *nitems = B->nitems;
    return IGAF_OK;
}

igaf_status igaf_batch_integrate_assemble(igaf_batch* B, const double* const* kappa,
                                          double* const* Mval, double* const* Kval, void* stream)
{
    if (!B || !kappa || (!Mval && !Kval)) return set_error(IGAF_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    const int n = (int)B->plans.size();
    bool changed = !B->uploaded;
    for (int i = 0; i < n && !changed; ++i) {
        const BatchPatch& b = B->h_patches[i];
        changed = b.kappa != kappa[i] || b.Mv != (Mval ? Mval[i] : nullptr) ||
                  b.Kv != (Kval ? Kval[i] : nullptr);
    }
    for (int i = 0; i < n; ++i)
        if (!kappa[i] || (!(Mval && Mval[i]) && !(Kval && Kval[i])))
            return set_error(IGAF_EINVAL, "patch without kappa or without outputs");
    if (changed) {
        // the staging buffer may still be read by a queued copy: wait first
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
            return set_error(IGAF_EINVAL,
                             "batch pointer tables changed during stream capture (call once eagerly first)");
        if (hipStreamSynchronize(s) != hipSuccess) return set_error(IGAF_EDEVICE, "stream sync failed");
        for (int i = 0; i < n; ++i) {
            B->h_patches[i].kappa = kappa[i];
            B->h_patches[i].Mv = Mval ? Mval[i] : nullptr;
            B->h_patches[i].Kv = Kval ? Kval[i] : nullptr;
        }
        B->uploaded = true;
    }
    if (hipMemcpyAsync(B->d_patches, B->h_patches, sizeof(BatchPatch) * n, hipMemcpyHostToDevice, s) !=
        hipSuccess)
        return set_error(IGAF_EDEVICE, "patch table upload failed");
    if (launch_rows_batch(B->d_patches, B->d_items, B->nitems, s))
        return set_error(IGAF_EDEVICE, "batched launch failed");
    return IGAF_OK;
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

}  // extern "C"
