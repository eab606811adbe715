// Batched integration + assembly of many independent patches (the paper's
// first concurrency level: parts of the mesh computed concurrently) in ONE
// persistent launch.  Host side: per-patch plans, the cost-sorted work list,
// the device patch table, and the autotuner that picks the work-item family
// (how finely the z column offsets of a row are split) and the persistent
// grid size by timing candidates on one representative patch per degree.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "batch.h"
#include "launch.h"

using namespace igaf;

namespace {

struct Tuned {
    int fam = 0;
    int grid = 0;
};

std::mutex g_tune_mu;
std::map<std::pair<int, unsigned>, Tuned> g_tune_cache;   // (device, degree mask) -> choice

struct WorkList {
    std::vector<int2> items;
};

WorkList build_items(const std::vector<igaf_plan*>& plans, int fam)
{
    struct C {
        double cost;
        int2 it;
    };
    std::vector<C> all;
    for (size_t i = 0; i < plans.size(); ++i) {
        const PatchDev& pd = plan_dev(plans[i]);
        int n = rows_item_count(pd.p, fam, pd.d[1].N, pd.d[2].N);
        double c = rows_item_cost(pd.p, fam, pd.d[0].K);
        for (int k = 0; k < n; ++k) all.push_back({c, make_int2((int)i, k)});
    }
    // longest first; stable so that items of one patch stay in order (their
    // neighbouring pencils share kappa and tables in cache)
    std::stable_sort(all.begin(), all.end(), [](const C& a, const C& b) { return a.cost > b.cost; });
    WorkList w;
    w.items.reserve(all.size());
    for (auto& c : all) w.items.push_back(c.it);
    return w;
}

}  // namespace

struct igaf_batch {
    std::vector<igaf_plan*> plans;
    int device = 0;
    int fam = 0, grid = 0;
    int nitems = 0;
    BatchPatch* d_patches = nullptr;
    BatchPatch* h_patches = nullptr;   // pinned staging of the device table
    int2* d_items = nullptr;
    int* d_ctr = nullptr;
    bool uploaded = false;
};

static void batch_free(igaf_batch* B)
{
    if (!B) return;
    if (B->d_patches) (void)hipFree(B->d_patches);
    if (B->h_patches) (void)hipHostFree(B->h_patches);
    if (B->d_items) (void)hipFree(B->d_items);
    if (B->d_ctr) (void)hipFree(B->d_ctr);
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

// Install the items of `plans` for family `fam` into the device list `d_items`
// (reallocated as needed); returns the number of items or -1.
static int install_items(const std::vector<igaf_plan*>& plans, int fam, int2** d_items)
{
    WorkList w = build_items(plans, fam);
    if (*d_items) (void)hipFree(*d_items);
    *d_items = nullptr;
    if (hipMalloc(d_items, sizeof(int2) * std::max<size_t>(1, w.items.size())) != hipSuccess) return -1;
    if (hipMemcpy(*d_items, w.items.data(), sizeof(int2) * w.items.size(), hipMemcpyHostToDevice) !=
        hipSuccess)
        return -1;
    return (int)w.items.size();
}

// Time the candidates on one representative (largest) patch per degree.
static igaf_status autotune(igaf_batch* B, Tuned* out)
{
    unsigned mask = 0;
    std::map<int, igaf_plan*> rep;
    for (auto* p : B->plans) {
        const PatchDev& pd = plan_dev(p);
        mask |= 1u << pd.p;
        auto it = rep.find(pd.p);
        if (it == rep.end() || plan_dev(it->second).E < pd.E) rep[pd.p] = p;
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find({B->device, mask});
        if (it != g_tune_cache.end()) {
            *out = it->second;
            return IGAF_OK;
        }
    }
    int ncu = 256;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, B->device) != hipSuccess)
        ncu = 256;
    std::vector<igaf_plan*> mini;
    for (auto& kv : rep) mini.push_back(kv.second);
    // scratch inputs / outputs for the representative patches
    std::vector<BatchPatch> hp;
    std::vector<void*> bufs;
    bool ok = true;
    for (auto* p : mini) {
        BatchPatch b = make_patch(p);
        const PatchDev& pd = b.pd;
        int64_t nq = (int64_t)pd.d[0].Q * pd.d[1].Q * pd.d[2].Q;
        double *k = nullptr, *m = nullptr, *kk = nullptr;
        ok = ok && hipMalloc(&k, sizeof(double) * pd.E * nq) == hipSuccess;
        ok = ok && hipMalloc(&m, sizeof(double) * pd.nnz) == hipSuccess;
        ok = ok && hipMalloc(&kk, sizeof(double) * pd.nnz) == hipSuccess;
        bufs.push_back(k);
        bufs.push_back(m);
        bufs.push_back(kk);
        if (!ok) break;
        ok = launch_fill_zero(k, pd.E * nq, nullptr) == 0;   // any finite coefficient times the same
        b.kappa = k;
        b.Mv = m;
        b.Kv = kk;
        hp.push_back(b);
    }
    BatchPatch* dp = nullptr;
    int2* di = nullptr;
    int* ctr = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ok = ok && hipMalloc(&dp, sizeof(BatchPatch) * hp.size()) == hipSuccess &&
         hipMemcpy(dp, hp.data(), sizeof(BatchPatch) * hp.size(), hipMemcpyHostToDevice) == hipSuccess &&
         hipMalloc(&ctr, 2 * sizeof(int)) == hipSuccess && hipMemset(ctr, 0, 2 * sizeof(int)) == hipSuccess &&
         hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
    Tuned best;
    float best_ms = 1e30f;
    for (int fam = 0; ok && fam < 2; ++fam) {
        int n = install_items(mini, fam, &di);
        if (n < 0) {
            ok = false;
            break;
        }
        for (int wpc : {1, 2, 3, 4, 6, 8}) {
            int grid = wpc * ncu;
            float ms = 1e30f;
            for (int rep = 0; rep < 3 && ok; ++rep) {
                ok = hipEventRecord(e0, nullptr) == hipSuccess &&
                     launch_rows_batch(fam, grid, dp, di, n, ctr, nullptr) == 0 &&
                     hipEventRecord(e1, nullptr) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
                float t = 0.f;
                if (ok && hipEventElapsedTime(&t, e0, e1) == hipSuccess && rep > 0) ms = std::min(ms, t);
            }
            if (ok && ms < best_ms) {
                best_ms = ms;
                best.fam = fam;
                best.grid = grid;
            }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (dp) (void)hipFree(dp);
    if (di) (void)hipFree(di);
    if (ctr) (void)hipFree(ctr);
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (!ok || best.grid == 0) return set_error(IGAF_EDEVICE, "batch autotuning failed");
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[{B->device, mask}] = best;
    }
    *out = best;
    return IGAF_OK;
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
    Tuned t;
    igaf_status st = autotune(B, &t);
    if (st) {
        batch_free(B);
        return st;
    }
    B->fam = t.fam;
    B->grid = t.grid;
    B->nitems = install_items(B->plans, B->fam, &B->d_items);
    bool ok = B->nitems >= 0 &&
              hipMalloc(&B->d_patches, sizeof(BatchPatch) * npatch) == hipSuccess &&
              hipHostMalloc(&B->h_patches, sizeof(BatchPatch) * npatch, hipHostMallocDefault) == hipSuccess &&
              hipMalloc(&B->d_ctr, 2 * sizeof(int)) == hipSuccess &&
              hipMemset(B->d_ctr, 0, 2 * sizeof(int)) == hipSuccess && hipDeviceSynchronize() == hipSuccess;
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
    if (family) *family = B->fam;
    if (grid) *grid = B->grid;
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
    if (launch_rows_batch(B->fam, B->grid, B->d_patches, B->d_items, B->nitems, B->d_ctr, s))
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
