// Batched integration + assembly of many independent patches (the paper's
// first concurrency level: parts of the mesh computed concurrently) in one
// launch per degree present (each with that degree's tile, whose block size
// and LDS differ).  Host side: per-patch plans, the device patch table and
// the work list of (patch, tile, x segment) items, grouped by degree and
// sorted longest first within a degree so that the hardware's in-order
// workgroup dispatch balances each launch, and the autotuner that picks the
// work split (segments per tile, items per XCD chunk) by timing the launches
// on the caller's data.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <iterator>
#include <new>
#include <vector>

#include "batch.h"
#include "launch.h"

using namespace igaf;

namespace {

constexpr int kSplits[] = {1, 2, 4, 8};
constexpr int kChunks[] = {4, 16, 64};
constexpr int kDefaultChunk = 16;
constexpr int kMaxDegree = 5;

// A work list: items of degree p at [off[p], off[p + 1]).
struct WorkList {
    std::vector<int4> items;
    int off[kMaxDegree + 2] = {};
};

// Every (tile, x segment) of every patch, grouped by degree and longest first
// within a degree; stable, so that the tiles of one patch stay in order
// (neighbouring tiles share kappa and tables in cache).  A patch's rows are
// cut into at most `split` segments of at least 2(p+1) rows; a segment that
// does not start at row 0 sweeps p warm-up elements first, which its cost
// includes.
WorkList build_items(const std::vector<igaf_plan*>& plans, int split)
{
    struct C {
        int p;
        double cost;
        int4 it;
    };
    std::vector<C> all;
    for (size_t i = 0; i < plans.size(); ++i) {
        const PatchDev& pd = plan_dev(plans[i]);
        int n = 0;
        double per_elem = 0.0;
        if (rows_tile_info(pd.p, pd.d[1].N, pd.d[2].N, &n, &per_elem) != 0) continue;
        const int Nx = pd.d[0].N;
        const int nseg = std::max(1, std::min(split, Nx / (2 * (pd.p + 1))));
        const int seglen = (Nx + nseg - 1) / nseg;
        for (int k = 0; k < n; ++k)
            for (int sgi = 0; sgi < nseg; ++sgi) {
                const int X0 = sgi * seglen, X1 = std::min(Nx, X0 + seglen);
                if (X0 >= X1) continue;
                const double cost = per_elem * (X1 - std::max(0, X0 - pd.p));
                all.push_back({pd.p, cost, make_int4((int)i, k, sgi, seglen)});
            }
    }
    std::stable_sort(all.begin(), all.end(),
                     [](const C& a, const C& b) { return a.p != b.p ? a.p < b.p : a.cost > b.cost; });
    WorkList w;
    w.items.reserve(all.size());
    for (auto& c : all) {
        w.items.push_back(c.it);
        ++w.off[c.p + 1];
    }
    for (int p = 1; p <= kMaxDegree + 1; ++p) w.off[p] += w.off[p - 1];
    return w;
}

}  // namespace

struct igaf_batch {
    std::vector<igaf_plan*> plans;
    int device = 0;
    int nitems = 0;
    int off[kMaxDegree + 2] = {};           // items of degree p: [off[p], off[p + 1]) of `items`
    int split = 1, chunk = kDefaultChunk;   // work split in use
    double tuned_ms = 0.0;                  // its time when the autotuner chose it
    // one immutable device list per split (kSplits order), uploaded at
    // creation: a re-split only selects another list, so a graph captured
    // with an earlier split keeps reading the items it was captured with
    WorkList lists[std::size(kSplits)];
    int4* d_lists = nullptr;
    const int4* items = nullptr;            // the list of the split in use
    BatchPatch* d_patches = nullptr;
    BatchPatch* h_patches = nullptr;   // pinned staging of the device table
    bool uploaded = false;
};

static void batch_free(igaf_batch* B)
{
    if (!B) return;
    if (B->d_patches) (void)hipFree(B->d_patches);
    if (B->h_patches) (void)hipHostFree(B->h_patches);
    if (B->d_lists) (void)hipFree(B->d_lists);
    for (auto* p : B->plans) igaf_plan_destroy(p);
    delete B;
}

// Build every split's work list and upload them into one device buffer
// (synchronous, at creation).
static bool upload_work_lists(igaf_batch* B)
{
    size_t total = 0;
    for (size_t k = 0; k < std::size(kSplits); ++k) {
        B->lists[k] = build_items(B->plans, kSplits[k]);
        total += B->lists[k].items.size();
    }
    if (hipMalloc(&B->d_lists, sizeof(int4) * std::max<size_t>(1, total)) != hipSuccess) return false;
    size_t base = 0;
    for (auto& w : B->lists) {
        if (!w.items.empty() &&
            hipMemcpy(B->d_lists + base, w.items.data(), sizeof(int4) * w.items.size(), hipMemcpyHostToDevice) !=
                hipSuccess)
            return false;
        base += w.items.size();
    }
    return true;
}

// Select the work list of one split and the chunking of its launches.
static void set_work_list(igaf_batch* B, int split, int chunk)
{
    size_t base = 0, k = 0;
    for (; kSplits[k] != split; ++k) base += B->lists[k].items.size();
    B->items = B->d_lists + base;
    B->nitems = (int)B->lists[k].items.size();
    std::copy(std::begin(B->lists[k].off), std::end(B->lists[k].off), B->off);
    B->split = split;
    B->chunk = chunk;
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
    bool ok = upload_work_lists(B) && hipMalloc(&B->d_patches, sizeof(BatchPatch) * npatch) == hipSuccess &&
              hipHostMalloc(&B->h_patches, sizeof(BatchPatch) * npatch, hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        batch_free(B);
        return set_error(IGAF_ENOMEM, "batch device allocation failed");
    }
    set_work_list(B, 1, kDefaultChunk);
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
    if (grid) {
        *grid = 0;
        for (int p = 1; p <= kMaxDegree; ++p) *grid += rows_batch_grid(B->off[p + 1] - B->off[p], B->chunk);
    }
    if (nitems) *nitems = B->nitems;
    return IGAF_OK;
}

igaf_status igaf_batch_set_split(igaf_batch* B, int32_t split, int32_t chunk)
{
    if (!B) return set_error(IGAF_EINVAL, "batch is NULL");
    if (std::find(std::begin(kSplits), std::end(kSplits), split) == std::end(kSplits) ||
        std::find(std::begin(kChunks), std::end(kChunks), chunk) == std::end(kChunks))
        return set_error(IGAF_EINVAL, "split must be 1, 2, 4 or 8 and chunk 4, 16 or 64");
    set_work_list(B, split, chunk);
    B->tuned_ms = 0.0;
    return IGAF_OK;
}

igaf_status igaf_batch_split(const igaf_batch* B, int32_t* split, int32_t* chunk, double* tuned_ms)
{
    if (!B) return set_error(IGAF_EINVAL, "batch is NULL");
    if (split) *split = B->split;
    if (chunk) *chunk = B->chunk;
    if (tuned_ms) *tuned_ms = B->tuned_ms;
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
    for (int p = kMaxDegree; p >= 1; --p)   // the costliest degrees first
        if (launch_rows_batch(p, B->d_patches, B->items + B->off[p], B->off[p + 1] - B->off[p], B->chunk, s))
            return set_error(IGAF_EDEVICE, "batched launch failed");
    return IGAF_OK;
}

igaf_status igaf_batch_autotune(igaf_batch* B, const double* const* kappa, double* const* Mval,
                                double* const* Kval, int32_t reps, void* stream)
{
    if (!B || !kappa || (!Mval && !Kval)) return set_error(IGAF_EINVAL, "NULL argument");
    if (reps < 1 || reps > 100) return set_error(IGAF_EINVAL, "reps outside [1, 100]");
    hipStream_t s = (hipStream_t)stream;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
        return set_error(IGAF_EINVAL, "the autotuner times launches: not under stream capture");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return set_error(IGAF_EDEVICE, "event creation failed");
    }
    igaf_status st = IGAF_OK;
    int best_split = 1, best_chunk = kDefaultChunk;
    double best = INFINITY;
    for (int split : kSplits) {
        for (int chunk : kChunks) {
            set_work_list(B, split, chunk);
            std::vector<float> ms;
            st = igaf_batch_integrate_assemble(B, kappa, Mval, Kval, stream);   // warm-up
            for (int r = 0; r < reps && !st; ++r) {
                float t = 0.f;
                if (hipEventRecord(e0, s) != hipSuccess) { st = set_error(IGAF_EDEVICE, "event record failed"); break; }
                st = igaf_batch_integrate_assemble(B, kappa, Mval, Kval, stream);
                if (st) break;
                if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
                    st = set_error(IGAF_EDEVICE, "timing failed");
                    break;
                }
                ms.push_back(t);
            }
            if (st) break;
            std::sort(ms.begin(), ms.end());
            const double med = ms[ms.size() / 2];
            if (med < best) {
                best = med;
                best_split = split;
                best_chunk = chunk;
            }
        }
        if (st) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    set_work_list(B, st ? 1 : best_split, st ? kDefaultChunk : best_chunk);
    if (st) return st;
    B->tuned_ms = best;
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
