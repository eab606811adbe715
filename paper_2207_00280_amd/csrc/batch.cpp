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
constexpr int kNumSplits = 4;
constexpr int kChunks[] = {4, 16, 64};
constexpr int kDefaultChunk = 16;
constexpr int kMaxDegree = 5;

int split_index(int split)
{
    for (int k = 0; k < kNumSplits; ++k)
        if (kSplits[k] == split) return k;
    return -1;
}

// The work list of the degree-p patches for one tile shape and split: every
// (tile, x segment) of every such patch, longest first; stable, so that the
// tiles of one patch stay in order (neighbouring tiles share kappa and
// tables in cache).  A patch's rows are cut into at most `split` segments
// of at least 2(p+1) rows; a segment that does not start at row 0 sweeps p
// warm-up elements first, which its cost includes.
std::vector<int4> build_items(const std::vector<igaf_plan*>& plans, int p, int variant, int split)
{
    struct C {
        double cost;
        int4 it;
    };
    std::vector<C> all;
    for (size_t i = 0; i < plans.size(); ++i) {
        const PatchDev& pd = plan_dev(plans[i]);
        if (pd.p != p) continue;
        int n = 0;
        double per_elem = 0.0;
        if (rows_tile_info(pd.p, variant, pd.d[1].N, pd.d[2].N, &n, &per_elem) != 0) continue;
        const int Nx = pd.d[0].N;
        const int nseg = std::max(1, std::min(split, Nx / (2 * (pd.p + 1))));
        const int seglen = (Nx + nseg - 1) / nseg;
        for (int k = 0; k < n; ++k)
            for (int sgi = 0; sgi < nseg; ++sgi) {
                const int X0 = sgi * seglen, X1 = std::min(Nx, X0 + seglen);
                if (X0 >= X1) continue;
                const double cost = per_elem * (X1 - std::max(0, X0 - pd.p));
                all.push_back({cost, make_int4((int)i, k, sgi, seglen)});
            }
    }
    std::stable_sort(all.begin(), all.end(), [](const C& a, const C& b) { return a.cost > b.cost; });
    std::vector<int4> items;
    items.reserve(all.size());
    for (auto& c : all) items.push_back(c.it);
    return items;
}

// The launch configuration of one degree
struct DegreeCfg {
    int variant = 0, split = 1, chunk = kDefaultChunk;
    double tuned_ms = 0.0;   // its median launch time when the autotuner chose it
};

}  // namespace

struct igaf_batch {
    std::vector<igaf_plan*> plans;
    int device = 0;
    // one immutable device list per (degree, tile shape, split), uploaded at
    // creation: a new configuration only selects other lists, so a graph
    // captured earlier keeps reading the items it was captured with
    int4* d_lists = nullptr;
    int64_t base[kMaxDegree + 1][kTileVariants][kNumSplits] = {};
    int count[kMaxDegree + 1][kTileVariants][kNumSplits] = {};
    DegreeCfg cfg[kMaxDegree + 1];
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

// Build every work list and upload them into one device buffer (synchronous,
// at creation).
static bool upload_work_lists(igaf_batch* B)
{
    std::vector<int4> all;
    for (int p = 1; p <= kMaxDegree; ++p)
        for (int v = 0; v < kTileVariants; ++v)
            for (int k = 0; k < kNumSplits; ++k) {
                std::vector<int4> items = build_items(B->plans, p, v, kSplits[k]);
                B->base[p][v][k] = (int64_t)all.size();
                B->count[p][v][k] = (int)items.size();
                all.insert(all.end(), items.begin(), items.end());
            }
    if (hipMalloc(&B->d_lists, sizeof(int4) * std::max<size_t>(1, all.size())) != hipSuccess) return false;
    return all.empty() ||
           hipMemcpy(B->d_lists, all.data(), sizeof(int4) * all.size(), hipMemcpyHostToDevice) == hipSuccess;
}

static int degree_items(const igaf_batch* B, int p)
{
    const DegreeCfg& c = B->cfg[p];
    return B->count[p][c.variant][split_index(c.split)];
}

// The batched launch of the degree-p patches with the degree's configuration
static int launch_degree(igaf_batch* B, int p, hipStream_t s)
{
    const DegreeCfg& c = B->cfg[p];
    const int k = split_index(c.split);
    return launch_rows_batch(p, c.variant, B->d_patches, B->d_lists + B->base[p][c.variant][k],
                             B->count[p][c.variant][k], c.chunk, s);
}

// Copy the patch pointer tables of this call to the device (see
// igaf_batch_integrate_assemble).
static igaf_status upload_pointers(igaf_batch* B, const double* const* kappa, double* const* Mval,
                                   double* const* Kval, hipStream_t s)
{
    const int n = (int)B->plans.size();
    bool changed = !B->uploaded;
    for (int i = 0; i < n && !changed; ++i) {
        const BatchPatch& b = B->h_patches[i];
        changed = b.kappa != kappa[i] || b.Mv != (Mval ? Mval[i] : nullptr) || b.Kv != (Kval ? Kval[i] : nullptr);
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
    if (hipMemcpyAsync(B->d_patches, B->h_patches, sizeof(BatchPatch) * n, hipMemcpyHostToDevice, s) != hipSuccess)
        return set_error(IGAF_EDEVICE, "patch table upload failed");
    return IGAF_OK;
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
    int g = 0, n = 0;
    for (int p = 1; p <= kMaxDegree; ++p) {
        g += rows_batch_grid(degree_items(B, p), B->cfg[p].chunk);
        n += degree_items(B, p);
    }
    if (grid) *grid = g;
    if (nitems) *nitems = n;
    return IGAF_OK;
}

static bool valid_split_chunk(int split, int chunk)
{
    return split_index(split) >= 0 && std::find(std::begin(kChunks), std::end(kChunks), chunk) != std::end(kChunks);
}

igaf_status igaf_batch_set_split(igaf_batch* B, int32_t split, int32_t chunk)
{
    if (!B) return set_error(IGAF_EINVAL, "batch is NULL");
    if (!valid_split_chunk(split, chunk))
        return set_error(IGAF_EINVAL, "split must be 1, 2, 4 or 8 and chunk 4, 16 or 64");
    for (int p = 1; p <= kMaxDegree; ++p) B->cfg[p] = DegreeCfg{0, split, chunk, 0.0};
    return IGAF_OK;
}

igaf_status igaf_batch_set_degree_config(igaf_batch* B, int32_t degree, int32_t tile, int32_t split, int32_t chunk)
{
    if (!B) return set_error(IGAF_EINVAL, "batch is NULL");
    if (degree < 1 || degree > kMaxDegree) return set_error(IGAF_EINVAL, "degree outside 1..5");
    if (tile < 0 || tile >= kTileVariants) return set_error(IGAF_EINVAL, "tile must be 0 or 1");
    if (!valid_split_chunk(split, chunk))
        return set_error(IGAF_EINVAL, "split must be 1, 2, 4 or 8 and chunk 4, 16 or 64");
    B->cfg[degree] = DegreeCfg{tile, split, chunk, 0.0};
    return IGAF_OK;
}

igaf_status igaf_batch_degree_config(const igaf_batch* B, int32_t degree, int32_t* tile, int32_t* split,
                                     int32_t* chunk, double* tuned_ms, int32_t* nitems)
{
    if (!B) return set_error(IGAF_EINVAL, "batch is NULL");
    if (degree < 1 || degree > kMaxDegree) return set_error(IGAF_EINVAL, "degree outside 1..5");
    const DegreeCfg& c = B->cfg[degree];
    if (tile) *tile = c.variant;
    if (split) *split = c.split;
    if (chunk) *chunk = c.chunk;
    if (tuned_ms) *tuned_ms = c.tuned_ms;
    if (nitems) *nitems = degree_items(B, degree);
    return IGAF_OK;
}

igaf_status igaf_batch_split(const igaf_batch* B, int32_t* split, int32_t* chunk, double* tuned_ms)
{
    if (!B) return set_error(IGAF_EINVAL, "batch is NULL");
    int top = 1;
    double ms = 0.0;
    for (int p = 1; p <= kMaxDegree; ++p) {
        if (degree_items(B, p) > 0) top = p;
        ms += B->cfg[p].tuned_ms;
    }
    if (split) *split = B->cfg[top].split;
    if (chunk) *chunk = B->cfg[top].chunk;
    if (tuned_ms) *tuned_ms = ms;
    return IGAF_OK;
}

igaf_status igaf_batch_integrate_assemble(igaf_batch* B, const double* const* kappa,
                                          double* const* Mval, double* const* Kval, void* stream)
{
    if (!B || !kappa || (!Mval && !Kval)) return set_error(IGAF_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    igaf_status st = upload_pointers(B, kappa, Mval, Kval, s);
    if (st) return st;
    for (int p = kMaxDegree; p >= 1; --p)   // the costliest degrees first
        if (launch_degree(B, p, s)) return set_error(IGAF_EDEVICE, "batched launch failed");
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
    igaf_status st = upload_pointers(B, kappa, Mval, Kval, s);
    if (st) return st;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return set_error(IGAF_EDEVICE, "event creation failed");
    }
    // each degree's launch is independent of the others': tune them one at a time
    for (int p = 1; p <= kMaxDegree && !st; ++p) {
        bool any = false;
        for (int v = 0; v < kTileVariants; ++v)
            for (int k = 0; k < kNumSplits; ++k) any = any || B->count[p][v][k] > 0;
        if (!any) continue;
        DegreeCfg best = B->cfg[p];
        best.tuned_ms = INFINITY;
        for (int v = 0; v < kTileVariants && !st; ++v)
            for (int split : kSplits) {
                if (st) break;
                for (int chunk : kChunks) {
                    B->cfg[p] = DegreeCfg{v, split, chunk, 0.0};
                    if (launch_degree(B, p, s)) {   // warm-up
                        st = set_error(IGAF_EDEVICE, "batched launch failed");
                        break;
                    }
                    std::vector<float> ms;
                    for (int r = 0; r < reps; ++r) {
                        float t = 0.f;
                        if (hipEventRecord(e0, s) != hipSuccess || launch_degree(B, p, s) ||
                            hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
                            st = set_error(IGAF_EDEVICE, "timing failed");
                            break;
                        }
                        ms.push_back(t);
                    }
                    if (st) break;
                    std::sort(ms.begin(), ms.end());
                    const double med = ms[ms.size() / 2];
                    if (med < best.tuned_ms) best = DegreeCfg{v, split, chunk, med};
                }
            }
        B->cfg[p] = st ? DegreeCfg{} : best;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st)
        for (int p = 1; p <= kMaxDegree; ++p) B->cfg[p] = DegreeCfg{};
    return st;
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
