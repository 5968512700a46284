// Batched filtering: many volumes of mixed size, dtype and radius in one call.
//
// The jobs are grouped into classes of equal (radius, voxel type).  Each class
// runs as ONE kernel launch over the tiles of all its volumes, in one of two
// modes:
//   - grid (LNF_BATCH_GRID, the default): workgroup b takes tile b of the class
//     (XCD-aware order), finds its volume by binary search over the jobs'
//     first-tile indices, and runs the same tile body as the single-volume
//     kernels (same registers, same occupancy).  Larger volumes come first, so
//     the class's tail consists of small tiles;
//   - queue (LNF_BATCH_PERSISTENT): one workgroup per resident slot takes tiles
//     from an atomic counter in the job table until the class is done.
// The hardware dispatcher (grid) or the queue keeps the GPU full across volume
// boundaries, and a class pays one launch and one tail instead of one per
// volume.  Geometry-variant contexts run the cluster kernel of cluster.hip the
// same way (grid mode).
//
// Per call: one H2D copy of the job table (from one of four pinned staging
// slots, queue counters uploaded as zero, so the call can be captured in a
// graph without memset nodes) and one launch per non-empty class, all on the
// caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "device_common.h"
#include "lnf_ctx.h"
#include "lnf_internal.h"
#include "batch_table.h"
#include "mean9_tile.h"
#include "plane_tile.h"

namespace lnf {

namespace {

constexpr int kSlots = 4;         // job-table staging slots of eager calls, used in turn
constexpr int kCaptureSlots = 4;  // slots of calls captured in a graph, one per capture

template <int R, int TY, typename T, bool GATE, int TXW, bool QUEUE>
__global__ __launch_bounds__((M9Geo<R, TY, TXW>::THREADS))
__attribute__((amdgpu_waves_per_eu((m9_waves<R, M9Geo<R, TY, TXW>::THREADS>())))) void mean9_multi(
    BatchTable* __restrict__ tab, int cls, uint32_t gate)
{
    __shared__ __align__(16) M9SmemAny<R, TY, TXW, T> sm;
    __shared__ int s_t;
    constexpr int n = (2 * R + 1) * (2 * R + 1) * (2 * R + 1);
    for_class_tiles<TXW, TY, QUEUE>(tab, cls, &s_t, [&](const BatchJobDesc& d, int x0, int y0,
                                                       int z0, int z1, int tid) {
        mean9_tile<R, TY, T, GATE, TXW>(sm, d.pairs != 0, static_cast<const T*>(d.in),
                                        static_cast<T*>(d.out), Geom{d.nx, d.ny, d.nz}, x0, y0,
                                        z0, z1, gate, 1.0 / (9.0 * n), tid);
    });
}

template <int R, typename T, bool GATE, bool WT, bool QUEUE>
__global__ __launch_bounds__((MV9Shape<R, WT>::THREADS))
__attribute__((amdgpu_waves_per_eu((MV9Shape<R, WT>::WAVES)))) void minvar9_multi(
    BatchTable* __restrict__ tab, int cls, uint32_t gate)
{
    using S = MV9Shape<R, WT>;
    __shared__ __align__(16) MV9Lds<R, T, WT> sm;
    __shared__ int s_t;
    constexpr int n = (2 * R + 1) * (2 * R + 1) * (2 * R + 1);
    for_class_tiles<S::TX, S::TY, QUEUE>(tab, cls, &s_t, [&](const BatchJobDesc& d, int x0,
                                                            int y0, int z0, int z1, int tid) {
        minvar9_tile<R, T, GATE, WT>(sm, static_cast<const T*>(d.in), static_cast<T*>(d.out),
                                     Geom{d.nx, d.ny, d.nz}, x0, y0, z0, z1, gate, (double)n,
                                     1.0 / n, tid);
    });
}

template <int R, typename T, bool GATE, int TY, int TXW, bool QUEUE>
ClassKernel mean9_kernel()
{
    return {reinterpret_cast<const void*>(mean9_multi<R, TY, T, GATE, TXW, QUEUE>),
            M9Geo<R, TY, TXW>::THREADS};
}

// Queue mode is compiled for the 64 x 16 tile only.
template <int R, typename T, bool GATE>
ClassKernel mean9_kernel_v(int variant, bool queue)
{
    if (queue) return mean9_kernel<R, T, GATE, 16, 64, true>();
    switch (variant) {
    case 1: return mean9_kernel<R, T, GATE, 32, 64, false>();
    case 2: return mean9_kernel<R, T, GATE, 16, 32, false>();
    case 3: return mean9_kernel<R, T, GATE, 32, 32, false>();
    default: return mean9_kernel<R, T, GATE, 16, 64, false>();  // variant 0: 64 x 16
    }
}

template <int R, typename T, bool GATE, bool WT>
ClassKernel minvar9_kernel(bool queue)
{
    if (queue)
        return {reinterpret_cast<const void*>(minvar9_multi<R, T, GATE, WT, true>),
                MV9Shape<R, WT>::THREADS};
    return {reinterpret_cast<const void*>(minvar9_multi<R, T, GATE, WT, false>),
            MV9Shape<R, WT>::THREADS};
}

template <int R, typename T>
ClassKernel class_kernel_rt(int rule, bool gate, int variant, bool queue)
{
    if (rule == LNF_MEAN9)
        return gate ? mean9_kernel_v<R, T, true>(variant, queue)
                    : mean9_kernel_v<R, T, false>(variant, queue);
    if (variant == 1)
        return gate ? minvar9_kernel<R, T, true, true>(queue) : minvar9_kernel<R, T, false, true>(queue);
    return gate ? minvar9_kernel<R, T, true, false>(queue) : minvar9_kernel<R, T, false, false>(queue);
}

template <typename T>
ClassKernel class_kernel_t(int rule, int r, bool gate, int variant, bool queue)
{
    switch (r) {
    case 1: return class_kernel_rt<1, T>(rule, gate, variant, queue);
    case 2: return class_kernel_rt<2, T>(rule, gate, variant, queue);
    case 3: return class_kernel_rt<3, T>(rule, gate, variant, queue);
    default: return class_kernel_rt<4, T>(rule, gate, variant, queue);
    }
}

// Kernel of class c (= batch_class(r, dtype)) for a tile variant.
ClassKernel class_kernel(int rule, int c, bool gate, int variant, bool queue)
{
    const int r = c / 2 + 1;
    return (c & 1) ? class_kernel_t<uint16_t>(rule, r, gate, variant, queue)
                   : class_kernel_t<uint8_t>(rule, r, gate, variant, queue);
}

// ---- job table of lnf_filter_batch_noalloc ----------------------------------
// A file-scope device array: one copy per GPU, at its own address on each,
// kept until the process ends.  In host code the name `scratch` is only a
// host-side stand-in; host code uses the device address that
// hipGetSymbolAddress returns for the current device (static_table_init).
struct StaticBatchTable {
    BatchClass c[kClasses];
    BatchJobDesc jobs[LNF_BATCH_NOALLOC_MAX];
};
static_assert(offsetof(StaticBatchTable, jobs) == offsetof(BatchTable, jobs),
              "the static table is a prefix of BatchTable");
static_assert(sizeof(StaticBatchTable) == 20608, "size stated in lnf.h");
static __device__ __align__(256) unsigned char scratch[sizeof(StaticBatchTable)];

std::mutex g_static_mu;
std::map<int, BatchTable*> g_static_table;  // device -> address of its `scratch`

// Address of `scratch` on `device`, which must be the current device; looked
// up once per device.  Null when the lookup fails.
BatchTable* static_table_init(int device)
{
    std::lock_guard<std::mutex> lk(g_static_mu);
    auto it = g_static_table.find(device);
    if (it != g_static_table.end()) return it->second;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
        (void)hipGetLastError();
        return nullptr;
    }
    BatchTable* t = static_cast<BatchTable*>(p);
    g_static_table[device] = t;
    return t;
}

struct BatchSlot {
    BatchTable* host = nullptr;  // pinned staging copy of the table
    BatchTable* dev = nullptr;
    hipEvent_t done = nullptr;
    bool pending = false;
};

}  // namespace

struct BatchState {
    std::mutex mu;
    BatchSlot slot[kSlots];
    int next = 0;
    // A call captured in a HIP graph keeps its table for the graph's lifetime:
    // its replays copy that host table again.  Those slots are allocated with
    // the rest (no allocation may happen during a capture) and never reused.
    BatchSlot captured[kCaptureSlots];
    int ncaptured = 0;
    BatchTable* static_dev = nullptr;  // this device's `scratch` (lnf_filter_batch_noalloc)
};

namespace {

void free_slot(BatchSlot& s)
{
    if (s.done) {
        (void)hipEventSynchronize(s.done);
        (void)hipEventDestroy(s.done);
    }
    if (s.dev) (void)hipFree(s.dev);
    if (s.host) (void)hipHostFree(s.host);
    s = BatchSlot{};
}

int build_slot(BatchSlot& s)
{
    if (hipHostMalloc((void**)&s.host, sizeof(BatchTable), hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void**)&s.dev, sizeof(BatchTable)) != hipSuccess) {
        (void)hipGetLastError();
        return LNF_ENOMEM;
    }
    std::memset(s.host, 0, sizeof(BatchTable));
    if (hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) return LNF_EHIP;
    return LNF_OK;
}

}  // namespace

int batch_state_init(lnf_ctx* h)
{
    BatchState* st = new (std::nothrow) BatchState();
    if (!st) return LNF_ENOMEM;
    h->batch = st;
    for (auto& s : st->slot)
        if (int rc = build_slot(s)) return rc;
    for (auto& s : st->captured)
        if (int rc = build_slot(s)) return rc;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || !(st->static_dev = static_table_init(dev)))
        return LNF_EHIP;
    return LNF_OK;
}

void batch_state_free(lnf_ctx* h)
{
    BatchState* st = h->batch;
    if (!st) return;
    for (auto& s : st->slot) free_slot(s);
    for (auto& s : st->captured) free_slot(s);
    delete st;
    h->batch = nullptr;
}

// Validate every job, as lnf_filter would, plus cross-job overlap of outputs.
int validate_jobs(const lnf_ctx* h, const lnf_job* jobs, int n, std::vector<Geom>* geoms)
{
    if (n < 0 || n > LNF_BATCH_MAX || (n > 0 && !jobs)) return LNF_EINVAL;
    geoms->resize(n);
    std::vector<std::pair<uintptr_t, uintptr_t>> outs, ins;
    for (int i = 0; i < n; ++i) {
        size_t bytes = 0;
        int rc = check_volume_args(h, jobs[i].in, jobs[i].dims, jobs[i].dtype, jobs[i].radius,
                                   jobs[i].out, &(*geoms)[i], &bytes);
        if (rc) return rc;
        if ((rc = check_device_range(jobs[i].in, bytes, h->device))) return rc;
        if ((rc = check_device_range(jobs[i].out, bytes, h->device))) return rc;
        outs.push_back({(uintptr_t)jobs[i].out, (uintptr_t)jobs[i].out + bytes});
        ins.push_back({(uintptr_t)jobs[i].in, (uintptr_t)jobs[i].in + bytes});
    }
    // an output may not overlap another output or any input (inputs may be shared)
    std::vector<std::pair<uintptr_t, uintptr_t>> all = outs;
    std::sort(all.begin(), all.end());
    for (size_t i = 1; i < all.size(); ++i)
        if (all[i].first < all[i - 1].second) return LNF_EINVAL;
    for (const auto& o : outs)
        for (const auto& in : ins)
            if (o.first < in.second && in.first < o.second) return LNF_EINVAL;
    return LNF_OK;
}

// dev_table: where the table goes on the device (null: the slot's own buffer).
int batch_launch(lnf_ctx* h, const lnf_job* jobs, int n, const std::vector<Geom>& geoms,
                 hipStream_t stream, bool queue, BatchTable* dev_table = nullptr)
{
    BatchState* st = h->batch;
    if (!st) return LNF_ENOMEM;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cap) != hipSuccess) return LNF_EHIP;
    const bool capturing = cap != hipStreamCaptureStatusNone;
    std::lock_guard<std::mutex> lk(st->mu);
    BatchSlot* sp;
    if (capturing) {
        if (st->ncaptured == kCaptureSlots) return LNF_EBUSY;
        sp = &st->captured[st->ncaptured++];
    } else {
        sp = &st->slot[st->next];
        st->next = (st->next + 1) % kSlots;
        // the slot's previous table may still be read by its kernels
        if (sp->pending && hipEventSynchronize(sp->done) != hipSuccess) return LNF_EHIP;
        sp->pending = false;
    }
    BatchSlot& s = *sp;

    // order: by class, then larger jobs first (their tiles get the low indices)
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    auto vox = [&](int i) { return (double)geoms[i].nx * geoms[i].ny * geoms[i].nz; };
    std::sort(order.begin(), order.end(), [&](int a, int b) {
        const int ca = batch_class(jobs[a].radius, jobs[a].dtype);
        const int cb = batch_class(jobs[b].radius, jobs[b].dtype);
        if (ca != cb) return ca < cb;
        if (vox(a) != vox(b)) return vox(a) > vox(b);
        return a < b;
    });
    BatchTable* tab = s.host;
    ClassKernel kern[kClasses];
    GeomClassKernel gk[kClasses];
    int grid[kClasses] = {};
    int k = 0;
    for (int c = 0; c < kClasses; ++c) {
        BatchClass& cl = tab->c[c];
        cl = BatchClass{0, 0, k, 0, {}};
        int kend = k;
        while (kend < n && batch_class(jobs[order[kend]].radius, jobs[order[kend]].dtype) == c)
            ++kend;
        if (kend == k) continue;
        const int r = c / 2 + 1, dtype = (c & 1) ? LNF_U16 : LNF_U8;
        // tile variant: the tuned one of the class's largest volume, else the
        // default for that volume
        int variant = 0, tx = 32, ty = 8;
        const TileCfg cfg = ctx_tile(h, h->rule, dtype, r, geoms[order[k]]);
        if (h->geom) {
            gk[c] = geometry_class_kernel(h->rule, h->geom, dtype, r);
            kern[c] = gk[c].k;
            tx = gk[c].tx;
            ty = gk[c].ty;
        } else {
            if (h->rule == LNF_MEAN9) {
                variant = queue ? 0
                          : cfg.variant >= 0 && cfg.variant < mean9_variants()
                              ? cfg.variant
                              : mean9_default_variant(dtype, r);
                mean9_tile_shape(variant, &tx, &ty);
            } else {
                variant = cfg.variant >= 0 && cfg.variant < minvar9_variants()
                              ? cfg.variant
                              : minvar9_default_variant(dtype, r, geoms[order[k]]);
                minvar9_tile_shape(variant, r, &tx, &ty);
            }
            kern[c] = class_kernel(h->rule, c, h->gate != 0, variant, queue);
        }
        // z-strips: the class's volumes differ in depth, so its workgroups
        // differ in length and the launch ends on a tail of the longest ones.
        // About 16 workgroups per resident slot keep that tail short (measured
        // on 64 mixed volumes: 1.38 ms against 1.61 ms for one strip per
        // column); strips stay at least 16 slices deep
        const long long target = resident_groups(kern[c].fn, kern[c].threads);
        long long cols = 0;
        for (int q = k; q < kend; ++q) {
            const Geom& g = geoms[order[q]];
            cols += (long long)((g.nx + tx - 1) / tx) * ((g.ny + ty - 1) / ty);
        }
        const int nzs_want = (int)std::min<long long>(1 << 20, std::max<long long>(1, (16 * target + cols - 1) / cols));
        for (int q = k; q < kend; ++q) {
            const int i = order[q];
            const Geom& g = geoms[i];
            BatchJobDesc& d = tab->jobs[q];
            d.in = jobs[i].in;
            d.out = jobs[i].out;
            d.nx = g.nx;
            d.ny = g.ny;
            d.nz = g.nz;
            d.pairs = mean9_pairs_ok(d.in, g.nx, dtype == LNF_U8 ? 1 : 2) ? 1 : 0;
            const int nzs = std::min(nzs_want, std::max(1, g.nz / 16));
            d.zs = (g.nz + nzs - 1) / nzs;
            d.tiles_x = (g.nx + tx - 1) / tx;
            d.tiles_y = (g.ny + ty - 1) / ty;
            const long long tiles = (long long)d.tiles_x * d.tiles_y * ((g.nz + d.zs - 1) / d.zs);
            if ((long long)cl.total + tiles > INT32_MAX) return LNF_EINVAL;
            d.tile_begin = cl.total;
            cl.total += (int)tiles;
        }
        cl.njobs = kend - k;
        cl.variant = variant;
        // queue mode: one workgroup per resident slot, at most one per tile
        grid[c] = queue ? (int)std::min<long long>(cl.total, target) : cl.total;
        k = kend;
    }
    const size_t used = offsetof(BatchTable, jobs) + (size_t)std::max(n, 1) * sizeof(BatchJobDesc);
    BatchTable* dtab = dev_table ? dev_table : s.dev;
    if (hipMemcpyAsync(dtab, s.host, used, hipMemcpyHostToDevice, stream) != hipSuccess)
        return LNF_EHIP;
    for (int c = 0; c < kClasses; ++c) {
        if (tab->c[c].total == 0) continue;
        int cls = c;
        uint32_t gate = h->gate;
        hipError_t e;
        if (h->geom) {
            const void* nul = nullptr;
            void* nulo = nullptr;
            Geom g0{0, 0, 0};
            int z = 0, total = tab->c[c].total;
            double dn = gk[c].dn, inv = gk[c].inv;
            void* args[] = {&dtab, &cls, &nul, &nulo, &g0, &z, &z, &z, &total, &gate, &dn, &inv};
            e = hipLaunchKernel(kern[c].fn, dim3(grid[c]), dim3(kern[c].threads), args, 0, stream);
        } else {
            void* args[] = {&dtab, &cls, &gate};
            e = hipLaunchKernel(kern[c].fn, dim3(grid[c]), dim3(kern[c].threads), args, 0, stream);
        }
        if (e != hipSuccess) return LNF_EHIP;
    }
    if (!capturing) {
        if (hipEventRecord(s.done, stream) != hipSuccess) return LNF_EHIP;
        s.pending = true;
    }
    return LNF_OK;
}

}  // namespace lnf

using namespace lnf;

extern "C" int lnf_filter_batch_mode(lnf_handle h, const lnf_job* jobs, int n, hipStream_t stream,
                                     int mode)
{
    if (!h || (mode != LNF_BATCH_GRID && mode != LNF_BATCH_PERSISTENT)) return LNF_EINVAL;
    // queue mode runs the default geometry only
    if (mode == LNF_BATCH_PERSISTENT && h->geom) return LNF_EINVAL;
    std::vector<Geom> geoms;
    DeviceGuard dg(h->device);
    if (!dg.ok()) return LNF_EHIP;
    int rc = validate_jobs(h, jobs, n, &geoms);
    if (rc || n == 0) return rc;
    return batch_launch(h, jobs, n, geoms, stream, mode == LNF_BATCH_PERSISTENT);
}

extern "C" int lnf_filter_batch(lnf_handle h, const lnf_job* jobs, int n, hipStream_t stream)
{
    return lnf_filter_batch_mode(h, jobs, n, stream, LNF_BATCH_GRID);
}

// Grid mode with the job table in this GPU's static `scratch` array: no
// allocation of any kind on the device (the host staging slot and the table
// address were set up by lnf_create).
extern "C" int lnf_filter_batch_noalloc(lnf_handle h, const lnf_job* jobs, int n,
                                        hipStream_t stream)
{
    if (!h) return LNF_EINVAL;
    if (n > LNF_BATCH_NOALLOC_MAX) return LNF_ERANGE;
    std::vector<Geom> geoms;
    DeviceGuard dg(h->device);
    if (!dg.ok()) return LNF_EHIP;
    int rc = validate_jobs(h, jobs, n, &geoms);
    if (rc || n == 0) return rc;
    if (!h->batch || !h->batch->static_dev) return LNF_EHIP;
    return batch_launch(h, jobs, n, geoms, stream, false, h->batch->static_dev);
}
