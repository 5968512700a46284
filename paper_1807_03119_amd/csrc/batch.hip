// Batched filtering: many volumes of mixed size, dtype and radius in one call.
//
// The jobs are grouped into classes of equal (radius, voxel type).  Each class
// runs as ONE kernel launch over the tiles of all its volumes: workgroup b
// takes tile b of the class (XCD-aware order), finds its volume by binary
// search over the jobs' first-tile indices, and runs the same streaming tile
// body as the single-volume kernels (same registers, same occupancy).  The
// hardware dispatcher then keeps the GPU full across volume boundaries, and a
// class pays one launch and one tail instead of one per volume.  Larger
// volumes come first in a class, so its tail consists of small tiles.
//
// Per call: one H2D copy of the job table (from one of four pinned staging
// slots) and one launch per non-empty class, all on the caller's stream.
// These are plain launches rather than a graph: with this runtime a graph of a
// copy and one kernel costs about 15 us per launch and parallel kernel
// branches 45-95 us, against about 5 us for the copy and a kernel launched
// directly.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "device_common.h"
#include "lnf_ctx.h"
#include "lnf_internal.h"
#include "mean9_tile.h"
#include "minvar9_tile.h"

namespace lnf {

struct BatchJobDesc {
    const void* in;
    void* out;
    int nx, ny, nz;
    int tiles_x, tiles_y, zs, tile_begin;  // tile_begin: first tile in its class
    int pairs;                             // MEAN9 stages element pairs (mean9_pairs_ok)
};

struct BatchClass {
    int total;      // tiles in this class
    int njobs;      // jobs in this class
    int job_begin;  // index of its first job in `jobs`
    int variant;    // MEAN9 tile variant of the class
};

constexpr int kClasses = 2 * LNF_RADIUS_MAX;  // (radius, voxel type)

// Class of a (radius, dtype) pair.
constexpr int batch_class(int r, int dtype) { return 2 * (r - 1) + (dtype == LNF_U16 ? 1 : 0); }

struct BatchTable {
    BatchClass c[kClasses];
    BatchJobDesc jobs[LNF_BATCH_MAX];
};

namespace {

constexpr int kSlots = 4;

// Job of class tile t: the last job whose first tile is <= t (uniform per
// workgroup, so these are scalar loads).
__device__ __forceinline__ const BatchJobDesc& job_of(const BatchTable* tab, const BatchClass& c,
                                                      int t)
{
    int lo = c.job_begin, hi = c.job_begin + c.njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab->jobs[mid].tile_begin <= t) lo = mid;
        else hi = mid - 1;
    }
    return tab->jobs[lo];
}

template <int R, int TY, typename T, bool GATE, int TXW>
__global__ __launch_bounds__((M9Geo<R, TY, TXW>::THREADS))
__attribute__((amdgpu_waves_per_eu(R <= 3 ? 3 : 2))) void mean9_multi(
    const BatchTable* __restrict__ tab, int cls, uint32_t gate)
{
    __shared__ __align__(16) M9SmemAny<R, TY, TXW, T> sm;
    constexpr int n = (2 * R + 1) * (2 * R + 1) * (2 * R + 1);
    const BatchClass c = tab->c[cls];
    const int t = xcd_tile(blockIdx.x, c.total);
    const BatchJobDesc d = job_of(tab, c, t);
    const int local = t - d.tile_begin;
    const int bx = local % d.tiles_x;
    const int rest = local / d.tiles_x;
    const int by = rest % d.tiles_y;
    const int bz = rest / d.tiles_y;
    const Geom g{d.nx, d.ny, d.nz};
    const int z0 = bz * d.zs;
    mean9_tile<R, TY, T, GATE, TXW>(sm, d.pairs != 0, static_cast<const T*>(d.in),
                                    static_cast<T*>(d.out), g, bx * TXW, by * TY, z0,
                                    min(z0 + d.zs, d.nz), gate, 1.0 / (9.0 * n));
}

template <int R, typename T, bool GATE>
__global__ __launch_bounds__(MV9Shape<R>::THREADS)
__attribute__((amdgpu_waves_per_eu(MV9Shape<R>::WAVES))) void minvar9_multi(const BatchTable* __restrict__ tab, int cls,
                                                     uint32_t gate)
{
    __shared__ __align__(16) MV9Smem<R, T> sm;
    constexpr int n = (2 * R + 1) * (2 * R + 1) * (2 * R + 1);
    const BatchClass c = tab->c[cls];
    const int t = xcd_tile(blockIdx.x, c.total);
    const BatchJobDesc d = job_of(tab, c, t);
    const int local = t - d.tile_begin;
    const int bx = local % d.tiles_x;
    const int rest = local / d.tiles_x;
    const int by = rest % d.tiles_y;
    const int bz = rest / d.tiles_y;
    const Geom g{d.nx, d.ny, d.nz};
    const int z0 = bz * d.zs;
    minvar9_tile<R, T, GATE>(sm, static_cast<const T*>(d.in), static_cast<T*>(d.out), g,
                             bx * MV9Shape<R>::TX, by * MV9Shape<R>::TY, z0,
                             min(z0 + d.zs, d.nz), gate, (double)n, 1.0 / n);
}

// A launchable class kernel: function, block size.
struct ClassKernel {
    const void* fn = nullptr;
    int threads = 0;
};

template <int R, typename T, bool GATE, int TY, int TXW>
ClassKernel mean9_kernel()
{
    return {reinterpret_cast<const void*>(mean9_multi<R, TY, T, GATE, TXW>),
            M9Geo<R, TY, TXW>::THREADS};
}

template <int R, typename T, bool GATE>
ClassKernel mean9_kernel_v(int variant)
{
    switch (variant) {
    case 1: return mean9_kernel<R, T, GATE, 32, 64>();
    case 2: return mean9_kernel<R, T, GATE, 16, 32>();
    case 3: return mean9_kernel<R, T, GATE, 32, 32>();
    default: return mean9_kernel<R, T, GATE, 16, 64>();  // variant 0: 64 x 16
    }
}

template <int R, typename T>
ClassKernel class_kernel_rt(int rule, bool gate, int variant)
{
    if (rule == LNF_MEAN9)
        return gate ? mean9_kernel_v<R, T, true>(variant) : mean9_kernel_v<R, T, false>(variant);
    if (gate) return {reinterpret_cast<const void*>(minvar9_multi<R, T, true>), MV9Shape<R>::THREADS};
    return {reinterpret_cast<const void*>(minvar9_multi<R, T, false>), MV9Shape<R>::THREADS};
}

template <typename T>
ClassKernel class_kernel_t(int rule, int r, bool gate, int variant)
{
    switch (r) {
    case 1: return class_kernel_rt<1, T>(rule, gate, variant);
    case 2: return class_kernel_rt<2, T>(rule, gate, variant);
    case 3: return class_kernel_rt<3, T>(rule, gate, variant);
    default: return class_kernel_rt<4, T>(rule, gate, variant);
    }
}

// Kernel of class c (= batch_class(r, dtype)) for a tile variant.
ClassKernel class_kernel(int rule, int c, bool gate, int variant)
{
    const int r = c / 2 + 1;
    return (c & 1) ? class_kernel_t<uint16_t>(rule, r, gate, variant)
                   : class_kernel_t<uint8_t>(rule, r, gate, variant);
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

void batch_state_free(lnf_ctx* h)
{
    BatchState* st = h->batch;
    if (!st) return;
    for (auto& s : st->slot) free_slot(s);
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

int batch_launch(lnf_ctx* h, const lnf_job* jobs, int n, const std::vector<Geom>& geoms,
                 hipStream_t stream)
{
    if (h->geom) {  // geometry variants: the cluster-gather kernel, one launch per job
        for (int i = 0; i < n; ++i) {
            const TileCfg cfg = ctx_tile(h, h->rule, jobs[i].dtype, jobs[i].radius, geoms[i]);
            if (launch_rule(h->rule, h->geom, jobs[i].in, jobs[i].out, jobs[i].dtype,
                            jobs[i].radius, geoms[i], h->gate, cfg, stream) != hipSuccess)
                return LNF_EHIP;
        }
        return LNF_OK;
    }
    {
        std::lock_guard<std::mutex> lk(h->mu);
        if (!h->batch) {
            h->batch = new (std::nothrow) BatchState();
            if (!h->batch) return LNF_ENOMEM;
        }
    }
    BatchState* st = h->batch;
    std::lock_guard<std::mutex> lk(st->mu);
    BatchSlot& s = st->slot[st->next];
    st->next = (st->next + 1) % kSlots;
    if (!s.host) {
        const int rc = build_slot(s);
        if (rc) {
            free_slot(s);
            return rc;
        }
    }
    // the slot's previous table may still be read by its kernels
    if (s.pending && hipEventSynchronize(s.done) != hipSuccess) return LNF_EHIP;
    s.pending = false;

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
    int k = 0;
    for (int c = 0; c < kClasses; ++c) {
        BatchClass& cl = tab->c[c];
        cl = BatchClass{0, 0, k, 0};
        int kend = k;
        while (kend < n && batch_class(jobs[order[kend]].radius, jobs[order[kend]].dtype) == c)
            ++kend;
        if (kend == k) continue;
        const int r = c / 2 + 1, dtype = (c & 1) ? LNF_U16 : LNF_U8;
        // tile variant: the tuned one of the class's largest volume, else the
        // default for (dtype, r)
        int variant = 0, tx = 32, ty = 8;
        if (h->rule == LNF_MEAN9) {
            const TileCfg cfg = ctx_tile(h, h->rule, dtype, r, geoms[order[k]]);
            variant = cfg.variant >= 0 && cfg.variant < mean9_variants()
                          ? cfg.variant
                          : mean9_default_variant(dtype, r);
            mean9_tile_shape(variant, &tx, &ty);
        } else {
            minvar9_tile_shape(0, r, &tx, &ty);
        }
        kern[c] = class_kernel(h->rule, c, h->gate != 0, variant);
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
        k = kend;
    }
    const size_t used = offsetof(BatchTable, jobs) + (size_t)std::max(n, 1) * sizeof(BatchJobDesc);
    if (hipMemcpyAsync(s.dev, s.host, used, hipMemcpyHostToDevice, stream) != hipSuccess)
        return LNF_EHIP;
    for (int c = 0; c < kClasses; ++c) {
        if (tab->c[c].total == 0) continue;
        const BatchTable* dtab = s.dev;
        int cls = c;
        uint32_t gate = h->gate;
        void* args[] = {&dtab, &cls, &gate};
        if (hipLaunchKernel(kern[c].fn, dim3(tab->c[c].total), dim3(kern[c].threads), args, 0,
                            stream) != hipSuccess)
            return LNF_EHIP;
    }
    if (hipEventRecord(s.done, stream) != hipSuccess) return LNF_EHIP;
    s.pending = true;
    return LNF_OK;
}

}  // namespace lnf

using namespace lnf;

extern "C" int lnf_filter_batch(lnf_handle h, const lnf_job* jobs, int n, hipStream_t stream)
{
    if (!h) return LNF_EINVAL;
    std::vector<Geom> geoms;
    DeviceGuard dg(h->device);
    if (!dg.ok()) return LNF_EHIP;
    int rc = validate_jobs(h, jobs, n, &geoms);
    if (rc || n == 0) return rc;
    return batch_launch(h, jobs, n, geoms, stream);
}
