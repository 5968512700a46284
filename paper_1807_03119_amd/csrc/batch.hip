// Batched filtering: many volumes of mixed size, dtype and radius in one graph
// launch.  The tiles of all jobs with the same radius form one work queue; a
// persistent kernel per radius class (the tile body is specialised on r) lets
// every workgroup pull tiles with an atomic counter until the queue is empty,
// so the GPU stays full across job boundaries instead of draining at the end
// of every volume.  The four class kernels are parallel branches of the graph.
//
// The graph of a context is built once per staging slot:
//     H2D copy of the job table  ->  {class kernel r=1, r=2, r=3, r=4}
// and reused for every batch: only the host-side table and the copy size
// change between launches.  The queue counters live in the table, so the copy
// itself resets them (no memset node).
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
    int nx, ny, nz, dtype;
    int tiles_x, tiles_y, zs, tile_begin;  // tile_begin: first tile in its class queue
    int pairs;                             // MEAN9 stages element pairs (mean9_pairs_ok)
};

struct BatchQueue {
    int total;      // tiles in this class
    int njobs;      // jobs in this class
    int job_begin;  // index of its first job in `jobs`
    int counter;    // next tile to hand out (reset to 0 by the upload)
};

struct BatchTable {
    BatchQueue q[LNF_RADIUS_MAX];
    BatchJobDesc jobs[LNF_BATCH_MAX];
};

namespace {

constexpr int kSlots = 4;
constexpr int kMean9TY = 16;  // batch tiles use the 64 x 16 streaming body

// Thread 0 takes the next tile of the class queue and finds its job by binary
// search over the jobs' first-tile indices; the pair is broadcast through LDS.
__device__ __forceinline__ bool next_tile(BatchTable* tab, BatchQueue* q, int* s_tile,
                                          int* s_job, int* tile, int* job)
{
    if (threadIdx.x == 0) {
        const int t = atomicAdd(&q->counter, 1);
        int j = -1;
        if (t < q->total) {
            int lo = q->job_begin, hi = q->job_begin + q->njobs - 1;
            while (lo < hi) {  // last job with tile_begin <= t
                const int mid = (lo + hi + 1) >> 1;
                if (tab->jobs[mid].tile_begin <= t) lo = mid;
                else hi = mid - 1;
            }
            j = lo;
        }
        *s_tile = t;
        *s_job = j;
    }
    __syncthreads();
    *tile = *s_tile;
    *job = *s_job;
    __syncthreads();
    return *job >= 0;
}

template <int R, bool GATE>
__global__ __launch_bounds__((M9Shape<R, kMean9TY>::THREADS)) void mean9_batch(BatchTable* tab,
                                                                             uint32_t gate)
{
    __shared__ __align__(16) M9SmemAny<R, kMean9TY> sm;
    __shared__ int s_tile, s_job;
    constexpr int n = (2 * R + 1) * (2 * R + 1) * (2 * R + 1);
    const double inv9n = 1.0 / (9.0 * n);
    BatchQueue* q = &tab->q[R - 1];
    int t, j;
    while (next_tile(tab, q, &s_tile, &s_job, &t, &j)) {
        const BatchJobDesc d = tab->jobs[j];
        const int local = t - d.tile_begin;
        const int bx = local % d.tiles_x;
        const int rest = local / d.tiles_x;
        const int by = rest % d.tiles_y;
        const int bz = rest / d.tiles_y;
        const Geom g{d.nx, d.ny, d.nz};
        const int z0 = bz * d.zs, z1 = min(z0 + d.zs, d.nz);
        const int x0 = bx * 64, y0 = by * kMean9TY;
        if (d.dtype == LNF_U8)
            mean9_tile<R, kMean9TY, uint8_t, GATE>(sm, d.pairs != 0, (const uint8_t*)d.in,
                                                   (uint8_t*)d.out, g, x0, y0, z0, z1, gate,
                                                   inv9n);
        else
            mean9_tile<R, kMean9TY, uint16_t, GATE>(sm, d.pairs != 0, (const uint16_t*)d.in,
                                                    (uint16_t*)d.out, g, x0, y0, z0, z1, gate,
                                                    inv9n);
    }
}

template <int R, bool GATE>
__global__ __launch_bounds__(256) void minvar9_batch(BatchTable* tab, uint32_t gate)
{
    __shared__ __align__(16) MV9Smem<R> sm;
    __shared__ int s_tile, s_job;
    constexpr int n = (2 * R + 1) * (2 * R + 1) * (2 * R + 1);
    const double dn = (double)n, invn = 1.0 / n;
    BatchQueue* q = &tab->q[R - 1];
    int t, j;
    while (next_tile(tab, q, &s_tile, &s_job, &t, &j)) {
        const BatchJobDesc d = tab->jobs[j];
        const int local = t - d.tile_begin;
        const int bx = local % d.tiles_x;
        const int rest = local / d.tiles_x;
        const int by = rest % d.tiles_y;
        const int bz = rest / d.tiles_y;
        const Geom g{d.nx, d.ny, d.nz};
        const int z0 = bz * d.zs, z1 = min(z0 + d.zs, d.nz);
        if (d.dtype == LNF_U8)
            minvar9_tile<R, uint8_t, GATE>(sm, (const uint8_t*)d.in, (uint8_t*)d.out, g, bx * 32,
                                           by * 8, z0, z1, gate, dn, invn);
        else
            minvar9_tile<R, uint16_t, GATE>(sm, (const uint16_t*)d.in, (uint16_t*)d.out, g,
                                            bx * 32, by * 8, z0, z1, gate, dn, invn);
    }
}

using BatchKernel = void (*)(BatchTable*, uint32_t);

BatchKernel batch_kernel(int rule, int r, bool gate)
{
#define LNF_PICK(K)                                                                  \
    switch (r) {                                                                     \
    case 1: return gate ? (BatchKernel)K<1, true> : (BatchKernel)K<1, false>;         \
    case 2: return gate ? (BatchKernel)K<2, true> : (BatchKernel)K<2, false>;         \
    case 3: return gate ? (BatchKernel)K<3, true> : (BatchKernel)K<3, false>;         \
    default: return gate ? (BatchKernel)K<4, true> : (BatchKernel)K<4, false>;        \
    }
    if (rule == LNF_MEAN9) {
        LNF_PICK(mean9_batch)
    }
    LNF_PICK(minvar9_batch)
#undef LNF_PICK
}

int batch_threads(int rule, int r)
{
    if (rule == LNF_MEAN9) {
        switch (r) {
        case 1: return M9Shape<1, kMean9TY>::THREADS;
        case 2: return M9Shape<2, kMean9TY>::THREADS;
        case 3: return M9Shape<3, kMean9TY>::THREADS;
        default: return M9Shape<4, kMean9TY>::THREADS;
        }
    }
    return 256;
}

struct BatchSlot {
    BatchTable* host = nullptr;  // pinned staging copy of the table
    BatchTable* dev = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t copy = nullptr;
    hipEvent_t done = nullptr;
    bool pending = false;
};

}  // namespace

struct BatchState {
    std::mutex mu;
    BatchSlot slot[kSlots];
    int next = 0;
    int grid[LNF_RADIUS_MAX] = {0, 0, 0, 0};
};

namespace {

void free_slot(BatchSlot& s)
{
    if (s.done) {
        (void)hipEventSynchronize(s.done);
        (void)hipEventDestroy(s.done);
    }
    if (s.exec) (void)hipGraphExecDestroy(s.exec);
    if (s.graph) (void)hipGraphDestroy(s.graph);
    if (s.dev) (void)hipFree(s.dev);
    if (s.host) (void)hipHostFree(s.host);
    s = BatchSlot{};
}

int build_slot(const lnf_ctx* h, BatchState* st, BatchSlot& s)
{
    if (hipHostMalloc((void**)&s.host, sizeof(BatchTable), hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void**)&s.dev, sizeof(BatchTable)) != hipSuccess) {
        (void)hipGetLastError();
        return LNF_ENOMEM;
    }
    std::memset(s.host, 0, sizeof(BatchTable));
    if (hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) return LNF_EHIP;
    if (hipGraphCreate(&s.graph, 0) != hipSuccess) return LNF_EHIP;
    if (hipGraphAddMemcpyNode1D(&s.copy, s.graph, nullptr, 0, s.dev, s.host, sizeof(BatchTable),
                                hipMemcpyHostToDevice) != hipSuccess)
        return LNF_EHIP;
    const bool gate = h->gate != 0;
    for (int r = 1; r <= LNF_RADIUS_MAX; ++r) {
        BatchTable* tab = s.dev;
        uint32_t g = h->gate;
        void* args[] = {&tab, &g};
        hipKernelNodeParams p{};
        p.func = reinterpret_cast<void*>(batch_kernel(h->rule, r, gate));
        p.gridDim = dim3(st->grid[r - 1]);
        p.blockDim = dim3(batch_threads(h->rule, r));
        p.sharedMemBytes = 0;
        p.kernelParams = args;
        p.extra = nullptr;
        hipGraphNode_t kn;
        if (hipGraphAddKernelNode(&kn, s.graph, &s.copy, 1, &p) != hipSuccess) return LNF_EHIP;
    }
    if (hipGraphInstantiate(&s.exec, s.graph, nullptr, nullptr, 0) != hipSuccess) return LNF_EHIP;
    return LNF_OK;
}

int init_batch_state(lnf_ctx* h, BatchState** out)
{
    BatchState* st = new (std::nothrow) BatchState();
    if (!st) return LNF_ENOMEM;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, h->device) != hipSuccess) {
        delete st;
        return LNF_EHIP;
    }
    for (int r = 1; r <= LNF_RADIUS_MAX; ++r) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, reinterpret_cast<const void*>(batch_kernel(h->rule, r, h->gate != 0)),
                batch_threads(h->rule, r), 0) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        st->grid[r - 1] = prop.multiProcessorCount * per_cu;
    }
    *out = st;
    return LNF_OK;
}

// Default z-strip depth of a batch job: deep enough to keep the z-halo small,
// shallow enough to give the queue many tiles for load balance.
int batch_default_zs(int nz) { return std::min(nz, 128); }

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
    {
        std::lock_guard<std::mutex> lk(h->mu);
        if (!h->batch) {
            BatchState* st = nullptr;
            const int rc = init_batch_state(h, &st);
            if (rc) return rc;
            h->batch = st;
        }
    }
    BatchState* st = h->batch;
    std::lock_guard<std::mutex> lk(st->mu);
    BatchSlot& s = st->slot[st->next];
    st->next = (st->next + 1) % kSlots;
    if (!s.exec) {
        const int rc = build_slot(h, st, s);
        if (rc) {
            free_slot(s);
            return rc;
        }
    }
    if (s.pending && hipEventSynchronize(s.done) != hipSuccess) return LNF_EHIP;
    s.pending = false;

    // order: by class, then larger jobs first (their tiles enter the queue first)
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b) {
        if (jobs[a].radius != jobs[b].radius) return jobs[a].radius < jobs[b].radius;
        const double va = (double)geoms[a].nx * geoms[a].ny * geoms[a].nz;
        const double vb = (double)geoms[b].nx * geoms[b].ny * geoms[b].nz;
        if (va != vb) return va > vb;
        return a < b;
    });
    BatchTable* tab = s.host;
    std::memset(tab->q, 0, sizeof(tab->q));
    int tx = 64, ty = 16;
    if (h->rule == LNF_MEAN9) mean9_tile_shape(1, &tx, &ty);
    else minvar9_tile_shape(0, &tx, &ty);
    for (int k = 0; k < n; ++k) {
        const int i = order[k];
        const Geom& g = geoms[i];
        BatchQueue& q = tab->q[jobs[i].radius - 1];
        if (q.njobs == 0) q.job_begin = k;
        BatchJobDesc& d = tab->jobs[k];
        d.in = jobs[i].in;
        d.out = jobs[i].out;
        d.nx = g.nx;
        d.ny = g.ny;
        d.nz = g.nz;
        d.dtype = jobs[i].dtype;
        d.pairs = mean9_pairs_ok(d.in, g.nx, jobs[i].dtype == LNF_U8 ? 1 : 2) ? 1 : 0;
        const TileCfg cfg = ctx_tile(h, h->rule, jobs[i].dtype, jobs[i].radius, g);
        d.zs = cfg.zs > 0 ? std::min(cfg.zs, g.nz) : batch_default_zs(g.nz);
        d.tiles_x = (g.nx + tx - 1) / tx;
        d.tiles_y = (g.ny + ty - 1) / ty;
        const long long tiles = (long long)d.tiles_x * d.tiles_y * ((g.nz + d.zs - 1) / d.zs);
        if ((long long)q.total + tiles > INT32_MAX) return LNF_EINVAL;
        d.tile_begin = q.total;
        q.total += (int)tiles;
        q.njobs += 1;
    }
    const size_t used = offsetof(BatchTable, jobs) + (size_t)std::max(n, 1) * sizeof(BatchJobDesc);
    if (hipGraphExecMemcpyNodeSetParams1D(s.exec, s.copy, s.dev, s.host, used,
                                          hipMemcpyHostToDevice) != hipSuccess)
        return LNF_EHIP;
    if (hipGraphLaunch(s.exec, stream) != hipSuccess) return LNF_EHIP;
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
