// C ABI of the local noise filter: argument validation, context state and
// dispatch to the HIP kernels.  Declarations and the contract: include/lnf.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>

#include "lnf.h"
#include "lnf_internal.h"
#include "lnf_ctx.h"

namespace lnf {

// z-strip depth of a launch over tiles_xy tile columns.  The strip count
// minimises (rounds of resident workgroups) x (slices per strip + the slices a
// strip reads beyond its own), so the last round is not a thin tail; strips
// are no shallower than 16 slices.
int default_zs(int tiles_xy, int nz, int target_groups)
{
    constexpr int kMinDepth = 16;  // shallower strips re-read too much z-halo
    constexpr int kHalo = 12;      // extra slices per strip (4r at r = 3)
    tiles_xy = std::max(tiles_xy, 1);
    target_groups = std::max(target_groups, 1);
    const int max_nzs = std::max(1, (nz + kMinDepth - 1) / kMinDepth);
    int best = 1;
    long long best_cost = -1;
    for (int nzs = 1; nzs <= max_nzs; ++nzs) {
        const long long rounds = ((long long)tiles_xy * nzs + target_groups - 1) / target_groups;
        const long long cost = rounds * ((nz + nzs - 1) / nzs + kHalo);
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = nzs;
        }
    }
    return (nz + best - 1) / best;
}

int resident_groups(const void* kernel, int threads)
{
    constexpr int kMaxDev = 64;
    static std::atomic<int> cus[kMaxDev];  // CU count per device, 0 = not queried yet
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, int> per_cu;  // resident groups per CU
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) {
        (void)hipGetLastError();
        return 1024;
    }
    int n = cus[dev].load(std::memory_order_relaxed);
    if (n <= 0) {
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            n <= 0) {
            (void)hipGetLastError();
            n = 256;
        }
        cus[dev].store(n, std::memory_order_relaxed);
    }
    int k = 0;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = per_cu.find({kernel, threads});
        if (it != per_cu.end()) {
            k = it->second;
        } else {
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&k, kernel, threads, 0) != hipSuccess ||
                k <= 0) {
                (void)hipGetLastError();
                k = 2;
            }
            per_cu[{kernel, threads}] = k;
        }
    }
    return n * k;
}

int check_volume_args(const lnf_ctx* h, const void* vol, const int64_t dims[3], int dtype,
                      int radius, const void* out, Geom* g, size_t* bytes)
{
    if (!h || !vol || !out || !dims) return LNF_EINVAL;
    if (dtype != LNF_U8 && dtype != LNF_U16) return LNF_EINVAL;
    if (radius < 1 || radius > LNF_RADIUS_MAX) return LNF_EINVAL;
    for (int i = 0; i < 3; ++i)
        if (dims[i] < 1 || dims[i] > INT_MAX) return LNF_EINVAL;
    if (dims[0] * dims[1] > INT_MAX) return LNF_EINVAL;
    const size_t es = dtype == LNF_U8 ? 1 : 2;
    const size_t nbytes = (size_t)dims[0] * (size_t)dims[1] * (size_t)dims[2] * es;
    const uintptr_t a = (uintptr_t)vol, b = (uintptr_t)out;
    if (a < b + nbytes && b < a + nbytes) return LNF_EINVAL;  // stencil: no in-place
    g->nx = (int)dims[0];
    g->ny = (int)dims[1];
    g->nz = (int)dims[2];
    *bytes = nbytes;
    return LNF_OK;
}

// The pointer must be device memory of `device` with `bytes` bytes behind it.
int check_device_range(const void* p, size_t bytes, int device)
{
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return LNF_EDEVICE;
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged) return LNF_EDEVICE;
    if (attr.device != device) return LNF_EDEVICE;
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p) != hipSuccess) {
        (void)hipGetLastError();
        return LNF_EDEVICE;
    }
    const uintptr_t lo = (uintptr_t)base, hi = lo + size, q = (uintptr_t)p;
    if (q < lo || q + bytes > hi) return LNF_EINVAL;
    return LNF_OK;
}

// Make the context's device current for the duration of a call.
DeviceGuard::DeviceGuard(int dev)
{
    if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
    if (prev_ != dev) {
        ok_ = hipSetDevice(dev) == hipSuccess;
        switched_ = true;
    }
}

DeviceGuard::~DeviceGuard()
{
    if (switched_ && prev_ >= 0) (void)hipSetDevice(prev_);
}

TileCfg ctx_tile(const lnf_ctx* h, int rule, int dtype, int radius, Geom g)
{
    TileCfg cfg{-1, 0};  // -1: the rule's default variant
    const TuneKey key = tune_key(rule, dtype, radius, g);
    std::lock_guard<std::mutex> lk(h->mu);
    auto it = h->tuned.find(key);
    if (it != h->tuned.end()) cfg = it->second;
    return cfg;
}

hipError_t launch_rule(int rule, uint32_t geom, const void* in, void* out, int dtype, int r,
                       Geom g, uint32_t gate, TileCfg cfg, hipStream_t s, TileCfg* plan)
{
    if (geom) return launch_geometry(rule, geom, in, out, dtype, r, g, gate, cfg.zs, s, plan);
    if (rule == LNF_MEAN9) return launch_mean9(in, out, dtype, r, g, gate, cfg, s, plan);
    return launch_minvar9(in, out, dtype, r, g, gate, cfg, s, plan);
}

TuneKey tune_key(int rule, int dtype, int radius, Geom g)
{
    // size class: log2 of the voxel count, so one tuning covers similar volumes
    const double vox = (double)g.nx * g.ny * g.nz;
    int cls = 0;
    while (cls < 40 && (double)(1ull << cls) < vox) ++cls;
    return ((uint64_t)rule << 48) | ((uint64_t)dtype << 40) | ((uint64_t)radius << 32) |
           (uint64_t)cls;
}

int ctx_init_device_state(lnf_ctx* c)
{
    c->dev_state = nullptr;
    DeviceGuard dg(c->device);
    if (!dg.ok()) return LNF_EHIP;
    const int rc = batch_state_init(c);
    if (rc != LNF_OK) batch_state_free(c);
    return rc;
}

void ctx_free_device_state(lnf_ctx* c)
{
    batch_state_free(c);
    otsu_scratch_free(c);
    entropy_scratch_free(c);
    c->dev_state = nullptr;
}

}  // namespace lnf

using namespace lnf;

extern "C" {

int lnf_version(void) { return 10000; }

const char* lnf_strerror(int code)
{
    switch (code) {
    case LNF_OK: return "success";
    case LNF_EINVAL: return "invalid argument";
    case LNF_EDEVICE: return "pointer is not device memory of the context's device";
    case LNF_ENOMEM: return "out of memory";
    case LNF_EHIP: return "HIP runtime error";
    case LNF_EBUSY: return "admission would exceed the memory cap";
    case LNF_ENOTFOUND: return "unknown volume id or ticket";
    case LNF_ECANCELED: return "request cancelled or failed";
    case LNF_ETIMEDOUT: return "timed out";
    case LNF_ERANGE: return "more jobs than the static job table of lnf_filter_batch_noalloc holds";
    default: return "unknown status code";
    }
}

int lnf_create(lnf_handle* h, const lnf_options* opt)
{
    if (!h) return LNF_EINVAL;
    *h = nullptr;
    lnf_options o{sizeof(lnf_options), LNF_MEAN9, 0, -1, 0};
    if (opt) {
        if (opt->size < sizeof(lnf_options)) return LNF_EINVAL;
        o = *opt;
    }
    if (o.rule != LNF_MEAN9 && o.rule != LNF_MINVAR9) return LNF_EINVAL;
    constexpr uint32_t kGeom = LNF_GEOM_CROSS | LNF_GEOM_OFFSET_1 | LNF_GEOM_OFFSET_2R1;
    if ((o.flags & ~kGeom) ||
        (o.flags & (LNF_GEOM_OFFSET_1 | LNF_GEOM_OFFSET_2R1)) == (LNF_GEOM_OFFSET_1 | LNF_GEOM_OFFSET_2R1))
        return LNF_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        return LNF_EDEVICE;
    }
    int dev = o.device;
    if (dev < 0 && hipGetDevice(&dev) != hipSuccess) return LNF_EHIP;
    if (dev >= ndev) return LNF_EDEVICE;
    lnf_ctx* c = new (std::nothrow) lnf_ctx();
    if (!c) return LNF_ENOMEM;
    c->device = dev;
    c->rule = o.rule;
    c->gate = o.gate_T;
    c->geom = o.flags;
    const int rc = ctx_init_device_state(c);
    if (rc != LNF_OK) {
        delete c;
        return rc;
    }
    if (const char* cache = std::getenv("LNF_TUNE_CACHE")) (void)lnf_tune_load(c, cache);
    *h = c;
    return LNF_OK;
}

int lnf_destroy(lnf_handle h)
{
    if (!h) return LNF_OK;
    {
        DeviceGuard dg(h->device);
        ctx_free_device_state(h);
    }
    delete h;
    return LNF_OK;
}

int lnf_tile_variants(int rule, int dtype, int radius)
{
    if (dtype != LNF_U8 && dtype != LNF_U16) return LNF_EINVAL;
    if (radius < 1 || radius > LNF_RADIUS_MAX) return LNF_EINVAL;
    if (rule == LNF_MEAN9) return mean9_variants();
    if (rule == LNF_MINVAR9) return minvar9_variants();
    return LNF_EINVAL;
}

int lnf_filter_tiled(lnf_handle h, const void* vol, const int64_t dims[3], int dtype, int radius,
                     void* out, hipStream_t stream, const lnf_tile* tile)
{
    Geom g;
    size_t bytes = 0;
    int rc = check_volume_args(h, vol, dims, dtype, radius, out, &g, &bytes);
    if (rc) return rc;
    TileCfg cfg = ctx_tile(h, h->rule, dtype, radius, g);
    if (tile) {
        const int nv = h->rule == LNF_MEAN9 ? mean9_variants() : minvar9_variants();
        if (tile->variant >= nv || tile->variant < -1 || tile->zs < 0) return LNF_EINVAL;
        if (tile->variant >= 0) cfg.variant = tile->variant;
        if (tile->zs > 0) cfg.zs = tile->zs;
    }
    DeviceGuard dg(h->device);
    if (!dg.ok()) return LNF_EHIP;
    if ((rc = check_device_range(vol, bytes, h->device))) return rc;
    if ((rc = check_device_range(out, bytes, h->device))) return rc;
    if (launch_rule(h->rule, h->geom, vol, out, dtype, radius, g, h->gate, cfg, stream) !=
        hipSuccess)
        return LNF_EHIP;
    return LNF_OK;
}

int lnf_tile_config(lnf_handle h, const int64_t dims[3], int dtype, int radius, lnf_tile* tile)
{
    if (!h || !dims || !tile) return LNF_EINVAL;
    if (dtype != LNF_U8 && dtype != LNF_U16) return LNF_EINVAL;
    if (radius < 1 || radius > LNF_RADIUS_MAX) return LNF_EINVAL;
    for (int i = 0; i < 3; ++i)
        if (dims[i] < 1 || dims[i] > INT_MAX) return LNF_EINVAL;
    if (dims[0] * dims[1] > INT_MAX) return LNF_EINVAL;
    const Geom g{(int)dims[0], (int)dims[1], (int)dims[2]};
    TileCfg plan{-1, 0};
    DeviceGuard dg(h->device);
    if (!dg.ok()) return LNF_EHIP;
    if (launch_rule(h->rule, h->geom, nullptr, nullptr, dtype, radius, g, h->gate,
                    ctx_tile(h, h->rule, dtype, radius, g), nullptr, &plan) != hipSuccess)
        return LNF_EHIP;
    tile->variant = plan.variant;
    tile->zs = plan.zs;
    return LNF_OK;
}

int lnf_filter(lnf_handle h, const void* vol, const int64_t dims[3], int dtype, int radius,
               void* out, hipStream_t stream)
{
    return lnf_filter_tiled(h, vol, dims, dtype, radius, out, stream, nullptr);
}

}  // extern "C"
