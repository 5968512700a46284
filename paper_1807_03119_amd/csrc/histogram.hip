// Grey-level histogram of a volume and Otsu's data threshold (paper, Section
// "Our Method", eq. 1), and the paper's automatic pipeline: threshold, then
// the nine-cluster filter gated at that threshold.
//
// Histogram kernels privatise the bins in LDS and flush them with global
// atomics once per workgroup:
//   - uint8: 256 uint32 counters per workgroup;
//   - uint16: 65536 bins as two 16-bit counters per LDS word (128 KiB of the
//     160 KiB LDS, one 1024-thread workgroup per CU); a workgroup takes at
//     most 65528 voxels (eight per 16-byte load), so neither half of a word
//     can carry into the other.
// The output histogram is cleared by a fill kernel (no memset node), so the
// sequence can be captured in a graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>

#include "device_common.h"
#include "lnf.h"
#include "lnf_ctx.h"
#include "lnf_internal.h"

namespace lnf {
namespace {

constexpr int kThreads = 256;
constexpr int kThreads16 = 1024;  // uint16: one 128 KiB workgroup per CU, 16 waves
constexpr int kChunk16 = 65528;   // voxels per uint16 workgroup: below 65536, a multiple of 8

__global__ __launch_bounds__(kThreads) void fill_u64(unsigned long long* p, int n)
{
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) p[i] = 0;
}

__global__ __launch_bounds__(kThreads) void hist_u8(const uint8_t* __restrict__ in, size_t n,
                                                     size_t chunk, unsigned long long* hist)
{
    __shared__ uint32_t bins[256];
    bins[threadIdx.x] = 0;
    __syncthreads();
    const size_t begin = (size_t)blockIdx.x * chunk;
    const size_t end = begin + chunk < n ? begin + chunk : n;
    for (size_t i = begin + threadIdx.x; i < end; i += kThreads) atomicAdd(&bins[in[i]], 1u);
    __syncthreads();
    const uint32_t c = bins[threadIdx.x];
    if (c) atomicAdd(&hist[threadIdx.x], (unsigned long long)c);
}

__global__ __launch_bounds__(kThreads16) void hist_u16(const uint16_t* __restrict__ in, size_t n,
                                                        unsigned long long* hist, int vec)
{
    __shared__ uint32_t pairs[32768];  // bin 2i in the low half, bin 2i+1 in the high half
    for (int i = threadIdx.x; i < 32768; i += kThreads16) pairs[i] = 0;
    __syncthreads();
    const size_t begin = (size_t)blockIdx.x * kChunk16;
    const size_t end = begin + kChunk16 < n ? begin + kChunk16 : n;
    auto add = [&](uint32_t v) { atomicAdd(&pairs[v >> 1], (v & 1) ? 65536u : 1u); };
    size_t tail = begin;
    if (vec) {
        // 16-byte aligned volume: eight voxels per load (begin is a multiple
        // of 8 voxels, so every workgroup's range starts aligned)
        const size_t nv = (end - begin) / 8;
        const uint4* p = reinterpret_cast<const uint4*>(in + begin);
        for (size_t i = threadIdx.x; i < nv; i += kThreads16) {
            const uint4 w = p[i];
            add(w.x & 0xffffu);
            add(w.x >> 16);
            add(w.y & 0xffffu);
            add(w.y >> 16);
            add(w.z & 0xffffu);
            add(w.z >> 16);
            add(w.w & 0xffffu);
            add(w.w >> 16);
        }
        tail = begin + nv * 8;
    }
    for (size_t i = tail + threadIdx.x; i < end; i += kThreads16) add(in[i]);
    __syncthreads();
    for (int i = threadIdx.x; i < 32768; i += kThreads16) {
        const uint32_t w = pairs[i];
        if (w & 0xffffu) atomicAdd(&hist[2 * i], (unsigned long long)(w & 0xffffu));
        if (w >> 16) atomicAdd(&hist[2 * i + 1], (unsigned long long)(w >> 16));
    }
}

// ---- exact Otsu on the host ------------------------------------------------
// Fixed-width unsigned integers of 12 x 64 bits (least significant limb
// first): wide enough for every product below with counts up to 2^64.
struct Big {
    static constexpr int L = 12;
    uint64_t w[L] = {};
};

Big big(unsigned __int128 v)
{
    Big r;
    r.w[0] = (uint64_t)v;
    r.w[1] = (uint64_t)(v >> 64);
    return r;
}

Big mul(const Big& a, const Big& b)
{
    Big r;
    for (int i = 0; i < Big::L; ++i) {
        if (!a.w[i]) continue;
        unsigned __int128 carry = 0;
        for (int j = 0; i + j < Big::L; ++j) {
            const unsigned __int128 cur = (unsigned __int128)a.w[i] * b.w[j] + r.w[i + j] + carry;
            r.w[i + j] = (uint64_t)cur;
            carry = cur >> 64;
        }
    }
    return r;
}

int cmp(const Big& a, const Big& b)
{
    for (int i = Big::L - 1; i >= 0; --i)
        if (a.w[i] != b.w[i]) return a.w[i] < b.w[i] ? -1 : 1;
    return 0;
}

Big sub(const Big& a, const Big& b)  // a >= b
{
    Big r;
    unsigned __int128 borrow = 0;
    for (int i = 0; i < Big::L; ++i) {
        const unsigned __int128 x = (unsigned __int128)a.w[i] - b.w[i] - borrow;
        r.w[i] = (uint64_t)x;
        borrow = (x >> 64) ? 1 : 0;
    }
    return r;
}

}  // namespace

// T maximising the between-class variance (N*s0 - n0*S)^2 / (n0*n1), which is
// the T minimising eq. 1's within-class variance (their sum is the constant
// total variance).  Class 0 is v < T; lowest T among maxima; with fewer than
// two levels present, T = the present level (0 for an empty histogram).
// Exact for any counts: N < 2^64, S < 2^80, every product below < 2^640.
uint32_t otsu_from_hist(const uint64_t* hist, int levels)
{
    unsigned __int128 N = 0, S = 0;
    for (int v = 0; v < levels; ++v) {
        N += hist[v];
        S += (unsigned __int128)hist[v] * (unsigned)v;
    }
    const Big bN = big(N), bS = big(S);
    unsigned __int128 n0 = 0, s0 = 0;
    int best_t = -1;
    Big best_num, best_den;
    for (int t = 1; t < levels; ++t) {
        // an empty level t-1 leaves both classes, so the criterion, as they
        // were at t-1: a tie, which the lower threshold keeps
        if (!hist[t - 1]) continue;
        n0 += hist[t - 1];
        s0 += (unsigned __int128)hist[t - 1] * (unsigned)(t - 1);
        const unsigned __int128 n1 = N - n0;
        if (n0 == 0 || n1 == 0) continue;
        const Big a = mul(bN, big(s0)), b = mul(big(n0), bS);
        const Big d = cmp(a, b) >= 0 ? sub(a, b) : sub(b, a);
        const Big num = mul(d, d);
        const Big den = mul(big(n0), big(n1));
        if (best_t < 0 || cmp(mul(num, best_den), mul(best_num, den)) > 0) {
            best_t = t;
            best_num = num;
            best_den = den;
        }
    }
    if (best_t >= 0) return (uint32_t)best_t;
    for (int v = 0; v < levels; ++v)
        if (hist[v]) return (uint32_t)v;
    return 0;
}

hipError_t launch_histogram(const void* vol, size_t n, int dtype, uint64_t* hist, hipStream_t s)
{
    const int levels = dtype == LNF_U8 ? 256 : 65536;
    auto* h = reinterpret_cast<unsigned long long*>(hist);
    hipLaunchKernelGGL(fill_u64, dim3((levels + kThreads - 1) / kThreads), dim3(kThreads), 0, s, h,
                       levels);
    if (n == 0) return hipGetLastError();
    if (dtype == LNF_U8) {
        const size_t groups = std::min<size_t>(4096, (n + 65535) / 65536);
        const size_t chunk = (n + groups - 1) / groups;
        hipLaunchKernelGGL(hist_u8, dim3((unsigned)groups), dim3(kThreads), 0, s,
                           static_cast<const uint8_t*>(vol), n, chunk, h);
    } else {
        const size_t groups = (n + kChunk16 - 1) / kChunk16;
        const int vec = (reinterpret_cast<uintptr_t>(vol) % 16) == 0;
        hipLaunchKernelGGL(hist_u16, dim3((unsigned)groups), dim3(kThreads16), 0, s,
                           static_cast<const uint16_t*>(vol), n, h, vec);
    }
    return hipGetLastError();
}

}  // namespace lnf

namespace lnf {

void otsu_scratch_free(lnf_ctx* h)
{
    if (h->otsu_dev) (void)hipFree(h->otsu_dev);
    if (h->otsu_host) (void)hipHostFree(h->otsu_host);
    h->otsu_dev = nullptr;
    h->otsu_host = nullptr;
}

}  // namespace lnf

using namespace lnf;

extern "C" int lnf_histogram(lnf_handle h, const void* vol, const int64_t dims[3], int dtype,
                             uint64_t* hist, hipStream_t stream)
{
    if (!h || !vol || !hist || !dims || (dtype != LNF_U8 && dtype != LNF_U16)) return LNF_EINVAL;
    for (int i = 0; i < 3; ++i)
        if (dims[i] < 1 || dims[i] > INT32_MAX) return LNF_EINVAL;
    const size_t n = (size_t)dims[0] * (size_t)dims[1] * (size_t)dims[2];
    const size_t bytes = n * (dtype == LNF_U8 ? 1 : 2);
    const size_t hbytes = (dtype == LNF_U8 ? 256 : 65536) * sizeof(uint64_t);
    const uintptr_t a = (uintptr_t)vol, b = (uintptr_t)hist;
    if (a < b + hbytes && b < a + bytes) return LNF_EINVAL;
    DeviceGuard dg(h->device);
    if (!dg.ok()) return LNF_EHIP;
    int rc;
    if ((rc = check_device_range(vol, bytes, h->device))) return rc;
    if ((rc = check_device_range(hist, hbytes, h->device))) return rc;
    return launch_histogram(vol, n, dtype, hist, stream) == hipSuccess ? LNF_OK : LNF_EHIP;
}

extern "C" int lnf_otsu_threshold(const uint64_t* hist, int levels, uint32_t* T)
{
    if (!hist || !T || levels < 1 || levels > 65536) return LNF_EINVAL;
    *T = otsu_from_hist(hist, levels);
    return LNF_OK;
}

extern "C" int lnf_filter_otsu(lnf_handle h, const void* vol, const int64_t dims[3], int dtype,
                               int radius, void* out, hipStream_t stream, uint32_t* T)
{
    Geom g;
    size_t bytes = 0;
    int rc = check_volume_args(h, vol, dims, dtype, radius, out, &g, &bytes);
    if (rc) return rc;
    DeviceGuard dg(h->device);
    if (!dg.ok()) return LNF_EHIP;
    if ((rc = check_device_range(vol, bytes, h->device))) return rc;
    if ((rc = check_device_range(out, bytes, h->device))) return rc;
    std::lock_guard<std::mutex> lk(h->otsu_mu);
    if (!h->otsu_dev) {
        if (hipMalloc((void**)&h->otsu_dev, 65536 * sizeof(uint64_t)) != hipSuccess ||
            hipHostMalloc((void**)&h->otsu_host, 65536 * sizeof(uint64_t),
                          hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            otsu_scratch_free(h);
            return LNF_ENOMEM;
        }
    }
    const int levels = dtype == LNF_U8 ? 256 : 65536;
    const size_t n = (size_t)g.nx * g.ny * g.nz;
    if (launch_histogram(vol, n, dtype, h->otsu_dev, stream) != hipSuccess) return LNF_EHIP;
    if (hipMemcpyAsync(h->otsu_host, h->otsu_dev, levels * sizeof(uint64_t),
                       hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return LNF_EHIP;
    const uint32_t t = otsu_from_hist(h->otsu_host, levels);
    if (T) *T = t;
    if (launch_rule(h->rule, h->geom, vol, out, dtype, radius, g, t,
                    ctx_tile(h, h->rule, dtype, radius, g), stream) != hipSuccess)
        return LNF_EHIP;
    return LNF_OK;
}
