// The paper's comparison filters (Section "Other Filters"), as second
// workloads beside the nine-cluster filter:
//   - mean (eq. 4): the box term of the MEAN9 streaming tile (mean9.hip,
//     launch_box_mean);
//   - sigma (eq. 5), Okada (eq. 6): data-dependent window filters, computed
//     by a direct window kernel.  A workgroup streams a 32 x 8 output column
//     down z with an LDS ring of the last 2r+1 raw planes ((32+2r) x (8+2r)
//     voxels each); every thread evaluates one output voxel per slice from
//     the ring;
//   - entropy (eq. 7): the window sum of per-voxel weights is a box sum, run
//     separably (entropy_box).
// Readings of the formulas (garbled or silent in the paper) follow the
// declarations in include/lnf.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "device_common.h"
#include "lnf.h"
#include "lnf_ctx.h"
#include "lnf_internal.h"

namespace lnf {
namespace {

constexpr int kWX = 32, kWY = 8, kWThreads = 256;

template <int R, typename T, int KIND>
__global__ __launch_bounds__(kWThreads) void window_planes(const T* __restrict__ in,
                                                           T* __restrict__ out, Geom g, int zs,
                                                           int tiles_x, int tiles_y, int total,
                                                           int64_t param,
                                                           const int64_t* __restrict__ weights,
                                                           uint32_t gate)
{
    constexpr int LX = kWX + 2 * R, LY = kWY + 2 * R, NPL = 2 * R + 1;
    constexpr int NRAW = LX * LY, NLOAD = (NRAW + kWThreads - 1) / kWThreads;
    static_assert(KIND == kWinSigma || KIND == kWinOkada, "entropy runs on entropy_box");
    // planes of the window loop unrolled only at r = 1: a fully unrolled
    // (2r+1)^3 window hoists all its LDS reads (266 VGPRs at r = 3)
    constexpr int UZ = R <= 1 ? NPL : 1;
    __shared__ uint32_t raw[NPL][NRAW];

    const int tile = xcd_tile(blockIdx.x, total);
    const int bx = tile % tiles_x;
    const int rest = tile / tiles_x;
    const int by = rest % tiles_y;
    const int bz = rest / tiles_y;
    const int x0 = bx * kWX, y0 = by * kWY, z0 = bz * zs, z1 = min(z0 + zs, g.nz);
    const int tid = threadIdx.x;
    const size_t plane = (size_t)g.nx * g.ny;
    const uint32_t pbytes = (uint32_t)(plane * sizeof(T));

    uint32_t off[NLOAD];
#pragma unroll
    for (int i = 0; i < NLOAD; ++i) {
        const int e = min(tid + i * kWThreads, NRAW - 1);
        const int row = e / LX, col = e - row * LX;
        off[i] = (uint32_t)(clampi(y0 - R + row, 0, g.ny - 1) * g.nx +
                            clampi(x0 - R + col, 0, g.nx - 1)) * (uint32_t)sizeof(T);
    }
    uint32_t v[NLOAD];
    auto load = [&](int zi) {
        const rsrc_t rs = make_rsrc(in + (size_t)clampi(zi, 0, g.nz - 1) * plane, pbytes);
#pragma unroll
        for (int i = 0; i < NLOAD; ++i) v[i] = buffer_load<T>(rs, off[i]);
    };

    const int ox = tid % kWX, oy = tid / kWX;
    const int ns = (z1 - z0) + 2 * R;  // input slices z0-r .. z1-1+r
    load(z0 - R);
    for (int k = 0; k < ns; ++k) {
        const int slot = k % NPL;
#pragma unroll
        for (int i = 0; i < NLOAD; ++i) {
            const int e = tid + i * kWThreads;
            if (e < NRAW) raw[slot][e] = v[i];
        }
        if (k + 1 < ns) load(z0 - R + k + 1);
        barrier_lds();
        if (k >= 2 * R) {  // output slice z = (slice k) - r: planes k-2r .. k
            const int z = z0 + k - 2 * R;
            const int cslot = (k - R) % NPL;
            const int c = (oy + R) * LX + ox + R;
            const uint32_t p0 = raw[cslot][c];
            uint32_t o = 0;
            if constexpr (KIND == kWinOkada) {
                // centre and six face neighbours (r = 1)
                const uint32_t nb[7] = {p0, raw[cslot][c - 1], raw[cslot][c + 1],
                                        raw[cslot][c - LX], raw[cslot][c + LX],
                                        raw[(k - 2) % NPL][c], raw[k % NPL][c]};
                // |w - p0| < param  <=>  lo <= w <= hi with lo = p0 - param + 1,
                // hi = p0 + param - 1, tested as (w - lo) <= hi - lo; no value
                // passes when param <= 0
                uint32_t sum = 0, cnt = 0;
                if (param > 0) {
                    const int64_t lo64 = (int64_t)p0 - param + 1;
                    const uint64_t hi64 = (uint64_t)p0 + (uint64_t)param - 1;
                    const uint32_t lo = lo64 > 0 ? (uint32_t)lo64 : 0u;
                    const uint32_t span =
                        (uint32_t)(hi64 < 0xffffffffull ? hi64 : 0xffffffffull) - lo;
#pragma unroll
                    for (int i = 0; i < 7; ++i) {
                        const bool in = nb[i] - lo <= span;
                        sum += in ? nb[i] : 0u;
                        cnt += in ? 1u : 0u;
                    }
                }
                o = cnt ? (uint32_t)((double)(2 * sum + cnt) / (double)(2 * cnt)) : 0u;
            } else if constexpr (KIND == kWinSigma) {
                // |w - p0| <= param  <=>  lo <= w <= hi, tested as one unsigned
                // compare (w - lo) <= hi - lo (values and bounds below 2^32)
                const uint64_t hi64 = (uint64_t)p0 + (uint64_t)param;
                const uint32_t lo = (int64_t)p0 > param ? (uint32_t)((int64_t)p0 - param) : 0u;
                const uint32_t span = (uint32_t)(hi64 < 0xffffffffull ? hi64 : 0xffffffffull) - lo;
                uint32_t sum = 0, cnt = 0;
#pragma unroll UZ
                for (int dz = 0; dz < NPL; ++dz) {
                    const uint32_t* pl = raw[(k - 2 * R + dz) % NPL];
#pragma unroll
                    for (int dy = 0; dy <= 2 * R; ++dy)
#pragma unroll
                        for (int dx = 0; dx <= 2 * R; ++dx) {
                            const uint32_t w = pl[(oy + dy) * LX + ox + dx];
                            const bool in = w - lo <= span;
                            sum += in ? w : 0u;
                            cnt += in ? 1u : 0u;
                        }
                }
                // (2 sum + cnt) / (2 cnt) < 2^27 / 2: its fp64 quotient never
                // rounds across an integer, so truncation is the exact floor
                o = (uint32_t)((double)(2 * sum + cnt) / (double)(2 * cnt));
            }
            if (o < gate) o = 0;
            const int x = x0 + ox, y = y0 + oy;
            if (x < g.nx && y < g.ny) {
                const rsrc_t wr = make_rsrc(out + (size_t)z * plane, pbytes);
                buffer_store<T>(o, wr, (uint32_t)(y * g.nx + x) * (uint32_t)sizeof(T), 0);
            }
        }
        barrier_lds();  // the next slice overwrites the oldest plane
    }
}

// Entropy (eq. 7) as a box sum: the window's sum of per-voxel weights
// -p log2 p is the (2r+1)^3 box sum of the weight volume, computed separably.
// Each thread keeps, for its raw columns of the (32+2r) x (8+2r) tile, a
// register ring of the last 2r+1 weights and their running sum over z; the
// sums go to LDS, an x-pass sums 2r+1 columns, and each output thread sums
// 2r+1 rows.  Weights are below 2^32 (-p log2 p <= 0.531 in 2^-32 fixed point)
// and at most 729 of them are added, so the fp64 sums are exact integers.
template <int R, typename T>
__global__ __launch_bounds__(kWThreads) void entropy_box(const T* __restrict__ in,
                                                         T* __restrict__ out, Geom g, int zs,
                                                         int tiles_x, int tiles_y, int total,
                                                         int64_t param,
                                                         const int64_t* __restrict__ weights,
                                                         uint32_t gate)
{
    constexpr int M = 2 * R + 1;
    constexpr int LX = kWX + 2 * R, LY = kWY + 2 * R, NRAW = LX * LY;
    constexpr int NZ = (NRAW + kWThreads - 1) / kWThreads;
    constexpr int XS = 8, NXS = kWX / XS, XW = XS + 2 * R, XW2 = (XW + 1) / 2 * 2;
    constexpr int ZP = (NXS - 1) * XS + XW2 > LX ? (NXS - 1) * XS + XW2 : LX;  // even
    static_assert(LY * NXS <= kWThreads && ZP % 2 == 0, "entropy tile shape");
    __shared__ __align__(16) double zsum[LY * ZP + 2];
    __shared__ __align__(16) double xsum[LY * kWX];

    const int tile = xcd_tile(blockIdx.x, total);
    const int bx = tile % tiles_x;
    const int rest = tile / tiles_x;
    const int by = rest % tiles_y;
    const int bz = rest / tiles_y;
    const int x0 = bx * kWX, y0 = by * kWY, z0 = bz * zs, z1 = min(z0 + zs, g.nz);
    const int tid = threadIdx.x;
    const size_t plane = (size_t)g.nx * g.ny;
    const uint32_t pbytes = (uint32_t)(plane * sizeof(T));
    const uint32_t* w32 = reinterpret_cast<const uint32_t*>(weights);  // low halves

    uint32_t off[NZ];
    int zi[NZ];
#pragma unroll
    for (int i = 0; i < NZ; ++i) {
        const int e = min(tid + i * kWThreads, NRAW - 1);
        const int row = e / LX, col = e - row * LX;
        off[i] = (uint32_t)(clampi(y0 - R + row, 0, g.ny - 1) * g.nx +
                            clampi(x0 - R + col, 0, g.nx - 1)) * (uint32_t)sizeof(T);
        zi[i] = row * ZP + col;
    }
    const bool zlast = tid + (NZ - 1) * kWThreads < NRAW;
    auto wload = [&](uint32_t(&w)[NZ], int zsl) {
        const rsrc_t rs = make_rsrc(in + (size_t)clampi(zsl, 0, g.nz - 1) * plane, pbytes);
        uint32_t v[NZ];
#pragma unroll
        for (int i = 0; i < NZ; ++i) v[i] = buffer_load<T>(rs, off[i]);
#pragma unroll
        for (int i = 0; i < NZ; ++i) w[i] = w32[2 * v[i]];
    };
    const int ox = tid % kWX, oy = tid / kWX;
    const int x = x0 + ox, y = y0 + oy;
    const uint32_t soff = (x < g.nx && y < g.ny) ? (uint32_t)(y * g.nx + x) * (uint32_t)sizeof(T)
                                                 : pbytes;
    const int xrow = tid % LY, xseg = tid / LY;  // x-pass: consecutive lanes, consecutive rows

    // ring of the last 2r+1 weights per column and their sum, for slice z0-1
    uint32_t ring[M][NZ];
    double zw[NZ];
#pragma unroll
    for (int i = 0; i < NZ; ++i) zw[i] = 0.0;
#pragma unroll
    for (int u = 0; u < M; ++u) {
        wload(ring[u], z0 - 1 - R + u);  // slot u holds slice z0-1-r+u
#pragma unroll
        for (int i = 0; i < NZ; ++i) zw[i] += (double)ring[u][i];
    }
    uint32_t wn[NZ];
    wload(wn, z0 + R);
    for (int zb = z0; zb < z1; zb += M) {
#pragma unroll
        for (int u = 0; u < M; ++u) {
            const int z = zb + u;
            if (z >= z1) break;
            // slice z+r enters, slice z-r-1 (ring slot u) leaves
#pragma unroll
            for (int i = 0; i < NZ; ++i) {
                zw[i] += (double)wn[i] - (double)ring[u][i];
                ring[u][i] = wn[i];
                if (i < NZ - 1 || zlast) zsum[zi[i]] = zw[i];
            }
            wload(wn, z + 1 + R);
            const T p0 = in[(size_t)clampi(z, 0, g.nz - 1) * plane +
                            (size_t)clampi(y, 0, g.ny - 1) * g.nx + clampi(x, 0, g.nx - 1)];
            barrier_lds();
            if (xseg < NXS) {
                const double* rp = zsum + xrow * ZP + xseg * XS;
                double c[XW2];
#pragma unroll
                for (int i = 0; i < XW2; i += 2) {
                    const double2 t = *reinterpret_cast<const double2*>(rp + i);
                    c[i] = t.x;
                    c[i + 1] = t.y;
                }
#pragma unroll
                for (int i = 1; i < XW; ++i) c[i] += c[i - 1];
                double* dp = xsum + xrow * kWX + xseg * XS;
#pragma unroll
                for (int m = 0; m < XS; m += 2)
                    *reinterpret_cast<double2*>(dp + m) = make_double2(
                        c[m + 2 * R] - (m ? c[m - 1] : 0.0), c[m + 1 + 2 * R] - c[m]);
            }
            barrier_lds();
            double h = 0.0;
#pragma unroll
            for (int t = 0; t < M; ++t) h += xsum[(oy + t) * kWX + ox];
            uint32_t o = h > (double)param ? (uint32_t)p0 : 0u;
            if (o < gate) o = 0;
            const rsrc_t wr = make_rsrc(out + (size_t)z * plane, pbytes);
            buffer_store<T>(o, wr, soff, 0);
        }
    }
}

template <int R, typename T, int KIND>
hipError_t launch_win(const void* in, void* out, Geom g, int64_t param, const int64_t* weights,
                      uint32_t gate, hipStream_t s)
{
    const auto kern = [] {
        if constexpr (KIND == kWinEntropy) return entropy_box<R, T>;
        else return window_planes<R, T, KIND>;
    }();
    const int tiles_x = (g.nx + kWX - 1) / kWX, tiles_y = (g.ny + kWY - 1) / kWY;
    const int zs = default_zs(tiles_x * tiles_y, g.nz, resident_groups((const void*)kern, 256));
    const int total = tiles_x * tiles_y * ((g.nz + zs - 1) / zs);
    hipLaunchKernelGGL(kern, dim3(total), dim3(kWThreads), 0, s, static_cast<const T*>(in),
                       static_cast<T*>(out), g, zs, tiles_x, tiles_y, total, param, weights, gate);
    return hipGetLastError();
}

template <typename T, int KIND>
hipError_t dispatch_win(int r, const void* in, void* out, Geom g, int64_t param,
                        const int64_t* weights, uint32_t gate, hipStream_t s)
{
    if constexpr (KIND == kWinOkada) {
        return launch_win<1, T, KIND>(in, out, g, param, weights, gate, s);
    } else {
        switch (r) {
        case 1: return launch_win<1, T, KIND>(in, out, g, param, weights, gate, s);
        case 2: return launch_win<2, T, KIND>(in, out, g, param, weights, gate, s);
        case 3: return launch_win<3, T, KIND>(in, out, g, param, weights, gate, s);
        case 4: return launch_win<4, T, KIND>(in, out, g, param, weights, gate, s);
        default: return hipErrorInvalidValue;
        }
    }
}

template <typename T>
hipError_t dispatch_kind(int kind, int r, const void* in, void* out, Geom g, int64_t param,
                         const int64_t* weights, uint32_t gate, hipStream_t s)
{
    switch (kind) {
    case kWinSigma: return dispatch_win<T, kWinSigma>(r, in, out, g, param, weights, gate, s);
    case kWinOkada: return dispatch_win<T, kWinOkada>(r, in, out, g, param, weights, gate, s);
    default: return dispatch_win<T, kWinEntropy>(r, in, out, g, param, weights, gate, s);
    }
}

// floor(sqrt(n)) for n < 2^64
uint64_t isqrt64(unsigned __int128 n)
{
    uint64_t x = (uint64_t)std::sqrt((double)n);
    while ((unsigned __int128)x * x > n) --x;
    while ((unsigned __int128)(x + 1) * (x + 1) <= n) ++x;
    return x;
}

// Histogram of the volume into the context's scratch, copied to the host
// (synchronises `stream`).  Caller holds h->otsu_mu.
int host_histogram(lnf_ctx* h, const void* vol, size_t n, int dtype, hipStream_t stream)
{
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
    if (launch_histogram(vol, n, dtype, h->otsu_dev, stream) != hipSuccess ||
        hipMemcpyAsync(h->otsu_host, h->otsu_dev, levels * sizeof(uint64_t),
                       hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return LNF_EHIP;
    return LNF_OK;
}

int check_pair(lnf_handle h, const void* vol, const int64_t* dims, int dtype, int radius,
               const void* out, Geom* g, size_t* bytes)
{
    int rc = check_volume_args(h, vol, dims, dtype, radius, out, g, bytes);
    if (rc) return rc;
    if ((rc = check_device_range(vol, *bytes, h->device))) return rc;
    return check_device_range(out, *bytes, h->device);
}

}  // namespace

hipError_t launch_window(int kind, const void* in, void* out, int dtype, int r, Geom g,
                         int64_t param, const int64_t* weights, uint32_t gate, hipStream_t s)
{
    if (dtype == LNF_U8) return dispatch_kind<uint8_t>(kind, r, in, out, g, param, weights, gate, s);
    return dispatch_kind<uint16_t>(kind, r, in, out, g, param, weights, gate, s);
}

void entropy_scratch_free(lnf_ctx* h)
{
    if (h->entropy_dev) (void)hipFree(h->entropy_dev);
    h->entropy_dev = nullptr;
}

}  // namespace lnf

using namespace lnf;

extern "C" int lnf_filter_mean(lnf_handle h, const void* vol, const int64_t dims[3], int dtype,
                               int radius, void* out, hipStream_t stream)
{
    Geom g;
    size_t bytes = 0;
    if (!h) return LNF_EINVAL;
    DeviceGuard dg(h->device);
    if (!dg.ok()) return LNF_EHIP;
    int rc = check_pair(h, vol, dims, dtype, radius, out, &g, &bytes);
    if (rc) return rc;
    return launch_box_mean(vol, out, dtype, radius, g, h->gate, stream) == hipSuccess ? LNF_OK
                                                                                      : LNF_EHIP;
}

extern "C" int lnf_filter_sigma(lnf_handle h, const void* vol, const int64_t dims[3], int dtype,
                                int radius, int64_t half_width, void* out, hipStream_t stream,
                                int64_t* used_half_width)
{
    Geom g;
    size_t bytes = 0;
    if (!h) return LNF_EINVAL;
    DeviceGuard dg(h->device);
    if (!dg.ok()) return LNF_EHIP;
    int rc = check_pair(h, vol, dims, dtype, radius, out, &g, &bytes);
    if (rc) return rc;
    int64_t w = half_width;
    if (w < 0) {  // floor(2 sigma) of the whole volume, exact
        std::lock_guard<std::mutex> lk(h->otsu_mu);
        const size_t n = (size_t)g.nx * g.ny * g.nz;
        if ((rc = host_histogram(h, vol, n, dtype, stream))) return rc;
        const int levels = dtype == LNF_U8 ? 256 : 65536;
        unsigned __int128 N = 0, S = 0, Q = 0;
        for (int l = 0; l < levels; ++l) {
            const unsigned __int128 c = h->otsu_host[l];
            N += c;
            S += c * (unsigned)l;
            Q += c * (unsigned)l * (unsigned)l;
        }
        // (2 sigma)^2 = 4 (N Q - S^2) / N^2; floor(sqrt(a / b)) = isqrt(floor(a / b));
        // with N < 2^32, N Q < 2^96 and S^2 < 2^96 fit the 128-bit arithmetic
        if (N == 0 || N >> 32) return LNF_EINVAL;  // exact only below 2^32 voxels
        const unsigned __int128 num = 4 * (N * Q - S * S);
        w = (int64_t)isqrt64(num / (N * N));
    }
    if (used_half_width) *used_half_width = w;
    return launch_window(kWinSigma, vol, out, dtype, radius, g, w, nullptr, h->gate, stream) ==
                   hipSuccess
               ? LNF_OK
               : LNF_EHIP;
}

extern "C" int lnf_filter_okada(lnf_handle h, const void* vol, const int64_t dims[3], int dtype,
                                uint32_t t_d, void* out, hipStream_t stream)
{
    Geom g;
    size_t bytes = 0;
    if (!h) return LNF_EINVAL;
    DeviceGuard dg(h->device);
    if (!dg.ok()) return LNF_EHIP;
    int rc = check_pair(h, vol, dims, dtype, 1, out, &g, &bytes);
    if (rc) return rc;
    return launch_window(kWinOkada, vol, out, dtype, 1, g, (int64_t)t_d, nullptr, h->gate,
                         stream) == hipSuccess
               ? LNF_OK
               : LNF_EHIP;
}

extern "C" int lnf_filter_entropy(lnf_handle h, const void* vol, const int64_t dims[3], int dtype,
                                  int radius, double t_e, void* out, hipStream_t stream)
{
    Geom g;
    size_t bytes = 0;
    if (!h || !std::isfinite(t_e)) return LNF_EINVAL;
    DeviceGuard dg(h->device);
    if (!dg.ok()) return LNF_EHIP;
    int rc = check_pair(h, vol, dims, dtype, radius, out, &g, &bytes);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(h->otsu_mu);
    if (!h->entropy_dev && hipMalloc((void**)&h->entropy_dev, 65536 * sizeof(int64_t)) != hipSuccess) {
        (void)hipGetLastError();
        return LNF_ENOMEM;
    }
    const size_t n = (size_t)g.nx * g.ny * g.nz;
    if ((rc = host_histogram(h, vol, n, dtype, stream))) return rc;
    // weights -p log2 p of every level in 2^-32 fixed point, p = count / N,
    // written over the host histogram copy
    const int levels = dtype == LNF_U8 ? 256 : 65536;
    int64_t* wt = reinterpret_cast<int64_t*>(h->otsu_host);
    for (int l = 0; l < levels; ++l) {
        const uint64_t c = h->otsu_host[l];
        int64_t w = 0;
        if (c) {
            const double p = (double)c / (double)n;
            w = (int64_t)std::floor(-p * std::log2(p) * 4294967296.0 + 0.5);
        }
        wt[l] = w;
    }
    const double tf = std::floor(t_e * 4294967296.0 + 0.5);
    if (!(tf > -9.2e18 && tf < 9.2e18)) return LNF_EINVAL;
    if (hipMemcpyAsync(h->entropy_dev, wt, levels * sizeof(int64_t), hipMemcpyHostToDevice,
                       stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)  // the host buffer is reused by later calls
        return LNF_EHIP;
    return launch_window(kWinEntropy, vol, out, dtype, radius, g, (int64_t)tf, h->entropy_dev,
                         h->gate, stream) == hipSuccess
               ? LNF_OK
               : LNF_EHIP;
}
