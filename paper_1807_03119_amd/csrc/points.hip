// Surface-point mode: the filter evaluated only at a list of voxels.  In the
// paper the filter runs at the first surface intersection point of each ray
// inside the renderer (Section "Our Method"; Results, Performance), so the
// work is a sparse gather rather than a dense stencil.
//
// One 64-lane wavefront per point: the lanes split the (2r+1)^3 samples of each
// of the nine clusters (coordinates clamped into the volume), keep per-cluster
// partial sums (and sums of squares for MINVAR9) in registers, and combine them
// with butterfly wavefront reductions (cross-lane shuffles).  Lane 0 applies
// the rule, rounding and gate.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "lnf.h"
#include "lnf_ctx.h"
#include "lnf_internal.h"

namespace lnf {
namespace {

constexpr int kWaves = 4;  // points per workgroup

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_sum_f64(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int R, typename T, int RULE>
__global__ __launch_bounds__(64 * kWaves) void filter_points_kernel(const T* __restrict__ in,
                                                                     Geom g, const int32_t* xyz,
                                                                     int64_t n, uint32_t gate,
                                                                     uint32_t* out)
{
    constexpr int M = 2 * R + 1, NB = M * M * M;
    const int lane = threadIdx.x & 63;
    const int64_t p = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (p >= n) return;  // whole wavefront exits together
    const int px = xyz[3 * p], py = xyz[3 * p + 1], pz = xyz[3 * p + 2];
    if (px < 0 || py < 0 || pz < 0 || px >= g.nx || py >= g.ny || pz >= g.nz) {
        if (lane == 0) out[p] = 0xffffffffu;  // point outside the volume
        return;
    }
    const size_t nx = g.nx, plane = (size_t)g.nx * g.ny;
    uint32_t s[9];
    double q[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int j = k - 1;
        const int dx = k == 0 ? 0 : ((j & 1) ? R : -R);
        const int dy = k == 0 ? 0 : ((j & 2) ? R : -R);
        const int dz = k == 0 ? 0 : ((j & 4) ? R : -R);
        uint32_t acc = 0;
        double acq = 0.0;
        for (int e = lane; e < NB; e += 64) {
            const int ax = e % M - R, ay = (e / M) % M - R, az = e / (M * M) - R;
            const int x = clampi(px + dx + ax, 0, g.nx - 1);
            const int y = clampi(py + dy + ay, 0, g.ny - 1);
            const int z = clampi(pz + dz + az, 0, g.nz - 1);
            const uint32_t v = in[(size_t)z * plane + (size_t)y * nx + x];
            acc += v;
            if (RULE == LNF_MINVAR9) acq = __builtin_fma((double)v, (double)v, acq);
        }
        s[k] = wave_sum_u32(acc);
        if (RULE == LNF_MINVAR9) q[k] = wave_sum_f64(acq);
    }
    if (lane != 0) return;
    uint32_t o;
    if (RULE == LNF_MEAN9) {
        uint32_t total = 0;
#pragma unroll
        for (int k = 0; k < 9; ++k) total += s[k];
        o = round_div_odd(total, 1.0 / (9.0 * NB));
    } else {
        uint32_t best_s = s[0];
        double best_v = __builtin_fma((double)NB, q[0], -(double)s[0] * (double)s[0]);
#pragma unroll
        for (int k = 1; k < 9; ++k) {
            const double v = __builtin_fma((double)NB, q[k], -(double)s[k] * (double)s[k]);
            if (v < best_v) {
                best_v = v;
                best_s = s[k];
            }
        }
        o = round_div_odd(best_s, 1.0 / NB);
    }
    if (o < gate) o = 0;
    out[p] = o;
}

template <int R, typename T>
hipError_t launch_points_r(int rule, const void* vol, Geom g, const int32_t* xyz, int64_t n,
                           uint32_t gate, uint32_t* out, hipStream_t s)
{
    const dim3 grid((unsigned)((n + kWaves - 1) / kWaves)), block(64 * kWaves);
    const T* in = static_cast<const T*>(vol);
    if (rule == LNF_MEAN9)
        hipLaunchKernelGGL((filter_points_kernel<R, T, LNF_MEAN9>), grid, block, 0, s, in, g, xyz,
                           n, gate, out);
    else
        hipLaunchKernelGGL((filter_points_kernel<R, T, LNF_MINVAR9>), grid, block, 0, s, in, g,
                           xyz, n, gate, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_points(int rule, int r, const void* vol, Geom g, const int32_t* xyz, int64_t n,
                         uint32_t gate, uint32_t* out, hipStream_t s)
{
    switch (r) {
    case 1: return launch_points_r<1, T>(rule, vol, g, xyz, n, gate, out, s);
    case 2: return launch_points_r<2, T>(rule, vol, g, xyz, n, gate, out, s);
    case 3: return launch_points_r<3, T>(rule, vol, g, xyz, n, gate, out, s);
    default: return launch_points_r<4, T>(rule, vol, g, xyz, n, gate, out, s);
    }
}

}  // namespace
}  // namespace lnf

using namespace lnf;

extern "C" int lnf_filter_points(lnf_handle h, const void* vol, const int64_t dims[3], int dtype,
                                 int radius, const int32_t* xyz, int64_t n, uint32_t* out,
                                 hipStream_t stream)
{
    if (!h || !vol || !dims || n < 0 || (n > 0 && (!xyz || !out))) return LNF_EINVAL;
    if (h->geom) return LNF_EINVAL;  // default cluster geometry only
    if (dtype != LNF_U8 && dtype != LNF_U16) return LNF_EINVAL;
    if (radius < 1 || radius > LNF_RADIUS_MAX) return LNF_EINVAL;
    for (int i = 0; i < 3; ++i)
        if (dims[i] < 1 || dims[i] > INT32_MAX) return LNF_EINVAL;
    if (dims[0] * dims[1] > INT32_MAX) return LNF_EINVAL;
    if (n > (int64_t)INT32_MAX * 4) return LNF_EINVAL;
    if (n == 0) return LNF_OK;
    const Geom g{(int)dims[0], (int)dims[1], (int)dims[2]};
    const size_t bytes = (size_t)dims[0] * dims[1] * dims[2] * (dtype == LNF_U8 ? 1 : 2);
    DeviceGuard dg(h->device);
    if (!dg.ok()) return LNF_EHIP;
    int rc;
    if ((rc = check_device_range(vol, bytes, h->device))) return rc;
    if ((rc = check_device_range(xyz, (size_t)n * 3 * sizeof(int32_t), h->device))) return rc;
    if ((rc = check_device_range(out, (size_t)n * sizeof(uint32_t), h->device))) return rc;
    const hipError_t e =
        dtype == LNF_U8
            ? launch_points<uint8_t>(h->rule, radius, vol, g, xyz, n, h->gate, out, stream)
            : launch_points<uint16_t>(h->rule, radius, vol, g, xyz, n, h->gate, out, stream);
    return e == hipSuccess ? LNF_OK : LNF_EHIP;
}
