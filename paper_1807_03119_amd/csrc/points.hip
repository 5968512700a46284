// Surface-point mode: the filter evaluated only at a list of voxels.  In the
// paper the filter runs at the first surface intersection point of each ray
// inside the renderer (Section "Our Method"; Results, Performance), so the
// work is a sparse gather rather than a dense stencil.
//
// One 64-lane wavefront per point.  The nine clusters cover the (4r+1)^3 block
// around the point (coordinates clamped into the volume); the lanes split its
// (4r+1)^2 x-rows.  Each row is read once and summed over three x-ranges: left
// [-2r, 0], right [0, 2r] and centre [-r, r].  A row at (dy, dz) then belongs to
// the corner clusters whose y- and z-ranges hold it (left or right part by the
// cluster's x side) and, when |dy|, |dz| <= r, to the centre cluster.  Per-lane
// cluster sums (and sums of squares for MINVAR9) are combined with butterfly
// wavefront reductions (cross-lane shuffles); MEAN9 needs only their total.
// Lane 0 applies the rule, rounding and gate.
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
    constexpr int W = 4 * R + 1, NROW = W * W;  // side and x-rows of the nine clusters' block
    constexpr bool VAR = RULE == LNF_MINVAR9;
    const int lane = threadIdx.x & 63;
    const int64_t p = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (p >= n) return;  // whole wavefront exits together
    // the point is the same for the whole wavefront: keep it scalar
    const int px = __builtin_amdgcn_readfirstlane(xyz[3 * p]);
    const int py = __builtin_amdgcn_readfirstlane(xyz[3 * p + 1]);
    const int pz = __builtin_amdgcn_readfirstlane(xyz[3 * p + 2]);
    if (px < 0 || py < 0 || pz < 0 || px >= g.nx || py >= g.ny || pz >= g.nz) {
        if (lane == 0) out[p] = 0xffffffffu;  // point outside the volume
        return;
    }
    const size_t nx = g.nx, plane = (size_t)g.nx * g.ny;
    int xs[W];  // clamped x of the row's samples (the same for every row)
#pragma unroll
    for (int i = 0; i < W; ++i) xs[i] = clampi(px - 2 * R + i, 0, g.nx - 1);
    uint32_t s[9];
    double q[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        s[k] = 0;
        q[k] = 0.0;
    }
    for (int row = lane; row < NROW; row += 64) {
        const int dy = row % W - 2 * R, dz = row / W - 2 * R;
        const int y = clampi(py + dy, 0, g.ny - 1), z = clampi(pz + dz, 0, g.nz - 1);
        const T* rp = in + (size_t)z * plane + (size_t)y * nx;
        uint32_t v[W];
#pragma unroll
        for (int i = 0; i < W; ++i) v[i] = rp[xs[i]];
        uint32_t left = 0, right = 0, centre = 0;
        double ql = 0.0, qr = 0.0, qc = 0.0;
#pragma unroll
        for (int i = 0; i < W; ++i) {
            if (i <= 2 * R) left += v[i];
            if (i >= 2 * R) right += v[i];
            if (i >= R && i <= 3 * R) centre += v[i];
            if constexpr (VAR) {
                const double vv = (double)v[i] * (double)v[i];  // exact below 2^32
                if (i <= 2 * R) ql += vv;
                if (i >= 2 * R) qr += vv;
                if (i >= R && i <= 3 * R) qc += vv;
            }
        }
        const bool inc = dy >= -R && dy <= R && dz >= -R && dz <= R;
        s[0] += inc ? centre : 0u;
        if constexpr (VAR) q[0] += inc ? qc : 0.0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {  // cluster j + 1: x, y, z side by bits 0, 1, 2
            const bool in_yz = ((j & 2) ? dy >= 0 : dy <= 0) && ((j & 4) ? dz >= 0 : dz <= 0);
            s[j + 1] += in_yz ? ((j & 1) ? right : left) : 0u;
            if constexpr (VAR) q[j + 1] += in_yz ? ((j & 1) ? qr : ql) : 0.0;
        }
    }
    uint32_t o;
    if constexpr (!VAR) {
        uint32_t total = 0;
#pragma unroll
        for (int k = 0; k < 9; ++k) total += s[k];
        total = wave_sum_u32(total);
        o = round_div_odd(total, 1.0 / (9.0 * NB));
    } else {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            s[k] = wave_sum_u32(s[k]);
            q[k] = wave_sum_f64(q[k]);
        }
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
    if (lane != 0) return;
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
