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
//
// The first-hit pass produces that point list for rays parallel to z: per
// pixel (x, y), the first voxel of the column, in the ray's direction, whose
// value reaches the threshold (the surface, Otsu's T in the paper).  One lane
// per ray, 64 neighbouring x per wavefront, so every slice step of a
// wavefront reads one contiguous row segment; each step issues kHitStep
// independent slice loads before testing them, to keep enough reads in
// flight for HBM.  A lane stops at its hit (its loads are masked off from
// then on) and the wavefront at its deepest hit, so the bytes read are the
// columns up to their hits.
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

constexpr int kHitStep = 8;     // slices loaded per step of a ray
constexpr int kHitRows = 4;     // wavefronts (pixel rows) per workgroup

template <typename T, bool BACK>
__global__ __launch_bounds__(64 * kHitRows) void first_hit_kernel(const T* __restrict__ in,
                                                                  Geom g, uint32_t thr,
                                                                  int tiles_x,
                                                                  int32_t* __restrict__ xyz)
{
    const int bx = blockIdx.x % tiles_x, by = blockIdx.x / tiles_x;
    const int x = bx * 64 + (threadIdx.x & 63);
    const int y = by * kHitRows + (threadIdx.x >> 6);
    if (x >= g.nx || y >= g.ny) return;
    const size_t plane = (size_t)g.nx * g.ny;
    const T* col = in + (size_t)y * g.nx + x;
    int hit = -1;  // steps from the ray's first slice
    for (int s0 = 0; s0 < g.nz; s0 += kHitStep) {
        uint32_t v[kHitStep];
#pragma unroll
        for (int k = 0; k < kHitStep; ++k) {
            const int s = s0 + k;
            const int z = BACK ? g.nz - 1 - s : s;
            v[k] = s < g.nz ? (uint32_t)col[(size_t)z * plane] : 0u;
        }
#pragma unroll
        for (int k = kHitStep - 1; k >= 0; --k)  // the first qualifying step wins
            if (s0 + k < g.nz && v[k] >= thr) hit = s0 + k;
        if (hit >= 0) break;
    }
    int32_t* o = xyz + 3 * ((size_t)y * g.nx + x);
    o[0] = x;
    o[1] = y;
    o[2] = hit < 0 ? -1 : (BACK ? g.nz - 1 - hit : hit);
}

template <typename T>
hipError_t launch_first_hit(const void* vol, Geom g, uint32_t thr, int direction, int32_t* xyz,
                            hipStream_t s)
{
    const int tiles_x = (g.nx + 63) / 64;
    const long long blocks = (long long)tiles_x * ((g.ny + kHitRows - 1) / kHitRows);
    const dim3 grid((unsigned)blocks), block(64 * kHitRows);
    const T* in = static_cast<const T*>(vol);
    if (direction > 0)
        hipLaunchKernelGGL((first_hit_kernel<T, false>), grid, block, 0, s, in, g, thr, tiles_x,
                           xyz);
    else
        hipLaunchKernelGGL((first_hit_kernel<T, true>), grid, block, 0, s, in, g, thr, tiles_x,
                           xyz);
    return hipGetLastError();
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

namespace {

// Checks shared by the first-hit entry points: the volume and a hit list of
// nx * ny entries on the context's device.
int check_first_hit(lnf_handle h, const void* vol, const int64_t dims[3], int dtype,
                    int direction, const int32_t* xyz, Geom* g)
{
    if (!h || !vol || !dims || !xyz) return LNF_EINVAL;
    if (dtype != LNF_U8 && dtype != LNF_U16) return LNF_EINVAL;
    if (direction != 1 && direction != -1) return LNF_EINVAL;
    for (int i = 0; i < 3; ++i)
        if (dims[i] < 1 || dims[i] > INT32_MAX) return LNF_EINVAL;
    if (dims[0] * dims[1] > INT32_MAX) return LNF_EINVAL;
    *g = Geom{(int)dims[0], (int)dims[1], (int)dims[2]};
    const size_t bytes = (size_t)dims[0] * dims[1] * dims[2] * (dtype == LNF_U8 ? 1 : 2);
    int rc;
    if ((rc = check_device_range(vol, bytes, h->device))) return rc;
    return check_device_range(xyz, (size_t)dims[0] * dims[1] * 3 * sizeof(int32_t), h->device);
}

}  // namespace

extern "C" int lnf_first_hit(lnf_handle h, const void* vol, const int64_t dims[3], int dtype,
                             uint32_t threshold, int direction, int32_t* xyz, hipStream_t stream)
{
    if (!h) return LNF_EINVAL;
    DeviceGuard dg(h->device);
    if (!dg.ok()) return LNF_EHIP;
    Geom g;
    const int rc = check_first_hit(h, vol, dims, dtype, direction, xyz, &g);
    if (rc) return rc;
    const hipError_t e = dtype == LNF_U8
                             ? launch_first_hit<uint8_t>(vol, g, threshold, direction, xyz, stream)
                             : launch_first_hit<uint16_t>(vol, g, threshold, direction, xyz, stream);
    return e == hipSuccess ? LNF_OK : LNF_EHIP;
}

extern "C" int lnf_filter_surface(lnf_handle h, const void* vol, const int64_t dims[3], int dtype,
                                  int radius, uint32_t threshold, int direction, int32_t* xyz,
                                  uint32_t* out, hipStream_t stream)
{
    if (!h || !out) return LNF_EINVAL;
    if (h->geom) return LNF_EINVAL;  // default cluster geometry only, as lnf_filter_points
    if (radius < 1 || radius > LNF_RADIUS_MAX) return LNF_EINVAL;
    DeviceGuard dg(h->device);
    if (!dg.ok()) return LNF_EHIP;
    Geom g;
    int rc = check_first_hit(h, vol, dims, dtype, direction, xyz, &g);
    if (rc) return rc;
    const int64_t n = dims[0] * dims[1];
    if ((rc = check_device_range(out, (size_t)n * sizeof(uint32_t), h->device))) return rc;
    if ((rc = lnf_first_hit(h, vol, dims, dtype, threshold, direction, xyz, stream))) return rc;
    return lnf_filter_points(h, vol, dims, dtype, radius, xyz, n, out, stream);
}

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
