// MEAN9: every voxel becomes the rounded mean of its nine cluster means
// (paper, Section "Our Method", eqs. 2-3 and the nine-cluster figure).
//
// The nine clusters have equal size n = (2r+1)^3, so the mean of means is
// S / (9n) with S the sum over all nine clusters.  S is a convolution of the
// clamp-extended volume E with a kernel that splits into two separable parts:
//   S = box_x box_y box_z E  +  c_x c_y c_z E,
//   box = ones on [-r, r]   (the centre cluster S_0),
//   c   = ones on [-2r, 2r] plus one more at 0  (per axis, the two diagonal
//         clusters at -r and +r overlap on the centre voxel; the product over
//         the three axes enumerates the eight diagonal clusters).
// The kernel evaluates it as separable running sums in exact uint32
// arithmetic: per z-slice an x-pass and a y-pass through LDS, then a z-window
// that slides through a register ring while the workgroup streams down its
// z-strip.
#include "device_common.h"
#include "lnf_internal.h"
#include "mean9_tile.h"

namespace lnf {
namespace {

// Single-volume wrapper around the streaming tile body of mean9_tile.h.
template <int R, int TY, typename T, bool GATE, int TXW>
__global__ __launch_bounds__((M9Geo<R, TY, TXW>::THREADS))
__attribute__((amdgpu_waves_per_eu((m9_waves<R, M9Geo<R, TY, TXW>::THREADS>())))) void mean9_stream(
    const T* __restrict__ in, T* __restrict__ out, Geom g, int zs, int tiles_x, int tiles_y,
    int total, uint32_t gate, double inv9n, int pairs)
{
    __shared__ __align__(16) M9SmemAny<R, TY, TXW, T> sm;
    const int tile = xcd_tile(blockIdx.x, total);
    const int bx = tile % tiles_x;
    const int rest = tile / tiles_x;
    const int by = rest % tiles_y;
    const int bz = rest / tiles_y;
    const int z0 = bz * zs;
    mean9_tile<R, TY, T, GATE, TXW>(sm, pairs != 0, in, out, g, bx * TXW, by * TY, z0,
                                    min(z0 + zs, g.nz), gate, inv9n, (int)threadIdx.x);
}

// The paper's mean filter (eq. 4): the box term of the same streaming tile,
// 64 x 16 tiles.
template <int R, typename T, bool GATE>
__global__ __launch_bounds__((M9Geo<R, 16, 64>::THREADS))
__attribute__((amdgpu_waves_per_eu((m9_waves<R, M9Geo<R, 16, 64>::THREADS>())))) void box_mean_stream(
    const T* __restrict__ in, T* __restrict__ out, Geom g, int zs, int tiles_x, int tiles_y,
    int total, uint32_t gate, double invn, int pairs)
{
    __shared__ __align__(16) M9SmemAny<R, 16, 64, T, true> sm;
    const int tile = xcd_tile(blockIdx.x, total);
    const int bx = tile % tiles_x;
    const int rest = tile / tiles_x;
    const int by = rest % tiles_y;
    const int bz = rest / tiles_y;
    const int z0 = bz * zs;
    mean9_tile<R, 16, T, GATE, 64, true>(sm, pairs != 0, in, out, g, bx * 64, by * 16, z0,
                                         min(z0 + zs, g.nz), gate, invn, (int)threadIdx.x);
}

template <int R, typename T, bool GATE>
hipError_t launch_box(const T* in, T* out, Geom g, uint32_t gate, hipStream_t s)
{
    constexpr int threads = M9Geo<R, 16, 64>::THREADS;
    const auto kern = box_mean_stream<R, T, GATE>;
    const int tiles_x = (g.nx + 63) / 64, tiles_y = (g.ny + 15) / 16;
    const int zs = default_zs(tiles_x * tiles_y, g.nz, resident_groups((const void*)kern, threads));
    const int total = tiles_x * tiles_y * ((g.nz + zs - 1) / zs);
    const int n = (2 * R + 1) * (2 * R + 1) * (2 * R + 1);
    const int pairs = mean9_pairs_ok(in, g.nx, sizeof(T)) ? 1 : 0;
    hipLaunchKernelGGL(kern, dim3(total), dim3(threads), 0, s, in, out, g, zs, tiles_x, tiles_y,
                       total, gate, 1.0 / n, pairs);
    return hipGetLastError();
}

template <typename T>
hipError_t dispatch_box(int r, const void* in, void* out, Geom g, uint32_t gate, hipStream_t s)
{
    const T* pin = static_cast<const T*>(in);
    T* pout = static_cast<T*>(out);
    switch (r) {
    case 1: return gate ? launch_box<1, T, true>(pin, pout, g, gate, s) : launch_box<1, T, false>(pin, pout, g, gate, s);
    case 2: return gate ? launch_box<2, T, true>(pin, pout, g, gate, s) : launch_box<2, T, false>(pin, pout, g, gate, s);
    case 3: return gate ? launch_box<3, T, true>(pin, pout, g, gate, s) : launch_box<3, T, false>(pin, pout, g, gate, s);
    case 4: return gate ? launch_box<4, T, true>(pin, pout, g, gate, s) : launch_box<4, T, false>(pin, pout, g, gate, s);
    default: return hipErrorInvalidValue;
    }
}

struct Variant {
    int tx, ty, threads;
};
// output tiles of the compiled shapes: 64 or 32 wide, 16 or 32 high
constexpr Variant kVariants[] = {{64, 16, 256}, {64, 32, 512}, {32, 16, 128}, {32, 32, 256}};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

// Default variant per voxel type and radius (index r-1): the fastest at the
// default z-strip depth on 512^3 volumes (uint16 r = 1: 32 x 16 tiles, about
// 1080 against 960 Gvoxel/s for 64 x 16; uint8 r = 4: 64 x 16, about 690
// against 620 for 32 x 32).
constexpr int kDefaultU16[LNF_RADIUS_MAX] = {2, 0, 0, 3};
constexpr int kDefaultU8[LNF_RADIUS_MAX] = {0, 0, 0, 0};

template <int R, typename T, bool GATE, int TY, int TXW>
hipError_t launch_stream(const T* in, T* out, Geom g, uint32_t gate, int zs, hipStream_t s,
                         TileCfg* plan)
{
    constexpr int threads = M9Geo<R, TY, TXW>::THREADS;
    const auto kern = mean9_stream<R, TY, T, GATE, TXW>;
    const int tiles_x = (g.nx + TXW - 1) / TXW, tiles_y = (g.ny + TY - 1) / TY;
    // default z-strip depth: one full round of resident workgroups
    if (zs <= 0)
        zs = default_zs(tiles_x * tiles_y, g.nz, resident_groups((const void*)kern, threads));
    if (plan) {
        plan->zs = zs;
        return hipSuccess;
    }
    const int nzs = (g.nz + zs - 1) / zs;
    const int total = tiles_x * tiles_y * nzs;
    const int n = (2 * R + 1) * (2 * R + 1) * (2 * R + 1);
    const int pairs = mean9_pairs_ok(in, g.nx, sizeof(T)) ? 1 : 0;
    hipLaunchKernelGGL(kern, dim3(total), dim3(threads), 0, s, in, out, g, zs, tiles_x, tiles_y,
                       total, gate, 1.0 / (9.0 * n), pairs);
    return hipGetLastError();
}

template <int R, typename T, bool GATE>
hipError_t launch_variant(int variant, const void* in, void* out, Geom g, uint32_t gate, int zs,
                          hipStream_t s, TileCfg* plan)
{
    const T* pin = static_cast<const T*>(in);
    T* pout = static_cast<T*>(out);
    switch (variant) {
    case 0: return launch_stream<R, T, GATE, 16, 64>(pin, pout, g, gate, zs, s, plan);
    case 1: return launch_stream<R, T, GATE, 32, 64>(pin, pout, g, gate, zs, s, plan);
    case 2: return launch_stream<R, T, GATE, 16, 32>(pin, pout, g, gate, zs, s, plan);
    default: return launch_stream<R, T, GATE, 32, 32>(pin, pout, g, gate, zs, s, plan);
    }
}

template <int R, typename T>
hipError_t launch_r(int variant, const void* in, void* out, Geom g, uint32_t gate, int zs,
                    hipStream_t s, TileCfg* plan)
{
    if (gate) return launch_variant<R, T, true>(variant, in, out, g, gate, zs, s, plan);
    return launch_variant<R, T, false>(variant, in, out, g, gate, zs, s, plan);
}

template <typename T>
hipError_t dispatch_r(const void* in, void* out, int r, Geom g, uint32_t gate, TileCfg cfg,
                      hipStream_t s, TileCfg* plan)
{
    if (r < 1 || r > LNF_RADIUS_MAX) return hipErrorInvalidValue;
    const int v = (cfg.variant >= 0 && cfg.variant < kNumVariants)
                      ? cfg.variant
                      : mean9_default_variant(sizeof(T) == 1 ? LNF_U8 : LNF_U16, r);
    if (plan) plan->variant = v;
    switch (r) {
    case 1: return launch_r<1, T>(v, in, out, g, gate, cfg.zs, s, plan);
    case 2: return launch_r<2, T>(v, in, out, g, gate, cfg.zs, s, plan);
    case 3: return launch_r<3, T>(v, in, out, g, gate, cfg.zs, s, plan);
    default: return launch_r<4, T>(v, in, out, g, gate, cfg.zs, s, plan);
    }
}

}  // namespace

int mean9_variants() { return kNumVariants; }

int mean9_default_variant(int dtype, int r)
{
    r = r < 1 ? 1 : r > LNF_RADIUS_MAX ? LNF_RADIUS_MAX : r;
    return dtype == LNF_U8 ? kDefaultU8[r - 1] : kDefaultU16[r - 1];
}

void mean9_tile_shape(int variant, int* tx, int* ty)
{
    const Variant v = kVariants[(variant >= 0 && variant < kNumVariants) ? variant : 0];
    *tx = v.tx;
    *ty = v.ty;
}

hipError_t launch_box_mean(const void* in, void* out, int dtype, int r, Geom g, uint32_t gate,
                           hipStream_t s)
{
    if (dtype == LNF_U8) return dispatch_box<uint8_t>(r, in, out, g, gate, s);
    return dispatch_box<uint16_t>(r, in, out, g, gate, s);
}

hipError_t launch_mean9(const void* in, void* out, int dtype, int r, Geom g, uint32_t gate,
                        TileCfg cfg, hipStream_t s, TileCfg* plan)
{
    if (dtype == LNF_U8) return dispatch_r<uint8_t>(in, out, r, g, gate, cfg, s, plan);
    return dispatch_r<uint16_t>(in, out, r, g, gate, cfg, s, plan);
}

}  // namespace lnf
