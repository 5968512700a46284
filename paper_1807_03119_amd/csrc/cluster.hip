// Geometry variants of the nine-cluster filter (cross clusters of eq. 2, and
// diagonal offsets 1 or 2r+1), both rules: single-volume kernels around the
// per-plane cluster tile of plane_tile.h.  The default geometry (cubes at
// offset r) runs on the MEAN9 streaming kernel and the MINVAR9 kernel instead.
#include "batch_table.h"
#include "device_common.h"
#include "lnf.h"
#include "lnf_internal.h"
#include "plane_tile.h"

namespace lnf {
namespace {

// The gate is a runtime value here (0 = off): one instantiation per geometry.
// One volume (tab == nullptr: in, out, g and the tile grid given), or a class
// `cls` of a batch job table (the volume arguments unused).
template <int R, int D, int SHAPE, int RULE, typename T>
__global__ __launch_bounds__((PTShape<R, D, SHAPE, RULE>::THREADS))
__attribute__((amdgpu_waves_per_eu(PTShape<R, D, SHAPE, RULE>::WAVES))) void cluster_planes(
    const BatchTable* __restrict__ tab, int cls, const T* __restrict__ in, T* __restrict__ out,
    Geom g, int zs, int tiles_x, int tiles_y, int total, uint32_t gate, double dn, double inv)
{
    using S = PTShape<R, D, SHAPE, RULE>;
    __shared__ __align__(16) PTSmem<R, D, SHAPE, RULE, T> sm;
    int local = xcd_tile(blockIdx.x, total);
    if (tab) {
        const BatchClass& c = tab->c[cls];
        const BatchJobDesc& d = job_of(tab, c, local);
        local -= d.tile_begin;
        in = static_cast<const T*>(d.in);
        out = static_cast<T*>(d.out);
        g = Geom{d.nx, d.ny, d.nz};
        zs = d.zs;
        tiles_x = d.tiles_x;
        tiles_y = d.tiles_y;
    }
    const int bx = local % tiles_x;
    const int rest = local / tiles_x;
    const int by = rest % tiles_y;
    const int bz = rest / tiles_y;
    const int z0 = bz * zs;
    plane_tile<R, D, SHAPE, RULE, T, true>(sm, in, out, g, bx * S::TX, by * S::TY, z0,
                                           min(z0 + zs, g.nz), gate, dn, inv,
                                           (int)threadIdx.x);
}

template <int R, int D, int SHAPE, int RULE, typename T>
hipError_t launch_geom(const void* in, void* out, Geom g, uint32_t gate, int zs, hipStream_t s,
                       TileCfg* plan)
{
    using S = PTShape<R, D, SHAPE, RULE>;
    const auto kern = cluster_planes<R, D, SHAPE, RULE, T>;
    const int tiles_x = (g.nx + S::TX - 1) / S::TX, tiles_y = (g.ny + S::TY - 1) / S::TY;
    if (zs <= 0)
        zs = default_zs(tiles_x * tiles_y, g.nz, resident_groups((const void*)kern, S::THREADS));
    if (plan) {
        *plan = TileCfg{0, zs};
        return hipSuccess;
    }
    const int nzs = (g.nz + zs - 1) / zs;
    const int total = tiles_x * tiles_y * nzs;
    const double dn = (double)S::N;
    const double inv = S::VAR ? 1.0 / S::N : 1.0 / (9.0 * S::N);
    hipLaunchKernelGGL(kern, dim3(total), dim3(S::THREADS), 0, s, (const BatchTable*)nullptr, 0,
                       static_cast<const T*>(in), static_cast<T*>(out), g, zs, tiles_x, tiles_y,
                       total, gate, dn, inv);
    return hipGetLastError();
}

template <int R, int SHAPE, int RULE, typename T>
hipError_t launch_offset(int offset, const void* in, void* out, Geom g, uint32_t gate, int zs,
                         hipStream_t s, TileCfg* plan)
{
    switch (offset) {
    case LNF_GEOM_OFFSET_1: return launch_geom<R, 1, SHAPE, RULE, T>(in, out, g, gate, zs, s, plan);
    case LNF_GEOM_OFFSET_2R1:
        return launch_geom<R, 2 * R + 1, SHAPE, RULE, T>(in, out, g, gate, zs, s, plan);
    default: return launch_geom<R, R, SHAPE, RULE, T>(in, out, g, gate, zs, s, plan);
    }
}

template <int R, typename T>
hipError_t launch_r(int rule, uint32_t geom, const void* in, void* out, Geom g, uint32_t gate,
                    int zs, hipStream_t s, TileCfg* plan)
{
    const int offset = (int)(geom & (LNF_GEOM_OFFSET_1 | LNF_GEOM_OFFSET_2R1));
    const bool var = rule == LNF_MINVAR9;
    if (geom & LNF_GEOM_CROSS) {
        if (var)
            return launch_offset<R, kClusterCross, kRuleMinVar9, T>(offset, in, out, g, gate, zs, s, plan);
        return launch_offset<R, kClusterCross, kRuleMean9, T>(offset, in, out, g, gate, zs, s, plan);
    }
    if (var) return launch_offset<R, kClusterBox, kRuleMinVar9, T>(offset, in, out, g, gate, zs, s, plan);
    return launch_offset<R, kClusterBox, kRuleMean9, T>(offset, in, out, g, gate, zs, s, plan);
}

template <typename T>
hipError_t dispatch(int rule, uint32_t geom, int r, const void* in, void* out, Geom g,
                    uint32_t gate, int zs, hipStream_t s, TileCfg* plan)
{
    switch (r) {
    case 1: return launch_r<1, T>(rule, geom, in, out, g, gate, zs, s, plan);
    case 2: return launch_r<2, T>(rule, geom, in, out, g, gate, zs, s, plan);
    case 3: return launch_r<3, T>(rule, geom, in, out, g, gate, zs, s, plan);
    case 4: return launch_r<4, T>(rule, geom, in, out, g, gate, zs, s, plan);
    default: return hipErrorInvalidValue;
    }
}

template <int R, int D, int SHAPE, int RULE, typename T>
GeomClassKernel geom_kernel()
{
    using S = PTShape<R, D, SHAPE, RULE>;
    return {{reinterpret_cast<const void*>(cluster_planes<R, D, SHAPE, RULE, T>), S::THREADS},
            S::TX, S::TY, (double)S::N, S::VAR ? 1.0 / S::N : 1.0 / (9.0 * S::N)};
}

template <int R, int SHAPE, int RULE, typename T>
GeomClassKernel geom_kernel_offset(int offset)
{
    switch (offset) {
    case LNF_GEOM_OFFSET_1: return geom_kernel<R, 1, SHAPE, RULE, T>();
    case LNF_GEOM_OFFSET_2R1: return geom_kernel<R, 2 * R + 1, SHAPE, RULE, T>();
    default: return geom_kernel<R, R, SHAPE, RULE, T>();
    }
}

template <int R, typename T>
GeomClassKernel geom_kernel_r(int rule, uint32_t geom)
{
    const int offset = (int)(geom & (LNF_GEOM_OFFSET_1 | LNF_GEOM_OFFSET_2R1));
    const bool var = rule == LNF_MINVAR9;
    if (geom & LNF_GEOM_CROSS)
        return var ? geom_kernel_offset<R, kClusterCross, kRuleMinVar9, T>(offset)
                   : geom_kernel_offset<R, kClusterCross, kRuleMean9, T>(offset);
    return var ? geom_kernel_offset<R, kClusterBox, kRuleMinVar9, T>(offset)
               : geom_kernel_offset<R, kClusterBox, kRuleMean9, T>(offset);
}

template <typename T>
GeomClassKernel geom_kernel_t(int rule, uint32_t geom, int r)
{
    switch (r) {
    case 1: return geom_kernel_r<1, T>(rule, geom);
    case 2: return geom_kernel_r<2, T>(rule, geom);
    case 3: return geom_kernel_r<3, T>(rule, geom);
    default: return geom_kernel_r<4, T>(rule, geom);
    }
}

}  // namespace

GeomClassKernel geometry_class_kernel(int rule, uint32_t geom, int dtype, int r)
{
    return dtype == LNF_U8 ? geom_kernel_t<uint8_t>(rule, geom, r)
                           : geom_kernel_t<uint16_t>(rule, geom, r);
}

hipError_t launch_geometry(int rule, uint32_t geom, const void* in, void* out, int dtype, int r,
                           Geom g, uint32_t gate, int zs, hipStream_t s, TileCfg* plan)
{
    if (dtype == LNF_U8) return dispatch<uint8_t>(rule, geom, r, in, out, g, gate, zs, s, plan);
    return dispatch<uint16_t>(rule, geom, r, in, out, g, gate, zs, s, plan);
}

}  // namespace lnf
