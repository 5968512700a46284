// MINVAR9 single-volume kernel: a thin wrapper around the tile body of
// plane_tile.h (least-variance selection among the nine clusters).
#include "device_common.h"
#include "lnf_internal.h"
#include "plane_tile.h"

namespace lnf {
namespace {

template <int R, typename T, bool GATE, bool WT>
__global__ __launch_bounds__((MV9Shape<R, WT>::THREADS))
__attribute__((amdgpu_waves_per_eu(MV9Shape<R, WT>::WAVES))) void minvar9_planes(
    const T* __restrict__ in, T* __restrict__ out, Geom g, int zs, int tiles_x, int tiles_y,
    int total, uint32_t gate, double dn, double invn)
{
    using S = MV9Shape<R, WT>;
    __shared__ __align__(16) MV9Lds<R, T, WT> sm;
    const int tile = xcd_tile(blockIdx.x, total);
    const int bx = tile % tiles_x;
    const int rest = tile / tiles_x;
    const int by = rest % tiles_y;
    const int bz = rest / tiles_y;
    const int z0 = bz * zs;
    minvar9_tile<R, T, GATE, WT>(sm, in, out, g, bx * S::TX, by * S::TY, z0, min(z0 + zs, g.nz),
                                 gate, dn, invn, (int)threadIdx.x);
}

template <int R, typename T, bool WT>
hipError_t launch_planes(const void* in, void* out, Geom g, uint32_t gate, int zs, hipStream_t s,
                         TileCfg* plan)
{
    using S = MV9Shape<R, WT>;
    const int tiles_x = (g.nx + S::TX - 1) / S::TX, tiles_y = (g.ny + S::TY - 1) / S::TY;
    if (zs <= 0)
        zs = default_zs(tiles_x * tiles_y, g.nz,
                        resident_groups((const void*)minvar9_planes<R, T, false, WT>, S::THREADS));
    if (plan) {
        plan->zs = zs;
        return hipSuccess;
    }
    const int nzs = (g.nz + zs - 1) / zs;
    const int total = tiles_x * tiles_y * nzs;
    const int n = (2 * R + 1) * (2 * R + 1) * (2 * R + 1);
    const T* pin = static_cast<const T*>(in);
    T* pout = static_cast<T*>(out);
    if (gate)
        hipLaunchKernelGGL((minvar9_planes<R, T, true, WT>), dim3(total), dim3(S::THREADS), 0, s,
                           pin, pout, g, zs, tiles_x, tiles_y, total, gate, (double)n, 1.0 / n);
    else
        hipLaunchKernelGGL((minvar9_planes<R, T, false, WT>), dim3(total), dim3(S::THREADS), 0, s,
                           pin, pout, g, zs, tiles_x, tiles_y, total, gate, (double)n, 1.0 / n);
    return hipGetLastError();
}

template <int R, typename T>
hipError_t launch_variant(int variant, const void* in, void* out, Geom g, uint32_t gate, int zs,
                          hipStream_t s, TileCfg* plan)
{
    if (variant == 1) return launch_planes<R, T, true>(in, out, g, gate, zs, s, plan);
    return launch_planes<R, T, false>(in, out, g, gate, zs, s, plan);
}

template <typename T>
hipError_t dispatch_r(const void* in, void* out, int r, Geom g, uint32_t gate, TileCfg cfg,
                      hipStream_t s, TileCfg* plan)
{
    const int v = cfg.variant >= 0 ? cfg.variant
                                   : minvar9_default_variant(sizeof(T) == 1 ? LNF_U8 : LNF_U16, r, g);
    if (plan) plan->variant = v;
    switch (r) {
    case 1: return launch_variant<1, T>(v, in, out, g, gate, cfg.zs, s, plan);
    case 2: return launch_variant<2, T>(v, in, out, g, gate, cfg.zs, s, plan);
    case 3: return launch_variant<3, T>(v, in, out, g, gate, cfg.zs, s, plan);
    case 4: return launch_variant<4, T>(v, in, out, g, gate, cfg.zs, s, plan);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

// 0: 32 x 16 outputs, 256 threads; 1: 64 x 16 outputs, 512 threads (up to
// r = 3; the same tile as 0 at r = 4)
int minvar9_variants() { return 2; }

// The wide tile on large planes where it measured faster (uint16 up to r = 3,
// uint8 at r = 3), else 32 x 16.
int minvar9_default_variant(int dtype, int r, Geom g)
{
    return (g.nx >= 256 && g.ny >= 256 && r <= 3 && (dtype == LNF_U16 || r == 3)) ? 1 : 0;
}

void minvar9_tile_shape(int variant, int r, int* tx, int* ty)
{
    const bool w = variant == 1;
    switch (r) {
    case 1: *tx = w ? MV9Shape<1, true>::TX : MV9Shape<1>::TX; *ty = MV9Shape<1>::TY; return;
    case 2: *tx = w ? MV9Shape<2, true>::TX : MV9Shape<2>::TX; *ty = MV9Shape<2>::TY; return;
    case 3: *tx = w ? MV9Shape<3, true>::TX : MV9Shape<3>::TX; *ty = MV9Shape<3>::TY; return;
    default: *tx = MV9Shape<4>::TX; *ty = MV9Shape<4>::TY; return;
    }
}

hipError_t launch_minvar9(const void* in, void* out, int dtype, int r, Geom g, uint32_t gate,
                          TileCfg cfg, hipStream_t s, TileCfg* plan)
{
    if (dtype == LNF_U8) return dispatch_r<uint8_t>(in, out, r, g, gate, cfg, s, plan);
    return dispatch_r<uint16_t>(in, out, r, g, gate, cfg, s, plan);
}

}  // namespace lnf
