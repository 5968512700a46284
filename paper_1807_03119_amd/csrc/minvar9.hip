// MINVAR9 single-volume kernel: a thin wrapper around the tile body of
// minvar9_tile.h (least-variance selection among the nine clusters).
#include "device_common.h"
#include "lnf_internal.h"
#include "minvar9_tile.h"

namespace lnf {
namespace {

template <int R, typename T, bool GATE>
__global__ __launch_bounds__(MV9Shape<R>::THREADS)
__attribute__((amdgpu_waves_per_eu(MV9Shape<R>::WAVES))) void minvar9_planes(const T* __restrict__ in, T* __restrict__ out,
                                                      Geom g, int zs, int tiles_x, int tiles_y,
                                                      int total, uint32_t gate, double dn,
                                                      double invn)
{
    __shared__ __align__(16) MV9Smem<R, T> sm;
    const int tile = xcd_tile(blockIdx.x, total);
    const int bx = tile % tiles_x;
    const int rest = tile / tiles_x;
    const int by = rest % tiles_y;
    const int bz = rest / tiles_y;
    const int z0 = bz * zs;
    minvar9_tile<R, T, GATE>(sm, in, out, g, bx * MV9Shape<R>::TX, by * MV9Shape<R>::TY, z0,
                             min(z0 + zs, g.nz), gate, dn, invn);
}

template <int R, typename T>
hipError_t launch_planes(const void* in, void* out, Geom g, uint32_t gate, int zs, hipStream_t s)
{
    using S = MV9Shape<R>;
    const int tiles_x = (g.nx + S::TX - 1) / S::TX, tiles_y = (g.ny + S::TY - 1) / S::TY;
    if (zs <= 0)
        zs = default_zs(tiles_x * tiles_y, g.nz,
                        resident_groups((const void*)minvar9_planes<R, T, false>, S::THREADS));
    const int nzs = (g.nz + zs - 1) / zs;
    const int total = tiles_x * tiles_y * nzs;
    const int n = (2 * R + 1) * (2 * R + 1) * (2 * R + 1);
    const T* pin = static_cast<const T*>(in);
    T* pout = static_cast<T*>(out);
    if (gate)
        hipLaunchKernelGGL((minvar9_planes<R, T, true>), dim3(total), dim3(S::THREADS), 0, s,
                           pin, pout, g, zs, tiles_x, tiles_y, total, gate, (double)n, 1.0 / n);
    else
        hipLaunchKernelGGL((minvar9_planes<R, T, false>), dim3(total), dim3(S::THREADS), 0, s,
                           pin, pout, g, zs, tiles_x, tiles_y, total, gate, (double)n, 1.0 / n);
    return hipGetLastError();
}

template <typename T>
hipError_t dispatch_r(const void* in, void* out, int r, Geom g, uint32_t gate, TileCfg cfg,
                      hipStream_t s)
{
    switch (r) {
    case 1: return launch_planes<1, T>(in, out, g, gate, cfg.zs, s);
    case 2: return launch_planes<2, T>(in, out, g, gate, cfg.zs, s);
    case 3: return launch_planes<3, T>(in, out, g, gate, cfg.zs, s);
    case 4: return launch_planes<4, T>(in, out, g, gate, cfg.zs, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

int minvar9_variants() { return 1; }

void minvar9_tile_shape(int variant, int* tx, int* ty)
{
    (void)variant;
    *tx = MV9Shape<1>::TX;  // one tile shape for every radius
    *ty = MV9Shape<1>::TY;
}

hipError_t launch_minvar9(const void* in, void* out, int dtype, int r, Geom g, uint32_t gate,
                          TileCfg cfg, hipStream_t s)
{
    if (dtype == LNF_U8) return dispatch_r<uint8_t>(in, out, r, g, gate, cfg, s);
    return dispatch_r<uint16_t>(in, out, r, g, gate, cfg, s);
}

}  // namespace lnf
