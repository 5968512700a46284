// Internal declarations of the GPU library (kernels, launchers, context).
// Nothing here is part of the C ABI; see include/lnf.h for that.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lnf.h"

namespace lnf {

constexpr int kXcds = 8;  // MI355X: 8 accelerator complex dies, one L2 each

// Geometry of one dense x-fastest volume.
struct Geom {
    int nx, ny, nz;
};

// Launch configuration chosen by the tuner or the caller.
struct TileCfg {
    int variant;  // index into the rule's table of compiled tile shapes
    int zs;       // output slices per workgroup (z-strip depth), > 0
};

// ---- MEAN9 (mean of the nine cluster means) -------------------------------
int mean9_variants();
int mean9_default_variant(int dtype, int r);
// Tile footprint of a variant: output tile width/height in x/y.
void mean9_tile_shape(int variant, int* tx, int* ty);
// With plan != nullptr the launchers only resolve the configuration they
// would launch (tile variant and z-strip depth) into *plan and launch nothing.
hipError_t launch_mean9(const void* in, void* out, int dtype, int r, Geom g, uint32_t gate,
                        TileCfg cfg, hipStream_t s, TileCfg* plan = nullptr);
// Whether a volume can be staged as element pairs: even row length and a base
// address aligned to a pair of elements.
inline bool mean9_pairs_ok(const void* base, int nx, size_t elem)
{
    return nx % 2 == 0 && reinterpret_cast<uintptr_t>(base) % (2 * elem) == 0;
}

// ---- geometry variants (plane_tile.h): LNF_GEOM_* bits, both rules ---------
hipError_t launch_geometry(int rule, uint32_t geom, const void* in, void* out, int dtype, int r,
                           Geom g, uint32_t gate, int zs, hipStream_t s, TileCfg* plan = nullptr);
// The paper's mean filter (eq. 4): rounded mean of the (2r+1)^3 cube, gated.
hipError_t launch_box_mean(const void* in, void* out, int dtype, int r, Geom g, uint32_t gate,
                           hipStream_t s);
// Sigma / Okada / entropy comparison filters (window.hip).
constexpr int kWinSigma = 0, kWinOkada = 1, kWinEntropy = 2;
hipError_t launch_window(int kind, const void* in, void* out, int dtype, int r, Geom g,
                         int64_t param, const int64_t* weights, uint32_t gate, hipStream_t s);

// ---- MINVAR9 (least-variance cluster) -------------------------------------
int minvar9_variants();
// Default tile variant for a volume of plane g.nx x g.ny.
int minvar9_default_variant(int dtype, int r, Geom g);
void minvar9_tile_shape(int variant, int r, int* tx, int* ty);  // output tile of (variant, r)
hipError_t launch_minvar9(const void* in, void* out, int dtype, int r, Geom g, uint32_t gate,
                          TileCfg cfg, hipStream_t s, TileCfg* plan = nullptr);

// Default z-strip depth: the strip count that minimises (rounds of
// target_groups resident workgroups over tiles_xy * strips) x (strip depth +
// 12 halo slices), strips at least 16 slices deep.
int default_zs(int tiles_xy, int nz, int target_groups);
// Workgroups of `kernel` (launched with `threads` threads, no dynamic LDS) that
// the current device holds at once: CUs x resident workgroups per CU.
int resident_groups(const void* kernel, int threads);

}  // namespace lnf
