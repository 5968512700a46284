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
int mean9_default_variant();
// Tile footprint of a variant: output tile width/height in x/y.
void mean9_tile_shape(int variant, int* tx, int* ty);
// narrow: x-pass sums fit 16 bits (uint8 data, or 12-bit uint16 data with r <= 3)
hipError_t launch_mean9(const void* in, void* out, int dtype, int r, Geom g, uint32_t gate,
                        TileCfg cfg, hipStream_t s, bool narrow);
// Whether the narrow MEAN9 path is valid for (dtype, r) under the context flags.
inline bool mean9_narrow(int dtype, int r, uint32_t flags)
{
    return dtype == LNF_U8 || ((flags & LNF_FLAG_DATA_12BIT) && r <= 3);
}

// ---- MINVAR9 (least-variance cluster) -------------------------------------
int minvar9_variants();
void minvar9_tile_shape(int variant, int* tx, int* ty);
hipError_t launch_minvar9(const void* in, void* out, int dtype, int r, Geom g, uint32_t gate,
                          TileCfg cfg, hipStream_t s);

// Default z-strip depth: enough workgroups to give every CU several tiles.
int default_zs(int tiles_xy, int nz, int target_groups);

}  // namespace lnf
