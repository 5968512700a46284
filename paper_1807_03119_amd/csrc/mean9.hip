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

constexpr int kThreads = 256;

// Output tile 64 (x) x 16 (y) per workgroup, streaming `zs` slices in z.
// Per input slice:
//   1. the raw (64+4r) x (16+4r) slice tile (clamped at the volume faces) is
//      written from registers into LDS, and the next slice's loads are issued;
//   2. x-pass: 8-wide row segments, prefix sums over the 8+4r raw values give
//      px = box_x E and qx = c_x E for the 16+4r rows;
//   3. y-pass: each thread owns one column x and four consecutive rows and
//      forms P = box_y px and Q = c_y qx from prefix sums over the column;
//   4. z-window: a ring of the last 4r+2 (P, Q) slices in registers keeps the
//      running sums B = box_z P (lagging 2r slices) and W = sum of Q over
//      [-2r, 2r]; the output slice z = zi - 2r is S = B + W + Q(z).
template <int R, typename T, bool GATE>
__global__ __launch_bounds__(kThreads) void mean9_ring_64x16(const T* __restrict__ in,
                                                             T* __restrict__ out, Geom g, int zs,
                                                             int tiles_x, int tiles_y, int total,
                                                             uint32_t gate, double inv9n)
{
    constexpr int TX = 64, TY = 16, H = 2 * R;
    constexpr int LX = TX + 2 * H, LY = TY + 2 * H;
    constexpr int NRAW = LX * LY;
    constexpr int NLOAD = (NRAW + kThreads - 1) / kThreads;
    constexpr int NFULL = NRAW / kThreads;
    constexpr int D = 4 * R + 2;  // ring period (slices kept per output column)
    constexpr int SEG = 8, NSEG = TX / SEG, SW = SEG + 4 * R;
    constexpr int YO = 4;  // outputs per thread along y
    constexpr int NPV = YO + 2 * R, NQV = YO + 4 * R;
    static_assert(LY * NSEG <= kThreads, "x-pass needs one thread per row segment");
    static_assert(TX * (TY / YO) == kThreads, "y-pass needs one thread per column quad");

    __shared__ __align__(16) uint32_t s_raw[LY * LX];
    __shared__ __align__(16) uint32_t s_px[LY * TX];
    __shared__ __align__(16) uint32_t s_qx[LY * TX];

    const int tid = threadIdx.x;
    const int tile = xcd_tile(blockIdx.x, total);
    const int bx = tile % tiles_x;
    const int rest = tile / tiles_x;
    const int by = rest % tiles_y;
    const int bz = rest / tiles_y;
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * zs;
    const int z1 = min(z0 + zs, g.nz);
    const size_t plane = (size_t)g.nx * g.ny;

    // In-slice offsets of the raw elements this thread stages (clamped).
    int off[NLOAD];
#pragma unroll
    for (int i = 0; i < NLOAD; ++i) {
        const int e = min(tid + i * kThreads, NRAW - 1);
        const int row = e / LX, col = e - row * LX;
        const int gy = clampi(y0 - H + row, 0, g.ny - 1);
        const int gx = clampi(x0 - H + col, 0, g.nx - 1);
        off[i] = gy * g.nx + gx;
    }
    const bool last_ok = tid + (NLOAD - 1) * kThreads < NRAW;

    uint32_t v[NLOAD];
    auto load = [&](int zi) {
        const T* base = in + (size_t)clampi(zi, 0, g.nz - 1) * plane;
#pragma unroll
        for (int i = 0; i < NLOAD; ++i) v[i] = base[off[i]];
    };

    const int xrow = tid / NSEG, xseg = tid % NSEG;
    const bool xactive = xrow < LY;
    const int xq = tid % TX, yg = tid / TX;

    uint32_t pr[D][YO], qr[D][YO], bacc[YO], wacc[YO];
#pragma unroll
    for (int m = 0; m < YO; ++m) {
        bacc[m] = wacc[m] = 0;
#pragma unroll
        for (int u = 0; u < D; ++u) pr[u][m] = qr[u][m] = 0;
    }

    const int ns = (z1 - z0) + 2 * H;  // input slices z0-2r .. z1-1+2r
    load(z0 - H);
    for (int kb = 0; kb < ns; kb += D) {
#pragma unroll
        for (int u = 0; u < D; ++u) {
            const int k = kb + u;
            if (k >= ns) break;
            // 1. stage slice k, prefetch slice k+1
#pragma unroll
            for (int i = 0; i < NLOAD; ++i)
                if (i < NFULL || last_ok) s_raw[tid + i * kThreads] = v[i];
            if (k + 1 < ns) load(z0 - H + k + 1);
            __syncthreads();

            // 2. x-pass
            if (xactive) {
                uint32_t w[SW], c[SW];
                const uint32_t* rp = s_raw + xrow * LX + xseg * SEG;
#pragma unroll
                for (int i = 0; i < SW; i += 4) {
                    const uint4 t4 = *reinterpret_cast<const uint4*>(rp + i);
                    w[i] = t4.x;
                    w[i + 1] = t4.y;
                    w[i + 2] = t4.z;
                    w[i + 3] = t4.w;
                }
                c[0] = w[0];
#pragma unroll
                for (int i = 1; i < SW; ++i) c[i] = c[i - 1] + w[i];
                uint32_t pp[SEG], qq[SEG];
#pragma unroll
                for (int m = 0; m < SEG; ++m) {
                    qq[m] = c[m + 4 * R] - (m ? c[m - 1] : 0u) + w[m + 2 * R];
                    pp[m] = c[m + 3 * R] - c[m + R - 1];
                }
                uint32_t* pd = s_px + xrow * TX + xseg * SEG;
                uint32_t* qd = s_qx + xrow * TX + xseg * SEG;
#pragma unroll
                for (int m = 0; m < SEG; m += 4) {
                    *reinterpret_cast<uint4*>(pd + m) = make_uint4(pp[m], pp[m + 1], pp[m + 2], pp[m + 3]);
                    *reinterpret_cast<uint4*>(qd + m) = make_uint4(qq[m], qq[m + 1], qq[m + 2], qq[m + 3]);
                }
            }
            __syncthreads();

            // 3. y-pass for rows yg*4 .. yg*4+3 of column xq
            uint32_t cp[NPV], cq[NQV], qc[YO];
            cp[0] = s_px[(yg * YO + R) * TX + xq];
#pragma unroll
            for (int i = 1; i < NPV; ++i) cp[i] = cp[i - 1] + s_px[(yg * YO + R + i) * TX + xq];
            {
                uint32_t qv[NQV];
#pragma unroll
                for (int i = 0; i < NQV; ++i) qv[i] = s_qx[(yg * YO + i) * TX + xq];
                cq[0] = qv[0];
#pragma unroll
                for (int i = 1; i < NQV; ++i) cq[i] = cq[i - 1] + qv[i];
#pragma unroll
                for (int m = 0; m < YO; ++m) qc[m] = qv[m + 2 * R];
            }

            // 4. z-window over the register ring
#pragma unroll
            for (int m = 0; m < YO; ++m) {
                const uint32_t P = cp[m + 2 * R] - (m ? cp[m - 1] : 0u);
                const uint32_t Q = cq[m + 4 * R] - (m ? cq[m - 1] : 0u) + qc[m];
                bacc[m] += pr[(u + D - R) % D][m] - pr[(u + R + 1) % D][m];
                wacc[m] += Q - qr[(u + 1) % D][m];
                pr[u][m] = P;
                qr[u][m] = Q;
            }
            if (k >= 2 * H) {
                const int z = z0 + k - 2 * H;
                T* op = out + (size_t)z * plane;
                const int x = x0 + xq;
#pragma unroll
                for (int m = 0; m < YO; ++m) {
                    const uint32_t S = bacc[m] + wacc[m] + qr[(u + D - 2 * R) % D][m];
                    uint32_t o = round_div_odd(S, inv9n);
                    if (GATE && o < gate) o = 0;
                    const int y = y0 + yg * YO + m;
                    if (x < g.nx && y < g.ny) op[(size_t)y * g.nx + x] = (T)o;
                }
            }
        }
    }
}

// Single-volume wrapper around the streaming tile body of mean9_tile.h.
// At least 2 waves per SIMD: at r = 4 the tile would take 274-285 VGPRs (one
// wave per SIMD); capped at 256 it spills a little and still runs faster
// (512^3, r = 4: uint16 406 -> 425, uint8 418 -> 466 Gvox/s); r <= 3 fits anyway.
template <int R, int TY, typename T, bool GATE, int TXW>
__global__ __launch_bounds__((M9Shape<R, TY, TXW>::THREADS))
__attribute__((amdgpu_waves_per_eu(2))) void mean9_stream(
    const T* __restrict__ in, T* __restrict__ out, Geom g, int zs, int tiles_x, int tiles_y,
    int total, uint32_t gate, double inv9n, int pairs)
{
    __shared__ __align__(16) M9SmemAny<R, TY, TXW> sm;
    const int tile = xcd_tile(blockIdx.x, total);
    const int bx = tile % tiles_x;
    const int rest = tile / tiles_x;
    const int by = rest % tiles_y;
    const int bz = rest / tiles_y;
    const int z0 = bz * zs;
    mean9_tile<R, TY, T, GATE, TXW>(sm, pairs != 0, in, out, g, bx * TXW, by * TY, z0,
                                    min(z0 + zs, g.nz), gate, inv9n);
}

// The paper's mean filter (eq. 4): the box term of the same streaming tile,
// 64 x 16 tiles.
template <int R, typename T, bool GATE>
__global__ __launch_bounds__((M9Shape<R, 16, 64>::THREADS)) void box_mean_stream(
    const T* __restrict__ in, T* __restrict__ out, Geom g, int zs, int tiles_x, int tiles_y,
    int total, uint32_t gate, double invn, int pairs)
{
    __shared__ __align__(16) M9SmemAny<R, 16, 64, true> sm;
    const int tile = xcd_tile(blockIdx.x, total);
    const int bx = tile % tiles_x;
    const int rest = tile / tiles_x;
    const int by = rest % tiles_y;
    const int bz = rest / tiles_y;
    const int z0 = bz * zs;
    mean9_tile<R, 16, T, GATE, 64, true>(sm, pairs != 0, in, out, g, bx * 64, by * 16, z0,
                                         min(z0 + zs, g.nz), gate, invn);
}

template <int R, typename T, bool GATE>
hipError_t launch_box(const T* in, T* out, Geom g, uint32_t gate, hipStream_t s)
{
    constexpr int threads = M9Shape<R, 16, 64>::THREADS;
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
// 0: first design (two barriers per slice, register staging)
// 1-4: LDS-DMA staging ring, one barrier per slice; 64 or 32 wide, 16 or 32 high
constexpr Variant kVariants[] = {{64, 16, 256}, {64, 16, 256}, {64, 32, 512}, {32, 16, 128},
                                 {32, 32, 256}};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

// Default variant per voxel type and radius (index r-1): the fastest at the
// default z-strip depth on 512^3 volumes.
constexpr int kDefaultU16[LNF_RADIUS_MAX] = {2, 1, 1, 4};
constexpr int kDefaultU8[LNF_RADIUS_MAX] = {2, 4, 3, 3};

template <int R, typename T, bool GATE, int TY, int TXW>
hipError_t launch_stream(const T* in, T* out, Geom g, uint32_t gate, int zs, hipStream_t s)
{
    static_assert(M9Shape<R, TY, TXW, true>::THREADS == M9Shape<R, TY, TXW>::THREADS, "");
    constexpr int threads = M9Shape<R, TY, TXW>::THREADS;
    const auto kern = mean9_stream<R, TY, T, GATE, TXW>;
    const int tiles_x = (g.nx + TXW - 1) / TXW, tiles_y = (g.ny + TY - 1) / TY;
    // default z-strip depth: one full round of resident workgroups
    if (zs <= 0)
        zs = default_zs(tiles_x * tiles_y, g.nz, resident_groups((const void*)kern, threads));
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
                          hipStream_t s)
{
    const T* pin = static_cast<const T*>(in);
    T* pout = static_cast<T*>(out);
    switch (variant) {
    case 0: {
        const int tiles_x = (g.nx + 63) / 64, tiles_y = (g.ny + 15) / 16;
        if (zs <= 0) zs = default_zs(tiles_x * tiles_y, g.nz, 1024);
        const int total = tiles_x * tiles_y * ((g.nz + zs - 1) / zs);
        const int n = (2 * R + 1) * (2 * R + 1) * (2 * R + 1);
        hipLaunchKernelGGL((mean9_ring_64x16<R, T, GATE>), dim3(total), dim3(kThreads), 0, s, pin,
                           pout, g, zs, tiles_x, tiles_y, total, gate, 1.0 / (9.0 * n));
        return hipGetLastError();
    }
    case 1: return launch_stream<R, T, GATE, 16, 64>(pin, pout, g, gate, zs, s);
    case 2: return launch_stream<R, T, GATE, 32, 64>(pin, pout, g, gate, zs, s);
    case 3: return launch_stream<R, T, GATE, 16, 32>(pin, pout, g, gate, zs, s);
    default: return launch_stream<R, T, GATE, 32, 32>(pin, pout, g, gate, zs, s);
    }
}

template <int R, typename T>
hipError_t launch_r(int variant, const void* in, void* out, Geom g, uint32_t gate, int zs,
                    hipStream_t s)
{
    if (gate) return launch_variant<R, T, true>(variant, in, out, g, gate, zs, s);
    return launch_variant<R, T, false>(variant, in, out, g, gate, zs, s);
}

template <typename T>
hipError_t dispatch_r(const void* in, void* out, int r, Geom g, uint32_t gate, TileCfg cfg,
                      hipStream_t s)
{
    if (r < 1 || r > LNF_RADIUS_MAX) return hipErrorInvalidValue;
    const int v = (cfg.variant >= 0 && cfg.variant < kNumVariants)
                      ? cfg.variant
                      : mean9_default_variant(sizeof(T) == 1 ? LNF_U8 : LNF_U16, r);
    switch (r) {
    case 1: return launch_r<1, T>(v, in, out, g, gate, cfg.zs, s);
    case 2: return launch_r<2, T>(v, in, out, g, gate, cfg.zs, s);
    case 3: return launch_r<3, T>(v, in, out, g, gate, cfg.zs, s);
    default: return launch_r<4, T>(v, in, out, g, gate, cfg.zs, s);
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
    const Variant v = kVariants[(variant >= 0 && variant < kNumVariants) ? variant : 1];
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
                        TileCfg cfg, hipStream_t s)
{
    if (dtype == LNF_U8) return dispatch_r<uint8_t>(in, out, r, g, gate, cfg, s);
    return dispatch_r<uint16_t>(in, out, r, g, gate, cfg, s);
}

}  // namespace lnf
