// Per-plane cluster tile: one workgroup filters a TX x TY column of output
// voxels over the z-range [z0, z1), for every cluster geometry and both rules.
//
// Geometry (paper, Section "Our Method", nine-cluster figure and eq. 2):
// cluster 0 is centred on the voxel, clusters 1..8 at (-+D, -+D, -+D), x
// varying fastest; a cluster is the (2r+1)^3 cube around its centre, or the
// cross of the three axis lines of 2r+1 voxels through it (the centre counted
// once per line).  Rules: MEAN9 writes round(sum of the nine cluster sums /
// 9n); MINVAR9 (not in the paper) writes the rounded mean of the cluster with
// the least n*q - s^2, the lowest index winning ties.
//
// The nine centres of output (x, y, z) lie on three planes, z and z -+ D, and
// the four of one plane keep the cluster order, so the tile runs one centre
// plane p at a time:
//   1. z-sums: each thread owns raw columns of the (TX+2(D+r)) x (TY+2(D+r))
//      tile and keeps Zb = sum of E and Zq = sum of E^2 over slices p-r .. p+r,
//      adding slice p+r and removing slice p-r-1 (loaded one plane ahead; the
//      removed slice was read 2r+1 planes earlier and comes from L2); crosses
//      also load slice p itself.  All go to LDS;
//   2. cubes: x-pass, sums over 2r+1 columns of Zb (Zq) on every raw row.
//      Crosses: x-lines and y-lines of slice p through every centre;
//   3. cubes: y-pass, sums over 2r+1 rows of the x-pass output.  Crosses: the
//      z-line (Zb at the centre) plus the two lines.  Either gives the cluster
//      sums B (and Q) at every centre of the (TX+2D) x (TY+2D) region; MINVAR9
//      turns them into v = n*Q - B^2 (fp64, exact: every value is an integer
//      below 2^53) and the rounded mean, MEAN9 keeps B; one LDS plane;
//   4. gather: each output reads its centre entry C and the four corner
//      entries (x -+ D, y -+ D) of the plane.  MEAN9 adds them up (K = corner
//      sum), MINVAR9 takes their first minimum in cluster order (G).  Output
//      z combines C(z) with the corner groups of planes z - D and z + D, in
//      that order; a register ring per output keeps the z - D group for D
//      planes and the combination with C(z) for D more.
// Each step reads what the previous one wrote to LDS, so a plane takes three
// barriers; the narrow MINVAR9 tiles from r = 2 overlap steps 3-4 of plane
// p - 1 with steps 1-2 of plane p instead (two barriers, two keys planes).
// Sums of squares are fp64 for uint16 data (below 2^42) and uint32 for uint8
// data (below 2^26); MINVAR9 cubes on uint16 data keep them in uint32 through
// the z- and x-passes while the tile's values allow it (NQ below).
#pragma once

#include <cstddef>
#include <type_traits>

#include "device_common.h"
#include "lnf_internal.h"

namespace lnf {

constexpr int kClusterBox = 0, kClusterCross = 1;
constexpr int kRuleMean9 = 0, kRuleMinVar9 = 1;

// LDS layout.  Bank conflicts come from lane groups that span two rows of an
// array (the z-sum writes: 64 lanes over rows of the raw tile; the y-pass:
// lanes over the centre columns, one row segment after the other), and from
// 16-byte accesses whose eight lanes per bank cycle fall in the same bank
// group.  The pitches below make the rows such a group spans continue each
// other in bank space, and give the eight rows of one 16-byte access distinct
// bank groups.
//
// Smallest pitch p >= lo with p = 2 mod 4 (when asked) and ys * p = g (mod m).
constexpr int pt_find_pitch(int ys, int g, int lo, int m, bool two_mod4)
{
    for (int p = lo; p < lo + 64; ++p)
        if ((!two_mod4 || p % 4 == 2) && (ys * p - g) % m == 0) return p;
    return -1;
}
// The y-pass segment height: the smallest that fits the threads and admits
// all three pitches, else the smallest that fits.
constexpr int pt_pick_ys(int gx, int gy, int xw, int threads)
{
    int first = 0;
    for (int ys = 1; ys <= gy; ++ys) {
        if ((gy + ys - 1) / ys * gx > threads) continue;
        if (!first) first = ys;
        if (pt_find_pitch(ys, gx, xw, 32, true) > 0 && pt_find_pitch(ys, gx, xw, 16, true) > 0 &&
            pt_find_pitch(ys, gx, gx, 32, false) > 0)
            return ys;
    }
    return first;
}
// The pitch found, else lo rounded up to even (8-byte rows of pairs).
constexpr int pt_pitch(int ys, int g, int lo, int m, bool two_mod4)
{
    return pt_find_pitch(ys, g, lo, m, two_mod4) > 0 ? pt_find_pitch(ys, g, lo, m, two_mod4)
                                                      : lo + (lo & 1);
}

// WT (wide tile): MINVAR9 cubes at offset r up to r = 3 fit 4 waves per SIMD,
// so 64 x 16 tiles in 512-thread workgroups cost less halo at the same
// occupancy: faster on large uint16 planes (r = 3: 214 -> 228 Gvox/s), slower
// on small volumes and on uint8 at r = 2.  A tile variant, chosen per launch.
template <int R, int D, int SHAPE, int RULE, bool WT = false>
struct PTShape {
    static constexpr bool CROSS = SHAPE == kClusterCross;
    static constexpr bool VAR = RULE == kRuleMinVar9;
    static constexpr bool BIG = WT && VAR && !CROSS && D == R && R <= 3;
    static constexpr int THREADS = BIG ? 512 : 256;
    // 16 output rows, except where a deep ring (D > r) of MINVAR9 entries
    // would push registers past about 200: crosses from r = 3, every r = 4
    static constexpr int TX = BIG ? 64 : 32, TY = (D <= R || !VAR || R <= 2 || (R == 3 && !CROSS)) ? 16 : 8;
    static constexpr int M = 2 * R + 1;
    static constexpr int N = CROSS ? 3 * M : M * M * M;   // voxels per cluster
    static constexpr int E = D + R;                       // raw halo
    static constexpr int LX = TX + 2 * E, LY = TY + 2 * E;  // raw tile
    static constexpr int GX = TX + 2 * D, GY = TY + 2 * D;  // centre region
    static constexpr int NRAW = LX * LY;
    static constexpr int NZ = (NRAW + THREADS - 1) / THREADS;  // raw columns per thread
    // x-pass: XS centre columns per row segment; consecutive lanes take
    // consecutive rows of a segment, XR rows per segment.  Cubes run it over
    // every raw row, crosses over the raw rows through centres (from row r).
    // Rows padded to a multiple of 8 keep the 16-byte reads of eight lanes in
    // distinct bank groups; unpadded rows are used where they need fewer
    // waves (the x-pass runs on as many waves as its items fill: 28 rows x 9
    // segments fit 4 waves, 32 x 9 take 5, and the fifth shares a SIMD with
    // the first; MINVAR9 r = 3, 64 x 16 tiles: 551 -> 527 us per 512^3).
    static constexpr int XIN = CROSS ? GY : LY;
    static constexpr int XROW0 = CROSS ? R : 0;
    static constexpr int XS = 8;
    static constexpr int NXS = (GX + XS - 1) / XS;
    static constexpr int XR8 = (XIN + 7) / 8 * 8;
    static constexpr int XR = (XIN * NXS + 63) / 64 < (XR8 * NXS + 63) / 64 ? XIN : XR8;
    static constexpr int NXI = XR * NXS;                  // x-pass work items
    // MINVAR9 cubes run the x-passes of the sums and of the squares as
    // separate items on separate waves where both fit the workgroup: the
    // sums on the threads below QOFF, the squares on those from QOFF
    // (512-thread tiles: r = 3 527 -> 514 us, r = 1 357 -> 335 us)
    static constexpr int QOFF = (NXI + 63) / 64 * 64;
    static constexpr bool XSPLIT = VAR && !CROSS && QOFF + NXI <= THREADS;
    static constexpr int XW = XS + 2 * R;                 // raw values a segment reads
    static constexpr int XW4 = (XW + 3) / 4 * 4;          // ... rounded to 16-byte reads
    // y-pass: YS centre rows per column segment
    static constexpr int YS = pt_pick_ys(GX, GY, NXS * XS, THREADS);
    static_assert(YS > 0, "y-pass does not fit the workgroup");
    static constexpr int NYS = (GY + YS - 1) / YS;
    static constexpr int YW = YS + 2 * R;                 // rows a segment reads
    static constexpr int YROWS = NYS * YS + 2 * R > LY ? NYS * YS + 2 * R : LY;
    // z-sum rows (32-bit words): the pitch is the row length when that is
    // 4 mod 8 (rows continue each other, and eight rows of a 16-byte x-pass
    // read start in distinct bank groups), else the next such length.  The
    // x-pass reads XW4 words from each segment start, past the row end into
    // the next row, and the cross y-lines read rows past the tile: those
    // values only feed centres outside the region.
    static constexpr int ZP = LX + (12 - LX % 8) % 8;
    static constexpr int ZROWS = CROSS ? YROWS : LY;
    static constexpr int ZN = ((ZROWS - 1) * ZP + (NXS - 1) * XS + XW4 + 3) / 4 * 4;
    // x-pass output rows (cubes: written 8 bytes per lane by 16 consecutive
    // rows, read by the y-pass; crosses: x- and y-lines at the centres) and
    // centre planes: pitches whose rows YS apart continue each other
    static constexpr int XROWS = CROSS ? GY : YROWS;
    static constexpr int XPB = pt_pitch(YS, GX, NXS * XS, 32, true);
    static constexpr int XPD = pt_pitch(YS, GX, NXS * XS, 16, true);  // 64-bit
    static constexpr int VP = pt_pitch(YS, GX, GX, 32, false);
    static constexpr int OPT = TX * TY / THREADS;         // outputs per thread
    static constexpr int OROWS = THREADS / TX;            // output rows per pass
    static constexpr int U = D + 1;                       // register ring period
    // waves per SIMD the kernels are compiled for: MINVAR9 cubes at offset r
    // get 4 up to r = 3 (at most 128 VGPRs, no spills) and 3 at r = 4 (168
    // VGPRs; a few spills for uint16, still 13 % faster than 2 waves); the
    // others have no limit below 256 VGPRs
    static constexpr int WAVES = (VAR && !CROSS && D == R) ? (R <= 3 ? 4 : 3) : 2;
    static_assert(THREADS % TX == 0 && OPT * OROWS == TY, "gather mapping");
};

// Values below 2^nq_bits(R) keep every sum of squares that the z- and x-passes
// of a (2r+1)^3 cube form, (2r+1)^2 squares, below 2^32.
constexpr int nq_bits(int r)
{
    int b = 16;
    while (b > 0 && (double)(2 * r + 1) * (2 * r + 1) * ((1 << b) - 1.0) * ((1 << b) - 1.0) >= 4294967296.0)
        --b;
    return b;
}

// NQ (narrow squares, MINVAR9 cubes on uint16 data): the z- and x-passes keep
// the sums of squares in uint32, which is exact while every value is below
// 2^nq_bits(r) (14, 13, 13, 12 bits for r = 1..4: 12-bit CT data always); the
// y-pass adds them up in fp64.  The tile body checks the values it loads and
// gives up when one is too large; the caller then runs the tile again with
// fp64 sums.
template <int R, int D, int SHAPE, int RULE, typename T, bool WT = false, bool NQ = false>
struct PTSmem {
    using S = PTShape<R, D, SHAPE, RULE, WT>;
    // sums of squares: fp64 for uint16 data, staged in LDS as two 32-bit
    // halves (so they share the 32-bit layout); uint32 for uint8 data and NQ
    using QT = std::conditional_t<sizeof(T) == 1 || NQ, uint32_t, double>;
    // the y-pass sums of squares and the cluster sums Q
    using YQ = std::conditional_t<sizeof(T) == 1, uint32_t, double>;
    static constexpr bool VAR = S::VAR, CROSS = S::CROSS;
    static constexpr bool WIDE = sizeof(QT) == 8;
    // MINVAR9 centre entries as one 64-bit key v * 2^16 + rounded mean, when
    // every v fits 48 bits: v = n^2 times a variance of values in [0, vmax],
    // so v <= n^2 vmax^2 / 4 (uint16 cubes up to r = 3, crosses, all uint8)
    static constexpr double VMAX = sizeof(T) == 1 ? 255.0 : 65535.0;
    static constexpr bool PACK =
        VAR && (double)S::N * S::N * VMAX * VMAX / 4.0 < 281474976710656.0;  // 2^48
    static constexpr int XPQ = WIDE ? S::XPD : S::XPB;
    // every array a multiple of 16 bytes, so each starts 16-byte aligned
    static constexpr int a16(int n, int bytes) { return (n * bytes + 15) / 16 * 16 / bytes; }
    static constexpr int QN = VAR ? 1 : 0, CN = CROSS ? 1 : 0;
    QT xq[QN ? a16(S::XROWS * XPQ, sizeof(QT)) : a16(1, sizeof(QT))];
    QT yq[QN * CN ? a16(S::XROWS * XPQ, sizeof(QT)) : a16(1, sizeof(QT))];  // crosses: y-lines of E^2
    // MINVAR9: v, or the packed keys (two planes for NQ from r = 2, whose
    // tile body gathers from one plane while the next is written)
    double vv[QN ? (NQ && R >= 2 ? 2 : 1) * a16(S::GY * S::VP, 8) : 2];
    uint32_t zb[S::ZN];
    uint32_t zq0[QN ? S::ZN : 4];                // uint8: Zq; uint16: low half of Zq
    uint32_t zq1[QN && WIDE ? S::ZN : 4];        // uint16: high half of Zq
    uint32_t ec[CN ? S::ZN : 4];                 // crosses: slice p
    uint32_t xb[a16(S::XROWS * S::XPB, 4)];      // cubes: x-pass; crosses: x-lines
    uint32_t yb[CN ? a16(S::XROWS * S::XPB, 4) : 4];  // crosses: y-lines
    uint32_t vo[PACK ? 4 : a16(S::GY * S::VP, 4)];  // MINVAR9: rounded means; MEAN9: B
};

// dn = n; inv = 1/n (MINVAR9) or 1/(9n) (MEAN9); tid: threadIdx.x (see
// tile_tid for loops over several tiles).  NQ: narrow sums of squares; `flag`
// is an LDS word of the caller's, and the body returns false, with every
// thread, when a value of the tile is too large for them (whatever it stored
// is then to be written again).  Otherwise it returns true.
template <int R, int D, int SHAPE, int RULE, typename T, bool GATE, bool WT = false,
          bool NQ = false>
__device__ __forceinline__ bool plane_tile(PTSmem<R, D, SHAPE, RULE, T, WT, NQ>& sm,
                                           const T* __restrict__ in, T* __restrict__ out, Geom g,
                                           int x0, int y0, int z0, int z1, uint32_t gate,
                                           double dn, double inv, int tid, int* flag = nullptr)
{
    using S = PTShape<R, D, SHAPE, RULE, WT>;
    using SM = PTSmem<R, D, SHAPE, RULE, T, WT, NQ>;
    using QT = typename SM::QT;
    using YQ = typename SM::YQ;
    constexpr bool VAR = S::VAR, CROSS = S::CROSS, WIDE = SM::WIDE, PACK = SM::PACK;
    static_assert(!NQ || (VAR && !CROSS && sizeof(T) == 2 && PACK),
                  "narrow squares: MINVAR9 cubes, uint16, packed keys");
    constexpr uint32_t kNQLimit = 1u << nq_bits(R);
    static_assert(offsetof(SM, vv) % 16 == 0 && offsetof(SM, zb) % 16 == 0 &&
                      offsetof(SM, zq0) % 16 == 0 && offsetof(SM, zq1) % 16 == 0 &&
                      offsetof(SM, ec) % 16 == 0 && offsetof(SM, xb) % 16 == 0 &&
                      offsetof(SM, yb) % 16 == 0 && offsetof(SM, vo) % 16 == 0,
                  "16-byte LDS accesses need 16-byte aligned arrays");
    constexpr int kT = S::THREADS, LX = S::LX, GX = S::GX, XS = S::XS, YS = S::YS;
    constexpr int U = S::U, OPT = S::OPT, VP = S::VP;
    const size_t plane = (size_t)g.nx * g.ny;
    const uint32_t pbytes = (uint32_t)(plane * sizeof(T));

    // NQ tiles from r = 2 run as a two-barrier pipeline (below)
    constexpr bool PIPE = NQ && R >= 2;
    // ---- raw columns owned for the z-sums.  Pipelined tiles rotate them so
    // that the partial last round falls on the highest threads, whose waves
    // have no y-pass work in the same phase.
    constexpr unsigned ZROT = PIPE ? (unsigned)(S::NRAW - (S::NZ - 1) * kT) : 0u;
    const int zt = PIPE ? (int)(((unsigned)tid + ZROT) % (unsigned)kT) : tid;
    uint32_t off[S::NZ];
    int zi[S::NZ];  // LDS index of each owned column
#pragma unroll
    for (int i = 0; i < S::NZ; ++i) {
        const int e = min(zt + i * kT, S::NRAW - 1);
        const int row = e / LX, col = e - row * LX;
        off[i] = (uint32_t)(clampi(y0 - S::E + row, 0, g.ny - 1) * g.nx +
                            clampi(x0 - S::E + col, 0, g.nx - 1)) * (uint32_t)sizeof(T);
        zi[i] = row * S::ZP + col;
    }
    // lanes past the tile in the last round own no column
    const bool zlast = zt + (S::NZ - 1) * kT < S::NRAW;
    auto load = [&](uint32_t(&v)[S::NZ], int zs) {
        const rsrc_t rs = make_rsrc(in + (size_t)clampi(zs, 0, g.nz - 1) * plane, pbytes);
#pragma unroll
        for (int i = 0; i < S::NZ; ++i) v[i] = buffer_load<T>(rs, off[i]);
    };
    auto sq = [](uint32_t e) -> QT {
        if constexpr (WIDE) return (double)e * (double)e;  // exact: below 2^32
        else return e * e;
    };

    // ---- output columns (gather) and their store offsets
    const int ox = tid % S::TX, oyb = tid / S::TX;
    uint32_t soff[OPT];
#pragma unroll
    for (int j = 0; j < OPT; ++j) {
        const int x = x0 + ox, y = y0 + oyb + j * S::OROWS;
        soff[j] = (x < g.nx && y < g.ny) ? (uint32_t)(y * g.nx + x) * (uint32_t)sizeof(T) : pbytes;
    }

    // ---- z-sums over the first plane's window but its newest slice
    const int p0 = z0 - D;
    uint32_t zb[S::NZ];
    QT zq[S::NZ];
    uint32_t orv = 0;  // NQ: OR of every value loaded
    if constexpr (NQ)
        if (tid == 0) *flag = 0;
#pragma unroll
    for (int i = 0; i < S::NZ; ++i) {
        zb[i] = 0;
        zq[i] = 0;
    }
#pragma unroll
    for (int s = 0; s < 2 * R; ++s) {
        uint32_t e[S::NZ];
        load(e, p0 - R + s);
#pragma unroll
        for (int i = 0; i < S::NZ; ++i) {
            zb[i] += e[i];
            if constexpr (VAR) zq[i] += sq(e[i]);
            if constexpr (NQ) orv |= e[i];
        }
    }
    uint32_t en[S::NZ], eo[S::NZ], ec[S::NZ];
    load(en, p0 + R);
    if constexpr (CROSS) load(ec, p0);
#pragma unroll
    for (int i = 0; i < S::NZ; ++i) eo[i] = 0;

    // ---- register rings of the pending outputs: MINVAR9 (value, rounded
    // mean) of the best so far, MEAN9 partial sums
    double av[U][OPT], mv[U][OPT];
    uint32_t ao[U][OPT], mo[U][OPT];
    uint64_t ak[U][OPT], mk[U][OPT];  // packed keys
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int j = 0; j < OPT; ++j) {
            av[u][j] = mv[u][j] = 0.0;
            ao[u][j] = mo[u][j] = 0;
            ak[u][j] = mk[u][j] = 0;
        }
    uint64_t* const keys = reinterpret_cast<uint64_t*>(sm.vv);
    constexpr uint64_t kHigh = ~0xffffull;  // a key's v part (key & kHigh = v * 2^16)

    // y-pass mapping: consecutive lanes take consecutive centre columns
    const int ycol = tid % GX, yseg = tid / GX;
    const bool yact = yseg < S::NYS;

    // x-pass over the 32-bit array `src`: row segments of raw rows XROW0 +
    // row, box sums over 2r+1 columns for the centre columns, written to xb at
    // x-pass row `row`; for MINVAR9 the same for the squares, written to xq.
    // Crosses square the raw values of `src`; cubes read Zq from `src0` (low
    // halves, or the uint32 sums) and `src1` (high halves, uint16 data).
    auto xpass_items = [&](const uint32_t* src, const uint32_t* src0, const uint32_t* src1,
                           int it0, bool do_b, bool do_q) {
        for (int it = it0; it < S::NXI; it += kT) {
            const int xrow = it % S::XR, xseg = it / S::XR;
            if (xrow >= S::XIN) continue;
            const int cbase = xseg * XS;
            const int zr = (S::XROW0 + xrow) * S::ZP + cbase;
            // sums first, then squares: one row segment live at a time keeps
            // the x-pass within the 4-waves-per-SIMD register budget
            uint32_t w[S::XW4];
            auto read_row = [&](const uint32_t* a) {
#pragma unroll
                for (int i = 0; i < S::XW4; i += 4) {
                    const uint4 t = *reinterpret_cast<const uint4*>(a + zr + i);
                    w[i] = t.x;
                    w[i + 1] = t.y;
                    w[i + 2] = t.z;
                    w[i + 3] = t.w;
                }
            };
            uint32_t* db = sm.xb + xrow * S::XPB + cbase;
            QT* dq = sm.xq + xrow * SM::XPQ + cbase;
            if (do_b || CROSS) read_row(src);
            if (do_b) {
                uint32_t cb[S::XW];
                cb[0] = w[0];
#pragma unroll
                for (int i = 1; i < S::XW; ++i) cb[i] = cb[i - 1] + w[i];
                uint32_t ob[XS];
#pragma unroll
                for (int m = 0; m < XS; ++m) ob[m] = cb[m + 2 * R] - (m ? cb[m - 1] : 0u);
#pragma unroll
                for (int m = 0; m < XS; m += 2)
                    *reinterpret_cast<uint2*>(db + m) = make_uint2(ob[m], ob[m + 1]);
            }
            if constexpr (VAR) if (do_q) {
                QT cq[S::XW];
                if constexpr (CROSS) {  // squares of the raw row just read
#pragma unroll
                    for (int i = 0; i < S::XW; ++i) cq[i] = sq(w[i]);
                } else if constexpr (WIDE) {  // Zq from its two 32-bit halves
                    uint32_t lo[S::XW4];
                    read_row(src0);
#pragma unroll
                    for (int i = 0; i < S::XW4; ++i) lo[i] = w[i];
                    read_row(src1);
#pragma unroll
                    for (int i = 0; i < S::XW; ++i)
                        cq[i] = __builtin_bit_cast(double, ((uint64_t)w[i] << 32) | lo[i]);
                } else {
                    read_row(src0);
#pragma unroll
                    for (int i = 0; i < S::XW; ++i) cq[i] = w[i];
                }
#pragma unroll
                for (int i = 1; i < S::XW; ++i) cq[i] += cq[i - 1];
                QT oq[XS];
#pragma unroll
                for (int m = 0; m < XS; ++m) oq[m] = cq[m + 2 * R] - (m ? cq[m - 1] : (QT)0);
#pragma unroll
                for (int m = 0; m < XS; m += 2) {
                    if constexpr (WIDE)
                        *reinterpret_cast<double2*>(dq + m) = make_double2(oq[m], oq[m + 1]);
                    else
                        *reinterpret_cast<uint2*>(dq + m) = make_uint2(oq[m], oq[m + 1]);
                }
            }
        }
    };
    auto xpass = [&](const uint32_t* src, const uint32_t* src0, const uint32_t* src1) {
        if constexpr (S::XSPLIT) {
            if (tid < S::QOFF) xpass_items(src, src0, src1, tid, true, false);
            else xpass_items(src, src0, src1, tid - S::QOFF, false, true);
        } else {
            xpass_items(src, src0, src1, tid, true, true);
        }
    };

    // the centre statistics of one centre: MINVAR9 (v, rounded mean), MEAN9 B
    auto centre_out = [&](int gy, int gx, uint32_t b, YQ qv) {
        if constexpr (PACK) {
            // v + 2^52 is exact (v < 2^48), so its mantissa field is v
            const double db = (double)b;
            const double vb = __builtin_fma(dn, (double)qv, __builtin_fma(-db, db, 0x1p52));
            const uint64_t v = __builtin_bit_cast(uint64_t, vb) & ((1ull << 52) - 1);
            keys[gy * VP + gx] = (v << 16) | round_div_odd(b, inv);
        } else if constexpr (VAR) {
            const double db = (double)b;
            sm.vv[gy * VP + gx] = __builtin_fma(dn, (double)qv, -db * db);
            sm.vo[gy * VP + gx] = round_div_odd(b, inv);
        } else {
            sm.vo[gy * VP + gx] = b;
        }
    };

    // centre planes z0-D .. z1-1+D, in whole blocks of U (no exit inside the
    // unrolled block); the planes past the end read clamped slices and store
    // nothing
    const int npl = (z1 - z0) + 2 * D;
    // NQ tiles from r = 2 run as a pipeline with two barriers per plane: the
    // y-pass of the previous plane shares a phase with the z-sums of this one,
    // and its gather (issued first) a phase with this plane's x-pass; the keys
    // planes alternate (512^3, 12-bit: r = 3 467 -> 445 us per launch, 288 ->
    // 302 Gvoxel/s; r = 2 428 -> 394 us; r = 1 was slower, 440 -> 392).  The other tiles take the four phases in
    // turn, three barriers a plane, in the loop below the pipelined one (kept
    // apart: folding the two into shared helpers cost r = 1 13 %).
    if constexpr (PIPE) {
        constexpr int KSZ = SM::a16(S::GY * VP, 8);  // keys per plane
        auto kbuf = [&](int q) { return keys + ((q & 1) ? KSZ : 0); };
        // the packed key of one centre, written to plane kb
        auto centre_key = [&](uint64_t* kb, int gy, int gx, uint32_t b, YQ qv) {
            const double db = (double)b;
            const double vb = __builtin_fma(dn, (double)qv, __builtin_fma(-db, db, 0x1p52));
            const uint64_t v = __builtin_bit_cast(uint64_t, vb) & ((1ull << 52) - 1);
            kb[gy * VP + gx] = (v << 16) | round_div_odd(b, inv);
        };
        // cluster sums at every centre of the region, as keys in plane kb
        auto ypass_cubes = [&](uint64_t* kb) {
            // y-pass: centre row c covers x-pass rows c .. c+2r
            if (yact) {
                const int rbase = yseg * YS;
                uint32_t cb[S::YW];
                YQ cq[S::YW];
#pragma unroll
                for (int t = 0; t < S::YW; ++t) {
                    const uint32_t b = sm.xb[(rbase + t) * S::XPB + ycol];
                    cb[t] = t ? cb[t - 1] + b : b;
                    if constexpr (VAR) {
                        const YQ qv = (YQ)sm.xq[(rbase + t) * SM::XPQ + ycol];
                        cq[t] = t ? cq[t - 1] + qv : qv;
                    }
                }
#pragma unroll
                for (int m = 0; m < YS; ++m) {
                    const int gy = rbase + m;
                    if (m + (S::NYS - 1) * YS < S::GY || gy < S::GY) {
                        const uint32_t b = cb[m + 2 * R] - (m ? cb[m - 1] : 0u);
                        YQ qv = 0;
                        if constexpr (VAR) qv = cq[m + 2 * R] - (m ? cq[m - 1] : (YQ)0);
                        centre_key(kb, gy, ycol, b, qv);
                    }
                }
            }
        };
        // gather of plane q (ring slot u): C and the corner group of the plane;
        // the rings finish output q - D
        auto gather = [&](uint64_t* kb, int u, int q) {
            const int p = p0 + q;
            const int ur = (u + U - D % U) % U;  // slot written D planes ago
            const rsrc_t wr = make_rsrc(out + (size_t)max(p - D, 0) * plane,
                                        (q >= 2 * D && q < npl) ? pbytes : 0u);
#pragma unroll
            for (int j = 0; j < OPT; ++j) {
                const int oy = oyb + j * S::OROWS;
                const int ic = (oy + D) * VP + ox + D;
                uint32_t o;
                if constexpr (PACK) {
                    // c.v < b.v  <=>  c.key < (b.key & kHigh): the same
                    // first minima as the unpacked branch below
                    const uint64_t ck = kb[ic];
                    uint64_t gk = kb[oy * VP + ox];
#pragma unroll
                    for (int k = 1; k < 4; ++k) {
                        const int ik = (oy + ((k & 2) ? 2 * D : 0)) * VP + ox + ((k & 1) ? 2 * D : 0);
                        const uint64_t kk = kb[ik];
                        gk = kk < (gk & kHigh) ? kk : gk;
                    }
                    o = (uint32_t)(gk < (mk[ur][j] & kHigh) ? gk : mk[ur][j]) & 0xffffu;
                    mk[u][j] = ak[ur][j] < (ck & kHigh) ? ak[ur][j] : ck;
                    ak[u][j] = gk;
                } else if constexpr (VAR) {
                    const double cv = sm.vv[ic];
                    const uint32_t co = sm.vo[ic];
                    double gv = sm.vv[oy * VP + ox];
                    uint32_t go = sm.vo[oy * VP + ox];
#pragma unroll
                    for (int k = 1; k < 4; ++k) {
                        const int ik = (oy + ((k & 2) ? 2 * D : 0)) * VP + ox + ((k & 1) ? 2 * D : 0);
                        const double v = sm.vv[ik];
                        if (v < gv) {
                            gv = v;
                            go = sm.vo[ik];
                        }
                    }
                    // output p - D: firstmin(C, G(p - 2D)) kept D planes, then G(p)
                    o = gv < mv[ur][j] ? go : mo[ur][j];
                    // output p: firstmin(C(p), G(p - D))
                    const bool ta = av[ur][j] < cv;
                    mv[u][j] = ta ? av[ur][j] : cv;
                    mo[u][j] = ta ? ao[ur][j] : co;
                    av[u][j] = gv;
                    ao[u][j] = go;
                } else {
                    const uint32_t c = sm.vo[ic];
                    const uint32_t k = sm.vo[oy * VP + ox] + sm.vo[oy * VP + ox + 2 * D] +
                                       sm.vo[(oy + 2 * D) * VP + ox] +
                                       sm.vo[(oy + 2 * D) * VP + ox + 2 * D];
                    // output p - D: C + K(p - 2D) kept D planes, plus K(p)
                    o = round_div_odd(mo[ur][j] + k, inv);
                    // output p: C(p) + K(p - D)
                    mo[u][j] = c + ao[ur][j];
                    ao[u][j] = k;
                }
                if (GATE && o < gate) o = 0;
                buffer_store<T>(o, wr, soff[j], 0u);
            }
        };
        for (int qb = 0; qb < npl; qb += U) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int q = qb + u;
                const int p = p0 + q;
                if (q > 0) ypass_cubes(kbuf(q - 1));
                // 1. z-sums of plane p (en = slice p+r, eo = slice p-r-1 or zeros)
#pragma unroll
                for (int i = 0; i < S::NZ; ++i) {
                    const int d = (int)en[i] - (int)eo[i];
                    zb[i] += (uint32_t)d;
                    if constexpr (VAR) {
                        const uint32_t s = en[i] + eo[i];
                        if constexpr (WIDE) zq[i] = __builtin_fma((double)d, (double)s, zq[i]);
                        else if constexpr (NQ) zq[i] += (uint32_t)d * s;  // modulo 2^32
                        else zq[i] += (uint32_t)(d * (int)s);
                    }
                    if constexpr (NQ) orv |= en[i];
                }
#pragma unroll
                for (int i = 0; i < S::NZ; ++i) {
                    if (i < S::NZ - 1 || zlast) {
                        sm.zb[zi[i]] = zb[i];
                        if constexpr (VAR) {
                            if constexpr (WIDE) {
                                const uint64_t w = __builtin_bit_cast(uint64_t, zq[i]);
                                sm.zq0[zi[i]] = (uint32_t)w;
                                sm.zq1[zi[i]] = (uint32_t)(w >> 32);
                            } else {
                                sm.zq0[zi[i]] = zq[i];
                            }
                        }
                        if constexpr (CROSS) sm.ec[zi[i]] = ec[i];
                    }
                }
                load(en, p + 1 + R);
                load(eo, p - R);
                if constexpr (CROSS) load(ec, p + 1);
                // NQ: at each block after the first, the values summed so far are
                // checked (later planes of the block are checked at the next one,
                // or after the loop)
                if constexpr (NQ)
                    if (u == 0 && qb > 0 && orv >= kNQLimit) *flag = 1;
                barrier_lds();
                if constexpr (NQ)
                    if (u == 0 && qb > 0 && *flag) return false;
                if (q > 0) gather(kbuf(q - 1), (u + U - 1) % U, q - 1);

                // 2. cubes: x-pass of the z-sums.  Crosses: x-lines and y-lines
                //    of slice p through every centre.
                if constexpr (!CROSS) {
                    xpass(sm.zb, sm.zq0, sm.zq1);
                } else {
                    xpass(sm.ec, nullptr, nullptr);
                    if (yact) {
                        // y-line of centre (ycol, c) covers raw rows c .. c+2r of
                        // raw column ycol + r
                        const int rbase = yseg * YS;
                        uint32_t cb[S::YW];
                        QT cq[S::YW];
#pragma unroll
                        for (int t = 0; t < S::YW; ++t) {
                            const uint32_t e = sm.ec[(rbase + t) * S::ZP + ycol + R];
                            cb[t] = t ? cb[t - 1] + e : e;
                            if constexpr (VAR) cq[t] = t ? cq[t - 1] + sq(e) : sq(e);
                        }
#pragma unroll
                        for (int m = 0; m < YS; ++m) {
                            const int gy = rbase + m;
                            if (m + (S::NYS - 1) * YS < S::GY || gy < S::GY) {
                                sm.yb[gy * S::XPB + ycol] = cb[m + 2 * R] - (m ? cb[m - 1] : 0u);
                                if constexpr (VAR)
                                    sm.yq[gy * SM::XPQ + ycol] = cq[m + 2 * R] - (m ? cq[m - 1] : (QT)0);
                            }
                        }
                    }
                }
                barrier_lds();
            }
        }
        // the y-pass and the gather of the last plane
        const int ql = (npl + U - 1) / U * U - 1;
        ypass_cubes(kbuf(ql));
        barrier_lds();
        gather(kbuf(ql), U - 1, ql);
    } else {
        for (int qb = 0; qb < npl; qb += U) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int q = qb + u;
                const int p = p0 + q;
                // 1. z-sums of plane p (en = slice p+r, eo = slice p-r-1 or zeros)
#pragma unroll
                for (int i = 0; i < S::NZ; ++i) {
                    const int d = (int)en[i] - (int)eo[i];
                    zb[i] += (uint32_t)d;
                    if constexpr (VAR) {
                        const uint32_t s = en[i] + eo[i];
                        if constexpr (WIDE) zq[i] = __builtin_fma((double)d, (double)s, zq[i]);
                        else if constexpr (NQ) zq[i] += (uint32_t)d * s;  // modulo 2^32
                        else zq[i] += (uint32_t)(d * (int)s);
                    }
                    if constexpr (NQ) orv |= en[i];
                }
#pragma unroll
                for (int i = 0; i < S::NZ; ++i) {
                    if (i < S::NZ - 1 || zlast) {
                        sm.zb[zi[i]] = zb[i];
                        if constexpr (VAR) {
                            if constexpr (WIDE) {
                                const uint64_t w = __builtin_bit_cast(uint64_t, zq[i]);
                                sm.zq0[zi[i]] = (uint32_t)w;
                                sm.zq1[zi[i]] = (uint32_t)(w >> 32);
                            } else {
                                sm.zq0[zi[i]] = zq[i];
                            }
                        }
                        if constexpr (CROSS) sm.ec[zi[i]] = ec[i];
                    }
                }
                load(en, p + 1 + R);
                load(eo, p - R);
                if constexpr (CROSS) load(ec, p + 1);
                // NQ: at each block after the first, the values summed so far are
                // checked (later planes of the block are checked at the next one,
                // or after the loop)
                if constexpr (NQ)
                    if (u == 0 && qb > 0 && orv >= kNQLimit) *flag = 1;
                barrier_lds();
                if constexpr (NQ)
                    if (u == 0 && qb > 0 && *flag) return false;

                // 2. cubes: x-pass of the z-sums.  Crosses: x-lines and y-lines
                //    of slice p through every centre.
                if constexpr (!CROSS) {
                    xpass(sm.zb, sm.zq0, sm.zq1);
                } else {
                    xpass(sm.ec, nullptr, nullptr);
                    if (yact) {
                        // y-line of centre (ycol, c) covers raw rows c .. c+2r of
                        // raw column ycol + r
                        const int rbase = yseg * YS;
                        uint32_t cb[S::YW];
                        QT cq[S::YW];
#pragma unroll
                        for (int t = 0; t < S::YW; ++t) {
                            const uint32_t e = sm.ec[(rbase + t) * S::ZP + ycol + R];
                            cb[t] = t ? cb[t - 1] + e : e;
                            if constexpr (VAR) cq[t] = t ? cq[t - 1] + sq(e) : sq(e);
                        }
#pragma unroll
                        for (int m = 0; m < YS; ++m) {
                            const int gy = rbase + m;
                            if (m + (S::NYS - 1) * YS < S::GY || gy < S::GY) {
                                sm.yb[gy * S::XPB + ycol] = cb[m + 2 * R] - (m ? cb[m - 1] : 0u);
                                if constexpr (VAR)
                                    sm.yq[gy * SM::XPQ + ycol] = cq[m + 2 * R] - (m ? cq[m - 1] : (QT)0);
                            }
                        }
                    }
                }
                barrier_lds();

                // 3. cluster sums at every centre of the region
                if constexpr (!CROSS) {
                    // y-pass: centre row c covers x-pass rows c .. c+2r
                    if (yact) {
                        const int rbase = yseg * YS;
                        uint32_t cb[S::YW];
                        YQ cq[S::YW];
#pragma unroll
                        for (int t = 0; t < S::YW; ++t) {
                            const uint32_t b = sm.xb[(rbase + t) * S::XPB + ycol];
                            cb[t] = t ? cb[t - 1] + b : b;
                            if constexpr (VAR) {
                                const YQ qv = (YQ)sm.xq[(rbase + t) * SM::XPQ + ycol];
                                cq[t] = t ? cq[t - 1] + qv : qv;
                            }
                        }
#pragma unroll
                        for (int m = 0; m < YS; ++m) {
                            const int gy = rbase + m;
                            if (m + (S::NYS - 1) * YS < S::GY || gy < S::GY) {
                                const uint32_t b = cb[m + 2 * R] - (m ? cb[m - 1] : 0u);
                                YQ qv = 0;
                                if constexpr (VAR) qv = cq[m + 2 * R] - (m ? cq[m - 1] : (YQ)0);
                                centre_out(gy, ycol, b, qv);
                            }
                        }
                    }
                } else {
                    // z-line (the z-sum at the centre) + x-line + y-line
                    for (int c = tid; c < S::GX * S::GY; c += kT) {
                        const int gy = c / GX, gx = c - gy * GX;
                        const int iz = (gy + R) * S::ZP + gx + R;
                        const int il = gy * S::XPB + gx;
                        const uint32_t b = sm.zb[iz] + sm.xb[il] + sm.yb[il];
                        QT qv = 0;
                        if constexpr (VAR) {
                            QT zqv;
                            if constexpr (WIDE)
                                zqv = __builtin_bit_cast(double, ((uint64_t)sm.zq1[iz] << 32) | sm.zq0[iz]);
                            else
                                zqv = sm.zq0[iz];
                            const int iq = gy * SM::XPQ + gx;
                            qv = zqv + sm.xq[iq] + sm.yq[iq];
                        }
                        centre_out(gy, gx, b, qv);
                    }
                }
                barrier_lds();

                // 4. gather: C and the corner group of plane p; the rings finish
                //    output p - D
                const int ur = (u + U - D % U) % U;  // slot written D planes ago
                const rsrc_t wr = make_rsrc(out + (size_t)max(p - D, 0) * plane,
                                            (q >= 2 * D && q < npl) ? pbytes : 0u);
#pragma unroll
                for (int j = 0; j < OPT; ++j) {
                    const int oy = oyb + j * S::OROWS;
                    const int ic = (oy + D) * VP + ox + D;
                    uint32_t o;
                    if constexpr (PACK) {
                        // c.v < b.v  <=>  c.key < (b.key & kHigh): the same
                        // first minima as the unpacked branch below
                        const uint64_t ck = keys[ic];
                        uint64_t gk = keys[oy * VP + ox];
#pragma unroll
                        for (int k = 1; k < 4; ++k) {
                            const int ik = (oy + ((k & 2) ? 2 * D : 0)) * VP + ox + ((k & 1) ? 2 * D : 0);
                            const uint64_t kk = keys[ik];
                            gk = kk < (gk & kHigh) ? kk : gk;
                        }
                        o = (uint32_t)(gk < (mk[ur][j] & kHigh) ? gk : mk[ur][j]) & 0xffffu;
                        mk[u][j] = ak[ur][j] < (ck & kHigh) ? ak[ur][j] : ck;
                        ak[u][j] = gk;
                    } else if constexpr (VAR) {
                        const double cv = sm.vv[ic];
                        const uint32_t co = sm.vo[ic];
                        double gv = sm.vv[oy * VP + ox];
                        uint32_t go = sm.vo[oy * VP + ox];
#pragma unroll
                        for (int k = 1; k < 4; ++k) {
                            const int ik = (oy + ((k & 2) ? 2 * D : 0)) * VP + ox + ((k & 1) ? 2 * D : 0);
                            const double v = sm.vv[ik];
                            if (v < gv) {
                                gv = v;
                                go = sm.vo[ik];
                            }
                        }
                        // output p - D: firstmin(C, G(p - 2D)) kept D planes, then G(p)
                        o = gv < mv[ur][j] ? go : mo[ur][j];
                        // output p: firstmin(C(p), G(p - D))
                        const bool ta = av[ur][j] < cv;
                        mv[u][j] = ta ? av[ur][j] : cv;
                        mo[u][j] = ta ? ao[ur][j] : co;
                        av[u][j] = gv;
                        ao[u][j] = go;
                    } else {
                        const uint32_t c = sm.vo[ic];
                        const uint32_t k = sm.vo[oy * VP + ox] + sm.vo[oy * VP + ox + 2 * D] +
                                           sm.vo[(oy + 2 * D) * VP + ox] +
                                           sm.vo[(oy + 2 * D) * VP + ox + 2 * D];
                        // output p - D: C + K(p - 2D) kept D planes, plus K(p)
                        o = round_div_odd(mo[ur][j] + k, inv);
                        // output p: C(p) + K(p - D)
                        mo[u][j] = c + ao[ur][j];
                        ao[u][j] = k;
                    }
                    if (GATE && o < gate) o = 0;
                    buffer_store<T>(o, wr, soff[j], 0u);
                }
            }
        }
    }

    if constexpr (NQ) {
        // the last block's values; the second barrier keeps the next tile's
        // reset of the flag after every thread has read it
        if (orv >= kNQLimit) *flag = 1;
        barrier_lds();
        const bool ok = *flag == 0;
        barrier_lds();
        return ok;
    }
    return true;
}

// The paper's cluster geometry (cubes, diagonal offset r) under MINVAR9, as
// the single-volume and the batch kernels run it.  WT: the wide-tile variant
// (64 x 16 outputs, 512 threads, up to r = 3).
template <int R, bool WT = false>
using MV9Shape = PTShape<R, R, kClusterBox, kRuleMinVar9, WT>;
template <int R, typename T, bool WT = false>
using MV9Smem = PTSmem<R, R, kClusterBox, kRuleMinVar9, T, WT>;

// Narrow sums of squares first: uint16 data up to r = 3 (at r = 4 the two
// bodies in one kernel spill).
template <int R, typename T>
constexpr bool mv9_narrow()
{
    return sizeof(T) == 2 && R <= 3;
}

// LDS of a MINVAR9 tile: the narrow and the fp64 layouts share the space.
template <int R, typename T, bool WT = false>
struct MV9Lds {
    union {
        MV9Smem<R, T, WT> wide;
        PTSmem<R, R, kClusterBox, kRuleMinVar9, T, WT, mv9_narrow<R, T>()> narrow;
    };
    int flag;
};

// One MINVAR9 tile: uint16 data first with narrow sums of squares, and again
// with fp64 sums if a value of the tile is too large for them.
template <int R, typename T, bool GATE, bool WT>
__device__ __forceinline__ void minvar9_tile(MV9Lds<R, T, WT>& lds, const T* __restrict__ in,
                                             T* __restrict__ out, Geom g, int x0, int y0, int z0,
                                             int z1, uint32_t gate, double dn, double inv, int tid)
{
    if constexpr (mv9_narrow<R, T>()) {
        if (plane_tile<R, R, kClusterBox, kRuleMinVar9, T, GATE, WT, true>(
                lds.narrow, in, out, g, x0, y0, z0, z1, gate, dn, inv, tid, &lds.flag))
            return;
    }
    plane_tile<R, R, kClusterBox, kRuleMinVar9, T, GATE, WT>(lds.wide, in, out, g, x0, y0, z0, z1,
                                                             gate, dn, inv, tid);
}

}  // namespace lnf
