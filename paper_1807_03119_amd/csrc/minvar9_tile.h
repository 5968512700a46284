// MINVAR9 tile body: one workgroup filters a TX x TY column of output voxels
// over the z-range [z0, z1).  Shared by the single-volume kernel and the
// multi-volume batch kernel.
//
// The selection rule is not in the paper (its cluster geometry is: Section
// "Our Method" and the nine-cluster figure): the variance numerator
// v_k = n*q_k - s_k^2 (s_k = sum, q_k = sum of squares, n voxels) is minimised,
// the lowest cluster index winning ties, and the winner's rounded mean
// round(s_k / n) is written.
//
// Every cluster statistic is a box sum at the cluster's centre, and the nine
// centres of output (x, y, z) lie on three planes: cluster 0 at (x, y, z),
// clusters 1..4 at (x -+ r, y -+ r, z - r) and 5..8 at (x -+ r, y -+ r, z + r),
// x varying fastest.  So the filter runs one centre plane p at a time:
//   1. z-sums: each thread owns raw columns of the (TX+4r) x (TY+4r) tile and
//      keeps Zb = sum of E and Zq = sum of E^2 over slices p-r .. p+r, adding
//      slice p+r and removing slice p-r-1 (both loaded one plane ahead; the
//      removed slice was read 2r+1 planes earlier and comes from L2), and
//      writes them to LDS;
//   2. x-pass: sums over 2r+1 columns for the (TX+2r) centre columns on every
//      raw row, from prefix sums over 8-wide row segments;
//   3. y-pass: sums over 2r+1 rows for the (TY+2r) centre rows, giving the box
//      sums B, Q of every centre of the plane; each centre's v = n*Q - B^2
//      (fp64, exact: every value is an integer below 2^53) and rounded mean o
//      go to an LDS plane;
//   4. gather: each output reads its centre entry C and the four corner
//      entries (x -+ r, y -+ r) of the plane; the first minimum of the corners
//      in cluster order is G.  Output z's winner is the first minimum of
//      C(z), G(z - r), G(z + r), in that order: a register ring per output
//      keeps G(p) until plane p + r and firstmin(C(p), G(p - r)) until plane
//      p + r, where G(p + r) completes it.
// Sums of squares are fp64 for uint16 data (Zq < 2^36, Q < 2^42) and uint32
// for uint8 data (Q <= 729 * 255^2 < 2^26).
#pragma once

#include <cstddef>
#include <type_traits>

#include "device_common.h"
#include "lnf_internal.h"

namespace lnf {

// LDS layout.  Bank conflicts come from lane groups that span two rows of an
// array (the z-sum writes: 64 lanes over rows of TX+4r; the y-pass: lanes over
// rows of TX+2r, one column segment after the other), and from 16-byte
// accesses whose eight lanes per bank cycle fall in the same bank group.  The
// pitches below make the rows such a group spans continue each other in bank
// space, and give the eight rows of one 16-byte access distinct bank groups.
//
// Smallest pitch p >= lo with p = 2 mod 4 (when asked) and ys * p = g (mod m).
constexpr int mv9_find_pitch(int ys, int g, int lo, int m, bool two_mod4)
{
    for (int p = lo; p < lo + 64; ++p)
        if ((!two_mod4 || p % 4 == 2) && (ys * p - g) % m == 0) return p;
    return -1;
}
// The y-pass segment height: the smallest that fits the threads and admits
// all three pitches; 0 if none does.
constexpr int mv9_pick_ys(int gx, int gy, int xw, int threads)
{
    for (int ys = 1; ys <= gy; ++ys) {
        if ((gy + ys - 1) / ys * gx > threads) continue;
        if (mv9_find_pitch(ys, gx, xw, 32, true) > 0 && mv9_find_pitch(ys, gx, xw, 16, true) > 0 &&
            mv9_find_pitch(ys, gx, gx, 32, false) > 0)
            return ys;
    }
    return 0;
}

template <int R>
struct MV9Shape {
    static constexpr int THREADS = 256;
    static constexpr int TX = 32, TY = 16, H = 2 * R;
    static constexpr int LX = TX + 4 * R, LY = TY + 4 * R;  // raw tile
    static constexpr int GX = TX + 2 * R, GY = TY + 2 * R;  // centre region
    static constexpr int NRAW = LX * LY;
    static constexpr int NZ = (NRAW + THREADS - 1) / THREADS;  // raw columns per thread
    // x-pass: XS centre columns per row segment; lanes take consecutive rows
    // of a segment, rows padded to XR
    static constexpr int XS = 8;
    static constexpr int NXS = (GX + XS - 1) / XS;
    static constexpr int XR = (LY + 7) / 8 * 8;
    static_assert(XR * NXS <= THREADS, "x-pass: one thread per row segment");
    static constexpr int XW = XS + 2 * R;           // raw values a segment reads
    static constexpr int XW4 = (XW + 3) / 4 * 4;    // ... rounded to 16-byte reads
    // z-sum rows (32-bit words): the pitch is the row length when that is
    // 4 mod 8 (rows continue each other, and eight rows of a 16-byte x-pass
    // read start in distinct bank groups), else the next such length.  The
    // x-pass reads XW4 words from each segment start, past the row end into
    // the next row (those values only feed discarded centres).
    static constexpr int ZP = LX + (12 - LX % 8) % 8;
    static constexpr int ZN = ((LY - 1) * ZP + (NXS - 1) * XS + XW4 + 3) / 4 * 4;  // 16-byte multiple
    // y-pass: YS centre rows per column segment
    static constexpr int YS = mv9_pick_ys(GX, GY, NXS * XS, THREADS);
    static_assert(YS > 0, "no conflict-free y-pass layout");
    static constexpr int NYS = (GY + YS - 1) / YS;
    static constexpr int YW = YS + 2 * R;           // rows a segment reads
    static constexpr int XROWS = NYS * YS + 2 * R > LY ? NYS * YS + 2 * R : LY;
    // x-pass output rows (written 8 bytes per lane by 16 consecutive rows)
    // and centre planes: pitches whose rows YS apart continue each other
    static constexpr int XPB = mv9_find_pitch(YS, GX, NXS * XS, 32, true);
    static constexpr int XPD = mv9_find_pitch(YS, GX, NXS * XS, 16, true);  // 64-bit
    static constexpr int VP = mv9_find_pitch(YS, GX, GX, 32, false);
    static constexpr int OPT = TX * TY / THREADS;   // outputs per thread
    static constexpr int OROWS = THREADS / TX;      // output rows per pass
    static constexpr int U = R + 1;                 // register ring period
    // waves per SIMD the kernels are compiled for (r = 4 would spill at 3)
    static constexpr int WAVES = R <= 3 ? 3 : 2;
    static_assert(THREADS % TX == 0 && OPT * OROWS == TY, "gather mapping");
};

template <int R, typename T>
struct MV9Smem {
    using S = MV9Shape<R>;
    // sums of squares: fp64 for uint16 data, staged in LDS as two 32-bit
    // halves (so they share the 32-bit layout); uint32 for uint8 data
    using QT = std::conditional_t<sizeof(T) == 1, uint32_t, double>;
    static constexpr bool WIDE = sizeof(QT) == 8;
    static constexpr int XPQ = WIDE ? S::XPD : S::XPB;
    // every array a multiple of 16 bytes, so each starts 16-byte aligned
    static constexpr int a16(int n, int bytes) { return (n * bytes + 15) / 16 * 16 / bytes; }
    QT xq[a16(S::XROWS * XPQ, sizeof(QT))];
    double vv[a16(S::GY * S::VP, 8)];
    uint32_t zb[S::ZN];
    uint32_t zq0[S::ZN];               // uint8: Zq; uint16: low half of Zq
    uint32_t zq1[WIDE ? S::ZN : 4];    // uint16: high half of Zq
    uint32_t xb[a16(S::XROWS * S::XPB, 4)];
    uint32_t vo[a16(S::GY * S::VP, 4)];
};

// dn = n, invn = 1/n.
template <int R, typename T, bool GATE>
__device__ __forceinline__ void minvar9_tile(MV9Smem<R, T>& sm, const T* __restrict__ in,
                                             T* __restrict__ out, Geom g, int x0, int y0, int z0,
                                             int z1, uint32_t gate, double dn, double invn)
{
    using S = MV9Shape<R>;
    using SM = MV9Smem<R, T>;
    using QT = typename SM::QT;
    static_assert(offsetof(SM, vv) % 16 == 0 && offsetof(SM, zb) % 16 == 0 &&
                      offsetof(SM, zq0) % 16 == 0 && offsetof(SM, zq1) % 16 == 0 &&
                      offsetof(SM, xb) % 16 == 0 && offsetof(SM, vo) % 16 == 0,
                  "16-byte LDS accesses need 16-byte aligned arrays");
    constexpr int kT = S::THREADS, LX = S::LX, GX = S::GX, XS = S::XS, YS = S::YS;
    constexpr int U = S::U, OPT = S::OPT;
    const int tid = threadIdx.x;
    const size_t plane = (size_t)g.nx * g.ny;
    const uint32_t pbytes = (uint32_t)(plane * sizeof(T));

    // ---- raw columns owned for the z-sums
    uint32_t off[S::NZ];
    int zi[S::NZ];  // LDS index of each owned column
#pragma unroll
    for (int i = 0; i < S::NZ; ++i) {
        const int e = min(tid + i * kT, S::NRAW - 1);
        const int row = e / LX, col = e - row * LX;
        off[i] = (uint32_t)(clampi(y0 - S::H + row, 0, g.ny - 1) * g.nx +
                            clampi(x0 - S::H + col, 0, g.nx - 1)) * (uint32_t)sizeof(T);
        zi[i] = row * S::ZP + col;
    }
    // lanes past the tile in the last round own no column
    const bool zlast = tid + (S::NZ - 1) * kT < S::NRAW;
    auto slice_rsrc = [&](int zi) {
        return make_rsrc(in + (size_t)clampi(zi, 0, g.nz - 1) * plane, pbytes);
    };
    auto load = [&](uint32_t(&v)[S::NZ], int zi) {
        const rsrc_t rs = slice_rsrc(zi);
#pragma unroll
        for (int i = 0; i < S::NZ; ++i) v[i] = buffer_load<T>(rs, off[i]);
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
    const int p0 = z0 - R;
    uint32_t zb[S::NZ];
    QT zq[S::NZ];
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
            if constexpr (sizeof(QT) == 4) zq[i] += e[i] * e[i];
            else zq[i] = __builtin_fma((double)e[i], (double)e[i], zq[i]);
        }
    }
    uint32_t en[S::NZ], eo[S::NZ];
    load(en, p0 + R);
#pragma unroll
    for (int i = 0; i < S::NZ; ++i) eo[i] = 0;

    // ---- register rings of the pending selections (value, rounded mean)
    double av[U][OPT], mv[U][OPT];
    uint32_t ao[U][OPT], mo[U][OPT];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int j = 0; j < OPT; ++j) {
            av[u][j] = mv[u][j] = 0.0;
            ao[u][j] = mo[u][j] = 0;
        }

    // x-pass mapping: consecutive lanes take consecutive rows of one segment
    const int xrow = tid % S::XR, xseg = tid / S::XR;
    const bool xact = xrow < S::LY && xseg < S::NXS;
    // y-pass mapping: consecutive lanes take consecutive centre columns
    const int ycol = tid % GX, yseg = tid / GX;
    const bool yact = yseg < S::NYS;

    const int npl = (z1 - z0) + 2 * R;  // centre planes z0-r .. z1-1+r
    for (int qb = 0; qb < npl; qb += U) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int q = qb + u;
            if (q >= npl) break;
            const int p = p0 + q;
            // 1. z-sums of plane p (en = slice p+r, eo = slice p-r-1 or zeros)
#pragma unroll
            for (int i = 0; i < S::NZ; ++i) {
                const int d = (int)en[i] - (int)eo[i];
                const uint32_t s = en[i] + eo[i];
                zb[i] += (uint32_t)d;
                if constexpr (sizeof(QT) == 4) zq[i] += (uint32_t)(d * (int)s);
                else zq[i] = __builtin_fma((double)d, (double)s, zq[i]);
            }
            load(en, p + 1 + R);
            load(eo, p - R);
#pragma unroll
            for (int i = 0; i < S::NZ; ++i) {
                if (i < S::NZ - 1 || zlast) {
                    sm.zb[zi[i]] = zb[i];
                    if constexpr (SM::WIDE) {
                        const uint64_t w = __builtin_bit_cast(uint64_t, zq[i]);
                        sm.zq0[zi[i]] = (uint32_t)w;
                        sm.zq1[zi[i]] = (uint32_t)(w >> 32);
                    } else {
                        sm.zq0[zi[i]] = zq[i];
                    }
                }
            }
            barrier_lds();

            // 2. x-pass: centre column c of the region covers raw columns c .. c+2r
            if (xact) {
                const int cbase = xseg * XS;
                const int zr = xrow * S::ZP + cbase;
                uint32_t wb[S::XW4], w0[S::XW4], w1[S::XW4];
                auto read_row = [&](const uint32_t* src, uint32_t(&w)[S::XW4]) {
#pragma unroll
                    for (int i = 0; i < S::XW4; i += 4) {
                        const uint4 t = *reinterpret_cast<const uint4*>(src + zr + i);
                        w[i] = t.x;
                        w[i + 1] = t.y;
                        w[i + 2] = t.z;
                        w[i + 3] = t.w;
                    }
                };
                read_row(sm.zb, wb);
                read_row(sm.zq0, w0);
                if constexpr (SM::WIDE) read_row(sm.zq1, w1);
                auto wq = [&](int i) -> QT {
                    if constexpr (SM::WIDE)
                        return __builtin_bit_cast(double, ((uint64_t)w1[i] << 32) | w0[i]);
                    else
                        return w0[i];
                };
                uint32_t cb[S::XW];
                QT cq[S::XW];
                cb[0] = wb[0];
                cq[0] = wq(0);
#pragma unroll
                for (int i = 1; i < S::XW; ++i) {
                    cb[i] = cb[i - 1] + wb[i];
                    cq[i] = cq[i - 1] + wq(i);
                }
                uint32_t ob[XS];
                QT oq[XS];
#pragma unroll
                for (int m = 0; m < XS; ++m) {
                    ob[m] = cb[m + 2 * R] - (m ? cb[m - 1] : 0u);
                    oq[m] = cq[m + 2 * R] - (m ? cq[m - 1] : (QT)0);
                }
                uint32_t* db = sm.xb + xrow * S::XPB + cbase;
                QT* dq = sm.xq + xrow * SM::XPQ + cbase;
#pragma unroll
                for (int m = 0; m < XS; m += 2) {
                    *reinterpret_cast<uint2*>(db + m) = make_uint2(ob[m], ob[m + 1]);
                    if constexpr (SM::WIDE)
                        *reinterpret_cast<double2*>(dq + m) = make_double2(oq[m], oq[m + 1]);
                    else
                        *reinterpret_cast<uint2*>(dq + m) = make_uint2(oq[m], oq[m + 1]);
                }
            }
            barrier_lds();

            // 3. y-pass: centre row c covers x-pass rows c .. c+2r; then v and o
            if (yact) {
                const int rbase = yseg * YS;
                uint32_t cb[S::YW];
                QT cq[S::YW];
#pragma unroll
                for (int t = 0; t < S::YW; ++t) {
                    const uint32_t b = sm.xb[(rbase + t) * S::XPB + ycol];
                    const QT qv = sm.xq[(rbase + t) * SM::XPQ + ycol];
                    cb[t] = t ? cb[t - 1] + b : b;
                    cq[t] = t ? cq[t - 1] + qv : qv;
                }
#pragma unroll
                for (int m = 0; m < YS; ++m) {
                    const int gy = rbase + m;
                    if (m + (S::NYS - 1) * YS < S::GY || gy < S::GY) {
                        const uint32_t b = cb[m + 2 * R] - (m ? cb[m - 1] : 0u);
                        const QT qv = cq[m + 2 * R] - (m ? cq[m - 1] : (QT)0);
                        const double db = (double)b;
                        sm.vv[gy * S::VP + ycol] = __builtin_fma(dn, (double)qv, -db * db);
                        sm.vo[gy * S::VP + ycol] = round_div_odd(b, invn);
                    }
                }
            }
            barrier_lds();

            // 4. gather: C and G of plane p; the rings finish output p - r
            const int ur = (u + U - R % U) % U;  // slot written r planes ago
            const rsrc_t wr = make_rsrc(out + (size_t)max(p - R, 0) * plane,
                                        q >= 2 * R ? pbytes : 0u);
#pragma unroll
            for (int j = 0; j < OPT; ++j) {
                const int oy = oyb + j * S::OROWS;
                const int ic = (oy + R) * S::VP + ox + R;
                const double cv = sm.vv[ic];
                const uint32_t co = sm.vo[ic];
                double gv = sm.vv[oy * S::VP + ox];
                uint32_t go = sm.vo[oy * S::VP + ox];
#pragma unroll
                for (int k = 1; k < 4; ++k) {
                    const int ik = (oy + ((k & 2) ? 2 * R : 0)) * S::VP + ox + ((k & 1) ? 2 * R : 0);
                    const double v = sm.vv[ik];
                    if (v < gv) {
                        gv = v;
                        go = sm.vo[ik];
                    }
                }
                // output p - r: firstmin(C, G(p - 2r)) stored r planes ago, then G(p)
                uint32_t o = gv < mv[ur][j] ? go : mo[ur][j];
                if (GATE && o < gate) o = 0;
                buffer_store<T>(o, wr, soff[j], 0u);
                // output p: firstmin(C(p), G(p - r))
                const bool ta = av[ur][j] < cv;
                mv[u][j] = ta ? av[ur][j] : cv;
                mo[u][j] = ta ? ao[ur][j] : co;
                av[u][j] = gv;
                ao[u][j] = go;
            }
        }
    }
}

}  // namespace lnf
