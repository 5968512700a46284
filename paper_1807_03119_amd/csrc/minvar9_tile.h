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

#include <type_traits>

#include "device_common.h"
#include "lnf_internal.h"

namespace lnf {

// Row pitches: 32-bit arrays take 4 mod 8 words and 64-bit arrays 2 mod 4
// elements, so eight consecutive rows start in eight different groups of four
// LDS banks (16-byte reads of eight lanes per bank cycle are conflict free).
constexpr int mv9_pitch32(int n) { return n + ((12 - n % 8) % 8); }
constexpr int mv9_pitch64(int n) { return n + ((6 - n % 4) % 4); }
template <typename Q>
constexpr int mv9_pitch(int n)
{
    return sizeof(Q) == 4 ? mv9_pitch32(n) : mv9_pitch64(n);
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
    static constexpr int XW2 = (XW + 1) / 2 * 2;    // ... of 64-bit values
    // y-pass: YS centre rows per column segment
    static constexpr int NYS0 = THREADS / GX;
    static constexpr int YS = (GY + NYS0 - 1) / NYS0;
    static constexpr int NYS = (GY + YS - 1) / YS;
    static constexpr int YW = YS + 2 * R;           // rows a segment reads
    static constexpr int XROWS = NYS * YS + 2 * R > LY ? NYS * YS + 2 * R : LY;
    static constexpr int OPT = TX * TY / THREADS;   // outputs per thread
    static constexpr int OROWS = THREADS / TX;      // output rows per pass
    static constexpr int U = R + 1;                 // register ring period
    static_assert(THREADS % TX == 0 && OPT * OROWS == TY, "gather mapping");
};

template <int R, typename T>
struct MV9Smem {
    using S = MV9Shape<R>;
    using QT = std::conditional_t<sizeof(T) == 1, uint32_t, double>;
    static constexpr int ZW = (S::NXS - 1) * S::XS + S::XW4;   // words a Zb row is read to
    static constexpr int ZQW = (S::NXS - 1) * S::XS + (sizeof(QT) == 4 ? S::XW4 : S::XW2);
    static constexpr int ZPB = mv9_pitch32(ZW > S::LX ? ZW : S::LX);
    static constexpr int ZPQ = mv9_pitch<QT>(ZQW > S::LX ? ZQW : S::LX);
    static constexpr int XPB = mv9_pitch32(S::NXS * S::XS);
    static constexpr int XPQ = mv9_pitch<QT>(S::NXS * S::XS);
    QT zq[S::LY * ZPQ];
    QT xq[S::XROWS * XPQ];
    double vv[S::GY * S::GX];
    uint32_t zb[S::LY * ZPB];
    uint32_t xb[S::XROWS * XPB];
    uint32_t vo[S::GY * S::GX];
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
    constexpr int kT = S::THREADS, LX = S::LX, GX = S::GX, XS = S::XS, YS = S::YS;
    constexpr int U = S::U, OPT = S::OPT;
    const int tid = threadIdx.x;
    const size_t plane = (size_t)g.nx * g.ny;
    const uint32_t pbytes = (uint32_t)(plane * sizeof(T));

    // ---- raw columns owned for the z-sums
    uint32_t off[S::NZ];
    int zbi[S::NZ], zqi[S::NZ];  // LDS indexes of each owned column
#pragma unroll
    for (int i = 0; i < S::NZ; ++i) {
        const int e = min(tid + i * kT, S::NRAW - 1);
        const int row = e / LX, col = e - row * LX;
        off[i] = (uint32_t)(clampi(y0 - S::H + row, 0, g.ny - 1) * g.nx +
                            clampi(x0 - S::H + col, 0, g.nx - 1)) * (uint32_t)sizeof(T);
        zbi[i] = row * SM::ZPB + col;
        zqi[i] = row * SM::ZPQ + col;
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
                    sm.zb[zbi[i]] = zb[i];
                    sm.zq[zqi[i]] = zq[i];
                }
            }
            barrier_lds();

            // 2. x-pass: centre column c of the region covers raw columns c .. c+2r
            if (xact) {
                const int cbase = xseg * XS;
                uint32_t wb[S::XW4];
                QT wq[S::XW4];
                const uint32_t* rb = sm.zb + xrow * SM::ZPB + cbase;
                const QT* rq = sm.zq + xrow * SM::ZPQ + cbase;
#pragma unroll
                for (int i = 0; i < S::XW4; i += 4) {
                    const uint4 t = *reinterpret_cast<const uint4*>(rb + i);
                    wb[i] = t.x;
                    wb[i + 1] = t.y;
                    wb[i + 2] = t.z;
                    wb[i + 3] = t.w;
                }
                if constexpr (sizeof(QT) == 4) {
#pragma unroll
                    for (int i = 0; i < S::XW4; i += 4) {
                        const uint4 t = *reinterpret_cast<const uint4*>(rq + i);
                        wq[i] = t.x;
                        wq[i + 1] = t.y;
                        wq[i + 2] = t.z;
                        wq[i + 3] = t.w;
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < S::XW2; i += 2) {
                        const double2 t = *reinterpret_cast<const double2*>(rq + i);
                        wq[i] = t.x;
                        wq[i + 1] = t.y;
                    }
                }
                uint32_t cb[S::XW];
                QT cq[S::XW];
                cb[0] = wb[0];
                cq[0] = wq[0];
#pragma unroll
                for (int i = 1; i < S::XW; ++i) {
                    cb[i] = cb[i - 1] + wb[i];
                    cq[i] = cq[i - 1] + wq[i];
                }
                uint32_t ob[XS];
                QT oq[XS];
#pragma unroll
                for (int m = 0; m < XS; ++m) {
                    ob[m] = cb[m + 2 * R] - (m ? cb[m - 1] : 0u);
                    oq[m] = cq[m + 2 * R] - (m ? cq[m - 1] : (QT)0);
                }
                uint32_t* db = sm.xb + xrow * SM::XPB + cbase;
                QT* dq = sm.xq + xrow * SM::XPQ + cbase;
#pragma unroll
                for (int m = 0; m < XS; m += 4)
                    *reinterpret_cast<uint4*>(db + m) = make_uint4(ob[m], ob[m + 1], ob[m + 2], ob[m + 3]);
                if constexpr (sizeof(QT) == 4) {
#pragma unroll
                    for (int m = 0; m < XS; m += 4)
                        *reinterpret_cast<uint4*>(dq + m) =
                            make_uint4(oq[m], oq[m + 1], oq[m + 2], oq[m + 3]);
                } else {
#pragma unroll
                    for (int m = 0; m < XS; m += 2)
                        *reinterpret_cast<double2*>(dq + m) = make_double2(oq[m], oq[m + 1]);
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
                    const uint32_t b = sm.xb[(rbase + t) * SM::XPB + ycol];
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
                        sm.vv[gy * GX + ycol] = __builtin_fma(dn, (double)qv, -db * db);
                        sm.vo[gy * GX + ycol] = round_div_odd(b, invn);
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
                const int ic = (oy + R) * GX + ox + R;
                const double cv = sm.vv[ic];
                const uint32_t co = sm.vo[ic];
                double gv = sm.vv[oy * GX + ox];
                uint32_t go = sm.vo[oy * GX + ox];
#pragma unroll
                for (int k = 1; k < 4; ++k) {
                    const int ik = (oy + ((k & 2) ? 2 * R : 0)) * GX + ox + ((k & 1) ? 2 * R : 0);
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
