/*
 * CPU oracle of the nine-cluster local noise filter.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * statement of what the filter computes; it exists so that the HIP path can be
 * checked against it.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or helper
 * with the GPU library.
 *
 * What is computed (paper, Section "Our Method", equations 2 and 3, and the
 * figure of the nine average clusters):
 *   - an "average cluster" is the mean of a cubic region of side M = 2r+1 around
 *     a centre voxel; offsets run over i - (M-1)/2 for i = 0..M-1 (eq. 3);
 *   - S_0 is the cluster about the voxel itself; S_1..S_8 sit on the eight
 *     diagonal neighbours, sqrt(3) units away when M = 3 (r = 1).  For larger r
 *     the diagonal centres are placed at (+-r, +-r, +-r), so that each diagonal
 *     cluster is the octant box that still touches the centre voxel;
 *   - the voxel is replaced by the average of the nine cluster averages
 *     (rule MEAN9), rounded to the nearest integer;
 *   - values below a data threshold T (Otsu's, eq. 1) are noise: written as 0.
 * Rule MINVAR9 is not in the paper: it picks the cluster of least variance
 * (numerator n*sum(x^2) - (sum x)^2, lowest cluster index on ties) and writes
 * its rounded mean.
 *
 * Readings where the paper is silent: samples outside the volume take the value
 * of the nearest voxel (clamp each coordinate separately); rounding is
 * round-half-up, and no exact half can occur because both divisors (9n and n,
 * n = M^3) are odd; the output has the dtype of the input.
 *
 * Cluster index order: k = 0 is the centre; for k = 1..8, with j = k-1, bit 0
 * of j selects +d (else -d) along x, bit 1 along y, bit 2 along z.
 *
 * Geometry variants (the paper's own open questions, Section "Our Method" and
 * the conclusion's future work):
 *   - cluster shape: the cube of side M (the text's "3x3x3 region"), or the
 *     three-line cross that eq. 2 writes out: the M voxels along x, along y and
 *     along z through the cluster centre, the centre thus counted three times,
 *     n = 3M;
 *   - diagonal offset d of S_1..S_8: r (default; sqrt(3) units at r = 1), 1
 *     (sqrt(3) units at every r), or 2r+1 (the diagonal clusters just clear
 *     the centre cluster).
 * Both divisors stay odd (9n, n with n = M^3 or 3M), so no tie ever occurs.
 *
 * Volume layout: vol[z][y][x], x fastest; dtype 1 = uint8, 2 = uint16.
 */
#include <stdint.h>
#include <stddef.h>

#define LNFO_MEAN9 0
#define LNFO_MINVAR9 1
#define LNFO_BOX 0
#define LNFO_CROSS 1

typedef struct {
    int shape;  /* LNFO_BOX or LNFO_CROSS */
    int64_t d;  /* diagonal offset of S_1..S_8 */
} geom_t;

typedef struct {
    const void* vol;
    int64_t nx, ny, nz;
    int dtype;
} grid_t;

static int64_t clamp_index(int64_t v, int64_t n)
{
    if (v < 0) return 0;
    if (v > n - 1) return n - 1;
    return v;
}

/* Grey value of the voxel nearest to (x, y, z), which may lie outside the volume. */
static uint64_t sample(const grid_t* g, int64_t x, int64_t y, int64_t z)
{
    int64_t cx = clamp_index(x, g->nx);
    int64_t cy = clamp_index(y, g->ny);
    int64_t cz = clamp_index(z, g->nz);
    int64_t idx = (cz * g->ny + cy) * g->nx + cx;
    if (g->dtype == 1) return ((const uint8_t*)g->vol)[idx];
    return ((const uint16_t*)g->vol)[idx];
}

/* Centre offset of cluster k (see the index order above). */
static void cluster_offset(int k, int64_t d, int64_t off[3])
{
    if (k == 0) {
        off[0] = off[1] = off[2] = 0;
        return;
    }
    int j = k - 1;
    for (int axis = 0; axis < 3; ++axis)
        off[axis] = ((j >> axis) & 1) ? d : -d;
}

/* Number of voxels of one cluster, counted with multiplicity. */
static uint64_t cluster_size(int r, int shape)
{
    const uint64_t m = (uint64_t)(2 * r + 1);
    return shape == LNFO_CROSS ? 3 * m : m * m * m;
}

/* Sum and sum of squares of every cluster about (px, py, pz): the cube of side
 * 2r+1, or the three lines of 2r+1 voxels through the cluster centre. */
static void cluster_stats(const grid_t* g, int r, geom_t geo, int64_t px, int64_t py,
                          int64_t pz, uint64_t s[9], uint64_t q[9])
{
    for (int k = 0; k < 9; ++k) {
        int64_t d[3];
        cluster_offset(k, geo.d, d);
        const int64_t cx = px + d[0], cy = py + d[1], cz = pz + d[2];
        uint64_t sum = 0, sq = 0;
        if (geo.shape == LNFO_BOX) {
            for (int64_t az = -r; az <= r; ++az)
                for (int64_t ay = -r; ay <= r; ++ay)
                    for (int64_t ax = -r; ax <= r; ++ax) {
                        uint64_t v = sample(g, cx + ax, cy + ay, cz + az);
                        sum += v;
                        sq += v * v;
                    }
        } else {
            for (int64_t t = -r; t <= r; ++t) {
                uint64_t vx = sample(g, cx + t, cy, cz);
                uint64_t vy = sample(g, cx, cy + t, cz);
                uint64_t vz = sample(g, cx, cy, cz + t);
                sum += vx + vy + vz;
                sq += vx * vx + vy * vy + vz * vz;
            }
        }
        s[k] = sum;
        q[k] = sq;
    }
}

static uint32_t filter_voxel(const grid_t* g, int r, geom_t geo, int rule, uint32_t gate_T,
                             int64_t px, int64_t py, int64_t pz)
{
    uint64_t s[9], q[9];
    cluster_stats(g, r, geo, px, py, pz, s, q);
    const uint64_t n = cluster_size(r, geo.shape);
    uint64_t out;
    if (rule == LNFO_MEAN9) {
        /* mean of the nine cluster means = (sum of all nine sums) / (9n), rounded */
        uint64_t total = 0;
        for (int k = 0; k < 9; ++k) total += s[k];
        out = (2 * total + 9 * n) / (18 * n);
    } else {
        /* n^2 times the variance of each cluster; all quantities below 2^62 for r <= 8 */
        int best = 0;
        int64_t best_v = 0;
        for (int k = 0; k < 9; ++k) {
            int64_t v = (int64_t)(n * q[k]) - (int64_t)(s[k] * s[k]);
            if (k == 0 || v < best_v) {
                best = k;
                best_v = v;
            }
        }
        out = (2 * s[best] + n) / (2 * n);
    }
    if (out < gate_T) out = 0;
    return (uint32_t)out;
}

static int check_args(const void* vol, int64_t nx, int64_t ny, int64_t nz, int dtype, int r,
                      int rule)
{
    if (!vol || nx < 1 || ny < 1 || nz < 1) return -1;
    if (dtype != 1 && dtype != 2) return -1;
    if (r < 1 || r > 8) return -1;
    if (rule != LNFO_MEAN9 && rule != LNFO_MINVAR9) return -1;
    return 0;
}

/* shape: LNFO_BOX / LNFO_CROSS; offset_mode 0: d = r, 1: d = 1, 2: d = 2r+1. */
static int make_geom(int r, int shape, int offset_mode, geom_t* geo)
{
    if (shape != LNFO_BOX && shape != LNFO_CROSS) return -1;
    if (offset_mode < 0 || offset_mode > 2) return -1;
    geo->shape = shape;
    geo->d = offset_mode == 0 ? r : offset_mode == 1 ? 1 : 2 * r + 1;
    return 0;
}

/* Filter a whole volume with a cluster geometry; `out` has the dtype and
 * layout of `vol`. */
int lnfo_filter_geom(const void* vol, int64_t nx, int64_t ny, int64_t nz, int dtype, int r,
                     int rule, uint32_t gate_T, int shape, int offset_mode, void* out)
{
    geom_t geo;
    if (check_args(vol, nx, ny, nz, dtype, r, rule) || !out) return -1;
    if (make_geom(r, shape, offset_mode, &geo)) return -1;
    grid_t g = {vol, nx, ny, nz, dtype};
    int64_t plane = nx * ny;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t zy = 0; zy < nz * ny; ++zy) {
        int64_t z = zy / ny, y = zy % ny;
        for (int64_t x = 0; x < nx; ++x) {
            uint32_t v = filter_voxel(&g, r, geo, rule, gate_T, x, y, z);
            int64_t idx = z * plane + y * nx + x;
            if (dtype == 1) ((uint8_t*)out)[idx] = (uint8_t)v;
            else ((uint16_t*)out)[idx] = (uint16_t)v;
        }
    }
    return 0;
}

/* Filter a whole volume with the default geometry (cubes, d = r). */
int lnfo_filter(const void* vol, int64_t nx, int64_t ny, int64_t nz, int dtype, int r,
                int rule, uint32_t gate_T, void* out)
{
    return lnfo_filter_geom(vol, nx, ny, nz, dtype, r, rule, gate_T, LNFO_BOX, 0, out);
}

/* Filter the voxels listed in xyz[m][3] (x, y, z inside the volume) into out[m]. */
int lnfo_filter_points(const void* vol, int64_t nx, int64_t ny, int64_t nz, int dtype, int r,
                       int rule, uint32_t gate_T, const int64_t* xyz, int64_t m, uint32_t* out)
{
    if (check_args(vol, nx, ny, nz, dtype, r, rule) || (m > 0 && (!xyz || !out))) return -1;
    for (int64_t i = 0; i < m; ++i) {
        int64_t x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
        if (x < 0 || x >= nx || y < 0 || y >= ny || z < 0 || z >= nz) return -1;
    }
    grid_t g = {vol, nx, ny, nz, dtype};
    const geom_t geo = {LNFO_BOX, r};
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < m; ++i)
        out[i] = filter_voxel(&g, r, geo, rule, gate_T, xyz[3 * i], xyz[3 * i + 1],
                              xyz[3 * i + 2]);
    return 0;
}

/* The nine (sum, sum of squares) pairs at one voxel, for diagnostics and pins. */
int lnfo_cluster_stats_geom(const void* vol, int64_t nx, int64_t ny, int64_t nz, int dtype,
                            int r, int shape, int offset_mode, int64_t x, int64_t y, int64_t z,
                            uint64_t* s9, uint64_t* q9)
{
    geom_t geo;
    if (check_args(vol, nx, ny, nz, dtype, r, LNFO_MEAN9) || !s9 || !q9) return -1;
    if (make_geom(r, shape, offset_mode, &geo)) return -1;
    grid_t g = {vol, nx, ny, nz, dtype};
    cluster_stats(&g, r, geo, x, y, z, s9, q9);
    return 0;
}

int lnfo_cluster_stats(const void* vol, int64_t nx, int64_t ny, int64_t nz, int dtype, int r,
                       int64_t x, int64_t y, int64_t z, uint64_t* s9, uint64_t* q9)
{
    return lnfo_cluster_stats_geom(vol, nx, ny, nz, dtype, r, LNFO_BOX, 0, x, y, z, s9, q9);
}

/* Number of OpenMP threads a parallel region of this library uses. */
int lnfo_threads(void)
{
    int t = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            t = omp_get_num_threads();
#endif
        }
    }
    return t;
}

/* Use n OpenMP threads in the parallel regions that follow (n >= 1). */
void lnfo_set_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(n < 1 ? 1 : n);
#else
    (void)n;
#endif
}

/* ---- comparison filters (paper, Section "Other Filters") -------------------
 * TEST INFRASTRUCTURE ONLY, like everything in this file.  Readings where the
 * paper's formulas are garbled or silent (each filter starts from the same
 * clamped sampling as above; averages round half up, exactly):
 *   mean    (eq. 4)  mean of the (2r+1)^3 cube about the voxel;
 *   sigma   (eq. 5)  mean of the cube's values v with |v - P0| <= w, P0 the
 *                    centre value, w the half width of the accepted range (the
 *                    paper's 2 sigma; the caller passes it);
 *   Okada   (eq. 6)  mean of the centre and its six face neighbours whose
 *                    difference to the centre is below t_d (strictly); 0 when
 *                    none is (t_d = 0);
 *   entropy (eq. 7)  P0 when the sum over the cube of -p log2 p (p the global
 *                    frequency of each voxel's grey level, in fixed point:
 *                    weights[level] in units of 2^-32) exceeds te_fixed, else 0.
 * The gate (out < gate_T -> 0) applies to every output, as to the main filter. */
#define LNFO_CMP_MEAN 0
#define LNFO_CMP_SIGMA 1
#define LNFO_CMP_OKADA 2
#define LNFO_CMP_ENTROPY 3

static uint32_t compare_voxel(const grid_t* g, int kind, int r, int64_t param,
                              const int64_t* weights, uint32_t gate_T, int64_t px, int64_t py,
                              int64_t pz)
{
    const uint64_t p0 = sample(g, px, py, pz);
    uint64_t out = 0;
    if (kind == LNFO_CMP_OKADA) {
        static const int nb[7][3] = {{0, 0, 0}, {-1, 0, 0}, {1, 0, 0}, {0, -1, 0},
                                     {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
        uint64_t sum = 0, cnt = 0;
        for (int i = 0; i < 7; ++i) {
            uint64_t v = sample(g, px + nb[i][0], py + nb[i][1], pz + nb[i][2]);
            uint64_t diff = v > p0 ? v - p0 : p0 - v;
            if ((int64_t)diff < param) {
                sum += v;
                cnt += 1;
            }
        }
        out = cnt ? (2 * sum + cnt) / (2 * cnt) : 0;
    } else {
        uint64_t sum = 0, cnt = 0;
        int64_t h = 0;
        for (int64_t az = -r; az <= r; ++az)
            for (int64_t ay = -r; ay <= r; ++ay)
                for (int64_t ax = -r; ax <= r; ++ax) {
                    uint64_t v = sample(g, px + ax, py + ay, pz + az);
                    if (kind == LNFO_CMP_ENTROPY) {
                        h += weights[v];
                    } else {
                        uint64_t diff = v > p0 ? v - p0 : p0 - v;
                        if (kind == LNFO_CMP_MEAN || (int64_t)diff <= param) {
                            sum += v;
                            cnt += 1;
                        }
                    }
                }
        if (kind == LNFO_CMP_ENTROPY) out = h > param ? p0 : 0;
        else out = (2 * sum + cnt) / (2 * cnt);
    }
    if (out < gate_T) out = 0;
    return (uint32_t)out;
}

/* Whole-volume comparison filter; param: sigma half width, Okada t_d, or the
 * entropy threshold in 2^-32 units; weights: entropy only (levels entries). */
int lnfo_compare(const void* vol, int64_t nx, int64_t ny, int64_t nz, int dtype, int kind,
                 int r, int64_t param, const int64_t* weights, uint32_t gate_T, void* out)
{
    if (check_args(vol, nx, ny, nz, dtype, r, LNFO_MEAN9) || !out) return -1;
    if (kind < LNFO_CMP_MEAN || kind > LNFO_CMP_ENTROPY) return -1;
    if (kind == LNFO_CMP_ENTROPY && !weights) return -1;
    grid_t g = {vol, nx, ny, nz, dtype};
    int64_t plane = nx * ny;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t zy = 0; zy < nz * ny; ++zy) {
        int64_t z = zy / ny, y = zy % ny;
        for (int64_t x = 0; x < nx; ++x) {
            uint32_t v = compare_voxel(&g, kind, r, param, weights, gate_T, x, y, z);
            int64_t idx = z * plane + y * nx + x;
            if (dtype == 1) ((uint8_t*)out)[idx] = (uint8_t)v;
            else ((uint16_t*)out)[idx] = (uint16_t)v;
        }
    }
    return 0;
}
