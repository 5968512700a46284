/*
 * lnf.h -- C ABI of the MI355X (gfx950) local noise filter for 3D CT volumes.
 *
 * The filter (Tan Jerome et al., "Real-time Local Noise Filter in 3D
 * Visualization of CT Data", Section "Our Method", eqs. 2-3 and the figure of
 * the nine "average clusters"): every voxel is replaced by a combination of
 * nine cubic sub-regions ("average clusters") of side M = 2r+1 -- S_0 centred
 * on the voxel and S_1..S_8 centred on its diagonal neighbours at (+-r,+-r,+-r),
 * which is sqrt(3) units away for the paper's M = 3.  Values below the data
 * threshold T (Otsu's, eq. 1) are treated as noise and written as 0.
 *
 * Exact integer semantics (identical on every call, tile shape and batch mix):
 *   n      = (2r+1)^3
 *   s_k    = sum of the n voxels of cluster k, q_k = sum of their squares
 *   sample = voxel at the coordinate clamped into the volume, per axis
 *   LNF_MEAN9   (the paper's rule): out = round(sum_k s_k / (9n))
 *   LNF_MINVAR9 (not in the paper; least-variance selection): k* = the lowest k
 *               minimising n*q_k - s_k^2, out = round(s_k* / n)
 *   gate        out = (out >= T) ? out : 0   (T = 0 disables it)
 * Rounding is to nearest; no exact half can occur because 9n and n are odd.
 * Cluster order: k = 0 is the centre; for k = 1..8 with j = k-1, bit 0 of j
 * selects +r (else -r) along x, bit 1 along y, bit 2 along z.
 *
 * Volumes are dense, x fastest: element (x,y,z) at byte offset
 * ((z*ny + y)*nx + x) * sizeof(element).  dims[] = {nx, ny, nz}.
 *
 * All functions return LNF_OK (0) or a negative LNF_E* code and never throw or
 * abort across the ABI.  Device pointers are checked against the device
 * allocation that contains them (a region past its end is rejected); a buffer
 * carved out of a larger allocation by a caching allocator cannot be checked
 * more finely, so the caller guarantees that each buffer holds what its dims say.  Work is enqueued asynchronously on the given stream;
 * device-side faults surface at the caller's next synchronisation.
 */
#ifndef LNF_H
#define LNF_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define LNF_API __attribute__((visibility("default")))
#else
#define LNF_API
#endif

/* ---- status codes ---------------------------------------------------- */
#define LNF_OK 0
#define LNF_EINVAL (-1)     /* bad argument: null pointer, dtype, radius, dims, overlap */
#define LNF_EDEVICE (-2)    /* a pointer is not device memory of the handle's device */
#define LNF_ENOMEM (-3)     /* library-internal allocation failed */
#define LNF_EHIP (-4)       /* a HIP runtime call or kernel launch failed */
#define LNF_EBUSY (-5)      /* server: admission would exceed the memory cap */
#define LNF_ENOTFOUND (-6)  /* server: unknown volume id or ticket */
#define LNF_ECANCELED (-7)  /* server: request was cancelled or its batch failed */
#define LNF_ETIMEDOUT (-8)  /* server: wait timed out (request still pending) */
#define LNF_ERANGE (-9)     /* more jobs than lnf_filter_batch_noalloc's static table holds */

/* ---- enumerations ---------------------------------------------------- */
#define LNF_U8 1            /* uint8 voxels */
#define LNF_U16 2           /* uint16 voxels */

#define LNF_MEAN9 0         /* mean of the nine cluster means (the paper's rule) */
#define LNF_MINVAR9 1       /* mean of the least-variance cluster (not in the paper) */

#define LNF_RADIUS_MAX 4    /* largest supported r (cluster side M = 2r+1 <= 9) */

/* ---- context ----------------------------------------------------------- */
typedef struct lnf_ctx* lnf_handle;

typedef struct {
    uint32_t size;    /* sizeof(lnf_options), for forward compatibility */
    int32_t rule;     /* LNF_MEAN9 (default) or LNF_MINVAR9 */
    uint32_t gate_T;  /* data threshold T of the noise gate; 0 disables the gate */
    int32_t device;   /* HIP device ordinal; -1 = the device current at create time */
    uint32_t flags;   /* cluster geometry: 0 or LNF_GEOM_* bits below */
} lnf_options;

/*
 * Cluster geometry (Section "Our Method": eq. 2 writes each cluster as three
 * lines, the text as a cube; the diagonal distance is given only for M = 3).
 * Default (flags = 0): cubes of side 2r+1, diagonal centres at (+-r,+-r,+-r).
 *   LNF_GEOM_CROSS       clusters are the three axis lines of 2r+1 voxels
 *                        through the centre (eq. 2; n = 3(2r+1), the centre
 *                        counted on each line);
 *   LNF_GEOM_OFFSET_1    diagonal centres at (+-1,+-1,+-1) for every r;
 *   LNF_GEOM_OFFSET_2R1  diagonal centres at (+-(2r+1), ...): the outer
 *                        clusters just clear the centre one.
 * The two offset bits exclude each other.  Non-default geometries run on a
 * general cluster-gather kernel (lnf_filter, lnf_filter_tiled's z-strip depth,
 * lnf_filter_batch as one launch per job, lnf_filter_otsu, the server);
 * lnf_filter_points supports the default geometry only.
 */
#define LNF_GEOM_CROSS 1u
#define LNF_GEOM_OFFSET_1 2u
#define LNF_GEOM_OFFSET_2R1 4u

/*
 * Create a filter context.  opt == NULL gives the defaults (LNF_MEAN9, gate off,
 * current device).  Allocates only library-internal state: eight job-table
 * slots of lnf_filter_batch (about 200 KB of device memory and 200 KB of pinned
 * host memory each), and later the histogram and entropy scratch.
 * Errors: LNF_EINVAL (h NULL, bad rule, unknown or conflicting flags, size), LNF_EDEVICE (bad device),
 * LNF_ENOMEM, LNF_EHIP.
 */
LNF_API int lnf_create(lnf_handle* h, const lnf_options* opt);

/* Release a context's internal state; never touches caller buffers.  NULL is a no-op. */
LNF_API int lnf_destroy(lnf_handle h);

/*
 * Filter one volume: out = filter(vol) with the context's rule and gate.
 *   vol, out  device pointers on the context's device, same dtype and dims,
 *             non-overlapping (the filter is a stencil); owned by the caller,
 *             not retained after the call's work completes on `stream`.
 *   dims      {nx, ny, nz}, each >= 1, nx*ny < 2^31.
 *   dtype     LNF_U8 or LNF_U16.
 *   radius    r in [1, LNF_RADIUS_MAX]; cluster side M = 2r+1.
 *   stream    HIP stream the work is enqueued on (0 = null stream).
 * Errors: LNF_EINVAL, LNF_EDEVICE, LNF_EHIP.
 */
LNF_API int lnf_filter(lnf_handle h, const void* vol, const int64_t dims[3], int dtype,
                       int radius, void* out, hipStream_t stream);

/*
 * Tile configuration of the single-volume kernels.  Every configuration gives
 * byte-identical output; they differ only in speed.
 *   variant  index of a compiled tile shape (0 .. lnf_tile_variants()-1);
 *            -1 = the context's tuned/default choice.
 *   zs       z-strip depth (output slices per workgroup); 0 = default.
 */
typedef struct {
    int32_t variant;
    int32_t zs;
} lnf_tile;

/* Number of compiled tile shapes for (rule, dtype, radius); < 0 on bad arguments. */
LNF_API int lnf_tile_variants(int rule, int dtype, int radius);

/*
 * The tile configuration lnf_filter would use for a volume of these dims with
 * this context (its rule, geometry and tuned choices): the tile variant and
 * the z-strip depth, so that a caller can see where the z-strips of the launch
 * start (every multiple of tile->zs).  No device work; no device memory is
 * touched.  Geometry-variant contexts have one tile shape (variant 0).
 *   tile  written on success.
 * Errors: LNF_EINVAL (NULL arguments, dtype, radius, dims as lnf_filter),
 * LNF_EHIP.
 */
LNF_API int lnf_tile_config(lnf_handle h, const int64_t dims[3], int dtype, int radius,
                            lnf_tile* tile);

/* lnf_filter with an explicit tile configuration (tile == NULL: as lnf_filter). */
LNF_API int lnf_filter_tiled(lnf_handle h, const void* vol, const int64_t dims[3], int dtype,
                             int radius, void* out, hipStream_t stream, const lnf_tile* tile);

/* ---- batch ------------------------------------------------------------- */
/* One volume of a batch.  Same contract as the arguments of lnf_filter. */
typedef struct {
    const void* in;      /* device input volume */
    void* out;           /* device output volume: same dtype and dims, no overlap with any in */
    int64_t dims[3];     /* {nx, ny, nz} */
    int32_t dtype;       /* LNF_U8 or LNF_U16 */
    int32_t radius;      /* 1 .. LNF_RADIUS_MAX */
} lnf_job;

#define LNF_BATCH_MAX 4096 /* most jobs one lnf_filter_batch call accepts */

/*
 * Filter n volumes with the context's rule, geometry and gate in one call: the
 * jobs are grouped by (radius, dtype), and each group runs as ONE kernel launch
 * over the tiles of all its volumes (larger volumes first), after one copy of
 * the job table; everything is enqueued on `stream`.  Each output is byte-identical to
 * lnf_filter on the same job.  The job table is copied by the call, so `jobs`
 * may be reused as soon as it returns; the buffers must stay valid until the
 * work completes on `stream`.  n == 0 is a no-op.
 * A call may be captured in a HIP graph (stream capture): it then takes one of
 * four job-table slots kept for captures for the context's lifetime, since each
 * replay copies that table again; a fifth capture on one context returns
 * LNF_EBUSY.  Calls that are not captured take the other slots in turn.
 * Errors: LNF_EINVAL (n < 0 or > LNF_BATCH_MAX, a bad job, jobs whose outputs
 * overlap any input or output), LNF_EDEVICE, LNF_ENOMEM, LNF_EHIP, LNF_EBUSY.
 * Argument errors are found before anything is enqueued.
 */
LNF_API int lnf_filter_batch(lnf_handle h, const lnf_job* jobs, int n, hipStream_t stream);

#define LNF_BATCH_GRID 0       /* one workgroup per tile, hardware-dispatched (default) */
#define LNF_BATCH_PERSISTENT 1 /* one workgroup per resident slot, tiles from a queue */

/*
 * lnf_filter_batch with an explicit launch mode; both modes give the same
 * bytes.  LNF_BATCH_PERSISTENT launches, per group, as many workgroups as the
 * GPU holds at once; the group's tiles are cut into one contiguous range per
 * XCD, the workgroups of an XCD deal all but about one round of its range out
 * among themselves by stride, take the rest from that range's atomic counter
 * in the job table, then what is left of the other XCDs' ranges, until the
 * group is done
 * (MEAN9 with 64 x 16 tiles, MINVAR9 with its tuned or default tile).  The
 * grid mode is the faster of the two on the workloads measured; the
 * persistent mode keeps the number of workgroups fixed.  The counters are
 * uploaded as zero with the table,
 * so both modes can be captured in a HIP graph (no memset node).  Default
 * cluster geometry only.  Errors: as lnf_filter_batch; LNF_EINVAL also for an
 * unknown mode, or LNF_BATCH_PERSISTENT on a context with LNF_GEOM_* flags.
 */
LNF_API int lnf_filter_batch_mode(lnf_handle h, const lnf_job* jobs, int n, hipStream_t stream,
                                  int mode);

#define LNF_BATCH_NOALLOC_MAX 256 /* most jobs one lnf_filter_batch_noalloc call accepts */

/*
 * lnf_filter_batch (grid mode) for callers that cannot allocate device memory
 * during the call: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  The call allocates nothing: its job table
 * is a static device array of the library (one per GPU, 20,608 bytes for
 * LNF_BATCH_NOALLOC_MAX jobs, held until the process ends), filled from a
 * host staging slot that lnf_create preallocated; the caller passes the
 * inputs and outputs as for lnf_filter_batch, and the results are the same
 * bytes.  Every call on a GPU, from any context, shares that one table, which
 * keeps the last call's contents: calls whose work overlaps on one GPU
 * (launched on different streams, or from different threads, without
 * ordering between them) race on it and must be serialised by the caller;
 * calls on one stream are ordered by the stream.  A captured call replays
 * into the same table, so the same rule holds for graph replays.
 * Errors: LNF_ERANGE (n > LNF_BATCH_NOALLOC_MAX); otherwise as
 * lnf_filter_batch.
 */
LNF_API int lnf_filter_batch_noalloc(lnf_handle h, const lnf_job* jobs, int n,
                                     hipStream_t stream);

/*
 * Autotune: for every distinct (dtype, radius, volume-size class) among the
 * sample jobs, time each tile variant and z-strip depth on that job (its output
 * is overwritten) and keep the fastest for later lnf_filter / lnf_filter_batch
 * calls of this context.  Synchronous; uses an internal stream.
 * Errors: as lnf_filter_batch.
 */
LNF_API int lnf_tune(lnf_handle h, const lnf_job* sample, int n);

/* Write / read the context's tuned configurations (text, one per line). */
LNF_API int lnf_tune_save(lnf_handle h, const char* path);
LNF_API int lnf_tune_load(lnf_handle h, const char* path);

/* ---- Otsu threshold and the gated pipeline ---------------------------- */
/*
 * Grey-level histogram: hist[v] = number of voxels equal to v.  `hist` is
 * device memory of 256 (LNF_U8) or 65536 (LNF_U16) uint64 counters, cleared
 * and filled by the call (asynchronous on `stream`).
 * Errors: LNF_EINVAL (nulls, dtype, dims, hist overlapping vol), LNF_EDEVICE, LNF_EHIP.
 */
LNF_API int lnf_histogram(lnf_handle h, const void* vol, const int64_t dims[3], int dtype,
                          uint64_t* hist, hipStream_t stream);

/*
 * Otsu's data threshold of a host histogram (paper, Section "Our Method",
 * eq. 1): the T minimising the within-class variance, computed exactly as the
 * T maximising (N*s0 - n0*S)^2 / (n0*n1) with class 0 = levels below T.
 * Lowest T among equal optima; if fewer than two levels are present, T is
 * the present level (0 for an empty histogram).  Host only, no GPU.
 * Errors: LNF_EINVAL (nulls, levels not in 1..65536).
 */
LNF_API int lnf_otsu_threshold(const uint64_t* hist, int levels, uint32_t* T);

/*
 * The paper's automatic pipeline: T = Otsu threshold of `vol`, then the
 * context's rule gated at T (the context's own gate_T is not used).  Reads
 * the histogram back, so `stream` is synchronised once; *T (if not NULL)
 * receives the threshold.  Errors: as lnf_filter, LNF_ENOMEM.
 */
LNF_API int lnf_filter_otsu(lnf_handle h, const void* vol, const int64_t dims[3], int dtype,
                            int radius, void* out, hipStream_t stream, uint32_t* T);

/* ---- comparison filters (paper, Section "Other Filters") ----------------- */
/*
 * The four spatially variant filters the paper compares its method with, as
 * it adapts them to 3D.  Each samples like lnf_filter (coordinates clamped
 * into the volume), rounds averages half up in exact arithmetic, writes the
 * input dtype, and applies the context's gate (out < gate_T -> 0).  The
 * context's rule and geometry are not used.  Readings of the paper's garbled
 * or silent formulas:
 *   mean (eq. 4)     rounded mean of the (2r+1)^3 cube about the voxel;
 *   sigma (eq. 5)    rounded mean of the cube's values v with |v - P0| <= w (P0
 *                    the centre value): the paper's 2-sigma range with
 *                    w = half_width, or, for half_width < 0, w = floor(2 sigma)
 *                    with sigma the standard deviation of all voxel values
 *                    (computed exactly from a histogram; volumes below 2^32
 *                    voxels); *used_half_width (if not NULL) receives w;
 *   Okada (eq. 6)    rounded mean of the centre and its six face neighbours
 *                    whose difference to the centre is < t_d; 0 if none is
 *                    (t_d = 0);
 *   entropy (eq. 7)  P0 if H > t_e, else 0, where H sums -p log2 p over the
 *                    cube's voxels, p the frequency of the voxel's grey level
 *                    in the whole volume; weights and threshold in 2^-32 fixed
 *                    point (floor(x * 2^32 + 1/2), x in fp64 with the C
 *                    library's log2).
 * lnf_filter_mean and lnf_filter_okada are asynchronous on `stream`;
 * lnf_filter_sigma with half_width < 0 and lnf_filter_entropy read a
 * histogram back first (they synchronise `stream`).  Radius 1..LNF_RADIUS_MAX
 * (Okada: the six face neighbours only).
 * Errors: as lnf_filter; LNF_EINVAL also for a non-finite t_e; LNF_ENOMEM.
 */
LNF_API int lnf_filter_mean(lnf_handle h, const void* vol, const int64_t dims[3], int dtype,
                            int radius, void* out, hipStream_t stream);
LNF_API int lnf_filter_sigma(lnf_handle h, const void* vol, const int64_t dims[3], int dtype,
                             int radius, int64_t half_width, void* out, hipStream_t stream,
                             int64_t* used_half_width);
LNF_API int lnf_filter_okada(lnf_handle h, const void* vol, const int64_t dims[3], int dtype,
                             uint32_t t_d, void* out, hipStream_t stream);
LNF_API int lnf_filter_entropy(lnf_handle h, const void* vol, const int64_t dims[3], int dtype,
                               int radius, double t_e, void* out, hipStream_t stream);

/* ---- surface-point mode ------------------------------------------------ */
/*
 * The filter evaluated only at listed voxels, as the paper applies it at the
 * first surface intersection point of each ray.  xyz: device int32 [n][3]
 * (x, y, z); out: device uint32 [n] receives the filtered value (rule and gate
 * of the context), or 0xFFFFFFFF for a point outside the volume.  Same value
 * as lnf_filter at that voxel.  Asynchronous on `stream`.
 * Errors: LNF_EINVAL (also for a context with a non-default cluster geometry),
 * LNF_EDEVICE, LNF_EHIP.
 */
LNF_API int lnf_filter_points(lnf_handle h, const void* vol, const int64_t dims[3], int dtype,
                              int radius, const int32_t* xyz, int64_t n, uint32_t* out,
                              hipStream_t stream);

/*
 * First-hit pass: the point list of the paper's surface intersection points
 * (Section "Our Method") for rays parallel to z.  The ray through pixel
 * (x, y) travels towards +z from slice 0 (direction 1) or towards -z from
 * slice nz-1 (direction -1); its hit is the first voxel it meets whose value
 * is >= threshold (the surface level, e.g. Otsu's T from lnf_histogram and
 * lnf_otsu_threshold).  xyz: device int32 [ny*nx][3], written in full: entry
 * y*nx + x receives (x, y, z_hit), z_hit = -1 when no voxel of the column
 * reaches the threshold (lnf_filter_points reports 0xFFFFFFFF for such an
 * entry).  Context rule, gate and geometry are not used.  Asynchronous on
 * `stream`.  Errors: LNF_EINVAL (nulls, dtype, dims, direction not 1 or -1),
 * LNF_EDEVICE, LNF_EHIP.
 */
LNF_API int lnf_first_hit(lnf_handle h, const void* vol, const int64_t dims[3], int dtype,
                          uint32_t threshold, int direction, int32_t* xyz, hipStream_t stream);

/*
 * Surface pipeline: lnf_first_hit into xyz, then lnf_filter_points at those
 * nx*ny points into out (device uint32 [ny*nx]): the context's filter at
 * each ray's hit, 0xFFFFFFFF for a ray that meets nothing.  Both launches are
 * asynchronous on `stream`.  Errors: as the two calls (a context with a
 * non-default cluster geometry: LNF_EINVAL).
 */
LNF_API int lnf_filter_surface(lnf_handle h, const void* vol, const int64_t dims[3], int dtype,
                               int radius, uint32_t threshold, int direction, int32_t* xyz,
                               uint32_t* out, hipStream_t stream);

/* ---- serving ------------------------------------------------------------ */
/*
 * A request server with continuous batching.  Volumes are uploaded once and
 * stay resident in library-owned device memory; filter requests against them
 * (at any radius) are queued, admitted while their memory fits under the cap
 * (the server holds at most cap_bytes of device memory, allocated in chunks as
 * needed and kept until lnf_server_destroy; volumes and request outputs take
 * ranges of it, so evictions never free device memory), grouped
 * into micro-batches in arrival order, and launched through the batch path on
 * a pool of streams, so batches issued while others run overlap on the
 * device.  A micro-batch takes requests until it holds max_batch of them or
 * the next would take its voxels past the voxel budget (a request larger than
 * the budget runs alone: it fills the device by itself).  A new micro-batch
 * is launched while fewer than two are in flight or the voxels in flight stay
 * under twice the budget; everything else waits in the queue, where later
 * arrivals join it, so the device queue stays short and requests complete
 * close to arrival order.  The FIFO mode follows the same bound with one
 * request per launch.  Idle volumes are evicted least-recently-used first
 * when the cap is reached.  A worker thread owned by the server does the scheduling and
 * completion polling; every function below is thread-safe.
 * Latency of a request = completion observed by the worker - its arrival time
 * (the client's scheduled arrival, so queueing delay is never hidden).
 */
typedef struct lnf_server* lnf_server_handle;

#define LNF_SERVE_BATCHED 0   /* continuous batching over n_streams streams */
#define LNF_SERVE_FIFO 1      /* reference: one lnf_filter per request, in order, one stream */

typedef struct {
    uint32_t size;            /* sizeof(lnf_server_options) */
    int32_t mode;             /* LNF_SERVE_BATCHED or LNF_SERVE_FIFO */
    uint64_t cap_bytes;       /* device-memory cap of the server (> 0) */
    int32_t n_streams;        /* streams micro-batches are spread over (1..16) */
    int32_t max_batch;        /* most requests per micro-batch (1..LNF_BATCH_MAX) */
    int32_t fail_batch;       /* test hook: the n-th batch (1-based) fails on the host
                                 before launch and its requests end LNF_ECANCELED; 0 = off */
    int32_t batch_mvox;       /* voxel budget of a micro-batch, in units of 2^20 voxels
                                 (0: 32, i.e. 2^25 voxels); >= 0 */
} lnf_server_options;

typedef struct {
    uint64_t submitted, completed, failed, cancelled, batches, evictions, uploads;
    uint64_t voxels;          /* voxels filtered by completed requests */
    uint64_t bytes_in_use;    /* current device footprint (memory the server holds) */
    uint64_t peak_bytes;      /* largest footprint seen */
    double p50_ms, p99_ms, max_ms, mean_ms;  /* latency of completed requests */
    double busy_s;            /* first arrival to last completion */
    double gvox_per_s;        /* voxels / busy_s */
} lnf_server_stats_t;

/* Steady clock (ns) the server measures latency with; use it for arrival times. */
LNF_API int64_t lnf_server_now_ns(void);

/* Create a server over context h (its rule and gate apply).  opt NULL: batched,
 * 200 GB cap, 4 streams, max_batch 256, batch budget 2^25 voxels.
 * Errors: LNF_EINVAL, LNF_EHIP, LNF_ENOMEM. */
LNF_API int lnf_server_create(lnf_handle h, const lnf_server_options* opt, lnf_server_handle* srv);

/* Finish all admitted work, fail still-pending requests with LNF_ECANCELED, free
 * everything.  NULL is a no-op. */
LNF_API int lnf_server_destroy(lnf_server_handle srv);

/*
 * Upload a host volume (asynchronously; pinned host memory gives a true DMA)
 * into a new resident volume.  host_pitch, if not NULL, gives the source's row
 * and slice pitch in elements ({row, slice}), so a crop of a larger host
 * volume can be uploaded without packing it first.  The host buffer must stay
 * valid until a request on the volume completes (or lnf_server_sync).
 * Errors: LNF_EINVAL, LNF_EBUSY (cannot fit under the cap even after evicting
 * every idle volume), LNF_ENOMEM, LNF_EHIP.
 */
LNF_API int lnf_server_put_volume(lnf_server_handle srv, const void* host, const int64_t dims[3],
                                  int dtype, const int64_t* host_pitch, uint64_t* vol_id);

/* Drop a resident volume once no request uses it.  Errors: LNF_ENOTFOUND. */
LNF_API int lnf_server_release(lnf_server_handle srv, uint64_t vol_id);

/*
 * Queue a filter request: filter resident volume vol_id at `radius`.  If
 * host_out is not NULL the result is copied there (dense layout, included in
 * the latency).  arrival_ns: scheduled arrival on lnf_server_now_ns's clock;
 * 0 = now.  Errors: LNF_EINVAL, LNF_ENOTFOUND, LNF_EBUSY (the volume and its
 * output together exceed the cap, so the request could never run).  A queued
 * request that cannot get memory for its output while nothing else runs or
 * waits to run (every idle volume evicted) ends with status LNF_EBUSY.
 */
LNF_API int lnf_server_submit(lnf_server_handle srv, uint64_t vol_id, int radius, void* host_out,
                              int64_t arrival_ns, uint64_t* ticket);

/* Status of a request: *done = 1 once it completed or failed; returns LNF_OK,
 * or the request's failure code once done, or LNF_ENOTFOUND. */
LNF_API int lnf_server_poll(lnf_server_handle srv, uint64_t ticket, int* done);

/* Block until the request completes (LNF_OK / its failure code) or timeout_ms
 * passes (LNF_ETIMEDOUT; < 0 waits forever). */
LNF_API int lnf_server_wait(lnf_server_handle srv, uint64_t ticket, int timeout_ms);

/* Cancel a request that has not been admitted yet (LNF_OK), else LNF_EBUSY. */
LNF_API int lnf_server_cancel(lnf_server_handle srv, uint64_t ticket);

/* Block until every submitted request has finished. */
LNF_API int lnf_server_sync(lnf_server_handle srv);

/* Counters and latency percentiles; reset_latency != 0 clears the latency
 * record and counters afterwards (resident volumes are kept). */
LNF_API int lnf_server_stats(lnf_server_handle srv, lnf_server_stats_t* st, int reset);

/* Human-readable text of a status code (static storage). */
LNF_API const char* lnf_strerror(int code);

/* ABI version: major*10000 + minor*100 + patch. */
LNF_API int lnf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LNF_H */
