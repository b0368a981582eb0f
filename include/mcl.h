/*
 * mcl.h -- C ABI of the MI355X (gfx950) belief-tensor localization filter.
 *
 * The filter keeps a dense belief tensor B[theta][y][x] over every robot pose
 * of an occupancy grid and updates it from odometry and, optionally, range
 * scans, as in Peng and Weikersdorfer, "Map as The Hidden Sensor: Fast
 * Odometry-Based Global Localization" (arXiv 1910.00572), Sec. III and Alg. 1.
 *
 * Conventions used throughout
 *   - Grid cell (i, j) has column i (world x, metres = i * cell_m) and row j
 *     (world y).  Heading channel k of n_theta represents the world heading
 *     k * 2 pi / n_theta + theta_offset (Sec. III-A, belief tensor), where
 *     theta_offset is the running sum of odometry heading increments.
 *   - Odometry increments (u, v, w) are robot-frame: u forward, v to the
 *     left (metres), w counter-clockwise heading change (radians).
 *   - Host arrays are row-major and dense: occupancy[j * W + i],
 *     belief[(k * H + j) * W + i].
 *   - All device memory is owned by the caller.  The library never allocates
 *     device memory: the caller queries a workspace size, allocates that many
 *     bytes of device memory (256-byte aligned) and hands it over; the handle
 *     uses it until it is destroyed.  Host inputs are copied during the call.
 *   - Every call returns an mcl_status.  Argument errors are detected before
 *     any work is enqueued and leave the state unchanged; mcl_last_error()
 *     then holds a message (per thread).  Conditions found on the device (all
 *     probability mass removed, a HIP error) are sticky and are reported by
 *     the next synchronising call (mcl_normalize, mcl_read_belief,
 *     mcl_get_info with sync = 1).
 *   - "async" calls only enqueue work on the handle's stream and return.
 *   - A handle is not thread-safe; drive each handle from one host thread.
 */
#ifndef MCL_H_
#define MCL_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MCL_OK = 0,
  MCL_EINVAL = 1,      /* bad argument; nothing was enqueued */
  MCL_ENOMEM = 2,      /* workspace smaller than the queried size */
  MCL_EDEGENERATE = 3, /* a step removed all probability mass (belief kept) */
  MCL_EDEVICE = 4,     /* a HIP runtime error; message in mcl_last_error() */
  MCL_ESTATE = 5       /* call not valid in the current state (e.g. no range table) */
} mcl_status;

typedef enum { MCL_F32 = 0, MCL_BF16 = 1, MCL_F16 = 2 } mcl_dtype;

/* Map-level flags (Alg. 1).  Default MCL_MASK_BEFORE_BLUR | MCL_WALL_NORMALIZE. */
enum {
  MCL_MASK_BEFORE_BLUR = 1u, /* multiply by the traversability map after the warp */
  MCL_WALL_NORMALIZE = 2u,   /* divide by the kernel activation G(B_0) after the blur */
  MCL_SUBCELL_GATE = 4u,     /* accumulate motion until it reaches one cell (Alg. 1 IF) */
  MCL_SCAN_F32 = 8u,         /* scan cross term on FP32 operands instead of BF16 */
  MCL_INTEGER_SHIFT = 16u,   /* warp by whole cells: each channel moves by its displacement plus the
                                remainder it carries, rounded half up (floor(d + 1/2)), and carries
                                d - floor(d + 1/2) to the next warp; with MCL_SUBCELL_GATE the warp
                                happens when the gate fires */
  MCL_ANISOTROPIC = 32u      /* motion noise with covariance R(psi_k) diag(sf^2, sl^2) R(psi_k)^T
                                rotated to each channel's pre-step heading psi_k (eq. Gaussian
                                kernel): sf = sigma_xy_cells along the heading, sl =
                                sigma_lateral_cells across it; the theta blur runs first, then
                                each channel's 2-D blur, with its own kernel activation G(B_0, k) */
};

typedef struct {
  int32_t width, height;        /* W, H >= 1 */
  double cell_m;                /* cell size in metres, > 0 */
  const uint8_t* occupancy;     /* host, H*W, nonzero = occupied; copied */
  const float* range_table;     /* host, nullable: expected range in metres from the centre
                                   of each cell along world direction d * 2 pi / n_dirs,
                                   layout [(j*W + i) * n_dirs + d]; copied and quantised */
  int32_t n_dirs;               /* directions per cell (required if range_table != NULL) */
  double max_range_m;           /* sensor range; ranges are quantised to max_range_m / 256 */
} mcl_map_desc;

typedef struct {
  int32_t n_theta;              /* heading channels, 1 .. 360 */
  double sigma_xy_cells;        /* motion-noise std-dev in x and y, cells, >= 0 */
  double sigma_theta_bins;      /* motion-noise std-dev in theta, bins, >= 0 */
  int32_t radius_xy;            /* blur half-width in cells; < 0 => ceil(3 sigma) */
  int32_t radius_theta;         /* blur half-width in bins;  < 0 => ceil(3 sigma) */
  mcl_dtype storage;            /* belief storage type; arithmetic is always FP32 */
  uint32_t flags;               /* MCL_* flags above */
  double sigma_lateral_cells;   /* MCL_ANISOTROPIC: noise std-dev across the heading, cells, > 0
                                   (sigma_xy_cells is then the std-dev along it, > 0; the 2-D
                                   kernel radius is radius_xy, or ceil(3 max(sf, sl)), at most 6) */
  int32_t launch_shape[7];      /* testing and tuning only (filters; maps ignore it).  All zero:
                                   the library chooses the step kernel's launch shape.  Otherwise
                                   {tile width (0 = streaming kernel), rows per tile, threads per
                                   workgroup, heading chunks (0 = automatic), source-row buffers
                                   (streaming), variant (streaming: 0, 1 or 2), output strip
                                   alignment in bytes (streaming; 0 = 32)}; init_belief fails with
                                   EINVAL if no kernel has that shape */
} mcl_params;

typedef struct {
  int32_t i, j, k;              /* grid cell and heading channel */
  double x_m, y_m, theta_rad;   /* i*cell, j*cell, k*2pi/n_theta + theta_offset */
  double prob;                  /* normalised probability of that state */
} mcl_pose;

typedef struct {
  int32_t width, height, n_theta, pitch; /* device rows are `pitch` elements apart */
  int32_t storage;              /* mcl_dtype */
  int32_t radius;               /* blur radius the kernels run with */
  int32_t tile_x, tile_y, theta_chunks, workgroups; /* launch shape of the step kernel */
  int64_t steps;                /* odometry steps applied */
  double theta_offset_rad;      /* running heading offset */
  double log_norm;              /* sum over updates of ln(kept mass) (valid after a sync) */
  int32_t status;               /* sticky device status (valid after a sync) */
  const void* belief_device;    /* current stored belief (device, pitch layout, scaled) */
  uint64_t state_bytes;         /* belief bytes one step reads (= bytes it writes) */
} mcl_info;

typedef struct mcl_map_s* mcl_map;
typedef struct mcl_filter_s* mcl_filter;

/* Thread-local message describing the last non-OK status. */
const char* mcl_last_error(void);

/* ---- map ------------------------------------------------------------------ */

/* Device bytes a map needs for this description and these parameters
 * (traversability, wall weights, and the quantised range table if given).
 * Returns 0 if the arguments are invalid. */
size_t mcl_map_workspace_bytes(const mcl_map_desc* desc, const mcl_params* params);

/* Build a map: traversability M (Sec. III-A-3), the kernel activation
 * G(B_0) and the post-blur weights M / G(B_0) (Alg. 1, last statement), and
 * the range table quantised to centred counts of max_range/256 together with
 * its per-cell sum of squares (dense scan update, eq. sensor update).  Uses
 * sigma_xy / radius_xy / flags of `params`; the theta fields are ignored.
 * `stream` is a hipStream_t (NULL = default stream).  Synchronous.
 * EINVAL for a size out of [1, 65536], a non-positive cell size, n_dirs
 * outside [1, 1024], or a quantised range table of 4 GiB or more (cells x
 * n_dirs rounded up to 64 x 2 bytes, 4 with MCL_SCAN_F32); ENOMEM if
 * ws_bytes is below mcl_map_workspace_bytes.
 * The map must outlive every filter created on it. */
mcl_status mcl_map_create(const mcl_map_desc* desc, const mcl_params* params, void* dev_ws,
                          size_t ws_bytes, void* stream, mcl_map* out);
void mcl_map_destroy(mcl_map map);

/* ---- filter ---------------------------------------------------------------- */

/* Device bytes a filter needs: two belief buffers (storage type, pitch
 * layout), a one-slice FP32 staging area, reduction partials and the device
 * scalars; plus an FP32 scan scratch when the map has a range table. */
size_t mcl_filter_workspace_bytes(mcl_map map, const mcl_params* params);

/* init_belief: create a filter on `map` (Sec. III-A, belief tensor).
 * init_host == NULL: B_0 uniform over the free cells of every heading channel.
 * Otherwise init_host is a host FP32 array of n_theta*H*W non-negative values
 * (any scale; it is renormalised) that becomes B_0 (checkpoint resume); it is
 * stored multiplied by the power of two that brings its largest value into
 * [1/2, 1) (exact), as the steps store the belief near a peak of one, so a
 * sum-one export resumes in 16-bit storage without flushing small values.
 * theta0_rad sets the running heading offset.  sigma_xy / radius_xy / flags
 * must equal those the map was built with.  With init_host the call returns
 * once the upload is done; the uniform start is only enqueued on `stream`. */
mcl_status mcl_init_belief(mcl_map map, const mcl_params* params, void* dev_ws, size_t ws_bytes,
                           void* stream, const float* init_host, double theta0_rad,
                           mcl_filter* out);
void mcl_filter_destroy(mcl_filter f);

/* step_odometry (async): one odometry update, Alg. 1 followed by
 * renormalisation (eq. sensor update's eta applied to the motion update):
 * every channel k is warped bilinearly by R(theta_offset + k*2pi/n_theta)
 * [u, v] (Sec. III-A-1), multiplied by M, blurred by the separable Gaussian
 * (x, y zero-padded, theta circular; Sec. III-A-2), multiplied by
 * M / G(B_0), and renormalised; then theta_offset += w.  With
 * MCL_SUBCELL_GATE the motion is accumulated and applied once it reaches one
 * cell.  With MCL_INTEGER_SHIFT the warp is a whole-cell translation with a
 * per-channel remainder carry (the remainders are host state of the handle).
 * EINVAL for non-finite input or |(u, v)| above 1e6 cells. */
mcl_status mcl_step_odometry(mcl_filter f, double u_m, double v_m, double w_rad);

/* apply_scan (async): dense observation update (eq. sensor update) with a
 * per-beam Gaussian range model of std-dev sigma_m.  ranges_m holds n_beams
 * host FP32 ranges; beam b points at heading(k) + b * 2 pi / n_beams.
 * n_beams must equal the map's n_dirs; ESTATE if the map has no range table. */
mcl_status mcl_apply_scan(mcl_filter f, const float* ranges_m, int32_t n_beams, double sigma_m);

/* apply_scan_batch (async, serving): mcl_apply_scan for n distinct filters
 * of one map, driven on one stream.  ranges_m: host FP32, n scans of n_beams
 * beams (filter i's at ranges_m[i * n_beams]); sigma_m: one std-dev per
 * filter.  The cross-term products of all filters run in one launch in which
 * every workgroup takes its tile of the range table for each filter in turn,
 * so the table is read from memory once per launch instead of once per
 * filter (up to 16 filters of one storage type and heading count per
 * launch).  Each filter's result is bitwise that of mcl_apply_scan.  Errors
 * as mcl_apply_scan for any filter; EINVAL for a repeated filter, filters of
 * different maps or streams, or NULL pointers. */
mcl_status mcl_apply_scan_batch(mcl_filter* const filters, const float* ranges_m, int32_t n_beams,
                                const double* sigma_m, int32_t n);

/* normalize (sync): rescale the stored belief in place so it sums to one
 * (FP32, BF16) or peaks at one (FP16, whose range cannot hold a sum-one
 * belief), and return the accumulated log-normaliser ln prod(kept mass)
 * (eq. sensor update's eta) in *log_norm_out (nullable).  Reports sticky
 * device errors. */
mcl_status mcl_normalize(mcl_filter f, double* log_norm_out);

/* read_belief (sync): copy the normalised FP32 belief (sums to one) into
 * host_out (n_theta*H*W, nullable), the most probable state into *argmax
 * (nullable; lowest flat index (k, j, i) wins ties; the belief map is the max
 * over theta, Sec. III-A last paragraph), the running heading offset and the
 * log-normaliser (both nullable).  Reports sticky device errors. */
mcl_status mcl_read_belief(mcl_filter f, float* host_out, mcl_pose* argmax,
                           double* theta_offset_rad, double* log_norm);

/* export_belief (async): write the normalised FP32 belief into dev_out
 * (device, n_theta*H*W dense) and, if dev_map_out != NULL, the belief map
 * max_k B into dev_map_out (device, H*W). */
mcl_status mcl_export_belief(mcl_filter f, float* dev_out, float* dev_map_out);

/* export_scalars (async): dev_out (device, two doubles) receives the
 * log-normaliser and the sticky status (as a double: 0 = MCL_OK, 3 =
 * MCL_EDEGENERATE) as they stand after the work enqueued so far, so that a
 * serving loop can retire a filter without synchronising the stream. */
mcl_status mcl_export_scalars(mcl_filter f, double* dev_out);

/* scan_sqdist (async, diagnostic): the exact integer squared distance
 * D[k][j][i] = sum_b (zq_b - rq(i, j, beam b of channel k))^2 between the
 * quantised scan and the quantised table, as the scan update computes it
 * (cross term on the matrix cores).  dev_out: device int32, n_theta*H*W. */
mcl_status mcl_scan_sqdist(mcl_filter f, const float* ranges_m, int32_t n_beams,
                           int32_t* dev_out);

/* sample_cells (async): the Floyd-Steinberg sample set of the belief map
 * (Sec. III-B, dithering).  m(i, j) = max_k of the stored belief (Sec. III-A,
 * last paragraph); intensity I = min(1, n_samples * m / sum m), the sum in
 * FP64 rounded to FP32, product and quotient in FP32; then error diffusion as
 * mcl_dither.  About n_samples cells are selected.  dev_mask: device uint8,
 * H*W dense (row stride W), written with 1 (selected) or 0.  Uses the
 * filter's staging area.  EINVAL for n_samples < 0 or a map beyond the
 * dithering kernel (see mcl_dither). */
mcl_status mcl_sample_cells(mcl_filter f, int32_t n_samples, uint8_t* dev_mask);

/* apply_scan_sampled (async): the observation update (eq. sensor update) on
 * the sampled states only (Sec. III-B): every heading channel of each cell
 * whose dev_mask byte (device, H*W dense) is nonzero.  With D the squared
 * distance of mcl_scan_sqdist and D* its minimum over the sampled states, a
 * sampled state is multiplied by exp(-c (D - D*)), c = h^2 / (2 sigma_m^2),
 * h = max_range / 256; unsampled states keep their value (they take the
 * likelihood of the best-matching sample).  Then the belief is renormalised
 * and the log-normaliser grows by ln(kept mass) - c D*.  An empty mask
 * changes nothing.  If no mass is left the belief is kept and the filter
 * reports MCL_EDEGENERATE.  Arguments as mcl_apply_scan; ESTATE without a
 * range table; EINVAL for a NULL mask or 2^31 states or more. */
mcl_status mcl_apply_scan_sampled(mcl_filter f, const float* ranges_m, int32_t n_beams, double sigma_m,
                                  const uint8_t* dev_mask);

/* dither (async): Floyd-Steinberg error diffusion of a device FP32 image
 * (H*W dense, any values) into dev_mask (device uint8, H*W): raster order,
 * threshold 1/2 (selected if intensity plus received error >= 1/2), error
 * weights 7/16 right, 3/16 below-left, 5/16 below, 1/16 below-right, error
 * leaving the image dropped.  Received error is summed in raster arrival
 * order; every product and sum is FP32 rounded to nearest, no fused
 * multiply-add.  `stream` is a hipStream_t (NULL = default stream).  A zero
 * width or height does nothing.  EINVAL for negative sizes, NULL pointers,
 * W * H >= 2^29, or H >= 4096 together with W >= 8190 (the error ring of the
 * wavefront kernel lives in 64 KB of LDS). */
mcl_status mcl_dither(const float* dev_intensity, int32_t width, int32_t height, uint8_t* dev_mask,
                      void* stream);

/* Device bytes mcl_best_match needs for batches of up to `batch` queries
 * (0 if the map has no range table or the arguments are out of range): the
 * batch's circulant columns plus one 4-byte key per 128 cells and column,
 * about 4 * (H * pitch / 128) * batch * n_theta bytes. */
size_t mcl_match_workspace_bytes(mcl_map map, int32_t n_theta, int32_t batch);

/* best_match (sync): for each query scan, the state that matches it best
 * (map difficulty, Sec. IV, localisation robustness): the free cell q and
 * heading channel k with the smallest exact squared distance D of the scan
 * update (as mcl_scan_sqdist, channel k at heading k 2 pi / n_theta, no
 * heading offset), ties to the lowest k * H * W + q; occupied cells are not
 * candidates.  ranges_m: host FP32 n_queries x n_dirs (metres, quantised as
 * the scan update does).  out_cell: host int32 per query, j * W + i;
 * out_heading, out_dist: host int32 per query (nullable).  Runs in batches of
 * `batch` queries on the map's range table with dev_ws (caller-owned device
 * memory of at least mcl_match_workspace_bytes(map, n_theta, batch) bytes);
 * the next batch is quantised on the host while one runs, through two pinned
 * host staging buffers that the call allocates and frees itself.
 * ESTATE without a range table; EINVAL for n_theta outside [1, 360], a table
 * deeper than 384 directions, H * pitch >= 2^30 (pitch = W rounded up to a
 * multiple of 8), batch * n_theta columns of 2 GiB
 * or more (batch * n_theta * 384 * 2 bytes for BF16 operands, * 4 for FP32),
 * non-finite ranges or NULL pointers; ENOMEM for a small workspace. */
mcl_status mcl_best_match(mcl_map map, int32_t n_theta, const float* ranges_m, int32_t n_queries,
                          int32_t batch, int32_t* out_cell, int32_t* out_heading, int32_t* out_dist,
                          void* dev_ws, size_t ws_bytes, void* stream);

/* difficulty (host): D_M (Sec. IV), the fraction of the n query cells whose
 * best match lies more than threshold_m metres from them (distance between
 * cell centres, the map's cell size; a best cell of -1 counts as far).
 * query_cells, best_cells: host int32 j * W + i.  EINVAL for NULL pointers
 * with n > 0, n < 0, a query cell outside the map or a negative threshold;
 * n == 0 gives 0. */
mcl_status mcl_difficulty(mcl_map map, const int32_t* query_cells, const int32_t* best_cells, int32_t n,
                          double threshold_m, double* out);

/* Launch shape, sizes and scalars.  sync != 0 waits for the stream first so
 * log_norm and status are current. */
mcl_status mcl_get_info(mcl_filter f, int sync, mcl_info* out);

/* Device bytes the batch job tables of mcl_step_batch (which uses the first
 * half) and of mcl_batch_create (two parameter slots) need for up to
 * max_filters filters per step (0 if out of range). */
size_t mcl_batch_workspace_bytes(int32_t max_filters);

/* step_batch (async, serving): one odometry step (as mcl_step_odometry) for
 * each of n distinct filters, enqueued on `stream` as one launch per group of
 * filters that share a storage type, blur radius and launch shape; filters of
 * any grid size and heading count mix in one launch.  uvw holds 3 doubles
 * (u, v, w) per filter.  dev_ws is caller-owned device memory of at least
 * mcl_batch_workspace_bytes(n) bytes holding the job table; it must not be
 * reused until the launches complete (stream order).  Each filter's result is
 * bitwise identical to stepping it alone: its tiles, reduction order and
 * final reduction do not depend on the batch.  All filters must have been
 * created on `stream` or be ordered with it by the caller. */
mcl_status mcl_step_batch(mcl_filter* const filters, const double* uvw, int32_t n, void* dev_ws,
                          size_t ws_bytes, void* stream);

/* step_batch_noalloc (async): mcl_step_batch for callers that cannot
 * allocate memory (tight serving loops, harnesses that forbid allocation).
 * Each filter's host bookkeeping runs at call time, so a captured graph of
 * this call would replay one step's parameters: graph replay of batched steps
 * is mcl_batch_step's job.  It takes no workspace and allocates
 * nothing: the job table lives in a device array of the library (2 MiB per
 * GPU the library runs on, held until the process ends, addressed on the
 * current device, which must be the filters' device) and its host staging in
 * a host array of the library.  At most 256 filters per call (EINVAL above).
 * Calls share those arrays: concurrent calls from several threads are
 * serialised by a lock, and calls on one GPU whose launches overlap on
 * different streams race on the device array (drive them from one stream).
 * Results are bitwise those of mcl_step_batch; other errors as it. */
mcl_status mcl_step_batch_noalloc(mcl_filter* const filters, const double* uvw, int32_t n, void* stream);

/* ---- serving: graph-replayed batched steps ---------------------------------------- */
typedef struct mcl_batch_s* mcl_batch;

/* Create a batch runner on `stream` (a hipStream_t other than the default
 * NULL stream, which cannot be captured) for up to max_filters filters per
 * step (the continuous-batching pattern of the serving loop).
 * dev_ws: caller-owned device memory of mcl_batch_workspace_bytes(max_filters)
 * bytes, two parameter slots used in turn; the runner also allocates two
 * pinned host slots of the same size (host memory, freed by destroy).  EINVAL
 * for max_filters outside [1, 65536], NULL pointers or a NULL stream; ENOMEM
 * for a small workspace; EDEVICE if the pinned allocation fails. */
mcl_status mcl_batch_create(int32_t max_filters, void* dev_ws, size_t ws_bytes, void* stream, mcl_batch* out);

/* batch_step: one odometry step for each of n distinct filters, the same
 * work and the same bitwise results as mcl_step_batch, launched as a HIP
 * graph: the host writes every filter's step parameters (job table with the
 * odometry, per-channel shift tables) into a pinned slot; the graph copies
 * the slot into device memory and runs one launch per kernel group, which
 * read their parameters there.  Graphs are instantiated per launch structure
 * (groups, job and workgroup counts) and replayed while it repeats, so
 * filters joining or leaving cost one capture.  A slot is rewritten only after
 * the replay that read it has completed (the call may wait for it).  The
 * graphs hold no memset node.  Filters must be driven on the runner's stream.
 * Errors as mcl_step_batch; EINVAL for n above max_filters. */
mcl_status mcl_batch_step(mcl_batch b, mcl_filter* const filters, const double* uvw, int32_t n);

/* Graph captures and replays of the runner so far (diagnostics). */
mcl_status mcl_batch_counts(mcl_batch b, int64_t* captures, int64_t* replays);

/* Waits for the runner's outstanding replays, then frees it. */
void mcl_batch_destroy(mcl_batch b);

#ifdef __cplusplus
}
#endif

#endif /* MCL_H_ */
