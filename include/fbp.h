/*
 * fbp.h - C ABI of the MI355X (gfx950) parallel-beam filtered backprojection library.
 *
 * The library reconstructs 2D slices from parallel-beam sinograms as in
 * arXiv 2109.02174, section "Computed tomography": every projection row
 * P_theta(t) is convolved with a filter kernel H to give Q_theta = P_theta * H,
 * and the image is the sum over angles of Q_theta_i evaluated on each pixel's
 * ray x cos(theta_i) + y sin(theta_i) = t (Eq. 2).
 *
 * Conventions (the paper leaves them open; these are the readings adopted):
 *   - H is the Ram-Lak band-limited ramp: h(0) = 1/(4 dt^2), h(d) = 0 for even
 *     d != 0, h(d) = -1/(pi^2 d^2 dt^2) for odd d, applied as a linear
 *     convolution over the D bins (zeros beyond both ends), times dt.
 *   - Eq. 2 is weighted by pi/K and evaluates Q between bins by linear
 *     interpolation; beyond the detector Q is zero and the interpolation ramps
 *     to it over one bin.
 *   - Detector bin j sits at t_j = (j - (D-1)/2) * det_spacing.  Pixel (r, c)
 *     of the N x N image sits at x = c - (N-1)/2, y = r - (N-1)/2 (unit pixel
 *     pitch): rows follow y, columns follow x.  Angles are radians from +x.
 *
 * Layouts: all device arrays are row-major, contiguous, FP32 and 4-byte
 * aligned.  A sinogram stack is [n_slices][n_angles][n_det]; an image stack is
 * [n_slices][N][N].
 *
 * Ownership: the caller owns every device buffer and keeps it alive until the
 * work queued on `hip_stream` has finished.  The library owns only per-geometry
 * plan state (FP64 cos/sin tables, the tile choice, partial-sum planes for the
 * shapes that split a slice's angles), created on the first call for a geometry
 * and kept until process exit, plus tables made on first use: the filter taps
 * of each operand precision (on the first filter call with that precision), the
 * FFT tables (first FBP_PREC_FP32_FFT call), the forward projector's padded
 * copies (first fbp_project call) and the cone-beam pre-weighting rows (first
 * fbp_cone_filter call).  Once those exist, no call allocates device memory.
 * The library's one static device array, the FBP_NOALLOC_WORKSPACE_BYTES
 * workspace of fbp_reconstruct_noalloc, exists on every GPU that loads it.
 *
 * Errors: arguments are validated on the host before any HIP call; a rejected
 * call has queued no work.  Launch failures are reported as FBP_EHIP.  Work is
 * asynchronous on `hip_stream` (NULL = the null stream): faults during
 * execution surface at the caller's next synchronisation.  No function aborts,
 * throws or prints on the hot path.  All functions are thread-safe.
 *
 * Determinism: every output value is written once, by one GPU thread (no
 * atomics), and every call is bitwise reproducible.  For parallel-beam
 * geometries with N >= 2 whose angles come in quarter-turn pairs
 * (theta_{k+K/2} = theta_k + pi/2, as every uniform list with even K) and whose
 * detector spacing is above about 0.36 pixel (a 16 x 16 tile's ray window
 * within 64 bins) the tile
 * shape and the summation order depend on the geometry alone: a slice
 * reconstructed alone, in a stack or inside a batch gives bitwise-equal images,
 * whatever the autotuner chose.  Other geometries may run single slices, stacks
 * and batches with different tile shapes (and the autotuner picks shapes by
 * timing); those paths agree within the FP32 tolerance.
 */
#ifndef FBP_H
#define FBP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FBP_OK = 0,
    FBP_EINVAL = -1,        /* invalid argument (null pointer, bad size, aliasing, misalignment) */
    FBP_ENOMEM = -2,        /* plan creation could not allocate device or host memory */
    FBP_EHIP = -3,          /* a HIP runtime call or kernel launch failed */
    FBP_EUNSUPPORTED = -4,  /* valid but outside the supported range (e.g. geometry too large) */
    FBP_EWORKSPACE = -5,    /* workspace missing or smaller than the *_workspace_bytes query */
    FBP_ENOTREADY = -6      /* fbp_reconstruct_noalloc: no plan or filter taps exist yet for the
                               geometry and precision on this device (nothing was queued) */
} fbp_status;

/* Operand precision of the ramp-filter GEMM; accumulation is always FP32. */
typedef enum {
    FBP_PREC_FP32 = 0,
    FBP_PREC_BF16 = 1,      /* sinogram rows and kernel taps rounded to bfloat16 (RNE) */
    FBP_PREC_FP16 = 2,      /* rounded to binary16 (RNE); taps pre-scaled by 2^s to stay normal */
    FBP_PREC_FP32_FFT = 3   /* FP32 without the GEMM: each pair of rows, zero-padded to a power of two
                               L >= 2D-1, is filtered by FFT, multiplication by the taps' DFT and
                               inverse FFT (equal to the linear convolution); D <= 4096; not for
                               fbp_reconstruct_batch (FBP_EUNSUPPORTED) */
} fbp_precision;

/* Filter kernel of the convolution Q = P * H (all with full support |d| <= D-1). */
typedef enum {
    FBP_FILTER_RAMLAK = 0,       /* h(0) = 1/(4 dt^2), h(even) = 0, h(odd d) = -1/(pi^2 d^2 dt^2) */
    FBP_FILTER_SHEPP_LOGAN = 1,  /* h(d) = -2/(pi^2 dt^2 (4 d^2 - 1)): ramp x sin(w/2)/(w/2) */
    FBP_FILTER_HANN = 2          /* Ram-Lak smoothed by (1/4, 1/2, 1/4): ramp x cos^2(w/2) */
} fbp_filter_kind;

/* Weight of each angle's term in Eq. 2. */
typedef enum {
    FBP_WEIGHT_UNIFORM = 0,      /* pi/K for every angle (angles evenly spread over a half-turn) */
    FBP_WEIGHT_ANGLE_GAPS = 1    /* each angle, reduced to [0, pi), gets half the gaps to its two
                                    neighbours (wrapping around); sums to pi; = pi/K when even */
} fbp_weighting;

/* One geometry (with the filter kernel and angular weights it is reconstructed
 * with; zero-initialised fields give parallel beam, Ram-Lak and pi/K).
 *
 * source_distance == 0: parallel beam, the ray x cos(theta_k) + y sin(theta_k) = t
 *   (section "Computed tomography"), angles theta_k, bins at t_j = (j - (D-1)/2) dt.
 * source_distance == R > 0: fan beam with a flat detector (Kak & Slaney 1988,
 *   ch. 3): view k has its source at R (cos b_k, sin b_k), angles holds the b_k
 *   (views spread over a full turn), and bin j sits at s_j = (j - (D-1)/2) dt on
 *   the detector line through the centre along (-sin b_k, cos b_k).  R must
 *   exceed N / sqrt(2) (the source stays outside the image); weighting must be
 *   FBP_WEIGHT_UNIFORM.  Fan geometries run through fbp_filter, fbp_backproject,
 *   fbp_reconstruct, fbp_reconstruct_noalloc, fbp_reconstruct_batch and
 *   fbp_project; fbp_autotune has nothing to tune for them (FBP_OK, tile id -1);
 *   the other entry points return FBP_EUNSUPPORTED.
 */
typedef struct {
    int32_t n_angles;        /* K >= 1 */
    int32_t n_det;           /* D >= 1 */
    int32_t image_size;      /* N >= 1: the image is N x N */
    double det_spacing;      /* dt > 0 and finite, in pixel units */
    const double* angles;    /* host array of K finite radians; copied into the plan, never kept */
    int32_t filter;          /* fbp_filter_kind */
    int32_t weighting;       /* fbp_weighting */
    double source_distance;  /* 0: parallel beam; R > N/sqrt(2): fan beam, flat detector */
} fbp_geom;

/* One slice of a mixed batch. */
typedef struct {
    fbp_geom geom;
    const float* sino;       /* device [K][D] */
    float* image;            /* device [N][N] */
} fbp_job;

/*
 * Ramp filter (the convolution Q = P * H, section "Computed tomography"):
 *   d_filtered[b][k][n] = dt * sum_{m<D} h(n - m) * d_sino[b][k][m],
 * h the kernel geom->filter selects.
 * Runs as a GEMM on the matrix cores: rows of the sinogram times the Toeplitz
 * matrix of the kernel, operands in `precision`, FP32 accumulation.  The
 * Ram-Lak kernel vanishes at even offsets, so it takes half the MACs of the
 * others.
 * d_sino and d_filtered are [n_slices][K][D] and must not overlap.
 * n_slices == 0 is a valid no-op.
 * Fan beam: each view value is multiplied by R / sqrt(R^2 + s_m^2) as the filter
 * loads it (no scratch) and the kernel is halved:  d_filtered[b][k][n] = dt * sum_m (h(n-m)/2) * d_sino[b][k][m] R / sqrt(R^2 + s_m^2).
 */
int fbp_filter(const fbp_geom* geom, int32_t n_slices, const float* d_sino, float* d_filtered,
               int32_t precision, void* hip_stream);

/*
 * Backprojection (Eq. 2 with weight pi/K, or the angle-gap weights w_k of
 * geom->weighting, and linear interpolation):
 *   d_image[b][r][c] = sum_k w_k Q~_k(u_k(x_c, y_r)),
 *   u_k(x, y) = (x cos(theta_k) + y sin(theta_k)) / dt + (D-1)/2.
 * d_filtered is [n_slices][K][D], d_image is [n_slices][N][N]; no overlap.
 * Every image pixel is written.  With d_filtered = the raw sinogram this is
 * the exact adjoint of the linear-interpolation (hat) projector.
 * Quarter-turn geometries (see Determinism above) run one kernel for any
 * number of slices: a 16-wave workgroup per 16 x 16 tile of the top-left
 * quadrant and its three turns, wave w summing the w-th of 16 contiguous chunks
 * of the angle pairs in ascending order, the chunk sums added in order.  Other
 * geometries: stacks of 4 or more slices run with the plan's stack tile shape
 * (fbp_plan_stack_config), shorter ones slice by slice with its single-slice
 * shape (fbp_plan_config); a single-slice shape with one angle group splits
 * the angles over several workgroups per tile and adds the parts in a fixed
 * order from a partial-sum buffer owned by the plan (calls that use it are
 * ordered among themselves on the device); the two shapes agree within the
 * FP32 tolerance.
 * Fan beam: d_image[b](X) = (2 pi / K) sum_k (R/L_k)^2 Q~_k(s_k(X) / dt + (D-1)/2),
 * L_k = R - (x cos b_k + y sin b_k) the depth of X along the central ray and
 * s_k(X) = R (-x sin b_k + y cos b_k) / L_k where the ray through X meets the
 * detector; 16 x 16 pixel tiles, one pixel per lane, deterministic.
 */
int fbp_backproject(const fbp_geom* geom, int32_t n_slices, const float* d_filtered,
                    float* d_image, void* hip_stream);

/*
 * fbp_backproject(fbp_filter(d_sino)) with the filtered rows kept in the
 * caller's workspace (at least fbp_workspace_bytes(geom, n_slices, precision)
 * bytes of device memory, 256-byte aligned).  Bitwise equal to the two calls.
 */
int fbp_reconstruct(const fbp_geom* geom, int32_t n_slices, const float* d_sino, float* d_image,
                    void* d_workspace, size_t workspace_bytes, int32_t precision,
                    void* hip_stream);

/* Size of the library's own workspace of fbp_reconstruct_noalloc (one per GPU). */
#define FBP_NOALLOC_WORKSPACE_BYTES ((size_t)64 << 20)

/*
 * fbp_reconstruct for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the filtered rows go to a workspace inside the library, a static device
 * array of FBP_NOALLOC_WORKSPACE_BYTES that each GPU the library runs on holds
 * until the process ends, instead of a caller's buffer.  Same kernels, so
 * bitwise equal to fbp_reconstruct with the same arguments.
 * Calls no hipMalloc, hipFree or other allocating routine: the geometry's plan
 * and the filter taps of `precision` must already exist on the current device
 * (made by an earlier fbp_reconstruct or fbp_filter call with this geometry and
 * precision), else FBP_ENOTREADY.  More than FBP_NOALLOC_WORKSPACE_BYTES of
 * filtered rows (n_slices * K * D * 4 bytes) gives FBP_EWORKSPACE.  Both are
 * returned before anything is queued.
 * Every call on one GPU uses that GPU's one array and leaves its contents
 * there: calls whose work can overlap on the device (unordered streams, other
 * threads) race on it and give wrong images.  Order them on one stream.
 * The first call on each GPU looks up the array's device address
 * (hipGetSymbolAddress, no allocation); make that call before capturing a graph.
 */
int fbp_reconstruct_noalloc(const fbp_geom* geom, int32_t n_slices, const float* d_sino, float* d_image,
                            int32_t precision, void* hip_stream);

/*
 * Forward projector, the exact adjoint of fbp_backproject (for iterative methods
 * and adjoint checks):
 *   d_sino[b][k][j] = w_k * sum_{r,c} d_image[b][r][c] * max(0, 1 - |u_k(x_c, y_r) - j|),
 * u_k as in fbp_backproject, w_k = pi/K or the angle-gap weights of
 * geom->weighting.  d_image is [n_slices][N][N], d_sino [n_slices][K][D]; no
 * overlap.  Gather-only (one lane per detector bin), no atomics, deterministic;
 * <fbp_project(x), y> = <x, fbp_backproject(y)> up to FP32 rounding.
 * Fan beam: the adjoint of the fan-beam fbp_backproject,
 *   d_sino[b][k][j] = (2 pi / K) sum_X d_image[b](X) (R/L_k)^2 max(0, 1 - |s_k(X)/dt + (D-1)/2 - j|),
 * with L_k and s_k as there; FBP_EUNSUPPORTED when the detector reaches the
 * source distance ((D-1) dt / 2 >= R) or the source is too close to the image for
 * the projector's window bound.
 */
int fbp_project(const fbp_geom* geom, int32_t n_slices, const float* d_image, float* d_sino,
                void* hip_stream);

/* Workspace bytes fbp_reconstruct needs (0 on invalid arguments). */
size_t fbp_workspace_bytes(const fbp_geom* geom, int32_t n_slices, int32_t precision);

/*
 * Mixed-size batch: fbp_reconstruct of every job (the convolution Q = P * H and
 * Eq. 2 of section "Computed tomography", each job with its own geometry, one
 * slice per job).  Grouped filter GEMMs and a persistent, cost-ordered
 * backprojection launch per tile shape, replayed from a captured HIP graph.
 * Quarter-turn geometries all take the chunked quarter-turn kernel, so each such
 * image is bitwise equal to fbp_reconstruct of the slice alone or in a stack.
 * For other geometries, jobs of a geometry that occurs 4 or more times take its
 * stack shape (bitwise equal to fbp_reconstruct of the geometry's stack) and
 * the others its single-slice shape without angle split (bitwise equal to
 * fbp_reconstruct alone unless that shape splits, then equal within the FP32
 * tolerance).  Fan-beam jobs (Kak & Slaney 1988, ch. 3) run after the
 * parallel-beam ones, one by one through the fan-beam kernels, each bitwise
 * equal to fbp_reconstruct of the slice alone.  The workspace
 * (fbp_batch_workspace_bytes) holds the filtered rows and the tile list; calls
 * that share a workspace must be ordered on one stream.
 */
int fbp_reconstruct_batch(const fbp_job* jobs, int32_t n_jobs, void* d_workspace,
                          size_t workspace_bytes, int32_t precision, void* hip_stream);

/* Workspace bytes fbp_reconstruct_batch needs for these jobs (0 on invalid arguments). */
size_t fbp_batch_workspace_bytes(const fbp_job* jobs, int32_t n_jobs, int32_t precision);

/*
 * Tile-shape autotuning for one geometry: times each compiled backprojection
 * tile shape on synthetic data on `hip_stream` (allocates and frees scratch
 * memory, synchronises the stream), once for one slice and once per slice of a
 * 16-slice stack, and records the fastest of each for this geometry.  Where a
 * chunked quarter-turn shape fits the geometry only its window pitches are
 * timed; they compute the same bits, so tuning then never changes a result.  Later
 * plans of the geometry use them; a plan that already exists keeps its shapes,
 * so results never depend on when tuning ran relative to a call.  With the
 * environment variable FBP_TUNE_CACHE naming a file, the choice is appended to
 * it, and the file's entries apply to plans created afterwards.
 * `out_config` (may be NULL) receives the chosen single-slice tile id.
 */
int fbp_autotune(const fbp_geom* geom, void* hip_stream, int32_t* out_config);

/* Tile id the plan of this geometry uses for single slices (stacks of up to 3),
 * or a negative fbp_status. */
int fbp_plan_config(const fbp_geom* geom);

/* Tile id the plan of this geometry uses for stacks of 4 or more slices, or a
 * negative fbp_status. */
int fbp_plan_stack_config(const fbp_geom* geom);

/*
 * fbp_backproject with an explicit tile id in place of both of the plan's (for
 * tests and tuning).  Different tile ids may differ in the last bits (per-tile
 * FP32 coordinates, angle groups); each is deterministic.
 */
int fbp_backproject_with_config(const fbp_geom* geom, int32_t n_slices, const float* d_filtered,
                                float* d_image, int32_t config, void* hip_stream);

/* Number of compiled backprojection tile shapes and a description of one. */
int32_t fbp_num_tile_configs(void);
const char* fbp_tile_config_name(int32_t id);

/* Static text for a status code (never NULL). */
const char* fbp_status_string(int status);

/* The HIP call behind the calling thread's most recent FBP_EHIP or FBP_ENOMEM,
 * with HIP's error name, e.g. "hipMemcpy (filter taps): hipErrorInvalidValue (1)";
 * "" if there was none.  Thread-local; valid until the thread's next library call
 * that fails.  Never NULL. */
const char* fbp_last_error(void);

/* Library version string. */
const char* fbp_version(void);

/* ------------------------------------------------------------------ cone beam (FDK)
 *
 * Circular cone-beam geometry with a flat detector (the 3D extension of the fan
 * beam; Feldkamp, Davis & Kress 1984; Kak & Slaney 1988, ch. 3): view k has its
 * source at (R cos b_k, R sin b_k, 0); the detector is the plane through the
 * rotation axis perpendicular to the central ray, column i at
 * s_i = (i - (Du-1)/2) du along (-sin b_k, cos b_k, 0), row j at
 * z_j = (j - (Dv-1)/2) dv along z.  Voxel (p, r, c) of the Nz x N x N volume
 * sits at (c - (N-1)/2, r - (N-1)/2, p - (Nz-1)/2) in voxel units.
 * Projections are [K][Dv][Du] (device, FP32), volumes [Nz][N][N].
 */
typedef struct {
    int32_t n_views;          /* K >= 1: source angles, spread over a full turn */
    int32_t n_det_u;          /* Du >= 1 detector columns */
    int32_t n_det_v;          /* Dv >= 1 detector rows */
    int32_t volume_size;      /* N >= 1 */
    int32_t volume_depth;     /* Nz >= 1 */
    int32_t filter;           /* fbp_filter_kind */
    double det_spacing_u;     /* du > 0, finite */
    double det_spacing_v;     /* dv > 0, finite */
    double source_distance;   /* R > N / sqrt(2), finite */
    const double* angles;     /* host array of K finite radians; copied into the plan */
} fbp_cone_geom;

/*
 * FDK steps 1-2: d_filtered[k][j][n] = du * sum_m (h(n-m)/2) * d_proj[k][j][m] R / sqrt(R^2 + s_m^2 + z_j^2)
 * (pre-weight through a scratch buffer owned by the plan, calls ordered on the
 * device; then the FP32 filter GEMM over the K*Dv detector rows).  No overlap.
 */
int fbp_cone_filter(const fbp_cone_geom* geom, const float* d_proj, float* d_filtered, void* hip_stream);

/*
 * FDK step 3: d_volume(X) = (2 pi / K) sum_k (R/L_k)^2 Q~_k(u, v) with bilinear
 * interpolation (zero off the detector), L_k = R - (x cos b_k + y sin b_k),
 * u = R (-x sin b_k + y cos b_k) / (L_k du) + (Du-1)/2, v = R z / (L_k dv) + (Dv-1)/2.
 * Workgroups own 16 x 16 columns x 32 slices, stage detector windows in LDS,
 * sum the views in a fixed order (deterministic, no atomics).  No overlap.
 */
int fbp_cone_backproject(const fbp_cone_geom* geom, const float* d_filtered, float* d_volume,
                         void* hip_stream);

/* fbp_cone_backproject(fbp_cone_filter(d_proj)) with the filtered views in the
 * caller's workspace (fbp_cone_workspace_bytes, 256-byte aligned, no overlap). */
int fbp_cone_reconstruct(const fbp_cone_geom* geom, const float* d_proj, float* d_volume, void* d_workspace,
                         size_t workspace_bytes, void* hip_stream);

/* Workspace bytes fbp_cone_reconstruct needs (0 on invalid arguments). */
size_t fbp_cone_workspace_bytes(const fbp_cone_geom* geom);

#ifdef __cplusplus
}
#endif

#endif /* FBP_H */
