/*
 * gsdf.h -- C ABI of the MI355X (gfx950) Gradient-SDF tracking and fusion
 * library (libgsdf.so).
 *
 * The method is Gradient-SDF (Sommer, Sang, Schubert, Cremers, CVPR 2022):
 * a voxel SDF whose voxels also store an accumulated SDF gradient, fused
 * from depth images (Sec. 3.1 Eq. (1)-(2), Sec. 3.2 Eq. (3)) and used to
 * track the camera with one voxel lookup per pixel through a first-order
 * Taylor expansion (Sec. 4.1 Eq. (5), (14)-(16)), solved by Gauss-Newton
 * with a Cholesky decomposition (Sec. 5.1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every pointer argument named *_dev, and every buffer of gsdf_map, is
 *    DEVICE memory allocated by the caller (the library never allocates or
 *    frees device memory).  Struct arguments (gsdf_camera, *_params,
 *    gsdf_map itself) are HOST memory read during the call only.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls only
 *    enqueue work; none synchronises the stream.  Device buffers must stay
 *    valid until the stream reaches the work.
 *  - Return value: GSDF_OK, or a negative gsdf_status detected on the host
 *    (null pointer, bad size, mismatched storage, launch failure); on such
 *    an error nothing is enqueued.
 *  - Conditions found on the device are OR-ed into *status_dev as the bit
 *    (1u << -code) and are sticky until the caller clears the word.
 *  - Poses are camera-to-world (R, t) as 12 float64, row-major 3x4, kept on
 *    the device: a camera point x maps to R x + t (Eq. (5)).
 *  - Depth images are float32 z-depth in metres, row-major height x width,
 *    with the pixel centre of column u at x = u; a pixel is valid when its
 *    depth is finite and zmin <= D <= zmax (binary32 comparisons).
 *  - Sign: psi > 0 inside objects and < 0 in free space (Sec. 3.1); the
 *    stored gradient points into the object.
 *  - A map is used by one stream at a time.
 */
#ifndef GSDF_H
#define GSDF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GSDF_OK = 0,
    GSDF_EINVAL = -1,     /* bad argument (host); on the device: a non-finite pose, */
                          /* with which the call did no work                        */
    GSDF_ECAPACITY = -2,  /* hash table or block pool full (device): the block is  */
                          /* not allocated and later steps skip its voxels         */
    GSDF_EHIP = -3,       /* a HIP call failed (host), or tracking gave up waiting  */
                          /* for work-groups that never ran (device)                */
    GSDF_ENOTPD = -4,     /* a Gauss-Newton system was not positive definite        */
                          /* (device): that iteration's pose update is skipped      */
    GSDF_ELOST = -5       /* tracking used fewer than min_inlier_frac of the valid  */
                          /* pixels at the finest level (device)                    */
} gsdf_status;

typedef enum {
    GSDF_FP32 = 0,         /* voxel = float4 {sum w d, g_x, g_y, g_z} (16 B) + W   */
    GSDF_BF16 = 1,         /* voxel = 4 x bf16 {psi/T, gbar_x, gbar_y, gbar_z} + W */
    GSDF_FP16 = 2,         /* voxel = 4 x fp16 {psi/T, gbar_x, gbar_y, gbar_z} + W */
    GSDF_NOGRAD_FP32 = 3   /* voxel = float {sum w d} (4 B) + W: a plain SDF map     */
                           /* without gradients (Eq. (1)-(2) only), the baseline of  */
                           /* the paper's runtime comparison (Sec. 5.3); tracked     */
                           /* with GSDF_MODEL_TRILINEAR only, and the calls that     */
                           /* read gradients reject it with GSDF_EINVAL              */
} gsdf_storage;

/* Map geometry and capacity.  The grid is v_j = voxel_size * m_j (Sec. 3.1),
 * stored sparsely as 8^3-voxel blocks found through a hash table. */
typedef struct gsdf_map_desc {
    double voxel_size;    /* metres (float32 band constants are rounded from it) */
    double truncation;    /* T, metres: SDF values are clamped to [-T, T]        */
    int32_t storage;      /* gsdf_storage                                        */
    int32_t reserved0;
    int64_t hash_slots;   /* power of two, >= 2 * max_blocks recommended         */
    int64_t max_blocks;   /* block pool capacity, <= 2^24                        */
    int32_t bounded;      /* 1: only blocks b with bmin <= b < bmax are allocated */
    int32_t bmin[3];
    int32_t bmax[3];
    int32_t reserved1;
} gsdf_map_desc;

/* Per-kernel event timer (host object owned by the caller, see
 * gsdf_timer_create); NULL in gsdf_map.timer means no timing. */
typedef struct gsdf_timer gsdf_timer;

/* The four caller-allocated device buffers of a map (sizes from
 * gsdf_map_buffer_sizes).  Layout inside them is private to the library.
 * The library keeps no state of its own between calls: everything a map
 * needs lives in these buffers and in this struct. */
typedef struct gsdf_map {
    void* hash;     /* hash table                                             */
    void* vox;      /* voxel records, max_blocks * 512                          */
    void* weight;   /* float32 accumulated weight W per voxel, max_blocks * 512 */
    void* aux;      /* block keys, counters, per-frame accumulators and lists   */
    gsdf_map_desc desc;
    gsdf_timer* timer;  /* optional: launches on this map record events in it   */
} gsdf_map;

/* Pinhole camera (Sec. 4.1 back-projection x = D [(u-cx)/fx, (v-cy)/fy, 1]). */
typedef struct gsdf_camera {
    double fx, fy, cx, cy;
    int32_t width, height;
    float zmin, zmax;     /* valid depth range, metres */
} gsdf_camera;

/* Fusion parameters (Sec. 5.3 setup). */
typedef struct gsdf_fuse_params {
    float eps_weight;     /* linear weight: w(d) = 1 for d <= eps, (T-d)/(T-eps)  */
                          /* for eps < d < T, 0 for d >= T                        */
    float cos_max_angle;  /* integrate pixels whose normal/ray angle cosine is at */
                          /* least this (cos 75 deg in the paper)                 */
} gsdf_fuse_params;

/* Tracking parameters (Sec. 4.1, Sec. 5.1). */
typedef struct gsdf_track_params {
    int32_t levels;          /* pyramid levels, 1..4                              */
    int32_t iters[4];        /* Gauss-Newton iterations per level, iters[0] is    */
                             /* the finest level; levels run coarse to fine       */
    float huber_delta;       /* Huber threshold delta (metres)                    */
    double damping;          /* mu = damping * trace(H) / 6 added to H's diagonal */
    float min_inlier_frac;   /* GSDF_ELOST below this fraction at the finest level */
    int32_t model;           /* gsdf_residual_model                               */
    int32_t max_polls;       /* bound on the polls of each wait between work-     */
                             /* groups before the frame is given up with          */
                             /* GSDF_EHIP; 0 = the library default (2^20 for the  */
                             /* per-iteration sums, 2^24 for a level boundary)    */
    uint64_t* iter_clocks;   /* optional (device, 4 per iteration in execution    */
                             /* order): ticks of the device wall clock since the  */
                             /* launch started, as work-group 0 sees them after   */
                             /* its pixel sums, after its part of the exchange    */
                             /* (its partial stored, and for a leaf leader the    */
                             /* leaf sum too), after the total, after the solve;  */
                             /* rate from gsdf_wall_clock_khz.  NULL: not taken   */
    int32_t exchange_device_scope; /* nonzero: every per-iteration partial sum   */
                             /* goes through device-scope memory instead of the   */
                             /* L2 of the XCD its leaf shares (the same sums in   */
                             /* the same order, so the same pose bits; slower).   */
                             /* 0 is the normal setting                           */
} gsdf_track_params;

/* Residual model of tracking (Sec. 4.1). */
typedef enum gsdf_residual_model {
    GSDF_MODEL_TAYLOR = 0,     /* Eq. (14)-(16): one voxel, psi + g^ . (q - v)     */
    GSDF_MODEL_TRILINEAR = 1   /* Eq. (12)-(13): tri-linear interpolant of the 8   */
                               /* voxels around q and its derivative (the direct   */
                               /* SDF tracking the paper compares against; needs   */
                               /* all eight observed)                              */
} gsdf_residual_model;

/* ---------------------------------------------------------------------- */
/* Map buffers                                                             */
/* ---------------------------------------------------------------------- */

/* Byte sizes of the four map buffers for `desc` (host only, no GPU work).
 * sizes_out[0..3] = hash, vox, weight, aux.  Returns GSDF_EINVAL for a
 * hash_slots that is not a power of two, a non-positive capacity, a
 * voxel_size <= 0 or truncation < voxel_size. */
int gsdf_map_buffer_sizes(const gsdf_map_desc* desc, size_t sizes_out[4]);

/* Clear a map to empty (all hash slots free, all voxels zero). */
int gsdf_map_reset(gsdf_map* map, void* stream);

/* Number of allocated blocks, written to *n_dev (int32, device). */
int gsdf_map_num_blocks(const gsdf_map* map, int32_t* n_dev, void* stream);

/* ---------------------------------------------------------------------- */
/* The per-frame hot path                                                  */
/* ---------------------------------------------------------------------- */

/* allocate_blocks (Sec. 5.3 setup: fusion is driven by depth pixels, each
 * touching the voxels its viewing ray crosses inside the truncation band;
 * 8^3 blocks as in Sec. 3.1): insert into the map every block that holds a
 * voxel of a valid pixel's ray band.  The band is sampled at z_k = (D - T) + k v_s/2,
 * k = 0 .. 4T/v_s, each sample is mapped to its voxel floor(q / v_s + 1/2)
 * and the voxel to its block floor(m / 8), all in binary32 with a fixed
 * operation order, so the allocated key set is reproducible bit for bit.
 * The blocks found (new or old) are also recorded as the frame's touched
 * set, which the next gsdf_integrate_frame consumes; call the two in pairs
 * with the same depth, camera and pose.
 * T_wc_dev: 12 float64 (device).  A full table or pool sets GSDF_ECAPACITY. */
int gsdf_allocate_blocks(gsdf_map* map, const float* depth_dev, const gsdf_camera* cam,
                         const double* T_wc_dev, int32_t* status_dev, void* stream);

/* Scratch bytes gsdf_integrate_frame needs for `cam` (one float4 per pixel). */
size_t gsdf_integrate_scratch_bytes(const gsdf_camera* cam);

/* integrate_frame (Eq. (1)-(3)): for every valid pixel whose 5x5 normal fit
 * succeeds and whose normal/ray angle passes the filter, every voxel of its
 * ray band (as in gsdf_allocate_blocks) in an allocated block receives
 * d = clamp(n_w . (v - p), -T, T) with weight w(d); per voxel,
 * psi <- (W psi + sum w d) / (W + sum w), g <- g + sum w n_w, W <- W + sum w.
 * Blocks must have been allocated for this frame first. */
int gsdf_integrate_frame(gsdf_map* map, const float* depth_dev, const gsdf_camera* cam,
                         const double* T_wc_dev, const gsdf_fuse_params* params,
                         void* scratch_dev, size_t scratch_bytes, int32_t* status_dev,
                         void* stream);

/* allocate_blocks followed by integrate_frame for one frame (Sec. 5.3),
 * with the same results as the two calls in sequence, in two launches: the
 * allocation of each 16x16 pixel tile and the tile's normal fits share one
 * launch (neither reads what the other writes), then the per-block fusion.
 * Arguments as for gsdf_integrate_frame (scratch_dev: at least
 * gsdf_integrate_scratch_bytes(cam) bytes). */
int gsdf_fuse_frame(gsdf_map* map, const float* depth_dev, const gsdf_camera* cam, const double* T_wc_dev,
                    const gsdf_fuse_params* params, void* scratch_dev, size_t scratch_bytes,
                    int32_t* status_dev, void* stream);

/* Host call: rate of the device wall clock that iter_clocks counts, in kHz
 * (100000 on MI355X), for the current device. */
int gsdf_wall_clock_khz(int32_t* khz_out);

/* Scratch bytes gsdf_track_frame / gsdf_normal_equations need for `cam`. */
size_t gsdf_track_scratch_bytes(const gsdf_camera* cam, int32_t levels);

/* track_frame (Sec. 4.1 Eq. (5), (14)-(16); Sec. 5.1): coarse-to-fine
 * Gauss-Newton on E = sum_k rho_delta(r_k), r_k = psi_j + g^_j . (T x_k - v_j)
 * with j the voxel nearest to T x_k, Jacobian [g^ ; (T x) x g^] for a left
 * perturbation in the world frame, and a damped 6x6 Cholesky solve (its
 * square-root-free LDL^T form) in float64 on the device; T <- exp(dxi) T.
 * T_init_dev (device, 12 f64) holds
 * the initial pose and T_wc_out_dev (device, 12 f64) receives the estimate;
 * they may be the same buffer.  stats_dev (device, optional) receives 2
 * floats per iteration in execution order: the energy and the number of
 * pixels used at that linearisation.  scratch_dev must hold
 * gsdf_track_scratch_bytes(cam, levels) bytes; its contents on entry do not
 * matter (the call clears what it needs before its iterations), and calls
 * that may overlap in time (on different streams) need separate scratch.
 * The launch needs every one of its work-groups resident at once (one per
 * compute unit); every wait in it is bounded (params->max_polls), so a
 * device too busy to hold them fails the frame with GSDF_EHIP in
 * *status_dev rather than hanging; the estimate is then undefined.  A
 * non-finite initial pose runs no iteration: the estimate is the initial
 * pose and GSDF_EINVAL is raised.  GSDF_ENOTPD: some iteration's system was
 * not positive definite (its update skipped); GSDF_ELOST: fewer than
 * min_inlier_frac of the valid finest-level pixels found an observed voxel
 * at the last linearisation. */
int gsdf_track_frame(const gsdf_map* map, const float* depth_dev, const gsdf_camera* cam,
                     const gsdf_track_params* params, const double* T_init_dev, double* T_wc_out_dev,
                     float* stats_dev, void* scratch_dev, size_t scratch_bytes, int32_t* status_dev, void* stream);

/* gsdf_track_frame without a scratch argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation).  Its scratch is a fixed array
 * of gsdf_track_noalloc_max_bytes() bytes in the library's device memory,
 * one per GPU, held until the process ends; a camera whose
 * gsdf_track_scratch_bytes(cam, levels) exceeds it is rejected with
 * GSDF_EINVAL.  Every call on one GPU shares that GPU's array (the call
 * clears what it needs first), so calls that may overlap in time on one
 * GPU (on different streams) race and must not be issued.  Other arguments,
 * results and status as for gsdf_track_frame. */
size_t gsdf_track_noalloc_max_bytes(void);
int gsdf_track_frame_noalloc(const gsdf_map* map, const float* depth_dev, const gsdf_camera* cam,
                             const gsdf_track_params* params, const double* T_init_dev, double* T_wc_out_dev,
                             float* stats_dev, int32_t* status_dev, void* stream);

/* One linearisation of the tracking energy at T_wc_dev on the full-resolution
 * image (Eq. (5), (14)-(16)): out29_dev (device, 29 float64) = the 21 upper-
 * triangular entries of H = sum w J J^T (row-major), the 6 of b = sum w J r,
 * the energy sum rho_delta(r) and the number of pixels used. */
int gsdf_normal_equations(const gsdf_map* map, const float* depth_dev, const gsdf_camera* cam,
                          const double* T_wc_dev, float huber_delta, double* out29_dev,
                          void* scratch_dev, size_t scratch_bytes, void* stream);

/* One damped Gauss-Newton step of the tracking energy (Sec. 4.1 Eq. (5),
 * (14)-(16); Sec. 5.1) at full resolution for each of n_keyframes keyframes
 * on the current map, as joint refinement takes it once per step: for
 * keyframe i, with depth depth_dev + i*H*W (K x H x W float32, device) and
 * pose T_dev + 12 i (K x 12 float64, row-major 3x4 camera-to-world,
 * device, updated in place), the step gsdf_track_frame takes with one level
 * and one iteration (Huber threshold huber_delta, mu = damping * trace(H)/6
 * added to H's diagonal, left SE(3) update), in two launches for all
 * keyframes.  The normal equations are summed in another fixed order than
 * gsdf_track_frame's, so the poses agree with K such calls to rounding, and
 * are the same bits on every run.  Sticky bits in *status_dev:
 * GSDF_ENOTPD when a keyframe's system is not positive definite (its pose
 * unchanged), GSDF_ELOST when fewer than min_inlier_frac of a keyframe's
 * valid pixels found an observed voxel, GSDF_EINVAL for a non-finite pose
 * (left unchanged).  scratch_dev: at least gsdf_gn_scratch_bytes(cam, K)
 * bytes (contents on entry do not matter).  Returns GSDF_EINVAL for bad
 * sizes, null buffers, huber_delta <= 0, damping < 0, K outside
 * 1..65535 or a map without gradients. */
size_t gsdf_gn_scratch_bytes(const gsdf_camera* cam, int32_t n_keyframes);
int gsdf_gn_step_keyframes(const gsdf_map* map, const float* depth_dev, int32_t n_keyframes,
                           const gsdf_camera* cam, double* T_dev, float huber_delta, double damping,
                           float min_inlier_frac, void* scratch_dev, size_t scratch_bytes,
                           int32_t* status_dev, void* stream);

/* ---------------------------------------------------------------------- */
/* Differentiable form: keyframe loss and its adjoint                      */
/* ---------------------------------------------------------------------- */

/* Per-voxel parameters: `params` is a float32 buffer of param_blocks x 512
 * float4 {psi, g_x, g_y, g_z} indexed by pool slot, voxel (lx, ly, lz) of a
 * block at Morton index gsdf_voxel_order()[lx + 8 ly + 64 lz].  g is the
 * map's stored gradient (the accumulated gradient of Eq. (3) for FP32
 * storage, its weighted mean for BF16/FP16); only its direction enters the
 * residual.  Slots >= param_blocks count as unobserved. */

/* Copy the map's voxels into params (psi = sum w d / W for FP32 storage);
 * rows beyond the map's block count are zero.  params_dev holds
 * param_blocks x 512 x 4 float32 (device). */
int gsdf_export_params(const gsdf_map* map, float* params_dev, int64_t param_blocks, void* stream);

/* Write params back into the map's observed voxels (W > 0), keeping W
 * (for BF16/FP16 storage psi/T and g are rounded to the format). */
int gsdf_import_params(gsdf_map* map, const float* params_dev, int64_t param_blocks, void* stream);

/* Host call: order_out[lx + 8 ly + 64 lz] = that voxel's index inside its
 * block in the map's (and the params') layout. */
int gsdf_voxel_order(int32_t order_out[512]);

/* T_out[i] = exp(xi_i^) T0[i] for i < n (Sec. 5.1 left pose update):
 * T0_dev, T_out_dev n x 12 float64, xi_dev n x 6 float64 (device); T_out
 * may alias T0. */
int gsdf_compose_poses(int32_t n, const double* T0_dev, const double* xi_dev, double* T_out_dev,
                       void* stream);

/* Scratch bytes of gsdf_keyframe_loss / gsdf_backward for K keyframes and
 * a parameter buffer of param_blocks rows (scratch sized for the map's
 * max_blocks serves every param_blocks).  0 when the arguments are invalid
 * or K x W x H exceeds INT32_MAX (pixels are numbered in int32). */
size_t gsdf_keyframe_scratch_bytes(const gsdf_camera* cam, int32_t n_keyframes, int64_t param_blocks);

/* Keyframe loss (Sec. 4.1 Eq. (5), (14); Huber penalty of Sec. 5.1): for
 * each keyframe i, L_i = sum over its valid pixels of rho_delta(r) with
 * r = psi_j + g^_j . (q - v_j), q = T_i x, T_i = exp(xi_i^) T0_i, j the voxel
 * nearest to q, (psi_j, g_j) read from params, and pixels whose voxel is
 * absent, unobserved (W = 0) or has g = 0 skipped.
 *   depth_dev: K x H x W float32 (device), 0 = invalid;
 *   T0_dev: K x 12 float64 (device), row-major 3x4 camera-to-world;
 *   xi_dev: K x 6 float64 (device), twist (translation, rotation) of the
 *     left increment;
 *   assoc_dev (optional): K x H x W x 3 int32 voxel coordinates: freeze = 0
 *     writes each pixel's nearest voxel (INT32_MIN when unused), freeze = 1
 *     reads them instead of searching (for finite differences);
 *   loss_dev: K float64 (device); count_dev (optional): K float64 pixels used.
 * Errors: GSDF_EINVAL for bad sizes, null buffers, freeze without assoc or
 * scratch smaller than gsdf_keyframe_scratch_bytes(cam, K, param_blocks). */
int gsdf_keyframe_loss(const gsdf_map* map, const float* depth_dev, int32_t n_keyframes,
                       const gsdf_camera* cam, const double* T0_dev, const double* xi_dev,
                       const float* params_dev, int64_t param_blocks, float huber_delta,
                       int32_t* assoc_dev, int32_t freeze, double* loss_dev, double* count_dev,
                       void* scratch_dev, size_t scratch_bytes, void* stream);

/* backward: the adjoint of gsdf_keyframe_loss (the differentiable form of
 * the tracking energy of Sec. 4.1 Eq. (5), (14); g^ is differentiated
 * through its normalisation, the association of pixel to voxel is held
 * fixed as in Sec. 4.2), recomputing every residual (nothing per pixel is
 * stored between the two calls).  With s_i = grad_loss_dev[i]
 * (K float32, device), rho' the Huber derivative and g^ = g/|g|:
 *   dparams[j] += sum s_i rho'(r) {1, (I - g^ g^T)(q - v_j) / |g_j|}
 *     (added to what dparams_dev holds: clear it first),
 *   dxi_dev[i] = Jl(xi_i)^T sum_k s_i rho'(r_k) [g^ ; q x g^]
 *     (K x 6 float64, overwritten; Jl the left Jacobian of SE(3)),
 *   loss_dev (optional) as gsdf_keyframe_loss.
 * The voxel sums are exact (fixed point) and each voxel is written by one
 * thread; the keyframe sums are reduced in a fixed order; so the results
 * are the same bits on every run.  freeze = 1 reads
 * the association from assoc_dev; with freeze = 0 each pixel's nearest
 * voxel is used and assoc_dev is neither read nor written (the loss call
 * writes it).  Other argument rules as for gsdf_keyframe_loss. */
int gsdf_backward(const gsdf_map* map, const float* depth_dev, int32_t n_keyframes,
                  const gsdf_camera* cam, const double* T0_dev, const double* xi_dev,
                  const float* params_dev, int64_t param_blocks, float huber_delta,
                  int32_t* assoc_dev, int32_t freeze, const float* grad_loss_dev,
                  float* dparams_dev, double* dxi_dev, double* loss_dev,
                  void* scratch_dev, size_t scratch_bytes, void* stream);

/* ---------------------------------------------------------------------- */
/* Photometric term (joint refinement with colour)                         */
/* ---------------------------------------------------------------------- */

/* Surface point of voxel j (Sec. 4.2 Eq. (18)): p_j = v_j - psi_j g^_j with
 * g^_j = g_j/|g_j| held fixed while psi_j changes; voxels with W > 0, g != 0
 * whose cell contains p_j (max_k |psi_j g^_jk| <= v_s/2) take part.
 * Keyframe i sees p_j when x = R_i^T (p_j - t_i) has z >= zmin, projects
 * inside [0, width-1) x [0, height-1), the nearest pixel's depth D is valid
 * with |z - D| <= T, and g^_j . (p_j - t_i) > 0.  rgb_dev: K x H x W x 3
 * float32 colour (device), sampled bilinearly.  colors: param_blocks x 512
 * x 3 float32 per-voxel colour rho_j in the params' slot/voxel order.
 * T_i = exp(xi_i^) T0_i as for gsdf_keyframe_loss. */

/* Scratch bytes of the photometric calls. */
size_t gsdf_photometric_scratch_bytes(int64_t param_blocks, int32_t n_keyframes);

/* L_i = weight * sum_{j seen by i} sum_c huber_delta(I_i^c(pi(x)) - rho_j^c)
 * into loss_dev (K float64); count_dev (optional, K float64): (voxel,
 * keyframe) pairs seen. */
int gsdf_photometric_loss(const gsdf_map* map, const float* depth_dev, const float* rgb_dev,
                          int32_t n_keyframes, const gsdf_camera* cam, const double* T0_dev,
                          const double* xi_dev, const float* params_dev, const float* colors_dev,
                          int64_t param_blocks, float huber_delta, float weight, double* loss_dev,
                          double* count_dev, void* scratch_dev, size_t scratch_bytes, void* stream);

/* Adjoint of gsdf_photometric_loss, recomputing every sample; with
 * s_i = grad_loss_dev[i]: dparams[j].psi += sum_i s_i dL_i/dpsi_j (g^ held
 * fixed, so the g components get nothing), dcolors[j] += sum_i s_i
 * dL_i/drho_j, dxi_dev[i] = Jl(xi_i)^T (left-increment gradient of s_i L_i)
 * (overwritten); loss_dev optional.  Each voxel's entries are written by
 * one thread (no atomics); call after, not concurrently with, other writers
 * of dparams. */
int gsdf_photometric_backward(const gsdf_map* map, const float* depth_dev, const float* rgb_dev,
                              int32_t n_keyframes, const gsdf_camera* cam, const double* T0_dev,
                              const double* xi_dev, const float* params_dev, const float* colors_dev,
                              int64_t param_blocks, float huber_delta, float weight,
                              const float* grad_loss_dev, float* dparams_dev, float* dcolors_dev,
                              double* dxi_dev, double* loss_dev, void* scratch_dev,
                              size_t scratch_bytes, void* stream);

/* Mean colour of each taking-part voxel over the keyframes that see it
 * (Sec. 4.2 Eq. (21)): colors_out_dev (param_blocks x 512 x 3 float32, 0
 * where no keyframe sees the voxel) and count_out_dev (optional,
 * param_blocks x 512 float32, N_j). */
int gsdf_mean_color(const gsdf_map* map, const float* depth_dev, const float* rgb_dev, int32_t n_keyframes,
                    const gsdf_camera* cam, const double* T0_dev, const double* xi_dev,
                    const float* params_dev, int64_t param_blocks, float* colors_out_dev,
                    float* count_out_dev, void* scratch_dev, size_t scratch_bytes, void* stream);

/* Adjoint of gsdf_mean_color (Sec. 4.2 Eq. (21) differentiated, g^ held
 * fixed): given the upstream gradient G_j of the mean colours
 * (grad_colors_dev, param_blocks x 512 x 3) and the view counts N_j of the
 * forward call (counts_dev, param_blocks x 512), each view (i, j) adds
 * (G_j / N_j) . dI_ij: to dparams[j].psi (+=, one writer per voxel) and to
 * dxi_dev[i] (K x 6 float64, overwritten, through Jl(xi_i)^T).  Composed
 * with gsdf_photometric_backward at the mean colours this gives the
 * gradient of the coupled bundle-adjustment energy of Sec. 4.2 Eq. (17). */
int gsdf_mean_color_backward(const gsdf_map* map, const float* depth_dev, const float* rgb_dev,
                             int32_t n_keyframes, const gsdf_camera* cam, const double* T0_dev,
                             const double* xi_dev, const float* params_dev, int64_t param_blocks,
                             const float* grad_colors_dev, const float* counts_dev, float* dparams_dev,
                             double* dxi_dev, void* scratch_dev, size_t scratch_bytes, void* stream);

/* Regulariser of the bundle adjustment (Sec. 5 experiments): loss_dev (one
 * float64) = weight * sum over observed voxels of (psi_j - psi0_j)^2, with
 * params and params0 as for gsdf_export_params; dparams_dev (optional) gets
 * 2 weight (psi_j - psi0_j) added to its psi entries.  scratch_dev holds at
 * least param_blocks float64. */
int gsdf_psi_regulariser(const gsdf_map* map, const float* params_dev, const float* params0_dev,
                         int64_t param_blocks, float weight, double* loss_dev, float* dparams_dev,
                         void* scratch_dev, size_t scratch_bytes, void* stream);

/* ---------------------------------------------------------------------- */
/* Surface extraction                                                       */
/* ---------------------------------------------------------------------- */

/* Scratch bytes of gsdf_extract_surfels for this map. */
size_t gsdf_surfel_scratch_bytes(const gsdf_map* map);

/* Oriented point cloud (Sec. 4.3): every observed voxel whose surface point
 * v - psi g^ lies in its cell (|psi g^_k| <= v_s/2 for each axis) gives that
 * point with normal -g^ (level 0); level 1 splits each voxel into 2x2x2
 * subvoxels, takes their distance from the Taylor expansion
 * psi + g^ . (s - v) and keeps those with |psi(s) g^_k| <= v_s/4.  Order:
 * block slot, voxel lx + 8 ly + 64 lz, subvoxel sx + 2 sy + 4 sz.  Writes
 * min(count, capacity) surfels: points_dev / normals_dev (n x 3 float32),
 * ids_dev (n x 4 int32: voxel coordinates and subvoxel), and the full count
 * to *count_dev (int64, device); capacity 0 only counts. */
int gsdf_extract_surfels(const gsdf_map* map, int32_t level, float* points_dev, float* normals_dev,
                         int32_t* ids_dev, int64_t capacity, int64_t* count_dev, void* scratch_dev,
                         size_t scratch_bytes, void* stream);

/* Gradient quality against a known union of spheres (Sec. 5.2, App. A).
 * spheres_dev: n_spheres x (cx, cy, cz, r) float64, device, 1 <= n_spheres
 * <= 64.  Per observed voxel (W > 0, g != 0) the nearest sphere surface
 * minimises | |v - c| - r | and the true gradient of the distance is
 * (c - v)/|c - v|.  out_dev (device, float32) receives 5 planes of `stride`
 * values at index slot * 512 + lx + 8 ly + 64 lz: [0] distance to that
 * surface, [1] angle (degrees) of the stored gradient, [2]-[4] angles of the
 * forward, backward and central differences of the stored distance (step
 * v_s; they need the six face neighbours observed); NaN where undefined.
 * Blocks with slot >= stride / 512 are skipped; stride must be a multiple of
 * 512.  GSDF_EINVAL on bad arguments. */
int gsdf_gradient_quality(const gsdf_map* map, const double* spheres_dev, int32_t n_spheres, float* out_dev,
                          int64_t stride, void* stream);

/* ---------------------------------------------------------------------- */
/* Inspection, import (used for parity checks and checkpoints)             */
/* ---------------------------------------------------------------------- */

/* Block keys in pool-slot order: keys_out_dev (device, max_blocks x 3 int32)
 * and their count in *n_dev (int32, device).  Row i is the block whose
 * voxels are row i of gsdf_export_voxels and of gsdf_export_params, so the
 * order pairs keys with values; a caller that wants the keys as a set sorts
 * them (the parity tests compare sorted (x, y, z) triples). */
int gsdf_export_keys(const gsdf_map* map, int32_t* keys_out_dev, int32_t* n_dev, void* stream);

/* Work counters accumulated since the last reset (device, 16 uint64):
 * [0] fusion updates applied, [1] (block, pixel) visits of the fusion
 * gather, [2] voxels written by fusion, [3] blocks processed by fusion,
 * [4] distinct (16x16 tile, block) pairs probed by allocation, [5] valid pixel-iterations
 * of tracking, [6] tracking pixel-iterations that found an observed voxel. */
int gsdf_map_counters(const gsdf_map* map, uint64_t* out_dev, void* stream);

/* Voxel values of pool slots [0, n_blocks): psi (n x 512), g (n x 512 x 3:
 * the accumulated gradient of Eq. (3) for FP32 storage, the weighted-mean
 * gradient g/W for BF16/FP16), W (n x 512), all float32, device.  Voxel order
 * within a block is lx + 8 ly + 64 lz. */
int gsdf_export_voxels(const gsdf_map* map, int32_t n_blocks, float* psi_dev, float* g_dev,
                       float* w_dev, void* stream);

/* Insert n blocks with the given keys (device, n x 3 int32) and set their
 * voxels from psi/g/W (device float32, layouts as gsdf_export_voxels). */
int gsdf_import_blocks(gsdf_map* map, const int32_t* keys_dev, int32_t n, const float* psi_dev,
                       const float* g_dev, const float* w_dev, int32_t* status_dev, void* stream);

/* ---------------------------------------------------------------------- */
/* Timing of individual kernels (host bookkeeping with HIP events)        */
/* ---------------------------------------------------------------------- */

/* Kernel identifiers for gsdf_timing_read. */
enum {
    GSDF_K_ALLOCATE = 0,
    GSDF_K_INTEGRATE = 1,
    GSDF_K_TRACK = 2,
    GSDF_K_PYRAMID = 3,
    GSDF_K_NORMALS = 4,
    GSDF_K_BACKWARD = 5,
    GSDF_K_LOSS = 6,
    GSDF_K_PHOTOMETRIC = 7,
    GSDF_K_ALLOC_NORMALS = 8,
    GSDF_K_COUNT = 16
};

/* Create a timer that records HIP events around the launches of the kernel
 * ids whose bits are set in `mask` (two events per timed launch, on the
 * launch's stream).  Attach it to a map by setting gsdf_map.timer; the
 * caller owns it and destroys it after the last timed launch completed. */
int gsdf_timer_create(uint32_t mask, gsdf_timer** timer_out);
int gsdf_timer_destroy(gsdf_timer* timer);

/* Select the timed kernel ids (0 = none) and clear the accumulated totals. */
int gsdf_timer_select(gsdf_timer* timer, uint32_t mask);

/* Total milliseconds and launch count recorded for one kernel id since the
 * last select; synchronises the recorded events. */
int gsdf_timer_read(gsdf_timer* timer, int32_t kernel_id, double* total_ms, int64_t* launches);

const char* gsdf_status_string(int32_t code);

#ifdef __cplusplus
}
#endif

#endif /* GSDF_H */
