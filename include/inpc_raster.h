/*
 * inpc_raster.h -- C ABI of the MI355X (gfx950) point rasterizer of
 * "A Bag of Tricks for Efficient Implicit Neural Point Clouds".
 *
 * What is computed (paper, Sec. 2 "Rendering Feature Maps", Sec. 3.2 and
 * Appendix A): a point cloud with positions p_i, opacities o_i and feature
 * vectors f_i is projected into a pinhole camera; every point becomes a
 * bilinear 2x2 splat (weights summing to one) or, at inference, a small
 * isotropic screen-space Gaussian (dilation variance 0.16, cut at 3 sigma);
 * the fragments of every pixel are alpha-blended front to back in depth
 * order (Eq. (1)) and composited with a background; the backward pass
 * returns the exact gradients of Eq. (1), including zero-alpha fragments
 * (Eq. (2) and the surrounding text).  The screen is cut into square tiles
 * (Sec. 3.2 "Tiled Rendering"); each tile gets the list of points whose
 * footprint meets it, ordered by (depth key, point index).
 *
 * Conventions for every entry point
 *  - Array arguments are DEVICE pointers owned by the caller unless stated
 *    otherwise.  The library never allocates or frees device memory and
 *    keeps no device state between calls; the only scratch memory it uses
 *    is the caller's workspace `ws` of at least inpc_workspace_bytes().
 *  - Every call is asynchronous on `stream` (a hipStream_t passed as void*,
 *    NULL = the null stream) and never synchronises, except
 *    inpc_check_sync().
 *  - Host-side argument checks run before any launch and return
 *    INPC_ERR_INVALID (null pointer, n < 0, tile not 8/16/32, channels
 *    outside [1, 64], non-positive image size, tile count not fitting 32
 *    bits, workspace too small for n).  Launch failures return INPC_ERR_HIP;
 *    inpc_last_error() then holds a message for the calling thread.
 *  - Data-dependent capacity overflow (more tile copies than the workspace
 *    holds, e.g. Gaussians larger than opts.max_radius) cannot be seen on
 *    the host without a sync: the kernels set a flag in the workspace and
 *    skip their work, leaving every output undefined; inpc_check_sync()
 *    reports it as INPC_ERR_CAPACITY.  The flag is sticky: later builds on
 *    the same workspace skip their work too until inpc_check_sync() has
 *    reported (and cleared) it.  A new workspace must therefore start
 *    zeroed (at least its first 64 bytes).
 *  - Alignment: the workspace, proj, feat, grad_feat and the backward
 *    scratch are read or written as 16-byte vectors and must be 16-byte
 *    aligned, grad_uv 8-byte aligned (INPC_ERR_INVALID otherwise).
 *  - Discrete decisions (culling, footprints, tile membership, sort keys)
 *    use IEEE FP32 with one rounding per operation and no fused
 *    multiply-add, so they are reproducible bit for bit.
 *  - Layouts: positions [n][3], projection records [n][4], features [n][C]
 *    (row per point), images planar [C][H][W], per-pixel planes [H][W].
 */
#ifndef INPC_RASTER_H
#define INPC_RASTER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t inpc_status_t;
enum {
    INPC_OK = 0,
    INPC_ERR_INVALID = -1,     /* bad argument, detected on the host before any launch */
    INPC_ERR_CAPACITY = -2,    /* workspace copy capacity exceeded (reported by inpc_check_sync) */
    INPC_ERR_HIP = -3,         /* a HIP runtime call failed; see inpc_last_error() */
    INPC_ERR_UNSUPPORTED = -4  /* valid but not implemented combination */
};

/* Splat kinds (Sec. 3.2): bilinear 2x2 splats (training), isotropic
 * screen-space Gaussians of a per-point radius, and isotropic world-space
 * Gaussians of one standard deviation ewa_sigma projected with the affine
 * (EWA) approximation of the perspective map ("Rendering Points as Small
 * Gaussians"). */
enum { INPC_SPLAT_BILINEAR = 0, INPC_SPLAT_GAUSSIAN = 1, INPC_SPLAT_EWA = 2 };
enum { INPC_F32 = 0, INPC_F16 = 1, INPC_BF16 = 2 };

/* Pinhole camera, OpenCV axes (+z forward, +y down).  A world point p goes
 * to camera space as X = R p + t (R row-major), then u = fx X/Z + cx,
 * v = fy Y/Z + cy.  Pixel (x, y) covers [x, x+1) x [y, y+1).  Points with
 * Z <= z_near (or NaN) are culled. */
typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
    float R[9];
    float t[3];
    float z_near;
} inpc_camera_t;

typedef struct {
    int32_t splat;      /* INPC_SPLAT_BILINEAR, INPC_SPLAT_GAUSSIAN or INPC_SPLAT_EWA */
    int32_t tile;       /* tile edge in pixels: 8, 16 or 32 (Sec. 3.2 uses 8) */
    float t_min;        /* fragment k is blended iff the transmittance in front of it is >= t_min;
                           0 blends every fragment (exact Eq. (1)); typical 1e-4 */
    float dilation;     /* Gaussians: variance added to the projected covariance (paper: 0.16) */
    float cutoff;       /* Gaussians: truncation in standard deviations (paper: 3) */
    float max_radius;   /* Gaussians: largest projected standard deviation in pixels, before
                           dilation, of any point (screen-space: radius; world-space: the
                           square root of the larger diagonal entry of sigma^2 J J^T); sizes
                           the workspace */
    int32_t bin_points; /* points per workgroup of the counting and scatter passes of steps 1-2:
                           0 = automatic (8192, or n/256 when larger), else a multiple of
                           1024; never fewer than n/256 (a tuning knob: results do not
                           depend on it; the workspace size does) */
    int32_t bg_per_pixel; /* 0: the blend's background `bg` (and grad_bg) is one [C] vector;
                             1: a per-pixel image [C][H][W] (e.g. from inpc_envmap_forward),
                             and grad_bg is [C][H][W] as well */
    float ewa_sigma;    /* INPC_SPLAT_EWA: world-space standard deviation of every point
                           (finite, > 0); projected covariance sigma^2 J J^T + dilation I with
                           J the Jacobian of the perspective map at the point.  The paper's
                           default makes a point at the near plane that projects to the image
                           centre 5 px wide: sigma = 5 z_near / max(fx, fy).  Ignored for the
                           other splats. */
} inpc_opts_t;

/* Bytes of workspace needed for n points with this camera and options.
 * Worst case, no sync: bilinear splats make at most 4 tile copies per point,
 * Gaussians at most the tile count of a (2 R + 1)^2 box with R from
 * max_radius.  Returns 0 for invalid arguments. */
size_t inpc_workspace_bytes(int64_t n, const inpc_camera_t* cam, const inpc_opts_t* opts);

/* Bytes of the forward state the backward pass reads: 12 per pixel (how far
 * down its tile list the pixel blended, and the transmittance in front of
 * its last blended fragment with nonzero transmittance) plus 4 per tile.
 * 0 if invalid. */
size_t inpc_state_bytes(const inpc_camera_t* cam, const inpc_opts_t* opts);

/* Number of tiles, ceil(W/T) * ceil(H/T); tile t covers columns
 * [T (t mod ntx), ...) and rows [T (t div ntx), ...).  0 if invalid. */
int64_t inpc_num_tiles(const inpc_camera_t* cam, const inpc_opts_t* opts);

/*
 * Step 1 -- project, cull, key (Sec. 2: points rasterized into a calibrated
 * camera; Sec. 3.2: 32-bit depth keys).
 *   pos      [n][3] f32 world positions
 *   opacity  [n] f32 in [0, 1]
 *   radius   [n] f32 screen-space Gaussian standard deviation in pixels
 *            (before dilation); NULL for bilinear and world-space splats
 *   proj     [n][4] f32 out, 16-byte aligned: per point (u, v, opacity,
 *            w) with w the radius (screen-space Gaussians), the camera-space
 *            depth Z (world-space Gaussians: the projected covariance is a
 *            function of u, v and Z) or 0, the image coordinates next to
 *            what the blend
 *            passes read with them, so that one 16-byte load fetches all of
 *            a point's footprint data
 *   depth_key[n] u32 out: bit pattern of camera-space Z (monotone in Z > 0)
 *   ntiles   [n] u32 out: tiles the footprint meets, 0 for culled points
 * Also counts copies per tile into the workspace for step 2.
 */
inpc_status_t inpc_project(const inpc_camera_t* cam, const inpc_opts_t* opts, int64_t n,
                           const float* pos, const float* opacity, const float* radius,
                           float* proj, uint32_t* depth_key, uint32_t* ntiles, void* ws,
                           size_t ws_bytes, void* stream);

/*
 * Step 1 over a ring buffer of point clouds (Sec. 3.1 "Fast and Stable
 * View-Specific Sampling during Inference": instead of sampling several
 * view-specific clouds for every frame, each frame samples one and reuses
 * the clouds of the previous frames).  The ring is one allocation of
 * n_slots slots of slot_cap points: point j of slot s is index
 * s * slot_cap + j of pos, opacity, radius (and of feat in the blend), and
 * slot s holds counts[s] <= slot_cap live points at its start (counts: host
 * array); the rest of a slot is never interpreted (any contents).  Same
 * outputs as inpc_project for n = n_slots * slot_cap points, with the slot
 * tails culled (ntiles = 0), so the later steps render the union of the
 * slots' clouds in one pass, ordered by (depth key, ring index), and the
 * backward writes every slot's gradients in place (zero for the tails).
 * A frame overwrites the oldest slot and renders the ring; no cloud is
 * copied to assemble the union.  n_slots in [1, 16], n_slots * slot_cap
 * < 2^31; INPC_ERR_INVALID otherwise or for a count outside [0, slot_cap].
 */
inpc_status_t inpc_project_ring(const inpc_camera_t* cam, const inpc_opts_t* opts,
                                int32_t n_slots, int64_t slot_cap, const int64_t* counts,
                                const float* pos, const float* opacity, const float* radius,
                                float* proj, uint32_t* depth_key, uint32_t* ntiles, void* ws,
                                size_t ws_bytes, void* stream);

/*
 * Step 2 -- bin (Sec. 3.2 "Tiled Rendering": one copy of a point per tile
 * its footprint meets).  Exclusive scan of the per-tile counts gathered by
 * inpc_project into tile_ranges, then one (depth key, point index) copy per
 * touched tile into the workspace buckets.
 *   proj, depth_key, ntiles: outputs of inpc_project
 *   tile_ranges [num_tiles + 1] u32 out: tile t owns list[tile_ranges[t] ..
 *               tile_ranges[t+1]); tile_ranges[num_tiles] = total copies M
 *   tile_order  [num_tiles] u32 out, or NULL: a permutation of the tiles by
 *               decreasing copy count, for the blend passes (results do not
 *               depend on it; it only schedules long lists first)
 */
inpc_status_t inpc_bin(const inpc_camera_t* cam, const inpc_opts_t* opts, int64_t n,
                       const float* proj, const uint32_t* depth_key, const uint32_t* ntiles,
                       uint32_t* tile_ranges, uint32_t* tile_order, void* ws, size_t ws_bytes,
                       void* stream);

/*
 * Step 3 -- depth sort per tile (Sec. 3.2: depth-sorted per-tile lists).
 * Sorts every tile's bucket by (depth key ascending, point index
 * ascending) -- the same order the paper's split sort (stable depth sort,
 * then stable tile sort) produces -- and writes the point indices.  For
 * bilinear splats it also writes, per list entry, where the point's 2x2
 * footprint sits inside the tile, which the blend passes read instead of
 * the point positions to find which pixels a copy covers.
 *   n           the point count the workspace was prepared for by
 *               inpc_project / inpc_bin
 *   proj        output of inpc_project (bilinear splats only; may be NULL
 *               for Gaussians)
 *   tile_ranges output of inpc_bin
 *   tile_order  output of inpc_bin, or NULL
 *   list        [inpc_copy_capacity(n, cam, opts)] u32 out; the first
 *               tile_ranges[num_tiles] entries are written
 *   lpos        [inpc_copy_capacity(n, cam, opts)] u16 out (bilinear splats;
 *               ignored and may be NULL for Gaussians): entry q of tile
 *               (tx, ty) holds (x0 - T tx + 1) | (y0 - T ty + 1) << 8, with
 *               (x0, y0) the top-left pixel of the point's 2x2 splat
 */
inpc_status_t inpc_sort(const inpc_camera_t* cam, const inpc_opts_t* opts, int64_t n,
                        const float* proj, const uint32_t* tile_ranges,
                        const uint32_t* tile_order, uint32_t* list, uint16_t* lpos, void* ws,
                        size_t ws_bytes, void* stream);

/* Copy capacity (list entries) of a workspace sized for n points. */
int64_t inpc_copy_capacity(int64_t n, const inpc_camera_t* cam, const inpc_opts_t* opts);

/*
 * Step 4 -- blend forward (Eq. (1), front to back, then the background).
 * For every pixel, the fragments of its tile's list in order: alpha = o w
 * (w bilinear weight or Gaussian value), F += T alpha f, T *= 1 - alpha;
 * stops before the first fragment whose T < t_min; finally F += T f_bg.
 *   proj       output of inpc_project (position, opacity, radius or depth)
 *   feat       [n][C] features, dtype INPC_F32 / INPC_F16 / INPC_BF16
 *              (blending and accumulation are FP32 for every dtype)
 *   bg         [C] f32 constant background features, [C][H][W] per-pixel
 *              background when opts->bg_per_pixel, or NULL (zero)
 *   tile_ranges, list: outputs of inpc_bin / inpc_sort
 *   tile_order [num_tiles] from inpc_bin, or NULL (tile-index order)
 *   lpos       output of inpc_sort (bilinear splats; NULL for Gaussians)
 *   out        [C][H][W] f32 out: feature image
 *   t_final    [H][W] f32 out: transmittance behind the last blended fragment
 *   n_contrib  [H][W] u32 out: number of blended fragments
 *   state      inpc_state_bytes() bytes out, read by inpc_blend_backward;
 *              may be NULL when no backward pass follows
 */
inpc_status_t inpc_blend_forward(const inpc_camera_t* cam, const inpc_opts_t* opts, int64_t n,
                                 const float* proj, const void* feat, int32_t C, int32_t dtype,
                                 const float* bg,
                                 const uint32_t* tile_ranges, const uint32_t* tile_order,
                                 const uint32_t* list, const uint16_t* lpos, float* out,
                                 float* t_final, uint32_t* n_contrib, void* state, void* ws,
                                 size_t ws_bytes, void* stream);

/*
 * Step 5 -- blend backward (Appendix A, Eq. (2), with the sign of the
 * background term that differentiating Eq. (1) gives, and without skipping
 * zero-alpha fragments).  Replays every pixel's blended fragments back to
 * front and accumulates, for loss L = sum G . F + sum G_T T_final:
 *   dL/dalpha_k = T_k (G . f_k - G . B_k) - G_T T_k prod_{j>k} (1 - alpha_j),
 * B_k the blend of everything behind fragment k including the background;
 * then dL/df, dL/do = w dL/dalpha, dL/d(u,v) = o dw/d(u,v) dL/dalpha.
 * Every splat kind.  Screen-space Gaussians: w = exp(-|d|^2 / (2 s2)) with
 * s2 = r^2 + dilation, differentiated in (u, v) (not in the radius).
 * World-space Gaussians: w = exp(-d^T S^-1 d / 2) with S the projected
 * covariance, differentiated in (u, v) through both the offset d and S, and
 * in the depth Z through S (grad_z; inpc_project_backward adds it).
 *   proj, ntiles, tile_ranges, tile_order, list, lpos: from steps 1-3
 *              (recomputed or kept)
 *   t_final, state: from inpc_blend_forward with the same inputs
 *   grad_out   [C][H][W] f32 dL/dF
 *   grad_t     [H][W] f32 dL/dT_final, or NULL
 *   grad_feat  [n][C] f32 out (FP32 for every feature dtype)
 *   grad_opacity [n] f32 out
 *   grad_uv    [n][2] f32 out (input of inpc_project_backward)
 *   grad_z     [n] f32 out: dL/dZ at fixed (u, v) (world-space Gaussians;
 *              may be NULL for the other splats, else written with zeros)
 *   grad_bg    [C] f32 out (sum over pixels of T_final G), [C][H][W] (T_final G
 *              per pixel) when opts->bg_per_pixel, or NULL
 *   scratch    device scratch of inpc_backward_scratch_bytes(n, C, ...) bytes
 * Every output element is written (zero for culled points and for points no
 * blended fragment reached).  A point whose footprint lies in one tile gets
 * its gradient stored by that tile; a point split over several tiles gets
 * each tile's share added with float atomics, so the last bits of those
 * gradients depend on the order the tiles finish in.
 */
inpc_status_t inpc_blend_backward(const inpc_camera_t* cam, const inpc_opts_t* opts, int64_t n,
                                  const float* proj, const void* feat, int32_t C, int32_t dtype,
                                  const float* bg,
                                  const uint32_t* ntiles, const uint32_t* tile_ranges,
                                  const uint32_t* tile_order, const uint32_t* list,
                                  const uint16_t* lpos, const float* t_final, const void* state,
                                  const float* grad_out, const float* grad_t, float* grad_feat,
                                  float* grad_opacity, float* grad_uv, float* grad_z,
                                  float* grad_bg, void* scratch, size_t scratch_bytes, void* ws,
                                  size_t ws_bytes, void* stream);

/*
 * Step 5 split in two, so that the zero fill it starts with can run ahead on
 * another stream, overlapped with the list build that precedes the backward
 * (App. A, Eq. (2): the gradient rows are sums over blended fragments, and
 * a point no fragment reaches keeps zero).
 *
 * inpc_backward_zero writes zeros to grad_feat [n][C] f32 and to the first
 * 16 n bytes of `scratch` (the per-point scalar rows), on `stream`.  Both
 * must be 16-byte aligned; scratch_bytes >= 16 n.  n == 0 does nothing.
 * Errors: INPC_ERR_INVALID for n out of range, C outside [1, 32], a NULL or
 * misaligned buffer, or a short scratch.
 *
 * inpc_blend_backward_prezeroed takes the arguments of inpc_blend_backward
 * and gives its results, but does not zero grad_feat and the scalar rows
 * itself: the caller has run inpc_backward_zero on the same grad_feat and
 * scratch, ordered before this call (same stream, or an event wait), with
 * nothing writing to them in between.  Without that the gradients are
 * wrong; nothing checks it.
 */
inpc_status_t inpc_backward_zero(int64_t n, int32_t C, float* grad_feat, void* scratch,
                                 size_t scratch_bytes, void* stream);
inpc_status_t inpc_blend_backward_prezeroed(
    const inpc_camera_t* cam, const inpc_opts_t* opts, int64_t n, const float* proj,
    const void* feat, int32_t C, int32_t dtype, const float* bg, const uint32_t* ntiles,
    const uint32_t* tile_ranges, const uint32_t* tile_order, const uint32_t* list,
    const uint16_t* lpos, const float* t_final, const void* state, const float* grad_out,
    const float* grad_t, float* grad_feat, float* grad_opacity, float* grad_uv, float* grad_z,
    float* grad_bg, void* scratch, size_t scratch_bytes, void* ws, size_t ws_bytes,
    void* stream);

/*
 * Step 5 without allocation -- for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and errors as
 * inpc_blend_backward, minus `scratch`: the scratch comes from a static
 * device array of INPC_STATIC_SCRATCH_BYTES (64 MiB) that the library holds
 * on every GPU it runs on until the process ends.  Calls needing more than
 * that (inpc_backward_scratch_bytes(n, C, ...) > INPC_STATIC_SCRATCH_BYTES,
 * about 4 M points at C = 16 and 1080p) return INPC_ERR_INVALID.  The call
 * itself allocates nothing.  The device is the current HIP device (the one
 * `stream` belongs to).  Every call on a GPU shares that GPU's array, so
 * calls that overlap on one GPU (concurrent streams, threads) race: the
 * caller serialises them.
 */
#define INPC_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
inpc_status_t inpc_blend_backward_noalloc(
    const inpc_camera_t* cam, const inpc_opts_t* opts, int64_t n, const float* proj,
    const void* feat, int32_t C, int32_t dtype, const float* bg, const uint32_t* ntiles,
    const uint32_t* tile_ranges, const uint32_t* tile_order, const uint32_t* list,
    const uint16_t* lpos, const float* t_final, const void* state, const float* grad_out,
    const float* grad_t, float* grad_feat, float* grad_opacity, float* grad_uv, float* grad_z,
    float* grad_bg, void* ws, size_t ws_bytes, void* stream);

/* Bytes of the scratch inpc_blend_backward needs for n points and C channels:
 * 16 per point (the opacity, position and depth gradients as one row per point,
 * which the atomics of points split over tiles add to) plus 4 C per tile
 * (the per-tile shares of the background gradient).  0 if invalid. */
size_t inpc_backward_scratch_bytes(int64_t n, int32_t C, const inpc_camera_t* cam,
                                   const inpc_opts_t* opts);

/*
 * Step 6 -- project backward (Sec. 2: the chain rule through the pinhole
 * projection of step 1, so that the position gradients of App. A Eq. (2)
 * reach the points; Sec. 3.2 for the depth term of world-space Gaussians):
 * dL/dX = G_u fx/Z, dL/dY = G_v fy/Z,
 * dL/dZ = G_Z - (G_u fx X + G_v fy Y)/Z^2, dL/dp = R^T (dL/dX, dL/dY, dL/dZ);
 * zero for culled points (ntiles == 0).
 *   grad_uv [n][2] f32; grad_z [n] f32 (the blend's dL/dZ at fixed (u, v),
 *   world-space Gaussians) or NULL (G_Z = 0); grad_pos [n][3] f32 out
 */
inpc_status_t inpc_project_backward(const inpc_camera_t* cam, int64_t n, const float* pos,
                                    const uint32_t* ntiles, const float* grad_uv,
                                    const float* grad_z, float* grad_pos, void* stream);

/*
 * Background from a spherical environment map (Sec. 3.2 "Faster Background
 * Model Evaluation": the background model is distilled into an
 * equirectangular map sampled with bilinear interpolation along every
 * pixel's view direction; the local view directions depend only on the
 * intrinsics and are cached).  The sampled image is passed to the blend as
 * a per-pixel background (opts->bg_per_pixel = 1), which composites it
 * behind the points: F += T_final f_bg(pixel).
 *
 * inpc_view_dirs: dirs [H][W][3] f32 out, the unit camera-space direction
 *   through every pixel centre, normalize((x + 0.5 - cx) / fx,
 *   (y + 0.5 - cy) / fy, 1).  Computed once per set of intrinsics.
 * inpc_envmap_forward: bg [C][H][W] f32 out, sampled from env [Hm][Wm][C]
 *   f32 (texel-major) along w = R^T d: longitude phi = atan2(w_x, w_z),
 *   polar angle theta = acos(-w_y / |w|) (OpenCV axes, so -y is up); column
 *   coordinate (phi / (2 pi) + 1/2) Wm, row coordinate (theta / pi) Hm;
 *   texel (i, j) centred at (i + 1/2, j + 1/2); bilinear between the four
 *   surrounding centres, wrapping in longitude, clamping at the poles.
 * inpc_envmap_backward: grad_env [Hm][Wm][C] f32 out (zeroed by the call,
 *   then every pixel's grad_bg [C][H][W] is added onto its four texels with
 *   the same weights, float atomics: the last bits depend on their order).
 */
inpc_status_t inpc_view_dirs(const inpc_camera_t* cam, float* dirs, void* stream);
inpc_status_t inpc_envmap_forward(const inpc_camera_t* cam, const float* dirs, const float* env,
                                  int32_t Hm, int32_t Wm, int32_t C, float* bg, void* stream);
inpc_status_t inpc_envmap_backward(const inpc_camera_t* cam, const float* dirs,
                                   const float* grad_bg, int32_t Hm, int32_t Wm, int32_t C,
                                   float* grad_env, void* stream);

/*
 * Many views in one pass.  A training step or a frame renders several views
 * (the paper samples one cloud per view and combines several clouds per
 * frame, Sec. 3.1), with uneven point counts and resolutions.  The caller
 * describes every view in an inpc_view_t: its camera and points, and the
 * same per-view buffers the single-view calls take (sized by
 * inpc_workspace_bytes, inpc_copy_capacity, inpc_num_tiles,
 * inpc_state_bytes and inpc_backward_scratch_bytes for that view).  The
 * table lives twice: `views_dev`, in device memory, is what the batched
 * kernels read; `views_host`, the same records in host memory, sizes the
 * launches.  All views share opts, the channel count C and the feature
 * dtype.
 *
 * inpc_rasterize_batched(pass = INPC_PASS_FORWARD): every view's tile
 *   lists are built (steps 1-3), then ONE launch blends every (view, tile)
 *   item: a kernel lays out a device work queue of all items (the views
 *   interleaved quad by quad in proportion to their tile counts, every
 *   view's tiles longest first) and the blend takes one item per workgroup
 *   in queue order.  Writes out, t_final, n_contrib and state of every
 *   view, exactly as inpc_blend_forward would.
 * inpc_rasterize_batched(pass = INPC_PASS_BACKWARD): the lists are built
 *   again, ONE launch replays every (view, tile) item
 *   backwards, then every view's gradients are finished and chained to
 *   positions: grad_feat, grad_opacity, grad_uv, grad_pos and grad_bg as
 *   inpc_blend_backward + inpc_project_backward give them.
 * batch_ws: device scratch of inpc_batch_workspace_bytes(views_host, ...)
 *   bytes (per-view kernel arguments and the work queue).
 * Everything is ordered on `stream` and allocates no device memory, so a
 * pass can be captured into a HIP graph: the views' own steps (lists, the
 * backward's zero fill and finishing passes) run side by side on up to 8
 * library-owned streams (default priority, created on the first call on a
 * device and kept until the process ends), forked from `stream` and joined
 * back to it with events.  Host-side checks as for the single-view calls,
 * all before any launch; n_views must be in [1, 64].
 */
typedef struct {
    inpc_camera_t cam;
    int64_t n;
    const float* pos;          /* [n][3] */
    const float* opacity;      /* [n] */
    const float* radius;       /* [n] screen-space Gaussian radii, or NULL */
    const void* feat;          /* [n][C] of the batch's dtype */
    const float* bg;           /* [C] or [C][H][W] (opts->bg_per_pixel), or NULL */
    float* proj;               /* [n][4], 16-byte aligned */
    uint32_t* depth_key;       /* [n] */
    uint32_t* ntiles;          /* [n] */
    uint32_t* tile_ranges;     /* [num_tiles + 1] */
    uint32_t* tile_order;      /* [num_tiles] */
    uint32_t* list;            /* [copy capacity] */
    uint16_t* lpos;            /* [copy capacity] (bilinear) */
    void* state;               /* inpc_state_bytes() */
    void* ws;                  /* inpc_workspace_bytes(), zeroed when first allocated */
    size_t ws_bytes;
    void* scratch;             /* inpc_backward_scratch_bytes() (backward pass) */
    size_t scratch_bytes;
    float* out;                /* [C][H][W] */
    float* t_final;            /* [H][W] */
    uint32_t* n_contrib;       /* [H][W] */
    const float* grad_out;     /* [C][H][W] (backward) */
    const float* grad_t;       /* [H][W] or NULL */
    float* grad_feat;          /* [n][C] f32 */
    float* grad_opacity;       /* [n] */
    float* grad_uv;            /* [n][2] */
    float* grad_pos;           /* [n][3] */
    float* grad_bg;            /* like bg, or NULL */
    float* grad_z;             /* [n] (world-space Gaussians, backward), else NULL */
    int32_t ring_slots;        /* > 0: the points are a ring of ring_slots slots of
                                  n / ring_slots points (inpc_project_ring); 0: one cloud */
    const int64_t* ring_counts; /* host [ring_slots]: live points per slot (ring views) */
} inpc_view_t;

enum { INPC_PASS_FORWARD = 0, INPC_PASS_BACKWARD = 1 };

size_t inpc_batch_workspace_bytes(const inpc_view_t* views_host, int32_t n_views,
                                  const inpc_opts_t* opts);
inpc_status_t inpc_rasterize_batched(const inpc_view_t* views_host, const inpc_view_t* views_dev,
                                     int32_t n_views, const inpc_opts_t* opts, int32_t C,
                                     int32_t dtype, int32_t pass, void* batch_ws,
                                     size_t batch_ws_bytes, void* stream);

/*
 * View-dependent point features (Sec. 2 "Implicit Point Cloud": the
 * appearance field gives every point spherical-harmonics coefficients up to
 * degree two per feature channel, evaluated at the view direction).  The
 * step before the rasterizer: its output is the `feat` of step 4.
 *   view direction d = (p - c) / |p - c|, camera centre c = -R^T t;
 *   real orthonormal SH of degrees 0-2 in graphics order (Condon-Shortley
 *   phase): Y0 = k0, Y1 = -k1 y, Y2 = k1 z, Y3 = -k1 x, Y4 = k2 x y,
 *   Y5 = -k2 y z, Y6 = k3 (2 z^2 - x^2 - y^2), Y7 = -k2 x z, Y8 = k4 (x^2 - y^2),
 *   k0 = 1/(2 sqrt(pi)), k1 = sqrt(3/(4 pi)), k2 = sqrt(15/(4 pi)),
 *   k3 = sqrt(5/(16 pi)), k4 = sqrt(15/(16 pi));  feat[i][c] = sum_j Y_j sh[i][c][j].
 * inpc_sh_features: pos [n][3], sh [n][C][9] f32 -> feat [n][C] f32 (C in [1, 64]).
 * inpc_sh_features_backward: grad_feat [n][C] -> grad_sh [n][C][9] (written)
 *   and grad_pos [n][3] (written; the position gradient through the view
 *   direction only, to be added to the rasterizer's; NULL skips it).
 */
inpc_status_t inpc_sh_features(const inpc_camera_t* cam, int64_t n, const float* pos,
                               const float* sh, int32_t C, float* feat, void* stream);
inpc_status_t inpc_sh_features_backward(const inpc_camera_t* cam, int64_t n, const float* pos,
                                        const float* sh, int32_t C, const float* grad_feat,
                                        float* grad_sh, float* grad_pos, void* stream);

/* The only synchronising call: waits for `stream`, then returns
 * INPC_ERR_CAPACITY if any build on this workspace since the last
 * inpc_check_sync() ran out of copy capacity (and clears the flag, so the
 * next build runs), INPC_OK otherwise. */
inpc_status_t inpc_check_sync(void* ws, size_t ws_bytes, void* stream);

/* Static description of a status code. */
const char* inpc_status_string(inpc_status_t status);

/* Message of the last INPC_ERR_INVALID / INPC_ERR_HIP on the calling thread. */
const char* inpc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* INPC_RASTER_H */
