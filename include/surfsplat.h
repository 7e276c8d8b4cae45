/*
 * surfsplat: differentiable EWA surfel rasterizer of 3D Surface Splatting (3DSS)
 * on AMD Instinct MI355X (gfx950).  C ABI.
 *
 * Forward (render): per (surfel, view) projection through the T-matrix with a
 * centre-precomputed object-space MIP filter (Sec. 3.1, Sec. 3.3.2), per-surfel
 * split-sum shading against an HDR environment map (eq:ibl, Sec. 3.4.2), tile
 * binning and a radix sort keyed by the start of each surfel's depth interval
 * (Sec. 3.2.1), and per pixel: interval-merging surface separation (Alg. 1),
 * Shepard normalisation (eq:shepard), coverage opacity from the accumulated
 * weight (eq:alpha) and front-to-back layer compositing with at most K_max
 * layers (eq:compositing, App. A.1).
 * Backward (render_backward): the adjoint of all of the above (App. A.1,
 * "Backward Pass Implementation"), producing gradients with respect to surfel
 * positions, normals, tangents, scales, albedo, roughness, metallic and the
 * environment maps.
 *
 * Conventions (shared by every entry point):
 *   - All buffers named "device" are device memory owned by the caller; they
 *     must stay alive until the work queued on the given stream has finished.
 *   - Surfel attributes are structure-of-arrays float32 [C][N]: row c of
 *     attribute a is a + c*N.  N is the total surfel count over all scenes;
 *     scene s owns surfels [surfel_offset[s], surfel_offset[s+1]).
 *   - The surfel frame: n_hat = normal/|normal|, u_hat = Gram-Schmidt of
 *     tangent against n_hat, v_hat = n_hat x u_hat, t_u = scale[0] u_hat,
 *     t_v = scale[1] v_hat (world units; one standard deviation of the kernel).
 *   - Cameras: pinhole, world->camera rotation R (row-major) and translation t,
 *     OpenCV axes (x right, y down, z forward); pixel (i, j) has its centre at
 *     (i + 1/2, j + 1/2) in pixel units.
 *   - Images are float32 [sum_v H_v W_v][3] in view order, row-major per view;
 *     alpha is float32 [sum_v H_v W_v] (alpha = 1 - residual transmittance).
 *   - Environment maps are equirectangular float32 [H_e][W_e][3], z up; texel
 *     (a, b) looks along (sin th cos ph, sin th sin ph, cos th) with
 *     th = pi (a + 1/2)/H_e, ph = 2 pi (b + 1/2)/W_e.
 *   - Calls never abort and never throw.  Argument errors are reported
 *     synchronously; conditions found on the device (pair-capacity overflow)
 *     are latched and reported by ss_poll.  A forward that overflowed its pair
 *     capacity writes NaN into every pixel of its image and alpha, and a
 *     backward after it NaN into every surfel gradient, so the failure cannot
 *     pass unnoticed where nobody polls (for instance in replayed graphs).
 *   - One context serves one stream at a time.
 */
#ifndef SURFSPLAT_H
#define SURFSPLAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* ss_stream;  /* a hipStream_t */

typedef enum ss_status {
  SS_OK = 0,
  SS_ERR_INVALID_ARG = 1, /* a null pointer, a size out of range, bad options   */
  SS_ERR_HIP = 2,         /* a HIP runtime call failed                           */
  SS_ERR_CAPACITY = 3,    /* pair capacity too small; ss_reserve and call again  */
  SS_ERR_STATE = 4,       /* call out of order (backward without forward, ...)   */
  SS_ERR_UNSUPPORTED = 5, /* an option value this build does not implement       */
  SS_ERR_NOMEM = 6,       /* device allocation failed                            */
  SS_ERR_STATIC_LIMIT = 7 /* the batch does not fit the fixed workspace of
                             ss_render_static                                   */
} ss_status;

typedef enum ss_shade_mode {
  SS_SHADE_ALBEDO = 0,   /* colour = albedo                                      */
  SS_SHADE_SPLITSUM = 1, /* split-sum microfacet IBL, eq:ibl                     */
  SS_SHADE_NORMAL = 2    /* normal image (Sec. 4.2.3): the attribute is the world-space
                            unit normal, and each layer's Shepard mean is renormalised
                            to unit length before compositing                     */
} ss_shade_mode;

typedef enum ss_launch_mode {
  SS_LAUNCH_BATCHED = 0,  /* every view of the batch in one launch per stage    */
  SS_LAUNCH_PER_VIEW = 1  /* one launch sequence per view (comparison baseline) */
} ss_launch_mode;

typedef struct ss_options {
  float r_cut;    /* kernel cutoff radius in standard deviations (App. A.1: 3)   */
  int32_t k_max;  /* maximum composited layers per pixel, 1..16 (App. A.1: 16)   */
  float gamma;    /* coverage gain of eq:alpha (Sec. 3.5.1: 2 pi)                */
  float sigma_f;  /* screen-space prefilter variance, px^2 (eq:mip_cov)          */
  int32_t shade;  /* ss_shade_mode                                                */
  int32_t tile_w; /* tile width in pixels: 8, 16 or 32                           */
  int32_t tile_h; /* tile height in pixels: 8 or 16                              */
  int32_t lds_batch; /* surfels staged per LDS batch: 32, 64, 128 or 256; 0: the
                        library picks one at each reserve from the measured mean
                        tile-list length (the largest of 32..256 not above it)  */
  int32_t launch;    /* ss_launch_mode                                            */
  int32_t persistent; /* 1: raster blocks pull (view, tile) items from a queue   */
  int32_t depth_stats; /* 1: reserve per-layer depth statistics (8 bytes x 16 layers
                          per pixel) so that forwards may output the
                          depth-consolidation term (ss_outputs.cons)            */
  int32_t mip;         /* 0: centre-precomputed MIP filter (Sec. 3.3.2, default);
                          1: per-pixel Jacobian (Sec. 3.3.1): J = d(u,v)/d(x,y) at
                          every intersection, support = the binning rectangle of the
                          centre filter intersected with rho^2 < r_cut^2; the
                          backward differentiates the per-pixel filter as well   */
  int32_t env_lds;     /* split-sum backward: floats of environment-level gradients
                          the shading adjoint may accumulate in a block-private LDS
                          copy (levels in the order irradiance, 5, 4, ..., 0, each
                          only while it fits whole); the others take global atomics.
                          -1 (default): as many as fit (39936 floats); 0: none.
                          Results agree either way up to the order of float sums  */
  float t_min;         /* transmittance early-out: once a layer has been composited
                          and the transmittance left in front of the next one,
                          T_{k+1} = prod_{j<=k} (1 - alpha_j), is below t_min, the
                          pixel's walk ends and later groups are discarded, exactly
                          as after the K_max-th layer (App. A.1); the image keeps
                          T_{K+1} bg.  0 (default): off, the exact semantics        */
  int32_t deterministic; /* 1: ss_render_backward returns bitwise identical gradients
                          for identical inputs and options: the raster backward sums
                          each record's per-fragment gradients per (record, tile)
                          in a fixed order, stores that partial at the pair's
                          emission slot and adds a record's slots in emission order
                          (instead of float atomics in arrival order); the shading
                          adjoint adds environment texel gradients as 64-bit
                          integers (a per-scene power-of-two scale bounded from the
                          records, every level in global memory) and the
                          environment adjoint sums fixed chunks in a fixed order.
                          Slower; reserves 64 bytes per pair and 4 per record more */
  int32_t validate;    /* 1: every ss_render counts the non-finite surfel parameters
                          and environment texels, every ss_render_backward the
                          non-finite entries of d_image / d_alpha; the count of the
                          last call is reported by ss_poll (n_nonfinite)          */
  int32_t counters;    /* 1: the raster forward counts its work (ss_diag:
                          n_evaluated, n_fragments, n_layers, sum_layer_weight)   */
  int32_t tonemap;     /* 0 (default): the image is the composited linear (HDR) colour;
                          1: the image is passed per channel through the log-space
                          and sRGB transfer used for HDR targets with eq:photo_loss
                          (Sec. 3.7.1): y = srgb(log(1 + max(x, 0))), with
                          srgb(v) = 12.92 v for v <= 0.0031308, else
                          1.055 v^(1/2.4) - 0.055.  d_image is then dL/dy and the
                          backward applies dy/dx itself.  alpha is not mapped     */
  int32_t seg_len;     /* segment length of split tile lists.  A tile's list is
                          split into segments of this many entries, walked in
                          parallel, when it is longer than both seg_len and
                          2 P w / 6144 (P the pairs of the batch, w the wave64s
                          of a tile: twice an even share of the pairs over the
                          waves the chip keeps resident).  Persistent launches
                          without depth statistics only; the forward merges the
                          segments' layers per pixel in list order, so the
                          decisions are those of one walk and only the float
                          summation order of a layer that spans a segment
                          boundary changes.  0 (default): 2048; -1: never split;
                          otherwise a multiple of 256 from 256 to 32768           */
  int32_t bwd_walk;    /* how the raster backward (App. A.1 "Backward Pass
                          Implementation") walks a tile; both give the same
                          gradients to float summation order.  1: rows -- per
                          4 x 4 quadrant, four of its recorded records per wave
                          step, one per 16-lane row, reduced across the row;
                          2: record-major -- per 8 x 8 sub-tile, the records of
                          a quadrant one per lane, each summing its gradient
                          over the quadrant's pixels.  0 (default): record-major
                          when the LDS batch is 256 records, rows otherwise    */
} ss_options;

typedef struct ss_camera {
  int32_t scene;           /* index of the scene this view renders               */
  int32_t width, height;   /* pixels                                              */
  float fx, fy, cx, cy;    /* focal lengths and principal point, pixels          */
  float R[9];              /* world -> camera rotation, row-major                */
  float t[3];              /* world -> camera translation                        */
  float znear;             /* surfels not entirely beyond znear are culled      */
  float background[3];     /* constant background colour                         */
} ss_camera;

typedef struct ss_batch {
  int32_t n_scenes;
  const int64_t* surfel_offset; /* host [n_scenes + 1], surfel_offset[0] = 0     */
  const float* position;        /* device [3][N] */
  const float* normal;          /* device [3][N] */
  const float* tangent;         /* device [3][N] */
  const float* scale;           /* device [2][N] */
  const float* albedo;          /* device [3][N] */
  const float* roughness;       /* device [N]    */
  const float* metallic;        /* device [N]    */
  const float* const* envmap;   /* host [n_scenes] of device [H_e][W_e][3]; unused (may be NULL) in albedo mode */
  const int32_t* env_hw;        /* host [n_scenes][2] (H_e, W_e), each >= 4 x 8; unused in albedo mode */
  int32_t n_views;
  const ss_camera* cameras;     /* host [n_views] */
} ss_batch;

typedef struct ss_outputs {
  float* image;       /* device [sum HW][3], written */
  float* alpha;       /* device [sum HW], written    */
  uint8_t* n_layers;  /* device [sum HW] or NULL: layers composited per pixel */
  /* device [sum HW] or NULL: per-pixel depth-consolidation term of eq:cons_loss
   * (Sec. 3.7.1), sum_{i<j} w_i w_j |z_i - z_j| + sum_i w_i^2 var_i over the
   * composited layers, w_i = T_i alpha_i, z_i and var_i the Shepard-weighted
   * mean and variance of the layer's fragment depths (camera-space z of the
   * ray-surfel intersection).  The 1/|P| mean and the loss weight are the
   * caller's.  Needs options.depth_stats = 1 (else SS_ERR_INVALID_ARG). */
  float* cons;
  /* device [sum HW] or NULL: composited depth sum_k T_k alpha_k z_k with z_k the
   * layer's mean depth as above (divide by alpha for the expected depth of the
   * covered part).  Needs options.depth_stats = 1. */
  float* depth;
  /* host, or NULL: receives the generation number of this forward (1, 2, ...
   * per context); ss_render_static writes 0 (it leaves no state for a backward) */
  int64_t* generation;
} ss_outputs;

typedef struct ss_grad_in {
  const float* d_image; /* device [sum HW][3]: dL/dimage                       */
  const float* d_alpha; /* device [sum HW] or NULL: dL/dalpha                  */
  const float* d_cons;  /* device [sum HW] or NULL: dL/dcons; needs the last forward to
                           have written cons or depth (else SS_ERR_STATE)       */
  const float* d_depth; /* device [sum HW] or NULL: dL/ddepth; same condition  */
  int64_t generation;   /* 0: the context's last forward; otherwise the number that
                           forward reported: SS_ERR_STATE when a later forward has
                           replaced its state (two renders before one backward)   */
} ss_grad_in;

typedef struct ss_grads { /* every pointer may be NULL (skip); outputs are overwritten */
  float* d_position;  /* device [3][N] */
  float* d_normal;    /* device [3][N] */
  float* d_tangent;   /* device [3][N] */
  float* d_scale;     /* device [2][N] */
  float* d_albedo;    /* device [3][N] */
  float* d_roughness; /* device [N]    */
  float* d_metallic;  /* device [N]    */
  float* const* d_envmap; /* host [n_scenes] of device [H_e][W_e][3], or NULL */
  /* Densification statistic (Sec. 3.6.1, eq:ss_grad): for every pixel p of
   * every view and every surfel whose fragment reaches p, the per-pixel
   * screen-space positional gradient g = (dL_p/dT1z, dL_p/dT2z) T4z, with L_p
   * the pixel's share of the loss (d_image . image + d_alpha alpha) and T1z,
   * T2z, T4z the z entries of the surfel's T rows in that view (the MIP filter
   * differentiated with them).  screen_grad[s] = sum over views and pixels of
   * |g| (summation order not fixed).  visible_views[s] = number of views in
   * which the surfel passes the cull with a non-empty tile rectangle; the
   * paper's criterion is screen_grad / visible_views.  Both device [N], NULL to
   * skip; computing screen_grad adds work to the raster backward. */
  float* screen_grad;
  int32_t* visible_views;
} ss_grads;

typedef struct ss_diag {
  int32_t status;        /* latched device status (ss_status)                   */
  int64_t n_records;     /* (surfel, view) records of the last forward          */
  int64_t n_pairs;       /* (tile, surfel) pairs of the last forward            */
  int64_t pair_capacity; /* pairs the workspace holds                           */
  int64_t workspace_bytes;
  int64_t generation;    /* generation number of the last ss_render (0: none)   */
  int64_t n_nonfinite;   /* options.validate: non-finite inputs of the last render
                            plus those of the last backward                       */
  /* options.counters, the last forward: */
  int64_t n_evaluated;   /* (pixel, record) pairs the raster evaluated (E)        */
  int64_t n_fragments;   /* fragments accumulated into composited layers (F)      */
  int64_t n_layers;      /* layers composited over all pixels                     */
  double sum_layer_weight; /* sum of their accumulated weights W_k (eq:alpha)     */
  /* the last ss_render_static on the current device (any context): */
  int32_t static_status; /* its latched status (SS_OK or SS_ERR_CAPACITY)        */
  int64_t static_pairs;  /* its (tile, surfel) pair count                        */
  int64_t static_pair_capacity;
} ss_diag;

typedef struct ss_context ss_context;

/* Fills *opt with the paper's settings: r_cut 3, K_max 16, gamma 2 pi,
 * sigma_f 0.1 px^2, albedo shading, 16x16 tiles, LDS batch 128, batched,
 * persistent raster, no early-out, no tone map, atomics (not deterministic),
 * no validation, no counters. */
ss_status ss_default_options(ss_options* opt);

/* Creates a context on the current HIP device.  *out receives ownership. */
ss_status ss_create(const ss_options* opt, ss_context** out);
ss_status ss_destroy(ss_context* ctx);
/* Replaces the options (tile size, batch, launch mode, ...); the next forward
 * re-bins.  Invalidates the stored forward state. */
ss_status ss_set_options(ss_context* ctx, const ss_options* opt);

/* BRDF table of eq:ibl: (beta1, beta2) indexed by (n.w_o, roughness) on a
 * vertex-centred [n_r][n_nv][2] grid (r = i/(n_r-1), n.v = max(j/(n_nv-1), 1e-3)),
 * GGX (alpha = r^2) with separable Smith masking and Schlick Fresnel, integrated
 * with `samples` Hammersley samples.  Writes the table to `lut` (device,
 * [n_r][n_nv][2]) on `stream`.  n_nv, n_r in 2..1024, samples in 1..65536. */
ss_status ss_brdf_lut(float* lut, int32_t n_nv, int32_t n_r, int32_t samples, ss_stream stream);
/* Copies a table (device [n_r][n_nv][2]) into the context for split-sum shading. */
ss_status ss_set_brdf_lut(ss_context* ctx, const float* lut, int32_t n_nv, int32_t n_r, ss_stream stream);

/* Sizes the workspace for `batch` (runs the projection and the tile count once
 * and synchronises `stream`).  After it, ss_render/ss_render_backward on the
 * same batch shape allocate nothing and synchronise nothing (they may be
 * captured in a HIP graph).  *workspace_bytes (may be NULL) receives the size. */
ss_status ss_reserve(ss_context* ctx, const ss_batch* batch, ss_stream stream, size_t* workspace_bytes);

/* Forward.  Calls ss_reserve itself when the batch shape (surfel counts,
 * views, resolutions, environment sizes) differs from the reserved one.  When
 * the surfels moved so that the pairs no longer fit, the device latches
 * SS_ERR_CAPACITY (see ss_poll): the outputs of that call are invalid; call
 * ss_reserve and render again. */
ss_status ss_render(ss_context* ctx, const ss_batch* batch, const ss_outputs* out, ss_stream stream);

/* Backward of the last ss_render on this context with the same batch.
 * Returns SS_ERR_STATE without a matching forward.  With split-sum shading and
 * environment gradients requested, the environment adjoint runs on a stream of
 * the context, forked from `stream` and joined back into it by events before
 * the call returns (a captured graph holds both branches); work queued on
 * `stream` afterwards sees every output. */
ss_status ss_render_backward(ss_context* ctx, const ss_batch* batch, const ss_grad_in* gin,
                             const ss_grads* grads, ss_stream stream);

/* Synchronises the context's last stream and reports the latched status. */
ss_status ss_poll(ss_context* ctx, ss_diag* out);

/* Allocation-free forward, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The same computation as ss_render, with every buffer of its
 * workspace taken from one fixed device array of SS_STATIC_SCRATCH_BYTES per
 * GPU (held by each GPU the library runs on until the process ends) instead of
 * the context's workspace: it calls no allocating routine and does not
 * synchronise.  The context supplies only its options and BRDF table, and its
 * own forward state is left as it was (a backward still refers to the last
 * ss_render).  Tile lists are never split (options.seg_len is ignored), so the
 * result equals ss_render's with seg_len = -1 bit for bit.  Limits: batched
 * launch mode (else SS_ERR_UNSUPPORTED); records,
 * pixels, tiles and environment levels must fit the array with room for at
 * least 4096 pairs, else SS_ERR_STATIC_LIMIT before any device work.  The
 * pair capacity is what the array has left; an overflow latches
 * SS_ERR_CAPACITY (ss_poll: static_status) and the image and alpha are NaN.
 * Every call on a GPU shares that GPU's array and clears what must start at
 * zero; calls that overlap in time on one GPU (two streams, two threads)
 * race and their results are undefined. */
#define SS_STATIC_SCRATCH_BYTES (32u << 20)
ss_status ss_render_static(ss_context* ctx, const ss_batch* batch, const ss_outputs* out, ss_stream stream);

/* Test access to the last forward's binning: record keys (depth-interval start
 * bits, or 0xffffffff when culled), per-record pixel rectangles (int32
 * [R][4]: i_lo, j_lo, i_hi, j_hi, or empty), the sorted pair list
 * (keys = global tile << 32 | z_start bits, values = record index) and the
 * per-tile [start, end) ranges.  Device destinations; any may be NULL.
 * *n_pairs and *n_tiles receive the counts (synchronises the stream). */
ss_status ss_debug_binning(ss_context* ctx, uint32_t* rec_zbits, int32_t* rec_rect,
                           uint64_t* pair_keys, uint32_t* pair_vals, uint32_t* tile_ranges,
                           int64_t* n_pairs, int64_t* n_tiles, ss_stream stream);

/* Test access to the environment levels of the last ss_render (split-sum
 * shading, eq:ibl, Sec. 3.4.2): the GGX-prefiltered levels 1..5 and the
 * irradiance level of scene `scene`, copied into `levels` (host or device),
 * each level [row][column][rgb] float32 in that order, n = 3 x the sum of the
 * levels' texel counts (level l of an He x We map: max(He >> l, 4) x
 * max(We >> l, 8); irradiance 32 x 64).  SS_ERR_STATE without a split-sum
 * forward, SS_ERR_INVALID_ARG for a scene out of range, a null destination or
 * another n.  Synchronises the stream. */
ss_status ss_debug_env_levels(ss_context* ctx, int32_t scene, float* levels, int64_t n, ss_stream stream);

/* Stage timing.  While enabled, every stage of ss_render / ss_render_backward
 * is bracketed by HIP events on the caller's stream (not usable under graph
 * capture).  ss_profile_read synchronises the last stream and writes, for each
 * stage, the summed milliseconds and the number of timed launches since the
 * previous read (ms and count: arrays of SS_NUM_STAGES, may be NULL).
 * Stage order: envmap, preprocess, binning (scan, emission, sort, ranges),
 * raster_forward, raster_backward, preprocess_backward, envmap_backward. */
#define SS_NUM_STAGES 7
ss_status ss_profile_enable(ss_context* ctx, int32_t enable);
ss_status ss_profile_read(ss_context* ctx, double* ms, int64_t* count);

const char* ss_status_str(ss_status s);

#ifdef __cplusplus
}
#endif
#endif /* SURFSPLAT_H */
