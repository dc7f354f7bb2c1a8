/*
 * niv.h -- C interface of the MI355X Neural Irradiance Volume library
 * (libniv.so).
 *
 * The library evaluates and trains the model of Coomans, Nazzaro et al.,
 * "Real-time Rendering with a Neural Irradiance Volume" (Eurographics 2026):
 * a multi-level hash-grid encoding of the position plus spherical-harmonic
 * encoding of the normal, fed to a ReLU MLP with a linear RGB output
 * (Sec. 4.1), queried per G-buffer pixel and shaded with albedo * E / pi
 * (Sec. 4.4, Eq. 2).
 *
 * Conventions for every call:
 *  - Pointers named "device" point to memory on the current HIP device.  The
 *    caller owns every buffer it passes; the library never frees them.
 *  - Calls that take a hipStream_t only enqueue work on that stream and
 *    return; errors raised by a kernel surface as NIV_ERR_HIP on a later
 *    call.  Arguments are validated on the host before anything is enqueued;
 *    on an error nothing is enqueued.
 *  - A handle may be used from one host thread at a time.
 */
#ifndef NIV_H
#define NIV_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NIV_OK = 0,
    NIV_ERR_INVALID_ARG = 1,  /* null/misaligned pointer, bad size or value */
    NIV_ERR_UNSUPPORTED = 2,  /* valid model shape the kernels do not cover */
    NIV_ERR_HIP = 3,          /* a HIP runtime call failed */
    NIV_ERR_WORKSPACE = 4,    /* caller-provided scratch too small */
    NIV_ERR_STATE = 5,        /* call out of order (e.g. no prepared model) */
    NIV_ERR_NONFINITE = 6     /* a training step's loss or gradient was not finite */
} niv_status;

typedef enum { NIV_FP32 = 0, NIV_FP16 = 1, NIV_BF16 = 2 } niv_precision;

/* Model shape (Sec. 4.1).  Level l has resolution floor(base_res *
 * per_level_scale^l); it is stored densely ((N+1)^3 entries, x fastest) when
 * that fits in T = 2^log2_T entries, else hashed into T entries with the
 * primes 1, 2654435761, 805459861.  The input vector is the concatenation
 * of the n_levels * n_features grid features (level-major), the positional
 * code of x when pos_bands > 0 (the grid-free models of Table 1: u = the
 * position mapped onto the unit cube by the box, then per band k <
 * pos_bands sin(2^k pi u_x..z) and cos(2^k pi u_x..z), 3 + 6 pos_bands
 * values), sh_bands^2 real spherical harmonics of the unit normal, and for
 * each scene variable the 2*extra_bands values sin(2^k pi t), cos(2^k pi t)
 * (Sec. 6).  Hidden layers are width wide with ReLU, no biases; the output
 * layer is linear.
 * Supported by the kernels: sh_bands = 4, n_out = 3, and either a grid of
 * two features per entry (n_levels 8 or 16, pos_bands 0: width 64 with 2 or
 * 3 hidden layers, or width 128 with 4 hidden layers and one scene
 * variable), a grid of four features per entry (Table 1's grid networks:
 * n_levels 2, 4, 6 or 8, width 64, 3 hidden layers, no scene variable;
 * queries only, training gives NIV_ERR_UNSUPPORTED) or no grid (n_levels 0,
 * pos_bands 8, width 16, 32 or 64, 3 hidden layers). */
typedef struct {
    int32_t n_levels, log2_T, n_features;
    double  base_res, per_level_scale;
    int32_t sh_bands;
    int32_t n_extra, extra_bands;
    int32_t width, n_hidden, n_out;
    double  aabb_min[3], aabb_max[3];   /* box mapped onto every level */
    int32_t pos_bands;                  /* 0, or bands of the positional code */
} niv_config;

typedef struct niv_handle niv_handle;

/* Validates `cfg` and builds the level table and parameter layout on the
 * host.  *out receives a new handle (release with niv_destroy). */
niv_status niv_create(const niv_config *cfg, niv_handle **out);
void niv_destroy(niv_handle *h);

/* Sizes: number of FP32 master parameters (layout [grid entries][F] then
 * W_0, W_1, ... W_H row-major [out][in]), number of grid values, and the
 * bytes of a prepared model for `prec` (see niv_prepare).  NULL outputs are
 * skipped. */
niv_status niv_sizes(const niv_handle *h, niv_precision prec, int64_t *n_params,
                     int64_t *n_grid_values, int64_t *prepared_bytes);

/* Per-level resolution, dense flag, first entry and entry count; each array
 * has n_levels elements (host memory; NULL arrays are skipped). */
niv_status niv_level_info(const niv_handle *h, int64_t *res, int32_t *dense,
                          int64_t *offset, int64_t *size);

/* Converts FP32 master parameters (device, n_params floats) into a prepared
 * model (device, prepared_bytes, 256-byte aligned) for queries at `prec`:
 * weights re-laid out as matrix-core operands, grid latents and weights
 * rounded to nearest-even in FP16/BF16 (copied for FP32). */
niv_status niv_prepare(niv_handle *h, const float *params, void *prepared,
                       niv_precision prec, hipStream_t stream);

/* One G-buffer (or any list of `count` query points).  All arrays device,
 * row-major, 4-byte aligned:
 *   pos, nrm     [count][3] float   world position, surface normal (any length)
 *   albedo       [count][3] float   or NULL (then out_L must be NULL)
 *   mask         [count]    uint8   1 = pixel covered, 0 = skip; NULL = all
 *   extra_values                    the frame's scene variables (n_extra used)
 *   model        prepared model for the precision of the call
 *   out_E        [count][3] float   irradiance E_theta(x, n) (indirect, Sec. 3)
 *   out_L        [count][3] float   albedo * E / pi (Eq. 2), or NULL
 *   out_flags    [count]    uint8   or NULL: bit 0 position outside the box
 *                (clamped), bit 1 non-finite input or zero normal (E set to
 *                0), bit 2 non-finite E, bit 4 finite E with a negative
 *                channel (irradiance is non-negative, the linear output
 *                layer is not).  Masked-off pixels get E = L = 0, flags 0.
 *   out_inputs   [count][din] float or NULL: the encoded input vector of each
 *                pixel as fed to the network (grid features, SH, frequency
 *                code; rounded to the operand precision), for inspection.
 *   in_flags     [count] uint8 or NULL: caller's request (non-zero) to send a
 *                pixel to the Monte Carlo fallback (niv_query_fallback only).
 *   scene        scene of the frame for the fallback, or NULL (no fallback).
 * count < 2^28. */
struct mc_scene;
typedef struct {
    int64_t count;
    const float *pos, *nrm, *albedo;
    const uint8_t *mask;
    float extra_values[4];
    const void *model;
    float *out_E, *out_L;
    uint8_t *out_flags;
    float *out_inputs;
    const uint8_t *in_flags;
    const struct mc_scene *scene;
} niv_frame;

/* Evaluates every pixel of `n_frames` frames (Sec. 4.4: per-pixel E(x, n)
 * from the position and normal buffers, then Eq. 2), arithmetic of `prec`:
 * features in FP32, matrix products on the matrix cores with FP32
 * accumulation (FP32 operands for NIV_FP32). */
niv_status niv_query(niv_handle *h, const niv_frame *frames, int32_t n_frames,
                     niv_precision prec, hipStream_t stream);
/* Frames may differ in size and each may use its own prepared model of this
 * shape and precision; up to 16 frames go into one persistent launch whose
 * workgroups walk the frames' pixel tiles in order. */

/* Inspection of the encoding (Sec. 4.1): for points i < count (pos, device
 * [count][3] float) the grid entries that the query's encoding at `prec`
 * reads, out (device) [count][n_levels][8] uint32: the level's first entry
 * plus the corner's index within the level, corner c = cx + 2 cy + 4 cz of
 * the cell, dense x + (N+1)(y + (N+1) z) or the spatial hash.  The entries
 * come from the same device encoding function that niv_query (training != 0:
 * the forward pass of niv_backward) runs for this model and precision, with
 * positions clamped to the box: FP64 cell coordinates, except the FP16
 * query, which takes FP32 coordinates (at a cell face it may choose the
 * neighbouring cell).  `model` is a prepared model of `prec` (its level
 * table is read).  Non-finite positions give 0xFFFFFFFF.  count < 2^28;
 * grid-free models give NIV_ERR_UNSUPPORTED. */
niv_status niv_corner_indices(niv_handle *h, niv_precision prec, int32_t training, const void *model,
                              const float *pos, int64_t count, uint32_t *out, hipStream_t stream);

/* Measurement: the encoding stage of niv_query alone (grid gathers and
 * trilinear blends, spherical harmonics), with the query's launch shape,
 * pixel order and encoding functions, for one frame of a 16-level room model
 * (other shapes: NIV_ERR_UNSUPPORTED).  Instead of running the network it
 * writes one word per pixel, the XOR of the encoded input, to out_E[3 q]
 * (the rest of out_E, out_L and out_flags are not written).  Its time is a
 * floor for the fused query's time on the same frame. */
niv_status niv_probe_encode(niv_handle *h, const niv_frame *frame, niv_precision prec,
                            hipStream_t stream);

/* Measurement: one pass of n x 128 four-byte gathers (8 per level, 16 levels)
 * in the pattern `mode`: 0 random words over an 8 MiB table (64 cache lines
 * per instruction, the pattern of the training forward's encoding), 1
 * consecutive words (2 lines per instruction), 2 quads of lanes sharing a
 * line (16 lines), 3 a line per lane (64 lines); modes 1-3 read the first
 * 16 KiB only.  table: device, 8 MiB; out: device, 2048 x 256 words written.
 * 1 <= n <= 2^24.  The caller times the launch. */
niv_status niv_probe_gather(int32_t mode, int32_t n, const void *table, void *out, hipStream_t stream);

/* Monte Carlo fallback for pixels the network should not answer: after the
 * query, pixels whose flags intersect `flag_mask` (bits 0, 2 and 4 of
 * out_flags) or whose in_flags are set are appended to a list, and
 * their E is replaced by mc_irradiance(spp, bounces, mc_flags) of the frame's
 * scene (L = albedo E / pi); their flags gain bit 3.  Random stream: point
 * index (frame << 28) | pixel. */
typedef struct {
    uint32_t flag_mask;
    int32_t spp, bounces, mc_flags;
    uint64_t seed;
} niv_fallback;

/* Scratch for up to max_flagged fallback pixels per call. */
niv_status niv_fallback_sizes(const niv_handle *h, int64_t max_flagged, int64_t *workspace_bytes);

/* niv_query of up to 16 frames followed by the Monte Carlo fallback, all
 * enqueued on `stream` without host synchronisation (pixels beyond the
 * scratch capacity keep the network's answer).  workspace: device, 256-byte
 * aligned, niv_fallback_sizes bytes. */
niv_status niv_query_fallback(niv_handle *h, const niv_frame *frames, int32_t n_frames,
                              niv_precision prec, const niv_fallback *fb, void *workspace,
                              int64_t workspace_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * niv_query_fallback with the counter and the list of flagged pixels in a
 * fixed scratch array inside the library instead of a workspace argument.
 * Computes exactly what niv_query_fallback computes with a list of
 * max_flagged entries.  1 <= max_flagged <= NIV_NOALLOC_MAX_FLAGGED
 * (4 MiB of scratch); a larger value gives NIV_ERR_WORKSPACE, a smaller one
 * NIV_ERR_INVALID_ARG, and nothing is enqueued.  The scratch is held on
 * each device the library runs on until the process ends (its device
 * address is looked up on the first call on a device); every call on one
 * device shares it, so calls that overlap on one device, on different
 * streams or from different threads, race and must be serialised by the
 * caller.  The counter is cleared by each call.  Allocates nothing. */
#define NIV_NOALLOC_MAX_FLAGGED (1 << 20)
niv_status niv_query_fallback_noalloc(niv_handle *h, const niv_frame *frames, int32_t n_frames,
                                      niv_precision prec, const niv_fallback *fb,
                                      int64_t max_flagged, hipStream_t stream);

/* Half-resolution rendering (Sec. 4.4): the network runs at a quarter of
 * the pixels and the full-resolution albedo shades the result.  The
 * half-resolution samples are the G-buffer pixels (2x, 2y), x < ceil(W/2),
 * y < ceil(H/2).  Upsampling is joint bilateral (the cited method) with the
 * G-buffer as guide: pixel (X, Y) averages the usable samples (covered,
 * finite, non-zero normal) with |2x - X| <= 2 and |2y - Y| <= 2 that face
 * its way (n . n_s > 0), weighted by exp(-(dx^2 + dy^2) / (2 sigma_px^2))
 * (n . n_s)^normal_power exp(-|p - p_s|^2 / (2 sigma_pos^2)).  With no
 * sample facing its way it takes the nearest usable sample (flag bit 5); with
 * no usable sample in the window E = 0 (flag bit 6).  Full-resolution flags
 * also carry bit 0 (outside the box) and bit 1 (non-finite input or zero
 * normal, E = 0); masked-off pixels get E = L = 0, flags 0. */
typedef struct {
    float sigma_px;        /* spatial Gaussian in full-resolution pixels, > 0 */
    float sigma_pos;       /* position guide in world units, > 0 */
    int32_t normal_power;  /* exponent of the normal guide, 0..64 */
} niv_upsample_params;

/* One full-resolution G-buffer (device arrays, row-major, 4-byte aligned):
 *   pos, nrm     [height][width][3] float; albedo the same or NULL
 *   mask         [height][width] uint8 or NULL
 *   half_E       [ceil(height/2)][ceil(width/2)][3] float: written by
 *                niv_query_half, read by niv_upsample
 *   half_flags   [ceil(height/2)][ceil(width/2)] uint8 or NULL: query flags
 *                of the samples (niv_query_half)
 *   out_E, out_L [height][width][3] float (out_L NULL or albedo given)
 *   out_flags    [height][width] uint8 or NULL
 * width, height >= 1, width * height < 2^28. */
typedef struct {
    int32_t width, height;
    const float *pos, *nrm, *albedo;
    const uint8_t *mask;
    float extra_values[4];
    const void *model;
    float *half_E;
    uint8_t *half_flags;
    float *out_E, *out_L;
    uint8_t *out_flags;
} niv_half_frame;

/* Joint bilateral upsampling of f->half_E to every pixel, then L = albedo E
 * / pi (Eq. 2).  Uses the handle's box for bit 0; model and extra values
 * are not read. */
niv_status niv_upsample(niv_handle *h, const niv_half_frame *f, const niv_upsample_params *p,
                        hipStream_t stream);

/* The fused query at the half-resolution samples (E into half_E, flags into
 * half_flags), then niv_upsample; both enqueued on `stream`. */
niv_status niv_query_half(niv_handle *h, const niv_half_frame *f, const niv_upsample_params *p,
                          niv_precision prec, hipStream_t stream);

/* Times the fused query on these frames for each candidate launch shape
 * (workgroup of 256 or 512 threads, and 768 for the lane-sliced 6-D field at
 * FP16/BF16, x 1, 2 or all-resident workgroups per CU x tile order: plain,
 * or XCD-grouped, where each of the 8 XCDs walks a contiguous eighth of the
 * tiles so that neighbouring pixels share an L2; best of 10 launches) and
 * keeps the fastest for later calls at this precision.  Synchronises
 * `stream`; the frames' outputs are overwritten.  out (optional, host): the
 * n <= 24 candidates and their times, and the chosen shape. */
typedef struct {
    int32_t n;
    int32_t block[24], blocks_per_cu[24], xcd_order[24];
    float ms[24];
    int32_t chosen_block, chosen_blocks_per_cu, chosen_xcd_order;
    float chosen_ms;
} niv_tune_result;
niv_status niv_autotune(niv_handle *h, const niv_frame *frames, int32_t n_frames,
                        niv_precision prec, hipStream_t stream, niv_tune_result *out);

/* Sets the launch shape of later queries at `prec` directly (for instance a
 * shape niv_autotune chose in an earlier process): block 256, 512 or 768
 * threads (768 takes effect for the lane-sliced 6-D field at FP16/BF16 and
 * runs as 512 elsewhere), blocks_per_cu 0 (all resident) or more,
 * xcd_order 0 or 1.  Out-of-range values give NIV_ERR_INVALID_ARG and
 * change nothing. */
niv_status niv_set_tune(niv_handle *h, niv_precision prec, int32_t block, int32_t blocks_per_cu,
                        int32_t xcd_order);

/* A frame captured as a HIP graph: niv_query (fb == NULL) or
 * niv_query_fallback with the given buffers, replayed by niv_graph_launch.
 * Capturing runs the frame once eagerly first.  Buffers must outlive the
 * graph; their contents may change between launches. */
typedef struct niv_graph niv_graph;
niv_status niv_graph_capture(niv_handle *h, const niv_frame *frames, int32_t n_frames,
                             niv_precision prec, const niv_fallback *fb, void *workspace,
                             int64_t workspace_bytes, niv_graph **out);
niv_status niv_graph_launch(niv_graph *g, hipStream_t stream);
void niv_graph_destroy(niv_graph *g);

/* ------------------------------------------------------------------ */
/* Training (Sec. 4.5)                                                  */
/* ------------------------------------------------------------------ */

/* A batch of training samples (device arrays): x, nrm [count][3] float
 * position and direction; extra [count][n_extra] scene variables (NULL when
 * n_extra = 0); target [count][3] float irradiance; valid [count] uint8 or
 * NULL (0 = sample contributes nothing but stays in the mean). */
typedef struct {
    int64_t count;
    const float *x, *nrm, *extra, *target;
    const uint8_t *valid;
} niv_batch;

/* Training state, all device memory owned by the caller: FP32 master
 * parameters, their gradient, Adam moments (n_params floats each, moments
 * zero before step 1), the prepared model of the training precision (kept
 * equal to niv_prepare(params)), scratch of niv_train_sizes bytes (256-byte
 * aligned) and a scalar receiving the batch loss. */
typedef struct {
    float *params, *grads, *adam_m, *adam_v;
    void *model;
    void *workspace;
    int64_t workspace_bytes;
    float *loss;
} niv_train_state;

/* Adam hyper-parameters for one update; step is the 1-based iteration. */
typedef struct {
    float lr, beta1, beta2, eps;
    int64_t step;
} niv_adam;

/* Scratch bytes for batches of up to max_batch samples, 1 <= max_batch <=
 * 2^24 (FP32 or FP16 training; BF16 is NIV_ERR_UNSUPPORTED).  About 0.2 KB
 * per sample for the saved activations plus 12 B per (sample, level,
 * corner) for the binned grid scatter (0.5 GB at 2^18 samples and 16
 * levels). */
niv_status niv_train_sizes(const niv_handle *h, niv_precision prec, int64_t max_batch,
                           int64_t *workspace_bytes);

/* Loss and gradient of one batch (Eq. 3), 1 <= count <= 2^24: loss = mean over samples and RGB
 * channels of (E - y)^2 / (E^2 + 0.01), the denominator held constant; the
 * gradient of every parameter is written to st->grads (overwritten), the
 * loss to st->loss.  The forward pass uses st->model at `prec` (matrix
 * products on the matrix cores with FP32 accumulation); gradients are FP32.
 * The gradient does not depend on scheduling: weight gradients are summed
 * in a fixed order, and each grid value is the sum of its contributions
 * (the 8 trilinear corners of every level, Sec. 4.1) in 64-bit fixed point,
 * converted to FP32 once.  With NIV_FP16 each contribution is first rounded
 * to FP16 at a per-step power-of-two scale (11 significant bits, the
 * precision of that path's operands); with NIV_FP32 it is summed as computed.  A sample whose output or target gives a
 * non-finite d loss / dE marks the step non-finite (niv_train_status) and
 * contributes nothing to the grid.  One pass (the count of the grid scatter)
 * runs on a second stream that the library creates once per device
 * (default priority, kept until the process ends), forked from and joined
 * back to `stream` with events: the call's work is complete when `stream`'s
 * is. */
niv_status niv_backward(niv_handle *h, const niv_batch *b, const niv_train_state *st,
                        niv_precision prec, hipStream_t stream);

/* One Adam update (Kingma & Ba) of every parameter from st->grads. */
niv_status niv_adam_update(niv_handle *h, const niv_train_state *st, const niv_adam *ad,
                           hipStream_t stream);

/* niv_backward, niv_adam_update, then niv_prepare of st->model.  When the
 * step's loss or gradient is not finite the update is skipped on the device
 * (parameters and moments unchanged) and niv_train_status reports it; the
 * call itself stays asynchronous. */
niv_status niv_train_step(niv_handle *h, const niv_batch *b, const niv_train_state *st,
                          const niv_adam *ad, niv_precision prec, hipStream_t stream);

/* Waits for `stream`, then NIV_ERR_NONFINITE if the last niv_backward or
 * niv_train_step on this scratch (st->workspace) met a non-finite loss or
 * gradient (a diverged output or a non-finite target), else NIV_OK. */
niv_status niv_train_status(const niv_train_state *st, hipStream_t stream);

/* Learning rate of step `step` (1-based) of the schedule of Sec. 4.5: lr0
 * for the first hold_steps steps, then exponential decay reaching lr1 at
 * step total_steps (and lr1 after it).  The paper holds 1e-2 for 10k of its
 * iterations and decays to 1e-4; the bake takes hold_steps = total / 5,
 * that ratio at its own step budget.  Host only. */
niv_status niv_lr_schedule(int64_t step, int64_t hold_steps, int64_t total_steps, double lr0,
                           double lr1, double *lr);

/* Seeded initial parameters (device, n_params floats, the layout of
 * niv_sizes): grid values uniform on [grid_lo, grid_hi), weights of each
 * matrix Xavier-uniform on [-a, a), a = sqrt(6 / (fan_in + fan_out)) (the
 * paper does not state its initialisation; the cited hash encoding starts
 * its table near zero).  Parameter k draws uniform number 0 of generator
 * stream (seed, k, 0, 3) (Philox4x64-10 as in mc_irradiance), the value is
 * formed in FP64 and rounded once to FP32.  Enqueued on `stream`. */
niv_status niv_init_params(niv_handle *h, float *params, uint64_t seed, float grid_lo,
                           float grid_hi, hipStream_t stream);

/* ------------------------------------------------------------------ */
/* Monte Carlo irradiance (training targets and reference)              */
/* ------------------------------------------------------------------ */

/* Scene primitive, 64 bytes (host memory).  kind 0: solid axis-aligned box
 * p = min corner, q = max corner, faces look outward; kind 1: axis-aligned
 * rectangle centred at p, normal axis `axis`, front face looking along
 * sign * e_axis, half extents q[0], q[1] along axes (axis+1)%3 and
 * (axis+2)%3; kind 2: disk centred at p, unit normal q (front side), radius.
 * A primitive with non-zero emission (radiance leaving its front face) is a
 * light; lights must be rectangles or disks, at most 8. */
typedef struct {
    int32_t kind, axis;
    float sign;
    float p[3], q[3];
    float radius;
    float albedo[3], emission[3];
} niv_mc_prim;

typedef struct mc_scene mc_scene;

/* Copies `n_prims` (1..4096) primitives to the device and builds the light
 * list and the area table of non-emitting surfaces.  Allocates device memory
 * owned by the scene (released by mc_scene_destroy). */
niv_status mc_scene_create(const niv_mc_prim *prims, int32_t n_prims, mc_scene **out);
void mc_scene_destroy(mc_scene *s);

#define NIV_MC_NEE 1              /* next-event estimation at every bounce */
#define NIV_MC_EMIT_ON_HIT 2      /* gather emission found by continuation rays */
#define NIV_MC_INCLUDE_DIRECT 4   /* add emission seen at the first hit */
#define NIV_MC_DIRECT_AT_ORIGIN 8 /* direct irradiance at x by light sampling */

/* Monte Carlo estimate of the indirect irradiance E(x, n) of Eq. 1 (light
 * reflected 1..bounces times before reaching x, Sec. 3) at `count` points
 * (device x, nrm [count][3] float; nrm need not be unit).  Per sample: a
 * cosine-distributed direction about n; a first hit seen from behind is a
 * back face (counted, scores 0); emission at the first hit is direct and
 * skipped unless NIV_MC_INCLUDE_DIRECT; then at each bounce the light
 * reflected there is gathered (NIV_MC_NEE or NIV_MC_EMIT_ON_HIT, exactly one
 * of them) and the path continues with a cosine-sampled direction, throughput
 * times albedo.  Rays start 1e-4 x scene extent off the surface along the
 * normal.  Tracing in FP32, sums in FP64.  Random number `d` of sample s of
 * point i is dimension d of Philox4x64-10 with counter (i, s, d/8, 0) and key
 * (seed, 0): 0-1 first direction, bounce k >= 1 uses 2+(k-1)(2J+2)+2j for
 * light j and 2+(k-1)(2J+2)+2J for the continuation (J lights).
 * Outputs (device): out_E [count][3] double mean and/or out_E32 [count][3]
 * the same rounded to float (either may be NULL, not both); out_var
 * [count][3] variance of the mean or NULL; out_backfaces [count] or NULL; out_valid [count] or NULL:
 * 1 iff back faces <= spp/2 and some channel of E > 0 (Sec. 4.5 culling and
 * null-irradiance rejection). */
niv_status mc_irradiance(const mc_scene *s, const float *x, const float *nrm, int64_t count,
                         int32_t spp, int32_t bounces, int32_t flags, uint64_t seed,
                         double *out_E, float *out_E32, double *out_var, int32_t *out_backfaces,
                         uint8_t *out_valid, hipStream_t stream);

/* Scenes that change with a scene variable t (Sec. 6: moving emitters,
 * moving occluders): motion (host, [n_prims][3] float, or NULL for a static
 * scene) translates primitive k by t * motion[k]; t comes per point
 * (mc_irradiance_at) or per frame (extra value 0 of a niv_frame, for the
 * Monte Carlo fallback).  Training points on surfaces are drawn only on
 * primitives that do not move.  The ray offset uses the extent at t = 0. */
niv_status mc_scene_set_motion(mc_scene *s, const float *motion);

/* mc_irradiance with the scene variable of each point: t [count] float
 * (device), or NULL for t = 0. */
niv_status mc_irradiance_at(const mc_scene *s, const float *x, const float *nrm, const float *t,
                            int64_t count, int32_t spp, int32_t bounces, int32_t flags, uint64_t seed,
                            double *out_E, float *out_E32, double *out_var, int32_t *out_backfaces,
                            uint8_t *out_valid, hipStream_t stream);

/* Training points (Sec. 4.2 and 4.5): points [0, count - n_surface) uniform in
 * the box [lo, hi] (host arrays of 3) with a normal uniform on the sphere;
 * points [count - n_surface, count) uniform by area over the non-emitting
 * surfaces with the surface's front normal.  Philox stream 1, counter
 * (i, 0, d/8, 1).  out_x, out_n: device [count][3] float. */
niv_status mc_sample_points(const mc_scene *s, const double *lo, const double *hi, int64_t count,
                            int64_t n_surface, uint64_t seed, float *out_x, float *out_n,
                            hipStream_t stream);

/* mc_sample_points that also draws a scene variable per point, uniform on
 * [0, 1) (Sec. 6: the variable is sampled at random during training):
 * out_t [count] float (device), dimension 7 of the point's stream. */
niv_status mc_sample_points_t(const mc_scene *s, const double *lo, const double *hi, int64_t count,
                              int64_t n_surface, uint64_t seed, float *out_x, float *out_n,
                              float *out_t, hipStream_t stream);

/* ---------------------------------------------------------------------
 * Dynamic ambient occlusion (Sec. 4.4).  A model trained on the static
 * scene does not see geometry placed at render time; the shaded irradiance
 * is multiplied by the visibility V of the hemisphere at each pixel against
 * that dynamic geometry only: one minus the cosine-weighted share of
 * directions whose ray from pos + eps n meets a dynamic triangle (either
 * side) at a distance in (0, radius].  V is estimated from `rays` cosine-
 * distributed directions: direction k of pixel i uses dimensions 0 and 1 of
 * Philox4x64-10 with counter (i, k, 0, 2) and key (seed, 0), the directions
 * mapped as mc_irradiance's first direction.  Ray tests in FP32.
 * ------------------------------------------------------------------- */
typedef struct niv_ao niv_ao;

typedef struct {
    int32_t rays;        /* 1..4096 directions per pixel */
    float radius;        /* > 0: farther triangles do not occlude */
    float eps;           /* >= 0: ray origin offset along the unit normal */
    uint64_t seed;
} niv_ao_params;

/* Builds a bounding-volume hierarchy over `n_tris` (0..2^22) triangles
 * `tris` [n_tris][3 vertices][3] float (host memory, finite) on the host and
 * copies it to the device (owned by the returned object, released by
 * niv_ao_destroy).  A new set of dynamic objects (or new placements) needs
 * a new object. */
niv_status niv_ao_create(const float *tris, int64_t n_tris, niv_ao **out);
void niv_ao_destroy(niv_ao *ao);
/* Inner nodes of the hierarchy (each record holds its two children's
 * boxes) and its depth (root 0). */
niv_status niv_ao_info(const niv_ao *ao, int32_t *n_nodes, int32_t *depth);

/* For pixels i < count (device buffers): pos, nrm [count][3] float; mask
 * [count] uint8 or NULL (0: pixel left alone, V = 1).  Outputs, each may be
 * NULL: vis [count] float receives V; E and L [count][3] float are
 * multiplied by V in place (the query's outputs of the same pixels).
 * Pixels with a non-finite position or a zero normal get V = 1.  Enqueued
 * on `stream`; nothing is allocated. */
niv_status niv_ao_apply(const niv_ao *ao, const niv_ao_params *p, int64_t count, const float *pos,
                        const float *nrm, const uint8_t *mask, float *E, float *L, float *vis,
                        hipStream_t stream);

const char *niv_status_string(niv_status s);

#ifdef __cplusplus
}
#endif
#endif /* NIV_H */
