// Internal declarations shared by the host side and the kernels of libniv.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "niv.h"

namespace niv {

constexpr int kMaxLevels = 32;
constexpr uint32_t kPrime1 = 2654435761u;  // y prime of the spatial hash
constexpr uint32_t kPrime2 = 805459861u;   // z prime (x prime is 1)

// Per-level constants of the encoding.  The cell coordinate on axis a is
// s = fma(p, k[a], o[a]) in FP64 with k = N / (hi - lo), o = -(lo * k).
struct LevelConst {
    double k[3];
    double o[3];
    int32_t nm1;     // N - 1, largest cell index
    int32_t dense;   // 1: (N+1)^3 table, x fastest; 0: hashed into T entries
    uint32_t off;    // first entry of the level in the grid
    uint32_t s1;     // N + 1
    uint32_t s2;     // (N + 1)^2
    uint32_t pad;
    float kf[3], of[3];  // k and o rounded to FP32 (cell coordinates of the FP16 query)
};

// Prepared model: [level table, kLevelBytes][operand block][grid latents].
constexpr int kLevelBytes = kMaxLevels * (int)sizeof(LevelConst);
static_assert(kLevelBytes % 256 == 0, "level table keeps the operand block aligned");

struct LevelTable {
    LevelConst lv[kMaxLevels];
};

constexpr int kMaxFrames = 16;

// One G-buffer of a launch.  Pixels are split into tiles of (waves per
// block) x 64; the frame's tiles are [tile_begin, tile_begin + tiles).
struct FrameArgs {
    const float *pos, *nrm, *albedo;
    const uint8_t *mask, *in_flags;
    float *out_E, *out_L;
    uint8_t *out_flags;
    float *out_inputs;        // optional [count][din] encoded input vectors
    const uint8_t *model;     // prepared model of this frame
    int64_t count;
    int64_t tile_begin;
    float extra[4];           // scene variables of the frame
    // half-resolution samples: pixel q of a sub_w wide grid reads its inputs
    // at pixel (2 (q / sub_w), 2 (q % sub_w)) of a src_w wide G-buffer
    // (sub_w = 0: pixel q reads pixel q)
    int32_t sub_w, src_w;
};

struct QueryArgs {
    int32_t n_frames;
    uint32_t hash_mask;       // T - 1
    int64_t n_tiles;
    uint64_t grid_off;        // byte offset of the grid in a prepared model
    uint32_t grid_bytes;      // size of the grid latents (bounds of the buffer loads)
    uint32_t fb_mask;         // flag bits that send a pixel to the Monte Carlo fallback
    double lo[3], hi[3];      // box the positions are clamped to
    double pe_k[3], pe_o[3];  // u = fma(p, pe_k, pe_o) on the unit cube (positional code)
    uint32_t *fb_list;        // fallback list: (frame << 28) | pixel, or null
    uint32_t *fb_count;       // entries appended (may exceed fb_cap)
    uint32_t fb_cap;
    float loss_scale;         // training: 1/(3n)
    // training forward only (the fused kernel instantiated with TRAIN, frame 0):
    const float *extra_ps;    // per-sample scene variables [count][n_extra] or null
    const float *target;      // [count][3] irradiance targets
    const uint8_t *valid;     // [count] or null
    uint8_t *x_save;          // activations, per 64-sample chunk [rows][64]
    uint32_t *mask_save;      // ReLU masks, per chunk, layer, dword, lane
    float *dE;                // [count][3] d(loss)/dE without the 1/(3n) factor
    float *loss;              // device scalar, accumulates the Eq. 3 loss
    uint32_t *train_status;   // step words of the training scratch; [2] set by a non-finite dE
    float loss_eps;           // 0.01 (Eq. 3)
    uint32_t l0_words;        // FP16 training forward: entries of grid level 0 (dense) held in
    uint32_t l0_off;          // LDS, or 0; and the level's first entry
    int32_t xcd_order;        // tile order, see LaunchTune
    FrameArgs f[kMaxFrames];
};

// Shapes the fused kernels are instantiated for.
// kT1L2..kT1L8: Table 1's grid networks, 2 to 8 levels of four features.
enum ModelKind { kUnitCube = 0, kRoom = 1, kWide6D = 2, kPE16 = 3, kPE32 = 4, kPE64 = 5, kRoom6D = 6,
                 kT1L2 = 7, kT1L4 = 8, kT1L6 = 9, kT1L8 = 10, kNumKinds = 11 };

// Launch shape of the fused query: workgroup size and resident workgroups
// per CU (0 = as many as fit); chosen by niv_autotune, else defaults.
struct LaunchTune {
    int block;
    int blocks_per_cu;
    int xcd_order;   // 1: each XCD walks a contiguous eighth of the tiles
};
constexpr int kXcds = 8;  // workgroups are dealt to the XCDs round robin

// Operand-block layout of a prepared model (see the prepare kernel).
struct OpLayout {
    int64_t w_bytes;     // operand block
    int64_t grid_off;    // grid latents, 256-byte aligned
    int64_t total;
};

struct Model {
    niv_config cfg;
    int kind;
    int din;
    int64_t res[kMaxLevels], size[kMaxLevels], offset[kMaxLevels];
    int32_t dense[kMaxLevels];
    int64_t n_entries, n_grid_values, n_params;
    LevelConst lv[kMaxLevels];
    LaunchTune tune[3];  // per precision
    bool tuned[3];
};

// Defined in query.hip.
OpLayout op_layout(int kind, niv_precision prec);
hipError_t launch_prepare(const Model &m, const float *params, void *prepared,
                          niv_precision prec, hipStream_t stream);
// The weight operands of a prepared model only (trainable shapes, FP32/FP16).
hipError_t launch_prepare_operands(const Model &m, const float *params, void *prepared,
                                   niv_precision prec, hipStream_t stream);
LaunchTune default_tune(int kind, niv_precision prec);
hipError_t launch_query(const Model &m, QueryArgs &a, niv_precision prec, const LaunchTune &tu,
                        hipStream_t stream);
hipError_t launch_zero_u32(uint32_t *p, int n, hipStream_t stream);
hipError_t launch_query_probe(const Model &m, QueryArgs &a, niv_precision prec, const LaunchTune &tu,
                              hipStream_t stream);
struct Box6 {
    double v[6];  // lo x, y, z, hi x, y, z
};
hipError_t launch_trace_corners(const Model &m, niv_precision prec, bool train, const void *model,
                                const float *pos, int64_t count, uint32_t *out, hipStream_t stream);

// Joint bilateral upsampling (upsample.hip).
struct UpsampleArgs {
    const float *pos, *nrm, *albedo;
    const uint8_t *mask;
    const float *half_E;
    float *out_E, *out_L;
    uint8_t *out_flags;
    int32_t width, height, half_w, half_h;
    float lo[3], hi[3];        // box (flag bit 0)
    float c_px, c_pos;         // log2 weight factors: 1 / (2 sigma^2 ln 2)
    float normal_power;
};
hipError_t launch_upsample(const UpsampleArgs &a, hipStream_t stream);

// Monte Carlo fallback of flagged pixels (mc.hip).
struct FbFrame {
    const float *pos, *nrm, *albedo;
    float *out_E, *out_L;
    uint8_t *out_flags;
    const void *prims;        // device primitives of the frame's scene, or null
    const int32_t *lights;
    const void *motion;       // float4 per primitive (scene variable), or null
    const void *recs;         // trace list of the static scene
    int32_t nk[5];            // its counts: boxes, rectangles by axis, disks
    int32_t n_prims, n_lights;
    float eps;
    float t;                  // the frame's scene variable (extra value 0)
};
struct FbArgs {
    const uint32_t *list;
    const uint32_t *count;
    uint32_t cap;
    int32_t spp, bounces, flags;
    uint64_t seed;
    FbFrame f[kMaxFrames];
};
hipError_t launch_mc_fallback(const FbArgs &a, hipStream_t stream);
void mc_scene_device_view(const struct mc_scene *s, const void **prims, const int32_t **lights,
                          int32_t *n_prims, int32_t *n_lights, float *eps, const void **motion);
void mc_scene_trace_view(const struct mc_scene *s, const void **recs, int32_t nk[5]);

}  // namespace niv

struct niv_handle {
    niv::Model m;
};
