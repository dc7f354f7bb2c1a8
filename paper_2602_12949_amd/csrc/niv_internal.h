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
};

// Prepared model: [level table, kLevelBytes][operand block][grid latents].
constexpr int kLevelBytes = kMaxLevels * (int)sizeof(LevelConst);
static_assert(kLevelBytes % 256 == 0, "level table keeps the operand block aligned");

struct LevelTable {
    LevelConst lv[kMaxLevels];
};

struct QueryArgs {
    const float *pos, *nrm, *albedo;
    const uint8_t *mask;
    float *out_E, *out_L;
    uint8_t *out_flags;
    float *out_inputs;        // optional [count][din] encoded input vectors
    const uint8_t *model;     // prepared model
    int64_t count;
    uint64_t grid_off;        // byte offset of the grid in the prepared model
    uint32_t hash_mask;       // T - 1
    int32_t pad0;
    float extra[4];           // scene variables of the frame
    double lo[3], hi[3];      // box the positions are clamped to
    // training forward only (the fused kernel instantiated with TRAIN):
    const float *extra_ps;    // per-sample scene variables [count][n_extra] or null
    const float *target;      // [count][3] irradiance targets
    const uint8_t *valid;     // [count] or null
    uint8_t *x_save;          // activations, per 64-sample chunk [rows][64]
    uint32_t *mask_save;      // ReLU masks, per chunk, layer, dword, lane
    float *dE;                // [count][3] d(loss)/dE without the 1/(3n) factor
    float *loss;              // device scalar, accumulates the Eq. 3 loss
    float loss_scale;         // 1/(3n)
    float loss_eps;           // 0.01 (Eq. 3)
};

// Shapes the fused kernels are instantiated for.
enum ModelKind { kUnitCube = 0, kRoom = 1, kWide6D = 2, kNumKinds = 3 };

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
};

// Defined in query.hip.
OpLayout op_layout(int kind, niv_precision prec);
hipError_t launch_prepare(const Model &m, const float *params, void *prepared,
                          niv_precision prec, hipStream_t stream);
hipError_t launch_query(const Model &m, const QueryArgs &a, niv_precision prec,
                        hipStream_t stream);

}  // namespace niv

struct niv_handle {
    niv::Model m;
};
