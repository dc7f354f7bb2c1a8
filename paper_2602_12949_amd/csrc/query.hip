// Fused query: prepare kernels (level table, operand block, grid) and the
// host launchers of the fused per-pixel kernel defined in query_kernel.h.
#include <hip/hip_runtime.h>
#include <string.h>

#include "niv_internal.h"
#include "niv_device.h"
#include "query_kernel.h"

namespace niv {
template <int P, class S>
__global__ void k_prepare_operands(const float *__restrict__ params, uint8_t *__restrict__ out,
                                   int64_t n_grid, int n_out)
{
    using O = Ops<P, S>;
    int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= O::N_OPS * 64) return;
    int op = tid / 64, lane = tid % 64;
    int64_t off;
    int ne;
    operand_place<P, S>(op, &off, &ne);
    for (int e = 0; e < ne; ++e) {
        int64_t src = operand_source<P, S>(op, lane, e, n_grid, n_out);
        float v = src >= 0 ? params[src] : 0.0f;
        if constexpr (P == NIV_FP32) {
            reinterpret_cast<float *>(out + off)[lane * ne + e] = v;
        } else if constexpr (P == NIV_FP16) {
            reinterpret_cast<_Float16 *>(out + off)[lane * ne + e] = (_Float16)v;
        } else {
            reinterpret_cast<__bf16 *>(out + off)[lane * ne + e] = (__bf16)v;
        }
    }
}

__global__ void k_prepare_levels(const LevelTable t, LevelConst *__restrict__ out)
{
    if (threadIdx.x < kMaxLevels) out[threadIdx.x] = t.lv[threadIdx.x];
}

template <int P>
__global__ void k_prepare_grid(const float *__restrict__ params, uint8_t *__restrict__ out,
                               int64_t n_grid)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; k < n_grid; k += stride) {
        float v = params[k];
        if constexpr (P == NIV_FP32) reinterpret_cast<float *>(out)[k] = v;
        else if constexpr (P == NIV_FP16) reinterpret_cast<_Float16 *>(out)[k] = (_Float16)v;
        else reinterpret_cast<__bf16 *>(out)[k] = (__bf16)v;
    }
}

// ---------------------------------------------------------------- host side
template <int P, class S> OpLayout layout_of()
{
    using O = Ops<P, S>;
    OpLayout L;
    L.w_bytes = O::W_BYTES;
    L.grid_off = kLevelBytes + align256(O::W_BYTES);
    L.total = 0;
    return L;
}

OpLayout op_layout(int kind, niv_precision prec)
{
#define NIV_LAYOUT(P)                                                   \
    switch (kind) {                                                     \
    case kUnitCube: return layout_of<P, ShapeUnitCube>();               \
    case kRoom: return layout_of<P, ShapeRoom>();                       \
    case kPE16: return layout_of<P, ShapePE<16>>();                     \
    case kPE32: return layout_of<P, ShapePE<32>>();                     \
    case kPE64: return layout_of<P, ShapePE<64>>();                     \
    case kRoom6D: return layout_of<P, ShapeRoom6D>();                   \
    case kT1L2: return layout_of<P, ShapeT1<2>>();                      \
    case kT1L4: return layout_of<P, ShapeT1<4>>();                      \
    case kT1L6: return layout_of<P, ShapeT1<6>>();                      \
    case kT1L8: return layout_of<P, ShapeT1<8>>();                      \
    default: return layout_of<P, ShapeWide6DFor<P>>();                  \
    }
    if (prec == NIV_FP32) { NIV_LAYOUT(NIV_FP32) }
    if (prec == NIV_FP16) { NIV_LAYOUT(NIV_FP16) }
    NIV_LAYOUT(NIV_BF16)
#undef NIV_LAYOUT
}

template <int P, class S>
static hipError_t prepare_t(const Model &m, const float *params, void *prepared, hipStream_t st)
{
    using O = Ops<P, S>;
    uint8_t *out = static_cast<uint8_t *>(prepared);
    LevelTable lt;
    memset(&lt, 0, sizeof(lt));
    for (int l = 0; l < m.cfg.n_levels; ++l) lt.lv[l] = m.lv[l];
    hipLaunchKernelGGL(k_prepare_levels, dim3(1), dim3(64), 0, st, lt,
                       reinterpret_cast<LevelConst *>(out));
    int threads = O::N_OPS * 64;
    hipLaunchKernelGGL((k_prepare_operands<P, S>), dim3((threads + 255) / 256), dim3(256), 0, st,
                       params, out + kLevelBytes, m.n_grid_values, m.cfg.n_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (m.n_grid_values == 0) return hipSuccess;
    int64_t blocks = (m.n_grid_values + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL((k_prepare_grid<P>), dim3((unsigned)blocks), dim3(256), 0, st, params,
                       out + kLevelBytes + align256(O::W_BYTES), m.n_grid_values);
    return hipGetLastError();
}

template <int P, class S>
static hipError_t prepare_operands_t(const Model &m, const float *params, void *prepared, hipStream_t st)
{
    using O = Ops<P, S>;
    int threads = O::N_OPS * 64;
    hipLaunchKernelGGL((k_prepare_operands<P, S>), dim3((threads + 255) / 256), dim3(256), 0, st,
                       params, static_cast<uint8_t *>(prepared) + kLevelBytes, m.n_grid_values,
                       m.cfg.n_out);
    return hipGetLastError();
}

hipError_t launch_prepare_operands(const Model &m, const float *params, void *prepared,
                                   niv_precision prec, hipStream_t st)
{
#define NIV_PREPO(P)                                                                          \
    switch (m.kind) {                                                                         \
    case kUnitCube: return prepare_operands_t<P, ShapeUnitCube>(m, params, prepared, st);    \
    case kRoom: return prepare_operands_t<P, ShapeRoom>(m, params, prepared, st);            \
    case kRoom6D: return prepare_operands_t<P, ShapeRoom6D>(m, params, prepared, st);        \
    default: return hipErrorInvalidValue;                                                     \
    }
    if (prec == NIV_FP32) { NIV_PREPO(NIV_FP32) }
    if (prec == NIV_FP16) { NIV_PREPO(NIV_FP16) }
    return hipErrorInvalidValue;
#undef NIV_PREPO
}

hipError_t launch_prepare(const Model &m, const float *params, void *prepared,
                          niv_precision prec, hipStream_t st)
{
#define NIV_PREP(P)                                                                      \
    switch (m.kind) {                                                                    \
    case kUnitCube: return prepare_t<P, ShapeUnitCube>(m, params, prepared, st);        \
    case kRoom: return prepare_t<P, ShapeRoom>(m, params, prepared, st);                \
    case kPE16: return prepare_t<P, ShapePE<16>>(m, params, prepared, st);              \
    case kPE32: return prepare_t<P, ShapePE<32>>(m, params, prepared, st);              \
    case kPE64: return prepare_t<P, ShapePE<64>>(m, params, prepared, st);              \
    case kRoom6D: return prepare_t<P, ShapeRoom6D>(m, params, prepared, st);            \
    case kT1L2: return prepare_t<P, ShapeT1<2>>(m, params, prepared, st);               \
    case kT1L4: return prepare_t<P, ShapeT1<4>>(m, params, prepared, st);               \
    case kT1L6: return prepare_t<P, ShapeT1<6>>(m, params, prepared, st);               \
    case kT1L8: return prepare_t<P, ShapeT1<8>>(m, params, prepared, st);               \
    default: return prepare_t<P, ShapeWide6DFor<P>>(m, params, prepared, st);           \
    }
    if (prec == NIV_FP32) { NIV_PREP(NIV_FP32) }
    if (prec == NIV_FP16) { NIV_PREP(NIV_FP16) }
    NIV_PREP(NIV_BF16)
#undef NIV_PREP
}

// LDS of one workgroup: the operand block (WLDS) and the per-wave staging
// rows, or the level table for the lane-sliced encoding.
template <int P, class S, bool WLDS, int BLOCK> constexpr size_t query_lds()
{
    using O = Ops<P, S>;
    return (WLDS ? (size_t)O::W_BYTES : 0) +
           (S::SL ? (size_t)kLevelBytes : (size_t)(BLOCK / 64) * 64 * O::ROW_DW * 4);
}
constexpr size_t kLdsPerCu = 160 * 1024;

template <int P, class S, bool WLDS, int TB, int BLOCK, bool PROBE = false>
static hipError_t query_t(QueryArgs &a, int blocks_per_cu, hipStream_t st)
{
    constexpr int kWavesPerBlock = BLOCK / 64;
    auto kern = k_query<P, S, WLDS, TB, false, BLOCK, PROBE>;
    constexpr size_t lds = query_lds<P, S, WLDS, BLOCK>();
    static_assert(lds <= kLdsPerCu, "workgroup LDS");
    static int max_blocks = -1;  // resident workgroups per CU for this instantiation
    static int n_cu = 0;
    if (max_blocks < 0) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        int dev = 0;
        e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        int nb = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, BLOCK, lds);
        if (e != hipSuccess) return e;
        max_blocks = nb > 0 ? nb : 1;
    }
    // tiles: each block handles kWavesPerBlock chunks of 64 pixels of one frame
    int64_t t = 0;
    for (int f = 0; f < a.n_frames; ++f) {
        a.f[f].tile_begin = t;
        const int64_t chunks = (a.f[f].count + 63) / 64;
        t += (chunks + kWavesPerBlock - 1) / kWavesPerBlock;
    }
    a.n_tiles = t;
    if (t == 0) return hipSuccess;
    const int per_cu = (blocks_per_cu > 0 && blocks_per_cu < max_blocks) ? blocks_per_cu : max_blocks;
    const int64_t cap = (int64_t)per_cu * n_cu;
    const int64_t blocks = t < cap ? t : cap;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(BLOCK), lds, st, a);
    return hipGetLastError();
}

template <int P, class S, bool WLDS, int TB>
static hipError_t query_b(QueryArgs &a, const LaunchTune &tu, hipStream_t st)
{
    // lane-sliced shapes keep no per-wave rows in LDS: a 768-thread
    // workgroup (three waves per SIMD) fits beside their weights
    if constexpr (S::SL) {
        if (tu.block == 768) return query_t<P, S, WLDS, TB, 768>(a, tu.blocks_per_cu, st);
    }
    // shapes whose 512-thread workgroup would not fit in LDS run 256 threads
    if constexpr (query_lds<P, S, WLDS, 512>() > kLdsPerCu) {
        return query_t<P, S, WLDS, TB, 256>(a, tu.blocks_per_cu, st);
    } else {
        if (tu.block == 256) return query_t<P, S, WLDS, TB, 256>(a, tu.blocks_per_cu, st);
        return query_t<P, S, WLDS, TB, 512>(a, tu.blocks_per_cu, st);
    }
}

// The encoding stage alone (measurement), room model, at the query's launch shape.
template <int P>
static hipError_t probe_b(QueryArgs &a, const LaunchTune &tu, hipStream_t st)
{
    if constexpr (query_lds<P, ShapeRoom, true, 512>() > kLdsPerCu) {
        return query_t<P, ShapeRoom, true, 4, 256, true>(a, tu.blocks_per_cu, st);
    } else {
        if (tu.block == 256) return query_t<P, ShapeRoom, true, 4, 256, true>(a, tu.blocks_per_cu, st);
        return query_t<P, ShapeRoom, true, 4, 512, true>(a, tu.blocks_per_cu, st);
    }
}

hipError_t launch_query_probe(const Model &m, QueryArgs &a, niv_precision prec, const LaunchTune &tu,
                              hipStream_t st)
{
    if (m.kind != kRoom) return hipErrorInvalidValue;
    if (prec == NIV_FP32) return probe_b<NIV_FP32>(a, tu, st);
    if (prec == NIV_FP16) return probe_b<NIV_FP16>(a, tu, st);
    return probe_b<NIV_BF16>(a, tu, st);
}

LaunchTune default_tune(int kind, niv_precision prec)
{
    LaunchTune t;
    // FP32 operands need twice the LDS per wave; smaller workgroups fit more
    // of them; the lane-sliced 6-D field runs three waves per SIMD
    t.block = (prec == NIV_FP32 && kind != kWide6D) ? 256 : (kind == kWide6D && prec != NIV_FP32) ? 768 : 512;
    t.blocks_per_cu = 0;
    t.xcd_order = 1;
    return t;
}

hipError_t launch_query(const Model &m, QueryArgs &a, niv_precision prec, const LaunchTune &tu,
                        hipStream_t st)
{
    switch (m.kind) {
    case kUnitCube:
        if (prec == NIV_FP32) return query_b<NIV_FP32, ShapeUnitCube, true, 4>(a, tu, st);
        if (prec == NIV_FP16) return query_b<NIV_FP16, ShapeUnitCube, true, 4>(a, tu, st);
        return query_b<NIV_BF16, ShapeUnitCube, true, 4>(a, tu, st);
    case kRoom:
        if (prec == NIV_FP32) return query_b<NIV_FP32, ShapeRoom, true, 4>(a, tu, st);
        if (prec == NIV_FP16) return query_b<NIV_FP16, ShapeRoom, true, 4>(a, tu, st);
        return query_b<NIV_BF16, ShapeRoom, true, 4>(a, tu, st);
    case kPE16:
        if (prec == NIV_FP32) return query_b<NIV_FP32, ShapePE<16>, true, 4>(a, tu, st);
        if (prec == NIV_FP16) return query_b<NIV_FP16, ShapePE<16>, true, 4>(a, tu, st);
        return query_b<NIV_BF16, ShapePE<16>, true, 4>(a, tu, st);
    case kPE32:
        if (prec == NIV_FP32) return query_b<NIV_FP32, ShapePE<32>, true, 4>(a, tu, st);
        if (prec == NIV_FP16) return query_b<NIV_FP16, ShapePE<32>, true, 4>(a, tu, st);
        return query_b<NIV_BF16, ShapePE<32>, true, 4>(a, tu, st);
    case kPE64:
        if (prec == NIV_FP32) return query_b<NIV_FP32, ShapePE<64>, true, 4>(a, tu, st);
        if (prec == NIV_FP16) return query_b<NIV_FP16, ShapePE<64>, true, 4>(a, tu, st);
        return query_b<NIV_BF16, ShapePE<64>, true, 4>(a, tu, st);
    case kRoom6D:
        if (prec == NIV_FP32) return query_b<NIV_FP32, ShapeRoom6D, true, 4>(a, tu, st);
        if (prec == NIV_FP16) return query_b<NIV_FP16, ShapeRoom6D, true, 4>(a, tu, st);
        return query_b<NIV_BF16, ShapeRoom6D, true, 4>(a, tu, st);
#define NIV_T1(K, NL)                                                                  \
    case K:                                                                            \
        if (prec == NIV_FP32) return query_b<NIV_FP32, ShapeT1<NL>, true, 4>(a, tu, st);  \
        if (prec == NIV_FP16) return query_b<NIV_FP16, ShapeT1<NL>, true, 4>(a, tu, st);  \
        return query_b<NIV_BF16, ShapeT1<NL>, true, 4>(a, tu, st);
    NIV_T1(kT1L2, 2)
    NIV_T1(kT1L4, 4)
    NIV_T1(kT1L6, 6)
    NIV_T1(kT1L8, 8)
#undef NIV_T1
    default:  // lane-sliced encoding: the LDS holds the whole weight block
        if (prec == NIV_FP32) return query_b<NIV_FP32, ShapeWide6DFor<NIV_FP32>, false, 2>(a, tu, st);
        if (prec == NIV_FP16) return query_b<NIV_FP16, ShapeWide6D, true, 2>(a, tu, st);
        return query_b<NIV_BF16, ShapeWide6D, true, 2>(a, tu, st);
    }
}

// Grid entries the query's encoding reads (inspection): one lane per point,
// the position clamped to the box as in k_query, then the same encoding
// function the fused kernel runs for this model and precision, which
// records each corner's entry.  Non-finite positions give 0xFFFFFFFF.
template <int P, bool F32C, bool SLICED, bool F4 = false>
__global__ __launch_bounds__(256) void k_trace_corners(const uint8_t *__restrict__ model,
                                                       uint64_t grid_off, uint32_t grid_bytes,
                                                       uint32_t hmask, const Box6 box,
                                                       const float *__restrict__ pos, int64_t count,
                                                       int n_levels, uint32_t *__restrict__ out)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(model + grid_off), (short)0, (int)grid_bytes, 0x00020000);
    const LevelConst *lvs = reinterpret_cast<const LevelConst *>(model);
    const float px = pos[3 * q], py = pos[3 * q + 1], pz = pos[3 * q + 2];
    uint32_t *o = out + q * n_levels * 8;
    if (!(__builtin_isfinite(px) && __builtin_isfinite(py) && __builtin_isfinite(pz))) {
        for (int k = 0; k < n_levels * 8; ++k) o[k] = 0xFFFFFFFFu;
        return;
    }
    double p[3] = {px, py, pz};
    for (int c = 0; c < 3; ++c)
        p[c] = p[c] < box.v[c] ? box.v[c] : (p[c] > box.v[3 + c] ? box.v[3 + c] : p[c]);
    const float pf[3] = {(float)p[0], (float)p[1], (float)p[2]};
    for (int l = 0; l < n_levels; ++l) {
        f2 f;
        if constexpr (F4) {
            const f4 f4v = encode_level_buf4<P, F32C, true>(lvs[l], p, hmask, rsrc, pf, o + 8 * l);
            f = (f2){f4v.x, f4v.y};
        } else if constexpr (SLICED) {
            const LevelRegs lc = load_level(lvs + l);
            LevelFetch<P> lf;
            level_issue_vec<P, true>(lc, p, hmask, rsrc, lf, o + 8 * l);
            f = level_blend<P>(lf);
        } else {
            if constexpr (F32C) {
                f = encode_level_buf<P, F32C, true>(lvs[l], p, hmask, rsrc, pf, o + 8 * l);
            } else {
                LevelFetch<P> lf;
                level_issue<P, false, true>(lvs[l], p, hmask, rsrc, pf, lf, o + 8 * l);
                f = level_blend<P>(lf);
            }
        }
        (void)f;
    }
}

hipError_t launch_trace_corners(const Model &m, niv_precision prec, bool train, const void *model,
                                const float *pos, int64_t count, uint32_t *out, hipStream_t st)
{
    Box6 box;
    for (int c = 0; c < 3; ++c) {
        box.v[c] = m.cfg.aabb_min[c];
        box.v[3 + c] = m.cfg.aabb_max[c];
    }
    const OpLayout L = op_layout(m.kind, prec);
    const uint64_t goff = (uint64_t)L.grid_off;
    const uint32_t gbytes = (uint32_t)(m.n_grid_values * (prec == NIV_FP32 ? 4 : 2));
    const uint32_t hmask = (uint32_t)((int64_t(1) << m.cfg.log2_T) - 1);
    const uint8_t *md = static_cast<const uint8_t *>(model);
    const dim3 grid((unsigned)((count + 255) / 256)), blk(256);
    const int nl = m.cfg.n_levels;
    const bool sliced = m.kind == kWide6D && prec != NIV_FP32;
    if (m.cfg.n_features == 4) {
        if (prec == NIV_FP32)
            hipLaunchKernelGGL((k_trace_corners<NIV_FP32, false, false, true>), grid, blk, 0, st, md, goff,
                               gbytes, hmask, box, pos, count, nl, out);
        else if (prec == NIV_FP16)
            hipLaunchKernelGGL((k_trace_corners<NIV_FP16, true, false, true>), grid, blk, 0, st, md, goff,
                               gbytes, hmask, box, pos, count, nl, out);
        else
            hipLaunchKernelGGL((k_trace_corners<NIV_BF16, false, false, true>), grid, blk, 0, st, md, goff,
                               gbytes, hmask, box, pos, count, nl, out);
    } else if (prec == NIV_FP32)
        hipLaunchKernelGGL((k_trace_corners<NIV_FP32, false, false>), grid, blk, 0, st, md, goff, gbytes,
                           hmask, box, pos, count, nl, out);
    else if (sliced && prec == NIV_FP16)
        hipLaunchKernelGGL((k_trace_corners<NIV_FP16, false, true>), grid, blk, 0, st, md, goff, gbytes,
                           hmask, box, pos, count, nl, out);
    else if (sliced)
        hipLaunchKernelGGL((k_trace_corners<NIV_BF16, false, true>), grid, blk, 0, st, md, goff, gbytes,
                           hmask, box, pos, count, nl, out);
    else if (prec == NIV_FP16 && !train)
        hipLaunchKernelGGL((k_trace_corners<NIV_FP16, true, false>), grid, blk, 0, st, md, goff, gbytes,
                           hmask, box, pos, count, nl, out);
    else if (prec == NIV_FP16)
        hipLaunchKernelGGL((k_trace_corners<NIV_FP16, false, false>), grid, blk, 0, st, md, goff, gbytes,
                           hmask, box, pos, count, nl, out);
    else
        hipLaunchKernelGGL((k_trace_corners<NIV_BF16, false, false>), grid, blk, 0, st, md, goff, gbytes,
                           hmask, box, pos, count, nl, out);
    return hipGetLastError();
}

__global__ void k_fill_u32(uint32_t *__restrict__ p, int n)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = 0u;
}

hipError_t launch_zero_u32(uint32_t *p, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_u32, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

}  // namespace niv
