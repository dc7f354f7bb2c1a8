// Fused per-pixel Neural Irradiance Volume query for gfx950 (CDNA4).
//
// One launch evaluates E_theta(x, n) for every pixel of a G-buffer (Sec. 4.4)
// and shades it with albedo * E / pi (Eq. 2):
//   1. each lane loads one pixel (coalesced) and builds its input vector:
//      per level the cell, the 8 corner indices (dense or spatially hashed),
//      8 gathers and a trilinear blend in FP32 (Sec. 3.1); 16 real SH of the
//      normal; the frequency code of the frame's scene variables (Sec. 6);
//   2. the wave's 64 input vectors go through a per-wave LDS block into the
//      operand layout of the matrix cores;
//   3. the MLP runs on MFMA with FP32 accumulation, four 16-pixel tiles per
//      wave, weights resident in LDS;
//   4. each lane writes its pixel's E, albedo * E / pi and flags.
//
// Operand layout.  A layer y = W x is computed transposed, D = W * X^T, with
// the weights as the A operand (16 output rows) and 16 pixels as the B
// operand columns.  A 16x16 accumulator leaves lane (g = lane/16, j =
// lane%16) holding rows 4g..4g+3 of pixel j.  The contraction index of the
// next layer can be permuted freely as long as A and B agree, so the prepared
// weights are stored with their input columns permuted such that a lane's own
// accumulator values, after ReLU and rounding, ARE its next B operand: no
// cross-lane traffic between layers.
#include <hip/hip_runtime.h>
#include <string.h>

#include "niv_internal.h"

namespace niv {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));
typedef uint32_t u2 __attribute__((ext_vector_type(2)));

// Scalar bit casts.  They take their operand by value: this compiler reads
// element 0 when __builtin_bit_cast is applied directly to an element of an
// ext_vector_type value (v.y, v.z, ...), so vector elements are first copied
// into a scalar.
__device__ inline uint32_t f2u(float x) { return __builtin_bit_cast(uint32_t, x); }
__device__ inline float u2f(uint32_t x) { return __builtin_bit_cast(float, x); }

// ---------------------------------------------------------------- precision
template <int P> struct Prec;

template <> struct Prec<NIV_FP16> {
    static constexpr int ES = 2;    // bytes per element
    static constexpr int EPO = 8;   // elements per lane of a full operand
    __device__ static f4 mma(u4 a, u4 b, f4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a),
                                                      __builtin_bit_cast(h8, b), c, 0, 0, 0);
    }
    __device__ static f4 mma_half(u2 a, u2 b, f4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(h4, a),
                                                     __builtin_bit_cast(h4, b), c, 0, 0, 0);
    }
    __device__ static uint32_t pack(float x, float y) {
        h2 v = __builtin_convertvector((f2){x, y}, h2);
        return __builtin_bit_cast(uint32_t, v);
    }
    __device__ static f2 unpack(uint32_t w) {
        return __builtin_convertvector(__builtin_bit_cast(h2, w), f2);
    }
};

template <> struct Prec<NIV_BF16> {
    static constexpr int ES = 2;
    static constexpr int EPO = 8;
    __device__ static f4 mma(u4 a, u4 b, f4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a),
                                                       __builtin_bit_cast(bf8, b), c, 0, 0, 0);
    }
    __device__ static f4 mma_half(u2 a, u2 b, f4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4, a),
                                                         __builtin_bit_cast(s4, b), c, 0, 0, 0);
    }
    __device__ static uint32_t pack(float x, float y) {
        bf2 v = __builtin_convertvector((f2){x, y}, bf2);
        return __builtin_bit_cast(uint32_t, v);
    }
    __device__ static f2 unpack(uint32_t w) {
        // a bf16 is the upper half of the float with the same bits
        return (f2){__builtin_bit_cast(float, w << 16), __builtin_bit_cast(float, w & 0xffff0000u)};
    }
    // x = hi + lo with hi = bf16(x), lo = bf16(x - hi): the pair carries 16
    // significant bits, so BF16 operands lose little to rounding.
    __device__ static uint32_t pack_lo(float x, float y, uint32_t hi) {
        f2 h = unpack(hi);
        return pack(x - h.x, y - h.y);
    }
};

template <> struct Prec<NIV_FP32> {
    static constexpr int ES = 4;
    static constexpr int EPO = 1;
    __device__ static f4 mma1(float a, float b, f4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

// ---------------------------------------------------------------- shapes
template <int L_, int NEX_, int W_, int H_> struct Shape {
    static constexpr int L = L_, NEX = NEX_, W = W_, H = H_;
    static constexpr int DIN = 2 * L + 16 + 16 * NEX;  // F = 2, 16 SH, 16 per variable
    static constexpr int KLG = DIN / 4;                // input slots per lane group
    static constexpr int NOB = W / 16;                 // 16-row output blocks
    static_assert(DIN % 16 == 0, "input width must be a multiple of 16");
    static_assert(L % 4 == 0 && W % 32 == 0, "shape");
};

using ShapeUnitCube = Shape<8, 0, 64, 2>;
using ShapeRoom = Shape<16, 0, 64, 3>;
using ShapeWide6D = Shape<16, 1, 128, 4>;

// Byte layout of the operand block of a prepared model.
template <int P, class S> struct Ops {
    static constexpr bool F32 = (P == NIV_FP32);
    static constexpr int ES = F32 ? 4 : 2;
    static constexpr int EPO = F32 ? 1 : 8;
    static constexpr int OPB = 64 * EPO * ES;                       // full operand
    static constexpr int OPS = 64 * 4 * ES;                         // half-depth operand
    static constexpr int L0_FULL = F32 ? S::KLG : S::KLG / 8;       // per output block
    static constexpr int L0_HALF = F32 ? 0 : (S::KLG % 8) / 4;
    static constexpr int L0_OB = L0_FULL * OPB + L0_HALF * OPS;    // bytes per output block
    static constexpr int L0_BYTES = S::NOB * L0_OB;
    static constexpr int HOPS = F32 ? S::W / 4 : S::W / 32;         // operands per block row
    static constexpr int HID_BYTES = S::NOB * HOPS * OPB;
    static constexpr int OUT_BYTES = 4 * HOPS * OPB;
    static constexpr int W_BYTES = L0_BYTES + (S::H - 1) * HID_BYTES + OUT_BYTES;
    static constexpr int N_OPS = S::NOB * (L0_FULL + L0_HALF) + (S::H - 1) * S::NOB * HOPS + 4 * HOPS;
    // BF16 operands are split into hi + lo parts (two products each)
    static constexpr int NS = (P == NIV_BF16) ? 2 : 1;
    static constexpr int PART_DW = S::DIN * ES / 4;                 // one part of a row
    // staging row (one pixel's input vector) in dwords, padded against bank conflicts
    static constexpr int ROW_DW = NS * PART_DW + (F32 ? 4 : 2);
    static constexpr int LANE_DW = S::KLG * ES / 4;                 // dwords a lane group reads
};

__host__ __device__ constexpr int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

// ---------------------------------------------------------------- prepare
// Source parameter index of element `e` of lane `lane` of operand `op`, or -1
// for a zero.  Parameters: [grid][W_0 (W x DIN)][W_1..W_{H-1} (W x W)][W_H (3 x W)].
template <int P, class S>
__device__ int64_t operand_source(int op, int lane, int e, int64_t n_grid, int n_out)
{
    using O = Ops<P, S>;
    const int i = lane & 15, g = lane >> 4;
    const int64_t w0 = n_grid;
    const int64_t wh = w0 + (int64_t)S::W * S::DIN;
    const int64_t wo = wh + (int64_t)(S::H - 1) * S::W * S::W;
    const int n0 = S::NOB * (O::L0_FULL + O::L0_HALF);
    const int nh = (S::H - 1) * S::NOB * O::HOPS;
    if (op < n0) {  // layer 0: [ob][chunk]
        int ob = op / (O::L0_FULL + O::L0_HALF), c = op % (O::L0_FULL + O::L0_HALF);
        int slot = O::F32 ? c : (c < O::L0_FULL ? c * 8 + e : O::L0_FULL * 8 + e);
        int row = 16 * ob + i, col = S::KLG * g + slot;
        return w0 + (int64_t)row * S::DIN + col;
    }
    op -= n0;
    int col;
    auto hidden_col = [&](int kb) {
        return O::F32 ? 16 * (kb / 4) + 4 * g + (kb % 4)
                      : 16 * (2 * kb + e / 4) + 4 * g + (e % 4);
    };
    if (op < nh) {  // hidden layers: [layer][ob][kb]
        int layer = op / (S::NOB * O::HOPS);
        int r = op % (S::NOB * O::HOPS);
        int ob = r / O::HOPS, kb = r % O::HOPS;
        col = hidden_col(kb);
        int row = 16 * ob + i;
        return wh + (int64_t)layer * S::W * S::W + (int64_t)row * S::W + col;
    }
    op -= nh;  // output layer: [tile][kb]; tile t occupies rows 4t..4t+n_out-1
    int t = op / O::HOPS, kb = op % O::HOPS;
    col = hidden_col(kb);
    if ((i >> 2) != t || (i & 3) >= n_out) return -1;
    return wo + (int64_t)(i & 3) * S::W + col;
}

// Byte offset and element count of operand `op`.
template <int P, class S>
__device__ void operand_place(int op, int64_t *off, int *n_elem)
{
    using O = Ops<P, S>;
    const int n0 = S::NOB * (O::L0_FULL + O::L0_HALF);
    if (op < n0) {
        int ob = op / (O::L0_FULL + O::L0_HALF), c = op % (O::L0_FULL + O::L0_HALF);
        *off = (int64_t)ob * O::L0_OB + (int64_t)c * O::OPB;
        *n_elem = (c < O::L0_FULL) ? O::EPO : 4;
        return;
    }
    *off = O::L0_BYTES + (int64_t)(op - n0) * O::OPB;
    *n_elem = O::EPO;
}

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

// ---------------------------------------------------------------- encoding
// Real SH of degree <= 3 with the Condon-Shortley phase, Cartesian form of
// the unit normal (x, y, z); index l^2 + l + m.
__device__ inline void sh16(float x, float y, float z, float *o)
{
    const float xx = x * x, yy = y * y, zz = z * z;
    o[0] = 0.28209479177387814f;
    o[1] = -0.4886025119029199f * y;
    o[2] = 0.4886025119029199f * z;
    o[3] = -0.4886025119029199f * x;
    o[4] = 1.0925484305920792f * x * y;
    o[5] = -1.0925484305920792f * y * z;
    o[6] = 0.31539156525252005f * (3.0f * zz - 1.0f);
    o[7] = -1.0925484305920792f * x * z;
    o[8] = 0.5462742152960396f * (xx - yy);
    o[9] = -0.5900435899266435f * y * (3.0f * xx - yy);
    o[10] = 2.890611442640554f * x * y * z;
    o[11] = -0.4570457994644658f * y * (5.0f * zz - 1.0f);
    o[12] = 0.3731763325901154f * z * (5.0f * zz - 3.0f);
    o[13] = -0.4570457994644658f * x * (5.0f * zz - 1.0f);
    o[14] = 1.445305721320277f * z * (xx - yy);
    o[15] = -0.5900435899266435f * x * (xx - 3.0f * yy);
}

template <int P>
__device__ inline f2 load_latent(const uint8_t *grid, uint32_t entry)
{
    if constexpr (P == NIV_FP32) {
        return reinterpret_cast<const f2 *>(grid)[entry];
    } else {
        return Prec<P>::unpack(reinterpret_cast<const uint32_t *>(grid)[entry]);
    }
}

// Trilinear blend of one level (Sec. 3.1).  Returns the F = 2 features.
template <int P, class LV>
__device__ inline f2 encode_level(const LV &lv, const double p[3], uint32_t hmask,
                                  const uint8_t *grid)
{
    int32_t ci[3];
    float fr[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double s = __builtin_fma(p[a], lv.k[a], lv.o[a]);
        int32_t c = (int32_t)s;               // s > -1, so truncation = floor clamped at 0
        c = c < lv.nm1 ? c : lv.nm1;
        ci[a] = c;
        fr[a] = (float)(s - (double)c);
    }
    uint32_t idx[8];
    if (lv.dense) {
        uint32_t b = (uint32_t)ci[0] + lv.s1 * ((uint32_t)ci[1] + lv.s1 * (uint32_t)ci[2]) + lv.off;
        idx[0] = b;           idx[1] = b + 1;
        idx[2] = b + lv.s1;   idx[3] = b + lv.s1 + 1;
        idx[4] = b + lv.s2;   idx[5] = b + lv.s2 + 1;
        idx[6] = b + lv.s2 + lv.s1;  idx[7] = b + lv.s2 + lv.s1 + 1;
    } else {
        uint32_t x0 = (uint32_t)ci[0], x1 = x0 + 1;
        uint32_t y0 = (uint32_t)ci[1] * kPrime1, y1 = y0 + kPrime1;
        uint32_t z0 = (uint32_t)ci[2] * kPrime2, z1 = z0 + kPrime2;
        // x < T on every hashed level (checked on the host), so the mask
        // can be applied to the y/z part alone.
        uint32_t t00 = (y0 ^ z0) & hmask, t10 = (y1 ^ z0) & hmask;
        uint32_t t01 = (y0 ^ z1) & hmask, t11 = (y1 ^ z1) & hmask;
        idx[0] = (x0 ^ t00) + lv.off;  idx[1] = (x1 ^ t00) + lv.off;
        idx[2] = (x0 ^ t10) + lv.off;  idx[3] = (x1 ^ t10) + lv.off;
        idx[4] = (x0 ^ t01) + lv.off;  idx[5] = (x1 ^ t01) + lv.off;
        idx[6] = (x0 ^ t11) + lv.off;  idx[7] = (x1 ^ t11) + lv.off;
    }
    f2 v[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) v[c] = load_latent<P>(grid, idx[c]);
    const float wx1 = fr[0], wx0 = 1.0f - fr[0];
    const float wy1 = fr[1], wy0 = 1.0f - fr[1];
    const float wz1 = fr[2], wz0 = 1.0f - fr[2];
    const float w00 = wy0 * wz0, w10 = wy1 * wz0, w01 = wy0 * wz1, w11 = wy1 * wz1;
    const float w[8] = {wx0 * w00, wx1 * w00, wx0 * w10, wx1 * w10,
                        wx0 * w01, wx1 * w01, wx0 * w11, wx1 * w11};
    f2 acc = {0.0f, 0.0f};
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        acc.x = __builtin_fmaf(w[c], v[c].x, acc.x);
        acc.y = __builtin_fmaf(w[c], v[c].y, acc.y);
    }
    return acc;
}

// ---------------------------------------------------------------- fused query
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / 64;

template <int P, class S, bool WLDS, int TB>
__global__ __launch_bounds__(kBlock) void k_query(const QueryArgs a)
{
    using O = Ops<P, S>;
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const uint8_t *model = a.model + kLevelBytes;   // operand block
    const uint8_t *grid = a.model + a.grid_off;

    // Operand block -> LDS, once per workgroup.
    const uint8_t *wsrc = model;
    uint32_t *stage;
    if constexpr (WLDS) {
        const u4 *src = reinterpret_cast<const u4 *>(model);
        u4 *dst = reinterpret_cast<u4 *>(smem);
        for (int k = threadIdx.x; k < O::W_BYTES / 16; k += kBlock) dst[k] = src[k];
        __syncthreads();
        wsrc = smem;
        stage = reinterpret_cast<uint32_t *>(smem + O::W_BYTES) + wave * 64 * O::ROW_DW;
    } else {
        stage = reinterpret_cast<uint32_t *>(smem) + wave * 64 * O::ROW_DW;
    }

    const int64_t n_chunks = (a.count + 63) / 64;
    const int64_t wave_id = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    const int64_t n_waves = (int64_t)gridDim.x * kWavesPerBlock;
    const int g = lane >> 4, j = lane & 15;

    // Frequency code of the frame's scene variables (uniform over the launch).
    float gam[16 * (S::NEX > 0 ? S::NEX : 1)];
    if constexpr (S::NEX > 0) {
#pragma unroll
        for (int e = 0; e < S::NEX; ++e)
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                float t = a.extra[e] * (float)(1 << k);   // exact scaling by 2^k
                gam[16 * e + 2 * k] = sinpif(t);
                gam[16 * e + 2 * k + 1] = cospif(t);
            }
    }

    for (int64_t chunk = wave_id; chunk < n_chunks; chunk += n_waves) {
        // Re-read the level constants from the argument segment every chunk
        // (scalar loads) instead of keeping 16 levels of them in registers.
        uint32_t zero = 0;
        asm volatile("" : "+s"(zero));
        // constant address space: uniform, read-only, so scalar loads
        typedef const __attribute__((address_space(4))) LevelConst *ConstLevels;
        ConstLevels lvs = (ConstLevels)(a.model + zero);
        const uint8_t *wop = wsrc;
        if constexpr (!WLDS) {
            // same for operands read from global memory: load them where used
            wop = a.model + kLevelBytes + zero;
        }
        const int64_t q = chunk * 64 + lane;
        const bool live = q < a.count;
        // ---- 1. load and encode this lane's pixel
        float px = 0.f, py = 0.f, pz = 0.f, nx = 0.f, ny = 0.f, nz = 0.f;
        bool on = false;
        if (live) {
            on = a.mask ? (a.mask[q] != 0) : true;
            if (on) {
                px = a.pos[3 * q]; py = a.pos[3 * q + 1]; pz = a.pos[3 * q + 2];
                nx = a.nrm[3 * q]; ny = a.nrm[3 * q + 1]; nz = a.nrm[3 * q + 2];
            }
        }
        bool bad = !(__builtin_isfinite(px) && __builtin_isfinite(py) && __builtin_isfinite(pz) &&
                     __builtin_isfinite(nx) && __builtin_isfinite(ny) && __builtin_isfinite(nz));
        if constexpr (S::NEX > 0) {
#pragma unroll
            for (int e = 0; e < S::NEX; ++e) bad |= !__builtin_isfinite(a.extra[e]);
        }
        // scale by the largest component first so that tiny or huge normals
        // normalise without underflow or overflow
        const float nm = fmaxf(fabsf(nx), fmaxf(fabsf(ny), fabsf(nz)));
        bad |= !(nm > 0.0f);
        const float ns = (nm > 0.0f) ? 1.0f / nm : 0.0f;
        nx *= ns; ny *= ns; nz *= ns;
        const float n2 = nx * nx + ny * ny + nz * nz;
        const bool work = on && !bad;
        uint32_t flags = (on && bad) ? 2u : 0u;
        double p[3] = {px, py, pz};
        bool outside = false;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            outside |= (p[c] < a.lo[c]) | (p[c] > a.hi[c]);
            p[c] = p[c] < a.lo[c] ? a.lo[c] : (p[c] > a.hi[c] ? a.hi[c] : p[c]);
        }
        if (work && outside) flags |= 1u;

        uint32_t *row = stage + lane * O::ROW_DW;
        if (work) {
            if constexpr (P == NIV_FP32) {
#pragma unroll
                for (int l = 0; l < S::L; ++l) {
                    f2 f = encode_level<P>(lvs[l], p, a.hash_mask, grid);
                    row[2 * l] = f2u(f.x);
                    row[2 * l + 1] = f2u(f.y);
                }
            } else {
#pragma unroll
                for (int l = 0; l < S::L; ++l) {
                    f2 f = encode_level<P>(lvs[l], p, a.hash_mask, grid);
                    row[l] = Prec<P>::pack(f.x, f.y);
                    if constexpr (O::NS == 2) row[O::PART_DW + l] = Prec<P>::pack_lo(f.x, f.y, row[l]);
                }
            }
            const float rn = __builtin_amdgcn_rsqf(n2);
            float sh[16];
            sh16(nx * rn, ny * rn, nz * rn, sh);
            constexpr int base = (P == NIV_FP32) ? 2 * S::L : S::L;
            if constexpr (P == NIV_FP32) {
#pragma unroll
                for (int k = 0; k < 16; ++k) row[base + k] = f2u(sh[k]);
#pragma unroll
                for (int k = 0; k < 16 * S::NEX; ++k)
                    row[base + 16 + k] = f2u(gam[k]);
            } else {
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    row[base + k] = Prec<P>::pack(sh[2 * k], sh[2 * k + 1]);
                    if constexpr (O::NS == 2)
                        row[O::PART_DW + base + k] = Prec<P>::pack_lo(sh[2 * k], sh[2 * k + 1], row[base + k]);
                }
#pragma unroll
                for (int k = 0; k < 8 * S::NEX; ++k) {
                    row[base + 8 + k] = Prec<P>::pack(gam[2 * k], gam[2 * k + 1]);
                    if constexpr (O::NS == 2)
                        row[O::PART_DW + base + 8 + k] =
                            Prec<P>::pack_lo(gam[2 * k], gam[2 * k + 1], row[base + 8 + k]);
                }
            }
        } else {
            // no bias anywhere: an all-zero input gives E = 0
#pragma unroll
            for (int k = 0; k < O::NS * O::PART_DW; ++k) row[k] = 0u;
        }
        if (a.out_inputs && live) {
            float *dst = a.out_inputs + q * S::DIN;
            if constexpr (P == NIV_FP32) {
#pragma unroll
                for (int k = 0; k < S::DIN; ++k) dst[k] = u2f(row[k]);
            } else {
#pragma unroll
                for (int k = 0; k < S::DIN / 2; ++k) {
                    f2 v = Prec<P>::unpack(row[k]);
                    if constexpr (O::NS == 2) {
                        f2 w = Prec<P>::unpack(row[O::PART_DW + k]);
                        v.x += w.x;
                        v.y += w.y;
                    }
                    dst[2 * k] = v.x;
                    dst[2 * k + 1] = v.y;
                }
            }
        }
        // LDS accesses of one wave complete in order; the fence keeps the
        // compiler from moving the operand reads above the row writes.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        // ---- 2/3. MLP on the matrix cores, TB tiles of 16 pixels at a time
        f4 acc_out = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t0 = 0; t0 < 4; t0 += TB) {
            f4 acc[TB][S::NOB];
            // layer 0
            if constexpr (P == NIV_FP32) {
                float b0[TB][S::KLG];
#pragma unroll
                for (int t = 0; t < TB; ++t) {
                    const uint32_t *r = stage + (16 * (t0 + t) + j) * O::ROW_DW + O::LANE_DW * g;
#pragma unroll
                    for (int k = 0; k < S::KLG; k += 4) {
                        f4 v = *reinterpret_cast<const f4 *>(r + k);
                        b0[t][k] = v.x;
                        b0[t][k + 1] = v.y;
                        b0[t][k + 2] = v.z;
                        b0[t][k + 3] = v.w;
                    }
                }
#pragma unroll
                for (int ob = 0; ob < S::NOB; ++ob) {
#pragma unroll
                    for (int t = 0; t < TB; ++t) acc[t][ob] = (f4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int c = 0; c < S::KLG; ++c) {
                        float av = reinterpret_cast<const float *>(wop + ob * O::L0_OB + c * O::OPB)[lane];
#pragma unroll
                        for (int t = 0; t < TB; ++t) acc[t][ob] = Prec<P>::mma1(av, b0[t][c], acc[t][ob]);
                    }
                }
            } else {
                uint32_t b0[O::NS][TB][O::LANE_DW];
#pragma unroll
                for (int sp = 0; sp < O::NS; ++sp)
#pragma unroll
                for (int t = 0; t < TB; ++t) {
                    const uint32_t *r = stage + (16 * (t0 + t) + j) * O::ROW_DW + sp * O::PART_DW +
                                        O::LANE_DW * g;
#pragma unroll
                    for (int k = 0; k < O::LANE_DW; k += 2) {
                        u2 v = *reinterpret_cast<const u2 *>(r + k);
                        b0[sp][t][k] = v.x;
                        b0[sp][t][k + 1] = v.y;
                    }
                }
#pragma unroll
                for (int ob = 0; ob < S::NOB; ++ob) {
#pragma unroll
                    for (int t = 0; t < TB; ++t) acc[t][ob] = (f4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int c = 0; c < O::L0_FULL; ++c) {
                        u4 av = reinterpret_cast<const u4 *>(wop + ob * O::L0_OB + c * O::OPB)[lane];
#pragma unroll
                        for (int sp = 0; sp < O::NS; ++sp)
#pragma unroll
                        for (int t = 0; t < TB; ++t) {
                            u4 bv = {b0[sp][t][4 * c], b0[sp][t][4 * c + 1], b0[sp][t][4 * c + 2],
                                     b0[sp][t][4 * c + 3]};
                            acc[t][ob] = Prec<P>::mma(av, bv, acc[t][ob]);
                        }
                    }
                    if constexpr (O::L0_HALF) {
                        u2 av = reinterpret_cast<const u2 *>(wop + ob * O::L0_OB + O::L0_FULL * O::OPB)[lane];
#pragma unroll
                        for (int sp = 0; sp < O::NS; ++sp)
#pragma unroll
                        for (int t = 0; t < TB; ++t) {
                            u2 bv = {b0[sp][t][4 * O::L0_FULL], b0[sp][t][4 * O::L0_FULL + 1]};
                            acc[t][ob] = Prec<P>::mma_half(av, bv, acc[t][ob]);
                        }
                    }
                }
            }
            // hidden layers and output: the accumulator of a lane is its next operand
#pragma unroll
            for (int layer = 1; layer <= S::H; ++layer) {
                const bool last = (layer == S::H);
                const uint8_t *lw = last ? wop + O::L0_BYTES + (S::H - 1) * O::HID_BYTES
                                         : wop + O::L0_BYTES + (layer - 1) * O::HID_BYTES;
                if constexpr (P == NIV_FP32) {
                    float bh[TB][S::W / 4];
#pragma unroll
                    for (int t = 0; t < TB; ++t)
#pragma unroll
                        for (int ob = 0; ob < S::NOB; ++ob) {
                            bh[t][4 * ob] = fmaxf(acc[t][ob].x, 0.f);
                            bh[t][4 * ob + 1] = fmaxf(acc[t][ob].y, 0.f);
                            bh[t][4 * ob + 2] = fmaxf(acc[t][ob].z, 0.f);
                            bh[t][4 * ob + 3] = fmaxf(acc[t][ob].w, 0.f);
                        }
                    if (last) {
#pragma unroll
                        for (int t = 0; t < TB; ++t)
#pragma unroll
                            for (int c = 0; c < O::HOPS; ++c) {
                                float av = reinterpret_cast<const float *>(lw + ((t0 + t) * O::HOPS + c) * O::OPB)[lane];
                                acc_out = Prec<P>::mma1(av, bh[t][c], acc_out);
                            }
                    } else {
#pragma unroll
                        for (int ob = 0; ob < S::NOB; ++ob) {
#pragma unroll
                            for (int t = 0; t < TB; ++t) acc[t][ob] = (f4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
                            for (int c = 0; c < O::HOPS; ++c) {
                                float av = reinterpret_cast<const float *>(lw + (ob * O::HOPS + c) * O::OPB)[lane];
#pragma unroll
                                for (int t = 0; t < TB; ++t) acc[t][ob] = Prec<P>::mma1(av, bh[t][c], acc[t][ob]);
                            }
                        }
                    }
                } else {
                    uint32_t bh[O::NS][TB][S::W / 8];
#pragma unroll
                    for (int t = 0; t < TB; ++t)
#pragma unroll
                        for (int ob = 0; ob < S::NOB; ++ob) {
                            const float r0 = fmaxf(acc[t][ob].x, 0.f), r1 = fmaxf(acc[t][ob].y, 0.f);
                            const float r2 = fmaxf(acc[t][ob].z, 0.f), r3 = fmaxf(acc[t][ob].w, 0.f);
                            bh[0][t][2 * ob] = Prec<P>::pack(r0, r1);
                            bh[0][t][2 * ob + 1] = Prec<P>::pack(r2, r3);
                            if constexpr (O::NS == 2) {
                                bh[O::NS - 1][t][2 * ob] = Prec<P>::pack_lo(r0, r1, bh[0][t][2 * ob]);
                                bh[O::NS - 1][t][2 * ob + 1] = Prec<P>::pack_lo(r2, r3, bh[0][t][2 * ob + 1]);
                            }
                        }
                    if (last) {
#pragma unroll
                        for (int t = 0; t < TB; ++t)
#pragma unroll
                            for (int kb = 0; kb < O::HOPS; ++kb) {
                                u4 av = reinterpret_cast<const u4 *>(lw + ((t0 + t) * O::HOPS + kb) * O::OPB)[lane];
#pragma unroll
                                for (int sp = 0; sp < O::NS; ++sp) {
                                    u4 bv = {bh[sp][t][4 * kb], bh[sp][t][4 * kb + 1], bh[sp][t][4 * kb + 2],
                                             bh[sp][t][4 * kb + 3]};
                                    acc_out = Prec<P>::mma(av, bv, acc_out);
                                }
                            }
                    } else {
#pragma unroll
                        for (int ob = 0; ob < S::NOB; ++ob) {
#pragma unroll
                            for (int t = 0; t < TB; ++t) acc[t][ob] = (f4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
                            for (int kb = 0; kb < O::HOPS; ++kb) {
                                u4 av = reinterpret_cast<const u4 *>(lw + (ob * O::HOPS + kb) * O::OPB)[lane];
#pragma unroll
                                for (int sp = 0; sp < O::NS; ++sp)
#pragma unroll
                                for (int t = 0; t < TB; ++t) {
                                    u4 bv = {bh[sp][t][4 * kb], bh[sp][t][4 * kb + 1], bh[sp][t][4 * kb + 2],
                                             bh[sp][t][4 * kb + 3]};
                                    acc[t][ob] = Prec<P>::mma(av, bv, acc[t][ob]);
                                }
                            }
                        }
                    }
                }
            }
        }
        // ---- 4. lane (g, j) holds rows 4g..4g+2 = RGB of pixel 16g + j = this lane's pixel
        if (live) {
            float E0 = work ? acc_out.x : 0.f, E1 = work ? acc_out.y : 0.f, E2 = work ? acc_out.z : 0.f;
            if (work && !(__builtin_isfinite(E0) && __builtin_isfinite(E1) && __builtin_isfinite(E2)))
                flags |= 4u;
            a.out_E[3 * q] = E0;
            a.out_E[3 * q + 1] = E1;
            a.out_E[3 * q + 2] = E2;
            if (a.out_L) {
                const float ip = 0.3183098861837907f;  // 1/pi
                float r0 = 0.f, r1 = 0.f, r2 = 0.f;
                if (on) { r0 = a.albedo[3 * q]; r1 = a.albedo[3 * q + 1]; r2 = a.albedo[3 * q + 2]; }
                a.out_L[3 * q] = r0 * E0 * ip;
                a.out_L[3 * q + 1] = r1 * E1 * ip;
                a.out_L[3 * q + 2] = r2 * E2 * ip;
            }
            if (a.out_flags) a.out_flags[q] = (uint8_t)flags;
        }
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
    default: return layout_of<P, ShapeWide6D>();                        \
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
    int64_t blocks = (m.n_grid_values + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL((k_prepare_grid<P>), dim3((unsigned)blocks), dim3(256), 0, st, params,
                       out + kLevelBytes + align256(O::W_BYTES), m.n_grid_values);
    return hipGetLastError();
}

hipError_t launch_prepare(const Model &m, const float *params, void *prepared,
                          niv_precision prec, hipStream_t st)
{
#define NIV_PREP(P)                                                                      \
    switch (m.kind) {                                                                    \
    case kUnitCube: return prepare_t<P, ShapeUnitCube>(m, params, prepared, st);        \
    case kRoom: return prepare_t<P, ShapeRoom>(m, params, prepared, st);                \
    default: return prepare_t<P, ShapeWide6D>(m, params, prepared, st);                 \
    }
    if (prec == NIV_FP32) { NIV_PREP(NIV_FP32) }
    if (prec == NIV_FP16) { NIV_PREP(NIV_FP16) }
    NIV_PREP(NIV_BF16)
#undef NIV_PREP
}

template <int P, class S, bool WLDS, int TB>
static hipError_t query_t(const QueryArgs &a, hipStream_t st)
{
    using O = Ops<P, S>;
    auto kern = k_query<P, S, WLDS, TB>;
    const size_t lds = (WLDS ? O::W_BYTES : 0) + (size_t)kWavesPerBlock * 64 * O::ROW_DW * 4;
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
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, kBlock, lds);
        if (e != hipSuccess) return e;
        max_blocks = nb > 0 ? nb : 1;
    }
    const int64_t n_chunks = (a.count + 63) / 64;
    int64_t want = (n_chunks + kWavesPerBlock - 1) / kWavesPerBlock;
    int64_t cap = (int64_t)max_blocks * n_cu;
    int64_t blocks = want < cap ? want : cap;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kBlock), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_query(const Model &m, const QueryArgs &a, niv_precision prec, hipStream_t st)
{
    if (a.count <= 0) return hipSuccess;
    switch (m.kind) {
    case kUnitCube:
        if (prec == NIV_FP32) return query_t<NIV_FP32, ShapeUnitCube, true, 4>(a, st);
        if (prec == NIV_FP16) return query_t<NIV_FP16, ShapeUnitCube, true, 4>(a, st);
        return query_t<NIV_BF16, ShapeUnitCube, true, 4>(a, st);
    case kRoom:
        if (prec == NIV_FP32) return query_t<NIV_FP32, ShapeRoom, true, 4>(a, st);
        if (prec == NIV_FP16) return query_t<NIV_FP16, ShapeRoom, true, 4>(a, st);
        return query_t<NIV_BF16, ShapeRoom, true, 4>(a, st);
    default:
        if (prec == NIV_FP32) return query_t<NIV_FP32, ShapeWide6D, false, 2>(a, st);
        if (prec == NIV_FP16) return query_t<NIV_FP16, ShapeWide6D, false, 2>(a, st);
        return query_t<NIV_BF16, ShapeWide6D, false, 2>(a, st);
    }
}

}  // namespace niv
