// Device-side pieces shared by the query and training kernels of libniv:
// vector types, precision traits, model shapes, the operand layout of a
// prepared model and the per-level encoding (Sec. 4.1).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

#include "niv_internal.h"

namespace niv {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef short s2 __attribute__((ext_vector_type(2)));
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
    // A K = 16 product issued as the K = 32 instruction with the upper half
    // of each lane's operands zero: lane (g, j) then pairs the same four
    // products as the K = 16 layout, and the sum is unchanged.  (The K = 16
    // instruction reading as its accumulator the result of a K = 32 one
    // needs 5 wait states between them on gfx950, measured; the compiler
    // inserts none when the registers coincide exactly, as they do when a
    // half-depth product continues a full one.  Same-opcode chains are
    // correct with none.)
    __device__ static f4 mma_half(u2 a, u2 b, f4 c) {
        return mma((u4){a.x, a.y, 0u, 0u}, (u4){b.x, b.y, 0u, 0u}, c);
    }
    __device__ static uint32_t pack(float x, float y) {
        h2 v = __builtin_convertvector((f2){x, y}, h2);
        return __builtin_bit_cast(uint32_t, v);
    }
    // ReLU after rounding: a half with its sign bit set is a negative 16-bit
    // integer, so a packed integer max with 0 zeroes exactly the negative
    // halves (rounding preserves the sign, so this equals rounding the ReLU).
    __device__ static uint32_t pack_relu(float x, float y) {
        s2 v = __builtin_bit_cast(s2, __builtin_convertvector((f2){x, y}, h2));
        return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(v, (s2){0, 0}));
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
    // as for FP16 (the K = 16 BF16 instruction has the same dependency on a
    // K = 32 one that wrote its accumulator)
    __device__ static f4 mma_half(u2 a, u2 b, f4 c) {
        return mma((u4){a.x, a.y, 0u, 0u}, (u4){b.x, b.y, 0u, 0u}, c);
    }
    __device__ static uint32_t pack(float x, float y) {
        bf2 v = __builtin_convertvector((f2){x, y}, bf2);
        return __builtin_bit_cast(uint32_t, v);
    }
    __device__ static f2 unpack(uint32_t w) {
        // a bf16 is the upper half of the float with the same bits
        return (f2){__builtin_bit_cast(float, w << 16), __builtin_bit_cast(float, w & 0xffff0000u)};
    }
    // x = hi + lo: hi is x cut to its upper 16 bits (a BF16 by truncation),
    // lo = x - hi (exact in FP32) rounded to BF16; the pair carries at least
    // 16 significant bits, so BF16 operands lose little to rounding.  Two
    // values per call: one byte permute for the two his, one conversion for
    // the two los.
    __device__ static void split(float x, float y, uint32_t &hi, uint32_t &lo) {
        const uint32_t xb = f2u(x), yb = f2u(y);
        hi = __builtin_amdgcn_perm(yb, xb, 0x07060302u);
        lo = pack(x - u2f(xb & 0xffff0000u), y - u2f(yb & 0xffff0000u));
    }
    // the same after a ReLU, done as a signed integer max on the FP32 bits
    __device__ static void split_relu(float x, float y, uint32_t &hi, uint32_t &lo) {
        const int32_t xi = (int32_t)f2u(x), yi = (int32_t)f2u(y);
        split(u2f((uint32_t)(xi > 0 ? xi : 0)), u2f((uint32_t)(yi > 0 ? yi : 0)), hi, lo);
    }
};

template <> struct Prec<NIV_FP32> {
    static constexpr int ES = 4;
    static constexpr int EPO = 1;
    // ReLU as a signed integer max: negative floats are negative integers
    __device__ static float relu(float x) {
        const int32_t i = (int32_t)f2u(x);
        return u2f((uint32_t)(i > 0 ? i : 0));
    }
    __device__ static f4 mma1(float a, float b, f4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

// ---------------------------------------------------------------- shapes
// SL_: lane-sliced encoding.  Each lane encodes exactly the layer-0 operand
// elements it feeds to the matrix cores (for the four pixels it serves, one
// per 16-pixel tile), so no per-wave staging block in LDS is needed and the
// whole LDS can hold the weights.
// PB_: bands of the positional code of x (grid-free models, L_ = 0).
// F_: features per grid entry (2, or 4 for Table 1's grid networks).
//
// Layer-0 columns.  The parameters of W_0 follow the input vector of the
// model: [grid F L][u 3, bands 6 PB][SH 16][scene variables 16 NEX].  The
// kernels order the columns as [grid F L][bands 6 PB][u 3][0][SH 16][scene
// variables][0 ...] so that 16-bit pairs never straddle two parts, padded
// with zero columns to a multiple of 16; in_col maps a kernel column to its
// parameter column (or -1 for a zero column).
template <int L_, int NEX_, int W_, int H_, bool SL_ = false, int PB_ = 0, int F_ = 2> struct Shape {
    static constexpr int L = L_, NEX = NEX_, W = W_, H = H_, PB = PB_, F = F_;
    static constexpr bool SL = SL_;
    static constexpr int GF = F * L;                              // grid features
    static constexpr int PEW_IN = PB > 0 ? 3 + 6 * PB : 0;       // positional code
    static constexpr int PEW = PB > 0 ? PEW_IN + 1 : 0;           // with its zero column
    static constexpr int DIN_IN = GF + PEW_IN + 16 + 16 * NEX;    // 16 SH, 16 per variable
    static constexpr int DIN = (GF + PEW + 16 + 16 * NEX + 15) / 16 * 16;
    static constexpr int KLG = DIN / 4;                // input slots per lane group
    static constexpr int NOB = W / 16;                 // 16-row output blocks
    static_assert(!SL || (L == 16 && F == 2 && DIN == 64 && PB == 0), "lane slices need 16 levels and 64 inputs");
    static_assert((F == 2 || F == 4) && GF % 4 == 0 && W % 16 == 0 && W >= 16, "shape");
    static_assert(PB == 0 || L == 0, "positional code only without grid levels");
    __host__ __device__ static constexpr int in_col(int kc)
    {
        if (kc < GF) return kc;
        int r = kc - GF;
        if (PB > 0) {
            if (r < 6 * PB) return GF + 3 + r;          // bands
            if (r < 6 * PB + 3) return GF + (r - 6 * PB);  // u
            if (r == 6 * PB + 3) return -1;
            r -= PEW;
        }
        return r < 16 + 16 * NEX ? GF + PEW_IN + r : -1;
    }
};

using ShapeUnitCube = Shape<8, 0, 64, 2>;
using ShapeRoom = Shape<16, 0, 64, 3>;
using ShapeWide6D = Shape<16, 1, 128, 4, true>;
// FP32 weights of the wide network (232 KB) do not fit in LDS: that
// precision stages the inputs and reads the weights from memory.
template <int P> using ShapeWide6DFor =
    typename std::conditional<P == NIV_FP32, Shape<16, 1, 128, 4>, ShapeWide6D>::type;
template <int W> using ShapePE = Shape<0, 0, W, 3, false, 8>;
// the room network with one scene variable (Sec. 6), trainable
using ShapeRoom6D = Shape<16, 1, 64, 3>;
// Table 1's grid rows: 2, 4, 6 or 8 levels of 4 features, width 64
template <int L> using ShapeT1 = Shape<L, 0, 64, 3, false, 0, 4>;

// Lane-sliced layer-0 input order.  Virtual element v (0..15) of lane group
// g: v < 8 is feature v % 2 of level 4 (v / 2) + g; then SH coefficients
// 4g..4g+3 and frequency-code entries 4g..4g+3.  (16 levels, 16 SH, one
// scene variable: 64 inputs.)
__host__ __device__ constexpr int slice_col(int v, int g)
{
    return v < 8 ? 2 * (4 * (v >> 1) + g) + (v & 1) : (v < 12 ? 32 + 4 * g + (v - 8) : 48 + 4 * g + (v - 12));
}

// Byte layout of the operand block of a prepared model.  16-bit layers
// whose contraction depth is not a multiple of 32 end with one half-depth
// (K = 16) operand per output block.
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
    static constexpr int HF = F32 ? S::W / 4 : S::W / 32;           // full operands per block row
    static constexpr int HH = F32 ? 0 : (S::W % 32) / 16;           // half-depth operands per row
    static constexpr int HOPS = HF + HH;
    static constexpr int HROW = HF * OPB + HH * OPS;                // bytes per block row
    static constexpr int HID_BYTES = S::NOB * HROW;
    static constexpr int OUT_BYTES = HROW;                          // rows 0..2 = W_H
    static constexpr int W_BYTES = L0_BYTES + (S::H - 1) * HID_BYTES + OUT_BYTES;
    static constexpr int N_OPS = S::NOB * (L0_FULL + L0_HALF) + (S::H - 1) * S::NOB * HOPS + HOPS;
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
// for a zero.  Parameters: [grid][W_0 (W x DIN_IN)][W_1..W_{H-1} (W x W)][W_H (3 x W)].
template <int P, class S>
__device__ int64_t operand_source(int op, int lane, int e, int64_t n_grid, int n_out)
{
    using O = Ops<P, S>;
    const int i = lane & 15, g = lane >> 4;
    const int64_t w0 = n_grid;
    const int64_t wh = w0 + (int64_t)S::W * S::DIN_IN;
    const int64_t wo = wh + (int64_t)(S::H - 1) * S::W * S::W;
    const int n0 = S::NOB * (O::L0_FULL + O::L0_HALF);
    const int nh = (S::H - 1) * S::NOB * O::HOPS;
    if (op < n0) {  // layer 0: [ob][chunk]
        int ob = op / (O::L0_FULL + O::L0_HALF), c = op % (O::L0_FULL + O::L0_HALF);
        int slot = O::F32 ? c : (c < O::L0_FULL ? c * 8 + e : O::L0_FULL * 8 + e);
        int row = 16 * ob + i, col = S::SL ? slice_col(slot, g) : S::KLG * g + slot;
        const int pc = S::in_col(col);
        if (pc < 0) return -1;
        return w0 + (int64_t)row * S::DIN_IN + pc;
    }
    op -= n0;
    int col;
    // contraction column of element e of lane group g in operand kb of a
    // block row (a half-depth operand covers 16 columns, 4 per lane group)
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
    op -= nh;  // output layer: [kb]; rows 0..n_out-1 hold W_H, the rest zero
    const int kb = op;
    col = hidden_col(kb);
    if (i >= n_out) return -1;
    return wo + (int64_t)i * S::W + col;
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
    op -= n0;  // hidden rows, then the output row: HOPS operands per block row
    const int row = op / O::HOPS, kb = op % O::HOPS;
    *off = O::L0_BYTES + (int64_t)row * O::HROW + (int64_t)kb * O::OPB;
    *n_elem = kb < O::HF ? O::EPO : 4;
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

// sin(pi r) and cos(pi r) for |r| <= 1/2 from their Taylor series about 0,
// to degree 11 and 12; on that range the first omitted terms are below
// 5.7e-8 and 6.4e-9.  Coefficients (-1)^k pi^n / n! are formed at compile
// time in double precision.
constexpr double taylor_pi(int n)
{
    double v = 1.0;
    for (int k = 1; k <= n; ++k) v *= 3.14159265358979323846 / k;
    return (n / 2) % 2 ? -v : v;
}
__device__ inline void sincospi_half(float r, float &s, float &c)
{
    const float x2 = r * r;
    float ps = (float)taylor_pi(11);
    ps = __builtin_fmaf(ps, x2, (float)taylor_pi(9));
    ps = __builtin_fmaf(ps, x2, (float)taylor_pi(7));
    ps = __builtin_fmaf(ps, x2, (float)taylor_pi(5));
    ps = __builtin_fmaf(ps, x2, (float)taylor_pi(3));
    ps = __builtin_fmaf(ps, x2, (float)taylor_pi(1));
    s = ps * r;
    float pc = (float)taylor_pi(12);
    pc = __builtin_fmaf(pc, x2, (float)taylor_pi(10));
    pc = __builtin_fmaf(pc, x2, (float)taylor_pi(8));
    pc = __builtin_fmaf(pc, x2, (float)taylor_pi(6));
    pc = __builtin_fmaf(pc, x2, (float)taylor_pi(4));
    pc = __builtin_fmaf(pc, x2, (float)taylor_pi(2));
    c = __builtin_fmaf(pc, x2, 1.0f);
}

// Positional code of one coordinate u in [0, 1] given as u = uh + ul (two
// floats): sin and cos of 2^b pi u for b < PB.  2^b u = th + tl exactly;
// n = rint(th) and th - n are exact (Sterbenz), so r = (th - n) + tl is the
// reduced argument with one rounding, and sin(pi (n + r)) = (-1)^n sin(pi r)
// (the same for cos).  EVERY (16-bit operands): only every EVERY-th band
// is evaluated so; the bands after it follow from the double-angle formulas
// sin 2a = 2 sin a cos a, cos 2a = (cos a - sin a)(cos a + sin a).  That
// step is twice a rotation, so it doubles the error of the evaluated band
// and no more (1 - 2 sin^2 a would multiply it by up to 4): EVERY = 4 (BF16,
// whose hi + lo operands keep ~16 bits) ends below 2e-6, EVERY = 8 (FP16, 11
// bits) below 3e-5, under the operand rounding either way.  EVERY = 1: all
// bands evaluated.
template <int PB, int EVERY>
__device__ inline void pos_code_axis(float uh, float ul, float *sv, float *cv)
{
#pragma unroll
    for (int b = 0; b < PB; ++b) {
        if ((b % EVERY) != 0) {
            const float s0 = sv[b - 1], c0 = cv[b - 1];
            sv[b] = 2.0f * (s0 * c0);
            cv[b] = (c0 - s0) * (c0 + s0);
            continue;
        }
        const float th = uh * (float)(1 << b), tl = ul * (float)(1 << b);
        const float n = __builtin_rintf(th);
        const float r = (th - n) + tl;
        float sr, cr;
        sincospi_half(r, sr, cr);
        const uint32_t flip = (uint32_t)(int32_t)n << 31;
        sv[b] = u2f(f2u(sr) ^ flip);
        cv[b] = u2f(f2u(cr) ^ flip);
    }
}

// Cell, corner indices (within the whole grid) and trilinear weights of one
// level (Sec. 4.1).  Corner c = cx + 2cy + 4cz.
template <class LV>
__device__ inline void level_corners(const LV &lv, const double p[3], uint32_t hmask,
                                     uint32_t idx[8], float w[8])
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
    const float wx1 = fr[0], wx0 = 1.0f - fr[0];
    const float wy1 = fr[1], wy0 = 1.0f - fr[1];
    const float wz1 = fr[2], wz0 = 1.0f - fr[2];
    const float w00 = wy0 * wz0, w10 = wy1 * wz0, w01 = wy0 * wz1, w11 = wy1 * wz1;
    w[0] = wx0 * w00; w[1] = wx1 * w00; w[2] = wx0 * w10; w[3] = wx1 * w10;
    w[4] = wx0 * w01; w[5] = wx1 * w01; w[6] = wx0 * w11; w[7] = wx1 * w11;
}

// The same blend with the 8 latents fetched by buffer loads: the per-level
// table offset rides in the scalar offset of the load, the hash primes are
// pre-scaled by the entry size, and dense corners differ only by scalar or
// immediate offsets, so no 64-bit address arithmetic is spent per corner.
// F32C: cell coordinates in FP32 (the FP16 query: an FP32 coordinate of
// ~2900 cells is off by ~2e-4 of a cell, below the operand rounding, and
// trilinear interpolation is continuous across cell faces, so a cell chosen
// differently at a face gives the same features); else in FP64.
// A level's eight latents in flight: the raw loaded words (FP16/BF16 pairs,
// or FP32 pairs) and the cell fractions.
template <int P> struct LevelFetch {
    typename std::conditional<P == NIV_FP32, u2, uint32_t>::type v[8];
    float fr[3];
};

// Issue phase: cell, corner offsets and the eight buffer loads of one level.
// F32C: cell coordinates in FP32 (the FP16 query: an FP32 coordinate of
// ~2900 cells is off by ~2e-4 of a cell, below the operand rounding, and
// trilinear interpolation is continuous across cell faces, so a cell chosen
// differently at a face gives the same features); else in FP64.
// TRACE (inspection only): also stores the grid entry of each corner, in
// corner order, to trace[0..7].
template <int P, bool F32C = false, bool TRACE = false, class LV>
__device__ inline void level_issue(const LV &lv, const double p[3], uint32_t hmask,
                                   __amdgpu_buffer_rsrc_t rsrc, const float *pf, LevelFetch<P> &out,
                                   uint32_t *trace = nullptr)
{
    constexpr int SH = (P == NIV_FP32) ? 3 : 2;   // log2 of the entry size in bytes
    constexpr uint32_t EB = 1u << SH;
    int32_t ci[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if constexpr (F32C) {
            const float s = __builtin_fmaf(pf[a], lv.kf[a], lv.of[a]);
            int32_t c = (int32_t)s;            // s > -1: truncation = floor clamped at 0
            c = c < lv.nm1 ? c : lv.nm1;
            ci[a] = c;
            out.fr[a] = s - (float)c;          // exact (Sterbenz)
        } else {
            double s = __builtin_fma(p[a], lv.k[a], lv.o[a]);
            int32_t c = (int32_t)s;
            c = c < lv.nm1 ? c : lv.nm1;
            ci[a] = c;
            out.fr[a] = (float)(s - (double)c);
        }
    }
    [[maybe_unused]] int nt = 0;
    auto ld = [&](int c, uint32_t voff, uint32_t soff) {
        if constexpr (TRACE) trace[nt++] = (voff + soff) >> SH;
        if constexpr (P == NIV_FP32) out.v[c] = __builtin_amdgcn_raw_buffer_load_b64(rsrc, voff, soff, 0);
        else out.v[c] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, voff, soff, 0);
    };
    // One set of loads for both storage kinds, with no branch, so that the
    // loads of consecutive levels can overlap.  Corner c = cx + 2cy + 4cz
    // reads (xb + cx EB) ^ t_c at scalar offset o_c: a hashed level has
    // xb = x << SH, t_c = the masked y/z hash terms and o_c its first entry;
    // a dense level has xb = (x + (N+1)(y + (N+1) z)) << SH, t_c = 0 (mask 0)
    // and o_c its first entry plus the y/z steps of the corner.
    const bool dn = lv.dense != 0;
    const uint32_t bd = ((uint32_t)ci[0] + lv.s1 * ((uint32_t)ci[1] + lv.s1 * (uint32_t)ci[2])) << SH;
    const uint32_t xb = dn ? bd : ((uint32_t)ci[0] << SH);
    const uint32_t m = dn ? 0u : (hmask << SH);
    const uint32_t p1 = kPrime1 << SH, p2 = kPrime2 << SH;
    const uint32_t y0 = (uint32_t)ci[1] * p1, y1 = y0 + p1;
    const uint32_t z0 = (uint32_t)ci[2] * p2, z1 = z0 + p2;
    const uint32_t t00 = (y0 ^ z0) & m, t10 = (y1 ^ z0) & m;
    const uint32_t t01 = (y0 ^ z1) & m, t11 = (y1 ^ z1) & m;
    const uint32_t o = lv.off << SH;
    const uint32_t o10 = dn ? (lv.off + lv.s1) << SH : o, o01 = dn ? (lv.off + lv.s2) << SH : o;
    const uint32_t o11 = dn ? (lv.off + lv.s2 + lv.s1) << SH : o;
    const uint32_t x0 = xb, x1 = xb + EB;
    ld(0, x0 ^ t00, o);   ld(1, x1 ^ t00, o);
    ld(2, x0 ^ t10, o10); ld(3, x1 ^ t10, o10);
    ld(4, x0 ^ t01, o01); ld(5, x1 ^ t01, o01);
    ld(6, x0 ^ t11, o11); ld(7, x1 ^ t11, o11);
}

// Blend phase: the trilinear weights and the FP32 sum of the eight latents.
template <int P>
__device__ inline f2 level_blend(const LevelFetch<P> &f)
{
    const float wx1 = f.fr[0], wx0 = 1.0f - f.fr[0];
    const float wy1 = f.fr[1], wy0 = 1.0f - f.fr[1];
    const float wz1 = f.fr[2], wz0 = 1.0f - f.fr[2];
    const float w00 = wy0 * wz0, w10 = wy1 * wz0, w01 = wy0 * wz1, w11 = wy1 * wz1;
    const float w[8] = {wx0 * w00, wx1 * w00, wx0 * w10, wx1 * w10,
                        wx0 * w01, wx1 * w01, wx0 * w11, wx1 * w11};
    f2 acc = {0.0f, 0.0f};
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        f2 v;
        if constexpr (P == NIV_FP32) v = (f2){u2f(f.v[c].x), u2f(f.v[c].y)};
        else v = Prec<P>::unpack(f.v[c]);
        acc.x = __builtin_fmaf(w[c], v.x, acc.x);
        acc.y = __builtin_fmaf(w[c], v.y, acc.y);
    }
    return acc;
}

// One level fetched and blended in one go, with the storage kind as a branch:
// the per-level table offset rides in the scalar offset of the load, the
// hash primes are pre-scaled by the entry size, and dense corners differ
// only by scalar or immediate offsets (the compiler pairs a dense level's
// x-neighbours into 8-byte loads).  The FP16 query uses it level by level:
// there the paired loads (fewer gather instructions) pay more than
// overlapping the levels' loads (level_issue), measured.
template <int P, bool F32C = false, bool TRACE = false, class LV>
__device__ inline f2 encode_level_buf(const LV &lv, const double p[3], uint32_t hmask,
                                      __amdgpu_buffer_rsrc_t rsrc, const float *pf = nullptr,
                                      uint32_t *trace = nullptr)
{
    constexpr int SH = (P == NIV_FP32) ? 3 : 2;   // log2 of the entry size in bytes
    constexpr uint32_t EB = 1u << SH;
    int32_t ci[3];
    float fr[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if constexpr (F32C) {
            const float s = __builtin_fmaf(pf[a], lv.kf[a], lv.of[a]);
            int32_t c = (int32_t)s;            // s > -1: truncation = floor clamped at 0
            c = c < lv.nm1 ? c : lv.nm1;
            ci[a] = c;
            fr[a] = s - (float)c;              // exact (Sterbenz)
        } else {
            double s = __builtin_fma(p[a], lv.k[a], lv.o[a]);
            int32_t c = (int32_t)s;
            c = c < lv.nm1 ? c : lv.nm1;
            ci[a] = c;
            fr[a] = (float)(s - (double)c);
        }
    }
    LevelFetch<P> f;
    [[maybe_unused]] int nt = 0;
    auto ld = [&](int c, uint32_t voff, uint32_t soff) {
        if constexpr (TRACE) trace[nt++] = (voff + soff) >> SH;
        if constexpr (P == NIV_FP32) f.v[c] = __builtin_amdgcn_raw_buffer_load_b64(rsrc, voff, soff, 0);
        else f.v[c] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, voff, soff, 0);
    };
    if (lv.dense) {
        const uint32_t b = ((uint32_t)ci[0] + lv.s1 * ((uint32_t)ci[1] + lv.s1 * (uint32_t)ci[2])) << SH;
        const uint32_t o00 = lv.off << SH, o10 = (lv.off + lv.s1) << SH;
        const uint32_t o01 = (lv.off + lv.s2) << SH, o11 = (lv.off + lv.s2 + lv.s1) << SH;
        ld(0, b, o00); ld(1, b + EB, o00);
        ld(2, b, o10); ld(3, b + EB, o10);
        ld(4, b, o01); ld(5, b + EB, o01);
        ld(6, b, o11); ld(7, b + EB, o11);
    } else {
        const uint32_t p1 = kPrime1 << SH, p2 = kPrime2 << SH, m = hmask << SH;
        const uint32_t x0 = (uint32_t)ci[0] << SH, x1 = x0 + EB;
        const uint32_t y0 = (uint32_t)ci[1] * p1, y1 = y0 + p1;
        const uint32_t z0 = (uint32_t)ci[2] * p2, z1 = z0 + p2;
        const uint32_t t00 = (y0 ^ z0) & m, t10 = (y1 ^ z0) & m;
        const uint32_t t01 = (y0 ^ z1) & m, t11 = (y1 ^ z1) & m;
        const uint32_t o = lv.off << SH;
        ld(0, x0 ^ t00, o); ld(1, x1 ^ t00, o);
        ld(2, x0 ^ t10, o); ld(3, x1 ^ t10, o);
        ld(4, x0 ^ t01, o); ld(5, x1 ^ t01, o);
        ld(6, x0 ^ t11, o); ld(7, x1 ^ t11, o);
    }
    f.fr[0] = fr[0]; f.fr[1] = fr[1]; f.fr[2] = fr[2];
    return level_blend<P>(f);
}

// A dense level read from a copy of its entries in LDS (tab[0] is the
// level's first entry): the cell, fractions and blend of encode_level_buf
// with FP64 cell coordinates, so the features are the same bit for bit.
template <int P, class LV>
__device__ inline f2 encode_dense_lds(const LV &lv, const double p[3], const uint32_t *tab)
{
    LevelFetch<P> f;
    int32_t ci[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double s = __builtin_fma(p[a], lv.k[a], lv.o[a]);
        int32_t c = (int32_t)s;
        c = c < lv.nm1 ? c : lv.nm1;
        ci[a] = c;
        f.fr[a] = (float)(s - (double)c);
    }
    const uint32_t b = (uint32_t)ci[0] + lv.s1 * ((uint32_t)ci[1] + lv.s1 * (uint32_t)ci[2]);
    const uint32_t o[4] = {b, b + lv.s1, b + lv.s2, b + lv.s2 + lv.s1};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        f.v[2 * k] = tab[o[k]];
        f.v[2 * k + 1] = tab[o[k] + 1];
    }
    return level_blend<P>(f);
}

// A level of four features per entry (Table 1's grid rows): eight
// corner entries of 8 bytes (16-bit) or 16 bytes (FP32), the storage kind as a
// branch as in encode_level_buf, FP32 trilinear blend of the four features.
template <int P, bool F32C = false, bool TRACE = false, class LV>
__device__ inline f4 encode_level_buf4(const LV &lv, const double p[3], uint32_t hmask,
                                       __amdgpu_buffer_rsrc_t rsrc, const float *pf = nullptr,
                                       uint32_t *trace = nullptr)
{
    constexpr int SH = (P == NIV_FP32) ? 4 : 3;   // log2 of the entry size in bytes
    constexpr uint32_t EB = 1u << SH;
    int32_t ci[3];
    float fr[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if constexpr (F32C) {
            const float s = __builtin_fmaf(pf[a], lv.kf[a], lv.of[a]);
            int32_t c = (int32_t)s;
            c = c < lv.nm1 ? c : lv.nm1;
            ci[a] = c;
            fr[a] = s - (float)c;
        } else {
            double s = __builtin_fma(p[a], lv.k[a], lv.o[a]);
            int32_t c = (int32_t)s;
            c = c < lv.nm1 ? c : lv.nm1;
            ci[a] = c;
            fr[a] = (float)(s - (double)c);
        }
    }
    f4 v[8];
    [[maybe_unused]] int nt = 0;
    auto ld = [&](int c, uint32_t voff, uint32_t soff) {
        if constexpr (TRACE) trace[nt++] = (voff + soff) >> SH;
        if constexpr (P == NIV_FP32) {
            const u4 w = __builtin_amdgcn_raw_buffer_load_b128(rsrc, voff, soff, 0);
            v[c] = (f4){u2f(w.x), u2f(w.y), u2f(w.z), u2f(w.w)};
        } else {
            const u2 w = __builtin_amdgcn_raw_buffer_load_b64(rsrc, voff, soff, 0);
            const f2 a = Prec<P>::unpack(w.x), b = Prec<P>::unpack(w.y);
            v[c] = (f4){a.x, a.y, b.x, b.y};
        }
    };
    if (lv.dense) {
        const uint32_t b = ((uint32_t)ci[0] + lv.s1 * ((uint32_t)ci[1] + lv.s1 * (uint32_t)ci[2])) << SH;
        const uint32_t o00 = lv.off << SH, o10 = (lv.off + lv.s1) << SH;
        const uint32_t o01 = (lv.off + lv.s2) << SH, o11 = (lv.off + lv.s2 + lv.s1) << SH;
        ld(0, b, o00); ld(1, b + EB, o00);
        ld(2, b, o10); ld(3, b + EB, o10);
        ld(4, b, o01); ld(5, b + EB, o01);
        ld(6, b, o11); ld(7, b + EB, o11);
    } else {
        const uint32_t p1 = kPrime1 << SH, p2 = kPrime2 << SH, m = hmask << SH;
        const uint32_t x0 = (uint32_t)ci[0] << SH, x1 = x0 + EB;
        const uint32_t y0 = (uint32_t)ci[1] * p1, y1 = y0 + p1;
        const uint32_t z0 = (uint32_t)ci[2] * p2, z1 = z0 + p2;
        const uint32_t t00 = (y0 ^ z0) & m, t10 = (y1 ^ z0) & m;
        const uint32_t t01 = (y0 ^ z1) & m, t11 = (y1 ^ z1) & m;
        const uint32_t o = lv.off << SH;
        ld(0, x0 ^ t00, o); ld(1, x1 ^ t00, o);
        ld(2, x0 ^ t10, o); ld(3, x1 ^ t10, o);
        ld(4, x0 ^ t01, o); ld(5, x1 ^ t01, o);
        ld(6, x0 ^ t11, o); ld(7, x1 ^ t11, o);
    }
    const float wx1 = fr[0], wx0 = 1.0f - fr[0];
    const float wy1 = fr[1], wy0 = 1.0f - fr[1];
    const float wz1 = fr[2], wz0 = 1.0f - fr[2];
    const float w00 = wy0 * wz0, w10 = wy1 * wz0, w01 = wy0 * wz1, w11 = wy1 * wz1;
    const float w[8] = {wx0 * w00, wx1 * w00, wx0 * w10, wx1 * w10,
                        wx0 * w01, wx1 * w01, wx0 * w11, wx1 * w11};
    f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        acc.x = __builtin_fmaf(w[c], v[c].x, acc.x);
        acc.y = __builtin_fmaf(w[c], v[c].y, acc.y);
        acc.z = __builtin_fmaf(w[c], v[c].z, acc.z);
        acc.w = __builtin_fmaf(w[c], v[c].w, acc.w);
    }
    return acc;
}

// The same blend for a level that differs between lanes (lane-sliced
// encoding): the level's constants are per-lane values, its first entry is
// added to the per-lane buffer offset.
struct LevelRegs {   // the per-lane part of a level's constants
    double k[3], o[3];
    int32_t nm1, dense;
    uint32_t off, s1, s2;
};

__device__ inline LevelRegs load_level(const LevelConst *lp)
{
    LevelRegs r;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r.k[a] = lp->k[a];
        r.o[a] = lp->o[a];
    }
    r.nm1 = lp->nm1;
    r.dense = lp->dense;
    r.off = lp->off;
    r.s1 = lp->s1;
    r.s2 = lp->s2;
    return r;
}

// Issue phase of a level that differs between lanes: cell, corner offsets
// and the eight loads with one set of instructions for dense and hashed
// levels (the level's kind is a per-lane value here, so a branch on it would
// diverge): corner c reads ((xb + cx EB) ^ t_c) + o_c, where a hashed level
// has xb = x << SH, t_c its masked y/z hash terms and o_c its first entry, a
// dense level xb = (x + (N+1)(y + (N+1) z)) << SH, t_c = 0 and o_c its first
// entry plus the corner's y/z steps.
template <int P, bool TRACE = false>
__device__ inline void level_issue_vec(const LevelRegs &lv, const double p[3], uint32_t hmask,
                                       __amdgpu_buffer_rsrc_t rsrc, LevelFetch<P> &out,
                                       uint32_t *trace = nullptr)
{
    constexpr int SH = (P == NIV_FP32) ? 3 : 2;
    constexpr uint32_t EB = 1u << SH;
    int32_t ci[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double s = __builtin_fma(p[a], lv.k[a], lv.o[a]);
        int32_t c = (int32_t)s;
        c = c < lv.nm1 ? c : lv.nm1;
        ci[a] = c;
        out.fr[a] = (float)(s - (double)c);
    }
    const bool dn = lv.dense != 0;
    const uint32_t bd = ((uint32_t)ci[0] + lv.s1 * ((uint32_t)ci[1] + lv.s1 * (uint32_t)ci[2])) << SH;
    const uint32_t xb = dn ? bd : ((uint32_t)ci[0] << SH);
    const uint32_t m = dn ? 0u : (hmask << SH);
    const uint32_t p1 = kPrime1 << SH, p2 = kPrime2 << SH;
    const uint32_t y0 = (uint32_t)ci[1] * p1, y1 = y0 + p1;
    const uint32_t z0 = (uint32_t)ci[2] * p2, z1 = z0 + p2;
    const uint32_t t00 = (y0 ^ z0) & m, t10 = (y1 ^ z0) & m;
    const uint32_t t01 = (y0 ^ z1) & m, t11 = (y1 ^ z1) & m;
    const uint32_t o = lv.off << SH;
    const uint32_t o10 = dn ? (lv.off + lv.s1) << SH : o, o01 = dn ? (lv.off + lv.s2) << SH : o;
    const uint32_t o11 = dn ? (lv.off + lv.s2 + lv.s1) << SH : o;
    [[maybe_unused]] int nt = 0;
    auto ld = [&](int c, uint32_t voff) {
        if constexpr (TRACE) trace[nt++] = voff >> SH;
        if constexpr (P == NIV_FP32) out.v[c] = __builtin_amdgcn_raw_buffer_load_b64(rsrc, voff, 0, 0);
        else out.v[c] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, voff, 0, 0);
    };
    const uint32_t x0 = xb, x1 = xb + EB;
    ld(0, (x0 ^ t00) + o);   ld(1, (x1 ^ t00) + o);
    ld(2, (x0 ^ t10) + o10); ld(3, (x1 ^ t10) + o10);
    ld(4, (x0 ^ t01) + o01); ld(5, (x1 ^ t01) + o01);
    ld(6, (x0 ^ t11) + o11); ld(7, (x1 ^ t11) + o11);
}

}  // namespace niv
