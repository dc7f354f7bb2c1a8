// Random numbers and hemisphere sampling shared by the Monte Carlo
// kernels: a counter-based generator keyed by (seed, point, sample,
// stream) and cosine-distributed directions.  Included after
// `#pragma clang fp contract(off)`, so no multiply-add is fused.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace niv {

// ---------------------------------------------------------------- Philox4x64-10
// Salmon et al., SC'11: ten rounds of two 64x64->128 products with the
// published multipliers, Weyl-sequence key schedule.
__device__ inline void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
        uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
        uint64_t y0 = hi1 ^ c[1] ^ k0, y2 = hi0 ^ c[3] ^ k1;
        c[0] = y0; c[1] = lo1; c[2] = y2; c[3] = lo0;
        k0 += W0;
        k1 += W1;
    }
}

// Stream of uniforms for one (point, sample): dimension d lives in block
// d / 8 at 32-bit half d % 8 (low half first); 24-bit mantissa.
struct Rng {
    uint64_t seed, a, b, stream;
    int block;
    uint64_t w[4];
    __device__ Rng(uint64_t s, uint64_t a_, uint64_t b_, uint64_t st)
        : seed(s), a(a_), b(b_), stream(st), block(-1) {}
    __device__ float u(int d)
    {
        int blk = d >> 3;
        if (blk != block) {
            w[0] = a; w[1] = b; w[2] = (uint64_t)blk; w[3] = stream;
            philox4x64_10(w, seed, 0);
            block = blk;
        }
        int k = (d & 7) >> 1;
        uint64_t x = k == 0 ? w[0] : k == 1 ? w[1] : k == 2 ? w[2] : w[3];
        uint32_t v = (d & 1) ? (uint32_t)(x >> 32) : (uint32_t)x;
        return (float)(v >> 8) * 0x1p-24f;
    }
};

// Orthonormal basis around a unit vector (Duff et al., JCGT 2017).
__device__ inline void onb(const float n[3], float t[3], float b[3])
{
    float s = n[2] >= 0.0f ? 1.0f : -1.0f;
    float a = -1.0f / (s + n[2]);
    float bb = n[0] * n[1] * a;
    t[0] = 1.0f + s * n[0] * n[0] * a; t[1] = s * bb; t[2] = -s * n[0];
    b[0] = bb; b[1] = s + n[1] * n[1] * a; b[2] = -n[1];
}

// Cosine-distributed direction about n (Malley: uniform disk point lifted).
__device__ inline void cosine_dir(const float n[3], float u1, float u2, float d[3])
{
    float t[3], b[3];
    onb(n, t, b);
    float r = sqrtf(u1), phi = 6.28318530717958647692f * u2;
    float sp, cp;
    __sincosf(phi, &sp, &cp);
    float x = r * cp, y = r * sp, z = sqrtf(fmaxf(0.0f, 1.0f - u1));
#pragma unroll
    for (int a = 0; a < 3; ++a) d[a] = x * t[a] + y * b[a] + z * n[a];
}

}  // namespace niv
