// Half-resolution rendering (Sec. 4.4): joint bilateral upsampling of the
// irradiance computed at the G-buffer pixels (2x, 2y) to every pixel, with
// the G-buffer's positions and normals as guides, then L = albedo * E / pi
// (Eq. 2).
//
// Sample x serves the pixels X with |2x - X| <= 2: 3 samples per axis for
// an even pixel, 2 for an odd one.
// Weights are formed from their base-2 logarithms relative to the largest
// one, so the average stays finite however small the weights get; the
// logarithms themselves are taken relative to the sample nearest in position
// so that no large terms cancel in FP32.
#include <hip/hip_runtime.h>

#include "niv_internal.h"

namespace niv {

namespace {
constexpr int kQuadsX = 32, kQuadsY = 8;   // workgroup: 32 x 8 quads = 64 x 16 pixels

__device__ inline bool finite3(const float *v)
{
    return __builtin_isfinite(v[0]) && __builtin_isfinite(v[1]) && __builtin_isfinite(v[2]);
}

// unit normal, scaled by the largest component first so tiny and huge
// normals normalise without underflow or overflow; false for a zero normal
// (branch-free: the result is only used where it returns true)
__device__ inline bool unit_normal(const float *v, float *u)
{
    const float m = fmaxf(fabsf(v[0]), fmaxf(fabsf(v[1]), fabsf(v[2])));
    const bool ok = m > 0.0f;
    const float s = ok ? __builtin_amdgcn_rcpf(m) : 0.0f;
    const float x = v[0] * s, y = v[1] * s, z = v[2] * s;
    const float r = ok ? __builtin_amdgcn_rsqf(x * x + y * y + z * z) : 0.0f;
    u[0] = x * r; u[1] = y * r; u[2] = z * r;
    return ok;
}

struct Sample {
    float e[3], p[3], n[3];
    bool usable;
};

// One full-resolution pixel from its window of samples: slots (sx, sy) of
// the quad's 3 x 3 samples, NX x NY of them starting at (X0S, Y0S); dx, dy
// of slot k are 2 (sx - 1) - i and 2 (sy - 1) - j for pixel (i, j) of the quad.
// Computes E and the flags (L = albedo E / pi is formed by the caller).
template <int I, int J>
__device__ inline void upsample_pixel(const UpsampleArgs &a, const Sample (&s)[9], int64_t pix,
                                      bool on, float (&E)[3], uint32_t &flags)
{
    constexpr int NX = I ? 2 : 3, NY = J ? 2 : 3, X0S = I, Y0S = J;
    E[0] = E[1] = E[2] = 0.f;
    flags = 0;
    const float p[3] = {a.pos[3 * pix], a.pos[3 * pix + 1], a.pos[3 * pix + 2]};
    const float nr[3] = {a.nrm[3 * pix], a.nrm[3 * pix + 1], a.nrm[3 * pix + 2]};
    if (on) {
        float n[3];
        const bool nok = unit_normal(nr, n);
        if (!(finite3(p) && finite3(nr) && nok)) {
            flags = 2u;
        } else {
            for (int c = 0; c < 3; ++c)
                if (p[c] < a.lo[c] || p[c] > a.hi[c]) flags |= 1u;
            bool fac[NX * NY], any = false, have = false;
            float lg[NX * NY], dp[NX * NY], lw[NX * NY];
            int nearest = -1, best = 1 << 30;
            int d2r = 0;
            float lgr = 0.f, pr[3] = {0.f, 0.f, 0.f}, dmin = __builtin_huge_valf();
#pragma unroll
            for (int k = 0; k < NX * NY; ++k) {
                const int sx = X0S + k % NX, sy = Y0S + k / NX, si = sy * 3 + sx;
                const int dx = 2 * (sx - 1) - I, dy = 2 * (sy - 1) - J, d2 = dx * dx + dy * dy;
                const Sample &q = s[si];
                if (q.usable && d2 < best) { best = d2; nearest = si; }
                any |= q.usable;
                const float cs = n[0] * q.n[0] + n[1] * q.n[1] + n[2] * q.n[2];
                fac[k] = q.usable && cs > 0.0f;
                lg[k] = fac[k] ? a.normal_power * __builtin_amdgcn_logf(cs) : 0.0f;
                const float q0 = p[0] - q.p[0], q1 = p[1] - q.p[1], q2 = p[2] - q.p[2];
                dp[k] = q0 * q0 + q1 * q1 + q2 * q2;
                // reference: the facing sample nearest in position
                const bool take = fac[k] && (!have || dp[k] < dmin);
                dmin = take ? dp[k] : dmin;
                d2r = take ? d2 : d2r;
                lgr = take ? lg[k] : lgr;
#pragma unroll
                for (int c = 0; c < 3; ++c) pr[c] = take ? q.p[c] : pr[c];
                have |= fac[k];
            }
            if (have) {
                // log2 weights relative to the reference r; the position term as
                // |p - p_k|^2 - |p - p_r|^2 = (p_r - p_k) . ((p - p_k) + (p - p_r)),
                // which keeps its precision however far the pixel is from the samples
                float lmax = -__builtin_huge_valf();
#pragma unroll
                for (int k = 0; k < NX * NY; ++k) {
                    const int sx = X0S + k % NX, sy = Y0S + k / NX;
                    const int dx = 2 * (sx - 1) - I, dy = 2 * (sy - 1) - J, d2 = dx * dx + dy * dy;
                    const Sample &q = s[sy * 3 + sx];
                    float dd = 0.f;
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        dd = __builtin_fmaf(pr[c] - q.p[c], (p[c] - q.p[c]) + (p[c] - pr[c]), dd);
                    lw[k] = (lg[k] - lgr) - (float)(d2 - d2r) * a.c_px - dd * a.c_pos;
                    if (fac[k]) lmax = fmaxf(lmax, lw[k]);
                }
                float ws = 0.f, acc[3] = {0.f, 0.f, 0.f};
#pragma unroll
                for (int k = 0; k < NX * NY; ++k) {
                    const int sx = X0S + k % NX, sy = Y0S + k / NX;
                    const Sample &q = s[sy * 3 + sx];
                    const float w = fac[k] ? __builtin_amdgcn_exp2f(lw[k] - lmax) : 0.0f;
                    ws += w;
                    acc[0] = __builtin_fmaf(w, q.e[0], acc[0]);
                    acc[1] = __builtin_fmaf(w, q.e[1], acc[1]);
                    acc[2] = __builtin_fmaf(w, q.e[2], acc[2]);
                }
                const float r = __builtin_amdgcn_rcpf(ws);
                E[0] = acc[0] * r; E[1] = acc[1] * r; E[2] = acc[2] * r;
            } else if (any) {
#pragma unroll
                for (int k = 0; k < 9; ++k)
                    if (k == nearest) { E[0] = s[k].e[0]; E[1] = s[k].e[1]; E[2] = s[k].e[2]; }
                flags |= 32u;
            } else {
                flags |= 64u;
            }
        }
    }
}
}  // namespace

// One lane per 2 x 2 pixel quad (2qx + i, 2qy + j): the union of its four
// windows is the 3 x 3 samples qx - 1 .. qx + 1, qy - 1 .. qy + 1, loaded
// once (neighbouring lanes' pixels, through the caches); each pixel then
// visits exactly its own 9, 6, 6 or 4 samples.
__global__ __launch_bounds__(kQuadsX * kQuadsY) void k_upsample(const UpsampleArgs a)
{
    const int qx = blockIdx.x * kQuadsX + (int)(threadIdx.x % kQuadsX);
    const int qy = blockIdx.y * kQuadsY + (int)(threadIdx.x / kQuadsX);
    if (qx >= a.half_w || qy >= a.half_h) return;
    // the 3 x 3 samples: loads at clamped coordinates, all issued before any
    // test, then validity by selects
    Sample s[9];
    float mk[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int x = qx - 1 + k % 3, y = qy - 1 + k / 3;
        const int xc = x < 0 ? 0 : (x >= a.half_w ? a.half_w - 1 : x);
        const int yc = y < 0 ? 0 : (y >= a.half_h ? a.half_h - 1 : y);
        const int64_t i = (int64_t)(2 * yc) * a.width + 2 * xc;
        const int64_t h = (int64_t)yc * a.half_w + xc;
        Sample &q = s[k];
        for (int c = 0; c < 3; ++c) {
            q.p[c] = a.pos[3 * i + c];
            q.n[c] = a.nrm[3 * i + c];
            q.e[c] = a.half_E[3 * h + c];
        }
        mk[k] = (x == xc && y == yc && (a.mask ? a.mask[i] != 0 : true)) ? 1.0f : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        Sample &q = s[k];
        const float raw[3] = {q.n[0], q.n[1], q.n[2]};
        const bool nok = unit_normal(raw, q.n);
        q.usable = mk[k] != 0.0f && finite3(q.p) && finite3(raw) && nok;
    }
    // per row of the quad: both pixels first, then their outputs stored
    // back to back (24 contiguous bytes of E and of L per lane)
    const int X = 2 * qx, Y = 2 * qy;
    const bool xin = X + 1 < a.width;
    const float ip = 0.3183098861837907f;  // 1/pi
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        if (Y + j >= a.height) break;
        const int64_t pa = (int64_t)(Y + j) * a.width + X, pb = pa + 1;
        const bool ona = a.mask ? a.mask[pa] != 0 : true;
        const bool onb = xin && (a.mask ? a.mask[pb] != 0 : true);
        float Ea[3], Eb[3] = {0.f, 0.f, 0.f};
        uint32_t fa, fb = 0;
        if (j == 0) upsample_pixel<0, 0>(a, s, pa, ona, Ea, fa);
        else upsample_pixel<0, 1>(a, s, pa, ona, Ea, fa);
        if (xin) {
            if (j == 0) upsample_pixel<1, 0>(a, s, pb, onb, Eb, fb);
            else upsample_pixel<1, 1>(a, s, pb, onb, Eb, fb);
        }
        float *oe = a.out_E + 3 * pa;
        oe[0] = Ea[0]; oe[1] = Ea[1]; oe[2] = Ea[2];
        if (xin) { oe[3] = Eb[0]; oe[4] = Eb[1]; oe[5] = Eb[2]; }
        if (a.out_L) {
            const float *al = a.albedo + 3 * pa;
            float ra[3] = {0.f, 0.f, 0.f}, rb[3] = {0.f, 0.f, 0.f};
            if (ona) { ra[0] = al[0]; ra[1] = al[1]; ra[2] = al[2]; }
            if (onb) { rb[0] = al[3]; rb[1] = al[4]; rb[2] = al[5]; }
            float *ol = a.out_L + 3 * pa;
            ol[0] = ra[0] * Ea[0] * ip; ol[1] = ra[1] * Ea[1] * ip; ol[2] = ra[2] * Ea[2] * ip;
            if (xin) { ol[3] = rb[0] * Eb[0] * ip; ol[4] = rb[1] * Eb[1] * ip; ol[5] = rb[2] * Eb[2] * ip; }
        }
        if (a.out_flags) {
            a.out_flags[pa] = (uint8_t)fa;
            if (xin) a.out_flags[pb] = (uint8_t)fb;
        }
    }
}

hipError_t launch_upsample(const UpsampleArgs &a, hipStream_t st)
{
    if (a.half_w == 0 || a.half_h == 0) return hipSuccess;
    const dim3 grid((a.half_w + kQuadsX - 1) / kQuadsX, (a.half_h + kQuadsY - 1) / kQuadsY);
    hipLaunchKernelGGL(k_upsample, grid, dim3(kQuadsX * kQuadsY), 0, st, a);
    return hipGetLastError();
}

}  // namespace niv
