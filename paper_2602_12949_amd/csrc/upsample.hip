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

// Samples a workgroup of QX x QY quads can reach: quads qx0 .. qx0 + QX - 1
// use samples qx0 - 1 .. qx0 + QX (the same in y).
constexpr int kSX = kQuadsX + 2, kSY = kQuadsY + 2, kStaged = kSX * kSY;

// Staged samples, one array per component (consecutive lanes read
// consecutive samples: no bank conflicts); u = 0 marks an unusable sample.
struct Staged {
    float ex[kStaged], ey[kStaged], ez[kStaged];
    float px[kStaged], py[kStaged], pz[kStaged];
    float nx[kStaged], ny[kStaged], nz[kStaged];
    float u[kStaged];
};

// E and flags of full-resolution pixel (2qx + I, 2qy + J) from its window
// of staged samples: sx = I .. 2, sy = J .. 2 around the quad's sample
// (sx, sy) = (1, 1) (3 per axis for an even pixel, 2 for an odd one).
template <int I, int J>
__device__ inline void upsample_pixel(const UpsampleArgs &a, const Staged &S, int base, int64_t pix,
                                      bool on, float (&E)[3], uint32_t &flags)
{
    constexpr int NX = I ? 2 : 3, NY = J ? 2 : 3, N = NX * NY;
    E[0] = E[1] = E[2] = 0.f;
    flags = 0;
    const float p[3] = {a.pos[3 * pix], a.pos[3 * pix + 1], a.pos[3 * pix + 2]};
    const float nr[3] = {a.nrm[3 * pix], a.nrm[3 * pix + 1], a.nrm[3 * pix + 2]};
    if (!on) return;
    float n[3];
    const bool nok = unit_normal(nr, n);
    if (!(finite3(p) && finite3(nr) && nok)) {
        flags = 2u;
        return;
    }
    for (int c = 0; c < 3; ++c)
        if (p[c] < a.lo[c] || p[c] > a.hi[c]) flags |= 1u;
    // pass 1: which samples face this pixel, the log2 normal term, the
    // nearest usable sample in pixels and the facing sample nearest in
    // position (the reference of the log-weights)
    bool fac[N];
    float lg[N];
    int nearest = -1, best = 1 << 30, ref = -1;
    float dmin = __builtin_huge_valf();
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const int sx = I + k % NX, sy = J + k / NX, si = base + sy * kSX + sx;
        const int dx = 2 * (sx - 1) - I, dy = 2 * (sy - 1) - J, d2 = dx * dx + dy * dy;
        const bool use = S.u[si] != 0.0f;
        if (use && d2 < best) { best = d2; nearest = si; }
        const float cs = n[0] * S.nx[si] + n[1] * S.ny[si] + n[2] * S.nz[si];
        fac[k] = use && cs > 0.0f;
        lg[k] = fac[k] ? a.normal_power * __builtin_amdgcn_logf(cs) : 0.0f;
        const float q0 = p[0] - S.px[si], q1 = p[1] - S.py[si], q2 = p[2] - S.pz[si];
        const float dp2 = q0 * q0 + q1 * q1 + q2 * q2;
        const bool take = fac[k] && (ref < 0 || dp2 < dmin);
        dmin = take ? dp2 : dmin;
        ref = take ? k : ref;
    }
    if (ref < 0) {
        if (nearest >= 0) {
            E[0] = S.ex[nearest]; E[1] = S.ey[nearest]; E[2] = S.ez[nearest];
            flags |= 32u;
        } else {
            flags |= 64u;
        }
        return;
    }
    // the reference's values (a runtime slot: selected, not indexed)
    float lgr = 0.f, pr[3] = {0.f, 0.f, 0.f};
    int d2r = 0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const int sx = I + k % NX, sy = J + k / NX, si = base + sy * kSX + sx;
        const int dx = 2 * (sx - 1) - I, dy = 2 * (sy - 1) - J, d2 = dx * dx + dy * dy;
        if (k == ref) { lgr = lg[k]; d2r = d2; pr[0] = S.px[si]; pr[1] = S.py[si]; pr[2] = S.pz[si]; }
    }
    // pass 2: log2 weights relative to the reference; the position term as
    // |p - p_k|^2 - |p - p_r|^2 = (p_r - p_k) . ((p - p_k) + (p - p_r)),
    // which keeps its precision however far the pixel is from the samples
    float lw[N], lmax = -__builtin_huge_valf();
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const int sx = I + k % NX, sy = J + k / NX, si = base + sy * kSX + sx;
        const int dx = 2 * (sx - 1) - I, dy = 2 * (sy - 1) - J, d2 = dx * dx + dy * dy;
        const float sp[3] = {S.px[si], S.py[si], S.pz[si]};
        float dd = 0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            dd = __builtin_fmaf(pr[c] - sp[c], (p[c] - sp[c]) + (p[c] - pr[c]), dd);
        lw[k] = (lg[k] - lgr) - (float)(d2 - d2r) * a.c_px - dd * a.c_pos;
        if (fac[k]) lmax = fmaxf(lmax, lw[k]);
    }
    float ws = 0.f, acc[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const int sx = I + k % NX, sy = J + k / NX, si = base + sy * kSX + sx;
        const float w = fac[k] ? __builtin_amdgcn_exp2f(lw[k] - lmax) : 0.0f;
        ws += w;
        acc[0] = __builtin_fmaf(w, S.ex[si], acc[0]);
        acc[1] = __builtin_fmaf(w, S.ey[si], acc[1]);
        acc[2] = __builtin_fmaf(w, S.ez[si], acc[2]);
    }
    const float r = __builtin_amdgcn_rcpf(ws);
    E[0] = acc[0] * r; E[1] = acc[1] * r; E[2] = acc[2] * r;
}
}  // namespace

// One lane per 2 x 2 pixel quad (2qx + i, 2qy + j).  The workgroup first
// stages every sample its quads can reach in LDS (loaded once, coalesced),
// then each pixel visits exactly its own 9, 6, 6 or 4 samples there.
__global__ __launch_bounds__(kQuadsX * kQuadsY) void k_upsample(const UpsampleArgs a)
{
    __shared__ Staged S;
    const int qx0 = blockIdx.x * kQuadsX, qy0 = blockIdx.y * kQuadsY;
    for (int t = threadIdx.x; t < kStaged; t += blockDim.x) {
        const int x = qx0 - 1 + t % kSX, y = qy0 - 1 + t / kSX;
        float e[3] = {0.f, 0.f, 0.f}, p[3] = {0.f, 0.f, 0.f}, n[3] = {0.f, 0.f, 0.f};
        float use = 0.f;
        if (x >= 0 && x < a.half_w && y >= 0 && y < a.half_h) {
            const int64_t i = (int64_t)(2 * y) * a.width + 2 * x;
            const int64_t h = (int64_t)y * a.half_w + x;
            const bool on = a.mask ? a.mask[i] != 0 : true;
            const float pp[3] = {a.pos[3 * i], a.pos[3 * i + 1], a.pos[3 * i + 2]};
            const float nn[3] = {a.nrm[3 * i], a.nrm[3 * i + 1], a.nrm[3 * i + 2]};
            const float ee[3] = {a.half_E[3 * h], a.half_E[3 * h + 1], a.half_E[3 * h + 2]};
            const bool nok = unit_normal(nn, n);
            if (on && finite3(pp) && finite3(nn) && nok) {
                use = 1.f;
                for (int c = 0; c < 3; ++c) { p[c] = pp[c]; e[c] = ee[c]; }
            }
        }
        S.ex[t] = e[0]; S.ey[t] = e[1]; S.ez[t] = e[2];
        S.px[t] = p[0]; S.py[t] = p[1]; S.pz[t] = p[2];
        S.nx[t] = n[0]; S.ny[t] = n[1]; S.nz[t] = n[2];
        S.u[t] = use;
    }
    __syncthreads();
    const int lx = (int)(threadIdx.x % kQuadsX), ly = (int)(threadIdx.x / kQuadsX);
    const int qx = qx0 + lx, qy = qy0 + ly;
    if (qx >= a.half_w || qy >= a.half_h) return;
    const int base = ly * kSX + lx;   // staged sample (qx - 1, qy - 1)
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
        if (j == 0) upsample_pixel<0, 0>(a, S, base, pa, ona, Ea, fa);
        else upsample_pixel<0, 1>(a, S, base, pa, ona, Ea, fa);
        if (xin) {
            if (j == 0) upsample_pixel<1, 0>(a, S, base, pb, onb, Eb, fb);
            else upsample_pixel<1, 1>(a, S, base, pb, onb, Eb, fb);
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
