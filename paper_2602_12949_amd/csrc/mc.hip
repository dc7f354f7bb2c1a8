// Monte Carlo estimate of indirect irradiance (Eq. 1) and the training-point
// sampler (Sec. 4.5, App. H), for gfx950.
//
// One wave per query point: the lanes take samples s = lane, lane+64, ...,
// trace in FP32, sum each sample's value in FP64, and the wave reduces the
// sums (wavefront shuffles) into the mean, the variance of the mean, the
// back-face count and the validity flag.  Random numbers come from a
// counter-based generator (Philox4x64-10) keyed by (seed, point, sample,
// dimension), so any point can be re-estimated independently.
#include <hip/hip_runtime.h>
#include <math.h>
#include <new>
#include <string.h>
#include <vector>

#include "niv_internal.h"

#pragma clang fp contract(off)

#include "mc_device.h"

namespace niv {

struct Prim {
    int32_t kind, axis;
    float sign;
    float p[3], q[3];
    float radius;
    float albedo[3], emission[3];
};
static_assert(sizeof(Prim) == 64, "primitive record is 64 bytes");

typedef const __attribute__((address_space(4))) Prim *ConstPrims;
typedef const __attribute__((address_space(4))) int32_t *ConstInts;

constexpr int kMaxPrims = 4096;
constexpr int kMaxLights = 8;

// ---------------------------------------------------------------- tracing (FP32)
struct Hit {
    float t;
    int prim;
    float n[3];
    bool back;
};

// Closest hit with t > 0; ties go to the lowest primitive index.  The
// slab and plane distances use the ray's reciprocal direction: a box costs
// six FMAs and a min/max tree, and only (t, primitive, back) is tracked in
// the loop; the normal of the winning primitive is rebuilt afterwards.
struct Ray {
    float o[3], d[3], inv[3], oi[3];  // oi = o * inv: a slab distance is fma(x, inv, -oi)
};

__device__ inline Ray make_ray(const float o[3], const float d[3])
{
    Ray r;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r.o[a] = o[a];
        r.d[a] = d[a];
        // a zero component gets a huge finite reciprocal: slab distances keep
        // the sign of (x - o) instead of turning into inf - inf
        r.inv[a] = d[a] != 0.0f ? 1.0f / d[a] : 1e30f;
        r.oi[a] = o[a] * r.inv[a];
    }
    return r;
}

__device__ inline float slab(float x, const Ray &r, int a) { return __builtin_fmaf(x, r.inv[a], -r.oi[a]); }

// Rectangle k perpendicular to axis A (a uniform value, so the caller
// branches once per primitive and every index below is a constant).
template <int A>
__device__ inline void rect_hit(ConstPrims prims, int k, const Ray &r, float &best, int &bp, bool &bback)
{
    constexpr int U = A == 2 ? 0 : A + 1, V = A == 0 ? 2 : A - 1;
    const float t = slab(prims[k].p[A], r, A);
    if (!(t > 0.0f) || !(t < best)) return;
    const float hu = __builtin_fmaf(t, r.d[U], r.o[U]), hv = __builtin_fmaf(t, r.d[V], r.o[V]);
    if (fabsf(hu - prims[k].p[U]) > prims[k].q[0] || fabsf(hv - prims[k].p[V]) > prims[k].q[1]) return;
    best = t;
    bp = k;
    bback = r.d[A] * prims[k].sign > 0.0f;
}

struct Motion4 {
    float x, y, z, w;   // translation per unit of the scene variable; w != 0: moving
};
typedef const __attribute__((address_space(4))) Motion4 *ConstMotion;

// Trace list of a static scene (built by mc_scene_create): the boxes, then
// the rectangles grouped by axis, then the disks, each list in primitive
// order and each record 32 bytes with the primitive's index, so that the
// closest-hit loop runs one kind at a time without a branch on the kind.
struct __attribute__((aligned(32))) TraceRec {
    float a[3];      // box: min corner; rectangle: centre (plane coordinate on its axis)
    int32_t idx;     // primitive index
    float b[3];      // box: max corner; rectangle: half extents u, v, then the facing sign
    int32_t pad;
};
static_assert(sizeof(TraceRec) == 32, "trace record is 32 bytes");
typedef const __attribute__((address_space(4))) TraceRec *ConstRecs;

struct SceneRefs {
    ConstPrims prims;
    int32_t n_prims;
    ConstRecs recs;        // null: test every primitive in order (moving scenes)
    int32_t nb, nr[3], nd;
};

// the ray origin moved by -shift (a primitive translated by shift is tested
// with the translated ray: same distance, side and normal)
__device__ inline Ray shifted(const Ray &r, float sx, float sy, float sz)
{
    Ray q = r;
    q.o[0] = r.o[0] - sx; q.o[1] = r.o[1] - sy; q.o[2] = r.o[2] - sz;
#pragma unroll
    for (int a = 0; a < 3; ++a) q.oi[a] = q.o[a] * q.inv[a];
    return q;
}

// Primitive k against ray r: updates (best, bp, bback).
__device__ inline void prim_hit(ConstPrims prims, int k, const Ray &r, float &best, int &bp, bool &bback)
{
    const int kind = prims[k].kind;
    if (kind == 0) {
        const float x1 = slab(prims[k].p[0], r, 0), x2 = slab(prims[k].q[0], r, 0);
        const float y1 = slab(prims[k].p[1], r, 1), y2 = slab(prims[k].q[1], r, 1);
        const float z1 = slab(prims[k].p[2], r, 2), z2 = slab(prims[k].q[2], r, 2);
        const float tn = fmaxf(fmaxf(fminf(x1, x2), fminf(y1, y2)), fminf(z1, z2));
        const float tf = fminf(fminf(fmaxf(x1, x2), fmaxf(y1, y2)), fmaxf(z1, z2));
        if (!(tn <= tf)) return;
        const bool front = tn > 0.0f;
        const float t = front ? tn : tf;      // from inside: the exit face, seen from behind
        if (t > 0.0f && t < best) { best = t; bp = k; bback = !front; }
    } else if (kind == 1) {
        const int a = prims[k].axis;
        if (a == 0) rect_hit<0>(prims, k, r, best, bp, bback);
        else if (a == 1) rect_hit<1>(prims, k, r, best, bp, bback);
        else rect_hit<2>(prims, k, r, best, bp, bback);
    } else {
        const float nx = prims[k].q[0], ny = prims[k].q[1], nz = prims[k].q[2];
        const float den = r.d[0] * nx + r.d[1] * ny + r.d[2] * nz;
        if (den == 0.0f) return;
        const float t = ((prims[k].p[0] - r.o[0]) * nx + (prims[k].p[1] - r.o[1]) * ny +
                         (prims[k].p[2] - r.o[2]) * nz) / den;
        if (!(t > 0.0f) || !(t < best)) return;
        float r2 = 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float e = __builtin_fmaf(t, r.d[c], r.o[c]) - prims[k].p[c];
            r2 = __builtin_fmaf(e, e, r2);
        }
        if (r2 > prims[k].radius * prims[k].radius) return;
        best = t; bp = k;
        bback = den > 0.0f;
    }
}

// Static scenes: closest hit over the trace list.  Boxes come first in
// primitive order with a strict comparison; rectangles and disks then take a
// hit at the same distance only from a lower primitive index, so ties go to
// the lowest index exactly as in one scan over the primitives.
__device__ inline void trace_list(const SceneRefs &sc, const Ray &r, float &best, int &bp, bool &bback)
{
    ConstRecs rb = sc.recs;
    // one 32-byte record per box, the next one loaded while this one is
    // tested (the list ends with a padding record, so rb[k + 1] is in bounds)
    auto load = [&](int k) {
        TraceRec q;
#pragma unroll
        for (int c = 0; c < 3; ++c) { q.a[c] = rb[k].a[c]; q.b[c] = rb[k].b[c]; }
        q.idx = rb[k].idx;
        q.pad = 0;
        return q;
    };
    TraceRec cur = load(0);
    for (int k = 0; k < sc.nb; ++k) {
        const TraceRec nxt = load(k + 1);
        const float x1 = slab(cur.a[0], r, 0), x2 = slab(cur.b[0], r, 0);
        const float y1 = slab(cur.a[1], r, 1), y2 = slab(cur.b[1], r, 1);
        const float z1 = slab(cur.a[2], r, 2), z2 = slab(cur.b[2], r, 2);
        const float tn = fmaxf(fmaxf(fminf(x1, x2), fminf(y1, y2)), fminf(z1, z2));
        const float tf = fminf(fminf(fmaxf(x1, x2), fmaxf(y1, y2)), fmaxf(z1, z2));
        const bool front = tn > 0.0f;
        const float t = front ? tn : tf;      // from inside: the exit face, seen from behind
        // t > 0 is tf > 0 here: with tn > 0, tn <= tf makes tf positive
        const bool take = (tn <= tf) && (tf > 0.0f) && (t < best);
        best = take ? t : best;
        bp = take ? cur.idx : bp;
        bback = take ? !front : bback;
        cur = nxt;
    }
    rb += sc.nb;
    auto rects = [&](auto axis, int n) {
        constexpr int A = decltype(axis)::value;
        constexpr int U = A == 2 ? 0 : A + 1, V = A == 0 ? 2 : A - 1;
        for (int k = 0; k < n; ++k) {
            const float t = slab(rb[k].a[A], r, A);
            const float hu = __builtin_fmaf(t, r.d[U], r.o[U]), hv = __builtin_fmaf(t, r.d[V], r.o[V]);
            const int id = rb[k].idx;
            const bool take = (t > 0.0f) && ((t < best) || ((t == best) && (id < bp))) &&
                              (fabsf(hu - rb[k].a[U]) <= rb[k].b[0]) && (fabsf(hv - rb[k].a[V]) <= rb[k].b[1]);
            best = take ? t : best;
            bp = take ? id : bp;
            bback = take ? (r.d[A] * rb[k].b[2] > 0.0f) : bback;
        }
        rb += n;
    };
    rects(std::integral_constant<int, 0>(), sc.nr[0]);
    rects(std::integral_constant<int, 1>(), sc.nr[1]);
    rects(std::integral_constant<int, 2>(), sc.nr[2]);
    for (int k = 0; k < sc.nd; ++k) {
        const int id = rb[k].idx;
        ConstPrims pd = sc.prims + id;
        const float nx = pd->q[0], ny = pd->q[1], nz = pd->q[2];
        const float den = r.d[0] * nx + r.d[1] * ny + r.d[2] * nz;
        const float t = ((pd->p[0] - r.o[0]) * nx + (pd->p[1] - r.o[1]) * ny + (pd->p[2] - r.o[2]) * nz) / den;
        float r2 = 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float e = __builtin_fmaf(t, r.d[c], r.o[c]) - pd->p[c];
            r2 = __builtin_fmaf(e, e, r2);
        }
        const bool take = (den != 0.0f) && (t > 0.0f) && ((t < best) || ((t == best) && (id < bp))) &&
                          (r2 <= pd->radius * pd->radius);
        best = take ? t : best;
        bp = take ? id : bp;
        bback = take ? (den > 0.0f) : bback;
    }
}

// MOVING: the scene changes with the point's scene variable tv (uniform over
// the wave): primitive k is translated by tv * motion[k] (motion[k].w != 0
// marks a moving primitive).
template <bool MOVING>
__device__ inline bool trace(const SceneRefs &sc, const float o[3], const float d[3],
                             Hit &h, ConstMotion motion = nullptr, float tv = 0.0f)
{
    ConstPrims prims = sc.prims;
    const Ray r = make_ray(o, d);
    float best = INFINITY;
    int bp = -1;
    bool bback = false;
    if (!MOVING && sc.recs) {
        trace_list(sc, r, best, bp, bback);
    } else {
        for (int k = 0; k < sc.n_prims; ++k) {
            if (MOVING && motion[k].w != 0.0f)
                prim_hit(prims, k, shifted(r, tv * motion[k].x, tv * motion[k].y, tv * motion[k].z),
                         best, bp, bback);
            else
                prim_hit(prims, k, r, best, bp, bback);
        }
    }
    h.t = best;
    h.prim = bp;
    h.back = bback;
    h.n[0] = h.n[1] = h.n[2] = 0.0f;
    if (bp < 0) return false;
    // the winning primitive differs between lanes: per-lane loads, and the
    // normal is assembled with selects (no indexing of a register array)
    const int kind = prims[bp].kind;
    if (kind == 0) {
        Ray rb = r;
        if constexpr (MOVING) {
            if (motion[bp].w != 0.0f)
                rb = shifted(r, tv * motion[bp].x, tv * motion[bp].y, tv * motion[bp].z);
        }
        // the face whose slab distance is the hit distance: entry (front) or exit (back)
        float n3[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float t1 = slab(prims[bp].p[c], rb, c), t2 = slab(prims[bp].q[c], rb, c);
            const float tc = bback ? fmaxf(t1, t2) : fminf(t1, t2);
            n3[c] = tc == best ? ((r.d[c] > 0.0f) != bback ? -1.0f : 1.0f) : 0.0f;
        }
        // a hit exactly on an edge matches two faces: keep the last, as a scan would
        if (n3[2] != 0.0f) { n3[0] = 0.0f; n3[1] = 0.0f; }
        else if (n3[1] != 0.0f) n3[0] = 0.0f;
        h.n[0] = n3[0]; h.n[1] = n3[1]; h.n[2] = n3[2];
        if (n3[0] == 0.0f && n3[1] == 0.0f && n3[2] == 0.0f) h.n[0] = (r.d[0] > 0.0f) != bback ? -1.0f : 1.0f;
    } else if (kind == 1) {
        const int ax = prims[bp].axis;
        const float sg = prims[bp].sign;
        h.n[0] = ax == 0 ? sg : 0.0f;
        h.n[1] = ax == 1 ? sg : 0.0f;
        h.n[2] = ax == 2 ? sg : 0.0f;
    } else {
        h.n[0] = prims[bp].q[0]; h.n[1] = prims[bp].q[1]; h.n[2] = prims[bp].q[2];
    }
    return true;
}

// Uniform point on a light's front surface; returns its area.
__device__ inline float light_point(ConstPrims prims, int k, float u1, float u2, float q[3],
                                    float nq[3])
{
    if (prims[k].kind == 1) {
        const int a = prims[k].axis, uu = (a + 1) % 3, vv = (a + 2) % 3;
        q[a] = prims[k].p[a];
        q[uu] = prims[k].p[uu] + (2.0f * u1 - 1.0f) * prims[k].q[0];
        q[vv] = prims[k].p[vv] + (2.0f * u2 - 1.0f) * prims[k].q[1];
        nq[0] = nq[1] = nq[2] = 0.0f;
        nq[a] = prims[k].sign;
        return 4.0f * prims[k].q[0] * prims[k].q[1];
    }
    float n[3] = {prims[k].q[0], prims[k].q[1], prims[k].q[2]}, t[3], b[3];
    onb(n, t, b);
    float r = prims[k].radius * sqrtf(u1), phi = 6.28318530717958647692f * u2;
    float sp, cp;
    sincosf(phi, &sp, &cp);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        q[a] = prims[k].p[a] + r * (cp * t[a] + sp * b[a]);
        nq[a] = n[a];
    }
    return 3.14159265358979323846f * prims[k].radius * prims[k].radius;
}

struct McArgs {
    const Prim *prims;
    const TraceRec *recs;     // trace list of the static scene
    int32_t nb, nr[3], nd;
    const int32_t *lights;
    const Motion4 *motion;    // [n_prims] (x, y, z, moving) or null
    const float *t;           // [count] scene variable per point or null (0)
    int32_t n_prims, n_lights;
    float eps;
    int32_t spp, bounces, flags;
    uint64_t seed;
    const float *x, *nrm;
    int64_t count;
    double *out_E, *out_var;
    float *out_E32;
    int32_t *out_backfaces;
    uint8_t *out_valid;
};

// Next-event estimate at y with normal ny toward light j: L cos cos / d^2 A.
template <bool MOVING>
__device__ inline bool nee(const SceneRefs &sc, int lk, const float oy[3],
                           const float ny[3], float u1, float u2, float &G, ConstMotion motion,
                           float tv)
{
    float q[3], nq[3];
    float A = light_point(sc.prims, lk, u1, u2, q, nq);
    if constexpr (MOVING) {
        q[0] += tv * motion[lk].x; q[1] += tv * motion[lk].y; q[2] += tv * motion[lk].z;
    }
    float w[3] = {q[0] - oy[0], q[1] - oy[1], q[2] - oy[2]};
    float d2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2], il = 1.0f / sqrtf(d2);
#pragma unroll
    for (int a = 0; a < 3; ++a) w[a] *= il;
    float cy = ny[0] * w[0] + ny[1] * w[1] + ny[2] * w[2];
    float cq = -(nq[0] * w[0] + nq[1] * w[1] + nq[2] * w[2]);
    if (cy <= 0.0f || cq <= 0.0f) return false;
    Hit hh;
    if (!trace<MOVING>(sc, oy, w, hh, motion, tv) || hh.prim != lk) return false;
    G = cy * cq / d2 * A;
    return true;
}

// Wave-cooperative estimate at one point: lanes take samples lane, lane+64,
// ...; returns (in every lane) the FP64 sums of the sample values and of
// their squares, and the back-face count.
template <bool MOVING>
__device__ inline void mc_point(const SceneRefs &sc, ConstInts lights, int J, float eps,
                                const float px[3], const float pn_in[3], int spp, int bounces,
                                int flags, uint64_t seed, uint64_t point, int lane, double s1[3],
                                double s2[3], int &backs, ConstMotion motion, float tv)
{
    ConstPrims prims = sc.prims;
    const int stride = 2 * J + 2;
    float pn[3] = {pn_in[0], pn_in[1], pn_in[2]};
    const float ln = sqrtf(pn[0] * pn[0] + pn[1] * pn[1] + pn[2] * pn[2]);
#pragma unroll
    for (int c = 0; c < 3; ++c) pn[c] /= ln;
    for (int c = 0; c < 3; ++c) { s1[c] = 0.0; s2[c] = 0.0; }
    backs = 0;
    for (int s = lane; s < spp; s += 64) {
        Rng rng(seed, point, (uint64_t)s, 0);
        float val[3] = {0.f, 0.f, 0.f};
        float o[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) o[c] = px[c] + eps * pn[c];
        if (flags & 8) {  // direct irradiance at x by light sampling (test mode)
            for (int j = 0; j < J; ++j) {
                int lk = lights[j];
                float G;
                if (nee<MOVING>(sc, lk, o, pn, rng.u(2 * j), rng.u(2 * j + 1), G, motion, tv))
                    for (int c = 0; c < 3; ++c) val[c] += prims[lk].emission[c] * G;
            }
        } else {
            float d[3];
            cosine_dir(pn, rng.u(0), rng.u(1), d);
            Hit h;
            bool ok = trace<MOVING>(sc, o, d, h, motion, tv);
            if (ok && h.back) { backs++; ok = false; }
            if (ok) {
                float rad[3] = {0.f, 0.f, 0.f};
                if (flags & 4)
                    for (int c = 0; c < 3; ++c) rad[c] += prims[h.prim].emission[c];
                float beta[3] = {1.f, 1.f, 1.f};
                float y[3], ny[3];
                for (int c = 0; c < 3; ++c) { y[c] = o[c] + h.t * d[c]; ny[c] = h.n[c]; }
                for (int k = 1; k <= bounces; ++k) {
                    const int pk = h.prim;
                    float rho[3] = {prims[pk].albedo[0], prims[pk].albedo[1], prims[pk].albedo[2]};
                    const int base = 2 + (k - 1) * stride;
                    float oy[3];
                    for (int c = 0; c < 3; ++c) oy[c] = y[c] + eps * ny[c];
                    if (flags & 1) {
                        for (int j = 0; j < J; ++j) {
                            int lk = lights[j];
                            float G;
                            if (nee<MOVING>(sc, lk, oy, ny, rng.u(base + 2 * j), rng.u(base + 2 * j + 1), G,
                                            motion, tv))
                                for (int c = 0; c < 3; ++c)
                                    rad[c] += beta[c] * rho[c] * 0.318309886183790672f * prims[lk].emission[c] * G;
                        }
                    }
                    const bool cont = (flags & 2) ? true : (k < bounces);
                    if (!cont) break;
                    for (int c = 0; c < 3; ++c) beta[c] *= rho[c];
                    if (beta[0] == 0.f && beta[1] == 0.f && beta[2] == 0.f) break;
                    cosine_dir(ny, rng.u(base + 2 * J), rng.u(base + 2 * J + 1), d);
                    if (!trace<MOVING>(sc, oy, d, h, motion, tv) || h.back) break;
                    if (flags & 2)
                        for (int c = 0; c < 3; ++c) rad[c] += beta[c] * prims[h.prim].emission[c];
                    for (int c = 0; c < 3; ++c) { y[c] = oy[c] + h.t * d[c]; ny[c] = h.n[c]; }
                }
                for (int c = 0; c < 3; ++c) val[c] = 3.14159265358979323846f * rad[c];
            }
        }
        for (int c = 0; c < 3; ++c) {
            double v = (double)val[c];
            s1[c] += v;
            s2[c] += v * v;
        }
    }
    // wave reduction (FP64 sums, integer back-face count)
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        for (int c = 0; c < 3; ++c) {
            s1[c] += __shfl_xor(s1[c], off);
            s2[c] += __shfl_xor(s2[c], off);
        }
        backs += __shfl_xor(backs, off);
    }
}

template <bool MOVING>
__global__ __launch_bounds__(256) void k_mc_irradiance(const McArgs a)
{
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= a.count) return;  // whole wave leaves together
    SceneRefs sc;
    sc.prims = (ConstPrims)a.prims;
    sc.n_prims = a.n_prims;
    sc.recs = (ConstRecs)a.recs;
    sc.nb = a.nb;
    sc.nr[0] = a.nr[0]; sc.nr[1] = a.nr[1]; sc.nr[2] = a.nr[2];
    sc.nd = a.nd;
    ConstInts lights = (ConstInts)a.lights;
    const float px[3] = {a.x[3 * i], a.x[3 * i + 1], a.x[3 * i + 2]};
    const float pn[3] = {a.nrm[3 * i], a.nrm[3 * i + 1], a.nrm[3 * i + 2]};
    double s1[3], s2[3];
    int backs;
    const float tv = (MOVING && a.t) ? a.t[i] : 0.0f;
    mc_point<MOVING>(sc, lights, a.n_lights, a.eps, px, pn, a.spp, a.bounces, a.flags,
                     a.seed, (uint64_t)i, lane, s1, s2, backs, (ConstMotion)a.motion, tv);
    if (lane == 0) {
        const double S = (double)a.spp;
        bool any = false;
        for (int c = 0; c < 3; ++c) {
            double mean = s1[c] / S;
            double var = a.spp > 1 ? (s2[c] - S * mean * mean) / (S - 1.0) / S : 0.0;
            if (var < 0.0) var = 0.0;
            if (a.out_E) a.out_E[3 * i + c] = mean;
            if (a.out_E32) a.out_E32[3 * i + c] = (float)mean;
            if (a.out_var) a.out_var[3 * i + c] = var;
            any |= mean > 0.0;
        }
        if (a.out_backfaces) a.out_backfaces[i] = backs;
        if (a.out_valid) a.out_valid[i] = (uint8_t)((2 * backs <= a.spp) && any);
    }
}

// Monte Carlo replacement of the pixels a query appended to its fallback
// list (one wave per pixel, persistent grid, length read on the device).
template <bool MOVING>
__global__ __launch_bounds__(256) void k_mc_fallback(const FbArgs a)
{
    typedef const __attribute__((address_space(4))) FbArgs *ConstFb;
    ConstFb ka = (ConstFb)__builtin_amdgcn_kernarg_segment_ptr();
    const int lane = threadIdx.x & 63;
    const uint32_t n = *a.count < a.cap ? *a.count : a.cap;
    for (uint32_t e = blockIdx.x * 4 + (threadIdx.x >> 6); e < n; e += gridDim.x * 4) {
        const uint32_t code = __builtin_amdgcn_readfirstlane(a.list[e]);
        const int fi = (int)(code >> 28);
        const int64_t q = code & 0x0fffffffu;
        if (!ka->f[fi].prims) continue;
        SceneRefs sc;
        sc.prims = (ConstPrims)ka->f[fi].prims;
        sc.n_prims = ka->f[fi].n_prims;
        sc.recs = (ConstRecs)ka->f[fi].recs;
        sc.nb = ka->f[fi].nk[0];
        sc.nr[0] = ka->f[fi].nk[1]; sc.nr[1] = ka->f[fi].nk[2]; sc.nr[2] = ka->f[fi].nk[3];
        sc.nd = ka->f[fi].nk[4];
        ConstInts lights = (ConstInts)ka->f[fi].lights;
        const float *pos = ka->f[fi].pos, *nrm = ka->f[fi].nrm;
        const float px[3] = {pos[3 * q], pos[3 * q + 1], pos[3 * q + 2]};
        const float pn[3] = {nrm[3 * q], nrm[3 * q + 1], nrm[3 * q + 2]};
        double s1[3], s2[3];
        int backs;
        // MOVING: the frames' scenes change with the frame's scene variable;
        // a static scene in such a launch has no motion table and reads none
        const bool moving = MOVING && ka->f[fi].motion != nullptr;
        if (moving)
            mc_point<MOVING>(sc, lights, ka->f[fi].n_lights, ka->f[fi].eps, px, pn,
                             a.spp, a.bounces, a.flags, a.seed, (uint64_t)code, lane, s1, s2, backs,
                             (ConstMotion)ka->f[fi].motion, ka->f[fi].t);
        else
            mc_point<false>(sc, lights, ka->f[fi].n_lights, ka->f[fi].eps, px, pn,
                            a.spp, a.bounces, a.flags, a.seed, (uint64_t)code, lane, s1, s2, backs,
                            nullptr, 0.0f);
        if (lane == 0) {
            float *oE = ka->f[fi].out_E, *oL = ka->f[fi].out_L;
            const float *alb = ka->f[fi].albedo;
            for (int c = 0; c < 3; ++c) {
                const float E = (float)(s1[c] / (double)a.spp);
                oE[3 * q + c] = E;
                if (oL) oL[3 * q + c] = alb[3 * q + c] * E * 0.3183098861837907f;
            }
            uint8_t *of = ka->f[fi].out_flags;
            if (of) of[q] = (uint8_t)(of[q] | 8u);
        }
    }
}

// ---------------------------------------------------------------- sampler
struct SampleArgs {
    const Prim *prims;
    const int32_t *face_prim;   // per non-emitting face: primitive
    const int32_t *face_id;     // -1 for a rectangle, 0..5 for a box face
    const double *cdf;          // cumulative area
    int32_t n_faces;
    double total_area;
    double lo[3], hi[3];
    int64_t count, n_surface;
    uint64_t seed;
    float *out_x, *out_n;
    float *out_t;               // scene variable per point (dimension 7), or null
};

__device__ inline double u64(Rng &r, int d) { return (double)r.u(d); }

__global__ __launch_bounds__(256) void k_sample_points(const SampleArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.count) return;
    ConstPrims prims = (ConstPrims)a.prims;
    Rng rng(a.seed, (uint64_t)i, 0, 1);
    double u0 = u64(rng, 0), u1 = u64(rng, 1), u2 = u64(rng, 2);
    double p[3], n[3] = {0.0, 0.0, 0.0};
    if (i < a.count - a.n_surface) {
        double u3 = u64(rng, 3), u4 = u64(rng, 4);
        for (int c = 0; c < 3; ++c) {
            double uc = c == 0 ? u0 : (c == 1 ? u1 : u2);
            p[c] = a.lo[c] + uc * (a.hi[c] - a.lo[c]);
        }
        double z = 1.0 - 2.0 * u3, phi = 2.0 * 3.14159265358979323846 * u4;
        double r = sqrt(fmax(0.0, 1.0 - z * z));
        double sp, cp;
        sincos(phi, &sp, &cp);
        n[0] = r * cp; n[1] = r * sp; n[2] = z;
    } else {
        double target = u0 * a.total_area;
        int lo_i = 0, hi_i = a.n_faces - 1;
        while (lo_i < hi_i) {
            int mid = (lo_i + hi_i) / 2;
            if (a.cdf[mid] > target) hi_i = mid; else lo_i = mid + 1;
        }
        const int k = a.face_prim[lo_i], f = a.face_id[lo_i];
        if (f < 0) {
            const int ax = prims[k].axis, uu = (ax + 1) % 3, vv = (ax + 2) % 3;
            p[ax] = prims[k].p[ax];
            p[uu] = prims[k].p[uu] + (2.0 * u1 - 1.0) * prims[k].q[0];
            p[vv] = prims[k].p[vv] + (2.0 * u2 - 1.0) * prims[k].q[1];
            n[ax] = prims[k].sign;
        } else {
            const int ax = f / 2, uu = (ax + 1) % 3, vv = (ax + 2) % 3;
            p[ax] = (f & 1) ? prims[k].q[ax] : prims[k].p[ax];
            p[uu] = prims[k].p[uu] + u1 * ((double)prims[k].q[uu] - prims[k].p[uu]);
            p[vv] = prims[k].p[vv] + u2 * ((double)prims[k].q[vv] - prims[k].p[vv]);
            n[ax] = (f & 1) ? 1.0 : -1.0;
        }
    }
    for (int c = 0; c < 3; ++c) {
        a.out_x[3 * i + c] = (float)p[c];
        a.out_n[3 * i + c] = (float)n[c];
    }
    if (a.out_t) a.out_t[i] = rng.u(7);
}

}  // namespace niv

using namespace niv;

struct mc_scene {
    Prim *d_prims = nullptr;       // device copy of the primitives
    int32_t *d_lights = nullptr;   // indices of emitting primitives
    int32_t *d_face_prim = nullptr, *d_face_id = nullptr;
    double *d_cdf = nullptr;
    Motion4 *d_motion = nullptr;   // per primitive (x, y, z, moving), or null: static scene
    TraceRec *d_recs = nullptr;    // trace list: boxes, rectangles by axis, disks
    int32_t nk[5] = {0, 0, 0, 0, 0};  // their counts (boxes, rectangles x/y/z, disks)
    int32_t n_prims = 0, n_lights = 0, n_faces = 0;
    double total_area = 0.0;
    float eps = 0.0f;
    std::vector<Prim> prims;       // host copy (rebuilds the sampler's face table)
};

namespace niv {
void mc_scene_device_view(const struct mc_scene *s, const void **prims, const int32_t **lights,
                          int32_t *n_prims, int32_t *n_lights, float *eps, const void **motion)
{
    *prims = s ? s->d_prims : nullptr;
    *lights = s ? s->d_lights : nullptr;
    *n_prims = s ? s->n_prims : 0;
    *n_lights = s ? s->n_lights : 0;
    *eps = s ? s->eps : 0.0f;
    *motion = s ? s->d_motion : nullptr;
}

void mc_scene_trace_view(const struct mc_scene *s, const void **recs, int32_t nk[5])
{
    *recs = s ? s->d_recs : nullptr;
    for (int k = 0; k < 5; ++k) nk[k] = s ? s->nk[k] : 0;
}

hipError_t launch_mc_fallback(const FbArgs &a, hipStream_t stream)
{
    static int n_cu = 0;
    if (n_cu == 0) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
    }
    bool moving = false;
    for (int f = 0; f < kMaxFrames; ++f) moving |= a.f[f].motion != nullptr;
    if (moving)
        hipLaunchKernelGGL(k_mc_fallback<true>, dim3((unsigned)(n_cu * 8)), dim3(256), 0, stream, a);
    else
        hipLaunchKernelGGL(k_mc_fallback<false>, dim3((unsigned)(n_cu * 8)), dim3(256), 0, stream, a);
    return hipGetLastError();
}
}  // namespace niv

namespace {
niv_status hs(hipError_t e) { return e == hipSuccess ? NIV_OK : NIV_ERR_HIP; }
bool is_light(const Prim &p) { return p.emission[0] > 0.f || p.emission[1] > 0.f || p.emission[2] > 0.f; }
void release(mc_scene *s)
{
    if (!s) return;
    (void)hipFree(s->d_prims);
    (void)hipFree(s->d_lights);
    (void)hipFree(s->d_face_prim);
    (void)hipFree(s->d_face_id);
    (void)hipFree(s->d_cdf);
    (void)hipFree(s->d_motion);
    (void)hipFree(s->d_recs);
    delete s;
}

// Trace list of the static scene: boxes, rectangles perpendicular to x, y
// and z, disks; each list in primitive order.
niv_status upload_trace_list(mc_scene *s)
{
    std::vector<TraceRec> lists[5];
    for (int k = 0; k < s->n_prims; ++k) {
        const Prim &p = s->prims[k];
        TraceRec r;
        memset(&r, 0, sizeof(r));
        r.idx = k;
        if (p.kind == 0) {
            for (int c = 0; c < 3; ++c) { r.a[c] = p.p[c]; r.b[c] = p.q[c]; }
            lists[0].push_back(r);
        } else if (p.kind == 1) {
            for (int c = 0; c < 3; ++c) r.a[c] = p.p[c];
            r.b[0] = p.q[0];
            r.b[1] = p.q[1];
            r.b[2] = p.sign;
            lists[1 + p.axis].push_back(r);
        } else {
            lists[4].push_back(r);
        }
    }
    std::vector<TraceRec> all;
    for (int l = 0; l < 5; ++l) {
        s->nk[l] = (int32_t)lists[l].size();
        all.insert(all.end(), lists[l].begin(), lists[l].end());
    }
    TraceRec pad;   // read ahead by the box loop, never tested
    memset(&pad, 0, sizeof(pad));
    all.push_back(pad);
    niv_status st = hs(hipMalloc(&s->d_recs, sizeof(TraceRec) * all.size()));
    if (st == NIV_OK)
        st = hs(hipMemcpy(s->d_recs, all.data(), sizeof(TraceRec) * all.size(), hipMemcpyHostToDevice));
    return st;
}
// Cumulative-area table of the sampler's surfaces: every rectangle and box
// face that does not emit and does not move.
niv_status upload_faces(mc_scene *s, const float *motion)
{
    const int n = s->n_prims;
    std::vector<int32_t> fp, ff;
    std::vector<double> cdf;
    double acc = 0.0;
    for (int k = 0; k < n; ++k) {
        const Prim &p = s->prims[k];
        if (is_light(p)) continue;
        if (motion && (motion[3 * k] != 0.f || motion[3 * k + 1] != 0.f || motion[3 * k + 2] != 0.f)) continue;
        if (p.kind == 1) {
            acc += 4.0 * (double)p.q[0] * p.q[1];
            fp.push_back(k); ff.push_back(-1); cdf.push_back(acc);
        } else if (p.kind == 0) {
            for (int f = 0; f < 6; ++f) {
                int ax = f / 2, u = (ax + 1) % 3, v = (ax + 2) % 3;
                acc += ((double)p.q[u] - p.p[u]) * ((double)p.q[v] - p.p[v]);
                fp.push_back(k); ff.push_back(f); cdf.push_back(acc);
            }
        }
    }
    const int nf = (int)fp.size();
    s->n_faces = nf;
    s->total_area = acc;
    niv_status st = NIV_OK;
    if (!s->d_face_prim) {
        // room for every face of every primitive, so a later table fits too
        st = hs(hipMalloc(&s->d_face_prim, sizeof(int32_t) * (6 * n + 1)));
        if (st == NIV_OK) st = hs(hipMalloc(&s->d_face_id, sizeof(int32_t) * (6 * n + 1)));
        if (st == NIV_OK) st = hs(hipMalloc(&s->d_cdf, sizeof(double) * (6 * n + 1)));
    }
    if (st == NIV_OK && nf > 0) {
        st = hs(hipMemcpy(s->d_face_prim, fp.data(), sizeof(int32_t) * nf, hipMemcpyHostToDevice));
        if (st == NIV_OK) st = hs(hipMemcpy(s->d_face_id, ff.data(), sizeof(int32_t) * nf, hipMemcpyHostToDevice));
        if (st == NIV_OK) st = hs(hipMemcpy(s->d_cdf, cdf.data(), sizeof(double) * nf, hipMemcpyHostToDevice));
    }
    return st;
}
}  // namespace

extern "C" {

niv_status mc_scene_create(const niv_mc_prim *prims, int32_t n_prims, mc_scene **out)
{
    if (!out || !prims || n_prims < 1 || n_prims > kMaxPrims) return NIV_ERR_INVALID_ARG;
    *out = nullptr;
    const Prim *P = reinterpret_cast<const Prim *>(prims);
    mc_scene *s = new (std::nothrow) mc_scene;
    if (!s) return NIV_ERR_INVALID_ARG;
    // lights, scene extent (for the ray offset), surface table for the sampler
    int32_t lights[kMaxLights];
    int n_lights = 0;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    niv_status st = NIV_OK;
    for (int k = 0; k < n_prims && st == NIV_OK; ++k) {
        const Prim &p = P[k];
        if (p.kind < 0 || p.kind > 2 || (p.kind == 1 && (p.axis < 0 || p.axis > 2))) {
            st = NIV_ERR_INVALID_ARG;
            break;
        }
        if (is_light(p)) {
            if (n_lights == kMaxLights || p.kind == 0) { st = NIV_ERR_UNSUPPORTED; break; }
            lights[n_lights++] = k;
        }
        double a[3], b[3];
        if (p.kind == 0) {
            for (int c = 0; c < 3; ++c) { a[c] = p.p[c]; b[c] = p.q[c]; }
        } else if (p.kind == 1) {
            int ax = p.axis, u = (ax + 1) % 3, v = (ax + 2) % 3;
            for (int c = 0; c < 3; ++c) a[c] = b[c] = p.p[c];
            a[u] -= p.q[0]; b[u] += p.q[0]; a[v] -= p.q[1]; b[v] += p.q[1];
        } else {
            for (int c = 0; c < 3; ++c) { a[c] = p.p[c] - p.radius; b[c] = p.p[c] + p.radius; }
        }
        for (int c = 0; c < 3; ++c) {
            if (a[c] < lo[c]) lo[c] = a[c];
            if (b[c] > hi[c]) hi[c] = b[c];
        }
    }
    if (st == NIV_OK) {
        double extent = 0.0;
        for (int c = 0; c < 3; ++c) extent = fmax(extent, hi[c] - lo[c]);
        s->eps = (float)(1e-4 * extent);
        s->n_prims = n_prims;
        s->n_lights = n_lights;
        s->prims.assign(P, P + n_prims);
        st = hs(hipMalloc(&s->d_prims, sizeof(Prim) * n_prims));
        if (st == NIV_OK) st = hs(hipMalloc(&s->d_lights, sizeof(int32_t) * kMaxLights));
        if (st == NIV_OK) st = hs(hipMemcpy(s->d_prims, P, sizeof(Prim) * n_prims, hipMemcpyHostToDevice));
        if (st == NIV_OK) st = hs(hipMemcpy(s->d_lights, lights, sizeof(int32_t) * kMaxLights, hipMemcpyHostToDevice));
        if (st == NIV_OK) st = upload_faces(s, nullptr);
        if (st == NIV_OK) st = upload_trace_list(s);
    }
    if (st != NIV_OK) {
        release(s);
        return st;
    }
    *out = s;
    return NIV_OK;
}

niv_status mc_scene_set_motion(mc_scene *s, const float *motion)
{
    if (!s) return NIV_ERR_INVALID_ARG;
    if (motion)
        for (int k = 0; k < 3 * s->n_prims; ++k)
            if (!isfinite(motion[k])) return NIV_ERR_INVALID_ARG;
    niv_status st = NIV_OK;
    if (!motion) {
        (void)hipFree(s->d_motion);
        s->d_motion = nullptr;
    } else {
        std::vector<Motion4> m(s->n_prims);
        for (int k = 0; k < s->n_prims; ++k) {
            const float x = motion[3 * k], y = motion[3 * k + 1], z = motion[3 * k + 2];
            m[k] = Motion4{x, y, z, (x != 0.f || y != 0.f || z != 0.f) ? 1.0f : 0.0f};
        }
        if (!s->d_motion) st = hs(hipMalloc(&s->d_motion, sizeof(Motion4) * s->n_prims));
        if (st == NIV_OK)
            st = hs(hipMemcpy(s->d_motion, m.data(), sizeof(Motion4) * s->n_prims, hipMemcpyHostToDevice));
    }
    // surface training points only on what does not move
    if (st == NIV_OK) st = upload_faces(s, motion);
    return st;
}

void mc_scene_destroy(mc_scene *s) { release(s); }

niv_status mc_irradiance_at(const mc_scene *s, const float *x, const float *nrm, const float *t,
                            int64_t count, int32_t spp, int32_t bounces, int32_t flags, uint64_t seed,
                            double *out_E, float *out_E32, double *out_var, int32_t *out_backfaces,
                            uint8_t *out_valid, hipStream_t stream)
{
    if (!s || count < 0 || spp < 1 || bounces < 0 || bounces > 16 || (flags & ~15)) return NIV_ERR_INVALID_ARG;
    if ((flags & 1) && (flags & 2)) return NIV_ERR_INVALID_ARG;  // NEE and emission-on-hit exclude each other
    if (count == 0) return NIV_OK;
    if (!x || !nrm || (!out_E && !out_E32)) return NIV_ERR_INVALID_ARG;
    if (2 + bounces * (2 * s->n_lights + 2) > 1 << 20) return NIV_ERR_INVALID_ARG;
    McArgs a;
    memset(&a, 0, sizeof(a));
    a.prims = s->d_prims;
    a.recs = s->d_recs;
    a.nb = s->nk[0];
    for (int c = 0; c < 3; ++c) a.nr[c] = s->nk[1 + c];
    a.nd = s->nk[4];
    a.lights = s->d_lights;
    a.motion = s->d_motion;
    a.t = t;
    a.n_prims = s->n_prims;
    a.n_lights = s->n_lights;
    a.eps = s->eps;
    a.spp = spp;
    a.bounces = bounces;
    a.flags = flags;
    a.seed = seed;
    a.x = x;
    a.nrm = nrm;
    a.count = count;
    a.out_E = out_E;
    a.out_E32 = out_E32;
    a.out_var = out_var;
    a.out_backfaces = out_backfaces;
    a.out_valid = out_valid;
    int64_t blocks = (count + 3) / 4;
    if (blocks > 0x7fffffff) return NIV_ERR_INVALID_ARG;
    if (s->d_motion)
        hipLaunchKernelGGL(k_mc_irradiance<true>, dim3((unsigned)blocks), dim3(256), 0, stream, a);
    else
        hipLaunchKernelGGL(k_mc_irradiance<false>, dim3((unsigned)blocks), dim3(256), 0, stream, a);
    return hs(hipGetLastError());
}

niv_status mc_irradiance(const mc_scene *s, const float *x, const float *nrm, int64_t count,
                         int32_t spp, int32_t bounces, int32_t flags, uint64_t seed,
                         double *out_E, float *out_E32, double *out_var, int32_t *out_backfaces,
                         uint8_t *out_valid, hipStream_t stream)
{
    return mc_irradiance_at(s, x, nrm, nullptr, count, spp, bounces, flags, seed, out_E, out_E32,
                            out_var, out_backfaces, out_valid, stream);
}

niv_status mc_sample_points_t(const mc_scene *s, const double *lo, const double *hi, int64_t count,
                              int64_t n_surface, uint64_t seed, float *out_x, float *out_n,
                              float *out_t, hipStream_t stream)
{
    if (!s || !lo || !hi || count < 0 || n_surface < 0 || n_surface > count) return NIV_ERR_INVALID_ARG;
    if (count == 0) return NIV_OK;
    if (!out_x || !out_n) return NIV_ERR_INVALID_ARG;
    if (n_surface > 0 && s->n_faces == 0) return NIV_ERR_INVALID_ARG;
    for (int c = 0; c < 3; ++c)
        if (!(hi[c] >= lo[c])) return NIV_ERR_INVALID_ARG;
    SampleArgs a;
    memset(&a, 0, sizeof(a));
    a.prims = s->d_prims;
    a.face_prim = s->d_face_prim;
    a.face_id = s->d_face_id;
    a.cdf = s->d_cdf;
    a.n_faces = s->n_faces;
    a.total_area = s->total_area;
    for (int c = 0; c < 3; ++c) { a.lo[c] = lo[c]; a.hi[c] = hi[c]; }
    a.count = count;
    a.n_surface = n_surface;
    a.seed = seed;
    a.out_x = out_x;
    a.out_n = out_n;
    a.out_t = out_t;
    int64_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(k_sample_points, dim3((unsigned)blocks), dim3(256), 0, stream, a);
    return hs(hipGetLastError());
}

niv_status mc_sample_points(const mc_scene *s, const double *lo, const double *hi, int64_t count,
                            int64_t n_surface, uint64_t seed, float *out_x, float *out_n,
                            hipStream_t stream)
{
    return mc_sample_points_t(s, lo, hi, count, n_surface, seed, out_x, out_n, nullptr, stream);
}

}  // extern "C"
