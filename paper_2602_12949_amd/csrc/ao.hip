// Dynamic ambient occlusion (Sec. 4.4) for gfx950.
//
// The irradiance a model learned from the static scene knows nothing of
// geometry placed at render time, so the shaded irradiance is multiplied by
// the visibility of the hemisphere against that dynamic geometry alone: the
// cosine-weighted share of directions whose ray leaves the point without
// meeting a dynamic triangle within a radius.  One lane per pixel estimates
// it from `rays` cosine-distributed directions drawn from the pixel's own
// random stream, so the estimate is a function of (seed, pixel) that the CPU
// replays exactly.
//
// The triangles sit in a bounding-volume hierarchy built on the host
// (binned surface-area splits near the root, centroid medians below, up to
// four triangles per leaf) and copied to the device once per set of dynamic
// objects.  A node record holds its two children's boxes, so one 64-byte
// load tests both; the nearer child is visited next and the farther one is
// pushed on a per-lane stack in LDS ([depth][lane]: a wave's pushes fall in
// distinct banks).  Rays take any hit (visibility needs no nearest one),
// and a pixel farther than the radius from both of the root's boxes is
// visible without tracing.
#include <hip/hip_runtime.h>
#include <math.h>
#include <algorithm>
#include <new>
#include <vector>

#include "niv_internal.h"

#pragma clang fp contract(off)

#include "mc_device.h"

namespace niv {
namespace {

// An inner node: the boxes of its two children and what they are.  Child
// item >= 0 is an inner node's index; item < 0 is a leaf, -1 - (first << 3 |
// count) with its first triangle and 1..4 triangles.  An absent child (the
// root of a tree that is a single leaf has one) is a leaf with no triangles.
struct BvhNode {          // 64 bytes, four 16-byte loads
    float lo0[3];
    int32_t item0;
    float hi0[3];
    int32_t pad0;
    float lo1[3];
    int32_t item1;
    float hi1[3];
    int32_t pad1;
};
static_assert(sizeof(BvhNode) == 64, "node record is 64 bytes");

struct Tri {              // vertex 0 and the two edges from it
    float v0[3], e1[3], e2[3];
};

constexpr int kLeaf = 4;
// Stack entries per lane: a ray pushes at most one node per level it
// descends, so the build keeps the depth within kStack.  20 entries (20 KB
// of LDS per 256-lane workgroup) let 8 workgroups share a CU, 8 waves per
// SIMD, which the latency-bound walk needs (32 entries, 5 waves: 8.0 ms
// instead of 7.0 on the 3840x2160 frame).
constexpr int kStack = 20;
constexpr int kAoBlock = 256;
constexpr int64_t kMaxTris = int64_t(kLeaf) << kStack;   // 2^22: the median levels alone fit the stack

struct AoArgs {
    const BvhNode *nodes;
    const Tri *tris;
    const float *pos, *nrm;
    const uint8_t *mask;
    float *E, *L, *vis;
    int64_t count;
    float lo0[3], hi0[3], lo1[3], hi1[3];   // the root's two boxes (empty without triangles)
    float radius, eps;
    int32_t rays;
    uint64_t seed;
};

// Moller-Trumbore: o + t d = v0 + u e1 + v e2 solved by Cramer's rule; both
// sides of the triangle count.
__device__ inline bool tri_hit(const Tri &T, const float o[3], const float d[3], float tmax)
{
    const float p0 = d[1] * T.e2[2] - d[2] * T.e2[1];
    const float p1 = d[2] * T.e2[0] - d[0] * T.e2[2];
    const float p2 = d[0] * T.e2[1] - d[1] * T.e2[0];
    const float det = T.e1[0] * p0 + T.e1[1] * p1 + T.e1[2] * p2;
    if (det == 0.0f) return false;
    const float s0 = o[0] - T.v0[0], s1 = o[1] - T.v0[1], s2 = o[2] - T.v0[2];
    const float u = (s0 * p0 + s1 * p1 + s2 * p2) / det;
    if (!(u >= 0.0f && u <= 1.0f)) return false;
    const float q0 = s1 * T.e1[2] - s2 * T.e1[1];
    const float q1 = s2 * T.e1[0] - s0 * T.e1[2];
    const float q2 = s0 * T.e1[1] - s1 * T.e1[0];
    const float v = (d[0] * q0 + d[1] * q1 + d[2] * q2) / det;
    if (!(v >= 0.0f && u + v <= 1.0f)) return false;
    const float t = (T.e2[0] * q0 + T.e2[1] * q1 + T.e2[2] * q2) / det;
    return t > 0.0f && t <= tmax;
}

// Entry distance of the segment t in [0, tmax] into a box (slab test with
// the reciprocal direction), or +inf when it misses.
__device__ inline float box_entry(const float lo[3], const float hi[3], const float inv[3], const float oi[3],
                                  float tmax)
{
    const float x0 = lo[0] * inv[0] - oi[0], x1 = hi[0] * inv[0] - oi[0];
    const float y0 = lo[1] * inv[1] - oi[1], y1 = hi[1] * inv[1] - oi[1];
    const float z0 = lo[2] * inv[2] - oi[2], z1 = hi[2] * inv[2] - oi[2];
    const float tn = fmaxf(fmaxf(fminf(x0, x1), fminf(y0, y1)), fmaxf(fminf(z0, z1), 0.0f));
    const float tf = fminf(fminf(fmaxf(x0, x1), fmaxf(y0, y1)), fminf(fmaxf(z0, z1), tmax));
    return tn <= tf ? tn : INFINITY;
}

__device__ inline float box_dist2(const float lo[3], const float hi[3], const float p[3])
{
    float r2 = 0.0f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float e = fmaxf(fmaxf(lo[c] - p[c], p[c] - hi[c]), 0.0f);
        r2 += e * e;
    }
    return r2;
}

__global__ __launch_bounds__(kAoBlock) void k_dynamic_ao(const AoArgs a)
{
    __shared__ int32_t stacks[kStack * kAoBlock];
    int32_t *stack = stacks + threadIdx.x;   // entry e at stack[e * kAoBlock]
    const int64_t i = (int64_t)blockIdx.x * kAoBlock + threadIdx.x;
    if (i >= a.count) return;   // no barriers below
    const bool use = !a.mask || a.mask[i];
    float p[3], n[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) { p[c] = a.pos[3 * i + c]; n[c] = a.nrm[3 * i + c]; }
    const float ln = sqrtf(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    bool trace = use && ln > 0.0f && __builtin_isfinite(ln);
#pragma unroll
    for (int c = 0; c < 3; ++c) trace = trace && __builtin_isfinite(p[c]);
    // a pixel out of reach of both of the root's boxes is visible without tracing
    const float reach = a.radius + a.eps;
    trace = trace && fminf(box_dist2(a.lo0, a.hi0, p), box_dist2(a.lo1, a.hi1, p)) <= reach * reach;
    float o[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        n[c] /= ln;
        o[c] = p[c] + a.eps * n[c];
    }
    int hits = 0;
    for (int k = 0; trace && k < a.rays; ++k) {
        Rng rng(a.seed, (uint64_t)i, (uint64_t)k, 2);
        float d[3], inv[3], oi[3];
        cosine_dir(n, rng.u(0), rng.u(1), d);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            inv[c] = d[c] != 0.0f ? 1.0f / d[c] : 1e30f;   // as in the Monte Carlo tracer
            oi[c] = o[c] * inv[c];
        }
        // depth-first from the root: `cur` is the item being visited
        int sp = 0;
        int32_t cur = 0;
        bool hit = false;
        while (true) {
            if (cur >= 0) {           // inner node: both children's boxes
                const float4 *w = reinterpret_cast<const float4 *>(a.nodes + cur);
                const float4 w0 = w[0], w1 = w[1], w2 = w[2], w3 = w[3];
                const float l0[3] = {w0.x, w0.y, w0.z}, h0[3] = {w1.x, w1.y, w1.z};
                const float l1[3] = {w2.x, w2.y, w2.z}, h1[3] = {w3.x, w3.y, w3.z};
                const float e0 = box_entry(l0, h0, inv, oi, a.radius);
                const float e1 = box_entry(l1, h1, inv, oi, a.radius);
                const int32_t c0 = __builtin_bit_cast(int32_t, w0.w), c1 = __builtin_bit_cast(int32_t, w2.w);
                if (e0 != INFINITY && e1 != INFINITY) {   // nearer child next, the other later
                    const bool first0 = e0 <= e1;
                    if (sp < kStack) {    // always true for trees the host accepted
                        stack[sp * kAoBlock] = first0 ? c1 : c0;
                        ++sp;
                    }
                    cur = first0 ? c0 : c1;
                    continue;
                }
                if (e0 != INFINITY) { cur = c0; continue; }
                if (e1 != INFINITY) { cur = c1; continue; }
            } else {                  // leaf: its triangles
                const int32_t code = -1 - cur;
                const int32_t first = code >> 3, cnt = code & 7;
                for (int32_t t = first; t < first + cnt && !hit; ++t) hit = tri_hit(a.tris[t], o, d, a.radius);
                if (hit) break;
            }
            if (sp == 0) break;
            --sp;
            cur = stack[sp * kAoBlock];
        }
        hits += hit ? 1 : 0;
    }
    const float vis = trace ? 1.0f - (float)hits / (float)a.rays : 1.0f;
    if (a.vis) a.vis[i] = vis;
    if (use && vis != 1.0f) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (a.E) a.E[3 * i + c] *= vis;
            if (a.L) a.L[3 * i + c] *= vis;
        }
    }
}

// ---------------------------------------------------------------- host: build
struct Item {
    float c[3], lo[3], hi[3];
    int32_t id;
};

// Binary tree by median splits; each inner node then becomes one record
// with its children's boxes.
struct Builder {
    struct Node {
        float lo[3], hi[3];
        int32_t left, begin, end;   // left: first of two children, or -1 for a leaf [begin, end)
    };
    std::vector<Item> items;
    std::vector<Node> tree;
    int depth = 0;
    int sah_levels = 0;   // levels split by the surface-area heuristic; median splits below

    // Binned surface-area heuristic (16 bins of the centroid range per
    // axis): the split minimising area(left) n(left) + area(right) n(right);
    // partitions [begin, end) and returns the split point, or -1 when all
    // centroids share a bin.
    int32_t sah_split(int32_t begin, int32_t end, const float clo[3], const float chi[3])
    {
        constexpr int NB = 16;
        float best = INFINITY;
        int best_axis = -1, best_b = -1;
        for (int ax = 0; ax < 3; ++ax) {
            const float ext = chi[ax] - clo[ax];
            if (!(ext > 0.0f)) continue;
            int cnt[NB] = {};
            float blo[NB][3], bhi[NB][3];
            for (int b = 0; b < NB; ++b)
                for (int c = 0; c < 3; ++c) { blo[b][c] = INFINITY; bhi[b][c] = -INFINITY; }
            for (int32_t k = begin; k < end; ++k) {
                int b = (int)((items[k].c[ax] - clo[ax]) / ext * NB);
                b = b < 0 ? 0 : (b >= NB ? NB - 1 : b);
                ++cnt[b];
                for (int c = 0; c < 3; ++c) {
                    blo[b][c] = std::min(blo[b][c], items[k].lo[c]);
                    bhi[b][c] = std::max(bhi[b][c], items[k].hi[c]);
                }
            }
            auto area = [](const float lo[3], const float hi[3]) {
                const float x = hi[0] - lo[0], y = hi[1] - lo[1], z = hi[2] - lo[2];
                return x * y + y * z + z * x;
            };
            float rlo[NB][3], rhi[NB][3];   // bounds of bins b..NB-1
            int rcnt[NB];
            for (int b = NB - 1; b >= 0; --b)
                for (int c = 0; c < 3; ++c) {
                    rlo[b][c] = b + 1 < NB ? std::min(rlo[b + 1][c], blo[b][c]) : blo[b][c];
                    rhi[b][c] = b + 1 < NB ? std::max(rhi[b + 1][c], bhi[b][c]) : bhi[b][c];
                    if (c == 0) rcnt[b] = (b + 1 < NB ? rcnt[b + 1] : 0) + cnt[b];
                }
            float llo[3] = {INFINITY, INFINITY, INFINITY}, lhi[3] = {-INFINITY, -INFINITY, -INFINITY};
            int lcnt = 0;
            for (int b = 0; b + 1 < NB; ++b) {   // split between bins b and b + 1
                lcnt += cnt[b];
                for (int c = 0; c < 3; ++c) { llo[c] = std::min(llo[c], blo[b][c]); lhi[c] = std::max(lhi[c], bhi[b][c]); }
                if (lcnt == 0 || rcnt[b + 1] == 0) continue;
                const float cost = area(llo, lhi) * lcnt + area(rlo[b + 1], rhi[b + 1]) * rcnt[b + 1];
                if (cost < best) { best = cost; best_axis = ax; best_b = b; }
            }
        }
        if (best_axis < 0) return -1;
        const int ax = best_axis;
        const float lo_ax = clo[ax], ext = chi[ax] - clo[ax];
        auto mid = std::partition(items.begin() + begin, items.begin() + end, [&](const Item &x) {
            int b = (int)((x.c[ax] - lo_ax) / ext * NB);
            b = b < 0 ? 0 : (b >= NB ? NB - 1 : b);
            return b <= best_b;
        });
        const int32_t m = (int32_t)(mid - items.begin());
        return (m > begin && m < end) ? m : -1;
    }

    void make(int32_t node, int32_t begin, int32_t end, int level)
    {
        float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        float clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int32_t k = begin; k < end; ++k)
            for (int c = 0; c < 3; ++c) {
                lo[c] = std::min(lo[c], items[k].lo[c]);
                hi[c] = std::max(hi[c], items[k].hi[c]);
                clo[c] = std::min(clo[c], items[k].c[c]);
                chi[c] = std::max(chi[c], items[k].c[c]);
            }
        for (int c = 0; c < 3; ++c) {
            tree[node].lo[c] = lo[c];
            tree[node].hi[c] = hi[c];
        }
        tree[node].begin = begin;
        tree[node].end = end;
        depth = std::max(depth, level);
        if (end - begin <= kLeaf) {
            tree[node].left = -1;
            return;
        }
        int32_t mid = level < sah_levels ? sah_split(begin, end, clo, chi) : -1;
        if (mid < 0) {   // median of the centroids along the longest axis
            int axis = 0;
            for (int c = 1; c < 3; ++c)
                if (chi[c] - clo[c] > chi[axis] - clo[axis]) axis = c;
            mid = begin + (end - begin) / 2;
            std::nth_element(items.begin() + begin, items.begin() + mid, items.begin() + end,
                             [axis](const Item &x, const Item &y) { return x.c[axis] < y.c[axis]; });
        }
        const int32_t left = (int32_t)tree.size();
        tree.push_back(Node{});
        tree.push_back(Node{});
        tree[node].left = left;
        make(left, begin, mid, level + 1);
        make(left + 1, mid, end, level + 1);
    }

    // Records of the inner nodes in tree order; a leaf-only tree gets one
    // record with the leaf and an empty box.
    std::vector<BvhNode> records() const
    {
        std::vector<int32_t> rec(tree.size(), -1);
        int32_t nrec = 0;
        for (size_t k = 0; k < tree.size(); ++k)
            if (tree[k].left >= 0 || k == 0) rec[k] = nrec++;
        std::vector<BvhNode> out((size_t)nrec);
        auto item = [&](int32_t k) {
            return tree[k].left >= 0 ? rec[k] : -1 - ((tree[k].begin << 3) | (tree[k].end - tree[k].begin));
        };
        auto put = [&](BvhNode &r, int side, int32_t k) {
            float *lo = side ? r.lo1 : r.lo0, *hi = side ? r.hi1 : r.hi0;
            for (int c = 0; c < 3; ++c) {
                lo[c] = k >= 0 ? tree[k].lo[c] : INFINITY;
                hi[c] = k >= 0 ? tree[k].hi[c] : -INFINITY;
            }
            (side ? r.item1 : r.item0) = k >= 0 ? item(k) : -1;   // a leaf of no triangles
            (side ? r.pad1 : r.pad0) = 0;
        };
        for (size_t k = 0; k < tree.size(); ++k) {
            if (rec[k] < 0) continue;
            BvhNode &r = out[(size_t)rec[k]];
            if (tree[k].left >= 0) {
                put(r, 0, tree[k].left);
                put(r, 1, tree[k].left + 1);
            } else {   // the root is a leaf
                put(r, 0, (int32_t)k);
                put(r, 1, -1);
            }
        }
        return out;
    }
};

niv_status hs(hipError_t e) { return e == hipSuccess ? NIV_OK : NIV_ERR_HIP; }

}  // namespace
}  // namespace niv

struct niv_ao {
    niv::BvhNode *d_nodes = nullptr;
    niv::Tri *d_tris = nullptr;
    int32_t n_nodes = 0, n_tris = 0, depth = 0;
    niv::BvhNode root;   // host copy of the root record (its two boxes cull pixels)
};

using namespace niv;

extern "C" {

niv_status niv_ao_create(const float *tris, int64_t n_tris, niv_ao **out)
{
    if (!out || n_tris < 0 || n_tris > kMaxTris || (n_tris > 0 && !tris)) return NIV_ERR_INVALID_ARG;
    *out = nullptr;
    for (int64_t k = 0; k < 9 * n_tris; ++k)
        if (!isfinite(tris[k])) return NIV_ERR_INVALID_ARG;
    niv_ao *ao = new (std::nothrow) niv_ao;
    if (!ao) return NIV_ERR_INVALID_ARG;
    for (int c = 0; c < 3; ++c) {   // empty boxes: no pixel is in reach
        ao->root.lo0[c] = ao->root.lo1[c] = INFINITY;
        ao->root.hi0[c] = ao->root.hi1[c] = -INFINITY;
    }
    if (n_tris == 0) {
        *out = ao;
        return NIV_OK;
    }
    Builder b;
    b.items.resize((size_t)n_tris);
    for (int64_t k = 0; k < n_tris; ++k) {
        Item &it = b.items[(size_t)k];
        it.id = (int32_t)k;
        for (int c = 0; c < 3; ++c) {
            const float x = tris[9 * k + c], y = tris[9 * k + 3 + c], z = tris[9 * k + 6 + c];
            it.lo[c] = std::min(x, std::min(y, z));
            it.hi[c] = std::max(x, std::max(y, z));
            it.c[c] = (it.lo[c] + it.hi[c]) * 0.5f;
        }
    }
    // surface-area splits near the root, medians below: with at most
    // ceil(log2(n / 4)) median levels the depth stays within the stack
    int median_levels = 0;
    while (((int64_t)kLeaf << median_levels) < n_tris) ++median_levels;
    b.sah_levels = std::max(0, kStack - median_levels);
    b.tree.reserve((size_t)(2 * n_tris / kLeaf + 4));
    b.tree.push_back(Builder::Node{});
    b.make(0, 0, (int32_t)n_tris, 0);
    if (b.depth > kStack) {   // cannot happen below kMaxTris triangles
        delete ao;
        return NIV_ERR_UNSUPPORTED;
    }
    const std::vector<BvhNode> rec = b.records();
    std::vector<Tri> T((size_t)n_tris);
    for (int64_t k = 0; k < n_tris; ++k) {
        const float *s = tris + 9 * (int64_t)b.items[(size_t)k].id;
        for (int c = 0; c < 3; ++c) {
            T[(size_t)k].v0[c] = s[c];
            T[(size_t)k].e1[c] = s[3 + c] - s[c];
            T[(size_t)k].e2[c] = s[6 + c] - s[c];
        }
    }
    ao->n_nodes = (int32_t)rec.size();
    ao->n_tris = (int32_t)n_tris;
    ao->depth = b.depth;
    ao->root = rec[0];
    niv_status st = hs(hipMalloc(&ao->d_nodes, sizeof(BvhNode) * rec.size()));
    if (st == NIV_OK) st = hs(hipMalloc(&ao->d_tris, sizeof(Tri) * T.size()));
    if (st == NIV_OK)
        st = hs(hipMemcpy(ao->d_nodes, rec.data(), sizeof(BvhNode) * rec.size(), hipMemcpyHostToDevice));
    if (st == NIV_OK) st = hs(hipMemcpy(ao->d_tris, T.data(), sizeof(Tri) * T.size(), hipMemcpyHostToDevice));
    if (st != NIV_OK) {
        niv_ao_destroy(ao);
        return st;
    }
    *out = ao;
    return NIV_OK;
}

void niv_ao_destroy(niv_ao *ao)
{
    if (!ao) return;
    if (ao->d_nodes) (void)hipFree(ao->d_nodes);
    if (ao->d_tris) (void)hipFree(ao->d_tris);
    delete ao;
}

niv_status niv_ao_info(const niv_ao *ao, int32_t *n_nodes, int32_t *depth)
{
    if (!ao) return NIV_ERR_INVALID_ARG;
    if (n_nodes) *n_nodes = ao->n_nodes;
    if (depth) *depth = ao->depth;
    return NIV_OK;
}

niv_status niv_ao_apply(const niv_ao *ao, const niv_ao_params *p, int64_t count, const float *pos,
                        const float *nrm, const uint8_t *mask, float *E, float *L, float *vis,
                        hipStream_t stream)
{
    if (!ao || !p || count < 0) return NIV_ERR_INVALID_ARG;
    if (p->rays < 1 || p->rays > 4096 || !(p->radius > 0.0f) || !isfinite(p->radius) || !(p->eps >= 0.0f) ||
        !isfinite(p->eps))
        return NIV_ERR_INVALID_ARG;
    if (count == 0) return NIV_OK;
    auto al4 = [](const void *q) { return ((uintptr_t)q & 3u) == 0; };
    if (!pos || !nrm || !al4(pos) || !al4(nrm) || !al4(E) || !al4(L) || !al4(vis)) return NIV_ERR_INVALID_ARG;
    AoArgs a;
    a.nodes = ao->d_nodes;
    a.tris = ao->d_tris;
    a.pos = pos;
    a.nrm = nrm;
    a.mask = mask;
    a.E = E;
    a.L = L;
    a.vis = vis;
    a.count = count;
    for (int c = 0; c < 3; ++c) {
        a.lo0[c] = ao->root.lo0[c];
        a.hi0[c] = ao->root.hi0[c];
        a.lo1[c] = ao->root.lo1[c];
        a.hi1[c] = ao->root.hi1[c];
    }
    a.radius = p->radius;
    a.eps = p->eps;
    a.rays = p->rays;
    a.seed = p->seed;
    const int64_t blocks = (count + kAoBlock - 1) / kAoBlock;
    hipLaunchKernelGGL(k_dynamic_ao, dim3((unsigned)blocks), dim3(kAoBlock), 0, stream, a);
    return hs(hipGetLastError());
}

}  // extern "C"
