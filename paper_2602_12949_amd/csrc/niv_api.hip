// C interface of libniv: argument checking, model tables, launches.
#include <math.h>
#include <string.h>

#include <mutex>
#include <new>

#include "niv_internal.h"

using namespace niv;

namespace {

bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// Level table (Sec. 4.1): resolution floor(N_min * b^l) (with a 2^-40
// relative guard so an exact integer product is not floored down), dense
// (N+1)^3 storage when it fits in T entries, else T hashed entries.
void build_levels(Model &m)
{
    const niv_config &c = m.cfg;
    const int64_t T = int64_t(1) << c.log2_T;
    int64_t total = 0;
    for (int l = 0; l < c.n_levels; ++l) {
        double x = c.base_res * pow(c.per_level_scale, (double)l);
        int64_t N = (int64_t)floor(x * (1.0 + 0x1p-40));
        int64_t side = N + 1;
        bool dense = side * side * side <= T;
        m.res[l] = N;
        m.dense[l] = dense ? 1 : 0;
        m.size[l] = dense ? side * side * side : T;
        m.offset[l] = total;
        total += m.size[l];
        LevelConst &lv = m.lv[l];
        for (int a = 0; a < 3; ++a) {
            double k = (double)N / (c.aabb_max[a] - c.aabb_min[a]);
            lv.k[a] = k;
            lv.o[a] = -(c.aabb_min[a] * k);
            lv.kf[a] = (float)lv.k[a];
            lv.of[a] = (float)lv.o[a];
        }
        lv.nm1 = (int32_t)(N - 1);
        lv.dense = dense ? 1 : 0;
        lv.off = (uint32_t)m.offset[l];
        lv.s1 = (uint32_t)side;
        lv.s2 = (uint32_t)(side * side);
        lv.pad = 0;
    }
    m.n_entries = total;
    m.n_grid_values = total * c.n_features;
    m.din = c.n_levels * c.n_features + (c.pos_bands > 0 ? 3 + 6 * c.pos_bands : 0) +
            c.sh_bands * c.sh_bands + c.n_extra * 2 * c.extra_bands;
    m.n_params = m.n_grid_values + (int64_t)c.width * m.din +
                 (int64_t)(c.n_hidden - 1) * c.width * c.width + (int64_t)c.n_out * c.width;
}

niv_status check_config(const niv_config *c)
{
    if (c->n_levels < 0 || c->n_levels > kMaxLevels || c->pos_bands < 0 || c->pos_bands > 16 ||
        (c->n_levels == 0 && c->pos_bands == 0) || c->log2_T < 1 || c->log2_T > 24 ||
        c->n_features < 1 || c->n_features > 8 || !(c->base_res >= 1.0) ||
        !(c->per_level_scale >= 1.0) || c->sh_bands < 0 || c->sh_bands > 8 || c->n_extra < 0 ||
        c->n_extra > 4 || c->extra_bands < 0 || c->extra_bands > 16 || c->width < 1 ||
        c->n_hidden < 1 || c->n_out < 1 || c->n_out > 4)
        return NIV_ERR_INVALID_ARG;
    for (int a = 0; a < 3; ++a)
        if (!(c->aabb_max[a] > c->aabb_min[a]) || !isfinite(c->aabb_min[a]) ||
            !isfinite(c->aabb_max[a]))
            return NIV_ERR_INVALID_ARG;
    if (c->n_levels > 0) {
        double top = c->base_res * pow(c->per_level_scale, (double)(c->n_levels - 1));
        if (!(top < 2147483647.0 / 2)) return NIV_ERR_INVALID_ARG;
    }
    return NIV_OK;
}

// Which fused-kernel shape serves this configuration, or -1.
int kernel_kind(const Model &m)
{
    const niv_config &c = m.cfg;
    if ((c.n_features != 2 && c.n_features != 4) || c.sh_bands != 4 || c.n_out != 3) return -1;
    if (c.n_extra > 0 && c.extra_bands != 8) return -1;
    // hashed levels rely on corner coordinates below T
    for (int l = 0; l < c.n_levels; ++l)
        if (!m.dense[l] && m.res[l] + 1 > (int64_t(1) << c.log2_T)) return -1;
    if (m.n_entries > (int64_t)0xFFFFFFFF / 2) return -1;
    if (c.n_features == 4) {  // grid networks of Table 1
        if (c.pos_bands != 0 || c.n_extra != 0 || c.width != 64 || c.n_hidden != 3) return -1;
        switch (c.n_levels) {
        case 2: return kT1L2;
        case 4: return kT1L4;
        case 6: return kT1L6;
        case 8: return kT1L8;
        default: return -1;
        }
    }
    if (c.n_levels == 0) {  // grid-free models of Table 1
        if (c.pos_bands != 8 || c.n_extra != 0 || c.n_hidden != 3) return -1;
        return c.width == 16 ? kPE16 : c.width == 32 ? kPE32 : c.width == 64 ? kPE64 : -1;
    }
    if (c.pos_bands != 0) return -1;
    if (c.n_levels == 8 && c.n_extra == 0 && c.width == 64 && c.n_hidden == 2) return kUnitCube;
    if (c.n_levels == 16 && c.n_extra == 0 && c.width == 64 && c.n_hidden == 3) return kRoom;
    if (c.n_levels == 16 && c.n_extra == 1 && c.width == 128 && c.n_hidden == 4) return kWide6D;
    if (c.n_levels == 16 && c.n_extra == 1 && c.width == 64 && c.n_hidden == 3) return kRoom6D;
    return -1;
}

niv_status hip_status(hipError_t e) { return e == hipSuccess ? NIV_OK : NIV_ERR_HIP; }

}  // namespace

extern "C" {

niv_status niv_create(const niv_config *cfg, niv_handle **out)
{
    if (!cfg || !out) return NIV_ERR_INVALID_ARG;
    *out = nullptr;
    niv_status s = check_config(cfg);
    if (s != NIV_OK) return s;
    niv_handle *h = new (std::nothrow) niv_handle;
    if (!h) return NIV_ERR_INVALID_ARG;
    memset(h, 0, sizeof(*h));
    h->m.cfg = *cfg;
    build_levels(h->m);
    h->m.kind = kernel_kind(h->m);
    *out = h;
    return NIV_OK;
}

void niv_destroy(niv_handle *h) { delete h; }

niv_status niv_sizes(const niv_handle *h, niv_precision prec, int64_t *n_params,
                     int64_t *n_grid_values, int64_t *prepared_bytes)
{
    if (!h) return NIV_ERR_INVALID_ARG;
    if (prec != NIV_FP32 && prec != NIV_FP16 && prec != NIV_BF16) return NIV_ERR_INVALID_ARG;
    if (n_params) *n_params = h->m.n_params;
    if (n_grid_values) *n_grid_values = h->m.n_grid_values;
    if (prepared_bytes) {
        if (h->m.kind < 0) return NIV_ERR_UNSUPPORTED;
        OpLayout L = op_layout(h->m.kind, prec);
        int64_t es = prec == NIV_FP32 ? 4 : 2;
        *prepared_bytes = L.grid_off + h->m.n_grid_values * es;
    }
    return NIV_OK;
}

niv_status niv_level_info(const niv_handle *h, int64_t *res, int32_t *dense, int64_t *offset,
                          int64_t *size)
{
    if (!h) return NIV_ERR_INVALID_ARG;
    for (int l = 0; l < h->m.cfg.n_levels; ++l) {
        if (res) res[l] = h->m.res[l];
        if (dense) dense[l] = h->m.dense[l];
        if (offset) offset[l] = h->m.offset[l];
        if (size) size[l] = h->m.size[l];
    }
    return NIV_OK;
}

niv_status niv_prepare(niv_handle *h, const float *params, void *prepared, niv_precision prec,
                       hipStream_t stream)
{
    if (!h || !params || !prepared) return NIV_ERR_INVALID_ARG;
    if (prec != NIV_FP32 && prec != NIV_FP16 && prec != NIV_BF16) return NIV_ERR_INVALID_ARG;
    if (!aligned(params, 4) || !aligned(prepared, 256)) return NIV_ERR_INVALID_ARG;
    if (h->m.kind < 0) return NIV_ERR_UNSUPPORTED;
    return hip_status(launch_prepare(h->m, params, prepared, prec, stream));
}

static niv_status check_frames(const niv_handle *h, const niv_frame *frames, int32_t n_frames,
                               niv_precision prec)
{
    if (!h || n_frames < 0 || (n_frames > 0 && !frames)) return NIV_ERR_INVALID_ARG;
    if (prec != NIV_FP32 && prec != NIV_FP16 && prec != NIV_BF16) return NIV_ERR_INVALID_ARG;
    if (h->m.kind < 0) return NIV_ERR_UNSUPPORTED;
    for (int f = 0; f < n_frames; ++f) {
        const niv_frame &fr = frames[f];
        if (fr.count < 0 || fr.count >= (int64_t(1) << 28)) return NIV_ERR_INVALID_ARG;
        if (fr.count == 0) continue;
        if (!fr.pos || !fr.nrm || !fr.out_E || !fr.model) return NIV_ERR_INVALID_ARG;
        if (fr.out_L && !fr.albedo) return NIV_ERR_INVALID_ARG;
        if (!aligned(fr.pos, 4) || !aligned(fr.nrm, 4) || !aligned(fr.out_E, 4) ||
            (fr.albedo && !aligned(fr.albedo, 4)) || (fr.out_L && !aligned(fr.out_L, 4)) ||
            (fr.out_inputs && !aligned(fr.out_inputs, 4)) || !aligned(fr.model, 256))
            return NIV_ERR_INVALID_ARG;
        for (int e = 0; e < h->m.cfg.n_extra; ++e)
            if (!isfinite(fr.extra_values[e])) return NIV_ERR_INVALID_ARG;
    }
    return NIV_OK;
}

// One launch for up to kMaxFrames frames.
static void fill_args(const niv_handle *h, const niv_frame *frames, int n, niv_precision prec,
                      QueryArgs &a)
{
    memset(&a, 0, sizeof(a));
    OpLayout L = op_layout(h->m.kind, prec);
    a.n_frames = n;
    a.grid_off = (uint64_t)L.grid_off;
    a.grid_bytes = (uint32_t)(h->m.n_grid_values * (prec == NIV_FP32 ? 4 : 2));
    a.hash_mask = (uint32_t)((int64_t(1) << h->m.cfg.log2_T) - 1);
    for (int c = 0; c < 3; ++c) {
        a.lo[c] = h->m.cfg.aabb_min[c];
        a.hi[c] = h->m.cfg.aabb_max[c];
        a.pe_k[c] = 1.0 / (a.hi[c] - a.lo[c]);
        a.pe_o[c] = -(a.lo[c] * a.pe_k[c]);
    }
    for (int f = 0; f < n; ++f) {
        const niv_frame &fr = frames[f];
        FrameArgs &d = a.f[f];
        d.pos = fr.pos;
        d.nrm = fr.nrm;
        d.albedo = fr.albedo;
        d.mask = fr.mask;
        d.in_flags = fr.in_flags;
        d.out_E = fr.out_E;
        d.out_L = fr.out_L;
        d.out_flags = fr.out_flags;
        d.out_inputs = fr.out_inputs;
        d.model = static_cast<const uint8_t *>(fr.model);
        d.count = fr.count;
        for (int e = 0; e < 4; ++e) d.extra[e] = fr.extra_values[e];
    }
}

static LaunchTune tune_of(const niv_handle *h, niv_precision prec)
{
    return h->m.tuned[prec] ? h->m.tune[prec] : default_tune(h->m.kind, prec);
}

niv_status niv_query(niv_handle *h, const niv_frame *frames, int32_t n_frames, niv_precision prec,
                     hipStream_t stream)
{
    niv_status s = check_frames(h, frames, n_frames, prec);
    if (s != NIV_OK) return s;
    const LaunchTune tu = tune_of(h, prec);
    for (int f0 = 0; f0 < n_frames; f0 += kMaxFrames) {
        const int n = n_frames - f0 < kMaxFrames ? n_frames - f0 : kMaxFrames;
        QueryArgs a;
        fill_args(h, frames + f0, n, prec, a);
        a.xcd_order = tu.xcd_order;
        if (launch_query(h->m, a, prec, tu, stream) != hipSuccess) return NIV_ERR_HIP;
    }
    return NIV_OK;
}

niv_status niv_probe_encode(niv_handle *h, const niv_frame *frame, niv_precision prec,
                            hipStream_t stream)
{
    niv_status s = check_frames(h, frame, 1, prec);
    if (s != NIV_OK) return s;
    if (h->m.kind != kRoom) return NIV_ERR_UNSUPPORTED;
    const LaunchTune tu = tune_of(h, prec);
    QueryArgs a;
    fill_args(h, frame, 1, prec, a);
    a.xcd_order = tu.xcd_order;
    return hip_status(launch_query_probe(h->m, a, prec, tu, stream));
}

// ---------------------------------------------------------------- half resolution
static niv_status check_half(const niv_handle *h, const niv_half_frame *f,
                             const niv_upsample_params *p)
{
    if (!h || !f || !p) return NIV_ERR_INVALID_ARG;
    if (f->width < 1 || f->height < 1 || (int64_t)f->width * f->height >= (int64_t(1) << 28))
        return NIV_ERR_INVALID_ARG;
    if (!f->pos || !f->nrm || !f->half_E || !f->out_E) return NIV_ERR_INVALID_ARG;
    if (f->out_L && !f->albedo) return NIV_ERR_INVALID_ARG;
    if (!aligned(f->pos, 4) || !aligned(f->nrm, 4) || !aligned(f->half_E, 4) ||
        !aligned(f->out_E, 4) || (f->albedo && !aligned(f->albedo, 4)) ||
        (f->out_L && !aligned(f->out_L, 4)))
        return NIV_ERR_INVALID_ARG;
    if (!(p->sigma_px > 0.0f) || !(p->sigma_pos > 0.0f) || !isfinite(p->sigma_px) ||
        !isfinite(p->sigma_pos) || p->normal_power < 0 || p->normal_power > 64)
        return NIV_ERR_INVALID_ARG;
    return NIV_OK;
}

static hipError_t upsample_launch(const niv_handle *h, const niv_half_frame *f,
                                  const niv_upsample_params *p, hipStream_t stream)
{
    UpsampleArgs u;
    memset(&u, 0, sizeof(u));
    u.pos = f->pos;
    u.nrm = f->nrm;
    u.albedo = f->albedo;
    u.mask = f->mask;
    u.half_E = f->half_E;
    u.out_E = f->out_E;
    u.out_L = f->out_L;
    u.out_flags = f->out_flags;
    u.width = f->width;
    u.height = f->height;
    u.half_w = (f->width + 1) / 2;
    u.half_h = (f->height + 1) / 2;
    for (int c = 0; c < 3; ++c) {
        u.lo[c] = (float)h->m.cfg.aabb_min[c];
        u.hi[c] = (float)h->m.cfg.aabb_max[c];
    }
    // log2 of the Gaussian weights: -d^2 / (2 sigma^2 ln 2)
    const double ln2 = 0.69314718055994531;
    u.c_px = (float)(1.0 / (2.0 * (double)p->sigma_px * p->sigma_px * ln2));
    u.c_pos = (float)(1.0 / (2.0 * (double)p->sigma_pos * p->sigma_pos * ln2));
    u.normal_power = (float)p->normal_power;
    return launch_upsample(u, stream);
}

niv_status niv_upsample(niv_handle *h, const niv_half_frame *f, const niv_upsample_params *p,
                        hipStream_t stream)
{
    niv_status s = check_half(h, f, p);
    if (s != NIV_OK) return s;
    return hip_status(upsample_launch(h, f, p, stream));
}

niv_status niv_query_half(niv_handle *h, const niv_half_frame *f, const niv_upsample_params *p,
                          niv_precision prec, hipStream_t stream)
{
    niv_status s = check_half(h, f, p);
    if (s != NIV_OK) return s;
    // the query at the half-resolution samples, as a frame of ceil(W/2) x
    // ceil(H/2) pixels that reads every other pixel of every other row
    niv_frame q;
    memset(&q, 0, sizeof(q));
    q.count = (int64_t)((f->width + 1) / 2) * ((f->height + 1) / 2);
    q.pos = f->pos;
    q.nrm = f->nrm;
    q.mask = f->mask;
    for (int e = 0; e < 4; ++e) q.extra_values[e] = f->extra_values[e];
    q.model = f->model;
    q.out_E = f->half_E;
    q.out_flags = f->half_flags;
    s = check_frames(h, &q, 1, prec);
    if (s != NIV_OK) return s;
    QueryArgs a;
    fill_args(h, &q, 1, prec, a);
    a.f[0].sub_w = (f->width + 1) / 2;
    a.f[0].src_w = f->width;
    const LaunchTune tu = tune_of(h, prec);
    a.xcd_order = tu.xcd_order;
    if (launch_query(h->m, a, prec, tu, stream) != hipSuccess) return NIV_ERR_HIP;
    return hip_status(upsample_launch(h, f, p, stream));
}

niv_status niv_corner_indices(niv_handle *h, niv_precision prec, int32_t training, const void *model,
                              const float *pos, int64_t count, uint32_t *out, hipStream_t stream)
{
    if (!h || (prec != NIV_FP32 && prec != NIV_FP16 && prec != NIV_BF16)) return NIV_ERR_INVALID_ARG;
    if (h->m.kind < 0) return NIV_ERR_UNSUPPORTED;
    if (h->m.cfg.n_levels == 0) return NIV_ERR_UNSUPPORTED;
    if (count < 0 || count >= (int64_t(1) << 28)) return NIV_ERR_INVALID_ARG;
    if (count == 0) return NIV_OK;
    if (!model || !pos || !out || !aligned(model, 256) || !aligned(pos, 4) || !aligned(out, 4))
        return NIV_ERR_INVALID_ARG;
    return hip_status(launch_trace_corners(h->m, prec, training != 0, model, pos, count, out, stream));
}

niv_status niv_fallback_sizes(const niv_handle *h, int64_t max_flagged, int64_t *workspace_bytes)
{
    if (!h || !workspace_bytes || max_flagged < 0 || max_flagged > 0x7fffffff) return NIV_ERR_INVALID_ARG;
    *workspace_bytes = 256 + 4 * max_flagged;
    return NIV_OK;
}

// niv_query_fallback with its scratch given as the counter and the list of
// `cap` entries.
static niv_status query_fallback_into(niv_handle *h, const niv_frame *frames, int32_t n_frames,
                                      niv_precision prec, const niv_fallback *fb, uint32_t *cnt,
                                      uint32_t *list, uint32_t cap, hipStream_t stream)
{
    // the counter is cleared by a kernel so that the whole call can be captured in a graph
    if (launch_zero_u32(cnt, 1, stream) != hipSuccess) return NIV_ERR_HIP;
    QueryArgs a;
    fill_args(h, frames, n_frames, prec, a);
    a.fb_list = list;
    a.fb_count = cnt;
    a.fb_cap = cap;
    a.fb_mask = fb->flag_mask;
    const LaunchTune tu = tune_of(h, prec);
    a.xcd_order = tu.xcd_order;
    if (launch_query(h->m, a, prec, tu, stream) != hipSuccess) return NIV_ERR_HIP;
    FbArgs b;
    memset(&b, 0, sizeof(b));
    b.list = list;
    b.count = cnt;
    b.cap = cap;
    b.spp = fb->spp;
    b.bounces = fb->bounces;
    b.flags = fb->mc_flags;
    b.seed = fb->seed;
    for (int f = 0; f < n_frames; ++f) {
        const niv_frame &fr = frames[f];
        FbFrame &d = b.f[f];
        d.pos = fr.pos;
        d.nrm = fr.nrm;
        d.albedo = fr.albedo;
        d.out_E = fr.out_E;
        d.out_L = fr.out_L;
        d.out_flags = fr.out_flags;
        mc_scene_device_view(fr.scene, &d.prims, &d.lights, &d.n_prims, &d.n_lights, &d.eps, &d.motion);
        mc_scene_trace_view(fr.scene, &d.recs, d.nk);
        d.t = fr.extra_values[0];
    }
    return launch_mc_fallback(b, stream) == hipSuccess ? NIV_OK : NIV_ERR_HIP;
}

static niv_status check_fallback(const niv_handle *h, const niv_frame *frames, int32_t n_frames,
                                 niv_precision prec, const niv_fallback *fb)
{
    niv_status s = check_frames(h, frames, n_frames, prec);
    if (s != NIV_OK) return s;
    if (n_frames > kMaxFrames || !fb) return NIV_ERR_INVALID_ARG;
    if (fb->spp < 1 || fb->bounces < 0 || fb->bounces > 16 || (fb->mc_flags & ~15) ||
        ((fb->mc_flags & 1) && (fb->mc_flags & 2)) || (fb->flag_mask & ~21u))
        return NIV_ERR_INVALID_ARG;
    return NIV_OK;
}

niv_status niv_query_fallback(niv_handle *h, const niv_frame *frames, int32_t n_frames,
                              niv_precision prec, const niv_fallback *fb, void *workspace,
                              int64_t workspace_bytes, hipStream_t stream)
{
    niv_status s = check_fallback(h, frames, n_frames, prec, fb);
    if (s != NIV_OK) return s;
    if (!workspace || !aligned(workspace, 256)) return NIV_ERR_INVALID_ARG;
    if (workspace_bytes < 256 + 4) return NIV_ERR_WORKSPACE;
    uint32_t *cnt = static_cast<uint32_t *>(workspace);
    uint32_t *list = reinterpret_cast<uint32_t *>(static_cast<uint8_t *>(workspace) + 256);
    const int64_t cap64 = (workspace_bytes - 256) / 4;
    const uint32_t cap = (uint32_t)(cap64 < 0x7fffffff ? cap64 : 0x7fffffff);
    return query_fallback_into(h, frames, n_frames, prec, fb, cnt, list, cap, stream);
}

}  // extern "C"

// Fallback scratch that needs no allocation: the counter (first 256 bytes)
// and a list of up to NIV_NOALLOC_MAX_FLAGGED entries, resident on every
// device the library runs on until the process ends.  Host code never uses
// this name as an address: the device address comes from
// hipGetSymbolAddress, once per device, and is kept in g_scratch_ptr.
static __device__ __align__(256) uint8_t scratch[256 + 4 * (size_t)NIV_NOALLOC_MAX_FLAGGED];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on the current device.
niv_status scratch_address(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return NIV_ERR_HIP;
    if (dev < 0 || dev >= kMaxDevices) return NIV_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return NIV_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return NIV_OK;
}
}  // namespace

extern "C" {

niv_status niv_query_fallback_noalloc(niv_handle *h, const niv_frame *frames, int32_t n_frames,
                                      niv_precision prec, const niv_fallback *fb,
                                      int64_t max_flagged, hipStream_t stream)
{
    niv_status s = check_fallback(h, frames, n_frames, prec, fb);
    if (s != NIV_OK) return s;
    if (max_flagged < 1) return NIV_ERR_INVALID_ARG;
    if (max_flagged > NIV_NOALLOC_MAX_FLAGGED) return NIV_ERR_WORKSPACE;
    void *base = nullptr;
    s = scratch_address(&base);
    if (s != NIV_OK) return s;
    uint32_t *cnt = static_cast<uint32_t *>(base);
    uint32_t *list = reinterpret_cast<uint32_t *>(static_cast<uint8_t *>(base) + 256);
    return query_fallback_into(h, frames, n_frames, prec, fb, cnt, list, (uint32_t)max_flagged,
                               stream);
}

niv_status niv_autotune(niv_handle *h, const niv_frame *frames, int32_t n_frames,
                        niv_precision prec, hipStream_t stream, niv_tune_result *out)
{
    niv_status s = check_frames(h, frames, n_frames, prec);
    if (s != NIV_OK) return s;
    if (n_frames < 1 || n_frames > kMaxFrames) return NIV_ERR_INVALID_ARG;
    static const int blocks[3] = {256, 512, 768};   // 768: lane-sliced shapes only
    const bool sliced = h->m.kind == kWide6D && prec != NIV_FP32;
    static const int per_cu[3] = {0, 1, 2};
    static const int orders[2] = {0, 1};
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return NIV_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return NIV_ERR_HIP; }
    LaunchTune best = default_tune(h->m.kind, prec);
    float best_ms = 1e30f;
    int k = 0;
    niv_status st = NIV_OK;
    for (int b = 0; b < (sliced ? 3 : 2) && st == NIV_OK; ++b)
        for (int c = 0; c < 3 && st == NIV_OK; ++c)
        for (int o = 0; o < 2 && st == NIV_OK; ++o, ++k) {
            LaunchTune tu = {blocks[b], per_cu[c], orders[o]};
            QueryArgs a;
            fill_args(h, frames, n_frames, prec, a);
            a.xcd_order = tu.xcd_order;
            float ms = 1e30f;
            for (int rep = 0; rep < 12 && st == NIV_OK; ++rep) {
                if (hipEventRecord(e0, stream) != hipSuccess ||
                    launch_query(h->m, a, prec, tu, stream) != hipSuccess ||
                    hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                    st = NIV_ERR_HIP;
                    break;
                }
                float t = 0.f;
                if (hipEventElapsedTime(&t, e0, e1) != hipSuccess) { st = NIV_ERR_HIP; break; }
                if (rep >= 2 && t < ms) ms = t;  // best of 10 after 2 warm-up launches
            }
            if (out && k < 24) {
                out->block[k] = tu.block;
                out->blocks_per_cu[k] = tu.blocks_per_cu;
                out->xcd_order[k] = tu.xcd_order;
                out->ms[k] = ms;
            }
            if (ms < best_ms) { best_ms = ms; best = tu; }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != NIV_OK) return st;
    h->m.tune[prec] = best;
    h->m.tuned[prec] = true;
    if (out) {
        out->n = k;
        out->chosen_block = best.block;
        out->chosen_blocks_per_cu = best.blocks_per_cu;
        out->chosen_xcd_order = best.xcd_order;
        out->chosen_ms = best_ms;
    }
    return NIV_OK;
}

niv_status niv_set_tune(niv_handle *h, niv_precision prec, int32_t block, int32_t blocks_per_cu,
                        int32_t xcd_order)
{
    if (!h || (prec != NIV_FP32 && prec != NIV_FP16 && prec != NIV_BF16)) return NIV_ERR_INVALID_ARG;
    if ((block != 256 && block != 512 && block != 768) || blocks_per_cu < 0 || blocks_per_cu > 64 ||
        (xcd_order != 0 && xcd_order != 1))
        return NIV_ERR_INVALID_ARG;
    h->m.tune[prec] = LaunchTune{block, blocks_per_cu, xcd_order};
    h->m.tuned[prec] = true;
    return NIV_OK;
}

}  // extern "C"

struct niv_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

niv_status niv_graph_capture(niv_handle *h, const niv_frame *frames, int32_t n_frames,
                             niv_precision prec, const niv_fallback *fb, void *workspace,
                             int64_t workspace_bytes, niv_graph **out)
{
    if (!out) return NIV_ERR_INVALID_ARG;
    *out = nullptr;
    niv_status s = check_frames(h, frames, n_frames, prec);
    if (s != NIV_OK) return s;
    hipStream_t cs;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return NIV_ERR_HIP;
    auto run = [&]() {
        return fb ? niv_query_fallback(h, frames, n_frames, prec, fb, workspace, workspace_bytes, cs)
                  : niv_query(h, frames, n_frames, prec, cs);
    };
    // eager run: initialises every launch parameter outside the capture
    s = run();
    if (s == NIV_OK && hipStreamSynchronize(cs) != hipSuccess) s = NIV_ERR_HIP;
    niv_graph *g = nullptr;
    if (s == NIV_OK) {
        g = new (std::nothrow) niv_graph;
        if (!g) s = NIV_ERR_INVALID_ARG;
    }
    if (s == NIV_OK && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess)
        s = NIV_ERR_HIP;
    if (s == NIV_OK) {
        niv_status rs = run();
        hipError_t e = hipStreamEndCapture(cs, &g->graph);
        if (rs != NIV_OK) s = rs;
        else if (e != hipSuccess) s = NIV_ERR_HIP;
    }
    if (s == NIV_OK && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
        s = NIV_ERR_HIP;
    (void)hipStreamDestroy(cs);
    if (s != NIV_OK) {
        niv_graph_destroy(g);
        return s;
    }
    *out = g;
    return NIV_OK;
}

niv_status niv_graph_launch(niv_graph *g, hipStream_t stream)
{
    if (!g || !g->exec) return NIV_ERR_INVALID_ARG;
    return hipGraphLaunch(g->exec, stream) == hipSuccess ? NIV_OK : NIV_ERR_HIP;
}

void niv_graph_destroy(niv_graph *g)
{
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

const char *niv_status_string(niv_status s)
{
    switch (s) {
    case NIV_OK: return "ok";
    case NIV_ERR_INVALID_ARG: return "invalid argument";
    case NIV_ERR_UNSUPPORTED: return "model shape not supported by the kernels";
    case NIV_ERR_HIP: return "HIP runtime error";
    case NIV_ERR_WORKSPACE: return "workspace too small";
    case NIV_ERR_STATE: return "call out of order";
    case NIV_ERR_NONFINITE: return "the training step's loss or gradient was not finite (update skipped)";
    }
    return "unknown status";
}

}  // extern "C"
