// Fused per-pixel Neural Irradiance Volume query for gfx950 (CDNA4).
//
// One launch evaluates E_theta(x, n) for every pixel of a G-buffer (Sec. 4.4)
// and shades it with albedo * E / pi (Eq. 2):
//   1. each lane loads one pixel (coalesced) and builds its input vector:
//      per level the cell, the 8 corner indices (dense or spatially hashed),
//      8 gathers and a trilinear blend in FP32 (Sec. 4.1); 16 real SH of the
//      normal; the frequency code of the frame's scene variables (Sec. 6);
//   2. the wave's 64 input vectors go through a per-wave LDS block into the
//      operand layout of the matrix cores;
//   3. the MLP runs on MFMA with FP32 accumulation, four 16-pixel tiles per
//      wave, weights resident in LDS;
//   4. the RGB of tile t sits in lanes 0..15 after the output layer; one
//      shuffle per channel hands every lane its own pixel's value, and each
//      lane writes its pixel's E, albedo * E / pi and flags.
//
// Operand layout.  A layer y = W x is computed transposed, D = W * X^T, with
// the weights as the A operand (16 output rows) and 16 pixels as the B
// operand columns.  A 16x16 accumulator leaves lane (g = lane/16, j =
// lane%16) holding rows 4g..4g+3 of pixel j.  The contraction index of the
// next layer can be permuted freely as long as A and B agree, so the prepared
// weights are stored with their input columns permuted such that a lane's own
// accumulator values, after ReLU and rounding, ARE its next B operand: no
// cross-lane traffic between layers.
#pragma once
#include <hip/hip_runtime.h>

#include "niv_internal.h"
#include "niv_device.h"

namespace niv {

// LDS accesses of one wave complete in order; the fences keep the compiler
// from moving LDS reads and writes of the wave across this point.
__device__ inline void wave_lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------- fused query
// Waves per SIMD the register allocation must allow: 4 for the FP16 query
// of the staged grid shapes (at most 128 VGPRs; the LDS of a 512-thread workgroup
// allows two workgroups per CU, i.e. four waves per SIMD), else no bound.
template <int P, class S, bool TRAIN> constexpr int query_min_waves()
{
    return (P == NIV_FP16 && !TRAIN && !S::SL && S::PB == 0) ? 4 : 1;
}

// PROBE (measurement only): the encoding stage alone, with the launch shape,
// pixel order and encoding functions of the query, writing one word per
// pixel (E[3q]) instead of running the network.
template <int P, class S, bool WLDS, int TB, bool TRAIN, int BLOCK, bool PROBE = false>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(query_min_waves<P, S, TRAIN>())))
void k_query(const QueryArgs a)
{
    static_assert(!PROBE || (!TRAIN && !S::SL), "probe: staged query encoding");
    constexpr int kWavesPerBlock = BLOCK / 64;
    using O = Ops<P, S>;
    static_assert(!TRAIN || (TB == 4 && P != NIV_BF16), "training: four tiles, FP32 or FP16");
    static_assert(!S::SL || WLDS, "lane slices read the level table from LDS");
    static_assert(!TRAIN || S::DIN == S::DIN_IN, "training: kernel columns are the parameter columns");
    // training saves: per 64-sample chunk, X_0 (DIN rows) then X_1..X_H (W rows), each [row][64]
    constexpr int64_t CHUNK_BYTES = (int64_t)(S::DIN + S::H * S::W) * 64 * O::ES;
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4, j = lane & 15;
    // The frame table is read from the argument segment with scalar loads,
    // indexed by the (block-uniform) frame of the current tile.
    typedef const __attribute__((address_space(4))) QueryArgs *ConstArgs;
    typedef const __attribute__((address_space(4))) LevelConst *ConstLevels;
    ConstArgs ka = (ConstArgs)__builtin_amdgcn_kernarg_segment_ptr();

    uint32_t *stage = reinterpret_cast<uint32_t *>(smem + (WLDS ? O::W_BYTES : 0)) + wave * 64 * O::ROW_DW;
    int staged = -1;  // frame whose operand block is in LDS (block-uniform)

    // Tile order.  Workgroup b runs on XCD b % 8; with xcd_order each XCD
    // takes a contiguous eighth of the tiles (pixels close on screen touch
    // the same grid cells and now share that XCD's L2), else tiles are
    // strided over all workgroups.  Both are uniform over the workgroup.
    const bool by_xcd = a.xcd_order && (gridDim.x % kXcds) == 0;
    const int64_t per_xcd = (a.n_tiles + kXcds - 1) / kXcds;
    const int64_t first = by_xcd ? (int64_t)(blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds
                                 : (int64_t)blockIdx.x;
    const int64_t last = by_xcd ? (int64_t)(blockIdx.x % kXcds + 1) * per_xcd : a.n_tiles;
    const int64_t step = by_xcd ? (int64_t)(gridDim.x / kXcds) : (int64_t)gridDim.x;
    for (int64_t tile = first; tile < last && tile < a.n_tiles; tile += step) {
        int fi = 0;
        for (int k = 1; k < a.n_frames; ++k)
            if (tile >= ka->f[k].tile_begin) fi = k;
        const uint8_t *fmodel = ka->f[fi].model;
        if constexpr (WLDS) {
            if (fi != staged) {  // operand block of this frame's model -> LDS
                __syncthreads();
                const u4 *src = reinterpret_cast<const u4 *>(fmodel + kLevelBytes);
                u4 *dst = reinterpret_cast<u4 *>(smem);
                for (int k = threadIdx.x; k < O::W_BYTES / 16; k += BLOCK) dst[k] = src[k];
                if constexpr (S::SL) {  // level table behind the weights (per-lane level reads)
                    const u4 *lsrc = reinterpret_cast<const u4 *>(fmodel);
                    u4 *ldst = reinterpret_cast<u4 *>(smem + O::W_BYTES);
                    for (int k = threadIdx.x; k < kLevelBytes / 16; k += BLOCK) ldst[k] = lsrc[k];
                }
                if constexpr (TRAIN && P == NIV_FP16) {  // grid level 0 behind the staging blocks
                    const uint32_t *gsrc = reinterpret_cast<const uint32_t *>(fmodel + a.grid_off) + a.l0_off;
                    uint32_t *l0 = reinterpret_cast<uint32_t *>(smem + O::W_BYTES) + kWavesPerBlock * 64 * O::ROW_DW;
                    for (uint32_t k = threadIdx.x; k < a.l0_words; k += BLOCK) l0[k] = gsrc[k];
                }
                __syncthreads();
                staged = fi;
            }
        }
        const int64_t count = ka->f[fi].count;
        const int64_t chunk = (tile - ka->f[fi].tile_begin) * kWavesPerBlock + wave;
        if (chunk * 64 >= count) continue;   // this wave has no pixels in the frame's last tile
        const __amdgpu_buffer_rsrc_t grid_rsrc = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(fmodel + a.grid_off), (short)0, (int)a.grid_bytes, 0x00020000);
        // frequency code of the frame's scene variables
        float gam[16 * (S::NEX > 0 ? S::NEX : 1)];
        if constexpr (S::NEX > 0) {
#pragma unroll
            for (int e = 0; e < S::NEX; ++e)
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    float t = ka->f[fi].extra[e] * (float)(1 << k);   // exact scaling by 2^k
                    gam[16 * e + 2 * k] = sinpif(t);
                    gam[16 * e + 2 * k + 1] = cospif(t);
                }
        }
        ConstLevels lvs = (ConstLevels)fmodel;
        const uint8_t *wop = WLDS ? smem : fmodel + kLevelBytes;
        const float *f_pos = ka->f[fi].pos, *f_nrm = ka->f[fi].nrm, *f_alb = ka->f[fi].albedo;
        const uint8_t *f_mask = ka->f[fi].mask;
        const int64_t q = chunk * 64 + lane;
        const bool live = q < count;
        // G-buffer pixel of this query (half-resolution samples read every
        // other pixel of every other row)
        int64_t qs = q;
        if (ka->f[fi].sub_w > 0) {
            const uint32_t sw = (uint32_t)ka->f[fi].sub_w;
            const uint32_t r = (uint32_t)q / sw, c = (uint32_t)q - r * sw;
            qs = 2 * ((int64_t)r * ka->f[fi].src_w + c);
        }
        float *f_inputs = ka->f[fi].out_inputs;
        bool on = false, work = false;
        uint32_t flags = 0u;
        // lane-sliced layer-0 operands of the TB tiles in flight: [part][tile][dword]
        constexpr int SL_DW = (P == NIV_FP32) ? 16 : 8;
        [[maybe_unused]] uint32_t sl[O::NS][TB][SL_DW];
        [[maybe_unused]] uint32_t tfl[4];
        [[maybe_unused]] bool ton[4], twk[4];
        // ---- 1'. lane-sliced encoding: lane (g, j) serves pixel 16t + j of
        // every tile t; it encodes grid levels 4s + g (s = 0..3) and SH /
        // frequency-code entries 4g..4g+3 of that pixel, i.e. exactly its own
        // layer-0 operand elements.  Runs per group of TB tiles, just before
        // their matrix products, so only TB tiles of operands are live.
        // each lane loads its own pixel (coalesced); the lanes serving it in
        // the sliced layout fetch it with a cross-lane permute
        [[maybe_unused]] uint32_t own[7];
        if constexpr (S::SL) {
            bool o = false;
            float v[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            if (live) {
                o = f_mask ? (f_mask[qs] != 0) : true;
                if (o) {
                    v[0] = f_pos[3 * qs]; v[1] = f_pos[3 * qs + 1]; v[2] = f_pos[3 * qs + 2];
                    v[3] = f_nrm[3 * qs]; v[4] = f_nrm[3 * qs + 1]; v[5] = f_nrm[3 * qs + 2];
                }
            }
#pragma unroll
            for (int c = 0; c < 6; ++c) own[c] = f2u(v[c]);
            own[6] = o ? 1u : 0u;
        }
        auto encode_tiles = [&](int tb0) {
            double pd[TB][3];
#pragma unroll
            for (int tt = 0; tt < TB; ++tt) {
                const int t = tb0 + tt;
                const int src = (16 * t + j) << 2;   // byte address of the pixel's own lane
                uint32_t r[7];
#pragma unroll
                for (int c = 0; c < 7; ++c) r[c] = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)own[c]);
                const bool o = r[6] != 0u;
                float x = u2f(r[0]), y = u2f(r[1]), z = u2f(r[2]);
                float mx = u2f(r[3]), my = u2f(r[4]), mz = u2f(r[5]);
                bool bd = !(__builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(z) &&
                            __builtin_isfinite(mx) && __builtin_isfinite(my) && __builtin_isfinite(mz));
#pragma unroll
                for (int e = 0; e < S::NEX; ++e) bd |= !__builtin_isfinite(ka->f[fi].extra[e]);
                const float nm = fmaxf(fabsf(mx), fmaxf(fabsf(my), fabsf(mz)));
                bd |= !(nm > 0.0f);
                const float ns = (nm > 0.0f) ? 1.0f / nm : 0.0f;
                mx *= ns; my *= ns; mz *= ns;
                const float n2 = mx * mx + my * my + mz * mz;
                const bool wk = o && !bd;
                uint32_t fl = (o && bd) ? 2u : 0u;
                double pp[3] = {x, y, z};
                bool out = false;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    out |= (pp[c] < a.lo[c]) | (pp[c] > a.hi[c]);
                    pd[tt][c] = pp[c] < a.lo[c] ? a.lo[c] : (pp[c] > a.hi[c] ? a.hi[c] : pp[c]);
                }
                if (wk && out) fl |= 1u;
                tfl[t] = fl; ton[t] = o; twk[t] = wk;
                const float rn = wk ? __builtin_amdgcn_rsqf(n2) : 0.0f;
                float sh[16];
                sh16(mx * rn, my * rn, mz * rn, sh);
                float se[4], fe[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    se[e] = g == 0 ? sh[e] : g == 1 ? sh[4 + e] : g == 2 ? sh[8 + e] : sh[12 + e];
                    fe[e] = g == 0 ? gam[e] : g == 1 ? gam[4 + e] : g == 2 ? gam[8 + e] : gam[12 + e];
                }
                if constexpr (P == NIV_FP32) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        sl[0][tt][8 + e] = f2u(se[e]);
                        sl[0][tt][12 + e] = f2u(fe[e]);
                    }
                } else {
                    if constexpr (O::NS == 2) {
                        Prec<P>::split(se[0], se[1], sl[0][tt][4], sl[O::NS - 1][tt][4]);
                        Prec<P>::split(se[2], se[3], sl[0][tt][5], sl[O::NS - 1][tt][5]);
                        Prec<P>::split(fe[0], fe[1], sl[0][tt][6], sl[O::NS - 1][tt][6]);
                        Prec<P>::split(fe[2], fe[3], sl[0][tt][7], sl[O::NS - 1][tt][7]);
                    } else {
                        sl[0][tt][4] = Prec<P>::pack(se[0], se[1]);
                        sl[0][tt][5] = Prec<P>::pack(se[2], se[3]);
                        sl[0][tt][6] = Prec<P>::pack(fe[0], fe[1]);
                        sl[0][tt][7] = Prec<P>::pack(fe[2], fe[3]);
                    }
                }
            }
            // grid levels 4s + g: the level's constants are per-lane LDS reads
            // (one set of loads for dense and hashed levels, the next slot's
            // gathers in flight while a slot is blended)
            const LevelConst *lt = reinterpret_cast<const LevelConst *>(smem + O::W_BYTES);
            LevelFetch<P> cur[TB], nxt[TB];
            {
                const LevelRegs lc = load_level(lt + g);
#pragma unroll
                for (int tt = 0; tt < TB; ++tt) level_issue_vec<P>(lc, pd[tt], a.hash_mask, grid_rsrc, cur[tt]);
            }
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2) {
                if (s2 + 1 < 4) {
                    const LevelRegs lc = load_level(lt + 4 * (s2 + 1) + g);
#pragma unroll
                    for (int tt = 0; tt < TB; ++tt)
                        level_issue_vec<P>(lc, pd[tt], a.hash_mask, grid_rsrc, nxt[tt]);
                }
#pragma unroll
                for (int tt = 0; tt < TB; ++tt) {
                    const f2 f = level_blend<P>(cur[tt]);
                    cur[tt] = nxt[tt];
                    if constexpr (P == NIV_FP32) {
                        sl[0][tt][2 * s2] = f2u(f.x);
                        sl[0][tt][2 * s2 + 1] = f2u(f.y);
                    } else {
                        if constexpr (O::NS == 2) Prec<P>::split(f.x, f.y, sl[0][tt][s2], sl[O::NS - 1][tt][s2]);
                        else sl[0][tt][s2] = Prec<P>::pack(f.x, f.y);
                    }
                }
            }
            // no bias anywhere: a pixel without valid inputs feeds zeros (E = 0)
#pragma unroll
            for (int tt = 0; tt < TB; ++tt)
#pragma unroll
                for (int sp = 0; sp < O::NS; ++sp)
#pragma unroll
                    for (int d = 0; d < SL_DW; ++d)
                        if (!twk[tb0 + tt]) sl[sp][tt][d] = 0u;
            if (f_inputs) {
#pragma unroll
                for (int tt = 0; tt < TB; ++tt) {
                    const int64_t qt = chunk * 64 + 16 * (tb0 + tt) + j;
                    if (qt >= count) continue;
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        float val;
                        if constexpr (P == NIV_FP32) {
                            val = u2f(sl[0][tt][v]);
                        } else {
                            f2 h = Prec<P>::unpack(sl[0][tt][v >> 1]);
                            val = (v & 1) ? h.y : h.x;
                            if constexpr (O::NS == 2) {
                                f2 l = Prec<P>::unpack(sl[1][tt][v >> 1]);
                                val += (v & 1) ? l.y : l.x;
                            }
                        }
                        f_inputs[qt * S::DIN_IN + slice_col(v, g)] = val;
                    }
                }
            }
        };
        if constexpr (S::SL) {
            static_assert(!TRAIN, "training uses the staged encoding");
        } else {
        // ---- 1. load and encode this lane's pixel
        float px = 0.f, py = 0.f, pz = 0.f, nx = 0.f, ny = 0.f, nz = 0.f;
        if (live) {
            on = f_mask ? (f_mask[qs] != 0) : true;
            if constexpr (TRAIN) on = a.valid ? (a.valid[q] != 0) : true;
            if (on) {
                px = f_pos[3 * qs]; py = f_pos[3 * qs + 1]; pz = f_pos[3 * qs + 2];
                nx = f_nrm[3 * qs]; ny = f_nrm[3 * qs + 1]; nz = f_nrm[3 * qs + 2];
            }
        }
        bool bad = !(__builtin_isfinite(px) && __builtin_isfinite(py) && __builtin_isfinite(pz) &&
                     __builtin_isfinite(nx) && __builtin_isfinite(ny) && __builtin_isfinite(nz));
        if constexpr (S::NEX > 0) {
            if (TRAIN && a.extra_ps) {
#pragma unroll
                for (int e = 0; e < S::NEX; ++e) {
                    const float te = live ? a.extra_ps[q * S::NEX + e] : 0.0f;
                    bad |= !__builtin_isfinite(te);
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        float t = te * (float)(1 << k);
                        gam[16 * e + 2 * k] = sinpif(t);
                        gam[16 * e + 2 * k + 1] = cospif(t);
                    }
                }
            } else {
#pragma unroll
                for (int e = 0; e < S::NEX; ++e) bad |= !__builtin_isfinite(ka->f[fi].extra[e]);
            }
        }
        // scale by the largest component first so that tiny or huge normals
        // normalise without underflow or overflow
        const float nm = fmaxf(fabsf(nx), fmaxf(fabsf(ny), fabsf(nz)));
        bad |= !(nm > 0.0f);
        const float ns = (nm > 0.0f) ? 1.0f / nm : 0.0f;
        nx *= ns; ny *= ns; nz *= ns;
        const float n2 = nx * nx + ny * ny + nz * nz;
        work = on && !bad;
        flags = (on && bad) ? 2u : 0u;
        double p[3] = {px, py, pz};
        bool outside = false;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            outside |= (p[c] < a.lo[c]) | (p[c] > a.hi[c]);
            p[c] = p[c] < a.lo[c] ? a.lo[c] : (p[c] > a.hi[c] ? a.hi[c] : p[c]);
        }
        if (work && outside) flags |= 1u;

        uint32_t *row = stage + lane * O::ROW_DW;
        // the FP16 query takes its cell coordinates in FP32
        constexpr bool F32C = (P == NIV_FP16) && !TRAIN;
        // the FP32 and BF16 queries overlap the levels' gathers; the FP16
        // query and the training forward go level by level (measured faster:
        // paired dense loads, and the training kernel's registers)
        constexpr bool PIPE = !F32C && !TRAIN && S::F == 2;
        if constexpr (S::L > 0 && PIPE) {
            // grid levels for every lane (lanes without work encode the box
            // corner and store zeros), so that the gathers are not inside a
            // divergent branch and the next level's loads are in flight while
            // a level is blended
#pragma unroll
            for (int c = 0; c < 3; ++c) p[c] = work ? p[c] : a.lo[c];
            const float pf[3] = {(float)p[0], (float)p[1], (float)p[2]};
            LevelFetch<P> cur, nxt;
            level_issue<P, F32C>(lvs[0], p, a.hash_mask, grid_rsrc, pf, cur);
#pragma unroll
            for (int l = 0; l < S::L; ++l) {
                if (l + 1 < S::L) level_issue<P, F32C>(lvs[l + 1], p, a.hash_mask, grid_rsrc, pf, nxt);
                f2 f = level_blend<P>(cur);
                f.x = work ? f.x : 0.0f;
                f.y = work ? f.y : 0.0f;
                if constexpr (P == NIV_FP32) {
                    row[2 * l] = f2u(f.x);
                    row[2 * l + 1] = f2u(f.y);
                } else if constexpr (O::NS == 2) {
                    Prec<P>::split(f.x, f.y, row[l], row[O::PART_DW + l]);
                } else {
                    row[l] = Prec<P>::pack(f.x, f.y);
                }
                cur = nxt;
            }
        }
        if (work) {
            if constexpr (S::L > 0 && S::F == 4) {
                // four features per entry: one 8- or 16-byte load per corner
                const float pf[3] = {(float)p[0], (float)p[1], (float)p[2]};
#pragma unroll
                for (int l = 0; l < S::L; ++l) {
                    const f4 f = encode_level_buf4<P, F32C>(lvs[l], p, a.hash_mask, grid_rsrc, pf);
                    if constexpr (P == NIV_FP32) {
                        row[4 * l] = f2u(f.x);
                        row[4 * l + 1] = f2u(f.y);
                        row[4 * l + 2] = f2u(f.z);
                        row[4 * l + 3] = f2u(f.w);
                    } else if constexpr (O::NS == 2) {
                        Prec<P>::split(f.x, f.y, row[2 * l], row[O::PART_DW + 2 * l]);
                        Prec<P>::split(f.z, f.w, row[2 * l + 1], row[O::PART_DW + 2 * l + 1]);
                    } else {
                        row[2 * l] = Prec<P>::pack(f.x, f.y);
                        row[2 * l + 1] = Prec<P>::pack(f.z, f.w);
                    }
                }
            } else if constexpr (S::L > 0 && !PIPE) {
                // level by level, the storage kind as a branch (paired 8-byte
                // loads on dense levels)
                const float pf[3] = {(float)p[0], (float)p[1], (float)p[2]};
#pragma unroll
                for (int l = 0; l < S::L; ++l) {
                    f2 f;
                    if (TRAIN && P == NIV_FP16 && l == 0 && a.l0_words) {
                        // the training forward's samples are spread over the
                        // volume: level 0 comes from its LDS copy instead of
                        // a gather touching a cache line per lane
                        const uint32_t *l0 = reinterpret_cast<const uint32_t *>(smem + O::W_BYTES) +
                                             kWavesPerBlock * 64 * O::ROW_DW;
                        f = encode_dense_lds<P>(lvs[0], p, l0);
                    } else {
                        f = encode_level_buf<P, F32C>(lvs[l], p, a.hash_mask, grid_rsrc, pf);
                    }
                    if constexpr (P == NIV_FP32) {
                        row[2 * l] = f2u(f.x);
                        row[2 * l + 1] = f2u(f.y);
                    } else if constexpr (O::NS == 2) {
                        Prec<P>::split(f.x, f.y, row[l], row[O::PART_DW + l]);
                    } else {
                        row[l] = Prec<P>::pack(f.x, f.y);
                    }
                }
            }
            if constexpr (S::PB > 0) {
                // positional code of the grid-free models (Sec. 4.1): u on the
                // unit cube in FP64, split into two floats, then sin and cos
                // of 2^k pi u with an exact argument reduction (16-bit
                // operands: the other bands by angle doubling)
                float pe[S::PEW];
                double ud[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    ud[c] = __builtin_fma(p[c], a.pe_k[c], a.pe_o[c]);
                    const float uh = (float)ud[c];
                    const float ul = (float)(ud[c] - (double)uh);
                    float sv[S::PB], cv[S::PB];
                    pos_code_axis<S::PB, P == NIV_FP32 ? 1 : (P == NIV_FP16 ? 8 : 4)>(uh, ul, sv, cv);
#pragma unroll
                    for (int b = 0; b < S::PB; ++b) {
                        pe[6 * b + c] = sv[b];
                        pe[6 * b + 3 + c] = cv[b];
                    }
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) pe[6 * S::PB + c] = (float)ud[c];
                pe[6 * S::PB + 3] = 0.0f;
                if constexpr (P == NIV_FP32) {
#pragma unroll
                    for (int k = 0; k < S::PEW; ++k) row[S::GF + k] = f2u(pe[k]);
                } else {
#pragma unroll
                    for (int k = 0; k < S::PEW / 2; ++k) {
                        if constexpr (O::NS == 2)
                            Prec<P>::split(pe[2 * k], pe[2 * k + 1], row[S::GF / 2 + k],
                                           row[O::PART_DW + S::GF / 2 + k]);
                        else
                            row[S::GF / 2 + k] = Prec<P>::pack(pe[2 * k], pe[2 * k + 1]);
                    }
                }
            }
            const float rn = __builtin_amdgcn_rsqf(n2);
            float sh[16];
            sh16(nx * rn, ny * rn, nz * rn, sh);
            constexpr int base = (P == NIV_FP32) ? S::GF + S::PEW : (S::GF + S::PEW) / 2;
            // zero columns that pad the input to a multiple of 16
            constexpr int used = S::GF + S::PEW + 16 + 16 * S::NEX;
            if constexpr (P == NIV_FP32) {
#pragma unroll
                for (int k = 0; k < 16; ++k) row[base + k] = f2u(sh[k]);
#pragma unroll
                for (int k = 0; k < 16 * S::NEX; ++k)
                    row[base + 16 + k] = f2u(gam[k]);
#pragma unroll
                for (int k = used; k < S::DIN; ++k) row[k] = 0u;
            } else {
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    if constexpr (O::NS == 2)
                        Prec<P>::split(sh[2 * k], sh[2 * k + 1], row[base + k], row[O::PART_DW + base + k]);
                    else
                        row[base + k] = Prec<P>::pack(sh[2 * k], sh[2 * k + 1]);
                }
#pragma unroll
                for (int k = 0; k < 8 * S::NEX; ++k) {
                    if constexpr (O::NS == 2)
                        Prec<P>::split(gam[2 * k], gam[2 * k + 1], row[base + 8 + k],
                                       row[O::PART_DW + base + 8 + k]);
                    else
                        row[base + 8 + k] = Prec<P>::pack(gam[2 * k], gam[2 * k + 1]);
                }
#pragma unroll
                for (int k = used / 2; k < S::DIN / 2; ++k)
#pragma unroll
                    for (int sp = 0; sp < O::NS; ++sp) row[sp * O::PART_DW + k] = 0u;
            }
        } else {
            // no bias anywhere: an all-zero input gives E = 0 (the
            // pipelined grid columns are already zero)
            constexpr int done = !PIPE ? 0 : (P == NIV_FP32 ? S::GF : S::GF / 2);
#pragma unroll
            for (int k = 0; k < O::NS * O::PART_DW; ++k)
                if (k % O::PART_DW >= done) row[k] = 0u;
        }
        if (f_inputs && live) {
            // in the order of the parameters of W_0
            float *dst = f_inputs + q * S::DIN_IN;
            if constexpr (P == NIV_FP32) {
#pragma unroll
                for (int k = 0; k < S::DIN; ++k)
                    if (S::in_col(k) >= 0) dst[S::in_col(k)] = u2f(row[k]);
            } else {
#pragma unroll
                for (int k = 0; k < S::DIN / 2; ++k) {
                    f2 v = Prec<P>::unpack(row[k]);
                    if constexpr (O::NS == 2) {
                        f2 w = Prec<P>::unpack(row[O::PART_DW + k]);
                        v.x += w.x;
                        v.y += w.y;
                    }
                    if (S::in_col(2 * k) >= 0) dst[S::in_col(2 * k)] = v.x;
                    if (S::in_col(2 * k + 1) >= 0) dst[S::in_col(2 * k + 1)] = v.y;
                }
            }
        }
        if constexpr (TRAIN) {
            uint8_t *xs = a.x_save + chunk * CHUNK_BYTES;
            if constexpr (P == NIV_FP32) {
#pragma unroll
                for (int k = 0; k < S::DIN; ++k)
                    reinterpret_cast<uint32_t *>(xs)[k * 64 + lane] = row[k];
            } else {
#pragma unroll
                for (int k = 0; k < S::DIN / 2; ++k) {
                    reinterpret_cast<uint16_t *>(xs)[(2 * k) * 64 + lane] = (uint16_t)(row[k] & 0xffffu);
                    reinterpret_cast<uint16_t *>(xs)[(2 * k + 1) * 64 + lane] = (uint16_t)(row[k] >> 16);
                }
            }
        }
        if constexpr (PROBE) {
            uint32_t xo = 0u;
#pragma unroll
            for (int k = 0; k < O::NS * O::PART_DW; ++k) xo ^= row[k];
            if (live) ka->f[fi].out_E[3 * q] = u2f(xo);
            continue;
        }
        }  // staged encoding
        // the operand reads below must not move above the row writes
        wave_lds_fence();

        // ---- 2/3. MLP on the matrix cores, TB tiles of 16 pixels at a time
        f4 acc_o[4];  // output layer per tile: RGB of pixel 16t + j in lane j
#pragma unroll
        for (int t = 0; t < 4; ++t) acc_o[t] = (f4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t0 = 0; t0 < 4; t0 += TB) {
            if constexpr (S::SL) encode_tiles(t0);
            f4 acc[TB][S::NOB];
            // layer 0
            if constexpr (P == NIV_FP32) {
                float b0[TB][S::KLG];
#pragma unroll
                for (int t = 0; t < TB; ++t) {
                    if constexpr (S::SL) {
#pragma unroll
                        for (int k = 0; k < S::KLG; ++k) b0[t][k] = u2f(sl[0][t][k]);
                        continue;
                    }
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
                    // wide layers: keep the weight loads of one output block together
                    if constexpr (S::W > 64) __builtin_amdgcn_sched_barrier(0);
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
                    if constexpr (S::SL) {
#pragma unroll
                        for (int k = 0; k < O::LANE_DW; ++k) b0[sp][t][k] = sl[sp][t][k];
                        continue;
                    }
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
                    // wide layers: keep the weight loads of one output block together
                    if constexpr (S::W > 64) __builtin_amdgcn_sched_barrier(0);
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
                            bh[t][4 * ob] = Prec<P>::relu(acc[t][ob].x);
                            bh[t][4 * ob + 1] = Prec<P>::relu(acc[t][ob].y);
                            bh[t][4 * ob + 2] = Prec<P>::relu(acc[t][ob].z);
                            bh[t][4 * ob + 3] = Prec<P>::relu(acc[t][ob].w);
                        }
                    if constexpr (TRAIN) {
                        uint32_t *xs = reinterpret_cast<uint32_t *>(a.x_save + chunk * CHUNK_BYTES) +
                                       (S::DIN + (layer - 1) * S::W) * 64;
                        uint32_t mk[S::W / 32];
#pragma unroll
                        for (int d = 0; d < S::W / 32; ++d) mk[d] = 0u;
#pragma unroll
                        for (int t = 0; t < TB; ++t)
#pragma unroll
                            for (int ob = 0; ob < S::NOB; ++ob)
#pragma unroll
                                for (int r = 0; r < 4; ++r) {
                                    const float v = bh[t][4 * ob + r];
                                    xs[(16 * ob + 4 * g + r) * 64 + 16 * t + j] = f2u(v);
                                    const int bit = (t * S::NOB + ob) * 4 + r;
                                    mk[bit >> 5] |= (v > 0.f ? 1u : 0u) << (bit & 31);
                                }
#pragma unroll
                        for (int d = 0; d < S::W / 32; ++d)
                            a.mask_save[((chunk * S::H + (layer - 1)) * (S::W / 32) + d) * 64 + lane] = mk[d];
                    }
                    if (last) {
#pragma unroll
                        for (int t = 0; t < TB; ++t)
#pragma unroll
                            for (int c = 0; c < O::HOPS; ++c) {
                                float av = reinterpret_cast<const float *>(lw + c * O::OPB)[lane];
                                acc_o[t0 + t] = Prec<P>::mma1(av, bh[t][c], acc_o[t0 + t]);
                            }
                    } else {
#pragma unroll
                        for (int ob = 0; ob < S::NOB; ++ob) {
                            // wide layers: keep the weight loads of one output block together
                            if constexpr (S::W > 64) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                            for (int t = 0; t < TB; ++t) acc[t][ob] = (f4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
                            for (int c = 0; c < O::HOPS; ++c) {
                                float av = reinterpret_cast<const float *>(lw + ob * O::HROW + c * O::OPB)[lane];
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
                            if constexpr (O::NS == 1) {
                                bh[0][t][2 * ob] = Prec<P>::pack_relu(acc[t][ob].x, acc[t][ob].y);
                                bh[0][t][2 * ob + 1] = Prec<P>::pack_relu(acc[t][ob].z, acc[t][ob].w);
                            } else {
                                Prec<P>::split_relu(acc[t][ob].x, acc[t][ob].y, bh[0][t][2 * ob],
                                                    bh[O::NS - 1][t][2 * ob]);
                                Prec<P>::split_relu(acc[t][ob].z, acc[t][ob].w, bh[0][t][2 * ob + 1],
                                                    bh[O::NS - 1][t][2 * ob + 1]);
                            }
                        }
                    if constexpr (TRAIN) {
                        // the layer's input, [neuron][64 samples], through this
                        // wave's staging block (free once layer 0 has read it)
                        // in halves of 32 neurons: 2-byte LDS writes, then
                        // coalesced 16-byte stores
                        uint8_t *xs = a.x_save + chunk * CHUNK_BYTES + (S::DIN + (layer - 1) * S::W) * 64 * 2;
                        constexpr int RS = 68;   // halves per staged row (64 samples + padding)
                        static_assert(32 * RS * 2 <= 64 * O::ROW_DW * 4, "half a layer fits the staging block");
                        uint16_t *tb16 = reinterpret_cast<uint16_t *>(stage);
                        uint32_t mk[S::W / 32];
#pragma unroll
                        for (int d = 0; d < S::W / 32; ++d) mk[d] = 0u;
#pragma unroll
                        for (int hf = 0; hf < 2; ++hf) {
                            wave_lds_fence();
#pragma unroll
                            for (int t = 0; t < TB; ++t)
#pragma unroll
                                for (int ob = 2 * hf; ob < 2 * hf + 2; ++ob)
#pragma unroll
                                    for (int r = 0; r < 4; ++r) {
                                        const uint32_t w2 = bh[0][t][2 * ob + (r >> 1)];
                                        const uint16_t hv = (uint16_t)((r & 1) ? (w2 >> 16) : (w2 & 0xffffu));
                                        tb16[(16 * (ob - 2 * hf) + 4 * g + r) * RS + 16 * t + j] = hv;
                                        const int bit = (t * S::NOB + ob) * 4 + r;
                                        mk[bit >> 5] |= (hv != 0 ? 1u : 0u) << (bit & 31);
                                    }
                            wave_lds_fence();
#pragma unroll
                            for (int i = 0; i < 4; ++i) {
                                const int ci = lane + 64 * i, row = ci >> 3, c = ci & 7;
                                const u2 lo = *reinterpret_cast<const u2 *>(tb16 + row * RS + 8 * c);
                                const u2 hi = *reinterpret_cast<const u2 *>(tb16 + row * RS + 8 * c + 4);
                                *reinterpret_cast<u4 *>(xs + ((32 * hf + row) * 64 + 8 * c) * 2) =
                                    (u4){lo.x, lo.y, hi.x, hi.y};
                            }
                        }
                        wave_lds_fence();   // the staging block is written again by the next tile
#pragma unroll
                        for (int d = 0; d < S::W / 32; ++d)
                            a.mask_save[((chunk * S::H + (layer - 1)) * (S::W / 32) + d) * 64 + lane] = mk[d];
                    }
                    // a block row of operands: HF full-depth, then HH half-depth
                    if (last) {
#pragma unroll
                        for (int t = 0; t < TB; ++t) {
#pragma unroll
                            for (int kb = 0; kb < O::HF; ++kb) {
                                u4 av = reinterpret_cast<const u4 *>(lw + kb * O::OPB)[lane];
#pragma unroll
                                for (int sp = 0; sp < O::NS; ++sp) {
                                    u4 bv = {bh[sp][t][4 * kb], bh[sp][t][4 * kb + 1], bh[sp][t][4 * kb + 2],
                                             bh[sp][t][4 * kb + 3]};
                                    acc_o[t0 + t] = Prec<P>::mma(av, bv, acc_o[t0 + t]);
                                }
                            }
                            if constexpr (O::HH) {
                                u2 av = reinterpret_cast<const u2 *>(lw + O::HF * O::OPB)[lane];
#pragma unroll
                                for (int sp = 0; sp < O::NS; ++sp) {
                                    u2 bv = {bh[sp][t][4 * O::HF], bh[sp][t][4 * O::HF + 1]};
                                    acc_o[t0 + t] = Prec<P>::mma_half(av, bv, acc_o[t0 + t]);
                                }
                            }
                        }
                    } else {
#pragma unroll
                        for (int ob = 0; ob < S::NOB; ++ob) {
                            // wide layers: keep the weight loads of one output block together
                            if constexpr (S::W > 64) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                            for (int t = 0; t < TB; ++t) acc[t][ob] = (f4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
                            for (int kb = 0; kb < O::HF; ++kb) {
                                u4 av = reinterpret_cast<const u4 *>(lw + ob * O::HROW + kb * O::OPB)[lane];
#pragma unroll
                                for (int sp = 0; sp < O::NS; ++sp)
#pragma unroll
                                for (int t = 0; t < TB; ++t) {
                                    u4 bv = {bh[sp][t][4 * kb], bh[sp][t][4 * kb + 1], bh[sp][t][4 * kb + 2],
                                             bh[sp][t][4 * kb + 3]};
                                    acc[t][ob] = Prec<P>::mma(av, bv, acc[t][ob]);
                                }
                            }
                            if constexpr (O::HH) {
                                u2 av = reinterpret_cast<const u2 *>(lw + ob * O::HROW + O::HF * O::OPB)[lane];
#pragma unroll
                                for (int sp = 0; sp < O::NS; ++sp)
#pragma unroll
                                for (int t = 0; t < TB; ++t) {
                                    u2 bv = {bh[sp][t][4 * O::HF], bh[sp][t][4 * O::HF + 1]};
                                    acc[t][ob] = Prec<P>::mma_half(av, bv, acc[t][ob]);
                                }
                            }
                        }
                    }
                }
            }
        }
        if constexpr (S::SL) {
            // this lane's own pixel 16g + j is the one it served in tile g
            on = g == 0 ? ton[0] : g == 1 ? ton[1] : g == 2 ? ton[2] : ton[3];
            work = g == 0 ? twk[0] : g == 1 ? twk[1] : g == 2 ? twk[2] : twk[3];
            flags = g == 0 ? tfl[0] : g == 1 ? tfl[1] : g == 2 ? tfl[2] : tfl[3];
        }
        // ---- 4. lane j (g = 0) holds the RGB of pixel 16t + j in acc_o[t]:
        // lane (g, j) takes channel c of its pixel 16g + j from lane j.
        f4 acc_out;
        {
            const int src = j << 2;  // byte address of lane j for ds_bpermute
            auto from_j = [&](float x) {
                return u2f((uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)f2u(x)));
            };
            float ch[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float e[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const f4 v = acc_o[t];
                    const float x = c == 0 ? v.x : (c == 1 ? v.y : v.z);
                    e[t] = from_j(x);
                }
                ch[c] = g == 0 ? e[0] : g == 1 ? e[1] : g == 2 ? e[2] : e[3];
            }
            acc_out = (f4){ch[0], ch[1], ch[2], 0.f};
        }
        if constexpr (TRAIN) {
            // Eq. 3: (E - y)^2 / (sg(E^2) + eps); d/dE = 2 (E - y) / (E^2 + eps)
            float lsum = 0.0f;
            bool nonfinite = false;
            if (live) {
                const float Ev[3] = {acc_out.x, acc_out.y, acc_out.z};
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float d = 0.0f;
                    if (work) {
                        const float r = Ev[c] - a.target[3 * q + c];
                        const float den = Ev[c] * Ev[c] + a.loss_eps;
                        d = 2.0f * r / den;
                        lsum += r * r / den;
                        nonfinite |= !__builtin_isfinite(d);
                    }
                    a.dE[3 * q + c] = d;
                }
            }
            // a diverged output or a non-finite target marks the whole step
            if (__ballot(nonfinite) != 0ull && lane == 0) atomicOr(a.train_status + 2, 1u);
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) lsum += __shfl_xor(lsum, off);
            if (lane == 0) atomicAdd(a.loss, lsum * a.loss_scale);
            continue;
        }
        float *f_E = ka->f[fi].out_E, *f_L = ka->f[fi].out_L;
        uint8_t *f_flags = ka->f[fi].out_flags;
        if (live) {
            float E0 = work ? acc_out.x : 0.f, E1 = work ? acc_out.y : 0.f, E2 = work ? acc_out.z : 0.f;
            if (work && !(__builtin_isfinite(E0) && __builtin_isfinite(E1) && __builtin_isfinite(E2)))
                flags |= 4u;
            else if (work && (E0 < 0.f || E1 < 0.f || E2 < 0.f))
                flags |= 16u;  // irradiance is non-negative; the linear output is not
            f_E[3 * q] = E0;
            f_E[3 * q + 1] = E1;
            f_E[3 * q + 2] = E2;
            if (f_L) {
                const float ip = 0.3183098861837907f;  // 1/pi
                float r0 = 0.f, r1 = 0.f, r2 = 0.f;
                if (on) { r0 = f_alb[3 * qs]; r1 = f_alb[3 * qs + 1]; r2 = f_alb[3 * qs + 2]; }
                f_L[3 * q] = r0 * E0 * ip;
                f_L[3 * q + 1] = r1 * E1 * ip;
                f_L[3 * q + 2] = r2 * E2 * ip;
            }
            if (f_flags) f_flags[q] = (uint8_t)flags;
        }
        // pixels the network should not be trusted with go to the Monte Carlo
        // fallback list: wave ballot, one atomic per wave
        if (a.fb_list) {
            const uint8_t *f_in = ka->f[fi].in_flags;
            // a pixel whose own inputs are not finite has nothing to estimate
            const bool fb = live && on && (flags & 2u) == 0u &&
                            (((flags & a.fb_mask) != 0u) || (f_in && f_in[q] != 0));
            const uint64_t bal = __ballot(fb);
            if (bal) {
                const uint32_t n = (uint32_t)__popcll(bal);
                const uint32_t before = (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
                uint32_t base = 0;
                if (lane == 0) base = atomicAdd(a.fb_count, n);
                base = __shfl(base, 0);
                if (fb && base + before < a.fb_cap)
                    a.fb_list[base + before] = ((uint32_t)fi << 28) | (uint32_t)q;
            }
        }
    }
}

}  // namespace niv
