// On-GPU training of the Neural Irradiance Volume (Sec. 4.5): Eq. 3 loss,
// backpropagation through the MLP on the matrix cores, scatter of the
// encoding gradient into the hash grid, and Adam.
//
// A step runs these stages on the caller's stream:
//   1. the fused query kernel in training mode: encodes each sample, runs
//      the MLP, saves every layer's input (per 64-sample chunk, row-major
//      [neuron][sample], the layout the weight-gradient products read) and
//      the ReLU masks, and writes d loss / dE (Eq. 3, stop-gradient
//      denominator) and the loss;
//   2. k_train_bwd: per chunk, the weight gradients dW_k = G_{k+1} X_k^T on
//      MFMA (the gradient is transposed through LDS), the input gradients
//      W_k^T G_{k+1} on MFMA with pre-permuted transposed weights so that
//      they come out in the same lane layout as the forward activations;
//      each wave keeps its weight gradient in the matrix-core accumulators
//      over its chunks, a workgroup's four waves add theirs in LDS and
//      write one row, and k_dw_sum adds the rows; the gradient of each
//      sample's grid features is written out level-major per chunk;
//   3. the scatter of those feature gradients to the 8 corners of every
//      level, without global atomics (device-scope atomics execute at the
//      memory side of this part, ~22 G/s): the contributions are counted
//      per bin of 4096 grid entries and workgroup (k_grid_count, on a
//      second stream beside the forward: it needs only the batch), the
//      counts are scanned (k_grid_scan_bins; the bins' totals at the start
//      of the write pass), the contributions are written bin by bin
//      (k_grid_write), and one or more workgroups per bin sum them in LDS
//      in 64-bit fixed point (k_grid_accum); a bin split over several
//      workgroups has its parts' integer sums added (k_grid_merge), so the
//      whole grid gradient is independent of scheduling;
//   4. k_adam over all parameters (it also writes the prepared model's
//      grid), then the prepared weight operands are rebuilt.
// Gradients are carried unscaled through the network and multiplied by
// 1/(3n) when they are added to the gradient buffer, so FP16 operands do not
// underflow.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "niv_internal.h"
#include "niv_device.h"
#include "mc_device.h"
#include "query_kernel.h"

namespace niv {

constexpr int kMaxMats = 12;   // weight matrices of a model (n_hidden + 1) niv_init_params takes
constexpr int kL0Words = 5120;  // LDS copy of grid level 0 in the FP16 training forward (20 KB)

// ---------------------------------------------------------------- layouts
template <int P, class S> struct Bwd {
    static constexpr bool F32 = (P == NIV_FP32);
    static constexpr int ES = F32 ? 4 : 2;
    static constexpr int EPO = F32 ? 1 : 8;
    static constexpr int OPB = 64 * EPO * ES;
    static constexpr int NIB = S::W / 16;              // row blocks of a hidden input
    static constexpr int NOB = S::W / 16;
    static constexpr int GIB = 2 * S::L / 16;          // row blocks of the grid features
    static constexpr int HOPS = F32 ? S::W / 4 : S::W / 32;
    static constexpr int OUT_OP = F32 ? 256 : 512;     // K = output channels
    static constexpr int OUT_BYTES = NIB * OUT_OP;
    static constexpr int HID_BYTES = NIB * HOPS * OPB;
    static constexpr int L0_BYTES = GIB * HOPS * OPB;
    static constexpr int BYTES = OUT_BYTES + (S::H - 1) * HID_BYTES + L0_BYTES;
    static constexpr int N_OPS = NIB + (S::H - 1) * NIB * HOPS + GIB * HOPS;
    static constexpr int64_t CHUNK_BYTES = (int64_t)(S::DIN + S::H * S::W) * 64 * ES;
    static constexpr int NMLP = S::W * S::DIN + (S::H - 1) * S::W * S::W + 3 * S::W;
    static constexpr int GB_BYTES = S::W * 64 * ES;            // gradient, [neuron][64]
    static constexpr int NFP = 2 * S::L + 2;                  // padded row of the grid-feature gradient
    static constexpr int DX_BYTES = 64 * NFP * 4;              // grid-feature gradient, [64][2L + 2]
    static constexpr int WB_BYTES = (GB_BYTES > DX_BYTES ? GB_BYTES : DX_BYTES) + 3 * 64 * 4;
    // LDS of a workgroup: four waves' blocks, reused at the end for the
    // workgroup's weight gradient
    static constexpr int LDS_BYTES = 4 * WB_BYTES > NMLP * 4 ? 4 * WB_BYTES : NMLP * 4;
    // weight-gradient tiles (16x16, f4 per lane) a wave accumulates in registers
    // over all its chunks: the output layer's, then layer H-1 down to 0
    static constexpr int T_OUT = S::W / 16;
    static constexpr int T_HID = NOB * NIB;
    static constexpr int N_TILES = T_OUT + (S::H - 1) * T_HID + NOB * (S::DIN / 16);
    static constexpr int tile_base(int k) { return T_OUT + (S::H - 1 - k) * T_HID; }
    static_assert(S::L % 8 == 0 && S::F == 2, "grid rows come in blocks of 16, two features a level");
    static_assert(S::DIN % 16 == 0, "input rows come in blocks of 16");
};

// Source parameter of element e of lane `lane` of backward operand `op`:
// the output layer's W_H^T (K = channels), then W_k^T for k = 1..H-1, then
// the grid-feature rows of W_0^T; the K index is permuted to match the lane
// layout of the gradient (as in the forward).
template <int P, class S>
__device__ int64_t bwd_source(int op, int lane, int e, int64_t n_grid)
{
    using B = Bwd<P, S>;
    const int i = lane & 15, g = lane >> 4;
    const int64_t w0 = n_grid;
    const int64_t wo = w0 + (int64_t)S::W * S::DIN + (int64_t)(S::H - 1) * S::W * S::W;
    auto out_neuron = [&](int kb) {
        return B::F32 ? 16 * (kb / 4) + 4 * g + (kb % 4) : 16 * (2 * kb + e / 4) + 4 * g + (e % 4);
    };
    if (op < B::NIB) {
        const int c = B::F32 ? g : 4 * g + e;
        if (c >= 3) return -1;
        return wo + (int64_t)c * S::W + 16 * op + i;
    }
    op -= B::NIB;
    if (op < (S::H - 1) * B::NIB * B::HOPS) {
        const int k = 1 + op / (B::NIB * B::HOPS);
        const int r = op % (B::NIB * B::HOPS);
        const int ib = r / B::HOPS, kb = r % B::HOPS;
        const int64_t wk = w0 + (int64_t)S::W * S::DIN + (int64_t)(k - 1) * S::W * S::W;
        return wk + (int64_t)out_neuron(kb) * S::W + 16 * ib + i;
    }
    op -= (S::H - 1) * B::NIB * B::HOPS;
    const int ib = op / B::HOPS, kb = op % B::HOPS;
    return w0 + (int64_t)out_neuron(kb) * S::DIN + 16 * ib + i;
}

// Also clears the step's words (status, loss) so that a step needs no
// separate fill launches (and stays capturable).
template <int P, class S>
__global__ void k_prepare_bwd(const float *__restrict__ params, uint8_t *__restrict__ out,
                              int64_t n_grid, uint32_t *__restrict__ status, int n_status,
                              float *__restrict__ loss)
{
    using B = Bwd<P, S>;
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid < n_status) status[tid] = 0u;
    if (tid == 0) *loss = 0.0f;
    if (tid >= B::N_OPS * 64) return;
    const int op = tid / 64, lane = tid % 64;
    int64_t off;
    int ne;
    if (op < B::NIB) {
        off = (int64_t)op * B::OUT_OP;
        ne = B::F32 ? 1 : 4;
    } else {
        off = B::OUT_BYTES + (int64_t)(op - B::NIB) * B::OPB;
        ne = B::EPO;
    }
    for (int e = 0; e < ne; ++e) {
        const int64_t src = bwd_source<P, S>(op, lane, e, n_grid);
        const float v = src >= 0 ? params[src] : 0.0f;
        if constexpr (B::F32) reinterpret_cast<float *>(out + off)[lane * ne + e] = v;
        else reinterpret_cast<_Float16 *>(out + off)[lane * ne + e] = (_Float16)v;
    }
}

// ---------------------------------------------------------------- backward
struct BwdArgs {
    const uint8_t *bwd;        // backward operands
    const uint8_t *x_save;
    const uint32_t *mask_save;
    const float *dE;           // [n][3], without the 1/(3n) factor
    const float *x;            // [n][3] sample positions
    const uint8_t *model;      // prepared model (level table first)
    float *grads;              // [n_params]
    float *dw_part;            // [workgroup][weights] each workgroup's weight gradient
    float *dx0;                // [chunk][L][64] float pairs: gradient of each sample's grid features
    uint8_t *sflag;            // [n] 1: the sample's features scatter into the grid
    uint32_t *vmax;            // step word [0]: largest |feature gradient| x loss_scale of a
                               // scattering sample (float bits; bounds every contribution)
    int64_t n, n_grid;
    float loss_scale;
    uint32_t hash_mask;
    double lo[3], hi[3];
};

template <int P> struct Mm;
template <> struct Mm<NIV_FP16> {
    __device__ static u4 h8(const float *v) {
        return (u4){Prec<NIV_FP16>::pack(v[0], v[1]), Prec<NIV_FP16>::pack(v[2], v[3]),
                    Prec<NIV_FP16>::pack(v[4], v[5]), Prec<NIV_FP16>::pack(v[6], v[7])};
    }
};

template <int P, class S>
__global__ __launch_bounds__(256) void k_train_bwd(const BwdArgs a)
{
    using B = Bwd<P, S>;
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, j = lane & 15;
    uint8_t *wbuf = smem + wave * B::WB_BYTES;
    float *debuf = reinterpret_cast<float *>(wbuf + (B::GB_BYTES > B::DX_BYTES ? B::GB_BYTES : B::DX_BYTES));
    // the wave's weight gradient, summed over its chunks in the matrix-core
    // accumulators (no LDS atomics per chunk)
    f4 dwacc[B::N_TILES];
#pragma unroll
    for (int t = 0; t < B::N_TILES; ++t) dwacc[t] = (f4){0.f, 0.f, 0.f, 0.f};

    const int64_t n_chunks = (a.n + 63) / 64;
    const int64_t n_waves = (int64_t)gridDim.x * 4;
    float gmax = 0.0f;   // largest |feature gradient| of this lane's scattering samples
    for (int64_t chunk = (int64_t)blockIdx.x * 4 + wave; chunk < n_chunks; chunk += n_waves) {
        const int64_t q = chunk * 64 + lane;
        const bool live = q < a.n;
        float dEl[3] = {0.f, 0.f, 0.f};
        if (live) {
            dEl[0] = a.dE[3 * q]; dEl[1] = a.dE[3 * q + 1]; dEl[2] = a.dE[3 * q + 2];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) debuf[c * 64 + lane] = dEl[c];
        wave_lds_fence();
        const uint8_t *xs = a.x_save + chunk * B::CHUNK_BYTES;
        const uint8_t *bw = a.bwd;

        // ---- output layer: dW_H[c][n] = sum_px dE[px][c] X_H[n][px]
        // (the X_H operands are loaded together first: one memory latency)
        {
            const int xrow = S::DIN + (S::H - 1) * S::W;
            if constexpr (B::F32) {
                const float *xf = reinterpret_cast<const float *>(xs);
                float xv[S::W / 16][16];
#pragma unroll
                for (int nb = 0; nb < S::W / 16; ++nb)
#pragma unroll
                    for (int s = 0; s < 16; ++s) xv[nb][s] = xf[(xrow + 16 * nb + j) * 64 + 4 * s + g];
#pragma unroll
                for (int nb = 0; nb < S::W / 16; ++nb) {
                    f4 acc = dwacc[nb];
#pragma unroll
                    for (int s = 0; s < 16; ++s) {
                        const float av = j < 3 ? debuf[j * 64 + 4 * s + g] : 0.f;
                        acc = Prec<NIV_FP32>::mma1(av, xv[nb][s], acc);
                    }
                    dwacc[nb] = acc;
                }
            } else {
                u4 xv[S::W / 16][2];
#pragma unroll
                for (int nb = 0; nb < S::W / 16; ++nb)
#pragma unroll
                    for (int h = 0; h < 2; ++h)
                        xv[nb][h] = *reinterpret_cast<const u4 *>(
                            xs + ((int64_t)(xrow + 16 * nb + j) * 64 + 32 * h + 8 * g) * 2);
                u4 av[2] = {{0u, 0u, 0u, 0u}, {0u, 0u, 0u, 0u}};
                if (j < 3) {
                    av[0] = Mm<P>::h8(debuf + j * 64 + 8 * g);
                    av[1] = Mm<P>::h8(debuf + j * 64 + 32 + 8 * g);
                }
#pragma unroll
                for (int nb = 0; nb < S::W / 16; ++nb) {
                    dwacc[nb] = Prec<P>::mma(av[0], xv[nb][0], dwacc[nb]);
                    dwacc[nb] = Prec<P>::mma(av[1], xv[nb][1], dwacc[nb]);
                }
            }
        }
        // ---- gradient w.r.t. x_H = W_H^T dE, lane layout of the forward
        f4 G[4][B::NOB];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int ib = 0; ib < B::NIB; ++ib) {
                const f4 z = {0.f, 0.f, 0.f, 0.f};
                if constexpr (B::F32) {
                    const float av = reinterpret_cast<const float *>(bw + ib * B::OUT_OP)[lane];
                    const float bv = g < 3 ? debuf[g * 64 + 16 * t + j] : 0.f;
                    G[t][ib] = Prec<NIV_FP32>::mma1(av, bv, z);
                } else {
                    const u2 av = reinterpret_cast<const u2 *>(bw + ib * B::OUT_OP)[lane];
                    u2 bv = {0u, 0u};
                    if (g == 0) {
                        bv.x = Prec<P>::pack(debuf[16 * t + j], debuf[64 + 16 * t + j]);
                        bv.y = Prec<P>::pack(debuf[128 + 16 * t + j], 0.f);
                    }
                    G[t][ib] = Prec<P>::mma_half(av, bv, z);
                }
            }
        // ---- hidden layers k = H-1 .. 0
#pragma unroll
        for (int k = S::H - 1; k >= 0; --k) {
            // G is d loss / d x_{k+1}; through the ReLU: x_{k+1} > 0
            uint32_t mk[S::W / 32];
#pragma unroll
            for (int d = 0; d < S::W / 32; ++d)
                mk[d] = a.mask_save[((chunk * S::H + k) * (S::W / 32) + d) * 64 + lane];
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int ob = 0; ob < B::NOB; ++ob) {
                    const int b0 = (t * B::NOB + ob) * 4;
                    if (!((mk[(b0 + 0) >> 5] >> ((b0 + 0) & 31)) & 1u)) G[t][ob].x = 0.f;
                    if (!((mk[(b0 + 1) >> 5] >> ((b0 + 1) & 31)) & 1u)) G[t][ob].y = 0.f;
                    if (!((mk[(b0 + 2) >> 5] >> ((b0 + 2) & 31)) & 1u)) G[t][ob].z = 0.f;
                    if (!((mk[(b0 + 3) >> 5] >> ((b0 + 3) & 31)) & 1u)) G[t][ob].w = 0.f;
                }
            // transpose G through LDS: [neuron][64 samples]
            if constexpr (B::F32) {
                float *gb = reinterpret_cast<float *>(wbuf);
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int ob = 0; ob < B::NOB; ++ob) {
                        gb[(16 * ob + 4 * g + 0) * 64 + 16 * t + j] = G[t][ob].x;
                        gb[(16 * ob + 4 * g + 1) * 64 + 16 * t + j] = G[t][ob].y;
                        gb[(16 * ob + 4 * g + 2) * 64 + 16 * t + j] = G[t][ob].z;
                        gb[(16 * ob + 4 * g + 3) * 64 + 16 * t + j] = G[t][ob].w;
                    }
            } else {
                _Float16 *gb = reinterpret_cast<_Float16 *>(wbuf);
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int ob = 0; ob < B::NOB; ++ob) {
                        gb[(16 * ob + 4 * g + 0) * 64 + 16 * t + j] = (_Float16)G[t][ob].x;
                        gb[(16 * ob + 4 * g + 1) * 64 + 16 * t + j] = (_Float16)G[t][ob].y;
                        gb[(16 * ob + 4 * g + 2) * 64 + 16 * t + j] = (_Float16)G[t][ob].z;
                        gb[(16 * ob + 4 * g + 3) * 64 + 16 * t + j] = (_Float16)G[t][ob].w;
                    }
            }
            wave_lds_fence();
            // dW_k += G X_k^T over the chunk's 64 samples; the X_k operands do
            // not depend on the output block and are loaded together first
            constexpr int DK_MAX = S::DIN > S::W ? S::DIN : S::W;
            const int dk = (k == 0) ? S::DIN : S::W;
            const int xrow = (k == 0) ? 0 : S::DIN + (k - 1) * S::W;
            const int tb = B::tile_base(k);   // this layer's tiles: ob * (dk / 16) + ib
            if constexpr (B::F32) {
                const float *gb = reinterpret_cast<const float *>(wbuf);
                const float *xf = reinterpret_cast<const float *>(xs);
                float xv[DK_MAX / 16][16];
#pragma unroll
                for (int ib = 0; ib < DK_MAX / 16; ++ib)
#pragma unroll
                    for (int s = 0; s < 16; ++s)
                        xv[ib][s] = ib * 16 < dk ? xf[(int64_t)(xrow + 16 * ib + j) * 64 + 4 * s + g] : 0.f;
#pragma unroll
                for (int ob = 0; ob < B::NOB; ++ob)
#pragma unroll
                    for (int ib = 0; ib < DK_MAX / 16; ++ib) {
                        if (ib * 16 >= dk) break;
                        f4 acc = dwacc[tb + ob * (dk / 16) + ib];
#pragma unroll
                        for (int s = 0; s < 16; ++s)
                            acc = Prec<NIV_FP32>::mma1(gb[(16 * ob + j) * 64 + 4 * s + g], xv[ib][s], acc);
                        dwacc[tb + ob * (dk / 16) + ib] = acc;
                    }
            } else {
                u4 xv[DK_MAX / 16][2];
#pragma unroll
                for (int ib = 0; ib < DK_MAX / 16; ++ib)
#pragma unroll
                    for (int h = 0; h < 2; ++h)
                        xv[ib][h] = ib * 16 < dk ? *reinterpret_cast<const u4 *>(
                                        xs + ((int64_t)(xrow + 16 * ib + j) * 64 + 32 * h + 8 * g) * 2)
                                                 : (u4){0u, 0u, 0u, 0u};
#pragma unroll
                for (int ob = 0; ob < B::NOB; ++ob) {
                    const u4 av0 = *reinterpret_cast<const u4 *>(wbuf + ((16 * ob + j) * 64 + 8 * g) * 2);
                    const u4 av1 = *reinterpret_cast<const u4 *>(wbuf + ((16 * ob + j) * 64 + 32 + 8 * g) * 2);
#pragma unroll
                    for (int ib = 0; ib < DK_MAX / 16; ++ib) {
                        if (ib * 16 >= dk) break;
                        f4 &acc = dwacc[tb + ob * (dk / 16) + ib];
                        acc = Prec<P>::mma(av0, xv[ib][0], acc);
                        acc = Prec<P>::mma(av1, xv[ib][1], acc);
                    }
                }
            }
            // d loss / d x_k = W_k^T G (grid rows only for k = 0)
            const int nib = (k == 0) ? B::GIB : B::NIB;
            const uint8_t *bk = (k == 0) ? bw + B::OUT_BYTES + (S::H - 1) * B::HID_BYTES
                                         : bw + B::OUT_BYTES + (k - 1) * B::HID_BYTES;
            f4 Gn[4][B::NOB];
            if constexpr (B::F32) {
#pragma unroll
                for (int ib = 0; ib < B::NIB; ++ib) {
                    if (ib >= nib) break;
#pragma unroll
                    for (int t = 0; t < 4; ++t) Gn[t][ib] = (f4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int c = 0; c < B::HOPS; ++c) {
                        const float av = reinterpret_cast<const float *>(bk + (ib * B::HOPS + c) * B::OPB)[lane];
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            const f4 gv = G[t][c / 4];
                            const float bv = (c % 4 == 0) ? gv.x : (c % 4 == 1) ? gv.y : (c % 4 == 2) ? gv.z : gv.w;
                            Gn[t][ib] = Prec<NIV_FP32>::mma1(av, bv, Gn[t][ib]);
                        }
                    }
                }
            } else {
                uint32_t bg[4][S::W / 8];
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int ob = 0; ob < B::NOB; ++ob) {
                        bg[t][2 * ob] = Prec<P>::pack(G[t][ob].x, G[t][ob].y);
                        bg[t][2 * ob + 1] = Prec<P>::pack(G[t][ob].z, G[t][ob].w);
                    }
#pragma unroll
                for (int ib = 0; ib < B::NIB; ++ib) {
                    if (ib >= nib) break;
#pragma unroll
                    for (int t = 0; t < 4; ++t) Gn[t][ib] = (f4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int kb = 0; kb < B::HOPS; ++kb) {
                        const u4 av = reinterpret_cast<const u4 *>(bk + (ib * B::HOPS + kb) * B::OPB)[lane];
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            const u4 bv = {bg[t][4 * kb], bg[t][4 * kb + 1], bg[t][4 * kb + 2], bg[t][4 * kb + 3]};
                            Gn[t][ib] = Prec<P>::mma(av, bv, Gn[t][ib]);
                        }
                    }
                }
            }
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int ob = 0; ob < B::NOB; ++ob) G[t][ob] = Gn[t][ob];
        }
        // ---- grid-feature gradients: rows 16ib + 4g + r of sample 16t + j,
        // through LDS ([sample][2L], rows padded by two floats so that a
        // level's column spreads over the banks), out as [chunk][level][64]
        // float pairs (one coalesced store per level)
        {
            float *dx = reinterpret_cast<float *>(wbuf);
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int ib = 0; ib < B::GIB; ++ib) {
                    float *d = dx + (16 * t + j) * B::NFP + 16 * ib + 4 * g;
                    d[0] = G[t][ib].x; d[1] = G[t][ib].y; d[2] = G[t][ib].z; d[3] = G[t][ib].w;
                }
            wave_lds_fence();
            // a sample scatters when its dE is finite and not zero (a non-finite
            // dE marks the step non-finite in the forward and never reaches the grid)
            bool scatter = live && (dEl[0] != 0.f || dEl[1] != 0.f || dEl[2] != 0.f) &&
                           __builtin_isfinite(dEl[0]) && __builtin_isfinite(dEl[1]) &&
                           __builtin_isfinite(dEl[2]);
            if (scatter) {
#pragma unroll
                for (int c = 0; c < 3; ++c) scatter &= __builtin_isfinite(a.x[3 * q + c]);
            }
            if (live) {
                const float2 *mine = reinterpret_cast<const float2 *>(dx + lane * B::NFP);
                float2 *dst = reinterpret_cast<float2 *>(a.dx0) + chunk * 64 * S::L + lane;
#pragma unroll
                for (int l = 0; l < S::L; ++l) {
                    const float2 v = mine[l];
                    dst[l * 64] = v;
                    if (scatter) gmax = fmaxf(gmax, fmaxf(fabsf(v.x), fabsf(v.y)));
                }
                a.sflag[q] = scatter ? 1 : 0;
            }
        }
    }
    // the step's bound on the grid contributions (|w g| <= |g|, weights <= 1):
    // the scale of the fixed-point sums and of 16-bit contribution records
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) gmax = fmaxf(gmax, __shfl_xor(gmax, off));
    const float cmax = gmax * a.loss_scale;
    if (lane == 0 && cmax == cmax && cmax > 0.0f) atomicMax(a.vmax, f2u(cmax));
    // the workgroup's weight gradient: the four waves add their tiles into
    // one LDS copy, wave after wave, and it goes out as one row; k_dw_sum adds
    // the rows (no atomics, a fixed summation order).  Tile element r of lane
    // (g, j) is row 16 ob + 4 g + r, column 16 ib + j of the layer's matrix.
    __syncthreads();   // every wave is done with its block
    float *red = reinterpret_cast<float *>(smem);
    for (int k = threadIdx.x; k < B::NMLP; k += 256) red[k] = 0.0f;
    __syncthreads();
    for (int w = 0; w < 4; ++w) {
        if (wave == w) {
            {
                const int woff = S::W * S::DIN + (S::H - 1) * S::W * S::W;   // output layer [3][W]
#pragma unroll
                for (int nb = 0; nb < S::W / 16; ++nb)
                    if (g == 0) {
                        red[woff + 0 * S::W + 16 * nb + j] += dwacc[nb].x;
                        red[woff + 1 * S::W + 16 * nb + j] += dwacc[nb].y;
                        red[woff + 2 * S::W + 16 * nb + j] += dwacc[nb].z;
                    }
            }
#pragma unroll
            for (int k = S::H - 1; k >= 0; --k) {
                const int dk = (k == 0) ? S::DIN : S::W;
                const int woff = (k == 0) ? 0 : S::W * S::DIN + (k - 1) * S::W * S::W;
                const int tb = B::tile_base(k);
#pragma unroll
                for (int ob = 0; ob < B::NOB; ++ob)
#pragma unroll
                    for (int ib = 0; ib < (S::DIN > S::W ? S::DIN : S::W) / 16; ++ib) {
                        if (ib * 16 >= dk) break;
                        const f4 v = dwacc[tb + ob * (dk / 16) + ib];
                        float *dst = red + woff + (16 * ob + 4 * g) * dk + 16 * ib + j;
                        dst[0] += v.x;
                        dst[dk] += v.y;
                        dst[2 * dk] += v.z;
                        dst[3 * dk] += v.w;
                    }
            }
        }
        __syncthreads();
    }
    float *row = a.dw_part + (int64_t)blockIdx.x * B::NMLP;
    for (int k = threadIdx.x; k < B::NMLP; k += 256) row[k] = red[k];
}

// Column sums of the per-workgroup weight gradients, scaled, into the
// gradient: a workgroup takes 16 columns; its 16 row groups each add rows
// g, g + 16, g + 32, ... of a column (eight loads in flight), and the 16
// partial sums are added in row-group order (a fixed summation order).
__global__ __launch_bounds__(256) void k_dw_sum(const float *__restrict__ part, int64_t nmlp, int rows,
                                               float *__restrict__ out, float scale)
{
    __shared__ float ps[16][17];
    const int c = threadIdx.x & 15, rg = threadIdx.x >> 4;
    const int64_t k = (int64_t)blockIdx.x * 16 + c;
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (k < nmlp) {
        int r = rg;
        for (; r + 7 * 16 < rows; r += 8 * 16)
#pragma unroll
            for (int u = 0; u < 8; ++u) s[u] += part[(int64_t)(r + 16 * u) * nmlp + k];
        for (; r < rows; r += 16) s[0] += part[(int64_t)r * nmlp + k];
#pragma unroll
        for (int u = 1; u < 8; ++u) s[0] += s[u];
    }
    ps[rg][c] = s[0];
    __syncthreads();
    if (rg == 0 && k < nmlp) {
        float t = 0.0f;
#pragma unroll
        for (int g = 0; g < 16; ++g) t += ps[g][c];
        out[k] = t * scale;
    }
}

// ---------------------------------------------------------------- grid scatter
// Contributions of (sample, level): the 8 corner entries e (with the level
// offset) and w_c * dL/dfeature.  Entries are binned by e >> kBinShift.
constexpr int kBinShift = 12;                 // 4096 entries (32 KB of FP32 pairs) per bin
constexpr int kBinEntries = 1 << kBinShift;
constexpr int kMaxBins = 2048;
constexpr int kBwdMaxBlocks = 512;            // workgroups of the backward (4 dW rows each)
constexpr int kScatterBlocks = 512;           // workgroups of the count and write passes
constexpr int kAccumRecords = 98304;          // records one accumulating workgroup takes (1.5x a
                                              // hashed level's bin at 2^18 samples: those stay whole)

// The first 256 bytes of the training scratch hold the step's words: [0]
// largest |grid contribution| (float bits), [1] records of the fullest bin,
// [2] non-zero when the step's loss or gradient was not finite (set by the
// forward pass; the Adam update of niv_train_step then does nothing).
constexpr int kStatusWords = 4;

struct ScatterArgs {
    const float *x;            // [n][3] sample positions
    const float *dx0;          // [chunk][L][64] float pairs
    const uint8_t *sflag;      // [n] 1: the sample's contributions are not zero (set by the backward)
    const uint8_t *valid;      // [n] the batch's valid flags, or NULL
    const uint8_t *model;      // prepared model (level table first)
    uint32_t *counts;          // [kScatterBlocks][cstride] per workgroup and bin, then their
                               // offsets within the bin
    uint32_t *totals;          // [kMaxBins] records of each bin
    uint32_t *bin_start;       // [bins + 1]
    uint32_t *work_start;      // [bins + 1] first accumulating workgroup of each bin
    uint32_t *split;           // [bins + 1] bins split over several workgroups, in order; [bins] count
    uint32_t *vmax;            // [0] bits of a bound M on every |contribution| of the step, set by
                               // the backward (>= 0 floats order as integers), [1] records of
                               // the fullest bin
    long long *parts;          // [accumulating workgroup][2 kBinEntries] fixed-point partial sums
    uint16_t *keys;            // [records] entry index within its bin
    float2 *vals;              // [records] contributions of the two features (FP32 records)
    uint32_t *vals16;          // [records] the same as an FP16 pair scaled by 2^(14 - e) (16-bit records)
    float *grads;              // grid part of the gradient: [entries][2]
    int64_t n, n_entries;
    int32_t n_levels, n_bins;
    int32_t cstride;           // row length of counts: n_bins rounded up to 4
    uint32_t hash_mask;
    float loss_scale;
    double lo[3], hi[3];
};

// Both passes: one wave takes a 64-sample chunk through every level (the
// level is wave-uniform, so its constants are scalar loads); workgroup b
// takes chunks kScatterWaves b + w, strided by kScatterWaves x the grid, in
// both passes, so a workgroup writes exactly the records it counted.
constexpr int kScatterWaves = 8;
constexpr int kScatterThreads = 64 * kScatterWaves;
constexpr int kScatterMaxLevels = 16;          // levels of the trainable shapes

// Inclusive scan over the 64 lanes of a wave.
__device__ inline uint32_t wave_scan_incl(uint32_t v, int lane)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_up(v, d);
        if (lane >= d) v += t;
    }
    return v;
}

// The samples that have records: every valid sample of the batch with a
// finite position (a superset of the samples that scatter, so the counts
// need nothing from the backward); the records of a sample the backward
// leaves out (sflag 0: its d loss / dE is zero, or the step is not finite)
// carry zeros.  p: the position clamped to the box, as the forward takes it.
__device__ inline bool scatter_sample(const ScatterArgs &a, int64_t q, double p[3])
{
    if (q >= a.n || (a.valid && !a.valid[q])) return false;
    const float x0 = a.x[3 * q], x1 = a.x[3 * q + 1], x2 = a.x[3 * q + 2];
    if (!(__builtin_isfinite(x0) && __builtin_isfinite(x1) && __builtin_isfinite(x2))) return false;
    const float xs[3] = {x0, x1, x2};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double v = xs[c];
        p[c] = v < a.lo[c] ? a.lo[c] : (v > a.hi[c] ? a.hi[c] : v);
    }
    return true;
}

__global__ __launch_bounds__(kScatterThreads) void k_grid_count(const ScatterArgs a)
{
    __shared__ uint32_t cnt[kMaxBins];
    typedef const __attribute__((address_space(4))) LevelConst *ConstLevels;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int b = threadIdx.x; b < a.n_bins; b += kScatterThreads) cnt[b] = 0u;
    __syncthreads();
    const int64_t n_chunks = (a.n + 63) / 64;
    ConstLevels lvs = (ConstLevels)a.model;
    for (int64_t chunk = (int64_t)blockIdx.x * kScatterWaves + wave; chunk < n_chunks;
         chunk += (int64_t)gridDim.x * kScatterWaves) {
        double p[3];
        if (!scatter_sample(a, chunk * 64 + lane, p)) continue;
        for (int l = 0; l < a.n_levels; ++l) {
            uint32_t idx[8];
            float w[8];
            level_corners(lvs[l], p, a.hash_mask, idx, w);
            // corners in the bin of corner 0 (all of them on coarse levels)
            // take one counter update together; the others one each
            const uint32_t b0 = idx[0] >> kBinShift;
            uint32_t n0 = 0;
#pragma unroll
            for (int c = 0; c < 8; ++c) n0 += (idx[c] >> kBinShift) == b0 ? 1u : 0u;
            atomicAdd(&cnt[b0], n0);
#pragma unroll
            for (int c = 0; c < 8; ++c)
                if ((idx[c] >> kBinShift) != b0) atomicAdd(&cnt[idx[c] >> kBinShift], 1u);
        }
    }
    __syncthreads();
    uint32_t *row = a.counts + (int64_t)blockIdx.x * a.cstride;
    for (int b = threadIdx.x; b < a.cstride; b += kScatterThreads) row[b] = b < a.n_bins ? cnt[b] : 0u;
}

// Write pass.  The waves of a workgroup order the records of their chunks
// at one level together, so that each bin receives one run of consecutive
// slots per workgroup (~128 records on a hashed level of 2^17 entries, for
// 8 chunks of 64 samples): per window of 64 of the level's bins, a histogram in LDS
// gives each record its rank in its bin, one wave scans the histogram and
// reserves each bin's run in the workgroup's segment of that bin, the
// records are staged in that order, and the workgroup stores them with
// consecutive threads on consecutive slots.  The feature gradients of a
// chunk are read one level at a time with a coalesced load (the backward
// stores them level-major per chunk).
// H16 (the FP16 training path): records carry the contributions as an FP16
// pair scaled by 2^(14 - e), M < 2^e, so every value is below 2^14 and keeps
// 11 significant bits (the operands of that path are FP16 already); 6 bytes
// per record instead of 10.
template <bool H16>
__global__ __launch_bounds__(kScatterThreads) void k_grid_write(const ScatterArgs a)
{
    // staged records: (bin in the window << 16 | entry within the bin) and
    // the value(s)
    using Val = typename std::conditional<H16, uint32_t, uint2>::type;
    constexpr int kWindow = 64;                     // bins ordered per pass
    __shared__ uint32_t cnt[kMaxBins];              // next free slot of each bin's segment
    __shared__ uint32_t hist[kWindow], lst[kWindow], gofs[kWindow];
    __shared__ uint32_t s_total;
    __shared__ uint32_t skey[kScatterThreads * 8];
    __shared__ Val sval[kScatterThreads * 8];
    typedef const __attribute__((address_space(4))) LevelConst *ConstLevels;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int L = a.n_levels;
    // Scans of the bins' totals, four bins per thread, in every workgroup:
    // the first slot of each bin's segment of this workgroup; workgroup 0
    // also stores the first record and the first accumulating workgroup
    // (ceil(total / kAccumRecords), at least one) of each bin, the list of
    // bins split over several workgroups and the records of the fullest bin.
    static_assert(kScatterThreads * 4 == kMaxBins, "four bins per thread");
    __shared__ uint32_t wtot[3][kScatterWaves];
    __shared__ uint32_t s_max;
    {
        const uint32_t *crow = a.counts + (int64_t)blockIdx.x * a.cstride;
        const int b0 = 4 * t;
        const uint4 tv = reinterpret_cast<const uint4 *>(a.totals)[t];
        const uint32_t tr[4] = {tv.x, tv.y, tv.z, tv.w};
        uint32_t tot[4], grp[4], spl[4], v[3] = {0u, 0u, 0u}, mx = 0u;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const bool in = b0 + i < a.n_bins;
            tot[i] = in ? tr[i] : 0u;
            grp[i] = in ? (tot[i] > kAccumRecords ? (tot[i] + kAccumRecords - 1) / kAccumRecords : 1u) : 0u;
            spl[i] = (in && tot[i] > kAccumRecords) ? 1u : 0u;
            v[0] += tot[i]; v[1] += grp[i]; v[2] += spl[i];
            mx = tot[i] > mx ? tot[i] : mx;
        }
        if (t == 0) s_max = 0u;
        uint32_t incl[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            incl[k] = wave_scan_incl(v[k], lane);
            if (lane == 63) wtot[k][wave] = incl[k];
        }
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t o = __shfl_xor(mx, d);
            mx = o > mx ? o : mx;
        }
        __syncthreads();
        if (lane == 0) atomicMax(&s_max, mx);
        uint32_t ex[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            uint32_t before = 0u;
            for (int u = 0; u < wave; ++u) before += wtot[k][u];
            ex[k] = before + incl[k] - v[k];
        }
        uint32_t s0 = ex[0], s1 = ex[1], s2 = ex[2];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int b = b0 + i;
            if (b < a.n_bins) cnt[b] = s0 + crow[b];
            s0 += tot[i];
            s1 += grp[i];
            if (blockIdx.x == 0 && b < a.n_bins) {
                a.bin_start[b + 1] = s0;
                a.work_start[b + 1] = s1;
                if (spl[i]) a.split[s2++] = (uint32_t)b;
            }
        }
        if (blockIdx.x == 0 && t == 0) {
            a.bin_start[0] = 0u;
            a.work_start[0] = 0u;
        }
        if (blockIdx.x == 0 && t == kScatterThreads - 1) a.split[a.n_bins] = s2;
    }
    if (t < kWindow) hist[t] = 0u;
    __syncthreads();
    if (blockIdx.x == 0 && t == 0) a.vmax[1] = s_max;
    const int64_t n_chunks = (a.n + 63) / 64;
    ConstLevels lvs = (ConstLevels)a.model;
    [[maybe_unused]] float rs = 1.0f;
    if constexpr (H16) {
        int e;
        (void)frexpf(u2f(a.vmax[0]), &e);
        rs = ldexpf(1.0f, 14 - e);
    }
    // the iteration count is uniform over the workgroup (barriers inside)
    for (int64_t g0 = (int64_t)blockIdx.x * kScatterWaves; g0 < n_chunks;
         g0 += (int64_t)gridDim.x * kScatterWaves) {
        const int64_t chunk = g0 + wave;
        const int64_t q0 = chunk * 64;
        const float2 *src = reinterpret_cast<const float2 *>(a.dx0) + q0 * L + lane;
        double p[3] = {a.lo[0], a.lo[1], a.lo[2]};
        const bool live = chunk < n_chunks && scatter_sample(a, q0 + lane, p);
        const bool sc = live && a.sflag[q0 + lane] != 0;   // else the records carry zeros
        // the next level's feature gradients are loaded while a level is ordered
        float2 gn = sc ? src[0] : make_float2(0.0f, 0.0f);
        for (int l = 0; l < L; ++l) {
            const float2 gg = gn;
            if (l + 1 < L) gn = sc ? src[(l + 1) * 64] : make_float2(0.0f, 0.0f);
            uint32_t idx[8];
            float w[8];
            level_corners(lvs[l], p, a.hash_mask, idx, w);
            const float g0v = gg.x * a.loss_scale, g1v = gg.y * a.loss_scale;
            const uint32_t off = lvs[l].off;
            const uint32_t size = lvs[l].dense ? lvs[l].s1 * lvs[l].s2 : a.hash_mask + 1u;
            const uint32_t fb = off >> kBinShift;                  // first bin of the level
            const uint32_t nlb = ((off + size - 1u) >> kBinShift) - fb + 1u;
            for (uint32_t w0 = 0; w0 < nlb; w0 += kWindow) {
                uint32_t rb[8], slot[8];
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    rb[c] = (idx[c] >> kBinShift) - fb - w0;      // >= kWindow (wrapped) outside the window
                    slot[c] = (live && rb[c] < (uint32_t)kWindow) ? atomicAdd(&hist[rb[c]], 1u) : ~0u;
                }
                __syncthreads();
                if (wave == 0) {
                    // runs of the window's bins: a bin with records is a bin of
                    // this level, so its cursor exists; one lane per bin
                    const uint32_t nb = hist[lane];
                    const uint32_t incl = wave_scan_incl(nb, lane);
                    uint32_t base = 0u;
                    if (nb) {
                        base = cnt[fb + w0 + lane];
                        cnt[fb + w0 + lane] = base + nb;
                    }
                    lst[lane] = incl - nb;
                    gofs[lane] = base - (incl - nb);   // slot of staged record k: gofs[bin] + k
                    hist[lane] = 0u;
                    if (lane == 63) s_total = incl;
                }
                __syncthreads();
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    if (slot[c] == ~0u) continue;
                    const float v0 = w[c] * g0v, v1 = w[c] * g1v;
                    const uint32_t k = lst[rb[c]] + slot[c];
                    skey[k] = (rb[c] << 16) | (idx[c] & (kBinEntries - 1));
                    if constexpr (H16) sval[k] = Prec<NIV_FP16>::pack(v0 * rs, v1 * rs);
                    else sval[k] = make_uint2(f2u(v0), f2u(v1));
                }
                __syncthreads();
                const uint32_t total = s_total;
                for (uint32_t k = t; k < total; k += kScatterThreads) {
                    const uint32_t key = skey[k];
                    const Val v = sval[k];
                    const uint32_t dst = gofs[key >> 16] + k;
                    a.keys[dst] = (uint16_t)(key & 0xFFFFu);
                    if constexpr (H16) a.vals16[dst] = v;
                    else a.vals[dst] = make_float2(u2f(v.x), u2f(v.y));
                }
                __syncthreads();   // the stage and the window's arrays are reused
            }
        }
    }
}

// Exclusive scans of the workgroups' counts of each bin, in place: workgroup
// i of this kernel takes bins 4 i .. 4 i + 3 and thread t the counts of
// workgroup t (one 16-byte piece of its row); the bins' totals go to
// totals[b].
__global__ __launch_bounds__(kScatterBlocks) void k_grid_scan_bins(const ScatterArgs a)
{
    constexpr int kW = kScatterBlocks / 64;
    __shared__ uint32_t wsum[4][kW];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int b0 = 4 * blockIdx.x;
    uint4 *row = reinterpret_cast<uint4 *>(a.counts + (int64_t)t * a.cstride + b0);
    const uint4 v = *row;
    const uint32_t c[4] = {v.x, v.y, v.z, v.w};
    uint32_t incl[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        incl[k] = wave_scan_incl(c[k], lane);
        if (lane == 63) wsum[k][wv] = incl[k];
    }
    __syncthreads();
    uint32_t ex[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        // totals of the waves before this one: lane u < wv holds wave u's,
        // summed over the whole wave
        uint32_t before = lane < wv ? wsum[k][lane] : 0u;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) before += __shfl_xor(before, d);
        ex[k] = before + incl[k] - c[k];
    }
    *row = make_uint4(ex[0], ex[1], ex[2], ex[3]);
    if (t < 4 && b0 + t < a.n_bins) {
        uint32_t total = 0u;
        for (int u = 0; u < kW; ++u) total += wsum[t][u];
        a.totals[b0 + t] = total;
    }
}

// Scale of the step's fixed-point sums: with M the largest |contribution| <
// 2^e and at most 2^c records in any bin, a value v becomes round(v 2^s),
// s = 62 - c - e, so every term is at most 2^(62-c) and every sum over a bin
// (whole, or any part of it) at most 2^62: no overflow in 64 bits, and each
// term is resolved to 2^(-62+c) M.
__device__ inline int fixed_shift(const uint32_t *vmax)
{
    int e;
    (void)frexpf(u2f(vmax[0]), &e);            // M < 2^e (M = 0 gives e = 0: all terms are zero)
    const uint32_t n = vmax[1];
    const int c = n > 1u ? 32 - __builtin_clz(n - 1u) : 0;   // n <= 2^c
    return 62 - c - e;
}

// Accumulation: the records of bin b are split over work_start[b+1] -
// work_start[b] workgroups of at most kAccumRecords records.  Each sums its
// share in LDS in 64-bit fixed point at the step's scale (fixed_shift; LDS
// integer atomics run far faster than LDS float atomics here, and integer
// sums do not depend on the order).  A bin taken by one workgroup is stored
// as is (every entry, zeros included); a shared bin (the coarse dense
// levels) stores each part's integer sums, which k_grid_merge adds.
template <bool H16>
__global__ __launch_bounds__(1024) void k_grid_accum(const ScatterArgs a)
{
    __shared__ unsigned long long acc[2 * kBinEntries];
    __shared__ int s_bin;
    const uint32_t w = blockIdx.x;
    if (w >= a.work_start[a.n_bins]) return;   // uniform over the workgroup
    if (threadIdx.x == 0) {                    // bin of this workgroup: last b with work_start[b] <= w
        int lo = 0, hi = a.n_bins - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.work_start[mid] <= w) lo = mid; else hi = mid - 1;
        }
        s_bin = lo;
    }
    for (int k = threadIdx.x; k < 2 * kBinEntries; k += 1024) acc[k] = 0ull;
    __syncthreads();
    const int b = s_bin;
    const uint32_t parts = a.work_start[b + 1] - a.work_start[b];
    const uint32_t part = w - a.work_start[b];
    const uint32_t b0 = a.bin_start[b], b1 = a.bin_start[b + 1];
    const uint32_t r0 = b0 + part * (uint32_t)kAccumRecords;
    const uint32_t r1 = parts == 1 ? b1 : (r0 + kAccumRecords < b1 ? r0 + kAccumRecords : b1);
    const int sh = fixed_shift(a.vmax);
    const double down = ldexp(1.0, -sh);
    double up = ldexp(1.0, sh);
    if constexpr (H16) {   // records hold v 2^(14 - e)
        int e;
        (void)frexpf(u2f(a.vmax[0]), &e);
        up = ldexp(1.0, sh - (14 - e));
    }
    auto fx = [&](float v) { return (unsigned long long)(long long)__builtin_rint((double)v * up); };
    auto val = [&](uint32_t r) -> float2 {
        if constexpr (H16) {
            const f2 h = Prec<NIV_FP16>::unpack(a.vals16[r]);
            return make_float2(h.x, h.y);
        } else {
            return a.vals[r];
        }
    };
    uint32_t r = r0 + threadIdx.x;
    // eight records per thread in flight before the LDS adds
    for (; r + 7 * 1024 < r1; r += 8 * 1024) {
        uint32_t i[8];
        float2 v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            i[k] = a.keys[r + k * 1024];
            v[k] = val(r + k * 1024);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            atomicAdd(&acc[2 * i[k]], fx(v[k].x));
            atomicAdd(&acc[2 * i[k] + 1], fx(v[k].y));
        }
    }
    for (; r < r1; r += 1024) {
        const uint32_t i = a.keys[r];
        const float2 v = val(r);
        atomicAdd(&acc[2 * i], fx(v.x));
        atomicAdd(&acc[2 * i + 1], fx(v.y));
    }
    __syncthreads();
    const int64_t e0 = (int64_t)b << kBinShift;
    if (parts > 1) {
        long long *dst = a.parts + (int64_t)w * (2 * kBinEntries);
        for (int k = threadIdx.x; k < 2 * kBinEntries; k += 1024) dst[k] = (long long)acc[k];
        return;
    }
    for (int k = threadIdx.x; k < 2 * kBinEntries; k += 1024) {
        const int64_t en = e0 + (k >> 1);
        if (en >= a.n_entries) continue;
        a.grads[2 * en + (k & 1)] = (float)((double)(long long)acc[k] * down);
    }
}

// Bins split over several workgroups: their parts' integer sums added, then
// scaled once.  Job (i, s) takes values 256 s .. 256 s + 255
// of the i-th split bin; a grid of at most kMergeBlocks workgroups walks the
// step's jobs.
constexpr int kMergeSlices = 2 * kBinEntries / 256;
constexpr int kMergeBlocks = 512;
__global__ __launch_bounds__(256) void k_grid_merge(const ScatterArgs a)
{
    const uint32_t jobs = a.split[a.n_bins] * (uint32_t)kMergeSlices;
    const double down = ldexp(1.0, -fixed_shift(a.vmax));
    for (uint32_t job = blockIdx.x; job < jobs; job += gridDim.x) {
        const int b = (int)a.split[job / kMergeSlices];
        const int k = (int)(job % kMergeSlices) * 256 + threadIdx.x;
        const uint32_t w0 = a.work_start[b], parts = a.work_start[b + 1] - w0;
        const int64_t en = ((int64_t)b << kBinShift) + (k >> 1);
        if (en >= a.n_entries) continue;
        const long long *src = a.parts + (int64_t)w0 * (2 * kBinEntries) + k;
        // integer sums: any order gives the same value, so the parts' loads
        // go out eight at a time
        long long sum = 0;
        uint32_t q = 0;
        for (; q + 8 <= parts; q += 8) {
            long long v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = src[(int64_t)(q + u) * (2 * kBinEntries)];
#pragma unroll
            for (int u = 0; u < 8; ++u) sum += v[u];
        }
        for (; q < parts; ++q) sum += src[(int64_t)q * (2 * kBinEntries)];
        a.grads[2 * en + (k & 1)] = (float)((double)sum * down);
    }
}

// ---------------------------------------------------------------- Adam
// Kingma & Ba, Algorithm 1, applied to every parameter; bc1 = 1 - beta1^t,
// bc2 = 1 - beta2^t.
// With `status` given (a training step), nothing is updated when the step's
// loss or gradient was not finite (status[2] set by the forward pass).
// With grid_out given, grid values k < n_grid are also stored, rounded to the
// model's precision (GP), into the prepared model's grid (the training step
// then rebuilds only the weight operands).
template <int GP>
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ gr, float *__restrict__ m,
                       float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float bc1, float bc2, const uint32_t *status, uint8_t *__restrict__ grid_out,
                       int64_t n_grid)
{
    if (status && status[2] != 0u) return;
    auto step = [&](float pv, float g, float mv, float vv, float &mk, float &vk) {
        mk = b1 * mv + (1.0f - b1) * g;
        vk = b2 * vv + (1.0f - b2) * g * g;
        return pv - lr * (mk / bc1) / (sqrtf(vk / bc2) + eps);
    };
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // four values per thread and iteration (16-byte accesses) where every
    // pointer is 16-byte aligned
    const bool vec = ((reinterpret_cast<uintptr_t>(p) | reinterpret_cast<uintptr_t>(gr) |
                       reinterpret_cast<uintptr_t>(m) | reinterpret_cast<uintptr_t>(v) |
                       reinterpret_cast<uintptr_t>(grid_out)) & 15u) == 0;
    int64_t k0 = 0;
    if (vec) {
        const int64_t n4 = n / 4;
        for (int64_t i = tid; i < n4; i += stride) {
            const f4 pv = reinterpret_cast<const f4 *>(p)[i], g = reinterpret_cast<const f4 *>(gr)[i];
            const f4 mv = reinterpret_cast<const f4 *>(m)[i], vv = reinterpret_cast<const f4 *>(v)[i];
            float mk4[4], vk4[4], pk4[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) pk4[c] = step(pv[c], g[c], mv[c], vv[c], mk4[c], vk4[c]);
            const f4 mk = {mk4[0], mk4[1], mk4[2], mk4[3]}, vk = {vk4[0], vk4[1], vk4[2], vk4[3]};
            const f4 pk = {pk4[0], pk4[1], pk4[2], pk4[3]};
            reinterpret_cast<f4 *>(m)[i] = mk;
            reinterpret_cast<f4 *>(v)[i] = vk;
            reinterpret_cast<f4 *>(p)[i] = pk;
            if (grid_out && 4 * i + 4 > n_grid && 4 * i < n_grid) {   // the group the grid ends in
                const float e[4] = {pk.x, pk.y, pk.z, pk.w};
                for (int c = 0; 4 * i + c < n_grid; ++c) {
                    if constexpr (GP == NIV_FP32) reinterpret_cast<float *>(grid_out)[4 * i + c] = e[c];
                    else reinterpret_cast<_Float16 *>(grid_out)[4 * i + c] = (_Float16)e[c];
                }
            } else if (grid_out && 4 * i < n_grid) {
                if constexpr (GP == NIV_FP32) {
                    reinterpret_cast<f4 *>(grid_out)[i] = pk;
                } else {
                    const h2 a = __builtin_convertvector((f2){pk.x, pk.y}, h2);
                    const h2 b = __builtin_convertvector((f2){pk.z, pk.w}, h2);
                    reinterpret_cast<u2 *>(grid_out)[i] =
                        (u2){__builtin_bit_cast(uint32_t, a), __builtin_bit_cast(uint32_t, b)};
                }
            }
        }
        k0 = n4 * 4;
    }
    for (int64_t k = k0 + tid; k < n; k += stride) {
        float mk, vk;
        const float pk = step(p[k], gr[k], m[k], v[k], mk, vk);
        m[k] = mk;
        v[k] = vk;
        p[k] = pk;
        if (grid_out && k < n_grid) {
            if constexpr (GP == NIV_FP32) reinterpret_cast<float *>(grid_out)[k] = pk;
            else reinterpret_cast<_Float16 *>(grid_out)[k] = (_Float16)pk;
        }
    }
}

// ---------------------------------------------------------------- initial parameters
// Seeded start of training: grid values uniform on [lo, hi), weights of
// matrix m uniform on [-a_m, a_m), a_m = sqrt(6 / (fan_in + fan_out))
// (Xavier-uniform).  Parameter k takes uniform number 0 of the generator
// stream (seed, k, 0, 3): Philox4x64-10, counter (k, 0, 0, 3), key (seed, 0),
// the low 32 bits of word 0 cut to 24.  FP64 arithmetic, one rounding to FP32.
struct InitArgs {
    float *params;
    int64_t n_grid, n;
    int32_t n_mats;
    int64_t mat_end[kMaxMats];
    double scale[kMaxMats];
    double lo, width;
    uint64_t seed;
};

__global__ void k_init_params(const InitArgs a)
{
#pragma clang fp contract(off)
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; k < a.n; k += stride) {
        uint64_t w[4] = {(uint64_t)k, 0ull, 0ull, 3ull};
        philox4x64_10(w, a.seed, 0);
        const double u = (double)((uint32_t)w[0] >> 8) * 0x1p-24;
        double v;
        if (k < a.n_grid) {
            v = __builtin_fma(a.width, u, a.lo);
        } else {
            int m = 0;
            while (m + 1 < a.n_mats && k >= a.mat_end[m]) ++m;
            v = a.scale[m] * (2.0 * u - 1.0);
        }
        a.params[k] = (float)v;
    }
}

// ---------------------------------------------------------------- host side
struct TrainLayout {
    int64_t bwd_off, x_off, mask_off, dE_off, dx0_off, sflag_off, counts_off, tot_off, start_off, work_off,
        split_off, vmax_off, keys_off, vals_off, dw_off, parts_off, total;
};

// Accumulating workgroups of a step: at most one per bin plus one per
// kAccumRecords records (the launch takes this many; the excess ones return
// at once).
static int64_t acc_group_bound(int64_t n, int n_levels, int64_t n_bins)
{
    const int64_t records = n * (int64_t)n_levels * 8;
    return n_bins + (records + kAccumRecords - 1) / kAccumRecords;
}

static int64_t grid_bins(const Model &m)
{
    return (m.n_grid_values / 2 + kBinEntries - 1) >> kBinShift;
}

template <int P, class S> TrainLayout train_layout_t(int64_t n, int64_t n_bins)
{
    using B = Bwd<P, S>;
    const int64_t nc = (n + 63) / 64;
    TrainLayout L;
    L.vmax_off = 0;   // step words first, at a fixed place (see kStatusWords)
    L.bwd_off = 256;
    L.x_off = L.bwd_off + align256(B::BYTES);
    L.mask_off = L.x_off + align256(nc * B::CHUNK_BYTES);
    L.dE_off = L.mask_off + align256(nc * S::H * (S::W / 32) * 64 * 4);
    L.dx0_off = L.dE_off + align256(n * 3 * 4);
    L.sflag_off = L.dx0_off + align256((n + 63) / 64 * 64 * 2 * S::L * 4);
    L.counts_off = L.sflag_off + align256(n);
    L.tot_off = L.counts_off + align256((int64_t)kMaxBins * kScatterBlocks * 4);
    L.start_off = L.tot_off + align256(kMaxBins * 4);
    L.work_off = L.start_off + align256((kMaxBins + 1) * 4);
    L.split_off = L.work_off + align256((kMaxBins + 1) * 4);
    L.keys_off = L.split_off + align256((kMaxBins + 1) * 4);
    const int64_t records = n * S::L * 8;
    L.vals_off = L.keys_off + align256(records * 2);
    L.dw_off = L.vals_off + align256(records * (B::F32 ? 8 : 4));   // FP32 pairs or scaled FP16 pairs
    // one weight-gradient row per backward wave: 4 per workgroup, at most
    // one workgroup per 4 chunks and kBwdMaxBlocks in all
    const int64_t bwd_blocks = std::min<int64_t>(kBwdMaxBlocks, std::max<int64_t>(1, (nc + 3) / 4));
    L.parts_off = L.dw_off + align256(bwd_blocks * Bwd<P, S>::NMLP * 4);
    // fixed-point partial sums: one row per accumulating workgroup
    L.total = L.parts_off + align256(acc_group_bound(n, S::L, n_bins) * 2 * kBinEntries * 8);
    return L;
}

// A second stream per device for work that runs beside the caller's stream
// (created once, default priority, kept until the process ends), and the
// two events of one fork and join (released when the call returns; an event
// still pending is released once it completes).
static std::mutex g_side_mu;
static hipStream_t g_side[64];
static hipError_t side_stream(hipStream_t *out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_side_mu);
    if (!g_side[dev] && (e = hipStreamCreateWithFlags(&g_side[dev], hipStreamNonBlocking)) != hipSuccess)
        return e;
    *out = g_side[dev];
    return hipSuccess;
}
struct SideFork {
    hipEvent_t fork = nullptr, join = nullptr;
    hipError_t create()
    {
        hipError_t e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
        return e != hipSuccess ? e : hipEventCreateWithFlags(&join, hipEventDisableTiming);
    }
    ~SideFork()
    {
        if (fork) (void)hipEventDestroy(fork);
        if (join) (void)hipEventDestroy(join);
    }
};

template <int P, class S>
static hipError_t backward_t(const Model &m, const niv_batch &b, const niv_train_state &st,
                             hipStream_t stream)
{
    using B = Bwd<P, S>;
    using O = Ops<P, S>;
    TrainLayout L = train_layout_t<P, S>(b.count, grid_bins(m));
    uint8_t *ws = static_cast<uint8_t *>(st.workspace);
    if (m.n_params - m.n_grid_values != B::NMLP) return hipErrorInvalidValue;   // shape mismatch
    // the loss and the step's words are cleared by kernels, so the step can be
    // captured; every gradient value is stored whole (the grid by the
    // accumulating and merging passes, the MLP by k_dw_sum)
    uint32_t *status = reinterpret_cast<uint32_t *>(ws + L.vmax_off);
    hipLaunchKernelGGL((k_prepare_bwd<P, S>), dim3((B::N_OPS * 64 + 255) / 256), dim3(256), 0,
                       stream, st.params, ws + L.bwd_off, m.n_grid_values, status, kStatusWords,
                       st.loss);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // 1. forward with saves, loss and d loss / dE (non-finite ones mark the step)
    QueryArgs a;
    memset(&a, 0, sizeof(a));
    a.n_frames = 1;
    a.f[0].pos = b.x;
    a.f[0].nrm = b.nrm;
    a.f[0].model = static_cast<const uint8_t *>(st.model);
    a.f[0].count = b.count;
    a.f[0].tile_begin = 0;
    a.grid_off = (uint64_t)op_layout(m.kind, (niv_precision)P).grid_off;
    a.grid_bytes = (uint32_t)(m.n_grid_values * (P == NIV_FP32 ? 4 : 2));
    a.hash_mask = (uint32_t)((int64_t(1) << m.cfg.log2_T) - 1);
    for (int c = 0; c < 3; ++c) {
        a.lo[c] = m.cfg.aabb_min[c];
        a.hi[c] = m.cfg.aabb_max[c];
    }
    a.extra_ps = b.extra;
    a.target = b.target;
    a.valid = b.valid;
    a.x_save = ws + L.x_off;
    a.mask_save = reinterpret_cast<uint32_t *>(ws + L.mask_off);
    a.dE = reinterpret_cast<float *>(ws + L.dE_off);
    a.loss = st.loss;
    a.train_status = status;
    a.loss_scale = (float)(1.0 / (3.0 * (double)b.count));  // used by the forward's loss sum
    a.loss_eps = 0.01f;
    // grid scatter arguments
    ScatterArgs sa;
    memset(&sa, 0, sizeof(sa));
    sa.x = b.x;
    sa.dx0 = reinterpret_cast<const float *>(ws + L.dx0_off);
    sa.sflag = ws + L.sflag_off;
    sa.valid = b.valid;
    sa.model = static_cast<const uint8_t *>(st.model);
    sa.counts = reinterpret_cast<uint32_t *>(ws + L.counts_off);
    sa.totals = reinterpret_cast<uint32_t *>(ws + L.tot_off);
    sa.bin_start = reinterpret_cast<uint32_t *>(ws + L.start_off);
    sa.work_start = reinterpret_cast<uint32_t *>(ws + L.work_off);
    sa.split = reinterpret_cast<uint32_t *>(ws + L.split_off);
    sa.vmax = status;
    sa.parts = reinterpret_cast<long long *>(ws + L.parts_off);
    sa.keys = reinterpret_cast<uint16_t *>(ws + L.keys_off);
    sa.vals = reinterpret_cast<float2 *>(ws + L.vals_off);
    sa.vals16 = reinterpret_cast<uint32_t *>(ws + L.vals_off);
    sa.grads = st.grads;
    sa.n = b.count;
    sa.n_entries = m.n_grid_values / 2;
    sa.n_levels = m.cfg.n_levels;
    sa.n_bins = (int32_t)((sa.n_entries + kBinEntries - 1) >> kBinShift);
    sa.hash_mask = a.hash_mask;
    sa.loss_scale = (float)(1.0 / (3.0 * (double)b.count));
    for (int c = 0; c < 3; ++c) { sa.lo[c] = a.lo[c]; sa.hi[c] = a.hi[c]; }
    sa.cstride = (sa.n_bins + 3) & ~3;
    if (sa.n_bins > kMaxBins) return hipErrorInvalidValue;
    if (sa.n_levels > kScatterMaxLevels) return hipErrorInvalidValue;
    // the count pass reads only the batch and the level table: it runs on a
    // second stream beside the forward (an event fork and join with the
    // caller's stream; both at the default priority)
    SideFork ev;
    hipStream_t side = nullptr;
    if ((e = side_stream(&side)) != hipSuccess) return e;
    if ((e = ev.create()) != hipSuccess) return e;
    if ((e = hipEventRecord(ev.fork, stream)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(side, ev.fork, 0)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_grid_count, dim3(kScatterBlocks), dim3(kScatterThreads), 0, side, sa);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipEventRecord(ev.join, side)) != hipSuccess) return e;
    // FP16: grid level 0, when dense and at most kL0Words entries, is read
    // from LDS (its random-sample gathers would touch a line per lane)
    if (P == NIV_FP16 && m.cfg.n_levels > 0 && m.dense[0] && m.size[0] <= kL0Words) {
        a.l0_words = (uint32_t)m.size[0];
        a.l0_off = (uint32_t)m.offset[0];
    }
    {
        constexpr int kBlock = 256, kWavesPerBlock = 4;
        auto kern = k_query<P, S, true, 4, true, kBlock>;
        const size_t lds = O::W_BYTES + (size_t)kWavesPerBlock * 64 * O::ROW_DW * 4 +
                           (P == NIV_FP16 ? (size_t)kL0Words * 4 : 0);
        static int max_blocks = -1, n_cu = 0;
        if (max_blocks < 0) {
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            int dev = 0;
            if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
            if ((e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
                return e;
            int nb = 0;
            if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, kBlock, lds)) != hipSuccess)
                return e;
            max_blocks = nb > 0 ? nb : 1;
        }
        const int64_t n_chunks = (b.count + 63) / 64;
        a.n_tiles = (n_chunks + kWavesPerBlock - 1) / kWavesPerBlock;
        int64_t blocks = a.n_tiles < (int64_t)max_blocks * n_cu ? a.n_tiles : (int64_t)max_blocks * n_cu;
        hipLaunchKernelGGL(kern, dim3((unsigned)(blocks < 1 ? 1 : blocks)), dim3(kBlock), lds, stream, a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // 2. backward
    BwdArgs ba;
    memset(&ba, 0, sizeof(ba));
    ba.bwd = ws + L.bwd_off;
    ba.x_save = ws + L.x_off;
    ba.mask_save = reinterpret_cast<const uint32_t *>(ws + L.mask_off);
    ba.dE = reinterpret_cast<const float *>(ws + L.dE_off);
    ba.x = b.x;
    ba.model = static_cast<const uint8_t *>(st.model);
    const float loss_scale = (float)(1.0 / (3.0 * (double)b.count));
    ba.grads = st.grads;
    ba.dw_part = reinterpret_cast<float *>(ws + L.dw_off);
    ba.dx0 = reinterpret_cast<float *>(ws + L.dx0_off);
    ba.sflag = ws + L.sflag_off;
    ba.vmax = status;
    ba.n = b.count;
    ba.n_grid = m.n_grid_values;
    ba.loss_scale = loss_scale;
    ba.hash_mask = a.hash_mask;
    for (int c = 0; c < 3; ++c) { ba.lo[c] = a.lo[c]; ba.hi[c] = a.hi[c]; }
    {
        auto kern = k_train_bwd<P, S>;
        const size_t lds = (size_t)B::LDS_BYTES;
        static int max_blocks = -1, n_cu = 0;
        if (max_blocks < 0) {
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            int dev = 0;
            if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
            if ((e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
                return e;
            int nb = 0;
            if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, 256, lds)) != hipSuccess)
                return e;
            max_blocks = nb > 0 ? nb : 1;
        }
        const int64_t n_chunks = (b.count + 63) / 64;
        int64_t blocks = (n_chunks + 3) / 4;
        blocks = blocks < (int64_t)max_blocks * n_cu ? blocks : (int64_t)max_blocks * n_cu;
        blocks = blocks < kBwdMaxBlocks ? blocks : kBwdMaxBlocks;
        blocks = blocks < 1 ? 1 : blocks;
        hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), lds, stream, ba);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // weight gradient: the workgroups' rows summed, one row per workgroup
        hipLaunchKernelGGL(k_dw_sum, dim3((unsigned)((B::NMLP + 15) / 16)), dim3(256), 0, stream, ba.dw_part,
                           (int64_t)B::NMLP, (int)blocks, st.grads + m.n_grid_values, ba.loss_scale);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // 3. grid scatter through bins (counted beside the forward, above)
    if ((e = hipStreamWaitEvent(stream, ev.join, 0)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_grid_scan_bins, dim3(sa.cstride / 4), dim3(kScatterBlocks), 0, stream, sa);
    constexpr bool H16 = !B::F32;
    hipLaunchKernelGGL(k_grid_write<H16>, dim3(kScatterBlocks), dim3(kScatterThreads), 0, stream, sa);
    const int64_t acc_groups = acc_group_bound(b.count, m.cfg.n_levels, sa.n_bins);
    hipLaunchKernelGGL(k_grid_accum<H16>, dim3((unsigned)acc_groups), dim3(1024), 0, stream, sa);
    // a split bin holds more than kAccumRecords records
    const int64_t records = b.count * (int64_t)m.cfg.n_levels * 8;
    const int64_t max_split = std::min<int64_t>(sa.n_bins, records / (kAccumRecords + 1));
    if (max_split > 0)
        hipLaunchKernelGGL(k_grid_merge, dim3((unsigned)std::min<int64_t>(max_split * kMergeSlices, kMergeBlocks)),
                           dim3(256), 0, stream, sa);
    return hipGetLastError();
}

static int64_t train_bytes(const Model &m, niv_precision prec, int64_t n)
{
    if (m.kind == kUnitCube)
        return prec == NIV_FP32 ? train_layout_t<NIV_FP32, ShapeUnitCube>(n, grid_bins(m)).total
                                : train_layout_t<NIV_FP16, ShapeUnitCube>(n, grid_bins(m)).total;
    if (m.kind == kRoom6D)
        return prec == NIV_FP32 ? train_layout_t<NIV_FP32, ShapeRoom6D>(n, grid_bins(m)).total
                                : train_layout_t<NIV_FP16, ShapeRoom6D>(n, grid_bins(m)).total;
    return prec == NIV_FP32 ? train_layout_t<NIV_FP32, ShapeRoom>(n, grid_bins(m)).total
                            : train_layout_t<NIV_FP16, ShapeRoom>(n, grid_bins(m)).total;
}

}  // namespace niv

using namespace niv;

namespace {
niv_status hst(hipError_t e) { return e == hipSuccess ? NIV_OK : NIV_ERR_HIP; }
bool al(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }
bool trainable(const Model &m) { return m.kind == kUnitCube || m.kind == kRoom || m.kind == kRoom6D; }
}  // namespace

extern "C" {

niv_status niv_train_sizes(const niv_handle *h, niv_precision prec, int64_t max_batch,
                           int64_t *workspace_bytes)
{
    if (!h || !workspace_bytes || max_batch < 1 || max_batch > (int64_t(1) << 24)) return NIV_ERR_INVALID_ARG;
    if (prec != NIV_FP32 && prec != NIV_FP16) return prec == NIV_BF16 ? NIV_ERR_UNSUPPORTED : NIV_ERR_INVALID_ARG;
    if (!trainable(h->m)) return NIV_ERR_UNSUPPORTED;
    *workspace_bytes = train_bytes(h->m, prec, max_batch);
    return NIV_OK;
}

niv_status niv_backward(niv_handle *h, const niv_batch *b, const niv_train_state *st,
                        niv_precision prec, hipStream_t stream)
{
    if (!h || !b || !st) return NIV_ERR_INVALID_ARG;
    if (prec != NIV_FP32 && prec != NIV_FP16) return prec == NIV_BF16 ? NIV_ERR_UNSUPPORTED : NIV_ERR_INVALID_ARG;
    if (!trainable(h->m)) return NIV_ERR_UNSUPPORTED;
    // the grid scatter indexes its 8 x levels contributions per sample with 32 bits
    if (b->count < 1 || b->count > (int64_t(1) << 24)) return NIV_ERR_INVALID_ARG;
    if (!b->x || !b->nrm || !b->target || (h->m.cfg.n_extra > 0 && !b->extra)) return NIV_ERR_INVALID_ARG;
    if (!st->params || !st->grads || !st->model || !st->workspace || !st->loss) return NIV_ERR_INVALID_ARG;
    if (!al(st->model, 256) || !al(st->workspace, 256) || !al(st->params, 4) || !al(st->grads, 4))
        return NIV_ERR_INVALID_ARG;
    if (st->workspace_bytes < train_bytes(h->m, prec, b->count)) return NIV_ERR_WORKSPACE;
    const Model &m = h->m;
    hipError_t e;
    if (m.kind == kUnitCube)
        e = prec == NIV_FP32 ? backward_t<NIV_FP32, ShapeUnitCube>(m, *b, *st, stream)
                             : backward_t<NIV_FP16, ShapeUnitCube>(m, *b, *st, stream);
    else if (m.kind == kRoom6D)
        e = prec == NIV_FP32 ? backward_t<NIV_FP32, ShapeRoom6D>(m, *b, *st, stream)
                             : backward_t<NIV_FP16, ShapeRoom6D>(m, *b, *st, stream);
    else
        e = prec == NIV_FP32 ? backward_t<NIV_FP32, ShapeRoom>(m, *b, *st, stream)
                             : backward_t<NIV_FP16, ShapeRoom>(m, *b, *st, stream);
    return hst(e);
}

static niv_status check_adam(const niv_train_state *st, const niv_adam *ad)
{
    if (!st || !ad || !st->params || !st->grads || !st->adam_m || !st->adam_v)
        return NIV_ERR_INVALID_ARG;
    if (ad->step < 1 || !(ad->lr >= 0.f) || !(ad->beta1 >= 0.f && ad->beta1 < 1.f) ||
        !(ad->beta2 >= 0.f && ad->beta2 < 1.f) || !(ad->eps > 0.f))
        return NIV_ERR_INVALID_ARG;
    return NIV_OK;
}

static niv_status adam_launch(const Model &m, const niv_train_state *st, const niv_adam *ad,
                              const uint32_t *status, uint8_t *grid_out, niv_precision prec,
                              hipStream_t stream)
{
    const double bc1 = 1.0 - pow((double)ad->beta1, (double)ad->step);
    const double bc2 = 1.0 - pow((double)ad->beta2, (double)ad->step);
    // one group of four values per thread (up to 2^22 groups; more loop)
    const int64_t groups = (m.n_params + 3) / 4;
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((groups + 255) / 256, 16384));
    if (prec == NIV_FP32)
        hipLaunchKernelGGL(k_adam<NIV_FP32>, dim3(blocks), dim3(256), 0, stream, st->params, st->grads,
                           st->adam_m, st->adam_v, m.n_params, ad->lr, ad->beta1, ad->beta2, ad->eps,
                           (float)bc1, (float)bc2, status, grid_out, m.n_grid_values);
    else
        hipLaunchKernelGGL(k_adam<NIV_FP16>, dim3(blocks), dim3(256), 0, stream, st->params, st->grads,
                           st->adam_m, st->adam_v, m.n_params, ad->lr, ad->beta1, ad->beta2, ad->eps,
                           (float)bc1, (float)bc2, status, grid_out, m.n_grid_values);
    return hst(hipGetLastError());
}

niv_status niv_adam_update(niv_handle *h, const niv_train_state *st, const niv_adam *ad,
                           hipStream_t stream)
{
    if (!h) return NIV_ERR_INVALID_ARG;
    niv_status s = check_adam(st, ad);
    if (s != NIV_OK) return s;
    return adam_launch(h->m, st, ad, nullptr, nullptr, NIV_FP32, stream);
}

niv_status niv_train_step(niv_handle *h, const niv_batch *b, const niv_train_state *st,
                          const niv_adam *ad, niv_precision prec, hipStream_t stream)
{
    if (!h) return NIV_ERR_INVALID_ARG;
    niv_status s = check_adam(st, ad);
    if (s != NIV_OK) return s;
    s = niv_backward(h, b, st, prec, stream);
    if (s != NIV_OK) return s;
    // the update reads the step's non-finite word and does nothing when it is
    // set; it stores the new grid into the prepared model, whose level table
    // never changes, so only the weight operands are rebuilt
    uint8_t *grid_out = static_cast<uint8_t *>(st->model) + op_layout(h->m.kind, prec).grid_off;
    s = adam_launch(h->m, st, ad, static_cast<const uint32_t *>(st->workspace), grid_out, prec, stream);
    if (s != NIV_OK) return s;
    return hst(launch_prepare_operands(h->m, st->params, st->model, prec, stream));
}

niv_status niv_train_status(const niv_train_state *st, hipStream_t stream)
{
    if (!st || !st->workspace || !al(st->workspace, 256)) return NIV_ERR_INVALID_ARG;
    uint32_t words[kStatusWords] = {0u, 0u, 0u, 0u};
    if (hipMemcpyAsync(words, st->workspace, sizeof(words), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return NIV_ERR_HIP;
    return words[2] ? NIV_ERR_NONFINITE : NIV_OK;
}

niv_status niv_lr_schedule(int64_t step, int64_t hold_steps, int64_t total_steps, double lr0,
                           double lr1, double *lr)
{
    if (!lr || step < 1 || hold_steps < 0 || total_steps < 1 || !(lr0 > 0.0) || !(lr1 > 0.0) ||
        !isfinite(lr0) || !isfinite(lr1))
        return NIV_ERR_INVALID_ARG;
    if (step <= hold_steps || total_steps <= hold_steps) {
        *lr = lr0;
        return NIV_OK;
    }
    double t = (double)(step - hold_steps) / (double)(total_steps - hold_steps);
    t = t < 1.0 ? t : 1.0;
    *lr = lr0 * pow(lr1 / lr0, t);
    return NIV_OK;
}

niv_status niv_init_params(niv_handle *h, float *params, uint64_t seed, float grid_lo, float grid_hi,
                           hipStream_t stream)
{
    if (!h || !params || !al(params, 4) || !isfinite(grid_lo) || !isfinite(grid_hi) ||
        !(grid_hi >= grid_lo))
        return NIV_ERR_INVALID_ARG;
    const niv_config &c = h->m.cfg;
    const int n_mats = c.n_hidden + 1;
    if (n_mats > kMaxMats) return NIV_ERR_UNSUPPORTED;
    InitArgs a;
    memset(&a, 0, sizeof(a));
    a.params = params;
    a.n_grid = h->m.n_grid_values;
    a.n = h->m.n_params;
    a.n_mats = n_mats;
    int64_t end = a.n_grid;
    for (int k = 0; k < n_mats; ++k) {
        const int64_t fan_in = k == 0 ? h->m.din : c.width;
        const int64_t fan_out = k == n_mats - 1 ? c.n_out : c.width;
        end += fan_in * fan_out;
        a.mat_end[k] = end;
        a.scale[k] = sqrt(6.0 / (double)(fan_in + fan_out));
    }
    a.lo = (double)grid_lo;
    a.width = (double)grid_hi - (double)grid_lo;
    a.seed = seed;
    hipLaunchKernelGGL(k_init_params, dim3(1024), dim3(256), 0, stream, a);
    return hst(hipGetLastError());
}

}  // extern "C"
