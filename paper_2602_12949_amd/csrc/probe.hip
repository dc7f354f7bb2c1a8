// Measurement kernels: gather rates of the texture path for the access
// patterns of the encoding (the query's ceilings are read against them).
// One pass reads n x 128 four-byte words, 8 per level of 16 levels.
#include <hip/hip_runtime.h>

#include "niv_internal.h"

namespace niv {
namespace {

__device__ inline uint32_t mix32(uint32_t x)
{
    x ^= x >> 16; x *= 0x7feb352du; x ^= x >> 15; x *= 0x846ca68bu; x ^= x >> 16;
    return x;
}

constexpr int kLevels = 16;
constexpr uint32_t kLevelWords = 1u << 17;   // 16 x 2^17 words = 8 MB, a hashed table's size class

// MODE 0: each lane reads words at random over the 8 MB table (64 lines per
// instruction, the training forward's pattern); 1: consecutive lanes read
// consecutive words (2 lines per instruction); 2: the four lanes of a quad
// share a line (16 lines per instruction); 3: every lane its own line (64
// lines per instruction).  Modes 1-3 stay within 16 KB (L1).
template <int MODE>
__global__ __launch_bounds__(256) void k_probe_gather(const uint32_t *__restrict__ tab, uint32_t *__restrict__ out,
                                                      int n)
{
    uint32_t acc = 0;
    const uint32_t lane = threadIdx.x & 63u;
    if constexpr (MODE == 0) {
        for (int s = blockIdx.x * 256 + threadIdx.x; s < n; s += gridDim.x * 256)
            for (int l = 0; l < kLevels; ++l) {
                const uint32_t base = mix32((uint32_t)s * 16u + (uint32_t)l) & (kLevelWords - 1);
#pragma unroll
                for (int c = 0; c < 8; ++c) acc += tab[l * kLevelWords + ((base ^ (c * 40503u)) & (kLevelWords - 1))];
            }
    } else {
        const uint32_t o = MODE == 1 ? lane : (MODE == 2 ? (lane >> 2) * 32u + (lane & 3u) : lane * 32u);
        for (int s = blockIdx.x * 256 + threadIdx.x; s < n; s += gridDim.x * 256) {
            // a wave-uniform shift per 64 samples, a multiple of the 128-byte
            // line, so that every pass loads anew (loop-invariant addresses
            // would be loaded once) with the same lines-per-instruction pattern
            const uint32_t w = ((uint32_t)s >> 6) * 1056u;
            for (int k = 0; k < kLevels * 8; k += 8) {
#pragma unroll
                for (int c = 0; c < 8; ++c) acc += tab[(o + (uint32_t)(k + c) * 64u + w) & 4095u];
            }
        }
    }
    out[blockIdx.x * 256 + threadIdx.x] = acc;
}

}  // namespace
}  // namespace niv

using namespace niv;

extern "C" niv_status niv_probe_gather(int32_t mode, int32_t n, const void *table, void *out,
                                       hipStream_t stream)
{
    if (mode < 0 || mode > 3 || n < 1 || n > (1 << 24) || !table || !out) return NIV_ERR_INVALID_ARG;
    const dim3 grid(2048), block(256);
    const uint32_t *t = static_cast<const uint32_t *>(table);
    uint32_t *o = static_cast<uint32_t *>(out);
    switch (mode) {
    case 0: hipLaunchKernelGGL(k_probe_gather<0>, grid, block, 0, stream, t, o, n); break;
    case 1: hipLaunchKernelGGL(k_probe_gather<1>, grid, block, 0, stream, t, o, n); break;
    case 2: hipLaunchKernelGGL(k_probe_gather<2>, grid, block, 0, stream, t, o, n); break;
    default: hipLaunchKernelGGL(k_probe_gather<3>, grid, block, 0, stream, t, o, n); break;
    }
    return hipGetLastError() == hipSuccess ? NIV_OK : NIV_ERR_HIP;
}
