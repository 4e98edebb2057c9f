// LDS-atomic ceiling of the dense scatter's access pattern (a measurement,
// not an operation of the paper).
//
// The dense scatter of a general tensor (Section 3.2: every entry added to
// bin sum_n h_n(i_n) with sign prod_n s_n(i_n)) keeps four sketch windows in
// LDS and adds each row of 1024 mode-0 entries to bins h_0(c) + o(row) of
// every window with 32-bit LDS atomics.  This kernel issues the same
// atomics and nothing else (no loads, no conversion, no flushes), so its
// time is what the LDS atomics alone cost on the same grid: with random
// column bins (pattern 0: the bank conflicts of random hashes) and with the
// 64 lanes of each atomic on consecutive bins (pattern 1: no conflicts).
//
// Layout of one workgroup (1024 threads, as in the dense scatter): a row of
// 1024 columns is covered by 4 waves of 64 lanes x 4 columns, so the 16
// waves keep 4 rows in flight; each lane adds its 4 columns to the 4
// windows (16 atomics per row).  Hashes come from the MurmurHash3 32-bit
// finaliser (Appleby) of a counter, so no table is read.
#include "fcs_internal.h"

namespace {

constexpr int PR_THREADS = 1024;
constexpr int PR_WINDOWS = 4;

__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

__global__ __launch_bounds__(PR_THREADS) void lds_atomic_probe_kernel(int rows, int W, int span, int pattern,
                                                                      uint32_t seed, uint32_t *sink) {
    extern __shared__ uint32_t bins[];                    // PR_WINDOWS x W
    __shared__ uint32_t red[PR_THREADS / 64];
    for (int k = threadIdx.x; k < PR_WINDOWS * W; k += PR_THREADS) bins[k] = 0u;
    __syncthreads();
    const int wave = threadIdx.x / 64;
    const int lane = threadIdx.x % 64;
    const int set = wave % 4;                             // which quarter of the row
    const int rl = wave / 4;                              // first row of the wave
    // column bins h_d(c) < span, fixed for the launch (as h_0 is)
    uint32_t h[PR_WINDOWS][4];
#pragma unroll
    for (int d = 0; d < PR_WINDOWS; ++d) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (pattern == 0) {
                const uint32_t c = (uint32_t)(set * 256 + lane * 4 + j);
                h[d][j] = fmix32(seed ^ (0x9e3779b9u * (uint32_t)(d + 1)) ^ (c << 3)) % (uint32_t)span;
            } else {
                h[d][j] = (uint32_t)(set * 256 + j * 64 + lane);
            }
        }
    }
    const uint32_t range = (uint32_t)(W - span + 1);     // row offsets o < range keep h + o < W
    for (int r = rl; r < rows; r += PR_THREADS / 256) {
        uint32_t o[PR_WINDOWS];
#pragma unroll
        for (int d = 0; d < PR_WINDOWS; ++d) {
            const uint32_t key = seed + 0x632be5abu * (uint32_t)blockIdx.x + 0x85157af5u * (uint32_t)(r * PR_WINDOWS + d);
            o[d] = (uint32_t)__builtin_amdgcn_readfirstlane((int)(fmix32(key) % range)) + (uint32_t)(d * W);
        }
#pragma unroll
        for (int d = 0; d < PR_WINDOWS; ++d) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                __hip_atomic_fetch_add(bins + o[d] + h[d][j], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    __syncthreads();
    // the workgroup's total (rows x 1024 x 4 when every atomic landed)
    uint32_t s = 0;
    for (int k = threadIdx.x; k < PR_WINDOWS * W; k += PR_THREADS) s += bins[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) red[wave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < PR_THREADS / 64; ++w) t += red[w];
        sink[blockIdx.x] = t;
    }
}

}  // namespace

extern "C" fcs_status fcs_probe_lds_atomics(int32_t blocks, int32_t rows, int32_t window, int32_t span,
                                            int32_t pattern, uint32_t seed, uint32_t *sink, void *stream) {
    fcs_clear_error();
    if (blocks < 1 || rows < 1) FCS_FAIL(FCS_EINVAL, "blocks=%d rows=%d", blocks, rows);
    if (rows >= (1 << 20)) FCS_FAIL(FCS_EINVAL, "rows=%d not below 2^20 (the per-workgroup total is 32-bit)", rows);
    if (pattern != 0 && pattern != 1) FCS_FAIL(FCS_EINVAL, "pattern=%d", pattern);
    if (span < 1024 || span > window || window > FCS_PROBE_MAX_WINDOW)
        FCS_FAIL(FCS_EINVAL, "need 1024 <= span <= window <= %d, got span=%d window=%d", FCS_PROBE_MAX_WINDOW,
                 span, window);
    if (!sink) FCS_FAIL(FCS_EINVAL, "null sink");
    const size_t lds = (size_t)PR_WINDOWS * (size_t)window * sizeof(uint32_t);
    fcs_allow_lds(reinterpret_cast<const void *>(lds_atomic_probe_kernel), lds);
    hipLaunchKernelGGL(lds_atomic_probe_kernel, dim3((unsigned)blocks), dim3(PR_THREADS), lds, (hipStream_t)stream,
                       (int)rows, (int)window, (int)span, (int)pattern, seed, sink);
    FCS_LAUNCH_CHECK();
    return FCS_OK;
}
