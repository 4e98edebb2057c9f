// Internal declarations shared by the translation units of libfcs.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <climits>
#include <cstdio>
#include <string>

#include "fcs.h"

// Packed hash word of sketch d, mode n, index i: bits 0..30 hold h_n(i),
// bit 31 is set when s_n(i) = -1.  Storing the sign as the float sign bit
// lets kernels apply it with one XOR.
constexpr uint32_t FCS_H_MASK = 0x7fffffffu;
constexpr uint32_t FCS_S_BIT = 0x80000000u;

// First-entry word of a hash bucket (inverse lists): bits 0..29 the index of
// the bucket's first entry, bit 30 set when the bucket holds more entries,
// bit 31 that entry's sign.  FCS_FIRST_EMPTY marks an empty bucket.
constexpr uint32_t FCS_IDX_MASK = 0x3fffffffu;
constexpr uint32_t FCS_MORE_BIT = 0x40000000u;
constexpr uint32_t FCS_FIRST_EMPTY = 0x7fffffffu;
constexpr int64_t FCS_MAX_GATHER_INDEX = (int64_t)1 << 30;

constexpr int FCS_MIN_FFT = 256;
constexpr size_t FCS_LDS_BYTES = 160 * 1024;   // LDS per CU on gfx950

struct fcs_plan {
    int N = 0, D = 0;
    int64_t I[FCS_MAX_ORDER] = {0}, J[FCS_MAX_ORDER] = {0};
    // hash values: h_n(i) = hmul[n] * lemire(y, Jh[n]), so J[n] = (Jh[n] - 1)
    // * hmul[n] + 1.  A sketch plan has hmul = 1 and Jh = J; a higher-order
    // count sketch plan has the mixed-radix strides hmul[n] = prod_{m<n} Jh[m],
    // so that sum_n h_n(i_n) is the flattened multi-index (mode 0 fastest)
    // and J~ = prod_n Jh[n]
    int64_t Jh[FCS_MAX_ORDER] = {0}, hmul[FCS_MAX_ORDER] = {0};
    bool hcs = false;
    int64_t off[FCS_MAX_ORDER] = {0};   // offset of mode n inside a sketch's table
    int64_t sumI = 0;
    uint64_t seed = 0;
    int64_t Jt = 0;                    // J~ = sum J_n - N + 1
    int64_t L = 0, P = 0;              // transform length L = Q * P, FFT size P
    int Q = 0, Qh = 0;                 // slices, stored slices floor(Q/2)+1
    // device layout inside the caller's table buffer
    size_t tab_off = 0, twP_off = 0, twL_off = 0, inv_off = 0, total = 0;
    const uint32_t *tab = nullptr;     // D x sumI packed hash words
    const float2 *twP = nullptr;       // exp(-2 pi i k / P), k < P
    const float2 *twL = nullptr;       // exp(-2 pi i k / L), k < L
    // inverse hash lists (buckets of h_n), per sketch a block of iblock words:
    // for mode n at ioff[n]: J_n + 1 bucket offsets, then I_n entries
    // (index i | sign bit), entries of bucket j at [off[j], off[j+1]), then
    // J_n first-entry words (FCS_IDX_MASK / FCS_MORE_BIT / FCS_FIRST_EMPTY),
    // then J_n second-entry words (the same fields; MORE: a third entry)
    const int32_t *inv = nullptr;
    int64_t ioff[FCS_MAX_ORDER] = {0};
    int64_t iblock = 0;
    // largest number of mode-0 indices that share one h_0 value, over all
    // sketches (bounds the additions one row makes to one bin); INT32_MAX
    // when too large to evaluate on the host
    int m0 = INT32_MAX;
    // lane order of the dense scatter: for each group of sketches and each
    // 256-column segment, the 16-byte column block each of the 64 lanes of a
    // wave loads (D x segs x 64 bytes; absent when perm_bytes == 0)
    // (computed on the first dense sketch of the plan, see perm_ready)
    size_t perm_off = 0, perm_bytes = 0;
    const uint8_t *perm = nullptr;
    bool perm_ready = false;
    bool bound = false;
};

// dense scatter lane order (scatter.hip): bytes reserved in the plan layout,
// and the search that fills them from the host's mode-0 hash values
// (h0[d * I_0 + i] = h_0 of sketch d); perm has perm_bytes entries
size_t fcs_dense_perm_bytes(const fcs_plan *p);
void fcs_dense_lane_order(const fcs_plan *p, const uint32_t *h0, uint8_t *perm);
// sketches per group of the dense kernel's first pass (0: HBM fallback)
int fcs_dense_group_size(const fcs_plan *p);
// h_0 of every sketch on the host (plan.hip), h0[d * I_0 + i]
void fcs_mode0_hashes(const fcs_plan *p, uint32_t *h0);

// error reporting ----------------------------------------------------------
void fcs_set_error(const char *fmt, ...);
void fcs_clear_error();

#define FCS_FAIL(code, ...)              \
    do {                                 \
        fcs_set_error(__VA_ARGS__);      \
        return (code);                   \
    } while (0)

#define FCS_HIP_CHECK(expr)                                                   \
    do {                                                                      \
        hipError_t e_ = (expr);                                               \
        if (e_ != hipSuccess)                                                 \
            FCS_FAIL(FCS_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define FCS_LAUNCH_CHECK()                                                     \
    do {                                                                       \
        hipError_t e_ = hipGetLastError();                                     \
        if (e_ != hipSuccess)                                                  \
            FCS_FAIL(FCS_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e_)); \
    } while (0)

static inline bool fcs_aligned(const void *p, size_t a) {
    return (reinterpret_cast<uintptr_t>(p) % a) == 0;
}

static inline int64_t fcs_ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// shared launch helpers (defined in plan.hip) --------------------------------
fcs_status fcs_zero_fill(float *p, int64_t n, hipStream_t s);
// Opt a kernel in to `bytes` of dynamic LDS above the 64 KB default, once per
// kernel and device (so that launches captured into a graph make no
// attribute calls after the first use).
void fcs_allow_lds(const void *kernel, size_t bytes);
int fcs_device_cu_count();

// workspace sizes of each operation (defined next to the kernels)
size_t fcs_ws_dense(const fcs_plan *p);
size_t fcs_ws_coo(const fcs_plan *p);
size_t fcs_ws_cp(const fcs_plan *p, int64_t R);
size_t fcs_ws_inner(const fcs_plan *p);
size_t fcs_ws_free_mode(const fcs_plan *p, int64_t P);
size_t fcs_ws_spectrum(const fcs_plan *p);
size_t fcs_ws_kron(const fcs_plan *p);
size_t fcs_ws_contraction(const fcs_plan *p, int64_t Lc);
size_t fcs_ws_full(const fcs_plan *p, int64_t Pn);
