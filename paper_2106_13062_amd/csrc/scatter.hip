// Dense and COO fast count sketch: the general-tensor formula of Section 3.2.
//
// Every element T[i_0..i_{N-1}] is added with sign S = prod_n s_n(i_n) to bin
// H = sum_n h_n(i_n) of each of the D sketches.  The long hash (H, S) of
// Definition 4 is never built: only the N short tables are read.
//
// Why integer bins.  On gfx950 an LDS float atomic add (ds_add_f32) retires
// about 0.3 lanes per clock per CU, while ds_add_u32 retires about 12 in the
// access pattern of this kernel (ds_add_f64 about 3).  The bins are therefore
// 32-bit fixed-point integers: each workgroup picks a power-of-two scale 2^F
// from the largest magnitude among its first rows, adds round(x 2^F) with
// ds_add_u32, and converts the bins back to float (exactly, by 2^-F) into
// per-thread register accumulators at the end of every "period" of rows.
//   * |round(x 2^F)| <= 2^21 - 1 for every element taken on this path;
//   * a row adds at most m0 elements to one bin, m0 the largest number of
//     mode-0 indices sharing one h_0 value (computed when the plan is bound);
//     a period of P rows with P * m0 <= 1023 therefore keeps every bin below
//     2^31 in magnitude: no overflow is possible.  Plans with m0 > 255
//     (a period shorter than 4 rows) take the HBM float-atomic kernel.
//   * precision: a block is sketched first at a speculative scale, the
//     largest sampled magnitude mapped into [2^19, 2^20).  That pass is kept
//     only if no element left the fixed-point range and the modelled
//     rounding error of every window is at most 3e-6 of its norm (about
//     2e-6 on Gaussian data).  Otherwise the block is redone at a scale from
//     its own root mean square (relative error at most 3.8e-6 of the
//     block's 2-norm), with the few elements beyond the range (at most 1/64
//     of them) added as float atomics.  Integer-valued data with small
//     magnitudes is exact.
//
// Dense kernel layout (gfx950, wave64):
//  * vec(T) is a sequence of rows along mode 0 (I_0 contiguous floats).  Along
//    a row H = c(row) + h_0(i_0), so the offset c and the row sign are
//    wave-uniform and the column part h_0 / s_0 is fixed for every row a wave
//    visits.  A wave owns a 256-column segment (one 16-byte load per lane) of
//    the rows it visits; its lanes keep the LDS byte address of bin h_0(i_0)
//    and the sign of s_0(i_0) of every sketch of the group in registers.  Per
//    element: one scale, one range test, one v_cvt_rpi (round); per element
//    and sketch: one v_mul_i32_i24 (column sign), half a 64-bit add (the
//    addresses of two sketches share one v_lshl_add_u64) and one ds_add_u32
//    or ds_sub_u32 (the row sign, uniform per wave).
//  * Each wave keeps four row loads in flight (rows k+1..k+4 while row k is
//    added); every row issues exactly one load, so each wait is "at most
//    three younger loads outstanding".  The row offsets and signs of a flush
//    period are computed into a small LDS table during the previous flush,
//    so the row loop issues no other memory loads.
//  * When N >= 2 a workgroup's rows share the last-mode index, so its bins lie
//    in h_{N-1}(i_{N-1}) + [0, J~ - J_{N-1} + 1) and only that window is held
//    (the last mode's sign is applied at the flush).  Sketches are split into
//    groups of DG windows that fit in LDS; the groups of one slab are
//    dispatched back to back onto one XCD (workgroups go round-robin over the
//    8 XCDs) so the second read of the slab hits that XCD's L2.
#include "fcs_internal.h"

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

namespace {

constexpr int DS_THREADS = 1024;        // 16 waves
constexpr int DS_WAVES = DS_THREADS / 64;
constexpr int SEG = 256;                // columns of a wave segment
constexpr int GSEG = 4;                 // segments per lane-order set (1024 columns)
constexpr int NXCD = 8;
constexpr int MAXACC = 32;              // register accumulators per thread
constexpr int SCALE_TOP = 20;           // first-rows max maps below 2^20
constexpr float QLIM = 2097150.0f;      // 2^21 - 2: larger |x 2^F| -> float path
constexpr int ADD_BOUND = 1023;         // P * m0 <= 1023 keeps |bin| < 2^31
constexpr size_t ROWTAB_BYTES = 16 * ADD_BOUND;   // row table of one flush period (<= ADD_BOUND rows)
constexpr int EXACT_TOP = 18;           // exact pass: root mean square maps into [2^17, 2^18)
constexpr int REDO_HEAD = 64;           // workspace words before the redo lists (counts of both launch passes)
// speculative pass accepted when the modelled rounding error of every window
// is at most 3e-6 of its norm (squared here)
constexpr double DENSE_TAU2 = 9e-12;

struct DenseArgs {
    const float *T;
    float *out;
    const uint32_t *tab;
    int32_t I[FCS_MAX_ORDER];
    int64_t off[FCS_MAX_ORDER];
    int64_t sumI;
    int64_t I0;
    int64_t rows;            // prod_{n>=1} I_n
    int64_t slab_rows;       // rows sharing one last-mode index
    int64_t block_rows;      // rows per row block
    int64_t blocks_per_slab;
    int64_t row_blocks;
    int64_t Jt;
    int W;                   // bins held per sketch in LDS
    int N;
    int D;
    int ngroups;             // groups of DG sketches in this launch
    int d_first;             // first sketch of this launch
    int windowed;            // 1: window anchored at h_{N-1}(i_{N-1})
    int segs;                // ceil(I0 / SEG)
    int seg_blocks;          // column blocks
    int segs_per_block;
    int period;              // rows per flush period
    int nrow_modes;          // modes 1..nrow_modes vary along a block's rows
    int dg_full;             // sketches per group of the first pass
    const uint8_t *perm;     // lane order per (group, segment); null: identity
    uint32_t *redo_n;        // entries of the redo list (blocks given up by the speculative pass)
    uint32_t *redo_list;     // their block indices
};

// 24-bit signed multiply (|a| < 2^22, b = +-1 here): one VALU op, with no
// sign extension of the operands
__device__ __forceinline__ int mul_i24(int a, int b) {
    int r;
    asm("v_mul_i32_i24 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// round to nearest (ties up) and convert: one VALU op
__device__ __forceinline__ int cvt_rpi(float x) {
    int r;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

__device__ __forceinline__ int64_t fcs_ceil_div_dev(int64_t a, int64_t b) { return (a + b - 1) / b; }

// LDS atomics on 32-bit LDS byte addresses: the base of the dynamic LDS
// array is folded into the per-lane addresses once, so each atomic needs a
// single v_add (lane address + uniform row offset)
typedef __attribute__((address_space(3))) uint32_t lds_u32;
__device__ __forceinline__ uint32_t lds_addr(uint32_t *p) { return (uint32_t)(uintptr_t)(lds_u32 *)p; }
__device__ __forceinline__ void lds_add(uint32_t addr, uint32_t v) {
    __hip_atomic_fetch_add((lds_u32 *)(uintptr_t)addr, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_sub(uint32_t addr, uint32_t v) {
    __hip_atomic_fetch_sub((lds_u32 *)(uintptr_t)addr, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ inline void dense_block_map(const DenseArgs &a, int64_t bid, int64_t &blk, int &grp) {
    const int64_t span = (int64_t)NXCD * a.ngroups;
    const int64_t super = bid / span;
    const int64_t rem = bid - super * span;
    grp = (int)(rem / NXCD);
    blk = super * NXCD + (rem % NXCD);
}

template <bool VEC4, bool FULL>
// the 4 columns of 16-byte block `blk` of a row segment
__device__ __forceinline__ void load_seg(const float *row, int blk, const bool (&valid)[4], float (&x)[4]) {
    if (FULL && VEC4) {
        const float4 q = reinterpret_cast<const float4 *>(row)[blk];
        x[0] = q.x; x[1] = q.y; x[2] = q.z; x[3] = q.w;
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) x[e] = (FULL || valid[e]) ? row[blk * 4 + e] : 0.f;
    }
}

// The LDS addresses of one element in two sketches of a pair sit in the low
// and high halves of a 64-bit register; one 64-bit add of the two uniform
// row offsets forms both (every address is below 2^18, so no carry crosses
// the halves).
__device__ __forceinline__ uint64_t add_pair(uint64_t v, uint64_t s) {
    uint64_t r;
    asm("v_lshl_add_u64 %0, %1, 0, %2" : "=v"(r) : "v"(v), "s"(s));
    return r;
}

// Out-of-range or non-finite entries of one row segment: float atomics into
// the HBM sketch, with every sign including the slab's last-mode sign.
template <int DG, bool CHECK>
__device__ __forceinline__ void scatter_slow(const DenseArgs &a, uint32_t qaddr, const float (&x)[4], float scale,
                                             int d0, const uint64_t (&A2)[(DG + 1) / 2][4], const int (&S)[DG][4],
                                             const bool (&valid)[4], const uint32_t (&C)[DG], const int (&base)[DG],
                                             const uint32_t (&wsign)[DG]) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const float xe = x[e];
        if ((!CHECK || valid[e]) && !(fabsf(xe * scale) < QLIM)) {
#pragma unroll
            for (int d = 0; d < DG; ++d) {
                const uint32_t ad = (d & 1) ? (uint32_t)(A2[d >> 1][e] >> 32) : (uint32_t)A2[d >> 1][e];
                const int bin = (int)((ad + (C[d] & FCS_H_MASK) - qaddr) / 4u) - d * a.W;
                const uint32_t sg = (S[d][e] < 0 ? FCS_S_BIT : 0u) ^ (C[d] & FCS_S_BIT) ^ wsign[d];
                unsafeAtomicAdd(a.out + (int64_t)(d0 + d) * a.Jt + base[d] + bin,
                                __uint_as_float(__float_as_uint(xe) ^ sg));
            }
        }
    }
}

// Add one row segment (4 values per lane, in `buf`) to the DG fixed-point
// windows, then reuse `buf` for the load of row `next`.  Each value is scaled
// and rounded once (v_cvt_rpi); the column sign of every sketch is a 24-bit
// integer multiply by +-1 and the row sign, uniform across the wave, selects
// ds_sub_u32 instead of ds_add_u32.  A wave with an out-of-range element in
// the row takes the float path for those elements and adds zero for them to
// the bins.  C holds the row's words (byte offset | sign bit) per sketch.
template <int DG, bool VEC4, bool FULL, bool EXACT>
__device__ __forceinline__ void scatter_row(const DenseArgs &a, uint32_t qaddr, float (&buf)[4], const float *next,
                                            float scale, int d0, int blk, const uint64_t (&A2)[(DG + 1) / 2][4],
                                            const int (&S)[DG][4], const bool (&valid)[4], const uint32_t (&C)[DG],
                                            const int (&base)[DG], const uint32_t (&wsign)[DG], bool process,
                                            uint32_t *ctl) {
    constexpr int DP = (DG + 1) / 2;
    constexpr bool CHECK = !FULL;
    int q[4];
    if (process) {
        bool slow = false;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float xs = buf[e] * scale;
            slow |= !(fabsf(xs) < QLIM) && (!CHECK || valid[e]);   // NaN / Inf too
            q[e] = cvt_rpi(xs);            // saturating; zeroed below when out of range
        }
        if (__builtin_expect(__builtin_amdgcn_ballot_w64(slow) != 0, 0)) {
            // the speculative pass gives the block up (it is redone with
            // the block's own statistics); the exact pass adds such entries
            // as floats
            if constexpr (EXACT)
                scatter_slow<DG, CHECK>(a, qaddr, buf, scale, d0, A2, S, valid, C, base, wsign);
            else
                *ctl = 1u;
#pragma unroll
            for (int e = 0; e < 4; ++e) q[e] = (fabsf(buf[e] * scale) < QLIM) ? q[e] : 0;
        }
    }
    // the load is issued whether or not the row is processed, so every
    // group of 4 rows issues exactly 4 loads (in-order waits stay exact)
    load_seg<VEC4, FULL>(next, blk, valid, buf);
    if (!process) return;
#pragma unroll
    for (int p = 0; p < DP; ++p) {
        const uint32_t lo = C[2 * p] & FCS_H_MASK;
        const uint32_t hi = C[2 * p + 1 < DG ? 2 * p + 1 : 2 * p] & FCS_H_MASK;
        const uint64_t cc = (uint64_t)lo | ((uint64_t)hi << 32);
        uint64_t ad[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) ad[e] = add_pair(A2[p][e], cc);
#pragma unroll
        for (int h = 0; h < 2 && 2 * p + h < DG; ++h) {
            const int d = 2 * p + h;
            if (C[d] & FCS_S_BIT) {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (!CHECK || valid[e])
                        lds_sub(h ? (uint32_t)(ad[e] >> 32) : (uint32_t)ad[e], (uint32_t)mul_i24(q[e], S[d][e]));
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (!CHECK || valid[e])
                        lds_add(h ? (uint32_t)(ad[e] >> 32) : (uint32_t)ad[e], (uint32_t)mul_i24(q[e], S[d][e]));
            }
        }
    }
}

// Row words of a flush period, kept in LDS after the bins: for each of the
// `cnt` block rows from r (global row index) on, 4 words (one per sketch of
// the group, unused ones zero): (byte offset of the row in the window) |
// (row sign bit), the row offset being sum_n h_n(i_n) over the modes that
// vary along the block's rows.  Filled by the whole workgroup between the
// barriers of a period flush, so the row loop issues no table loads.
template <int DG, int NV>
__device__ __forceinline__ void fill_rowtab(const DenseArgs &a, int d0, uint32_t *rowtab, int64_t r, int cnt) {
    for (int j = threadIdx.x; j < cnt; j += DS_THREADS) {
        int64_t rem = r + j;
        int idx[NV > 0 ? NV : 1];
#pragma unroll
        for (int n = 0; n < NV; ++n) {
            const int64_t In = a.I[n + 1];
            idx[n] = (int)(rem % In);
            rem /= In;
        }
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            uint32_t c = 0, sg = 0;
            if (d < DG) {
#pragma unroll
                for (int n = 0; n < NV; ++n) {
                    const uint32_t w = a.tab[(int64_t)(d0 + d) * a.sumI + a.off[n + 1] + idx[n]];
                    c += (w & FCS_H_MASK) * 4u;
                    sg ^= w & FCS_S_BIT;
                }
            }
            rowtab[j * 4 + d] = c | sg;
        }
    }
}

// One wave's rows r_first + k * wps (k < nk) of one column segment, in flush
// periods of pk rows.  Four row loads are in flight: row k + 4 is loaded into
// the buffer of row k as soon as row k is rounded.  Loads past the last row
// re-read it, so every row issues exactly one load and the wait for a row is
// always "at most three younger loads outstanding".  Every wave of the
// workgroup calls this with the same period count so all reach every barrier.
template <int DG, int NV, bool VEC4, bool FULL, bool EXACT>
__device__ __forceinline__ void wave_rows(const DenseArgs &a, uint32_t *qbins, uint32_t *rowtab, float (&acc)[MAXACC],
                                          float (&nrm)[DG],
                                          float scale, float inv, int d0, int seg, int lane, bool active, int64_t r0,
                                          int64_t nrows, int rl, int nk, int wps, int pk, int nperiods,
                                          const int (&base)[DG], const uint32_t (&wsign)[DG], uint32_t *ctl) {
    const int64_t r_first = r0 + rl;
    constexpr int DP = (DG + 1) / 2;
    const int W = a.W;
    const uint32_t qaddr = lds_addr(qbins);
    uint64_t A2[DP][4];
    int S[DG][4];
    bool valid[4];
    // the 16-byte column block this lane loads: with a lane order, any block
    // of the segment's set of GSEG segments (1024 columns), chosen at bind to
    // spread LDS banks; without one, block `lane` of its own segment
    const int64_t set_col = a.perm ? (int64_t)(seg / GSEG) * (GSEG * SEG) : (int64_t)seg * SEG;
    const int pb = a.perm ? (int)a.perm[((int64_t)(d0 / a.dg_full) * a.segs + seg) * 64 + lane] : lane;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t col = set_col + pb * 4 + e;
        valid[e] = active && col < a.I0;
        uint32_t Ad[DG];
#pragma unroll
        for (int d = 0; d < DG; ++d) {
            const uint32_t p = valid[e] ? a.tab[(int64_t)(d0 + d) * a.sumI + col] : 0u;
            Ad[d] = qaddr + (uint32_t)((d * W + (int)(p & FCS_H_MASK)) * 4);
            S[d][e] = (p & FCS_S_BIT) ? -1 : 1;
        }
#pragma unroll
        for (int p = 0; p < DP; ++p)
            A2[p][e] = (uint64_t)Ad[2 * p] | ((uint64_t)Ad[2 * p + 1 < DG ? 2 * p + 1 : 2 * p] << 32);
    }
    const float *Tseg = a.T + set_col;
    const int64_t I0 = a.I0;
    auto rowp = [&](int k) { return Tseg + (r_first + (int64_t)min(k, nk - 1) * wps) * I0; };
    float b0[4], b1[4], b2[4], b3[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        b0[e] = 0.f;
        b1[e] = 0.f;
        b2[e] = 0.f;
        b3[e] = 0.f;
    }
    if (active && nk > 0) {
        load_seg<VEC4, FULL>(rowp(0), pb, valid, b0);
        load_seg<VEC4, FULL>(rowp(1), pb, valid, b1);
        load_seg<VEC4, FULL>(rowp(2), pb, valid, b2);
        load_seg<VEC4, FULL>(rowp(3), pb, valid, b3);
    }
    // lane j holds the words of wave row k0 + j (64 rows of the period at a
    // time, read from the period's row table and broadcast with v_readlane)
    uint32_t CR[DG];
    auto refresh = [&](int k0, int kb, int ke) {
        const bool live = k0 + lane < ke;
        const int j = rl + (k0 + lane - kb) * wps;
#pragma unroll
        for (int d = 0; d < DG; ++d) CR[d] = live ? rowtab[j * 4 + d] : 0u;
        // take the wait for these reads here, once per 64 rows, so that the
        // row loop does not wait for its own atomics before v_readlane
#pragma unroll
        for (int d = 0; d < DG; ++d) asm volatile("" : "+v"(CR[d]));
    };
    auto row = [&](int k, int k0, float (&buf)[4], bool process) {
        uint32_t C[DG];
#pragma unroll
        for (int d = 0; d < DG; ++d) C[d] = process ? __builtin_amdgcn_readlane(CR[d], k - k0) : 0u;
        scatter_row<DG, VEC4, FULL, EXACT>(a, qaddr, buf, rowp(k + 4), scale, d0, pb, A2, S, valid, C, base,
                                           wsign, process, ctl);
    };

    // pk is a multiple of 4, so every period starts on buffer b0; only the
    // wave's last group can hold fewer than 4 rows
    int k = 0;
    for (int p = 0; p < nperiods; ++p) {
        const int kb = p * pk;
        const int ke = active ? min(kb + pk, nk) : 0;
        int k0 = k;
        if (k < ke) refresh(k0, kb, ke);
        for (; k < ke; k += 4) {
            if (k - k0 == 64) {
                k0 = k;
                refresh(k0, kb, ke);
            }
            row(k, k0, b0, true);
            row(k + 1, k0, b1, k + 1 < ke);
            row(k + 2, k0, b2, k + 2 < ke);
            row(k + 3, k0, b3, k + 3 < ke);
        }
        __syncthreads();
        // a block given up by the speculative pass stops here: every wave
        // reads the flag between the same two barriers (it is only written
        // in the row loops)
        if (!EXACT && *ctl) return;
        // period flush: integer bins -> float register accumulators (exact
        // scaling by 2^-F), bins back to zero.  Thread t holds bins
        // t + 1024 m of each window; nrm sums the squared bins (in units of
        // the quantum) for the check of the speculative pass.
#pragma unroll
        for (int d = 0; d < DG; ++d) {
#pragma unroll
            for (int m = 0; m < MAXACC / DG; ++m) {
                const int j = threadIdx.x + m * DS_THREADS;
                if (j < W) {
                    const float t = (float)(int)qbins[d * W + j];
                    acc[d * (MAXACC / DG) + m] += t * inv;
                    if constexpr (!EXACT) nrm[d] += t * t;
                    qbins[d * W + j] = 0u;
                }
            }
        }
        if (p + 1 < nperiods) {
            const int64_t jb = (int64_t)(p + 1) * pk * wps;
            fill_rowtab<DG, NV>(a, d0, rowtab, r0 + jb, (int)min<int64_t>((int64_t)pk * wps, nrows - jb));
        }
        __syncthreads();
    }
}

// Check of the speculative pass.  Rounding to the quantum q = 2^-F moves an
// entry by at most q/2, and the hash signs make those moves add like
// independent terms: the expected squared error of a window is at most
// n q^2 / 4 for n entries, and n q^2 / 12 when the moves are spread evenly
// over [-q/2, q/2].  The pass is kept when n q^2 / 12 is at most
// DENSE_TAU2 times the squared norm of every sketch's window (relative error
// 3e-6 in that model, at most 5.2e-6 in the worst case).  The squared norm
// is taken as the sum over flush periods of the squared bins, which has the
// window's squared norm as its expectation over the hash signs; both sides
// are in units of q^2, where the sums cannot overflow or underflow a float.
// Uses 16 * DG floats of scratch LDS; every thread returns the same answer.
template <int DG>
__device__ __forceinline__ bool dense_error_ok(const float (&nrm)[DG], float nelem, uint32_t *scratch, int wave,
                                               int lane) {
    float *red = reinterpret_cast<float *>(scratch);
#pragma unroll
    for (int d = 0; d < DG; ++d) {
        float v = nrm[d];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) red[wave * DG + d] = v;
    }
    __syncthreads();
    const float err2 = nelem * (1.0f / 12.0f);
    bool ok = true;
#pragma unroll
    for (int d = 0; d < DG; ++d) {
        float t = 0.f;
#pragma unroll
        for (int w = 0; w < DS_WAVES; ++w) t += red[w * DG + d];
        ok = ok && err2 <= (float)DENSE_TAU2 * t;
    }
    __syncthreads();
    return ok;
}

// Scale exponent of the exact pass: the root mean square of the block's
// finite entries maps into [2^17, 2^18).  An entry on the fixed-point path
// then moves by at most 2^-18 of that root mean square, so the expected
// squared error of a window is at most 2^-36 of the block's squared 2-norm
// (relative error 3.8e-6), and by Chebyshev's inequality at most 1/64 of the
// entries exceed the 2^21 range and take the float path.  Reads the block
// once more, 16 loads in flight per thread; uses 16 doubles of scratch LDS.
template <bool VEC4>
__device__ int dense_exact_exponent(const DenseArgs &a, int64_t r0, int64_t r1, int64_t c_lo, int64_t c_hi,
                                    double nelem, uint32_t *scratch, int wave, int lane) {
    constexpr int V = VEC4 ? 4 : 1;            // floats per load (VEC4: I_0 % 4 == 0, 16-byte aligned)
    constexpr int U = 16;
    const int64_t nb = (c_hi - c_lo) / V;      // loads per row (c_lo, c_hi multiples of 4 with VEC4)
    const int64_t total = (r1 - r0) * nb;
    const int64_t dr = DS_THREADS / nb, dc = DS_THREADS % nb;
    int64_t row = threadIdx.x / nb, col = threadIdx.x % nb;
    double s2 = 0.0;
    for (int64_t k = threadIdx.x; k < total; k += (int64_t)U * DS_THREADS) {
        float v[U][V];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool ok = k + (int64_t)u * DS_THREADS < total;
            const float *p = a.T + (r0 + row) * a.I0 + c_lo + col * V;
            if constexpr (VEC4) {
                const float4 t = ok ? *reinterpret_cast<const float4 *>(p) : make_float4(0.f, 0.f, 0.f, 0.f);
                v[u][0] = t.x;
                v[u][1] = t.y;
                v[u][2] = t.z;
                v[u][3] = t.w;
            } else {
                v[u][0] = ok ? *p : 0.f;
            }
            // position of the next load of this thread
            col += dc;
            row += dr;
            if (col >= nb) {
                col -= nb;
                ++row;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < V; ++e)
                if (fabsf(v[u][e]) <= 3.4028235e38f) s2 += (double)v[u][e] * (double)v[u][e];
    }
    double *red = reinterpret_cast<double *>(scratch);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s2 += __shfl_xor(s2, o, 64);
    if (lane == 0) red[wave] = s2;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < DS_WAVES; ++w) t += red[w];
    __syncthreads();
    const double ms = t / nelem;
    int F = 0;
    if (ms > 0.0) {
        int e;
        frexp(sqrt(ms), &e);
        F = EXACT_TOP - e;
    }
    return max(-120, min(126, F));
}

// One row block (all its rows, up to 16 column segments, DG sketches).
// The speculative form (EXACT false) takes its scale from the sampled
// leading rows and, when its check fails, appends the block to the redo
// list and writes nothing; the exact form takes its scale from the block's
// own mean square.
template <int DG, int NV, bool VEC4, bool FULL, bool EXACT>
__device__ __forceinline__ void dense_block(const DenseArgs &a, int64_t bid, uint32_t *qbins) {
    int64_t blk;
    int grp;
    dense_block_map(a, bid, blk, grp);
    if (blk >= a.row_blocks * a.seg_blocks) return;
    const int64_t rblk = blk / a.seg_blocks;
    const int sblk = (int)(blk - rblk * a.seg_blocks);
    const int d0 = a.d_first + grp * DG;

    // rows and column segments of this block (at most 16 segments)
    int64_t r0, r1;
    if (a.windowed) {
        const int64_t slab = rblk / a.blocks_per_slab;
        const int64_t sub = rblk - slab * a.blocks_per_slab;
        r0 = slab * a.slab_rows + sub * a.block_rows;
        r1 = min(r0 + a.block_rows, (slab + 1) * a.slab_rows);
    } else {
        r0 = rblk * a.block_rows;
        r1 = min(r0 + a.block_rows, a.rows);
    }
    const int s0 = sblk * a.segs_per_block;
    const int s1 = min(a.segs, s0 + a.segs_per_block);
    const int nseg = s1 - s0;

    // window base and sign per sketch: the last-mode hash pair of the slab
    int base[DG];
    uint32_t wsign[DG];
    const int64_t ilast = (a.windowed && a.N >= 2) ? (r0 / a.slab_rows) : 0;
#pragma unroll
    for (int d = 0; d < DG; ++d) {
        base[d] = 0;
        wsign[d] = 0;
        if (a.windowed && a.N >= 2) {
            const uint32_t p = a.tab[(int64_t)(d0 + d) * a.sumI + a.off[a.N - 1] + ilast];
            base[d] = (int)(p & FCS_H_MASK);
            wsign[d] = p & FCS_S_BIT;
        }
    }

    const int W = a.W;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    const int lane = threadIdx.x % 64;

    // speculative scale: largest magnitude among up to 16 leading rows
    // (first 4096 columns of the block's segments), mapped into
    // [2^19, 2^20); the wave maxima are exchanged through the (not yet
    // used) bin memory
    float M0 = 0.f;
    if constexpr (!EXACT) {
        const int64_t nrows = r1 - r0;
        const int64_t r = r0 + (wave % nrows);
        const int64_t c0 = (int64_t)s0 * SEG;
        const int64_t c1 = min<int64_t>(min<int64_t>((int64_t)s1 * SEG, a.I0), c0 + 4096);
        const float *rowp = a.T + r * a.I0;
        float m = 0.f;
        // 16 independent loads per pass (one memory latency per 1024
        // columns); indices past the end re-read the last column
        for (int64_t c = c0 + lane; c < c1; c += 1024) {
            float v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) v[u] = rowp[min<int64_t>(c + u * 64, c1 - 1)];
#pragma unroll
            for (int u = 0; u < 16; ++u) m = fmaxf(m, fabsf(v[u]));
        }
        // NaN / Inf in the sample are ignored here (they make the check fail)
        if (!(m <= 3.0e38f)) m = 0.f;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
        if (lane == 0) qbins[wave] = __float_as_uint(m);
        __syncthreads();
#pragma unroll
        for (int w = 0; w < DS_WAVES; ++w) M0 = fmaxf(M0, __uint_as_float(qbins[w]));
        __syncthreads();
    }
    // each wave owns at most one (segment, row lane) of the block; waves
    // per segment at most period / 4 so that a multiple of 4 rows per wave
    // fits a flush period (pk * wps <= period)
    const int wps = max(1, min(DS_WAVES / nseg, a.period / 4));
    const int64_t nrows = r1 - r0;
    const bool active = wave < nseg * wps;
    const int seg = s0 + (active ? wave % nseg : 0);
    const int rl = active ? wave / nseg : 0;
    const int nk = (active && rl < nrows) ? (int)((nrows - rl + wps - 1) / wps) : 0;
    const int pk = (a.period / wps) & ~3;                // >= 4, a multiple of 4
    const int nperiods = (int)((fcs_ceil_div_dev(nrows, wps) + pk - 1) / pk);
    // the row table of a period sits after the bins (16-byte aligned), the
    // give-up flag of the speculative pass after the row table
    uint32_t *rowtab = qbins + ((DG * W + 3) & ~3);
    uint32_t *ctl = rowtab + 4 * a.period;
    const int64_t c_lo = (int64_t)s0 * SEG;
    const int64_t c_hi = min<int64_t>((int64_t)s1 * SEG, a.I0);
    // entries of the block (a count, in single precision for the error model)
    const float nelem = (float)nrows * (float)(c_hi - c_lo);
    int F;
    if constexpr (EXACT) {
        F = dense_exact_exponent<VEC4>(a, r0, r1, c_lo, c_hi, (double)nrows * (double)(c_hi - c_lo), qbins, wave,
                                       lane);
    } else {
        F = SCALE_TOP - 1;
        if (M0 > 0.f) F = SCALE_TOP - __builtin_amdgcn_frexp_expf(M0);
        F = max(-100, min(100, F));
    }
    const float scale = ldexpf(1.0f, F);
    const float inv = ldexpf(1.0f, -F);
    for (int k = threadIdx.x; k < DG * W; k += DS_THREADS) qbins[k] = 0u;
    if (threadIdx.x == 0) *ctl = 0u;
    fill_rowtab<DG, NV>(a, d0, rowtab, r0, (int)min<int64_t>((int64_t)pk * wps, nrows));
    __syncthreads();

    float acc[MAXACC], nrm[DG];
#pragma unroll
    for (int m = 0; m < MAXACC; ++m) acc[m] = 0.f;
#pragma unroll
    for (int d = 0; d < DG; ++d) nrm[d] = 0.f;
    // FULL kernels are launched only when every segment is complete
    wave_rows<DG, NV, VEC4, FULL, EXACT>(a, qbins, rowtab, acc, nrm, scale, inv, d0, seg, lane, active, r0, nrows, rl,
                                         nk, wps, pk, nperiods, base, wsign, ctl);
    if constexpr (!EXACT) {
        // the speculative pass is kept when no entry left the fixed-point
        // range and the modelled rounding error is small beside every
        // window (the row loops ended at a barrier: the flag is final);
        // otherwise the block goes to the redo list of the exact kernel
        if (*ctl != 0u || !dense_error_ok<DG>(nrm, nelem, qbins, wave, lane)) {
            if (threadIdx.x == 0) {
                const uint32_t slot = atomicAdd(a.redo_n, 1u);
                a.redo_list[slot] = (uint32_t)bid;
            }
            return;
        }
    }

    // add the window to the HBM sketch, with the slab's last-mode sign
#pragma unroll
    for (int d = 0; d < DG; ++d) {
#pragma unroll
        for (int m = 0; m < MAXACC / DG; ++m) {
            const int j = threadIdx.x + m * DS_THREADS;
            const float v = __uint_as_float(__float_as_uint(acc[d * (MAXACC / DG) + m]) ^ wsign[d]);
            if (j < W && v != 0.f) unsafeAtomicAdd(a.out + (int64_t)(d0 + d) * a.Jt + base[d] + j, v);
        }
    }
}

// Speculative pass over every block of the launch.
template <int DG, int NV, bool VEC4, bool FULL>
// one workgroup per CU when the window fills LDS: allow 2 waves per SIMD
__global__ __launch_bounds__(DS_THREADS) __attribute__((amdgpu_waves_per_eu(2, 2))) void dense_scatter_kernel(
    DenseArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint32_t qbins[];     // DG x W fixed-point bins
    dense_block<DG, NV, VEC4, FULL, false>(a, blockIdx.x, qbins);
}

// Exact pass over the blocks the speculative pass gave up (the redo list);
// one persistent workgroup per CU, most of which find nothing to do.
template <int DG, int NV, bool VEC4, bool FULL>
__global__ __launch_bounds__(DS_THREADS) __attribute__((amdgpu_waves_per_eu(2, 2))) void dense_exact_kernel(
    DenseArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint32_t qbins[];
    const uint32_t n = __builtin_amdgcn_readfirstlane(*(volatile uint32_t *)a.redo_n);
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
        dense_block<DG, NV, VEC4, FULL, true>(a, (int64_t)a.redo_list[i], qbins);
        __syncthreads();
    }
}

// Fallback when not even one sketch window fits in LDS: float atomics in HBM.
__global__ __launch_bounds__(256) void dense_scatter_global_kernel(DenseArgs a) {
    const int64_t total = a.rows * a.I0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < total; l += stride) {
        const float x = a.T[l];
        int64_t rem = l;
        int64_t idx[FCS_MAX_ORDER];
        for (int n = 0; n < a.N; ++n) {
            idx[n] = rem % a.I[n];
            rem /= a.I[n];
        }
        for (int d = 0; d < a.D; ++d) {
            int64_t H = 0;
            uint32_t S = 0;
            for (int n = 0; n < a.N; ++n) {
                const uint32_t p = a.tab[(int64_t)d * a.sumI + a.off[n] + idx[n]];
                H += p & FCS_H_MASK;
                S ^= p & FCS_S_BIT;
            }
            unsafeAtomicAdd(a.out + (int64_t)d * a.Jt + H, __uint_as_float(__float_as_uint(x) ^ S));
        }
    }
}

struct DenseLaunch {
    int dg = 0;              // 0: global fallback
    bool windowed = false;
    int64_t W = 0;
    int64_t slab_rows = 0, block_rows = 0, blocks_per_slab = 0, row_blocks = 0;
    int segs = 0, seg_blocks = 1, segs_per_block = 0;
};

// A thread keeps the bins t + 1024 m (m < MAXACC / DG) of each of the DG
// windows in registers: fewer sketches per group when a window needs more.
static int fit_accumulators(int64_t W, int dg) {
    while (dg >= 1 && (int64_t)dg * fcs_ceil_div(W, DS_THREADS) > MAXACC) --dg;
    return std::max(dg, 0);
}

DenseLaunch plan_dense(const fcs_plan *p) {
    DenseLaunch L;
    int64_t rows = 1;
    for (int n = 1; n < p->N; ++n) rows *= p->I[n];
    const int64_t I0 = p->I[0];
    L.segs = (int)fcs_ceil_div(I0, SEG);
    // bins of DG windows plus the row table of one flush period
    const size_t budget = std::min<size_t>(FCS_LDS_BYTES - 1024 - ROWTAB_BYTES, (size_t)MAXACC * DS_THREADS * 4);
    const int64_t total = rows * I0;
    // windowed: a row block never spans two values of the last mode
    // a single row may not add more than ADD_BOUND elements to one bin
    if (4 * p->m0 > ADD_BOUND) return L;
    if (p->N >= 2) {
        const int64_t Wwin = p->Jt - p->J[p->N - 1] + 1;
        const int64_t slab_rows = rows / p->I[p->N - 1];
        if ((double)slab_rows * (double)I0 >= 16.0 * (double)Wwin) {
            int dg = (int)std::min<int64_t>(4, (int64_t)(budget / (4 * Wwin)));
            dg = fit_accumulators(Wwin, std::min(dg, p->D));
            if (dg >= 1) {
                L.dg = dg;
                L.windowed = true;
                L.W = Wwin;
                L.slab_rows = slab_rows;
                // split a slab only when there are too few slabs to fill the
                // chip, and keep >= 128 elements per bin per block (each block
                // ends with one flush of its window)
                const int64_t elems = slab_rows * I0;
                int64_t bps = fcs_ceil_div(1024, p->I[p->N - 1]);
                bps = std::min<int64_t>(bps, std::max<int64_t>(1, elems / (128 * Wwin)));
                bps = std::max<int64_t>(1, std::min<int64_t>(bps, slab_rows));
                L.block_rows = fcs_ceil_div(slab_rows, bps);
                L.blocks_per_slab = fcs_ceil_div(slab_rows, L.block_rows);
                L.row_blocks = L.blocks_per_slab * p->I[p->N - 1];
                L.segs_per_block = std::min(L.segs, DS_WAVES);
                L.seg_blocks = (int)fcs_ceil_div(L.segs, L.segs_per_block);
                return L;
            }
        }
    }
    int dg = (int)std::min<int64_t>(4, (int64_t)(budget / (4 * p->Jt)));
    dg = fit_accumulators(p->Jt, std::min(dg, p->D));
    if (dg < 1) return L;   // global fallback
    L.dg = dg;
    L.windowed = false;
    L.W = p->Jt;
    L.slab_rows = rows;
    // enough blocks to fill the chip, each sketching many more elements than
    // it has bins; few long rows are split by column segments instead
    int64_t nb = std::max<int64_t>(1, std::min<int64_t>(total / std::max<int64_t>(1, 16 * p->Jt), 2048));
    const int64_t rb = std::min(nb, rows);
    L.block_rows = fcs_ceil_div(rows, rb);
    L.row_blocks = fcs_ceil_div(rows, L.block_rows);
    const int64_t sb = std::max<int64_t>(1, std::min<int64_t>(nb / L.row_blocks, L.segs));
    // whole lane-order sets of GSEG segments per block
    L.segs_per_block = std::min<int>((int)fcs_ceil_div(fcs_ceil_div(L.segs, sb), GSEG) * GSEG, DS_WAVES);
    L.seg_blocks = (int)fcs_ceil_div(L.segs, L.segs_per_block);
    L.blocks_per_slab = L.row_blocks;
    return L;
}

// Kernels that use more than 64 KB of dynamic LDS opt in to that amount
// (static LDS of the kernel comes on top, within the 160 KB of a CU).
template <typename K>
void allow_lds(K kernel, size_t bytes) {
    fcs_allow_lds(reinterpret_cast<const void *>(kernel), bytes);
}

template <int DG, int NV>
void launch_dense_nv(const DenseArgs &a, bool vec4, size_t lds, unsigned grid, unsigned exact_grid, hipStream_t s) {
    if (vec4 && a.I0 % SEG == 0) {
        // every segment complete: the fast instance
        allow_lds(dense_scatter_kernel<DG, NV, true, true>, lds);
        allow_lds(dense_exact_kernel<DG, NV, true, true>, lds);
        hipLaunchKernelGGL((dense_scatter_kernel<DG, NV, true, true>), dim3(grid), dim3(DS_THREADS), lds, s, a);
        hipLaunchKernelGGL((dense_exact_kernel<DG, NV, true, true>), dim3(exact_grid), dim3(DS_THREADS), lds, s, a);
    } else {
        allow_lds(dense_scatter_kernel<DG, NV, false, false>, lds);
        allow_lds(dense_exact_kernel<DG, NV, false, false>, lds);
        hipLaunchKernelGGL((dense_scatter_kernel<DG, NV, false, false>), dim3(grid), dim3(DS_THREADS), lds, s, a);
        hipLaunchKernelGGL((dense_exact_kernel<DG, NV, false, false>), dim3(exact_grid), dim3(DS_THREADS), lds, s,
                           a);
    }
}

template <int DG>
void launch_dense(const DenseArgs &a, bool vec4, size_t lds, unsigned grid, unsigned exact_grid, hipStream_t s) {
    switch (a.nrow_modes) {
    case 0: launch_dense_nv<DG, 0>(a, vec4, lds, grid, exact_grid, s); break;
    case 1: launch_dense_nv<DG, 1>(a, vec4, lds, grid, exact_grid, s); break;
    case 2: launch_dense_nv<DG, 2>(a, vec4, lds, grid, exact_grid, s); break;
    case 3: launch_dense_nv<DG, 3>(a, vec4, lds, grid, exact_grid, s); break;
    case 4: launch_dense_nv<DG, 4>(a, vec4, lds, grid, exact_grid, s); break;
    case 5: launch_dense_nv<DG, 5>(a, vec4, lds, grid, exact_grid, s); break;
    case 6: launch_dense_nv<DG, 6>(a, vec4, lds, grid, exact_grid, s); break;
    default: launch_dense_nv<DG, 7>(a, vec4, lds, grid, exact_grid, s); break;
    }
}

// ---------------------------------------------------------------------------
// COO kernel.  Each workgroup holds the hash tables of DG sketches and their
// full J~ bins in LDS and streams a contiguous range of entries.  Entries are
// rounded to 32-bit integers at a per-workgroup power-of-two scale and added
// to 32-bit two's-complement bins with returning LDS atomics.  The returned
// old value shows exactly when an addition wraps a bin past the signed
// range: the bin's true sum then differs from its 32-bit value by one more
// +-2^32, which is added to the sketch at once as a float (rare: a bin
// collects a few hundred entries of magnitude below 2^28 per workgroup).
// The hash words of the group's sketches are interleaved per index, so one
// LDS read serves every sketch of the group.
// Precision does not depend on how well the sampled scale fits the data: an
// entry takes the fixed-point path only when |x 2^F| lies in [2^16, 2^31),
// so rounding moves it by at most 2^-17 of its own magnitude (the expected
// squared error of a sketch is then at most 2^-34 of the tensor's squared
// 2-norm, relative error 7.6e-6, over the hash signs).  Smaller nonzero
// entries, larger ones, NaN and Inf are added as floats to the HBM sketch.
// For Gaussian data about 0.1 % of the entries fall below the range.
// ---------------------------------------------------------------------------
constexpr int COO_THREADS = 1024;
constexpr float QLIM32 = 2147483520.0f;   // largest float below 2^31
constexpr float QMIN32 = 65536.0f;        // 2^16: smaller entries take the float path
constexpr int COO_TOP = 28;               // sample max maps into [2^27, 2^28)

struct CooArgs {
    const int32_t *idx;
    const float *val;
    float *out;
    const uint32_t *tab;
    int64_t off[FCS_MAX_ORDER];
    int64_t sumI;
    int64_t nnz;
    int64_t chunk;         // entries per workgroup
    int64_t nchunks;
    int64_t Jt;
    int N, D, ngroups;
};

// hash words of the DG sketches of index row `r` of the interleaved table
template <int DG>
__device__ __forceinline__ void coo_words(const uint32_t *tabs, int r, uint32_t (&w)[DG]) {
    if constexpr (DG == 2) {
        const uint2 v = *reinterpret_cast<const uint2 *>(tabs + 2 * r);
        w[0] = v.x;
        w[1] = v.y;
    } else if constexpr (DG == 4) {
        const uint4 v = *reinterpret_cast<const uint4 *>(tabs + 4 * r);
        w[0] = v.x;
        w[1] = v.y;
        w[2] = v.z;
        w[3] = v.w;
    } else {
#pragma unroll
        for (int d = 0; d < DG; ++d) w[d] = tabs[DG * r + d];
    }
}

template <int DG>
__global__ __launch_bounds__(COO_THREADS) void coo_scatter_kernel(CooArgs a) {
    extern __shared__ uint32_t smem32[];
    const int sumI = (int)a.sumI;
    const int Jt = (int)a.Jt;
    uint32_t *bins = smem32;                                        // DG x Jt
    uint32_t *tabs = smem32 + (((size_t)DG * Jt + 3) & ~(size_t)3);  // sumI x DG, 16-byte aligned
    __shared__ float wave_max[COO_THREADS / 64];
    const int64_t span = (int64_t)NXCD * a.ngroups;
    const int64_t super = blockIdx.x / span;
    const int64_t rem = blockIdx.x - super * span;
    const int grp = (int)(rem / NXCD);
    const int64_t chunk = super * NXCD + (rem % NXCD);
    if (chunk >= a.nchunks) return;
    const int d0 = grp * DG;
    const int nd = min(DG, a.D - d0);
    for (int k = threadIdx.x; k < DG * sumI; k += COO_THREADS) {
        const int i = k / DG, d = k - i * DG;
        tabs[k] = d < nd ? a.tab[(int64_t)(d0 + d) * a.sumI + i] : 0u;
    }
    for (int k = threadIdx.x; k < DG * Jt; k += COO_THREADS) bins[k] = 0u;
    const int64_t k0 = chunk * a.chunk;
    const int64_t k1 = min(k0 + a.chunk, a.nnz);
    // scale from the largest magnitude among the chunk's first 16K entries
    {
        float m = 0.f;
        for (int64_t k = k0 + threadIdx.x; k < min<int64_t>(k1, k0 + 16384); k += COO_THREADS)
            m = fmaxf(m, fabsf(a.val[k]));
        if (!(m <= 3.0e38f)) m = 0.f;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
        if ((threadIdx.x & 63) == 0) wave_max[threadIdx.x / 64] = m;
    }
    __syncthreads();
    float M0 = 0.f;
    for (int w = 0; w < COO_THREADS / 64; ++w) M0 = fmaxf(M0, wave_max[w]);
    int F = COO_TOP - 1;
    if (M0 > 0.f) F = COO_TOP - __builtin_amdgcn_frexp_expf(M0);
    F = max(-100, min(100, F));
    const float scale = ldexpf(1.0f, F);
    const float wrap = ldexpf(1.0f, 32 - F);           // one wrap of a bin, in sketch units

    // U entries per thread per step: their coordinate and value loads are
    // all issued before any is used, and their returning atomics before any
    // result is checked, so one workgroup per CU keeps enough of both in
    // flight (16 against 8: 1.19 against 1.29 ms on 1.07e8 entries, D = 8;
    // 32 spills, and so do 16 with more than two sketches per group)
    constexpr int U = DG <= 2 ? 16 : 8;
    // entries of the chunk are indexed in 32 bits from its start, and the
    // hash words of the modes are added as packed words: their hash parts
    // sum below J~ < 2^31, so bit 31 of the sum is the sign of the product
    const int nloc = (int)(k1 - k0);
    const float *vals = a.val + k0;
    for (int kb = threadIdx.x; kb < nloc; kb += COO_THREADS * U) {
        float x[U];
        uint32_t Wd[U][DG];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = kb + u * COO_THREADS;
            x[u] = k < nloc ? vals[k] : 0.f;
#pragma unroll
            for (int d = 0; d < DG; ++d) Wd[u][d] = 0u;
        }
        for (int n = 0; n < a.N; ++n) {
            const int32_t *col = a.idx + (int64_t)n * a.nnz + k0;
            int ix[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = kb + u * COO_THREADS;
                ix[u] = (k < nloc ? col[k] : 0) + (int)a.off[n];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                uint32_t w[DG];
                coo_words<DG>(tabs, ix[u], w);
#pragma unroll
                for (int d = 0; d < DG; ++d) Wd[u][d] += w[d];
            }
        }
        int q[U][DG];
        uint32_t old[U][DG];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool live = kb + u * COO_THREADS < nloc;
            const float xs = x[u] * scale;
            const float ax = fabsf(xs);
            const bool ok = ax >= QMIN32 && ax < QLIM32;
            const bool flt = !ok && x[u] != 0.f;     // NaN and Inf too
#pragma unroll
            for (int d = 0; d < DG; ++d) {
                const int H = (int)(Wd[u][d] & FCS_H_MASK);
                const uint32_t S = Wd[u][d] & FCS_S_BIT;
                q[u][d] = 0;
                old[u][d] = 0u;
                if (live && d < nd) {
                    if (ok) {
                        q[u][d] = cvt_rpi(__uint_as_float(__float_as_uint(xs) ^ S));
                        old[u][d] = __hip_atomic_fetch_add(&bins[d * Jt + H], (uint32_t)q[u][d],
                                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    } else if (flt) {
                        unsafeAtomicAdd(a.out + (int64_t)(d0 + d) * a.Jt + H,
                                        __uint_as_float(__float_as_uint(x[u]) ^ S));
                    }
                }
            }
        }
        // an addition that carried the bin past the signed 32-bit range
        // (operands of one sign, result of the other) owes it +-2^32
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int d = 0; d < DG; ++d) {
                const uint32_t nw = old[u][d] + (uint32_t)q[u][d];
                if ((old[u][d] ^ nw) & ((uint32_t)q[u][d] ^ nw) & 0x80000000u)
                    unsafeAtomicAdd(a.out + (int64_t)(d0 + d) * a.Jt + (int)(Wd[u][d] & FCS_H_MASK),
                                    q[u][d] > 0 ? wrap : -wrap);
            }
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nd * Jt; k += COO_THREADS) {
        const int qv = (int)bins[k];
        if (qv != 0) {
            const int d = k / Jt;
            unsafeAtomicAdd(a.out + (int64_t)(d0 + d) * a.Jt + (k - d * Jt), ldexpf((float)qv, -F));
        }
    }
}

__global__ __launch_bounds__(256) void coo_scatter_global_kernel(CooArgs a) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < a.nnz; k += stride) {
        const float x = a.val[k];
        for (int d = 0; d < a.D; ++d) {
            int64_t H = 0;
            uint32_t S = 0;
            for (int n = 0; n < a.N; ++n) {
                const uint32_t p = a.tab[(int64_t)d * a.sumI + a.off[n] + a.idx[(int64_t)n * a.nnz + k]];
                H += p & FCS_H_MASK;
                S ^= p & FCS_S_BIT;
            }
            unsafeAtomicAdd(a.out + (int64_t)d * a.Jt + H, __uint_as_float(__float_as_uint(x) ^ S));
        }
    }
}

int coo_dg(const fcs_plan *p) {
    const size_t budget = FCS_LDS_BYTES - 1024 - 16;
    const size_t per_d = 4 * (size_t)p->Jt + 4 * (size_t)p->sumI;
    int dg = (int)std::min<size_t>(4, budget / per_d);
    return std::min(dg, p->D);
}

}  // namespace

// Lane order of the dense kernel.  A wave issues each LDS atomic as two
// half-waves (lanes 0-31, 32-63), and a half-wave takes as many passes as
// the largest number of its lanes that hit one of the 32 LDS banks.  A lane
// keeps its 4 consecutive columns (one 16-byte load), and in sketch d the
// bank of column c is h_0(c) plus a row-uniform offset (mod 32), so the
// assignment of column blocks to half-waves fixes the conflicts of every
// row.  Within each set of GSEG segments (1024 columns, processed by GSEG
// waves of one workgroup), the set's blocks may go to any half-wave of those
// waves; any assignment is correct (each block is still loaded and added
// exactly once per row), and a local search picks one with a small sum, over
// the group's sketches and a block's 4 columns, of the largest bank load per
// half-wave.  Entry (group, segment, lane) holds the lane's block index
// within its set.
int fcs_dense_group_size(const fcs_plan *p) { return plan_dense(p).dg; }

size_t fcs_dense_perm_bytes(const fcs_plan *p) {
    const int64_t I0 = p->I[0];
    const int64_t segs = fcs_ceil_div(I0, SEG);
    if ((double)I0 * (double)p->D > 16777216.0 || segs * p->D > 65536) return 0;
    return (size_t)p->D * (size_t)segs * 64;
}

void fcs_dense_lane_order(const fcs_plan *p, const uint32_t *h0, uint8_t *perm) {
    const int64_t I0 = p->I[0];
    const int segs = (int)fcs_ceil_div(I0, SEG);
    // identity: lane l of segment s loads block (s % GSEG) * 64 + l of its set
    for (size_t k = 0; k < p->perm_bytes; ++k)
        perm[k] = (uint8_t)((((k / 64) % (size_t)segs) % GSEG) * 64 + k % 64);
    const DenseLaunch L = plan_dense(p);
    if (L.dg == 0) return;
    const int ngroups = (p->D + L.dg - 1) / L.dg;
    const int nsets = (segs + GSEG - 1) / GSEG;
    constexpr int MAX_SEARCHED = 16;     // (group, set) pairs searched; the rest keep the identity
    constexpr int ITERS = 100000;
    constexpr int NB = GSEG * 64;        // blocks of a full set
    constexpr int NH = 2 * GSEG;         // half-waves of a full set
    // per (half-wave, sketch-column pair): bank counts, how many banks hold
    // each count, and the largest count (kept exactly under +-1 updates)
    struct Hist {
        int cnt[32];
        int at[34];
        int mx;
    };
    std::vector<int> bank((size_t)NB * 16);
    std::vector<Hist> hist((size_t)NH * 16);
    int searched = 0;
    for (int gi = 0; gi < ngroups; ++gi) {
        const int d0 = gi * L.dg;
        const int nk = 4 * std::min(L.dg, p->D - d0);   // (sketch, column) pairs of a block
        for (int st = 0; st < nsets && searched < MAX_SEARCHED; ++st, ++searched) {
            const int ns = std::min(GSEG, segs - st * GSEG);   // segments (waves) in this set
            const int nb = ns * 64, nh = 2 * ns;
            if (nh < 2) continue;
            for (int b = 0; b < nb; ++b)
                for (int k = 0; k < nk; ++k) {
                    const int64_t c = (int64_t)st * GSEG * SEG + 4 * b + (k & 3);
                    bank[(size_t)b * 16 + k] = c < I0 ? (int)(h0[(size_t)(d0 + (k >> 2)) * I0 + c] & 31u) : -1;
                }
            std::vector<int> order(nb);
            for (int b = 0; b < nb; ++b) order[b] = b;
            for (int h = 0; h < nh; ++h)
                for (int k = 0; k < nk; ++k) {
                    Hist &t = hist[(size_t)h * 16 + k];
                    std::fill(t.cnt, t.cnt + 32, 0);
                    std::fill(t.at, t.at + 34, 0);
                    t.at[0] = 32;
                    t.mx = 0;
                }
            auto inc = [&](Hist &t, int b) {
                const int v = t.cnt[b]++;
                --t.at[v];
                ++t.at[v + 1];
                if (v + 1 > t.mx) t.mx = v + 1;
            };
            auto dec = [&](Hist &t, int b) {
                const int v = t.cnt[b]--;
                --t.at[v];
                ++t.at[v - 1];
                if (v == t.mx && t.at[v] == 0) t.mx = v - 1;
            };
            for (int b = 0; b < nb; ++b)
                for (int k = 0; k < nk; ++k)
                    if (bank[(size_t)b * 16 + k] >= 0) inc(hist[(size_t)(b >> 5) * 16 + k], bank[(size_t)b * 16 + k]);
            uint64_t rs = p->seed ^ ((uint64_t)gi << 32) ^ (uint64_t)st;
            for (int it = 0; it < ITERS; ++it) {
                rs += 0x9E3779B97F4A7C15ull;
                uint64_t z = rs;
                z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
                z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
                z ^= z >> 31;
                const int i = (int)(z % (uint64_t)nb), j = (int)((z >> 24) % (uint64_t)nb);
                const int hi = i >> 5, hj = j >> 5;
                if (hi == hj) continue;
                const int bi = order[i], bj = order[j];
                int delta = 0;
                auto move = [&](int bfrom, int hfrom, int hto) {
                    for (int k = 0; k < nk; ++k) {
                        const int bk = bank[(size_t)bfrom * 16 + k];
                        if (bk < 0) continue;
                        Hist &a = hist[(size_t)hfrom * 16 + k], &c = hist[(size_t)hto * 16 + k];
                        delta -= a.mx + c.mx;
                        dec(a, bk);
                        inc(c, bk);
                        delta += a.mx + c.mx;
                    }
                };
                move(bi, hi, hj);
                move(bj, hj, hi);
                if (delta <= 0) {
                    order[i] = bj;
                    order[j] = bi;
                } else {
                    move(bj, hi, hj);
                    move(bi, hj, hi);
                }
            }
            for (int ls = 0; ls < ns; ++ls)
                for (int l = 0; l < 64; ++l)
                    perm[((size_t)gi * segs + st * GSEG + ls) * 64 + l] = (uint8_t)order[ls * 64 + l];
        }
    }
}

// The lane order is searched on the host and uploaded on the plan's first
// dense sketch (one synchronisation of that stream).  A call made while the
// stream is being captured into a graph uses the identity order (same
// result, more bank conflicts).  Returns whether the order is on the device.
static bool dense_lane_order(fcs_plan *p, hipStream_t s) {
    static std::mutex mu;
    std::lock_guard<std::mutex> lock(mu);
    if (!p->perm_bytes || p->perm_ready) return p->perm_ready;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return false;
    std::vector<uint32_t> h0((size_t)p->D * (size_t)p->I[0]);
    fcs_mode0_hashes(p, h0.data());
    std::vector<uint8_t> perm(p->perm_bytes);
    fcs_dense_lane_order(p, h0.data(), perm.data());
    if (hipMemcpyAsync((void *)p->perm, perm.data(), perm.size(), hipMemcpyHostToDevice, s) != hipSuccess) return false;
    if (hipStreamSynchronize(s) != hipSuccess) return false;
    p->perm_ready = true;
    return true;
}

// Dense workspace: REDO_HEAD header words (the redo-list lengths of the two
// launch passes, full sketch groups and the tail group), then one redo list
// per pass with room for every block of its launch.
static int64_t dense_pass_grid(const fcs_plan *p, const DenseLaunch &L, int pass) {
    if (L.dg == 0) return 0;
    const int full_groups = p->D / L.dg;
    const int groups = pass == 0 ? full_groups : ((p->D - full_groups * L.dg) ? 1 : 0);
    const int64_t nblocks = L.row_blocks * L.seg_blocks;
    return fcs_ceil_div(nblocks, NXCD) * NXCD * groups;
}

size_t fcs_ws_dense(const fcs_plan *p) {
    const DenseLaunch L = plan_dense(p);
    const int64_t words = REDO_HEAD + dense_pass_grid(p, L, 0) + dense_pass_grid(p, L, 1);
    return ((size_t)words * 4 + 255) & ~(size_t)255;
}
size_t fcs_ws_coo(const fcs_plan *) { return 256; }

extern "C" fcs_status fcs_sketch_dense(fcs_plan_t p, const float *T, float *out, void *ws,
                                       size_t ws_bytes, void *stream) {
    fcs_clear_error();
    if (!p || !p->bound) FCS_FAIL(FCS_EINVAL, "plan is null or not bound");
    if (!T || !out) FCS_FAIL(FCS_EINVAL, "null tensor or output");
    const size_t need = fcs_ws_dense(p);
    if (!ws || ws_bytes < need) FCS_FAIL(FCS_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
    if (!fcs_aligned(ws, 4)) FCS_FAIL(FCS_EINVAL, "workspace not 4-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    const DenseLaunch L = plan_dense(p);
    DenseArgs a{};
    a.T = T;
    a.out = out;
    a.tab = p->tab;
    for (int n = 0; n < FCS_MAX_ORDER; ++n) {
        a.I[n] = n < p->N ? (int32_t)p->I[n] : 1;
        a.off[n] = n < p->N ? p->off[n] : 0;
    }
    a.sumI = p->sumI;
    a.I0 = p->I[0];
    a.rows = 1;
    for (int n = 1; n < p->N; ++n) a.rows *= p->I[n];
    a.Jt = p->Jt;
    a.N = p->N;
    a.D = p->D;
    fcs_status st = fcs_zero_fill(out, (int64_t)p->D * p->Jt, s);
    if (st != FCS_OK) return st;
    if (L.dg == 0) {
        const int64_t total = a.rows * a.I0;
        unsigned grid = (unsigned)std::min<int64_t>(fcs_ceil_div(total, 256), 65536);
        dense_scatter_global_kernel<<<grid, 256, 0, s>>>(a);
        FCS_LAUNCH_CHECK();
        return FCS_OK;
    }
    a.slab_rows = L.slab_rows;
    a.block_rows = L.block_rows;
    a.blocks_per_slab = L.blocks_per_slab;
    a.row_blocks = L.row_blocks;
    a.W = (int)L.W;
    a.windowed = L.windowed ? 1 : 0;
    a.nrow_modes = L.windowed ? p->N - 2 : p->N - 1;
    a.segs = L.segs;
    a.seg_blocks = L.seg_blocks;
    a.segs_per_block = L.segs_per_block;
    a.period = (int)std::max<int64_t>(1, ADD_BOUND / std::max(1, p->m0));
    a.dg_full = L.dg;
    a.perm = dense_lane_order(p, s) ? p->perm : nullptr;
    const bool vec4 = (a.I0 % 4 == 0) && fcs_aligned(T, 16);
    const int full_groups = p->D / L.dg;
    const int tail = p->D - full_groups * L.dg;
    const int64_t nblocks = L.row_blocks * L.seg_blocks;
    const int64_t blocks_rounded = fcs_ceil_div(nblocks, NXCD) * NXCD;
    // redo lists of the speculative pass, cleared by a kernel (no memset
    // node when the call is captured into a graph)
    uint32_t *wsw = static_cast<uint32_t *>(ws);
    st = fcs_zero_fill(reinterpret_cast<float *>(wsw), REDO_HEAD, s);
    if (st != FCS_OK) return st;
    const unsigned exact_grid = (unsigned)std::max(1, fcs_device_cu_count());
    for (int pass = 0; pass < 2; ++pass) {
        const int dg = pass == 0 ? L.dg : tail;
        const int groups = pass == 0 ? full_groups : (tail ? 1 : 0);
        if (groups == 0) continue;
        a.ngroups = groups;
        a.d_first = pass == 0 ? 0 : full_groups * L.dg;
        const int64_t grid64 = blocks_rounded * groups;
        if (grid64 > INT32_MAX) FCS_FAIL(FCS_EUNSUPPORTED, "grid too large");
        a.redo_n = wsw + pass;
        a.redo_list = wsw + REDO_HEAD + (pass == 0 ? 0 : dense_pass_grid(p, L, 0));
        // bins, the row table of a period and the give-up flag
        const size_t lds = (((size_t)dg * (size_t)L.W + 3) & ~(size_t)3) * sizeof(uint32_t) + 16 * (size_t)a.period +
                           16;
        switch (dg) {
        case 1: launch_dense<1>(a, vec4, lds, (unsigned)grid64, exact_grid, s); break;
        case 2: launch_dense<2>(a, vec4, lds, (unsigned)grid64, exact_grid, s); break;
        case 3: launch_dense<3>(a, vec4, lds, (unsigned)grid64, exact_grid, s); break;
        default: launch_dense<4>(a, vec4, lds, (unsigned)grid64, exact_grid, s); break;
        }
        FCS_LAUNCH_CHECK();
    }
    return FCS_OK;
}

extern "C" fcs_status fcs_sketch_coo(fcs_plan_t p, int64_t nnz, const int32_t *idx, const float *val,
                                     float *out, void *ws, size_t ws_bytes, void *stream) {
    fcs_clear_error();
    if (!p || !p->bound) FCS_FAIL(FCS_EINVAL, "plan is null or not bound");
    if (nnz < 0) FCS_FAIL(FCS_EINVAL, "nnz < 0");
    if (!out) FCS_FAIL(FCS_EINVAL, "null output");
    if (nnz > 0 && (!idx || !val)) FCS_FAIL(FCS_EINVAL, "null coordinates or values");
    (void)ws;
    (void)ws_bytes;
    hipStream_t s = (hipStream_t)stream;
    fcs_status st = fcs_zero_fill(out, (int64_t)p->D * p->Jt, s);
    if (st != FCS_OK || nnz == 0) return st;
    CooArgs a{};
    a.idx = idx;
    a.val = val;
    a.out = out;
    a.tab = p->tab;
    for (int n = 0; n < FCS_MAX_ORDER; ++n) a.off[n] = n < p->N ? p->off[n] : 0;
    a.sumI = p->sumI;
    a.nnz = nnz;
    a.Jt = p->Jt;
    a.N = p->N;
    a.D = p->D;
    const int dg = coo_dg(p);
    if (dg < 1) {
        unsigned grid = (unsigned)std::min<int64_t>(fcs_ceil_div(nnz, 256), 65536);
        coo_scatter_global_kernel<<<grid, 256, 0, s>>>(a);
        FCS_LAUNCH_CHECK();
        return FCS_OK;
    }
    a.ngroups = (int)fcs_ceil_div(p->D, dg);
    // chunks: each workgroup streams many more entries than it has bins
    int64_t nchunks = std::max<int64_t>(1, std::min<int64_t>(nnz / std::max<int64_t>(1, 8 * p->Jt),
                                                             (int64_t)2048 / a.ngroups + 1));
    // the kernel indexes a chunk's entries in 32 bits
    nchunks = std::max<int64_t>(nchunks, fcs_ceil_div(nnz, (int64_t)1 << 30));
    a.chunk = fcs_ceil_div(nnz, nchunks);
    a.nchunks = fcs_ceil_div(nnz, a.chunk);
    const size_t lds = ((((size_t)dg * p->Jt + 3) & ~(size_t)3) + (size_t)dg * p->sumI) * 4;
    const unsigned grid = (unsigned)(fcs_ceil_div(a.nchunks, NXCD) * NXCD * a.ngroups);
    allow_lds(coo_scatter_kernel<1>, lds);
    allow_lds(coo_scatter_kernel<2>, lds);
    allow_lds(coo_scatter_kernel<3>, lds);
    allow_lds(coo_scatter_kernel<4>, lds);
    switch (dg) {
    case 1: hipLaunchKernelGGL(coo_scatter_kernel<1>, dim3(grid), dim3(COO_THREADS), lds, s, a); break;
    case 2: hipLaunchKernelGGL(coo_scatter_kernel<2>, dim3(grid), dim3(COO_THREADS), lds, s, a); break;
    case 3: hipLaunchKernelGGL(coo_scatter_kernel<3>, dim3(grid), dim3(COO_THREADS), lds, s, a); break;
    default: hipLaunchKernelGGL(coo_scatter_kernel<4>, dim3(grid), dim3(COO_THREADS), lds, s, a); break;
    }
    FCS_LAUNCH_CHECK();
    return FCS_OK;
}
