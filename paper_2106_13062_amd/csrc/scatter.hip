// Dense and COO fast count sketch: the general-tensor formula of Section 3.2.
//
// Every element T[i_0..i_{N-1}] is added with sign S = prod_n s_n(i_n) to bin
// H = sum_n h_n(i_n) of each of the D sketches.  The long hash (H, S) of
// Definition 4 is never built: only the N short tables are read.
//
// Dense kernel design (gfx950):
//  * vec(T) is a sequence of rows along mode 0 (I_0 contiguous floats).  Along
//    a row, H = c(row) + h_0(i_0): the offset c and the row sign depend only
//    on the row, so they are wave-uniform scalars, and the per-column part
//    h_0 / s_0 of a wave's columns is fixed for all rows it visits.
//  * A wave owns a 512-column segment of the rows it visits (8 floats per
//    lane, two 16-byte loads); its lanes keep, for every sketch of the
//    workgroup, the LDS byte address of bin h_0(i_0) and the sign mask of
//    s_0(i_0) in registers.  Per element and sketch the hot loop is one
//    v_add (address + row offset), one v_bitop3 (value ^ column sign ^ row
//    sign) and one LDS float atomic add.
//  * Bins are privatised in LDS per workgroup.  When N >= 2 a workgroup's rows
//    share the last-mode index, so its bins lie in the window
//    h_{N-1}(i_{N-1}) + [0, J~ - J_{N-1} + 1) and only that window is held;
//    the sketches are split into groups of DG so DG windows fit in LDS.
//    At the end the window is added to the HBM sketch with coalesced float
//    atomics.
//  * The two (or more) sketch groups of one slab are dispatched to the same
//    XCD back to back (workgroups go round-robin over the 8 XCDs), so the
//    second read of the slab is served from that XCD's L2.
#include "fcs_internal.h"

#include <algorithm>

namespace {

constexpr int DS_THREADS = 1024;     // 16 waves
constexpr int DS_WAVES = DS_THREADS / 64;
constexpr int SEG = 512;             // columns of a wave segment
constexpr int NXCD = 8;

struct DenseArgs {
    const float *T;
    float *out;
    const uint32_t *tab;
    int64_t I[FCS_MAX_ORDER];
    int64_t off[FCS_MAX_ORDER];
    int64_t sumI;
    int64_t I0;
    int64_t rows;          // prod_{n>=1} I_n
    int64_t slab_rows;     // rows sharing one last-mode index (windowed mode)
    int64_t block_rows;    // rows per workgroup block
    int64_t blocks_per_slab;
    int64_t nblocks;
    int64_t Jt;
    int64_t W;             // bins held per sketch in LDS
    int N;
    int D;
    int ngroups;           // groups of DG sketches in this launch
    int d_first;           // first sketch of this launch
    int windowed;          // 1: window anchored at h_{N-1}(i_{N-1})
    int segs;              // ceil(I0 / SEG)
};

// Map the flat block id to (row block, sketch group) so that all groups of a
// row block land on one XCD consecutively.
__device__ inline void dense_block_map(const DenseArgs &a, int64_t bid, int64_t &blk, int &grp) {
    const int64_t span = (int64_t)NXCD * a.ngroups;
    const int64_t super = bid / span;
    const int64_t rem = bid - super * span;
    grp = (int)(rem / NXCD);
    blk = super * NXCD + (rem % NXCD);
}

// value ^ column sign ^ row sign in one VALU op (three-input xor, gfx950).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// Scatter one row segment of 8 values per lane into the LDS windows of the
// DG sketches.  Row offset C[d] (bytes) and row sign R[d] are wave-uniform.
// Per element and sketch: one v_bitop3, one v_add and one ds_add_f32.
template <int DG, bool CHECK>
__device__ __forceinline__ void scatter_row(float *bins, const float (&x)[8], const uint32_t (&A)[DG][8],
                                            const uint32_t (&M)[DG][8], const bool (&valid)[8],
                                            const uint32_t (&C)[DG], const uint32_t (&R)[DG]) {
#pragma unroll
    for (int d = 0; d < DG; ++d) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            if (!CHECK || valid[e]) {
                const float v = __uint_as_float(xor3(__float_as_uint(x[e]), M[d][e], R[d]));
                float *dst = reinterpret_cast<float *>(reinterpret_cast<char *>(bins) + (A[d][e] + C[d]));
                __hip_atomic_fetch_add(dst, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
    }
}

// Row offset (bytes) and row sign of every sketch of the group, from the
// hash words of modes 1..nvar-1 at the decoded row index.
template <int DG>
__device__ __forceinline__ void row_hash(const DenseArgs &a, int d0, int nvar, const int (&idx)[FCS_MAX_ORDER],
                                         uint32_t (&C)[DG], uint32_t (&R)[DG]) {
    uint32_t w[FCS_MAX_ORDER - 1][DG];
#pragma unroll
    for (int n = 1; n < FCS_MAX_ORDER; ++n) {
        if (n < nvar) {
#pragma unroll
            for (int d = 0; d < DG; ++d)
                w[n - 1][d] = __builtin_nontemporal_load(a.tab + (int64_t)(d0 + d) * a.sumI + a.off[n] + idx[n]);
        }
    }
#pragma unroll
    for (int d = 0; d < DG; ++d) {
        C[d] = 0;
        R[d] = 0;
    }
#pragma unroll
    for (int n = 1; n < FCS_MAX_ORDER; ++n) {
        if (n < nvar) {
#pragma unroll
            for (int d = 0; d < DG; ++d) {
                C[d] += (w[n - 1][d] & FCS_H_MASK) * 4u;
                R[d] ^= w[n - 1][d] & FCS_S_BIT;
            }
        }
    }
}

__device__ __forceinline__ void advance_rows(const DenseArgs &a, int nvar, int step, int (&idx)[FCS_MAX_ORDER]) {
    int carry = step;
#pragma unroll
    for (int n = 1; n < FCS_MAX_ORDER; ++n) {
        if (n < nvar && carry) {
            const uint32_t In = (uint32_t)a.I[n];
            const uint32_t t = (uint32_t)idx[n] + (uint32_t)carry;
            if (t < In) {
                idx[n] = (int)t;
                carry = 0;
            } else {
                idx[n] = (int)(t % In);
                carry = (int)(t / In);
            }
        }
    }
}

template <bool VEC4, bool FULL>
__device__ __forceinline__ void load_row(const float *row, int lane, const bool (&valid)[8], float (&x)[8]) {
    if (FULL && VEC4) {
        const float4 q0 = *reinterpret_cast<const float4 *>(row + lane * 4);
        const float4 q1 = *reinterpret_cast<const float4 *>(row + 256 + lane * 4);
        x[0] = q0.x; x[1] = q0.y; x[2] = q0.z; x[3] = q0.w;
        x[4] = q1.x; x[5] = q1.y; x[6] = q1.z; x[7] = q1.w;
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = (FULL || valid[e]) ? row[(e >> 2) * 256 + lane * 4 + (e & 3)] : 0.f;
    }
}

// All rows [r_first, r1) with stride wps of one segment; the next row's hash
// words and values are in flight while the current row is scattered.
template <int DG, bool VEC4, bool FULL>
__device__ __forceinline__ void segment_rows(const DenseArgs &a, float *bins, int d0, int nvar, int seg, int lane,
                                             int64_t r_first, int64_t r1, int wps, const uint32_t (&A)[DG][8],
                                             const uint32_t (&M)[DG][8], const bool (&valid)[8]) {
    if (r_first >= r1) return;
    int idx[FCS_MAX_ORDER];
    {
        int64_t rem = r_first;
#pragma unroll
        for (int n = 1; n < FCS_MAX_ORDER; ++n) {
            idx[n] = 0;
            if (n < nvar) {
                idx[n] = (int)(rem % a.I[n]);
                rem /= a.I[n];
            }
        }
    }
    const float *Tseg = a.T + (int64_t)seg * SEG;
    uint32_t C[DG], R[DG];
    float x[8];
    row_hash<DG>(a, d0, nvar, idx, C, R);
    load_row<VEC4, FULL>(Tseg + r_first * a.I0, lane, valid, x);
    for (int64_t r = r_first; r < r1; r += wps) {
        const int64_t rn = r + wps;
        uint32_t Cn[DG], Rn[DG];
        float xn[8];
        if (rn < r1) {
            advance_rows(a, nvar, wps, idx);
            row_hash<DG>(a, d0, nvar, idx, Cn, Rn);
            load_row<VEC4, FULL>(Tseg + rn * a.I0, lane, valid, xn);
        }
        scatter_row<DG, !FULL>(bins, x, A, M, valid, C, R);
        if (rn < r1) {
#pragma unroll
            for (int d = 0; d < DG; ++d) {
                C[d] = Cn[d];
                R[d] = Rn[d];
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) x[e] = xn[e];
        }
    }
}

template <int DG, bool VEC4>
__global__ __launch_bounds__(DS_THREADS) void dense_scatter_kernel(DenseArgs a) {
    extern __shared__ float bins[];   // DG x W
    int64_t blk;
    int grp;
    dense_block_map(a, blockIdx.x, blk, grp);
    if (blk >= a.nblocks) return;
    const int d0 = a.d_first + grp * DG;   // this launch covers whole groups of DG sketches

    // row range of this block
    int64_t r0, r1;
    if (a.windowed) {
        const int64_t slab = blk / a.blocks_per_slab;
        const int64_t sub = blk - slab * a.blocks_per_slab;
        r0 = slab * a.slab_rows + sub * a.block_rows;
        r1 = min(r0 + a.block_rows, (slab + 1) * a.slab_rows);
    } else {
        r0 = blk * a.block_rows;
        r1 = min(r0 + a.block_rows, a.rows);
    }

    // window base per sketch: the last-mode hash of this slab
    int base[DG];
    const int last = a.N - 1;
    const int64_t ilast = (a.windowed && a.N >= 2) ? (r0 / a.slab_rows) : 0;
#pragma unroll
    for (int d = 0; d < DG; ++d) {
        base[d] = 0;
        if (a.windowed && a.N >= 2)
            base[d] = (int)(a.tab[(int64_t)(d0 + d) * a.sumI + a.off[last] + ilast] & FCS_H_MASK);
    }

    const int W = (int)a.W;
    for (int k = threadIdx.x; k < DG * W; k += DS_THREADS) bins[k] = 0.f;
    __syncthreads();

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    const int lane = threadIdx.x % 64;
    const int wps = max(1, DS_WAVES / a.segs);             // waves per segment
    const int nvar = a.windowed ? a.N - 1 : a.N;           // modes 1..nvar-1 vary per row

    for (int sidx = wave; sidx < a.segs * wps; sidx += DS_WAVES) {
        const int seg = sidx % a.segs;
        const int rl = sidx / a.segs;
        // per-lane column data of this segment, kept in registers for all rows
        uint32_t A[DG][8], M[DG][8];
        bool valid[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int64_t col = (int64_t)seg * SEG + (e >> 2) * 256 + lane * 4 + (e & 3);
            valid[e] = col < a.I0;
#pragma unroll
            for (int d = 0; d < DG; ++d) {
                const uint32_t p = valid[e] ? a.tab[(int64_t)(d0 + d) * a.sumI + col] : 0u;
                A[d][e] = (uint32_t)((d * W + (int)(p & FCS_H_MASK)) * 4);
                M[d][e] = p & FCS_S_BIT;
            }
        }
        if ((int64_t)(seg + 1) * SEG <= a.I0)   // wave-uniform
            segment_rows<DG, VEC4, true>(a, bins, d0, nvar, seg, lane, r0 + rl, r1, wps, A, M, valid);
        else
            segment_rows<DG, VEC4, false>(a, bins, d0, nvar, seg, lane, r0 + rl, r1, wps, A, M, valid);
    }
    __syncthreads();
    // flush the window into the HBM sketch
    for (int k = threadIdx.x; k < DG * W; k += DS_THREADS) {
        const int d = k / W;
        const int j = k - d * W;
        const float v = bins[k];
        if (v != 0.f) unsafeAtomicAdd(a.out + (int64_t)(d0 + d) * a.Jt + base[d] + j, v);
    }
}

// Fallback when not even one sketch window fits in LDS: global atomics.
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
            unsafeAtomicAdd(a.out + (int64_t)d * a.Jt + H, __int_as_float(__float_as_int(x) ^ S));
        }
    }
}

struct DenseLaunch {
    int dg = 0;            // 0: global fallback
    bool windowed = false;
    int64_t W = 0;
    int64_t slab_rows = 0, block_rows = 0, blocks_per_slab = 0, nblocks = 0;
};

DenseLaunch plan_dense(const fcs_plan *p) {
    DenseLaunch L;
    const int64_t rows = p->sumI > 0 ? [&] {
        int64_t r = 1;
        for (int n = 1; n < p->N; ++n) r *= p->I[n];
        return r;
    }() : 1;
    const int64_t I0 = p->I[0];
    const size_t budget = FCS_LDS_BYTES - 1024;
    // windowed: workgroups never span two values of the last mode
    if (p->N >= 2) {
        const int64_t Wwin = p->Jt - p->J[p->N - 1] + 1;
        const int64_t slab_rows = rows / p->I[p->N - 1];
        // worth it when a slab holds many more elements than window bins
        if ((double)slab_rows * (double)I0 >= 16.0 * (double)Wwin) {
            int dg = (int)std::min<int64_t>(4, budget / (4 * Wwin));
            dg = std::min(dg, p->D);
            if (dg >= 1) {
                L.dg = dg;
                L.windowed = true;
                L.W = Wwin;
                L.slab_rows = slab_rows;
                // split a slab into several blocks only when there are too
                // few slabs to fill the chip, and never below 128 elements
                // per bin (each block ends with one flush of its window)
                const int64_t elems = slab_rows * I0;
                int64_t bps = fcs_ceil_div(1024, p->I[p->N - 1]);
                bps = std::min<int64_t>(bps, std::max<int64_t>(1, elems / (128 * Wwin)));
                bps = std::max<int64_t>(1, std::min<int64_t>(bps, slab_rows));
                L.block_rows = fcs_ceil_div(slab_rows, bps);
                L.blocks_per_slab = fcs_ceil_div(slab_rows, L.block_rows);
                L.nblocks = L.blocks_per_slab * p->I[p->N - 1];
                return L;
            }
        }
    }
    int dg = (int)std::min<int64_t>(4, budget / (4 * p->Jt));
    dg = std::min(dg, p->D);
    if (dg < 1) return L;   // global fallback
    L.dg = dg;
    L.windowed = false;
    L.W = p->Jt;
    L.slab_rows = rows;
    // enough blocks to fill the chip, but each block sketches many more
    // elements than it has bins
    const int64_t total = rows * I0;
    int64_t nb = std::max<int64_t>(1, std::min<int64_t>(total / std::max<int64_t>(1, 16 * p->Jt), 2048));
    nb = std::min(nb, rows);
    L.block_rows = fcs_ceil_div(rows, nb);
    L.nblocks = fcs_ceil_div(rows, L.block_rows);
    L.blocks_per_slab = L.nblocks;
    return L;
}

// Kernels that use more than 64 KB of dynamic LDS opt in once.
template <typename K>
void allow_lds(K kernel, size_t bytes) {
    if (bytes > 65536)
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)FCS_LDS_BYTES);
}

template <int DG>
void launch_dense(const DenseArgs &a, bool vec4, size_t lds, unsigned grid, hipStream_t s) {
    if (vec4) {
        allow_lds(dense_scatter_kernel<DG, true>, lds);
        hipLaunchKernelGGL((dense_scatter_kernel<DG, true>), dim3(grid), dim3(DS_THREADS), lds, s, a);
    } else {
        allow_lds(dense_scatter_kernel<DG, false>, lds);
        hipLaunchKernelGGL((dense_scatter_kernel<DG, false>), dim3(grid), dim3(DS_THREADS), lds, s, a);
    }
}

// ---------------------------------------------------------------------------
// COO kernel: each workgroup holds the hash tables and the full J~ bins of DG
// sketches in LDS and streams a contiguous range of entries.
// ---------------------------------------------------------------------------
constexpr int COO_THREADS = 1024;

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

template <int DG>
__global__ __launch_bounds__(COO_THREADS) void coo_scatter_kernel(CooArgs a) {
    extern __shared__ uint32_t smem[];
    uint32_t *tabs = smem;                                        // DG x sumI
    float *bins = reinterpret_cast<float *>(smem + DG * a.sumI);  // DG x Jt
    const int64_t span = (int64_t)NXCD * a.ngroups;
    const int64_t super = blockIdx.x / span;
    const int64_t rem = blockIdx.x - super * span;
    const int grp = (int)(rem / NXCD);
    const int64_t chunk = super * NXCD + (rem % NXCD);
    if (chunk >= a.nchunks) return;
    const int d0 = grp * DG;
    const int nd = min(DG, a.D - d0);
    const int sumI = (int)a.sumI;
    const int Jt = (int)a.Jt;
    for (int k = threadIdx.x; k < DG * sumI; k += COO_THREADS) {
        const int d = k / sumI;
        tabs[k] = d < nd ? a.tab[(int64_t)(d0 + d) * a.sumI + (k - d * sumI)] : 0u;
    }
    for (int k = threadIdx.x; k < DG * Jt; k += COO_THREADS) bins[k] = 0.f;
    __syncthreads();
    const int64_t k0 = chunk * a.chunk;
    const int64_t k1 = min(k0 + a.chunk, a.nnz);
    for (int64_t k = k0 + threadIdx.x; k < k1; k += COO_THREADS) {
        const float x = a.val[k];
        int ix[FCS_MAX_ORDER];
        for (int n = 0; n < a.N; ++n) ix[n] = a.idx[(int64_t)n * a.nnz + k] + (int)a.off[n];
#pragma unroll
        for (int d = 0; d < DG; ++d) {
            if (d < nd) {
                int H = 0;
                uint32_t S = 0;
                for (int n = 0; n < a.N; ++n) {
                    const uint32_t p = tabs[d * sumI + ix[n]];
                    H += (int)(p & FCS_H_MASK);
                    S ^= p & FCS_S_BIT;
                }
                __hip_atomic_fetch_add(&bins[d * Jt + H], __int_as_float(__float_as_int(x) ^ S),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nd * Jt; k += COO_THREADS) {
        const float v = bins[k];
        if (v != 0.f) {
            const int d = k / Jt;
            unsafeAtomicAdd(a.out + (int64_t)(d0 + d) * a.Jt + (k - d * Jt), v);
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
            unsafeAtomicAdd(a.out + (int64_t)d * a.Jt + H, __int_as_float(__float_as_int(x) ^ S));
        }
    }
}

int coo_dg(const fcs_plan *p) {
    const size_t budget = FCS_LDS_BYTES - 1024;
    const size_t per_d = 4 * ((size_t)p->sumI + (size_t)p->Jt);
    int dg = (int)std::min<size_t>(4, budget / per_d);
    return std::min(dg, p->D);
}

}  // namespace

size_t fcs_ws_dense(const fcs_plan *) { return 256; }
size_t fcs_ws_coo(const fcs_plan *) { return 256; }

extern "C" fcs_status fcs_sketch_dense(fcs_plan_t p, const float *T, float *out, void *ws,
                                       size_t ws_bytes, void *stream) {
    fcs_clear_error();
    if (!p || !p->bound) FCS_FAIL(FCS_EINVAL, "plan is null or not bound");
    if (!T || !out) FCS_FAIL(FCS_EINVAL, "null tensor or output");
    (void)ws;
    (void)ws_bytes;
    hipStream_t s = (hipStream_t)stream;
    const DenseLaunch L = plan_dense(p);
    DenseArgs a{};
    a.T = T;
    a.out = out;
    a.tab = p->tab;
    for (int n = 0; n < FCS_MAX_ORDER; ++n) {
        a.I[n] = n < p->N ? p->I[n] : 1;
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
    a.nblocks = L.nblocks;
    a.W = L.W;
    a.windowed = L.windowed ? 1 : 0;
    a.segs = (int)fcs_ceil_div(a.I0, SEG);
    const bool vec4 = (a.I0 % 4 == 0) && fcs_aligned(T, 16);
    // whole groups of dg sketches, then one launch for the remainder
    const int full_groups = p->D / L.dg;
    const int tail = p->D - full_groups * L.dg;
    const int64_t blocks_rounded = fcs_ceil_div(L.nblocks, NXCD) * NXCD;
    for (int pass = 0; pass < 2; ++pass) {
        const int dg = pass == 0 ? L.dg : tail;
        const int groups = pass == 0 ? full_groups : (tail ? 1 : 0);
        if (groups == 0) continue;
        a.ngroups = groups;
        a.d_first = pass == 0 ? 0 : full_groups * L.dg;
        const int64_t grid64 = blocks_rounded * groups;
        if (grid64 > INT32_MAX) FCS_FAIL(FCS_EUNSUPPORTED, "grid too large");
        const size_t lds = (size_t)dg * (size_t)L.W * sizeof(float);
        switch (dg) {
        case 1: launch_dense<1>(a, vec4, lds, (unsigned)grid64, s); break;
        case 2: launch_dense<2>(a, vec4, lds, (unsigned)grid64, s); break;
        case 3: launch_dense<3>(a, vec4, lds, (unsigned)grid64, s); break;
        default: launch_dense<4>(a, vec4, lds, (unsigned)grid64, s); break;
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
    a.chunk = fcs_ceil_div(nnz, nchunks);
    a.nchunks = fcs_ceil_div(nnz, a.chunk);
    const size_t lds = (size_t)dg * ((size_t)p->sumI + (size_t)p->Jt) * 4;
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
