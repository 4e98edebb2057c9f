// Decompression of fast count sketches.  Section 4.3 states the rule for the
// Kronecker product and for the tensor contraction, and it holds at any
// order: per sketch d, entry i of the recovered tensor is S_d(i) y_d[H_d(i)]
// with H_d = sum_n h_n(i_n) and S_d = prod_n s_n(i_n).  The D estimates are
// reduced by their median, since the method keeps D independent sketches and
// returns the median (Section 4).
//
// The output is written in a caller-chosen mode order, fastest first.  Its
// dimensions split into inner ones [0, ks) and outer ones [ks, N).  The outer
// indices fix a row whose hash part r_d = sum_{k >= ks} h(j_k) is the same
// for every entry of the row, so those entries read y_d only inside the
// window [r_d, r_d + W), with W = sum_{k < ks} (J_k - 1) + 1.
//
// A workgroup takes a tile (one row, one chunk of its inner entries) and
// stages the D windows in LDS with the row's sign applied.  After that, each
// entry costs one LDS read per sketch, the median, and its share of a 16-byte
// non-temporal store.  The kernel is therefore bound by HBM writes for small
// D.  Where the D windows would not fit in LDS, or a row is shorter than its
// staged windows, entries read y from global memory in place; y is D x J~
// floats and stays resident in L2, and the kernel is bound by those random
// L2 reads.
//
// Packed hash words (bits 0..30 the hash, bit 31 the sign) add as words: a
// sum of hashes stays below J~ < 2^31, so bit 31 of the word sum is the XOR
// of the signs, i.e. the sign of the product.
#include "fcs_internal.h"

#include <algorithm>

namespace {

constexpr int DC_T = 512;                   // threads of the in-place and larger-D kernels
constexpr int DC_T_SMALL = 1024;            // staged kernels with D <= 4
constexpr int DC_T_PHASE = 256;             // in-place kernel with D > 4, one sketch at a time
constexpr int64_t DC_LDS_FLOATS = 36864;    // 144 KB of staged windows
constexpr int DC_MAXD = 32;
constexpr int64_t DC_ROW_TARGET = 65536;    // inner entries per row worth aiming for

typedef float f32x4 __attribute__((ext_vector_type(4)));

struct DecompArgs {
    const float *y;                         // D x Jt
    float *out;
    const uint32_t *tab[FCS_MAX_ORDER];     // hash words of output dimension k, sketch 0
    uint32_t n[FCS_MAX_ORDER];              // sizes of the output dimensions
    int N, ks, D, W;
    int64_t sumI, Jt;
    uint32_t n_in;                          // entries per row
    uint32_t chunk;                         // inner entries per tile
    uint32_t chunks;                        // tiles per row
};

// Median of v[0..D) with the library's convention (mean of the middle pair
// for even D, formed in double).  D = 1, 2, 3 are exact forms; larger D sort
// a bitonic network over MAXD values padded with +inf, then pick the middle
// ranks.  Sketch values are finite.
template <int MAXD>
__device__ __forceinline__ float median_of(float (&v)[MAXD], int D) {
    if constexpr (MAXD == 1) {
        return v[0];
    } else if constexpr (MAXD == 2) {
        return (float)(0.5 * ((double)v[0] + (double)v[1]));
    } else if constexpr (MAXD == 3) {
        return __builtin_amdgcn_fmed3f(v[0], v[1], v[2]);
    } else {
#pragma unroll
        for (int i = 0; i < MAXD; ++i)
            if (i >= D) v[i] = __builtin_inff();
#pragma unroll
        for (int k = 2; k <= MAXD; k <<= 1) {
#pragma unroll
            for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
                for (int i = 0; i < MAXD; ++i) {
                    const int l = i ^ j;
                    if (l > i) {
                        const float a = v[i], b = v[l];
                        const bool up = (i & k) == 0;
                        v[i] = up ? fminf(a, b) : fmaxf(a, b);
                        v[l] = up ? fmaxf(a, b) : fminf(a, b);
                    }
                }
            }
        }
        const int t1 = (D - 1) >> 1, t2 = D >> 1;
        float m1 = v[0], m2 = v[0];
#pragma unroll
        for (int i = 0; i < MAXD; ++i) {
            m1 = (i == t1) ? v[i] : m1;
            m2 = (i == t2) ? v[i] : m2;
        }
        return (float)(0.5 * ((double)m1 + (double)m2));
    }
}

// Batcher's odd-even merge sort over slots [0, DN) of an NP-slot network
// (NP the power of two >= DN), all comparators ascending.  Slots at and
// above DN would hold +inf, so a comparator that reaches one of them moves
// nothing; it is left out at compile time (103 comparators for DN = 20
// against 240 for the bitonic network over 32 slots).
template <int NP, int DN>
__device__ __forceinline__ void sort_exact(float (&v)[DN]) {
#pragma unroll
    for (int p = 1; p < NP; p <<= 1) {
#pragma unroll
        for (int k = p; k >= 1; k >>= 1) {
#pragma unroll
            for (int j = k % p; j + k < NP; j += 2 * k) {
#pragma unroll
                for (int i = 0; i < k; ++i) {
                    const int a = i + j, b = i + j + k;
                    if (b < DN && a / (2 * p) == b / (2 * p)) {
                        const float x = v[a], y = v[b];
                        v[a] = fminf(x, y);
                        v[b] = fmaxf(x, y);
                    }
                }
            }
        }
    }
}

template <int DN>
__device__ __forceinline__ float median_exact(float (&v)[DN]) {
    constexpr int NP = DN <= 8 ? 8 : DN <= 16 ? 16 : 32;
    sort_exact<NP, DN>(v);
    if constexpr (DN & 1)
        return v[(DN - 1) / 2];
    else
        return (float)(0.5 * ((double)v[DN / 2 - 1] + (double)v[DN / 2]));
}

// Estimate of sketch d for an entry whose summed hash word is `word`
// (inner part only when the window is staged, the whole sum otherwise).
template <bool GLOBAL>
__device__ __forceinline__ float estimate(const DecompArgs &a, const float *win, int d, uint32_t word) {
    float v;
    if constexpr (GLOBAL)
        v = a.y[(int64_t)d * a.Jt + (word & FCS_H_MASK)];
    else
        v = win[d * a.W + (int)(word & FCS_H_MASK)];
    return __uint_as_float(__float_as_uint(v) ^ (word & FCS_S_BIT));
}

template <int MAXD, bool VEC, bool GLOBAL, int T>
__global__ __launch_bounds__(T) void decompress_kernel(DecompArgs a) {
    extern __shared__ float win[];           // D x W staged windows
    __shared__ uint32_t rowb[FCS_MAX_D];     // row hash word of each sketch
    const int t = threadIdx.x;
    const int D = MAXD <= 3 ? MAXD : a.D;
    const uint32_t r = blockIdx.x / a.chunks;
    const uint32_t c0 = (blockIdx.x - r * a.chunks) * a.chunk;
    const uint32_t c1 = min(c0 + a.chunk, a.n_in);
    if (t < D) {
        uint32_t rem = r, w = 0;
        for (int k = a.ks; k < a.N; ++k) {
            const uint32_t j = rem % a.n[k];
            rem /= a.n[k];
            w += a.tab[k][t * a.sumI + j];
        }
        rowb[t] = w;
    }
    __syncthreads();
    if constexpr (!GLOBAL) {
        for (int d = 0; d < D; ++d) {
            const uint32_t rb = rowb[d];
            const float *src = a.y + (int64_t)d * a.Jt + (rb & FCS_H_MASK);
            const uint32_t sg = rb & FCS_S_BIT;
            float *dst = win + d * a.W;
#pragma unroll 4
            for (int w = t; w < a.W; w += T) dst[w] = __uint_as_float(__float_as_uint(src[w]) ^ sg);
        }
        __syncthreads();
    }
    float *orow = a.out + (int64_t)r * a.n_in;
    if constexpr (VEC) {
        for (uint32_t e = c0 + 4 * t; e < c1; e += 4 * T) {
            const uint32_t j0 = e % a.n[0];
            uint32_t rem = e / a.n[0];
            uint32_t base[MAXD];
#pragma unroll
            for (int d = 0; d < MAXD; ++d) base[d] = (GLOBAL && d < D) ? rowb[d] : 0u;
            for (int k = 1; k < a.ks; ++k) {
                const uint32_t j = rem % a.n[k];
                rem /= a.n[k];
#pragma unroll
                for (int d = 0; d < MAXD; ++d)
                    if (d < D) base[d] += a.tab[k][d * a.sumI + j];
            }
            float res[4];
            constexpr int QU = MAXD <= 4 ? 4 : 1;
#pragma unroll QU
            for (int q = 0; q < 4; ++q) {
                float v[MAXD];
#pragma unroll
                for (int d = 0; d < MAXD; ++d)
                    v[d] = d < D ? estimate<GLOBAL>(a, win, d, base[d] + a.tab[0][d * a.sumI + j0 + q]) : 0.f;
                res[q] = median_of<MAXD>(v, D);
            }
            const f32x4 o = {res[0], res[1], res[2], res[3]};
            __builtin_nontemporal_store(o, reinterpret_cast<f32x4 *>(orow + e));
        }
    } else {
        for (uint32_t e = c0 + t; e < c1; e += T) {
            uint32_t rem = e;
            uint32_t word[MAXD];
#pragma unroll
            for (int d = 0; d < MAXD; ++d) word[d] = (GLOBAL && d < D) ? rowb[d] : 0u;
            for (int k = 0; k < a.ks; ++k) {
                const uint32_t j = rem % a.n[k];
                rem /= a.n[k];
#pragma unroll
                for (int d = 0; d < MAXD; ++d)
                    if (d < D) word[d] += a.tab[k][d * a.sumI + j];
            }
            float v[MAXD];
#pragma unroll
            for (int d = 0; d < MAXD; ++d) v[d] = d < D ? estimate<GLOBAL>(a, win, d, word[d]) : 0.f;
            __builtin_nontemporal_store(median_of<MAXD>(v, D), orow + e);
        }
    }
}

// In-place reads for larger D, one sketch at a time: a tile is four
// entries per thread of one row (leading output dimension a multiple of 4,
// out 16-byte aligned).  Every thread gathers its four estimates of sketch
// d from y_d, then the workgroup meets at a barrier before sketch d + 1, so
// its waves read inside one sketch's row window (W floats) at a time and
// mostly hit the CU's L1 instead of spreading over all D windows.  The D
// estimates stay in registers until the median, which a sorting network
// for exactly D values forms (one instance per D).
template <int D>
__global__ __launch_bounds__(DC_T_PHASE) void decompress_phase_kernel(DecompArgs a) {
    __shared__ uint32_t rowb[FCS_MAX_D];
    const int t = threadIdx.x;
    const uint32_t r = blockIdx.x / a.chunks;
    const uint32_t c0 = (blockIdx.x - r * a.chunks) * a.chunk;
    const uint32_t e = c0 + 4 * t;
    const bool live = e < min(c0 + a.chunk, a.n_in);
    if (t < D) {
        uint32_t rem = r, w = 0;
        for (int k = a.ks; k < a.N; ++k) {
            const uint32_t j = rem % a.n[k];
            rem /= a.n[k];
            w += a.tab[k][t * a.sumI + j];
        }
        rowb[t] = w;
    }
    // inner indices of the thread's first entry (a thread past the end of
    // the row takes entry 0, whose reads are in range, and stores nothing)
    uint32_t jk[FCS_MAX_ORDER];
    {
        uint32_t rem = live ? e : 0u;
#pragma unroll
        for (int k = 0; k < FCS_MAX_ORDER; ++k) {
            jk[k] = 0u;
            if (k < a.ks) {
                jk[k] = rem % a.n[k];
                rem /= a.n[k];
            }
        }
    }
    __syncthreads();
    float v[4][D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        uint32_t bw = rowb[d];
#pragma unroll
        for (int k = 1; k < FCS_MAX_ORDER; ++k)
            if (k < a.ks) bw += a.tab[k][d * a.sumI + jk[k]];
        const uint32_t *h0 = a.tab[0] + d * a.sumI + jk[0];
        const float *yd = a.y + (int64_t)d * a.Jt;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t w = bw + h0[q];
            v[q][d] = __uint_as_float(__float_as_uint(yd[w & FCS_H_MASK]) ^ (w & FCS_S_BIT));
        }
        __syncthreads();
    }
    if (!live) return;
    float res[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) res[q] = median_exact<D>(v[q]);
    const f32x4 o = {res[0], res[1], res[2], res[3]};
    __builtin_nontemporal_store(o, reinterpret_cast<f32x4 *>(a.out + (int64_t)r * a.n_in + e));
}

template <int MAXD, bool VEC, bool GLOBAL, int T>
void launch(const DecompArgs &a, uint32_t grid, size_t lds, hipStream_t s) {
    auto k = decompress_kernel<MAXD, VEC, GLOBAL, T>;
    fcs_allow_lds((const void *)k, lds);
    hipLaunchKernelGGL(k, dim3(grid), dim3(T), lds, s, a);
}

// the in-place kernel instance of the plan's D (5 .. DC_MAXD)
template <int DN>
void launch_phase(const DecompArgs &a, uint32_t grid, hipStream_t s) {
    if constexpr (DN <= DC_MAXD) {
        if (a.D == DN) {
            hipLaunchKernelGGL(decompress_phase_kernel<DN>, dim3(grid), dim3(DC_T_PHASE), 0, s, a);
            return;
        }
        launch_phase<DN + 1>(a, grid, s);
    }
}

template <int MAXD>
void launch_d(const DecompArgs &a, bool global, bool vec, uint32_t grid, size_t lds, hipStream_t s) {
    constexpr int TS = MAXD <= 4 ? DC_T_SMALL : DC_T;
    if constexpr (MAXD >= 8) {
        if (vec && global) {
            launch_phase<5>(a, grid, s);
            return;
        }
    }
    if (vec) {
        if (global) launch<MAXD, true, true, DC_T>(a, grid, lds, s);
        else launch<MAXD, true, false, TS>(a, grid, lds, s);
    } else {
        if (global) launch<MAXD, false, true, DC_T>(a, grid, lds, s);
        else launch<MAXD, false, false, TS>(a, grid, lds, s);
    }
}

}  // namespace

extern "C" fcs_status fcs_decompress(fcs_plan_t p, const float *y, const int32_t *order, float *out,
                                     void *stream) {
    fcs_clear_error();
    if (!p || !p->bound) FCS_FAIL(FCS_EINVAL, "plan is null or not bound");
    if (!y || !out) FCS_FAIL(FCS_EINVAL, "null sketch or output");
    if (!fcs_aligned(y, 4) || !fcs_aligned(out, 4)) FCS_FAIL(FCS_EINVAL, "sketch or output not 4-byte aligned");
    if (p->D > DC_MAXD) FCS_FAIL(FCS_EUNSUPPORTED, "decompression supports D <= %d (D=%d)", DC_MAXD, p->D);
    if (p->Jt >= ((int64_t)1 << 31)) FCS_FAIL(FCS_EUNSUPPORTED, "sketch length %lld too long", (long long)p->Jt);
    const int N = p->N;
    int perm[FCS_MAX_ORDER];
    bool seen[FCS_MAX_ORDER] = {false};
    for (int k = 0; k < N; ++k) {
        perm[k] = order ? order[k] : k;
        if (perm[k] < 0 || perm[k] >= N || seen[perm[k]])
            FCS_FAIL(FCS_EINVAL, "order is not a permutation of the %d modes", N);
        seen[perm[k]] = true;
    }
    DecompArgs a{};
    a.y = y;
    a.out = out;
    a.N = N;
    a.D = p->D;
    a.sumI = p->sumI;
    a.Jt = p->Jt;
    int64_t I[FCS_MAX_ORDER], J[FCS_MAX_ORDER];
    int64_t total = 1;
    for (int k = 0; k < N; ++k) {
        I[k] = p->I[perm[k]];
        J[k] = p->J[perm[k]];
        if (I[k] >= ((int64_t)1 << 31)) FCS_FAIL(FCS_EUNSUPPORTED, "mode size %lld too large", (long long)I[k]);
        if (total > ((int64_t)1 << 62) / I[k]) FCS_FAIL(FCS_EUNSUPPORTED, "output too large");
        total *= I[k];
        a.tab[k] = p->tab + p->off[perm[k]];
        a.n[k] = (uint32_t)I[k];
    }
    auto W_of = [&](int ks) {
        int64_t w = 1;
        for (int k = 0; k < ks; ++k) w += J[k] - 1;
        return w;
    };
    auto nin_of = [&](int ks) {
        int64_t n = 1;
        for (int k = 0; k < ks; ++k) n *= I[k];
        return n;
    };
    const int64_t D = p->D;
    const bool vec = (I[0] % 4 == 0) && fcs_aligned(out, 16);
    auto grow = [&](auto fits) {
        int ks = 1;
        while (ks < N && nin_of(ks) < DC_ROW_TARGET && nin_of(ks + 1) < ((int64_t)1 << 31) && fits(ks + 1))
            ++ks;
        return ks;
    };
    // the D windows staged in LDS, if they fit and a row is long enough to
    // repay the staging; otherwise entries read y in place
    bool global = true;
    int ks = 0;
    if (D * W_of(1) <= DC_LDS_FLOATS) {
        ks = grow([&](int k) { return D * W_of(k) <= DC_LDS_FLOATS; });
        global = nin_of(ks) < D * W_of(ks);
    }
    if (global) ks = grow([](int) { return true; });
    const int64_t n_in = nin_of(ks);
    const int64_t n_out = total / n_in;
    const int64_t W = global ? 0 : W_of(ks);
    const bool phase = global && vec && D > 4;      // decompress_phase_kernel
    const int64_t threads = phase ? DC_T_PHASE : (!global && D <= 4) ? DC_T_SMALL : DC_T;
    const int64_t unit = vec ? 4 * threads : threads;
    int64_t target = phase ? unit : global ? 16384 : std::max<int64_t>(8192, 4 * D * W);
    target = (target + unit - 1) / unit * unit;
    const int64_t chunk = std::min(n_in, target);
    const int64_t chunks = fcs_ceil_div(n_in, chunk);
    if (n_out > INT32_MAX / chunks) FCS_FAIL(FCS_EUNSUPPORTED, "output needs more than 2^31 tiles");
    a.ks = ks;
    a.W = (int)W;
    a.n_in = (uint32_t)n_in;
    a.chunk = (uint32_t)chunk;
    a.chunks = (uint32_t)chunks;
    const uint32_t grid = (uint32_t)(n_out * chunks);
    const size_t lds = global ? 0 : (size_t)(D * W) * sizeof(float);
    hipStream_t s = (hipStream_t)stream;
    if (D == 1) launch_d<1>(a, global, vec, grid, lds, s);
    else if (D == 2) launch_d<2>(a, global, vec, grid, lds, s);
    else if (D == 3) launch_d<3>(a, global, vec, grid, lds, s);
    else if (D <= 4) launch_d<4>(a, global, vec, grid, lds, s);
    else if (D <= 8) launch_d<8>(a, global, vec, grid, lds, s);
    else if (D <= 16) launch_d<16>(a, global, vec, grid, lds, s);
    else launch_d<32>(a, global, vec, grid, lds, s);
    FCS_LAUNCH_CHECK();
    return FCS_OK;
}
