// CP sketch, sketch spectra and T(I, u, v) contractions (Sections 3.1 and
// 4.1 of the paper).
//
// Transform layout.  The plan's transform length is L = Q * P with P a power
// of two held in LDS.  The L-point DFT of a sequence x supported on [0, M) is
// split into Q interleaved slices: X[Q k + q] = DFT_P(w_q)[k] with
// w_q[m] = sum_t x[m + tP] exp(-2 pi i q (m + tP) / L)  (a twisted fold), so
// every slice is one P-point FFT in LDS.  The spectrum of a real sequence is
// conjugate-symmetric, so only slices q = 0..floor(Q/2) are formed; the
// inverse combines them as
//   y[m] = (1/L) sum_q c_q Re( exp(+2 pi i q m / L) Z_q[m mod P] ),
// Z_q the unnormalised inverse P-point DFT of slice q, c_q = 1 for q = 0 and
// (Q even) q = Q/2, else 2.  Any L >= J~ gives the linear convolution of the
// paper's J~-point zero-padded transforms, truncated to J~.
//
// Count sketches inside the transforms are scattered into LDS bins as 64-bit
// fixed point scaled to each column's maximum (a small pre-kernel computes
// the maxima; integer LDS atomics, since float LDS atomics are slow on
// gfx950).  Hash lengths J_n > P fold several buckets onto one position
// with complex weights; those sketches are gathered over the plan's inverse
// hash lists (indices grouped by h_n) by the thread that owns the position.
#include "fcs_internal.h"

#include <algorithm>
#include <mutex>

#include "cp_tile.h"
#include "fft.h"
#include "median.h"

using namespace fcsfft;
using namespace fcscp;

namespace {

// ---------------------------------------------------------------------------
// CP sketch: forward tiles (sketch d, slice q, rank chunk) write partial
// spectra, one workgroup per sketch then sums and inverts them.  A plan with
// a single slice and a single chunk inverts inside the forward tile.
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(Shape<P>::T) void cp_forward_kernel(CpDesc c) {
    extern __shared__ float2 lds[];
    // tiles of the slices that pack two modes per transform (q = 0 and,
    // Q even, q = Q/2) cost less: the others are dispatched first
    const int tile = blockIdx.x;
    const int chunk = tile % c.nchunks;
    const int d = (tile / c.nchunks) % c.D;
    const int qi = tile / (c.nchunks * c.D);
    const int nfull = c.s.Qh - 1 - ((c.s.Q % 2 == 0 && c.s.Q > 1) ? 1 : 0);
    const int q = qi < nfull ? qi + 1 : (qi == nfull ? 0 : c.s.Q / 2);
    float2 acc[Shape<P>::E];
    cp_tile<P>(c, d, q, chunk, lds, acc);
    if (c.nchunks == 1)
        finish_slice<P>(c, d, q, lds, acc, slice_dst(c, d, q), false);
    else
        store_partial<P>(c, d, q, chunk, acc);
}

// Columns whose maxima scale the fixed-point count-sketch bins: column r
// of mode n is col[n][r * I[n] .. + I[n]) (modes with a null col are
// skipped), r < ncols.
struct ColMaxArgs {
    const float *col[FCS_MAX_ORDER];
    int I[FCS_MAX_ORDER];
    int ncols;
};

// max_i |col_n(i, r)| of every column, at umax[n * ncols + r].  A column
// that holds a NaN or an infinity gets +inf (its count sketch is then summed
// in float).  With uexp given, uexp[n * ncols + r] receives the exponent e
// with 2^(e-1) <= ||col_n(:, r)|| < 2^e (0 for a zero or non-finite column),
// the power-of-two scale that balances two modes packed into one transform.
__global__ __launch_bounds__(256) void column_absmax_kernel(ColMaxArgs a, float *umax, float *uexp) {
    __shared__ float part[4];
    __shared__ double psq[4];
    const int idx = blockIdx.x;
    const int n = idx / a.ncols, r = idx % a.ncols;
    if (!a.col[n]) {
        if (threadIdx.x == 0) {
            umax[idx] = 0.f;
            if (uexp) uexp[idx] = 0.f;
        }
        return;
    }
    const int In = a.I[n];
    const float *u = a.col[n] + (int64_t)r * In;
    constexpr int K = 4;
    float m = 0.f;
    double sq = 0.0;
    for (int i0 = threadIdx.x; i0 < In; i0 += K * 256) {
        float v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = i0 + k * 256 < In ? fabsf(u[i0 + k * 256]) : 0.f;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            m = (v[k] != v[k]) ? INFINITY : fmaxf(m, v[k]);
            sq += (double)v[k] * (double)v[k];
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        m = fmaxf(m, __shfl_xor(m, o));
        sq += __shfl_xor(sq, o);
    }
    if ((threadIdx.x & 63) == 0) {
        part[threadIdx.x >> 6] = m;
        psq[threadIdx.x >> 6] = sq;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const float mx = fmaxf(fmaxf(part[0], part[1]), fmaxf(part[2], part[3]));
        umax[idx] = mx;
        if (uexp) {
            const double nrm = sqrt(psq[0] + psq[1] + psq[2] + psq[3]);
            int e = 0;
            if (mx <= 3.4028234e38f && nrm > 0.0) (void)frexp(nrm, &e);
            uexp[idx] = (float)e;
        }
    }
}

void launch_column_absmax(const float *const *col, const int *I, int N, int ncols, float *umax, float *uexp,
                          hipStream_t s) {
    ColMaxArgs a{};
    for (int n = 0; n < N; ++n) {
        a.col[n] = col[n];
        a.I[n] = I[n];
    }
    a.ncols = ncols;
    hipLaunchKernelGGL(column_absmax_kernel, dim3((unsigned)(N * ncols)), dim3(256), 0, s, a, umax, uexp);
}

// Sum of the chunk partials of every (sketch, slice) into chunk slot 0, by
// many workgroups (bandwidth bound): thread k of (d, q, block b) adds the
// chunks of spectrum position b * 256 + k in chunk order.
__global__ __launch_bounds__(256) void reduce_chunks_kernel(float2 *partial, int nchunks, int P, int blocks) {
    const int dq = blockIdx.x / blocks;
    const int k = (blockIdx.x % blocks) * 256 + threadIdx.x;
    if (k >= P) return;
    float2 *base = partial + (int64_t)dq * nchunks * P + k;
    float2 acc = base[0];
    for (int ch = 1; ch < nchunks; ++ch) acc = cadd(acc, base[(int64_t)ch * P]);
    base[0] = acc;
}

// One workgroup per (sketch, slice): inverts the reduced spectrum.
template <int P>
__global__ __launch_bounds__(Shape<P>::T) void cp_finalize_kernel(CpDesc c) {
    extern __shared__ float2 lds[];
    slice_from_partials<P>(c, blockIdx.x / c.s.Qh, blockIdx.x % c.s.Qh, lds, 1);
}

// y_d = sum of the slice terms, in slice order.
__global__ __launch_bounds__(256) void sum_slices_kernel(CpDesc c) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= (int64_t)c.D * c.Jt) return;
    const int d = (int)(k / c.Jt);
    const int64_t m = k - (int64_t)d * c.Jt;
    const float *src = c.ytmp + (int64_t)d * c.s.Qh * c.Jt + m;
    float v = 0.f;
    for (int q = 0; q < c.s.Qh; ++q) v += src[(int64_t)q * c.Jt];
    c.out[k] = v;
}

// Kronecker product of two matrices: one workgroup per sketch.
template <int P>
__global__ __launch_bounds__(Shape<P>::T) void kron_kernel(CpDesc c) {
    extern __shared__ float2 lds[];
    kron_sketch<P>(c, blockIdx.x, lds);
}

// Contraction of two order-3 tensors over a shared index: the slice sketches
// (one workgroup per sketch and shared index), then forward tiles over
// chunks of the shared index laid out like the CP rank chunks, so the CP
// chunk reduction and finalisation complete it.
template <int P>
__global__ __launch_bounds__(Shape<P>::T) void contraction_factor_kernel(CpDesc c) {
    extern __shared__ float2 lds[];
    contraction_factors<Shape<P>::T>(c, blockIdx.x / c.R, blockIdx.x % c.R, lds);
}

template <int P>
__global__ __launch_bounds__(Shape<P>::T) void contraction_forward_kernel(CpDesc c) {
    extern __shared__ float2 lds[];
    const int tile = blockIdx.x;
    const int chunk = tile % c.nchunks;
    const int q = (tile / c.nchunks) % c.s.Qh;
    const int d = tile / (c.nchunks * c.s.Qh);
    float2 acc[Shape<P>::E];
    contraction_tile<P>(c, d, q, chunk, lds, acc);
    if (c.nchunks == 1)
        finish_slice<P>(c, d, q, lds, acc, slice_dst(c, d, q), false);
    else
        store_partial<P>(c, d, q, chunk, acc);
}

// ---------------------------------------------------------------------------
// Spectrum of given sketches: one workgroup per (sketch, slice).
// ---------------------------------------------------------------------------
struct SpecArgs {
    const float *y;
    float2 *spec;
    int64_t Jt;
    SliceArgs s;
};

template <int P>
__global__ __launch_bounds__(Shape<P>::T) void spectrum_kernel(SpecArgs a) {
    extern __shared__ float2 lds[];
    constexpr int E = Shape<P>::E;
    constexpr int T = Shape<P>::T;
    const int q = blockIdx.x % a.s.Qh;
    const int d = blockIdx.x / a.s.Qh;
    float2 v[E];
    build_seq_slice<P>(v, a.y + (int64_t)d * a.Jt, (int)a.Jt, q, a.s);
    forward_regs<P>(lds, a.s.twP, v);
    float2 *sp = a.spec + ((int64_t)d * a.s.Qh + q) * P;
#pragma unroll
    for (int e = 0; e < E; ++e) sp[threadIdx.x + e * T] = v[e];
}

// ---------------------------------------------------------------------------
// T(I, u, v)-type contraction (Section 4.1): one workgroup per (sketch d,
// vector tuple p).  z = F^-1(X_d prod_{n != f} conj(F(CS_n(v_n)))) over all
// slices, accumulated into zbuf[d][p][0..J_f); then
// est[p][i][d] = s_f(i) z[h_f(i)].
// ---------------------------------------------------------------------------
struct FreeArgs {
    const float2 *spec;
    const float *vecs[FCS_MAX_ORDER];
    const uint32_t *tab;
    int64_t off[FCS_MAX_ORDER];
    int64_t sumI;
    const int32_t *inv;
    int64_t ioff[FCS_MAX_ORDER];
    int64_t iblock;
    int I[FCS_MAX_ORDER];
    int J[FCS_MAX_ORDER];
    int N, D, Pn, free_mode;
    SliceArgs s;
    float *zbuf;            // [D][Pn][J_f]
    float *est;             // [Pn][I_f][D]
    const float *umax;      // free mode: max_i |v_n(i)| of tuple p at [n * Pn + p] (fixed-point
                            // scatter of the count sketches), or null (gather)
    const float *uexp;      // free mode: norm exponents of the same vectors (two modes packed per
                            // transform on the conjugate-symmetric slices), or null
    double *full;           // full contraction: [Pn][D]
};

template <int P>
__global__ __launch_bounds__(Shape<P>::T) void free_mode_kernel(FreeArgs a) {
    extern __shared__ float2 lds[];
    constexpr int E = Shape<P>::E;
    constexpr int T = Shape<P>::T;
    const int p = blockIdx.x % a.Pn;
    const int d = blockIdx.x / a.Pn;
    const int f = a.free_mode;
    const int Jf = a.J[f];
    float *z = a.zbuf + ((int64_t)d * a.Pn + p) * Jf;
    const int32_t *invd = a.inv + (int64_t)d * a.iblock;
    for (int q = 0; q < a.s.Qh; ++q) {
        float2 X[E];
        const float2 *sp = a.spec + ((int64_t)d * a.s.Qh + q) * P;
#pragma unroll
        for (int e = 0; e < E; ++e) X[e] = sp[threadIdx.x + e * T];
        const bool selfconj = (q == 0) || (2 * q == a.s.Q);
        for (int n = 0; n < a.N; ++n) {
            if (n == f) continue;
            const int32_t *off = invd + a.ioff[n];
            const float *vn = a.vecs[n] + (int64_t)p * a.I[n];
            float2 F[E];
            const int nb = (n + 1 == f) ? n + 2 : n + 1;     // the next mode with a vector
            if (selfconj && a.uexp && nb < a.N && a.J[n] <= P && a.J[nb] <= P) {
                // two vectors' count sketches share one transform (as in the
                // CP tiles), each scaled to a norm in [1/2, 1)
                const int ea = (int)a.uexp[(int64_t)n * a.Pn + p];
                const int eb = (int)a.uexp[(int64_t)nb * a.Pn + p];
                scatter_cs_slice<P>(F, lds, vn, a.tab + (int64_t)d * a.sumI + a.off[n], a.I[n], a.J[n], q, a.s,
                                    ldexpf(1.0f, -ea), a.umax[(int64_t)n * a.Pn + p]);
                scatter_cs_slice<P, true>(F, lds, a.vecs[nb] + (int64_t)p * a.I[nb],
                                          a.tab + (int64_t)d * a.sumI + a.off[nb], a.I[nb], a.J[nb], q, a.s,
                                          ldexpf(1.0f, -eb), a.umax[(int64_t)nb * a.Pn + p]);
                forward_regs<P>(lds, a.s.twP, F);
                split_pair_product<P>(F, lds, q != 0, ea + eb);
#pragma unroll
                for (int e = 0; e < E; ++e) X[e] = cmulc(X[e], F[e]);
                n = nb;
                continue;
            }
            if (a.umax && a.J[n] <= P) {
                scatter_cs_slice<P>(F, lds, vn, a.tab + (int64_t)d * a.sumI + a.off[n], a.I[n], a.J[n], q, a.s,
                                    1.0f, a.umax[(int64_t)n * a.Pn + p]);
            } else if (a.I[n] <= 2 * Lds<P>::elems) {
                // the vector fits in the transform's (free) LDS: stage it
                // there so the gather reads LDS, as in the CP tiles
                float *lv = reinterpret_cast<float *>(lds);
                stage_column<T>(lv, vn, a.I[n]);
                __syncthreads();
                build_cs_slice<P>(F, lv, off, off + a.J[n] + 1, off + a.J[n] + 1 + a.I[n], a.J[n], q, a.s, 1.0f);
                __syncthreads();
            } else {
                build_cs_slice<P>(F, vn, off, off + a.J[n] + 1, off + a.J[n] + 1 + a.I[n], a.J[n], q, a.s, 1.0f);
            }
            forward_regs<P>(lds, a.s.twP, F);
#pragma unroll
            for (int e = 0; e < E; ++e) X[e] = cmulc(X[e], F[e]);
        }
        store<P>(lds, X);
        __syncthreads();
        float2 Z[E];
        inverse<P>(lds, a.s.twP, Z);
        const int tt = tid_opaque();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = tt + e * T;
            InvTerms it(a.s, q, k, Z[e]);
            for (int m = k; m < Jf; m += P) {
                const float t = it.next();
                z[m] = (q == 0) ? t : z[m] + t;
            }
        }
        __syncthreads();
    }
    __threadfence_block();
    __syncthreads();
    const uint32_t *tf = a.tab + (int64_t)d * a.sumI + a.off[f];
    const int If = a.I[f];
    for (int i = threadIdx.x; i < If; i += T) {
        const uint32_t w = tf[i];
        const float v = z[w & FCS_H_MASK];
        a.est[((int64_t)p * If + i) * a.D + d] = __uint_as_float(__float_as_uint(v) ^ (w & FCS_S_BIT));
    }
}

// Full contraction (a vector at every mode), one workgroup per (sketch d,
// tuple p).  By Parseval, <y_d, g> with g the linear convolution of the
// modes' count sketches is (1/L) times the sum over all L frequencies of
// Y conj(G); the stored slices hold the frequencies Q k + q for
// q <= floor(Q/2), and the product is conjugate-symmetric, so slice q
// counts c_q times (1 for q = 0 and, Q even, q = Q/2, else 2) through its
// real part.  Sums are formed in double.
template <int P>
__global__ __launch_bounds__(Shape<P>::T) void full_contract_kernel(FreeArgs a) {
    extern __shared__ float2 lds[];
    constexpr int E = Shape<P>::E;
    constexpr int T = Shape<P>::T;
    const int p = blockIdx.x % a.Pn;
    const int d = blockIdx.x / a.Pn;
    const int32_t *invd = a.inv + (int64_t)d * a.iblock;
    double acc = 0.0;
    for (int q = 0; q < a.s.Qh; ++q) {
        float2 X[E];
        const float2 *sp = a.spec + ((int64_t)d * a.s.Qh + q) * P;
#pragma unroll
        for (int e = 0; e < E; ++e) X[e] = sp[threadIdx.x + e * T];
        for (int n = 0; n < a.N; ++n) {
            const int32_t *off = invd + a.ioff[n];
            const float *vn = a.vecs[n] + (int64_t)p * a.I[n];
            float2 F[E];
            if (a.I[n] <= 2 * Lds<P>::elems) {
                float *lv = reinterpret_cast<float *>(lds);
                stage_column<T>(lv, vn, a.I[n]);
                __syncthreads();
                build_cs_slice<P>(F, lv, off, off + a.J[n] + 1, off + a.J[n] + 1 + a.I[n], a.J[n], q, a.s, 1.0f);
                __syncthreads();
            } else {
                build_cs_slice<P>(F, vn, off, off + a.J[n] + 1, off + a.J[n] + 1 + a.I[n], a.J[n], q, a.s, 1.0f);
            }
            forward_regs<P>(lds, a.s.twP, F);
#pragma unroll
            for (int e = 0; e < E; ++e) X[e] = cmulc(X[e], F[e]);
        }
        double part = 0.0;
#pragma unroll
        for (int e = 0; e < E; ++e) part += (double)X[e].x;
        acc += ((q == 0 || 2 * q == a.s.Q) ? 1.0 : 2.0) * part;
        __syncthreads();
    }
    acc = fcs_block_sum_f64<T>(acc);
    if (threadIdx.x == 0) a.full[(int64_t)p * a.D + d] = acc / (double)a.s.L;
}

__global__ __launch_bounds__(256) void median_tuples_kernel(const double *v, int64_t Pn, int D, double *out) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < Pn) out[p] = fcs_median_small(v + p * D, D);
}

template <int MAXD>
__global__ __launch_bounds__(256) void median_rows_kernel(const float *est, int64_t rows, int D, double *out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= rows) return;
    float v[MAXD];
#pragma unroll
    for (int d = 0; d < MAXD; ++d) v[d] = d < D ? est[k * D + d] : 0.f;
    out[k] = fcs_median_reg<MAXD>(v, D);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
template <int P>
int forward_occupancy() {
    // resident forward workgroups per CU (LDS, registers, threads), asked of
    // the runtime once per device
    static int cached[64] = {0};
    int dev = 0;
    (void)hipGetDevice(&dev);
    int &k = cached[dev & 63];
    if (k == 0) {
        fcs_allow_lds(reinterpret_cast<const void *>(cp_forward_kernel<P>), Lds<P>::bytes);
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void *>(cp_forward_kernel<P>),
                                                         Shape<P>::T, Lds<P>::bytes) != hipSuccess || n < 1)
            n = 1;
        k = n;
    }
    return k;
}

// Rank chunks per (sketch, slice): the forward grid runs in rounds of
// (resident workgroups per CU x CUs); the busiest CU handles
// rounds x ceil(R / chunks) ranks.  Pick the count that minimises that
// load (each extra chunk also costs one partial spectrum), fewest chunks on
// ties.
int cp_chunks(const fcs_plan *p, int64_t R) {
    if (R <= 0) return 1;
    int occ = 1;
    FCS_DISPATCH_FFT_NOFAIL(p->P, occ = forward_occupancy<PP>());
    const int64_t slots = (int64_t)occ * fcs_device_cu_count();
    const int64_t tiles = (int64_t)p->D * p->Qh;
    int best = 1;
    double best_cost = 0.0;
    const int64_t hi = std::min<int64_t>(R, std::max<int64_t>(1, 4 * slots / std::max<int64_t>(1, tiles) + 1));
    for (int64_t nch = 1; nch <= hi; ++nch) {
        const int64_t rounds = fcs_ceil_div(tiles * nch, slots);
        const double cost = (double)rounds * (double)fcs_ceil_div(R, nch) + 0.02 * (double)nch;
        if (nch == 1 || cost < best_cost) {
            best_cost = cost;
            best = (int)nch;
        }
    }
    return best;
}

template <typename K>
void allow_lds_cp(K kernel, size_t bytes) {
    fcs_allow_lds(reinterpret_cast<const void *>(kernel), bytes);
}

template <int P>
void launch_cp(const CpDesc &c, hipStream_t s) {
    constexpr size_t lds = Lds<P>::bytes;
    allow_lds_cp(cp_forward_kernel<P>, lds);
    allow_lds_cp(cp_finalize_kernel<P>, lds);
    if (c.umax) launch_column_absmax(c.U, c.I, c.N, c.R, const_cast<float *>(c.umax), const_cast<float *>(c.uexp), s);
    hipLaunchKernelGGL(cp_forward_kernel<P>, dim3(c.D * c.s.Qh * c.nchunks), dim3(Shape<P>::T), lds, s, c);
    if (c.nchunks > 1) {
        const int blocks = P / 256;
        hipLaunchKernelGGL(reduce_chunks_kernel, dim3(c.D * c.s.Qh * blocks), dim3(256), 0, s, c.partial,
                           c.nchunks, P, blocks);
        hipLaunchKernelGGL(cp_finalize_kernel<P>, dim3(c.D * c.s.Qh), dim3(Shape<P>::T), lds, s, c);
    }
    if (c.s.Qh > 1 && c.out)
        hipLaunchKernelGGL(sum_slices_kernel, dim3((unsigned)fcs_ceil_div((int64_t)c.D * c.Jt, 256)), dim3(256), 0,
                           s, c);
}

template <int P>
void launch_kron(const CpDesc &c, hipStream_t s) {
    const size_t lds = cp_lds_bytes(P, c);
    allow_lds_cp(kron_kernel<P>, lds);
    hipLaunchKernelGGL(kron_kernel<P>, dim3(c.D), dim3(Shape<P>::T), lds, s, c);
}

template <int P>
void launch_contraction(const CpDesc &c, hipStream_t s) {
    const size_t lds = cp_lds_bytes(P, c);
    constexpr size_t flds = Lds<P>::bytes;
    allow_lds_cp(contraction_factor_kernel<P>, lds);
    allow_lds_cp(contraction_forward_kernel<P>, flds);
    allow_lds_cp(cp_finalize_kernel<P>, flds);
    hipLaunchKernelGGL(contraction_factor_kernel<P>, dim3(c.D * c.R), dim3(Shape<P>::T), lds, s, c);
    hipLaunchKernelGGL(contraction_forward_kernel<P>, dim3(c.D * c.s.Qh * c.nchunks), dim3(Shape<P>::T), flds, s,
                       c);
    if (c.nchunks > 1) {
        const int blocks = P / 256;
        hipLaunchKernelGGL(reduce_chunks_kernel, dim3(c.D * c.s.Qh * blocks), dim3(256), 0, s, c.partial,
                           c.nchunks, P, blocks);
        hipLaunchKernelGGL(cp_finalize_kernel<P>, dim3(c.D * c.s.Qh), dim3(Shape<P>::T), flds, s, c);
    }
    if (c.s.Qh > 1 && c.out)
        hipLaunchKernelGGL(sum_slices_kernel, dim3((unsigned)fcs_ceil_div((int64_t)c.D * c.Jt, 256)), dim3(256), 0,
                           s, c);
}

template <int P>
void launch_spectrum(const SpecArgs &sa, int D, int Qh, hipStream_t s) {
    constexpr size_t lds = Lds<P>::bytes;
    allow_lds_cp(spectrum_kernel<P>, lds);
    hipLaunchKernelGGL(spectrum_kernel<P>, dim3(D * Qh), dim3(Shape<P>::T), lds, s, sa);
}

template <int P>
void launch_free(const FreeArgs &fa, hipStream_t s) {
    constexpr size_t lds = Lds<P>::bytes;
    allow_lds_cp(free_mode_kernel<P>, lds);
    hipLaunchKernelGGL(free_mode_kernel<P>, dim3(fa.D * fa.Pn), dim3(Shape<P>::T), lds, s, fa);
}

template <int P>
void launch_full(const FreeArgs &fa, hipStream_t s) {
    constexpr size_t lds = Lds<P>::bytes;
    allow_lds_cp(full_contract_kernel<P>, lds);
    hipLaunchKernelGGL(full_contract_kernel<P>, dim3(fa.D * fa.Pn), dim3(Shape<P>::T), lds, s, fa);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// CP workspace: chunk partial spectra (several chunks) and slice terms
// (several slices)
static size_t cp_partial_bytes(const fcs_plan *p, int nch) {
    return nch > 1 ? align256((size_t)p->D * p->Qh * nch * p->P * sizeof(float2)) : 0;
}

static size_t cp_ytmp_bytes(const fcs_plan *p) {
    return p->Qh > 1 ? align256((size_t)p->D * p->Qh * p->Jt * sizeof(float)) : 0;
}

// column maxima of the factors (fixed-point count-sketch scales) and their
// norm exponents (scales of the modes packed into one transform)
static size_t cp_umax_bytes(const fcs_plan *p, int64_t R) {
    return align256(2 * (size_t)p->N * (size_t)std::max<int64_t>(R, 0) * sizeof(float));
}

size_t fcs_ws_cp(const fcs_plan *p, int64_t R) {
    if (p->P == 0) return 256;
    const int nch = cp_chunks(p, R);
    return std::max<size_t>(256, cp_partial_bytes(p, nch) + cp_ytmp_bytes(p) + cp_umax_bytes(p, R));
}

// factor sketches of a Kronecker or contraction plan whose 64-bit bins do
// not fit LDS are summed in global memory (after the float sketches in the
// workspace)
static bool factor_bins_in_lds(const fcs_plan *p) {
    const size_t nb = (size_t)std::max<int64_t>(p->J[0] + p->J[1] - 1, p->J[2] + p->J[3] - 1);
    return nb * 8 <= FCS_LDS_BYTES - 1024;
}

static size_t factor_float_bytes(const fcs_plan *p, int64_t pairs) {
    return align256((size_t)p->D * (size_t)pairs * (p->J[0] + p->J[1] - 1 + p->J[2] + p->J[3] - 1) * sizeof(float));
}

static size_t factor_bin_bytes(const fcs_plan *p, int64_t pairs) {
    if (factor_bins_in_lds(p)) return 0;
    return align256((size_t)p->D * (size_t)pairs * (p->J[0] + p->J[1] - 1 + p->J[2] + p->J[3] - 1) * 8);
}

// A Kronecker sketch with many stored slices runs as the contraction of
// shared length 1 (its slices spread over workgroups); otherwise one
// workgroup per sketch does the whole of it.
static bool kron_as_contraction(const fcs_plan *p) { return p->Qh > 2; }

size_t fcs_ws_contraction(const fcs_plan *p, int64_t Lc);

size_t fcs_ws_kron(const fcs_plan *p) {
    if (p->N != 4) return 256;
    if (kron_as_contraction(p)) return fcs_ws_contraction(p, 1);
    return factor_float_bytes(p, 1) + factor_bin_bytes(p, 1);
}

// contraction workspace: slice sketches, then the CP chunk partials and
// slice terms for chunks of the shared index
static size_t contraction_factor_bytes(const fcs_plan *p, int64_t Lc) {
    return factor_float_bytes(p, Lc) + factor_bin_bytes(p, Lc);
}

size_t fcs_ws_contraction(const fcs_plan *p, int64_t Lc) {
    if (p->N != 4 || Lc < 1 || p->P == 0) return 256;
    return contraction_factor_bytes(p, Lc) + cp_partial_bytes(p, cp_chunks(p, Lc)) + cp_ytmp_bytes(p);
}

size_t fcs_ws_spectrum(const fcs_plan *) { return 256; }

size_t fcs_ws_full(const fcs_plan *p, int64_t Pn) {
    return std::max<size_t>(256, align256((size_t)std::max<int64_t>(Pn, 0) * p->D * sizeof(double)));
}

size_t fcs_ws_free_mode(const fcs_plan *p, int64_t Pn) {
    if (Pn <= 0) return 256;
    int64_t Jmax = 0, Imax = 0;
    for (int n = 0; n < p->N; ++n) {
        Jmax = std::max<int64_t>(Jmax, p->J[n]);
        Imax = std::max<int64_t>(Imax, p->I[n]);
    }
    return align256((size_t)p->D * Pn * Jmax * 4) + align256((size_t)Pn * Imax * p->D * 4) +
           align256(2 * (size_t)p->N * Pn * 4);
}

// Argument checks shared by fcs_sketch_cp and fcs_sketch_cp_noalloc
// (nothing is enqueued before they pass).
static fcs_status cp_check_args(const fcs_plan *p, int64_t R, const float *const *U, const float *out,
                                const float *spec) {
    if (!p || !p->bound) FCS_FAIL(FCS_EINVAL, "plan is null or not bound");
    if (p->P == 0) FCS_FAIL(FCS_EUNSUPPORTED, "no transform length fits this plan");
    if (R < 0) FCS_FAIL(FCS_EINVAL, "R < 0");
    if (R > INT32_MAX / FCS_MAX_ORDER) FCS_FAIL(FCS_EUNSUPPORTED, "R too large");
    if (!out && !spec) FCS_FAIL(FCS_EINVAL, "neither out nor spec given");
    if (R > 0 && !U) FCS_FAIL(FCS_EINVAL, "null factor array");
    for (int n = 0; n < p->N; ++n)
        if (p->I[n] >= FCS_MAX_GATHER_INDEX) FCS_FAIL(FCS_EUNSUPPORTED, "CP sketches need I_n < 2^30");
    for (int n = 0; R > 0 && n < p->N; ++n)
        if (!U[n]) FCS_FAIL(FCS_EINVAL, "null factor %d", n);
    return FCS_OK;
}

// The CP sketch with `nchunks` rank chunks; buf holds the chunk partial
// spectra, the slice terms and the column maxima (cp_partial_bytes +
// cp_ytmp_bytes + cp_umax_bytes).
static fcs_status cp_run(const fcs_plan *p, int64_t R, const float *const *U, const float *lambda, float *out,
                         float *spec, void *buf, int nchunks, hipStream_t s) {
    if (R == 0) {
        if (out) {
            fcs_status st = fcs_zero_fill(out, (int64_t)p->D * p->Jt, s);
            if (st != FCS_OK) return st;
        }
        if (spec) return fcs_zero_fill(spec, (int64_t)p->D * p->Qh * p->P * 2, s);
        return FCS_OK;
    }
    CpDesc c{};
    desc_from_plan(c, p);
    c.kind = FCS_DESC_CP;
    for (int n = 0; n < p->N; ++n) c.U[n] = U[n];
    c.lambda = lambda;
    c.R = (int)R;
    c.nchunks = nchunks;
    c.rchunk = (int)fcs_ceil_div(R, c.nchunks);
    c.partial = (float2 *)buf;
    c.ytmp = (float *)((char *)buf + cp_partial_bytes(p, c.nchunks));
    c.umax = (const float *)((char *)buf + cp_partial_bytes(p, c.nchunks) + cp_ytmp_bytes(p));
    c.uexp = c.umax + (int64_t)p->N * R;
    c.out = out;
    c.spec = (float2 *)spec;
    FCS_DISPATCH_FFT(p->P, (launch_cp<PP>(c, s)));
    FCS_LAUNCH_CHECK();
    return FCS_OK;
}

extern "C" fcs_status fcs_sketch_cp(fcs_plan_t p, int64_t R, const float *const *U, const float *lambda,
                                    float *out, float *spec, void *ws, size_t ws_bytes, void *stream) {
    fcs_clear_error();
    fcs_status st = cp_check_args(p, R, U, out, spec);
    if (st != FCS_OK) return st;
    if (R > 0) {
        const size_t need = fcs_ws_cp(p, R);
        if (!ws || ws_bytes < need) FCS_FAIL(FCS_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
        if (!fcs_aligned(ws, 16)) FCS_FAIL(FCS_EINVAL, "workspace not 16-byte aligned");
    }
    return cp_run(p, R, U, lambda, out, spec, ws, R > 0 ? cp_chunks(p, R) : 1, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Allocation-free CP sketch.  Its chunk partials, slice terms and column
// maxima live in a file-scope device array of FCS_NOALLOC_SCRATCH_BYTES
// (each device the library runs on holds its own copy until the process
// ends).  Host code
// never passes the array's name to a kernel: its device address is looked
// up once per device with hipGetSymbolAddress on the first call made with
// that device current, and kept.  Every call on a device shares that
// device's array, so calls that overlap on one device race.  Nothing needs
// to start at zero: the kernels overwrite every word they later read.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[FCS_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

fcs_status noalloc_scratch(void **out) {
    int dev = 0;
    FCS_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) FCS_FAIL(FCS_EUNSUPPORTED, "device %d beyond %d", dev, NOALLOC_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        FCS_HIP_CHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) FCS_FAIL(FCS_EDEVICE, "no device address for the scratch array");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return FCS_OK;
}
}  // namespace

extern "C" fcs_status fcs_sketch_cp_noalloc(fcs_plan_t p, int64_t R, const float *const *U, const float *lambda,
                                            float *out, float *spec, void *stream) {
    fcs_clear_error();
    fcs_status st = cp_check_args(p, R, U, out, spec);
    if (st != FCS_OK) return st;
    // the rank chunks of fcs_sketch_cp, fewer when their partials would not
    // fit the array (the sums then group the ranks differently)
    int nch = R > 0 ? cp_chunks(p, R) : 1;
    const size_t fixed = cp_ytmp_bytes(p) + cp_umax_bytes(p, R);
    while (nch > 1 && cp_partial_bytes(p, nch) + fixed > FCS_NOALLOC_SCRATCH_BYTES) --nch;
    const size_t need = cp_partial_bytes(p, nch) + fixed;
    if (R > 0 && need > FCS_NOALLOC_SCRATCH_BYTES)
        FCS_FAIL(FCS_ENOMEM, "slice terms and column maxima need %zu bytes, more than the %zu-byte scratch array of "
                             "fcs_sketch_cp_noalloc (use fcs_sketch_cp with a workspace)",
                 need, (size_t)FCS_NOALLOC_SCRATCH_BYTES);
    void *buf = nullptr;
    if (R > 0) {
        st = noalloc_scratch(&buf);
        if (st != FCS_OK) return st;
    }
    return cp_run(p, R, U, lambda, out, spec, buf, nch, (hipStream_t)stream);
}

extern "C" fcs_status fcs_sketch_kron(fcs_plan_t p, const float *A, const float *B, float *out, float *spec,
                                      void *ws, size_t ws_bytes, void *stream) {
    fcs_clear_error();
    if (!p || !p->bound) FCS_FAIL(FCS_EINVAL, "plan is null or not bound");
    if (p->N != 4) FCS_FAIL(FCS_EINVAL, "a Kronecker sketch needs an order-4 plan (N=%d)", p->N);
    if (p->P == 0) FCS_FAIL(FCS_EUNSUPPORTED, "no transform length fits this plan");
    if (!A || !B) FCS_FAIL(FCS_EINVAL, "null factor matrix");
    if (!out && !spec) FCS_FAIL(FCS_EINVAL, "neither out nor spec given");
    const size_t need = fcs_ws_kron(p);
    if (!ws || ws_bytes < need) FCS_FAIL(FCS_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
    if (!fcs_aligned(ws, 16)) FCS_FAIL(FCS_EINVAL, "workspace not 16-byte aligned");
    // A (x) B is the contraction of A (I_0 x I_1 x 1) with B (1 x I_2 x I_3)
    if (kron_as_contraction(p)) return fcs_sketch_contraction(p, 1, A, B, out, spec, ws, ws_bytes, stream);
    CpDesc c{};
    desc_from_plan(c, p);
    c.kind = FCS_DESC_KRON;
    c.U[0] = A;
    c.U[1] = B;
    c.R = 1;
    c.nchunks = 1;
    c.rchunk = 1;
    c.kscratch = (float *)ws;
    c.kbins = factor_bins_in_lds(p) ? nullptr
                                    : reinterpret_cast<unsigned long long *>((char *)ws + factor_float_bytes(p, 1));
    c.out = out;
    c.spec = (float2 *)spec;
    hipStream_t s = (hipStream_t)stream;
    FCS_DISPATCH_FFT(p->P, (launch_kron<PP>(c, s)));
    FCS_LAUNCH_CHECK();
    return FCS_OK;
}

extern "C" fcs_status fcs_sketch_contraction(fcs_plan_t p, int64_t Lc, const float *A, const float *B,
                                             float *out, float *spec, void *ws, size_t ws_bytes, void *stream) {
    fcs_clear_error();
    if (!p || !p->bound) FCS_FAIL(FCS_EINVAL, "plan is null or not bound");
    if (p->N != 4) FCS_FAIL(FCS_EINVAL, "a contraction sketch needs an order-4 plan (N=%d)", p->N);
    if (p->P == 0) FCS_FAIL(FCS_EUNSUPPORTED, "no transform length fits this plan");
    if (Lc < 1 || Lc > (1 << 20)) FCS_FAIL(FCS_EINVAL, "shared index length %lld out of range", (long long)Lc);
    if (!A || !B) FCS_FAIL(FCS_EINVAL, "null factor tensor");
    if (!out && !spec) FCS_FAIL(FCS_EINVAL, "neither out nor spec given");
    CpDesc c{};
    desc_from_plan(c, p);
    c.kind = FCS_DESC_CONTRACTION;
    const size_t need = fcs_ws_contraction(p, Lc);
    if (!ws || ws_bytes < need) FCS_FAIL(FCS_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
    if (!fcs_aligned(ws, 16)) FCS_FAIL(FCS_EINVAL, "workspace not 16-byte aligned");
    c.U[0] = A;
    c.U[1] = B;
    c.R = (int)Lc;
    c.nchunks = cp_chunks(p, Lc);
    c.rchunk = (int)fcs_ceil_div(Lc, c.nchunks);
    c.kscratch = (float *)ws;
    c.kbins = factor_bins_in_lds(p) ? nullptr
                                    : reinterpret_cast<unsigned long long *>((char *)ws + factor_float_bytes(p, Lc));
    c.partial = (float2 *)((char *)ws + contraction_factor_bytes(p, Lc));
    c.ytmp = (float *)((char *)c.partial + cp_partial_bytes(p, c.nchunks));
    c.out = out;
    c.spec = (float2 *)spec;
    hipStream_t s = (hipStream_t)stream;
    FCS_DISPATCH_FFT(p->P, (launch_contraction<PP>(c, s)));
    FCS_LAUNCH_CHECK();
    return FCS_OK;
}

extern "C" fcs_status fcs_sketch_spectrum(fcs_plan_t p, const float *y, float *spec, void *ws, size_t ws_bytes,
                                          void *stream) {
    fcs_clear_error();
    (void)ws;
    (void)ws_bytes;
    if (!p || !p->bound) FCS_FAIL(FCS_EINVAL, "plan is null or not bound");
    if (p->P == 0) FCS_FAIL(FCS_EUNSUPPORTED, "no transform length fits this plan");
    if (!y || !spec) FCS_FAIL(FCS_EINVAL, "null sketch or spectrum");
    SpecArgs sa{};
    sa.y = y;
    sa.spec = (float2 *)spec;
    sa.Jt = p->Jt;
    sa.s = slice_args(p);
    hipStream_t s = (hipStream_t)stream;
    FCS_DISPATCH_FFT(p->P, (launch_spectrum<PP>(sa, p->D, p->Qh, s)));
    FCS_LAUNCH_CHECK();
    return FCS_OK;
}

extern "C" fcs_status fcs_contract_free_mode(fcs_plan_t p, const float *spec, int32_t free_mode, int64_t Pn,
                                             const float *const *vecs, double *out, void *ws, size_t ws_bytes,
                                             void *stream) {
    fcs_clear_error();
    if (!p || !p->bound) FCS_FAIL(FCS_EINVAL, "plan is null or not bound");
    if (p->P == 0) FCS_FAIL(FCS_EUNSUPPORTED, "no transform length fits this plan");
    if (free_mode < 0 || free_mode >= p->N) FCS_FAIL(FCS_EINVAL, "free_mode %d out of range", free_mode);
    if (Pn < 0) FCS_FAIL(FCS_EINVAL, "P < 0");
    if (Pn == 0) return FCS_OK;
    for (int n = 0; n < p->N; ++n)
        if (p->I[n] >= FCS_MAX_GATHER_INDEX) FCS_FAIL(FCS_EUNSUPPORTED, "contractions need I_n < 2^30");
    if (Pn > INT32_MAX / std::max<int>(FCS_MAX_ORDER, p->D)) FCS_FAIL(FCS_EUNSUPPORTED, "too many vector tuples");
    if (!spec || !out || !vecs) FCS_FAIL(FCS_EINVAL, "null spectrum, output or vector array");
    for (int n = 0; n < p->N; ++n)
        if (n != free_mode && !vecs[n]) FCS_FAIL(FCS_EINVAL, "null vector block %d", n);
    const size_t need = fcs_ws_free_mode(p, Pn);
    if (!ws || ws_bytes < need) FCS_FAIL(FCS_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
    if (!fcs_aligned(ws, 16)) FCS_FAIL(FCS_EINVAL, "workspace not 16-byte aligned");
    int64_t Jmax = 0;
    for (int n = 0; n < p->N; ++n) Jmax = std::max<int64_t>(Jmax, p->J[n]);
    FreeArgs fa{};
    fa.spec = (const float2 *)spec;
    for (int n = 0; n < p->N; ++n) {
        fa.vecs[n] = n == free_mode ? nullptr : vecs[n];
        fa.off[n] = p->off[n];
        fa.ioff[n] = p->ioff[n];
        fa.I[n] = (int)p->I[n];
        fa.J[n] = (int)p->J[n];
    }
    fa.tab = p->tab;
    fa.sumI = p->sumI;
    fa.inv = p->inv;
    fa.iblock = p->iblock;
    fa.N = p->N;
    fa.D = p->D;
    fa.Pn = (int)Pn;
    fa.free_mode = free_mode;
    fa.s = slice_args(p);
    fa.zbuf = (float *)ws;
    fa.est = (float *)((char *)ws + align256((size_t)p->D * Pn * Jmax * 4));
    int64_t Imax = 0;
    for (int n = 0; n < p->N; ++n) Imax = std::max<int64_t>(Imax, p->I[n]);
    float *vmax = (float *)((char *)fa.est + align256((size_t)Pn * Imax * p->D * 4));
    float *vexp = vmax + (int64_t)p->N * Pn;
    fa.umax = vmax;
    fa.uexp = vexp;
    hipStream_t s = (hipStream_t)stream;
    launch_column_absmax(fa.vecs, fa.I, p->N, (int)Pn, vmax, vexp, s);
    FCS_DISPATCH_FFT(p->P, (launch_free<PP>(fa, s)));
    FCS_LAUNCH_CHECK();
    const int64_t rows = Pn * p->I[free_mode];
    const unsigned grid = (unsigned)fcs_ceil_div(rows, 256);
    if (p->D <= 8)
        median_rows_kernel<8><<<grid, 256, 0, s>>>(fa.est, rows, p->D, out);
    else if (p->D <= 16)
        median_rows_kernel<16><<<grid, 256, 0, s>>>(fa.est, rows, p->D, out);
    else if (p->D <= 32)
        median_rows_kernel<32><<<grid, 256, 0, s>>>(fa.est, rows, p->D, out);
    else
        median_rows_kernel<64><<<grid, 256, 0, s>>>(fa.est, rows, p->D, out);
    FCS_LAUNCH_CHECK();
    return FCS_OK;
}

extern "C" fcs_status fcs_contract_full(fcs_plan_t p, const float *spec, int64_t Pn, const float *const *vecs,
                                        double *out, double *per_d, void *ws, size_t ws_bytes, void *stream) {
    fcs_clear_error();
    if (!p || !p->bound) FCS_FAIL(FCS_EINVAL, "plan is null or not bound");
    if (p->P == 0) FCS_FAIL(FCS_EUNSUPPORTED, "no transform length fits this plan");
    if (Pn < 0) FCS_FAIL(FCS_EINVAL, "P < 0");
    if (Pn == 0) return FCS_OK;
    for (int n = 0; n < p->N; ++n)
        if (p->I[n] >= FCS_MAX_GATHER_INDEX) FCS_FAIL(FCS_EUNSUPPORTED, "contractions need I_n < 2^30");
    if (Pn > INT32_MAX / std::max<int>(1, p->D)) FCS_FAIL(FCS_EUNSUPPORTED, "too many vector tuples");
    if (!spec || !out || !vecs) FCS_FAIL(FCS_EINVAL, "null spectrum, output or vector array");
    for (int n = 0; n < p->N; ++n)
        if (!vecs[n]) FCS_FAIL(FCS_EINVAL, "null vector block %d", n);
    double *buf = per_d;
    if (!buf) {
        const size_t need = fcs_ws_full(p, Pn);
        if (!ws || ws_bytes < need) FCS_FAIL(FCS_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
        if (!fcs_aligned(ws, 8)) FCS_FAIL(FCS_EINVAL, "workspace not 8-byte aligned");
        buf = (double *)ws;
    }
    FreeArgs fa{};
    fa.spec = (const float2 *)spec;
    for (int n = 0; n < p->N; ++n) {
        fa.vecs[n] = vecs[n];
        fa.off[n] = p->off[n];
        fa.ioff[n] = p->ioff[n];
        fa.I[n] = (int)p->I[n];
        fa.J[n] = (int)p->J[n];
    }
    fa.tab = p->tab;
    fa.sumI = p->sumI;
    fa.inv = p->inv;
    fa.iblock = p->iblock;
    fa.N = p->N;
    fa.D = p->D;
    fa.Pn = (int)Pn;
    fa.free_mode = -1;
    fa.s = slice_args(p);
    fa.full = buf;
    hipStream_t s = (hipStream_t)stream;
    FCS_DISPATCH_FFT(p->P, (launch_full<PP>(fa, s)));
    FCS_LAUNCH_CHECK();
    median_tuples_kernel<<<(unsigned)fcs_ceil_div(Pn, 256), 256, 0, s>>>(buf, Pn, p->D, out);
    FCS_LAUNCH_CHECK();
    return FCS_OK;
}
