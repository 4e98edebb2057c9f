// Device building blocks of the CP sketch (Section 3.1 of the paper) shared
// by the single-plan kernels and the persistent batch kernels:
//   - count sketches of factor columns, one interleaved slice of the
//     L-point transform at a time (L = Q * P, P a power of two held in LDS;
//     see cp.hip for the layout): scattered into 64-bit fixed-point LDS bins
//     when J_n <= P, gathered over the inverse hash lists when J_n > P (the
//     buckets fold onto P positions),
//   - on the conjugate-symmetric slices, two modes packed into one complex
//     transform and split through one LDS exchange,
//   - one CP work tile: for a rank range, N mode spectra of one slice formed
//     in LDS, multiplied in registers and summed,
//   - the inverse: slice partial spectra summed, inverted and accumulated
//     into y[0..J~),
//   - the Kronecker product of two matrices (Section 4.3): the order-2 FCS of
//     each factor matrix and their linear convolution.
#pragma once

#include "fcs_internal.h"
#include "fft.h"

// Instantiate CALL with the compile-time FFT size PP equal to P_.
#define FCS_DISPATCH_FFT(P_, CALL)                           \
    switch (P_) {                                            \
    case 256: { constexpr int PP = 256; CALL; } break;       \
    case 512: { constexpr int PP = 512; CALL; } break;       \
    case 1024: { constexpr int PP = 1024; CALL; } break;     \
    case 2048: { constexpr int PP = 2048; CALL; } break;     \
    case 4096: { constexpr int PP = 4096; CALL; } break;     \
    case 8192: { constexpr int PP = 8192; CALL; } break;     \
    case 16384: { constexpr int PP = 16384; CALL; } break;   \
    default: FCS_FAIL(FCS_EUNSUPPORTED, "FFT size %lld not built", (long long)(P_)); \
    }

// The same dispatch for helpers that cannot fail (unknown sizes do nothing).
#define FCS_DISPATCH_FFT_NOFAIL(P_, CALL)                    \
    switch (P_) {                                            \
    case 256: { constexpr int PP = 256; CALL; } break;       \
    case 512: { constexpr int PP = 512; CALL; } break;       \
    case 1024: { constexpr int PP = 1024; CALL; } break;     \
    case 2048: { constexpr int PP = 2048; CALL; } break;     \
    case 4096: { constexpr int PP = 4096; CALL; } break;     \
    case 8192: { constexpr int PP = 8192; CALL; } break;     \
    case 16384: { constexpr int PP = 16384; CALL; } break;   \
    default: break;                                          \
    }

namespace fcscp {

using namespace fcsfft;

struct SliceArgs {
    const float2 *twP;
    const float2 *twL;
    int L, P, Q, Qh;
};

// Slice q of the DFT of one mode's count sketch CS_n(u): the thread's
// positions m = t + e*T of w_q, returned in registers w[e] (the inputs of
// its first FFT pass).  u is the factor column (I_n floats); the inverse
// lists give the buckets of h_n: `first` holds each bucket's first entry
// (index, sign, more-entries flag) and is followed by the J_n second-entry
// words, `off` / `ent` all entries in bucket order.  A position costs two
// independent entry-word loads and then its factor values, unless its
// bucket holds three or more entries; the loads of G positions are issued
// together so that their latencies overlap.
template <int P>
__device__ __forceinline__ float bucket_rest(const float *__restrict__ u, const int32_t *__restrict__ off,
                                             const int32_t *__restrict__ ent, int j) {
    // entries from the third on (the first two come from the entry words):
    // the loads of up to four of them are issued together, a loop takes any
    // further ones
    constexpr int K = 4;
    const int k0 = off[j] + 2, c1 = off[j + 1];
    uint32_t w[K];
#pragma unroll
    for (int i = 0; i < K; ++i) w[i] = (k0 + i < c1) ? (uint32_t)ent[k0 + i] : 0u;
    float y = 0.f;
#pragma unroll
    for (int i = 0; i < K; ++i)
        if (k0 + i < c1) y += __uint_as_float(__float_as_uint(u[w[i] & FCS_H_MASK]) ^ (w[i] & FCS_S_BIT));
    for (int k = k0 + K; k < c1; ++k) {
        const uint32_t v = (uint32_t)ent[k];
        y += __uint_as_float(__float_as_uint(u[v & FCS_H_MASK]) ^ (v & FCS_S_BIT));
    }
    return y;
}

__device__ __forceinline__ float bucket_first(const float *__restrict__ u, uint32_t f) {
    const float v = (f != FCS_FIRST_EMPTY) ? u[f & FCS_IDX_MASK] : 0.f;
    return __uint_as_float(__float_as_uint(v) ^ (f & FCS_S_BIT));
}

// EAGER2: load every position's second-entry word with its first one (one
// latency for two-entry buckets, more registers); otherwise only for
// buckets whose first word flags a second entry.
template <int P, bool EAGER2 = true>
__device__ __forceinline__ void build_cs_slice(float2 (&wv)[Shape<P>::E], const float *__restrict__ u,
                                               const int32_t *__restrict__ off,
                                               const int32_t *__restrict__ ent,
                                               const int32_t *__restrict__ first, int Jn, int q,
                                               const SliceArgs &s, float scale) {
    constexpr int T = Shape<P>::T;
    constexpr int E = Shape<P>::E;
    const int t = tid_opaque();
    const int32_t *__restrict__ second = first + Jn;   // second-entry words follow the first ones
    if (Jn <= P) {
        // slice twist exp(-2 pi i q (t + eT) / L) = exp(-2 pi i q t / L) *
        // exp(-2 pi i q e T / L): one per-thread factor and E factors that
        // are the same for every thread (q e T < Q P = L)
        const float2 wt = (q == 0) ? make_float2(1.f, 0.f) : s.twL[q * t];
        // positions t + e*T in groups of G (smaller groups for 1024-thread
        // workgroups, whose register budget is half, and for the persistent
        // kernels, whose occupancy follows their register count)
        constexpr int G = (T >= 1024 || (!EAGER2 && T >= 128)) ? E / 2 : E;
#pragma unroll
        for (int g0 = 0; g0 < E; g0 += G) {
            uint32_t f[G], f2[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int j = t + (g0 + g) * T;
                f[g] = (j < Jn) ? (uint32_t)first[j] : FCS_FIRST_EMPTY;
                if (EAGER2) f2[g] = (j < Jn) ? (uint32_t)second[j] : FCS_FIRST_EMPTY;
            }
            if (!EAGER2) {
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const int j = t + (g0 + g) * T;
                    f2[g] = (f[g] != FCS_FIRST_EMPTY && (f[g] & FCS_MORE_BIT)) ? (uint32_t)second[j]
                                                                             : FCS_FIRST_EMPTY;
                }
            }
            float y[G];
#pragma unroll
            for (int g = 0; g < G; ++g) y[g] = bucket_first(u, f[g]) + bucket_first(u, f2[g]);
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if (f2[g] != FCS_FIRST_EMPTY && (f2[g] & FCS_MORE_BIT))
                    y[g] += bucket_rest<P>(u, off, ent, t + (g0 + g) * T);
            }
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const float ys = y[g] * scale;
                if (q == 0) {
                    wv[g0 + g] = make_float2(ys, 0.f);
                } else {
                    const float2 w = cmul(wt, s.twL[q * (g0 + g) * T]);
                    wv[g0 + g] = make_float2(ys * w.x, ys * w.y);
                }
            }
        }
        return;
    }
    // J_n > P: fold the buckets of m, m + P, m + 2P, ... onto position m.
    // exp(-2 pi i q (m + tP) / L) = exp(-2 pi i q m / L) exp(-2 pi i q t / Q):
    // the fold sums with the Q-th roots (index q t mod Q, kept incrementally)
    // and applies the position twist once.
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int m = t + e * T;
        float2 acc = make_float2(0.f, 0.f);
        int qt = 0;
        for (int j = m; j < Jn; j += P) {
            // the second-entry word only for buckets that have one (keeps
            // the registers of this unrolled loop low)
            const uint32_t f = (uint32_t)first[j];
            float y = bucket_first(u, f);
            if (f != FCS_FIRST_EMPTY && (f & FCS_MORE_BIT)) {
                const uint32_t f2 = (uint32_t)second[j];
                y += bucket_first(u, f2);
                if (f2 & FCS_MORE_BIT) y += bucket_rest<P>(u, off, ent, j);
            }
            if (q == 0) {
                acc.x += y;
            } else {
                const float2 w = s.twL[qt * P];
                acc.x += y * w.x;
                acc.y += y * w.y;
                qt += q;
                if (qt >= s.Q) qt -= s.Q;
            }
        }
        if (q != 0) acc = cmul(acc, s.twL[q * m]);
        wv[e] = make_float2(acc.x * scale, acc.y * scale);
    }
}

// Slice q of the DFT of CS_n(u) for J_n <= P, built by scattering instead
// of gathering: the thread clears its bucket positions t + eT of the bins
// (the workgroup's LDS), every entry i of u is added to bucket h_n(i) with
// sign s_n(i) by an LDS atomic (the I_n hash words and factor values are
// coalesced loads), and the thread reads its positions back.  The loads and
// VALU work scale with I_n instead of with the J_n bucket lists.
//
// Bins are 64-bit fixed point: with umax = max_i |u_i| < 2^e, every entry is
// scaled by 2^F, F = 62 - ceil(log2 I_n) - e, so that no bucket sum can
// reach 2^62, and added as an integer.  The sums are exact apart from the
// truncation of each scaled entry to an integer (less than 2^-F, which is
// at most 2^(ceil(log2 I_n) - 61) umax), and do not depend on the order of
// the atomics; each bin's 64-bit sum is then converted to float from its
// two signed 32-bit halves (one fused multiply-add, within about one ulp)
// and scaled back by 2^-F.  A column with a non-finite entry (umax not
// finite) is summed with float atomics instead, so infinities and NaNs
// reach the sketch as in a float sum.  The LDS must be free on entry (no
// thread still reading it); it is free again on return.  IMAG adds i times
// the slice to wv instead of overwriting it (two real sequences packed into
// one complex transform).
// Entries i = t, t + T, ... of a factor column added to their buckets h_n(i)
// with sign s_n(i): as 64-bit fixed point at scale 2^F (FIXED) or with float
// atomics.  Each round issues the loads of K entries per thread before any
// atomic; rounds whose K entries all exist skip the per-entry bounds test.
template <int T, int K, bool FIXED>
__device__ __forceinline__ void scatter_entries(float2 *lds, const float *__restrict__ u,
                                                const uint32_t *__restrict__ words, int In, int F, int t) {
    unsigned long long *bins = reinterpret_cast<unsigned long long *>(lds);
    float *fbins = reinterpret_cast<float *>(lds);
    auto add = [&](uint32_t w, float x) {
        const uint32_t h = w & FCS_H_MASK;
        const bool neg = (__float_as_uint(x) ^ w) & FCS_S_BIT;   // sign of s_n(i) u_i
        if constexpr (FIXED) {
            // |u_i| 2^F < 2^62 split into exact 32-bit halves, then negated
            // as a 64-bit integer when s_n(i) u_i < 0
            const float a = ldexpf(fabsf(x), F);
            const float ahi = floorf(ldexpf(a, -32));
            const float alo = fmaf(-ahi, 4294967296.0f, a);
            unsigned long long v = ((unsigned long long)(uint32_t)ahi << 32) | (uint32_t)alo;
            if (neg) v = 0ull - v;
            __hip_atomic_fetch_add(bins + h, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        } else {
            const float v = neg ? -fabsf(x) : fabsf(x);
            __hip_atomic_fetch_add(fbins + h, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    };
    int i0 = t;
    for (; i0 + (K - 1) * T < In; i0 += K * T) {
        uint32_t w[K];
        float x[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            w[k] = words[i0 + k * T];
            x[k] = u[i0 + k * T];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) add(w[k], x[k]);
    }
    if (i0 < In) {
        uint32_t w[K];
        float x[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = i0 + k * T;
            w[k] = i < In ? words[i] : 0u;
            x[k] = i < In ? u[i] : 0.f;
        }
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (i0 + k * T < In) add(w[k], x[k]);
    }
}

template <int P, bool IMAG = false>
__device__ __forceinline__ void scatter_cs_slice(float2 (&wv)[Shape<P>::E], float2 *lds,
                                                 const float *__restrict__ u,
                                                 const uint32_t *__restrict__ words, int In, int Jn, int q,
                                                 const SliceArgs &s, float scale, float umax) {
    constexpr int T = Shape<P>::T;
    constexpr int E = Shape<P>::E;
    constexpr int K = 8;        // entries per thread whose loads are in flight together
    static_assert(8 * P <= Lds<P>::bytes, "64-bit bins fit the transform's LDS");
    const int t = tid_opaque();
    unsigned long long *bins = reinterpret_cast<unsigned long long *>(lds);
    float *fbins = reinterpret_cast<float *>(lds);
    const bool fixed = umax <= 3.4028234e38f;       // false for inf and NaN
    int F = 0;
    if (fixed && umax > 0.f) {
        int e = 0;
        (void)frexpf(umax, &e);                      // umax < 2^e
        const int lgI = In > 1 ? 32 - __clz(In - 1) : 0;
        F = 62 - lgI - e;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int j = t + e * T;
        if (j < Jn) {
            if (fixed) bins[j] = 0ull;
            else fbins[j] = 0.f;
        }
    }
    __syncthreads();
    if (fixed) scatter_entries<T, K, true>(lds, u, words, In, F, t);
    else scatter_entries<T, K, false>(lds, u, words, In, F, t);
    __syncthreads();
    float y[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int j = t + e * T;
        if (j >= Jn) {
            y[e] = 0.f;
        } else if (fixed) {
            // v = hi 2^32 + lo with lo the signed low word, so that
            // |lo| <= 2^31 and a small negative sum keeps hi = 0 (|v| < 2^62)
            const long long v = (long long)bins[j];
            const int lo = (int)(uint32_t)v;
            const int hi = (int)(v >> 32) + (int)((uint32_t)lo >> 31);
            y[e] = ldexpf(fmaf((float)hi, 4294967296.0f, (float)lo), -F);
        } else {
            y[e] = fbins[j];
        }
    }
    __syncthreads();
    // slice twist exp(-2 pi i q (t + eT) / L), factorised as in build_cs_slice
    const float2 wt = (q == 0) ? make_float2(1.f, 0.f) : s.twL[q * t];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const float ys = y[e] * scale;
        float2 v;
        if (q == 0) {
            v = make_float2(ys, 0.f);
        } else {
            const float2 w = cmul(wt, s.twL[q * e * T]);
            v = make_float2(ys * w.x, ys * w.y);
        }
        if (IMAG) wv[e] = make_float2(wv[e].x - v.y, wv[e].y + v.x);
        else wv[e] = v;
    }
}

// Slices q = 0 and, Q even, q = Q/2 hold conjugate-symmetric spectra of a
// real sequence: with X the L-point DFT, conj(X[Qk + q]) = X[Qk' + q] for
// k' = (P - k) mod P (q = 0) or k' = P - 1 - k (q = Q/2).  Two real
// sequences a, b then share one P-point transform Z of the slice of a + i b:
// F(a)[k] = (Z[k] + conj(Z[k'])) / 2 and F(b)[k] = (Z[k] - conj(Z[k'])) / 2i.
// Given the thread's Z[t + eT] in z, returns F(a)[k] F(b)[k] at the same
// positions (the two modes' product) times 2^eab through one exchange in
// LDS (free on entry and on return).
template <int P>
__device__ __forceinline__ void split_pair_product(float2 (&z)[Shape<P>::E], float2 *lds, bool half, int eab) {
    constexpr int T = Shape<P>::T;
    constexpr int E = Shape<P>::E;
    store<P>(lds, z);
    __syncthreads();
    const int t = tid_opaque();
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = t + e * T;
        const int km = half ? P - 1 - k : (P - k) & (P - 1);
        const float2 m = lds[pad(km)];
        // 2 F(a) = (zr + mr, zi - mi), 2 F(b) = (zi + mi, mr - zr)
        const float2 a = make_float2(z[e].x + m.x, z[e].y - m.y);
        const float2 b = make_float2(z[e].y + m.y, m.x - z[e].x);
        const float2 ab = cmul(a, b);
        z[e] = make_float2(ldexpf(ab.x, eab - 2), ldexpf(ab.y, eab - 2));
    }
    __syncthreads();
}

// Slice q of the DFT of a dense real sequence y[0..M): the thread's
// positions of w_q in registers (same factorised twist as the fold above).
template <int P>
__device__ __forceinline__ void build_seq_slice(float2 (&wv)[Shape<P>::E], const float *__restrict__ y, int M,
                                                int q, const SliceArgs &s) {
    constexpr int T = Shape<P>::T;
    constexpr int E = Shape<P>::E;
    const int t = tid_opaque();
#pragma unroll
    for (int e = 0; e < E; ++e) wv[e] = make_float2(0.f, 0.f);
    // fold round k adds y[m + kP] for all E positions of the thread, so the
    // E loads of a round are in flight together (the rounds are few:
    // ceil(M / P)); the fold root exp(-2 pi i q k / Q) is the same for the
    // whole workgroup
    const int nfold = (M + P - 1) / P;
    int qt = 0;
    for (int k = 0; k < nfold; ++k) {
        float v[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int j = t + e * T + k * P;
            v[e] = j < M ? y[j] : 0.f;
        }
        if (q == 0) {
#pragma unroll
            for (int e = 0; e < E; ++e) wv[e].x += v[e];
        } else {
            const float2 w = s.twL[qt * P];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                wv[e].x += v[e] * w.x;
                wv[e].y += v[e] * w.y;
            }
            qt += q;
            if (qt >= s.Q) qt -= s.Q;
        }
    }
    if (q != 0) {
#pragma unroll
        for (int e = 0; e < E; ++e) wv[e] = cmul(wv[e], s.twL[q * (t + e * T)]);
    }
}

// Slice-q terms of the inverse at the positions m = k + tP (t = 0, 1, ...)
// of thread position k < P: c_q Re(exp(+2 pi i q m / L) Z) / L with
// exp(+2 pi i q m / L) = exp(+2 pi i q k / L) exp(+2 pi i q t / Q).
struct InvTerms {
    float2 v;        // c_q conj(w_L^{qk}) Z / L
    int q, qt, Q, P;
    const float2 *twL;
    __device__ __forceinline__ InvTerms(const SliceArgs &s, int q_, int k, float2 Z) {
        const float cq = (q_ == 0 || (2 * q_ == s.Q)) ? 1.f : 2.f;
        const float sc = cq / (float)s.L;
        q = q_;
        qt = 0;
        Q = s.Q;
        P = s.P;
        twL = s.twL;
        v = (q_ == 0) ? Z : cmulc(Z, s.twL[q_ * k]);
        v.x *= sc;
        v.y *= sc;
    }
    // term of the next position k + tP (t = 0, 1, ... in order)
    __device__ __forceinline__ float next() {
        if (q == 0) return v.x;
        const float2 w = twL[qt * P];      // exp(-2 pi i q t / Q)
        qt += q;
        if (qt >= Q) qt -= Q;
        return w.x * v.x + w.y * v.y;      // Re(conj(w) v)
    }
};
// Copy n floats from global memory to LDS with the workgroup's T threads:
// 16 independent loads per thread are in flight before any is written, so a
// column costs one memory latency per 16 T floats.
template <int T>
__device__ __forceinline__ void stage_column(float *dst, const float *__restrict__ src, int n) {
    constexpr int CU = 16;
    for (int i0 = tid_opaque(); i0 < n; i0 += T * CU) {
        float v[CU];
#pragma unroll
        for (int k = 0; k < CU; ++k) {
            const int i = i0 + k * T;
            v[k] = i < n ? src[i] : 0.f;
        }
#pragma unroll
        for (int k = 0; k < CU; ++k) {
            const int i = i0 + k * T;
            if (i < n) dst[i] = v[k];
        }
    }
}

// One CP (or Kronecker) sketch computation as the kernels see it.
enum { FCS_DESC_CP = 0, FCS_DESC_KRON = 1, FCS_DESC_CONTRACTION = 2 };

struct CpDesc {
    int kind;                        // FCS_DESC_CP, FCS_DESC_KRON or FCS_DESC_CONTRACTION
    int N, D, R;                     // CONTRACTION: R = length of the shared index
    int nchunks, rchunk;             // rank chunks of the forward tiles
    int I[FCS_MAX_ORDER];
    int J[FCS_MAX_ORDER];
    const float *U[FCS_MAX_ORDER];   // CP: factor n column-major (I_n x R); KRON: U[0] = vec(A), U[1] = vec(B)
    const float *lambda;             // R weights or null
    const int32_t *inv;              // inverse hash lists, iblock words per sketch
    int64_t ioff[FCS_MAX_ORDER];
    int64_t iblock;
    const uint32_t *tab;             // packed hash words, sumI per sketch
    int64_t off[FCS_MAX_ORDER];
    int64_t sumI;
    SliceArgs s;
    int64_t Jt;
    float2 *partial;                 // [D][Qh][nchunks][P] forward partial spectra (nchunks > 1)
    float *ytmp;                     // [D][Qh][Jt] inverse term of every slice (Qh > 1)
    float *kscratch;                 // KRON: [D][J_0 + J_1 - 1 + J_2 + J_3 - 1] factor sketches
                                     // CONTRACTION: [D][R][the same] (one pair per shared index);
                                     // rank chunks are chunks of the shared index
    float *out;                      // D x Jt or null
    float2 *spec;                    // D x (Qh * P) or null
    const float *umax;               // CP: max_i |U_n(i, r)| at [n * R + r] (fixed-point scatter of the
                                     // count sketches), or null (gather over the bucket lists)
    const float *uexp;               // CP: e with 2^(e-1) <= ||U_n(:, r)|| < 2^e at [n * R + r] (scales of
                                     // two modes packed into one transform), or null (no packing)
    unsigned long long *kbins;       // KRON / CONTRACTION: 64-bit factor-sketch bins in global memory, laid
                                     // out like kscratch, when they exceed LDS (null: bins in LDS)
    int cnt_slice;                   // batch: first (d, q) chunk counter (nchunks > 1)
    int cnt_sketch;                  // batch: first per-d slice counter (Qh > 1)
};

// Forward tile (d, q, rank chunk): sum over the chunk's ranks of
// lambda_r prod_n F_q(CS_n(U_n(:, r))); thread t returns X[t + e T] in acc.
template <int P, bool EAGER2 = true>
__device__ __forceinline__ void cp_tile(const CpDesc &c, int d, int q, int chunk, float2 *lds,
                                        float2 (&acc)[Shape<P>::E]) {
    constexpr int E = Shape<P>::E;
    constexpr int T = Shape<P>::T;
    const int r0 = chunk * c.rchunk;
    const int r1 = min(c.R, r0 + c.rchunk);
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = make_float2(0.f, 0.f);
    const int32_t *invd = c.inv + (int64_t)d * c.iblock;
    // with the column maxima given, count sketches with J_n <= P are
    // scattered into LDS bins; otherwise (and for J_n > P, folded onto P
    // positions) they are gathered over the bucket lists, with a factor
    // column that fits in the (not yet used) LDS of the transform first
    // copied there, so the gather's random reads of it are LDS reads
    constexpr int LDS_FLOATS = 2 * Lds<P>::elems;
    float *lu = reinterpret_cast<float *>(lds);
    __syncthreads();
    // slices 0 and Q/2 are conjugate-symmetric: there two modes' count
    // sketches share one transform (split_pair_product)
    const bool selfconj = (q == 0) || (2 * q == c.s.Q);
    for (int r = r0; r < r1; ++r) {
        float2 prod[E];
        const float lam = c.lambda ? c.lambda[r] : 1.0f;
        for (int n = 0; n < c.N; ++n) {
            const int32_t *off = invd + c.ioff[n];
            const float *un = c.U[n] + (int64_t)r * c.I[n];
            float2 v[E];
            if (selfconj && c.uexp && n + 1 < c.N && c.J[n] <= P && c.J[n + 1] <= P) {
                // both columns scaled to norms in [1/2, 1) so that the
                // rounding of the shared transform is relative to each
                // mode's own size; the product is scaled back exactly
                const int ea = (int)c.uexp[(int64_t)n * c.R + r];
                const int eb = (int)c.uexp[(int64_t)(n + 1) * c.R + r];
                scatter_cs_slice<P>(v, lds, un, c.tab + (int64_t)d * c.sumI + c.off[n], c.I[n], c.J[n], q, c.s,
                                    ldexpf(n == 0 ? lam : 1.0f, -ea), c.umax[(int64_t)n * c.R + r]);
                scatter_cs_slice<P, true>(v, lds, c.U[n + 1] + (int64_t)r * c.I[n + 1],
                                          c.tab + (int64_t)d * c.sumI + c.off[n + 1], c.I[n + 1], c.J[n + 1], q,
                                          c.s, ldexpf(1.0f, -eb), c.umax[(int64_t)(n + 1) * c.R + r]);
                forward_regs<P>(lds, c.s.twP, v);
                split_pair_product<P>(v, lds, q != 0, ea + eb);
                if (n == 0) {
#pragma unroll
                    for (int e = 0; e < E; ++e) prod[e] = v[e];
                } else {
#pragma unroll
                    for (int e = 0; e < E; ++e) prod[e] = cmul(prod[e], v[e]);
                }
                ++n;
                continue;
            }
            if (c.umax && c.J[n] <= P) {
                scatter_cs_slice<P>(v, lds, un, c.tab + (int64_t)d * c.sumI + c.off[n], c.I[n], c.J[n], q, c.s,
                                    n == 0 ? lam : 1.0f, c.umax[(int64_t)n * c.R + r]);
            } else if (c.I[n] <= LDS_FLOATS) {
                stage_column<T>(lu, un, c.I[n]);
                __syncthreads();
                build_cs_slice<P, EAGER2>(v, lu, off, off + c.J[n] + 1, off + c.J[n] + 1 + c.I[n], c.J[n], q, c.s,
                                  n == 0 ? lam : 1.0f);
                __syncthreads();
            } else {
                build_cs_slice<P, EAGER2>(v, un, off, off + c.J[n] + 1, off + c.J[n] + 1 + c.I[n], c.J[n], q, c.s,
                                  n == 0 ? lam : 1.0f);
            }
            forward_regs<P>(lds, c.s.twP, v);
#pragma unroll
            for (int e = 0; e < E; ++e) prod[e] = (n == 0) ? v[e] : cmul(prod[e], v[e]);
        }
#pragma unroll
        for (int e = 0; e < E; ++e) acc[e] = cadd(acc[e], prod[e]);
    }
}

template <int P>
__device__ __forceinline__ void store_partial(const CpDesc &c, int d, int q, int chunk, const float2 (&acc)[Shape<P>::E]) {
    constexpr int E = Shape<P>::E;
    constexpr int T = Shape<P>::T;
    float2 *dst = c.partial + (((int64_t)d * c.s.Qh + q) * c.nchunks + chunk) * P;
    const int t = tid_opaque();
#pragma unroll
    for (int e = 0; e < E; ++e) dst[t + e * T] = acc[e];
}

// Slice q of the spectrum of sketch d is complete in X (registers): store it
// if asked, invert it and write its term of y[0..J~) to dst (accumulate:
// add to what dst holds).  Each thread owns the same positions for every q.
// Ends with a barrier (lds is reused).
template <int P>
__device__ __forceinline__ void finish_slice(const CpDesc &c, int d, int q, float2 *lds,
                                             const float2 (&X)[Shape<P>::E], float *dst, bool accumulate) {
    constexpr int E = Shape<P>::E;
    constexpr int T = Shape<P>::T;
    if (c.spec) {
        float2 *sp = c.spec + ((int64_t)d * c.s.Qh + q) * P;
        const int t = tid_opaque();
#pragma unroll
        for (int e = 0; e < E; ++e) sp[t + e * T] = X[e];
    }
    if (!dst) return;
    store<P>(lds, X);
    __syncthreads();
    float2 Z[E];
    inverse<P>(lds, c.s.twP, Z);
    const int tt = tid_opaque();
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = tt + e * T;
        InvTerms it(c.s, q, k, Z[e]);
        for (int64_t m = k; m < c.Jt; m += P) {
            const float t = it.next();
            dst[m] = accumulate ? dst[m] + t : t;
        }
    }
    __syncthreads();
}

// Where the inverse term of slice q of sketch d goes: straight to the
// output when there is one slice, else to the slice's row of ytmp.
__device__ __forceinline__ float *slice_dst(const CpDesc &c, int d, int q) {
    if (!c.out) return nullptr;
    if (c.s.Qh == 1) return c.out + (int64_t)d * c.Jt;
    return c.ytmp + ((int64_t)d * c.s.Qh + q) * c.Jt;
}

// Slice q of sketch d from its chunk partials: the first `nsum` chunk
// slots are summed in a fixed order (1 when an earlier pass already reduced
// the chunks into slot 0).
template <int P>
__device__ __forceinline__ void slice_from_partials(const CpDesc &c, int d, int q, float2 *lds, int nsum) {
    constexpr int E = Shape<P>::E;
    constexpr int T = Shape<P>::T;
    float2 X[E];
#pragma unroll
    for (int e = 0; e < E; ++e) X[e] = make_float2(0.f, 0.f);
    const float2 *src = c.partial + ((int64_t)d * c.s.Qh + q) * c.nchunks * P + tid_opaque();
    for (int ch = 0; ch < nsum; ++ch) {
#pragma unroll
        for (int e = 0; e < E; ++e) X[e] = cadd(X[e], src[(int64_t)ch * P + e * T]);
    }
    finish_slice<P>(c, d, q, lds, X, slice_dst(c, d, q), false);
}

// y_d = sum over slices of their terms (fixed order), threads over positions.
template <int T>
__device__ __forceinline__ void sum_slices(const CpDesc &c, int d) {
    if (!c.out) return;
    const float *src = c.ytmp + (int64_t)d * c.s.Qh * c.Jt;
    float *dst = c.out + (int64_t)d * c.Jt;
    for (int64_t m = tid_opaque(); m < c.Jt; m += T) {
        float v = 0.f;
        for (int q = 0; q < c.s.Qh; ++q) v += src[(int64_t)q * c.Jt + m];
        dst[m] = v;
    }
}

// Order-2 FCS of the I_a x I_b column-major matrix M under the hash words
// ta (mode a) and tb (mode b) of one sketch: y[h_a(i) + h_b(j)] +=
// s_a(i) s_b(j) M[i, j] for nb = J_a + J_b - 1 bins, written to y (global).
// Entries are quantised to 64-bit integers and summed exactly in 64-bit LDS
// bins: the largest magnitude maps into [2^(B-1), 2^B) with
// B = min(40, 62 - ceil(log2(I_a I_b))), so no bin can overflow and rounding
// moves each entry by at most 2^-B of that largest magnitude (relative error
// of the sketch at most sqrt(I_a I_b) 2^-B, below 1e-7 up to 2^20 entries).
// The nb 64-bit bins are in LDS (lds must hold them), or in global memory
// at gbins when that is given (sketches too long for LDS; the bins are then
// read back with device-scope loads, past the L1 cache).  A matrix with a
// non-finite entry gives NaN bins.
// With STRIDED, entry k of the matrix is M[k * stride] (a slice of a
// larger tensor whose other index varies fastest).
template <int T, bool STRIDED = false>
__device__ __forceinline__ void kron_factor_sketch(const float *__restrict__ M, int Ia, int Ib,
                                                   const uint32_t *__restrict__ ta,
                                                   const uint32_t *__restrict__ tb, int nb, float *y,
                                                   float2 *lds, int64_t stride = 1,
                                                   unsigned long long *gbins = nullptr) {
    unsigned long long *bins = gbins ? gbins : reinterpret_cast<unsigned long long *>(lds);
    float *red = reinterpret_cast<float *>(lds);
    const int t = tid_opaque();
    const int64_t n = (int64_t)Ia * Ib;
    float m = 0.f;
    bool bad = false;
    for (int64_t k = t; k < n; k += T) {
        const float v = fabsf(M[STRIDED ? k * stride : k]);
        bad |= !(v <= 3.4e38f);
        m = fmaxf(m, v);
    }
    // workgroup max (non-finite entries flagged separately)
    m = bad ? -1.f : m;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const float w = __shfl_xor(m, o, 64);
        m = (m < 0.f || w < 0.f) ? -1.f : fmaxf(m, w);
    }
    float M0 = m;       // one wave: every lane holds the maximum already
    if constexpr (T > 64) {
        if ((t & 63) == 0) red[t >> 6] = m;
        __syncthreads();
        M0 = 0.f;
        for (int w = 0; w < T / 64; ++w) {
            const float v = red[w];
            M0 = (M0 < 0.f || v < 0.f) ? -1.f : fmaxf(M0, v);
        }
        __syncthreads();
    }
    if (M0 < 0.f) {
        for (int j = t; j < nb; j += T) y[j] = __builtin_nanf("");
        return;
    }
    if (gbins && n <= 4 * (int64_t)nb) {
        // bins in global memory and sparse (at most four entries per bin on
        // average): float atomics straight into y, whose clearing and reading
        // is then the only traffic besides the entries (the 64-bit bins would
        // be cleared, added to and read back in full)
        for (int j = t; j < nb; j += T) y[j] = 0.f;
        __threadfence();
        __syncthreads();
        int i = t % Ia, j = t / Ia;
        const int st_i = T % Ia, st_j = T / Ia;
        for (int64_t k = t; k < n; k += T) {
            const uint32_t wa = ta[i], wb = tb[j];
            const int bin = (int)(wa & FCS_H_MASK) + (int)(wb & FCS_H_MASK);
            const float v = M[STRIDED ? k * stride : k];
            unsafeAtomicAdd(&y[bin], ((wa ^ wb) & FCS_S_BIT) ? -v : v);
            i += st_i;
            j += st_j;
            if (i >= Ia) {
                i -= Ia;
                ++j;
            }
        }
        __threadfence();
        __syncthreads();
        return;
    }
    const int lgn = n > 1 ? 64 - __clzll((unsigned long long)(n - 1)) : 0;
    const int B = min(40, 62 - lgn);
    int F = B - 1;
    if (M0 > 0.f) F = B - __builtin_amdgcn_frexp_expf(M0);
    F = max(-120, min(127, F));
    const float scale = ldexpf(1.0f, F);
    for (int j = t; j < nb; j += T) bins[j] = 0ull;
    if (gbins) __threadfence();
    __syncthreads();
    int i = t % Ia, j = t / Ia;
    const int st_i = T % Ia, st_j = T / Ia;
    for (int64_t k = t; k < n; k += T) {
        const uint32_t wa = ta[i], wb = tb[j];
        const int bin = (int)(wa & FCS_H_MASK) + (int)(wb & FCS_H_MASK);
        long long qv = __float2ll_rn(M[STRIDED ? k * stride : k] * scale);
        if ((wa ^ wb) & FCS_S_BIT) qv = -qv;
        atomicAdd(&bins[bin], (unsigned long long)qv);
        i += st_i;
        j += st_j;
        if (i >= Ia) {
            i -= Ia;
            ++j;
        }
    }
    if (gbins) __threadfence();
    __syncthreads();
    // 2^-F in two normal factors (F may reach 127)
    const float inv1 = ldexpf(1.0f, -(F / 2)), inv2 = ldexpf(1.0f, -(F - F / 2));
    for (int b = t; b < nb; b += T) {
        const unsigned long long v =
            gbins ? __hip_atomic_load(&bins[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : bins[b];
        y[b] = (float)(long long)v * inv1 * inv2;
    }
    __syncthreads();
}

// Kronecker product A (x) B as an order-4 tensor (Section 4.3): FCS(A (x) B)
// is the linear convolution of the order-2 sketches of A (modes 0, 1) and B
// (modes 2, 3); computed slice by slice as F^-1(F(y_A) F(y_B)).
template <int P>
__device__ __forceinline__ void kron_sketch(const CpDesc &c, int d, float2 *lds) {
    constexpr int E = Shape<P>::E;
    constexpr int T = Shape<P>::T;
    const uint32_t *tab = c.tab + (int64_t)d * c.sumI;
    const int na = c.J[0] + c.J[1] - 1;
    const int nbb = c.J[2] + c.J[3] - 1;
    float *ya = c.kscratch + (int64_t)d * (na + nbb);
    float *yb = ya + na;
    unsigned long long *ga = c.kbins ? c.kbins + (int64_t)d * (na + nbb) : nullptr;
    kron_factor_sketch<T>(c.U[0], c.I[0], c.I[1], tab + c.off[0], tab + c.off[1], na, ya, lds, 1, ga);
    kron_factor_sketch<T>(c.U[1], c.I[2], c.I[3], tab + c.off[2], tab + c.off[3], nbb, yb, lds, 1,
                          ga ? ga + na : nullptr);
    __threadfence_block();
    __syncthreads();
    for (int q = 0; q < c.s.Qh; ++q) {
        float2 X[E];
        build_seq_slice<P>(X, ya, na, q, c.s);
        forward_regs<P>(lds, c.s.twP, X);
        float2 Y[E];
        build_seq_slice<P>(Y, yb, nbb, q, c.s);
        forward_regs<P>(lds, c.s.twP, Y);
#pragma unroll
        for (int e = 0; e < E; ++e) X[e] = cmul(X[e], Y[e]);
        finish_slice<P>(c, d, q, lds, X, c.out ? c.out + (int64_t)d * c.Jt : nullptr, q > 0);
    }
}

// Contraction C[i0,i1,i2,i3] = sum_l A[i0,i1,l] B[l,i2,i3] of an
// I_0 x I_1 x R tensor A with an R x I_2 x I_3 tensor B (both column-major,
// Section 4.3): FCS(C) = sum_l F^-1(F(FCS(A(:,:,l))) F(FCS(B(l,:,:)))).  By
// linearity the products of the slice spectra are summed over l before one
// inverse per transform slice.
//
// First step, one workgroup per (sketch d, shared index l): the order-2
// sketches of A(:,:,l) and of B(l,:,:) (a stride-R slice) into the
// workspace, [D][R][J_0 + J_1 - 1 + J_2 + J_3 - 1].
template <int T>
__device__ __forceinline__ void contraction_factors(const CpDesc &c, int d, int l, float2 *lds) {
    const uint32_t *tab = c.tab + (int64_t)d * c.sumI;
    const int na = c.J[0] + c.J[1] - 1;
    const int nbb = c.J[2] + c.J[3] - 1;
    float *ya = c.kscratch + ((int64_t)d * c.R + l) * (na + nbb);
    unsigned long long *ga = c.kbins ? c.kbins + ((int64_t)d * c.R + l) * (na + nbb) : nullptr;
    kron_factor_sketch<T>(c.U[0] + (int64_t)l * c.I[0] * c.I[1], c.I[0], c.I[1], tab + c.off[0], tab + c.off[1],
                          na, ya, lds, 1, ga);
    kron_factor_sketch<T, true>(c.U[1] + l, c.I[2], c.I[3], tab + c.off[2], tab + c.off[3], nbb, ya + na, lds,
                                c.R, ga ? ga + na : nullptr);
}

// Second step, forward tile (sketch d, slice q, chunk of shared indices):
// acc = sum over the chunk of F_q(sketch of A(:,:,l)) F_q(sketch of B(l,:,:)).
template <int P>
__device__ __forceinline__ void contraction_tile(const CpDesc &c, int d, int q, int chunk, float2 *lds,
                                                 float2 (&acc)[Shape<P>::E]) {
    constexpr int E = Shape<P>::E;
    const int na = c.J[0] + c.J[1] - 1;
    const int nbb = c.J[2] + c.J[3] - 1;
    const int l0 = chunk * c.rchunk;
    const int l1 = min(c.R, l0 + c.rchunk);
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = make_float2(0.f, 0.f);
    for (int l = l0; l < l1; ++l) {
        const float *ya = c.kscratch + ((int64_t)d * c.R + l) * (na + nbb);
        float2 X[E];
        build_seq_slice<P>(X, ya, na, q, c.s);
        forward_regs<P>(lds, c.s.twP, X);
        float2 Y[E];
        build_seq_slice<P>(Y, ya + na, nbb, q, c.s);
        forward_regs<P>(lds, c.s.twP, Y);
#pragma unroll
        for (int e = 0; e < E; ++e) acc[e] = cadd(acc[e], cmul(X[e], Y[e]));
    }
}

// Plan-derived part of a descriptor (host side).
inline SliceArgs slice_args(const fcs_plan *p) {
    SliceArgs s;
    s.twP = p->twP;
    s.twL = p->twL;
    s.L = (int)p->L;
    s.P = (int)p->P;
    s.Q = p->Q;
    s.Qh = p->Qh;
    return s;
}

inline void desc_from_plan(CpDesc &c, const fcs_plan *p) {
    c.N = p->N;
    c.D = p->D;
    for (int n = 0; n < p->N; ++n) {
        c.I[n] = (int)p->I[n];
        c.J[n] = (int)p->J[n];
        c.ioff[n] = p->ioff[n];
        c.off[n] = p->off[n];
    }
    c.inv = p->inv;
    c.iblock = p->iblock;
    c.tab = p->tab;
    c.sumI = p->sumI;
    c.s = slice_args(p);
    c.Jt = p->Jt;
}

// LDS bytes a kernel of FFT size P needs for a computation.
__host__ __device__ inline size_t cp_lds_bytes(int P, const CpDesc &c) {
    size_t b = (size_t)(P + P / 16) * 8;
    if ((c.kind == FCS_DESC_KRON || c.kind == FCS_DESC_CONTRACTION) && !c.kbins) {
        const size_t na = (size_t)(c.J[0] + c.J[1] - 1), nb = (size_t)(c.J[2] + c.J[3] - 1);
        b = na * 8 > b ? na * 8 : b;
        b = nb * 8 > b ? nb * 8 : b;
    }
    return b;
}

}  // namespace fcscp
