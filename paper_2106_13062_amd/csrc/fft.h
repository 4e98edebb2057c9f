// LDS-resident complex FFT of P = 2^p points (256 <= P <= 16384) for one
// workgroup, written for gfx950 wave64.
//
// Algorithm: Stockham autosort (natural order in and out, no bit reversal),
// radix-E passes where E = P / T elements live in each of the T threads; the
// first pass takes the leftover radix (2, 4 or 8) so the last pass is radix E
// with exactly one butterfly per thread.  Between passes the data goes
// through LDS with one padding slot per 16 complex values (b64 accesses by 16
// consecutive lanes then hit distinct banks).  The last pass leaves the
// transform in registers: thread t holds X[t + e*T], e = 0..E-1.
// Twiddles W_P^k = exp(-2 pi i k / P) come from a table built in double
// precision; the radix-E butterflies use exact constants.
#pragma once

#include <hip/hip_runtime.h>

namespace fcsfft {

__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }

// threadIdx.x through an opaque move: address arithmetic that depends on it
// is then not hoisted out of the callers' rank / mode / slice loops (hoisted
// addresses of every pass would stay live and spill to scratch)
__device__ __forceinline__ int tid_opaque() {
    int t;
    asm volatile("v_mov_b32 %0, %1" : "=v"(t) : "v"((int)threadIdx.x));
    return t;
}

template <int P>
struct Lds {
    static constexpr int elems = P + P / 16;
    static constexpr int bytes = elems * 8;
};

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {   // a * conj(b)
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }

// cos(2 pi k / 16) for k = 0..4 (the other values follow by symmetry)
constexpr float C16[5] = {1.0f, 0.923879532511286756f, 0.707106781186547524f, 0.382683432365089772f, 0.0f};

// multiply by W_16^k = exp(-2 pi i k / 16), exact special cases for k = 0, 4, 8, 12
template <int K>
__device__ __forceinline__ float2 w16(float2 v) {
    constexpr int k = K & 15;
    if constexpr (k == 0) {
        return v;
    } else if constexpr (k == 4) {               // -i
        return make_float2(v.y, -v.x);
    } else if constexpr (k == 8) {               // -1
        return make_float2(-v.x, -v.y);
    } else if constexpr (k == 12) {              // +i
        return make_float2(-v.y, v.x);
    } else {
        // cos and -sin of 2 pi k / 16
        constexpr int kc = (k <= 4) ? k : (k <= 8) ? 8 - k : (k <= 12) ? k - 8 : 16 - k;
        constexpr float c0 = C16[kc];
        constexpr float s0 = C16[4 - kc];
        constexpr float c = (k <= 4 || k >= 12) ? c0 : -c0;
        constexpr float s = (k <= 8) ? s0 : -s0;   // sin(2 pi k / 16)
        return make_float2(v.x * c + v.y * s, v.y * c - v.x * s);
    }
}

template <int R>
constexpr int bitrev(int i) {
    int r = 0;
    for (int b = 1; b < R; b <<= 1) {
        r = (r << 1) | (i & 1);
        i >>= 1;
    }
    return r;
}

// In-register forward DFT of R = 2, 4, 8 or 16 points (radix-2 DIT network
// with exact twiddles): X[k] = sum_n x[n] exp(-2 pi i n k / R).
template <int R>
__device__ __forceinline__ void dft(float2 (&v)[R]) {
    float2 t[R];
#pragma unroll
    for (int i = 0; i < R; ++i) t[bitrev<R>(i)] = v[i];
    // stage with butterfly half-size s uses W_{2s}^j = W_16^{j * 16 / (2s)}
#define FCS_STAGE(S)                                                              \
    if constexpr (R > S) {                                                        \
        _Pragma("unroll") for (int k = 0; k < R; k += 2 * S) {                    \
            _Pragma("unroll") for (int j = 0; j < S; ++j) {                       \
                float2 b = t[k + j + S];                                          \
                if (j == 0) {                                                     \
                } else if (S == 2) {                                              \
                    b = w16<4>(b);                                                \
                } else if (S == 4) {                                              \
                    if (j == 1) b = w16<2>(b);                                    \
                    if (j == 2) b = w16<4>(b);                                    \
                    if (j == 3) b = w16<6>(b);                                    \
                } else {                                                          \
                    if (j == 1) b = w16<1>(b);                                    \
                    if (j == 2) b = w16<2>(b);                                    \
                    if (j == 3) b = w16<3>(b);                                    \
                    if (j == 4) b = w16<4>(b);                                    \
                    if (j == 5) b = w16<5>(b);                                    \
                    if (j == 6) b = w16<6>(b);                                    \
                    if (j == 7) b = w16<7>(b);                                    \
                }                                                                 \
                const float2 a = t[k + j];                                        \
                t[k + j] = cadd(a, b);                                            \
                t[k + j + S] = csub(a, b);                                        \
            }                                                                     \
        }                                                                         \
    }
    FCS_STAGE(1)
    FCS_STAGE(2)
    FCS_STAGE(4)
    FCS_STAGE(8)
#undef FCS_STAGE
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = t[i];
}

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }

// Threads and elements per thread for a P-point transform.
template <int P>
struct Shape {
    static constexpr int T = P >= 1024 ? P / 16 : 64;
    static constexpr int E = P / T;                       // 4, 8 or 16
    static constexpr int LE = ilog2(E);
    static constexpr int LP = ilog2(P);
    static constexpr int R0 = 1 << (LP % LE == 0 ? LE : LP % LE);   // first-pass radix
    static constexpr int NPASS = (LP % LE == 0) ? LP / LE : LP / LE + 1;
};

// One Stockham pass of radix R with Ns = product of earlier radices, on the
// thread's E values v (B = E / R butterflies).  Reads every input of the
// thread first, synchronises, then writes (the same LDS buffer is used in
// place).  LAST leaves the outputs in v: v[r] = X[t + r*T].
template <int P, int R, int NS, bool LAST>
__device__ __forceinline__ void pass(float2 *lds, const float2 *__restrict__ tw, float2 (&v)[Shape<P>::E]) {
    constexpr int T = Shape<P>::T;
    constexpr int B = P / R / T;        // butterflies per thread
    const int t = tid_opaque();
    // the pass's twiddles do not depend on the data: their loads are issued
    // first so that the latency overlaps the LDS reads and the barrier.  For
    // radix 8 and 16 only W^1 and W^4 are loaded and the other powers are
    // formed by at most three complex products (error a few ulp).
    float2 w[NS > 1 ? B : 1][R];
    if constexpr (NS > 1) {
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int jm = (t + T * b) % NS;
            constexpr int st = P / (NS * R);
            if constexpr (R >= 8) {
                w[b][1] = tw[jm * st];
                w[b][4] = tw[4 * jm * st];
            } else {
#pragma unroll
                for (int r = 1; r < R; ++r) w[b][r] = tw[r * jm * st];
            }
        }
    }
    // pad(i + c) = pad(i) + c + c / 16 when c is a multiple of 16: one
    // padded base per butterfly and constant offsets
    constexpr int SR = P / R;
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int j = t + T * b;
        if constexpr (SR % 16 == 0) {
            const float2 *src = lds + pad(j);
#pragma unroll
            for (int r = 0; r < R; ++r) v[b * R + r] = src[r * (SR + SR / 16)];
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) v[b * R + r] = lds[pad(j + r * SR)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int j = t + T * b;
        float2 u[R];
#pragma unroll
        for (int r = 0; r < R; ++r) u[r] = v[b * R + r];
        if constexpr (NS > 1) {
            if constexpr (R >= 8) {
                float2 (&x)[R] = w[b];
                x[2] = cmul(x[1], x[1]);
                x[3] = cmul(x[2], x[1]);
                x[5] = cmul(x[4], x[1]);
                x[6] = cmul(x[4], x[2]);
                x[7] = cmul(x[4], x[3]);
                if constexpr (R == 16) {
                    x[8] = cmul(x[4], x[4]);
#pragma unroll
                    for (int r = 9; r < 16; ++r) x[r] = cmul(x[8], x[r - 8]);
                }
            }
#pragma unroll
            for (int r = 1; r < R; ++r) u[r] = cmul(u[r], w[b][r]);
        }
        dft<R>(u);
        if constexpr (LAST) {
            static_assert(B == 1, "last pass has one butterfly per thread");
#pragma unroll
            for (int r = 0; r < R; ++r) v[r] = u[r];
        } else {
            const int idxD = (j / NS) * NS * R + (j % NS);
            if constexpr (NS % 16 == 0) {
                float2 *dst = lds + pad(idxD);
#pragma unroll
                for (int r = 0; r < R; ++r) dst[r * (NS + NS / 16)] = u[r];
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) lds[pad(idxD + r * NS)] = u[r];
            }
        }
    }
    if constexpr (!LAST) __syncthreads();
}

// Forward FFT of the P values in lds (natural order, padded); returns
// X[t + e*T] in out[e].  lds is clobbered.
template <int P>
__device__ __forceinline__ void forward(float2 *lds, const float2 *__restrict__ tw, float2 (&out)[Shape<P>::E]) {
    using S = Shape<P>;
    constexpr int E = S::E;
    constexpr int R0 = S::R0;
    if constexpr (S::NPASS == 1) {
        pass<P, E, 1, true>(lds, tw, out);
    } else {
        pass<P, R0, 1, false>(lds, tw, out);
        if constexpr (S::NPASS == 2) {
            pass<P, E, R0, true>(lds, tw, out);
        } else {
            pass<P, E, R0, false>(lds, tw, out);
            if constexpr (S::NPASS == 3) {
                pass<P, E, R0 * E, true>(lds, tw, out);
            } else {
                pass<P, E, R0 * E, false>(lds, tw, out);
                static_assert(S::NPASS == 4, "P <= 16384");
                pass<P, E, R0 * E * E, true>(lds, tw, out);
            }
        }
    }
}

// Forward FFT of values the thread already holds: v[e] = x[t + e*T] (its own
// natural-order positions, which are exactly the inputs of its first-pass
// butterflies).  The first pass reads no LDS and needs no barrier before it;
// returns X[t + e*T] in v.  lds is clobbered and must not be in use.
template <int P>
__device__ __forceinline__ void forward_regs(float2 *lds, const float2 *__restrict__ tw, float2 (&v)[Shape<P>::E]) {
    using S = Shape<P>;
    constexpr int T = S::T;
    constexpr int E = S::E;
    constexpr int R0 = S::R0;
    constexpr int B = E / R0;
    static_assert(S::NPASS >= 2, "first pass is never the last");
    const int t = tid_opaque();
    // first pass (NS = 1): butterfly b takes x[j + r P/R0], j = t + T b,
    // that is v[b + r B]; its outputs go to positions j R0 + r
#pragma unroll
    for (int b = 0; b < B; ++b) {
        float2 u[R0];
#pragma unroll
        for (int r = 0; r < R0; ++r) u[r] = v[b + r * B];
        dft<R0>(u);
        const int j = t + T * b;
#pragma unroll
        for (int r = 0; r < R0; ++r) lds[pad(j * R0 + r)] = u[r];
    }
    __syncthreads();
    if constexpr (S::NPASS == 2) {
        pass<P, E, R0, true>(lds, tw, v);
    } else {
        pass<P, E, R0, false>(lds, tw, v);
        if constexpr (S::NPASS == 3) {
            pass<P, E, R0 * E, true>(lds, tw, v);
        } else {
            pass<P, E, R0 * E, false>(lds, tw, v);
            static_assert(S::NPASS == 4, "P <= 16384");
            pass<P, E, R0 * E * E, true>(lds, tw, v);
        }
    }
}

// Unnormalised inverse transform (exp(+2 pi i jk/P)) of the values in lds,
// through conj(FFT(conj(x))).  Returns x[t + e*T] in out[e].
template <int P>
__device__ __forceinline__ void inverse(float2 *lds, const float2 *__restrict__ tw, float2 (&out)[Shape<P>::E]) {
    constexpr int T = Shape<P>::T;
    for (int k = tid_opaque(); k < P; k += T) {
        float2 v = lds[pad(k)];
        lds[pad(k)] = conjf2(v);
    }
    __syncthreads();
    forward<P>(lds, tw, out);
#pragma unroll
    for (int e = 0; e < Shape<P>::E; ++e) out[e] = conjf2(out[e]);
}

// Store register values X[t + e*T] back to lds in natural order.
template <int P>
__device__ __forceinline__ void store(float2 *lds, const float2 (&v)[Shape<P>::E]) {
    constexpr int T = Shape<P>::T;
    static_assert(T % 16 == 0, "thread count is a multiple of 16");
    float2 *dst = lds + pad(tid_opaque());
#pragma unroll
    for (int e = 0; e < Shape<P>::E; ++e) dst[e * (T + T / 16)] = v[e];
}

}  // namespace fcsfft
