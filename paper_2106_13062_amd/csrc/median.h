// Device helpers for the median over D independent sketches (Section 4) and
// double-precision block reductions.
#pragma once

#include <hip/hip_runtime.h>

// Value of rank t (0-based, ascending) among v[0..n): the element whose
// interval [#less, #less + #equal) contains t.  O(n^2), for small n.
__device__ inline double fcs_rank_select(const double *v, int n, int t) {
    for (int j = 0; j < n; ++j) {
        int less = 0, eq = 0;
        for (int k = 0; k < n; ++k) {
            less += v[k] < v[j];
            eq += v[k] == v[j];
        }
        if (less <= t && t < less + eq) return v[j];
    }
    return v[0];
}

// Median with the usual convention: the middle value for odd n, the mean of
// the two middle values for even n.
__device__ inline double fcs_median_small(const double *v, int n) {
    const double lo = fcs_rank_select(v, n, (n - 1) / 2);
    if (n & 1) return lo;
    const double hi = fcs_rank_select(v, n, n / 2);
    return 0.5 * (lo + hi);
}

// Same selection on a register array whose first n of MAXD entries are live;
// float inputs, the mean of the middle pair is formed in double.
template <int MAXD>
__device__ inline double fcs_median_reg(const float (&v)[MAXD], int n) {
    const int t1 = (n - 1) / 2, t2 = n / 2;
    float m1 = v[0], m2 = v[0];
#pragma unroll
    for (int j = 0; j < MAXD; ++j) {
        int less = 0, eq = 0;
#pragma unroll
        for (int k = 0; k < MAXD; ++k) {
            const bool live = k < n;
            less += (live && v[k] < v[j]) ? 1 : 0;
            eq += (live && v[k] == v[j]) ? 1 : 0;
        }
        const bool livej = j < n;
        if (livej && less <= t1 && t1 < less + eq) m1 = v[j];
        if (livej && less <= t2 && t2 < less + eq) m2 = v[j];
    }
    return 0.5 * ((double)m1 + (double)m2);
}

template <int THREADS>
__device__ inline double fcs_block_sum_f64(double x) {
    __shared__ double part[THREADS / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) part[w] = x;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        for (int k = 0; k < THREADS / 64; ++k) t += part[k];
    }
    __syncthreads();
    return t;
}
