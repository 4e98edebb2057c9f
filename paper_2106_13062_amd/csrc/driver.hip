// Small dense steps of the decomposition drivers of Section 4.1 (the
// robust tensor power method of Section 4.1.1 and alternating least squares
// of Section 4.1.2) run on sketch-sized data: normalising estimated vectors,
// keeping the start with the largest eigenvalue, deflating a sketch by a
// rank-1 term, and the ALS solve against the Hadamard product of Gram
// matrices.  Reductions are in double (the norms of the estimates); the
// vectors the sketch kernels consume are float.
#include "fcs_internal.h"

#include <algorithm>

namespace {

constexpr int DRV_THREADS = 256;
constexpr int ALS_MAX_R = 90;       // R x R doubles of the Cholesky factor fit in LDS

template <int T>
__device__ __forceinline__ double block_sum(double v, double *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < T / 64; ++w) t += red[w];
    __syncthreads();
    return t;
}

// one workgroup per row: out = in / ||in||_2 (a zero row stays zero)
__global__ __launch_bounds__(DRV_THREADS) void normalize_rows_kernel(const double *in64, const float *in32,
                                                                     float *out, double *norms, int64_t n) {
    __shared__ double red[DRV_THREADS / 64];
    const int64_t r = blockIdx.x;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += DRV_THREADS) {
        const double v = in64 ? in64[r * n + i] : (double)in32[r * n + i];
        s += v * v;
    }
    const double nrm = sqrt(block_sum<DRV_THREADS>(s, red));
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int64_t i = threadIdx.x; i < n; i += DRV_THREADS) {
        const double v = in64 ? in64[r * n + i] : (double)in32[r * n + i];
        out[r * n + i] = (float)(v * inv);
    }
    if (norms && threadIdx.x == 0) norms[r] = nrm;
}

// one workgroup: the first index of the largest value (NaN never wins),
// its value, and a copy of that row
__global__ __launch_bounds__(DRV_THREADS) void select_max_kernel(const double *vals, int64_t P, const float *rows,
                                                                 int64_t n, float *row_out, float *val_out,
                                                                 double *val64_out, int32_t *index_out) {
    __shared__ double bv[DRV_THREADS];
    __shared__ int64_t bi[DRV_THREADS];
    double best = -INFINITY;
    int64_t bidx = -1;
    for (int64_t p = threadIdx.x; p < P; p += DRV_THREADS) {
        const double v = vals[p];
        if (v > best || (bidx < 0 && !(v != v))) {
            best = v;
            bidx = p;
        }
    }
    bv[threadIdx.x] = best;
    bi[threadIdx.x] = bidx;
    __syncthreads();
    for (int w = DRV_THREADS / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const double v = bv[threadIdx.x + w];
            const int64_t i = bi[threadIdx.x + w];
            const int64_t mi = bi[threadIdx.x];
            if (i >= 0 && (mi < 0 || v > bv[threadIdx.x] || (v == bv[threadIdx.x] && i < mi))) {
                bv[threadIdx.x] = v;
                bi[threadIdx.x] = i;
            }
        }
        __syncthreads();
    }
    const int64_t j = bi[0] < 0 ? 0 : bi[0];
    const double v = bi[0] < 0 ? __builtin_nan("") : bv[0];
    for (int64_t i = threadIdx.x; i < n; i += DRV_THREADS) row_out[i] = rows[j * n + i];
    if (threadIdx.x == 0) {
        if (val_out) *val_out = (float)v;
        if (val64_out) *val64_out = v;
        if (index_out) *index_out = (int32_t)j;
    }
}

__global__ __launch_bounds__(DRV_THREADS) void axpy_kernel(int64_t n, float a, const float *x, float *y) {
    const int64_t stride = (int64_t)gridDim.x * DRV_THREADS;
    for (int64_t i = (int64_t)blockIdx.x * DRV_THREADS + threadIdx.x; i < n; i += stride) y[i] += a * x[i];
}

struct AlsArgs {
    int R;
    int64_t In;
    const double *Mt;                    // R x In
    int nother;
    const float *F[FCS_MAX_ORDER];       // R x I_m, row-major
    int64_t Im[FCS_MAX_ORDER];
    double *L;                           // R x R Cholesky factor (lower)
    double *X;                           // R x In solution
};

// G = Hadamard product over the other modes of F_m F_m^T (R x R, double),
// then its Cholesky factor L (G = L L^T), in one workgroup; a non-positive
// pivot (G not positive definite) makes L NaN
__global__ __launch_bounds__(DRV_THREADS) void als_gram_kernel(AlsArgs a) {
    __shared__ double G[ALS_MAX_R * ALS_MAX_R];
    const int R = a.R;
    for (int e = threadIdx.x; e < R * R; e += DRV_THREADS) {
        const int r = e / R, c = e - r * R;
        double g = 1.0;
        if (c <= r) {
            for (int m = 0; m < a.nother; ++m) {
                const float *fr = a.F[m] + (int64_t)r * a.Im[m];
                const float *fc = a.F[m] + (int64_t)c * a.Im[m];
                double s = 0.0;
                for (int64_t i = 0; i < a.Im[m]; ++i) s += (double)fr[i] * (double)fc[i];
                g *= s;
            }
        }
        G[e] = g;
    }
    __syncthreads();
    // right-looking Cholesky on the lower triangle
    for (int k = 0; k < R; ++k) {
        if (threadIdx.x == 0) {
            const double p = G[k * R + k];
            G[k * R + k] = p > 0.0 ? sqrt(p) : __builtin_nan("");
        }
        __syncthreads();
        const double dkk = G[k * R + k];
        for (int i = k + 1 + threadIdx.x; i < R; i += DRV_THREADS) G[i * R + k] /= dkk;
        __syncthreads();
        for (int e = threadIdx.x; e < R * R; e += DRV_THREADS) {
            const int i = e / R, j = e - i * R;
            if (i > k && j > k && j <= i) G[e] -= G[i * R + k] * G[j * R + k];
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < R * R; e += DRV_THREADS) {
        const int i = e / R, j = e - i * R;
        a.L[e] = j <= i ? G[e] : 0.0;
    }
}

// one thread per column i: solve L L^T x = Mt[:, i] (forward then back
// substitution, the column kept in X)
__global__ __launch_bounds__(DRV_THREADS) void als_solve_kernel(AlsArgs a) {
    __shared__ double L[ALS_MAX_R * ALS_MAX_R];
    const int R = a.R;
    for (int e = threadIdx.x; e < R * R; e += DRV_THREADS) L[e] = a.L[e];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * DRV_THREADS + threadIdx.x;
    if (i >= a.In) return;
    double *x = a.X + i;
    const int64_t ld = a.In;
    for (int r = 0; r < R; ++r) {
        double v = a.Mt[(int64_t)r * ld + i];
        for (int j = 0; j < r; ++j) v -= L[r * R + j] * x[(int64_t)j * ld];
        x[(int64_t)r * ld] = v / L[r * R + r];
    }
    for (int r = R - 1; r >= 0; --r) {
        double v = x[(int64_t)r * ld];
        for (int j = r + 1; j < R; ++j) v -= L[j * R + r] * x[(int64_t)j * ld];
        x[(int64_t)r * ld] = v / L[r * R + r];
    }
}

}  // namespace

extern "C" fcs_status fcs_normalize_rows(int64_t P, int64_t n, const double *in64, const float *in32, float *out,
                                         double *norms, void *stream) {
    fcs_clear_error();
    if (P < 0 || n < 1) FCS_FAIL(FCS_EINVAL, "P=%lld rows of n=%lld entries", (long long)P, (long long)n);
    if ((in64 == nullptr) == (in32 == nullptr)) FCS_FAIL(FCS_EINVAL, "give exactly one of the double and float inputs");
    if (!out) FCS_FAIL(FCS_EINVAL, "null output");
    if (P > INT32_MAX) FCS_FAIL(FCS_EUNSUPPORTED, "too many rows");
    if (P == 0) return FCS_OK;
    normalize_rows_kernel<<<(unsigned)P, DRV_THREADS, 0, (hipStream_t)stream>>>(in64, in32, out, norms, n);
    FCS_LAUNCH_CHECK();
    return FCS_OK;
}

extern "C" fcs_status fcs_select_max(int64_t P, const double *vals, int64_t n, const float *rows, float *row_out,
                                     float *val_out, double *val64_out, int32_t *index_out, void *stream) {
    fcs_clear_error();
    if (P < 1 || n < 1) FCS_FAIL(FCS_EINVAL, "P=%lld values, rows of n=%lld", (long long)P, (long long)n);
    if (!vals || !rows || !row_out) FCS_FAIL(FCS_EINVAL, "null values, rows or output row");
    select_max_kernel<<<1, DRV_THREADS, 0, (hipStream_t)stream>>>(vals, P, rows, n, row_out, val_out, val64_out,
                                                                  index_out);
    FCS_LAUNCH_CHECK();
    return FCS_OK;
}

extern "C" fcs_status fcs_axpy(int64_t n, float a, const float *x, float *y, void *stream) {
    fcs_clear_error();
    if (n < 0) FCS_FAIL(FCS_EINVAL, "n < 0");
    if (n > 0 && (!x || !y)) FCS_FAIL(FCS_EINVAL, "null vector");
    if (n == 0) return FCS_OK;
    const unsigned grid = (unsigned)std::min<int64_t>(fcs_ceil_div(n, DRV_THREADS), 4096);
    axpy_kernel<<<grid, DRV_THREADS, 0, (hipStream_t)stream>>>(n, a, x, y);
    FCS_LAUNCH_CHECK();
    return FCS_OK;
}

extern "C" size_t fcs_als_workspace_bytes(int32_t R, int64_t In) {
    if (R < 1 || In < 1) return 0;
    return (((size_t)R * R * 8 + 255) & ~(size_t)255) + (size_t)R * (size_t)In * 8;
}

extern "C" fcs_status fcs_als_update(int32_t R, int64_t In, const double *Mt, int32_t nother,
                                     const float *const *others, const int64_t *Iother, float *Ft_out,
                                     double *lam, void *ws, size_t ws_bytes, void *stream) {
    fcs_clear_error();
    if (R < 1 || R > ALS_MAX_R) FCS_FAIL(FCS_EUNSUPPORTED, "R=%d outside [1, %d]", R, ALS_MAX_R);
    if (In < 1) FCS_FAIL(FCS_EINVAL, "In < 1");
    if (nother < 0 || nother > FCS_MAX_ORDER) FCS_FAIL(FCS_EINVAL, "nother=%d", nother);
    if (!Mt || !Ft_out || !lam) FCS_FAIL(FCS_EINVAL, "null input or output");
    if (nother > 0 && (!others || !Iother)) FCS_FAIL(FCS_EINVAL, "null factor arrays");
    const size_t need = fcs_als_workspace_bytes(R, In);
    if (!ws || ws_bytes < need) FCS_FAIL(FCS_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
    if (!fcs_aligned(ws, 8)) FCS_FAIL(FCS_EINVAL, "workspace not 8-byte aligned");
    AlsArgs a{};
    a.R = R;
    a.In = In;
    a.Mt = Mt;
    a.nother = nother;
    for (int m = 0; m < nother; ++m) {
        if (!others[m] || Iother[m] < 1) FCS_FAIL(FCS_EINVAL, "factor %d", m);
        a.F[m] = others[m];
        a.Im[m] = Iother[m];
    }
    a.L = static_cast<double *>(ws);
    a.X = reinterpret_cast<double *>(static_cast<char *>(ws) + (((size_t)R * R * 8 + 255) & ~(size_t)255));
    hipStream_t s = (hipStream_t)stream;
    als_gram_kernel<<<1, DRV_THREADS, 0, s>>>(a);
    FCS_LAUNCH_CHECK();
    als_solve_kernel<<<(unsigned)fcs_ceil_div(In, DRV_THREADS), DRV_THREADS, 0, s>>>(a);
    FCS_LAUNCH_CHECK();
    normalize_rows_kernel<<<(unsigned)R, DRV_THREADS, 0, s>>>(a.X, nullptr, Ft_out, lam, In);
    FCS_LAUNCH_CHECK();
    return FCS_OK;
}
