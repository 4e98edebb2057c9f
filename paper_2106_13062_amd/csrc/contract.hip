// Sketched inner products and the median over D independent sketches
// (Proposition 1; Section 4 computes D sketches and returns the median).
#include "fcs_internal.h"

#include "median.h"

namespace {

constexpr int IP_THREADS = 256;

// One workgroup per sketch d: ip_d = sum_j a[d][j] * b[d][j].  Each float
// product is exact in double; the sum is a double wavefront tree reduction.
__global__ __launch_bounds__(IP_THREADS) void inner_kernel(const float *a, const float *b, int64_t Jt,
                                                           double *per_d) {
    const int d = blockIdx.x;
    const float *x = a + (int64_t)d * Jt;
    const float *y = b + (int64_t)d * Jt;
    double acc = 0.0;
    for (int64_t j = threadIdx.x; j < Jt; j += IP_THREADS) acc += (double)x[j] * (double)y[j];
    acc = fcs_block_sum_f64<IP_THREADS>(acc);
    if (threadIdx.x == 0) per_d[d] = acc;
}

__global__ void median_kernel(const double *v, int D, double *out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *out = fcs_median_small(v, D);
}

}  // namespace

size_t fcs_ws_inner(const fcs_plan *p) {
    return (((size_t)p->D * sizeof(double)) + 255) & ~(size_t)255;
}

static fcs_status inner_median(int D, int64_t len, const float *a, const float *b, double *median, double *per_d,
                               void *ws, size_t ws_bytes, hipStream_t s) {
    if (!a || !b || !median) FCS_FAIL(FCS_EINVAL, "null sketch or output");
    if (D < 1 || D > FCS_MAX_D) FCS_FAIL(FCS_EINVAL, "D=%d outside [1, %d]", D, FCS_MAX_D);
    if (len < 1) FCS_FAIL(FCS_EINVAL, "sketch length %lld < 1", (long long)len);
    double *buf = per_d;
    if (!buf) {
        const size_t need = (((size_t)D * sizeof(double)) + 255) & ~(size_t)255;
        if (!ws) FCS_FAIL(FCS_EINVAL, "null workspace (needed when per_d is NULL)");
        if (ws_bytes < need) FCS_FAIL(FCS_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
        if (!fcs_aligned(ws, 8)) FCS_FAIL(FCS_EINVAL, "workspace not 8-byte aligned");
        buf = (double *)ws;
    }
    inner_kernel<<<D, IP_THREADS, 0, s>>>(a, b, len, buf);
    FCS_LAUNCH_CHECK();
    median_kernel<<<1, 64, 0, s>>>(buf, D, median);
    FCS_LAUNCH_CHECK();
    return FCS_OK;
}

extern "C" fcs_status fcs_contract_inner(fcs_plan_t p, const float *a, const float *b, double *median,
                                         double *per_d, void *ws, size_t ws_bytes, void *stream) {
    fcs_clear_error();
    if (!p) FCS_FAIL(FCS_EINVAL, "null plan");
    return inner_median(p->D, p->Jt, a, b, median, per_d, ws, ws_bytes, (hipStream_t)stream);
}

extern "C" fcs_status fcs_inner_median(int32_t D, int64_t len, const float *a, const float *b, double *median,
                                       double *per_d, void *ws, size_t ws_bytes, void *stream) {
    fcs_clear_error();
    return inner_median(D, len, a, b, median, per_d, ws, ws_bytes, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Tensor sketch (Definition 2) from a fast count sketch under the same hash
// pairs: with every J_n = J the tensor sketch's bin is (sum_n h_n) mod J, so
// TS[k] = sum over m = k (mod J) of FCS[m].  One thread per output entry
// adds its at most N terms in order of m.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void ts_fold_kernel(const float *y, float *ts, int D, int64_t Jt, int64_t J) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)D * J) return;
    const int64_t d = t / J;
    const int64_t k = t - d * J;
    const float *src = y + d * Jt;
    float v = 0.f;
    for (int64_t m = k; m < Jt; m += J) v += src[m];
    ts[t] = v;
}

extern "C" fcs_status fcs_ts_fold(fcs_plan_t p, const float *y, float *ts, void *stream) {
    fcs_clear_error();
    if (!p) FCS_FAIL(FCS_EINVAL, "null plan");
    if (!y || !ts) FCS_FAIL(FCS_EINVAL, "null sketch or output");
    if (p->hcs) FCS_FAIL(FCS_EINVAL, "a tensor sketch folds a fast count sketch, not a higher-order count sketch");
    for (int n = 1; n < p->N; ++n)
        if (p->J[n] != p->J[0]) FCS_FAIL(FCS_EINVAL, "a tensor sketch needs equal hash lengths (J_%d != J_0)", n);
    const int64_t J = p->J[0];
    const int64_t total = (int64_t)p->D * J;
    ts_fold_kernel<<<(unsigned)fcs_ceil_div(total, 256), 256, 0, (hipStream_t)stream>>>(y, ts, p->D, p->Jt, J);
    FCS_LAUNCH_CHECK();
    return FCS_OK;
}
