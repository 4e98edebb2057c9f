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

extern "C" fcs_status fcs_contract_inner(fcs_plan_t p, const float *a, const float *b, double *median,
                                         double *per_d, void *ws, size_t ws_bytes, void *stream) {
    fcs_clear_error();
    if (!p) FCS_FAIL(FCS_EINVAL, "null plan");
    if (!a || !b || !median) FCS_FAIL(FCS_EINVAL, "null sketch or output");
    double *buf = per_d;
    if (!buf) {
        if (!ws) FCS_FAIL(FCS_EINVAL, "null workspace (needed when per_d is NULL)");
        if (ws_bytes < fcs_ws_inner(p))
            FCS_FAIL(FCS_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, fcs_ws_inner(p));
        if (!fcs_aligned(ws, 8)) FCS_FAIL(FCS_EINVAL, "workspace not 8-byte aligned");
        buf = (double *)ws;
    }
    hipStream_t s = (hipStream_t)stream;
    inner_kernel<<<p->D, IP_THREADS, 0, s>>>(a, b, p->Jt, buf);
    FCS_LAUNCH_CHECK();
    median_kernel<<<1, 64, 0, s>>>(buf, p->D, median);
    FCS_LAUNCH_CHECK();
    return FCS_OK;
}
