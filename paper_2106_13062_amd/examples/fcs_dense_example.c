/*
 * The C ABI on its own (no Python): plan, hash tables, workspace and the
 * dense FCS (Definition 4, Section 3.2) of a small integer-valued order-3
 * tensor, printed as text.  Device memory comes from the HIP runtime; the
 * library allocates nothing.
 *
 * Tensor: vec(T)[i] = ((i * 7919) mod 7) - 3 for i < 20 * 15 * 10 (mode 0
 * fastest); hash lengths (16, 8, 4), D = 2 sketches, seed 5.
 * Output: a line "D J~", then one line of J~ values per sketch.
 * Exit status 0 on success, 1 on any error (reported on stderr).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "fcs.h"

#define HIP_OK(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));         \
            return 1;                                                                 \
        }                                                                             \
    } while (0)

#define FCS_OK_(call)                                                                 \
    do {                                                                              \
        fcs_status s_ = (call);                                                       \
        if (s_ != FCS_OK) {                                                           \
            fprintf(stderr, "%s failed: %s (%s)\n", #call, fcs_status_str(s_),        \
                    fcs_last_error());                                                \
            return 1;                                                                 \
        }                                                                             \
    } while (0)

int main(void) {
    const int64_t I[3] = {20, 15, 10};
    const int64_t J[3] = {16, 8, 4};
    const int32_t D = 2;
    fcs_plan_desc desc = {3, I, J, D, 5, 0};
    fcs_plan_t plan = NULL;
    FCS_OK_(fcs_plan_create(&desc, &plan));

    void *tables = NULL;
    HIP_OK(hipMalloc(&tables, fcs_plan_table_bytes(plan)));
    FCS_OK_(fcs_plan_bind(plan, tables, NULL));
    int64_t Jt = 0;
    FCS_OK_(fcs_plan_info(plan, &Jt, NULL, NULL, NULL));

    const size_t n = (size_t)(I[0] * I[1] * I[2]);
    float *host = (float *)malloc(n * sizeof(float));
    float *sketch = (float *)malloc((size_t)D * (size_t)Jt * sizeof(float));
    if (!host || !sketch) {
        fprintf(stderr, "host allocation failed\n");
        return 1;
    }
    for (size_t i = 0; i < n; ++i) host[i] = (float)((int)((i * 7919u) % 7u) - 3);

    float *T = NULL, *out = NULL;
    void *ws = NULL;
    const size_t ws_bytes = fcs_workspace_bytes(plan, FCS_OP_DENSE, 0, 0);
    HIP_OK(hipMalloc((void **)&T, n * sizeof(float)));
    HIP_OK(hipMalloc((void **)&out, (size_t)D * (size_t)Jt * sizeof(float)));
    HIP_OK(hipMalloc(&ws, ws_bytes));
    HIP_OK(hipMemcpy(T, host, n * sizeof(float), hipMemcpyHostToDevice));

    FCS_OK_(fcs_sketch_dense(plan, T, out, ws, ws_bytes, NULL));
    HIP_OK(hipDeviceSynchronize());
    HIP_OK(hipMemcpy(sketch, out, (size_t)D * (size_t)Jt * sizeof(float), hipMemcpyDeviceToHost));

    printf("%d %lld\n", D, (long long)Jt);
    for (int d = 0; d < D; ++d) {
        for (int64_t j = 0; j < Jt; ++j) printf(j ? " %.1f" : "%.1f", sketch[(size_t)d * Jt + j]);
        printf("\n");
    }

    HIP_OK(hipFree(ws));
    HIP_OK(hipFree(out));
    HIP_OK(hipFree(T));
    HIP_OK(hipFree(tables));
    FCS_OK_(fcs_plan_destroy(plan));
    free(sketch);
    free(host);
    return 0;
}
