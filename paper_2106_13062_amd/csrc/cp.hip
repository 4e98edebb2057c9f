// CP sketch, spectra and T(I, u, v) contractions (Sections 3.1 and 4.1).
#include "fcs_internal.h"

size_t fcs_ws_cp(const fcs_plan *, int64_t) { return 256; }
size_t fcs_ws_free_mode(const fcs_plan *, int64_t) { return 256; }
size_t fcs_ws_spectrum(const fcs_plan *) { return 256; }

extern "C" fcs_status fcs_sketch_cp(fcs_plan_t, int64_t, const float *const *, const float *, float *,
                                    float *, void *, size_t, void *) {
    FCS_FAIL(FCS_EUNSUPPORTED, "CP sketch not built yet");
}

extern "C" fcs_status fcs_sketch_spectrum(fcs_plan_t, const float *, float *, void *, size_t, void *) {
    FCS_FAIL(FCS_EUNSUPPORTED, "spectrum not built yet");
}

extern "C" fcs_status fcs_contract_free_mode(fcs_plan_t, const float *, int32_t, int64_t,
                                             const float *const *, double *, void *, size_t, void *) {
    FCS_FAIL(FCS_EUNSUPPORTED, "free-mode contraction not built yet");
}
