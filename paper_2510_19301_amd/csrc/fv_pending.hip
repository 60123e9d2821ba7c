// Entry points whose kernels are not in this build yet.
#include "fv_internal.h"

extern "C" fv_status fv_decode_beam(const fv_trans*, const float*, const float*, int64_t, int32_t, int32_t,
                                    int32_t, int32_t*, float*, int32_t*, uint32_t, void*, size_t, fv_stream_t) {
    return FV_E_UNSUPPORTED;
}
extern "C" fv_status fv_viterbi_backward(int32_t, int32_t, int32_t, const int32_t*, const int32_t*, const float*,
                                         float*, float*, float*, int32_t, void*, size_t, fv_stream_t) {
    return FV_E_UNSUPPORTED;
}
extern "C" fv_status fv_backward_workspace_size(int32_t, int32_t, int32_t, size_t*) { return FV_E_UNSUPPORTED; }
