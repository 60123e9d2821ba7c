// Entry points whose kernels are not in this build yet.
#include "fv_internal.h"

extern "C" fv_status fv_decode_beam(const fv_trans*, const float*, const float*, int64_t, int32_t, int32_t,
                                    int32_t, int32_t*, float*, int32_t*, uint32_t, void*, size_t, fv_stream_t) {
    return FV_E_UNSUPPORTED;
}
