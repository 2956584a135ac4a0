// spcn_pending.hip -- operations not built yet in this library: workspace sizes are 0 and the
// entry points report SPCN_E_UNSUPPORTED.
#include "spcn_internal.h"
namespace spcn {
size_t batched_workspace_bytes(int64_t, int64_t) { return 0; }
size_t f32_forward_workspace_bytes(int64_t, int64_t) { return 0; }
size_t f32_backward_workspace_bytes(int64_t, int64_t) { return 0; }
}  // namespace spcn
extern "C" {
spcn_status spcn_normalize_batched(const spcn_tile*, int32_t, int64_t, const float*, const float*, const float*,
                                   const float*, const spcn_params*, float*, float*, int32_t*, void*, size_t,
                                   hipStream_t) {
    return spcn::fail(SPCN_E_UNSUPPORTED, "spcn_normalize_batched is not built");
}
spcn_status spcn_normalize_f32(const float*, int64_t, int64_t, int64_t, const float*, int64_t, const float*, int64_t,
                               const float*, int64_t, const float*, const spcn_params*, float*, float*, float*,
                               int64_t*, int32_t*, void*, size_t, hipStream_t) {
    return spcn::fail(SPCN_E_UNSUPPORTED, "spcn_normalize_f32 is not built");
}
spcn_status spcn_normalize_backward(const float*, int64_t, int64_t, int64_t, const float*, int64_t, const float*,
                                    int64_t, const float*, int64_t, const float*, const spcn_params*, const float*,
                                    const int64_t*, const int32_t*, const float*, float*, float*, float*, void*,
                                    size_t, hipStream_t) {
    return spcn::fail(SPCN_E_UNSUPPORTED, "spcn_normalize_backward is not built");
}
}
