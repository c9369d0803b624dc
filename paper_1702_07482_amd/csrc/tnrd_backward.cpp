// Backward pass (in progress).
#include "tnrd.h"
#include "tnrd_api_internal.hpp"

namespace tnrd {
size_t backward_ws_bytes(int, int, int, const tnrd_model *, const tnrd_opts &, int) { return 0; }
}  // namespace tnrd

extern "C" {
int tnrd_backward(const float *, int, int, int, int, const tnrd_model *, const float *,
                  const float *, float *, float *, float *, float *, const tnrd_opts *, void *,
                  size_t, void *)
{
    return TNRD_ERR_UNSUPPORTED;
}
size_t tnrd_batched_workspace_bytes(int, const tnrd_image *, int, const tnrd_model *,
                                    const tnrd_opts *)
{
    return 0;
}
int tnrd_forward_batched(int, const tnrd_image *, int, const tnrd_model *, const tnrd_opts *,
                         void *, size_t, void *)
{
    return TNRD_ERR_UNSUPPORTED;
}
}
