// Batched forward over uneven images (in progress).
#include "tnrd.h"

extern "C" {
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
