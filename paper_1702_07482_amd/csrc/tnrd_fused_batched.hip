// Instantiations of the fused stage kernel for the batched forward (one launch
// per stage over the tiles of every image).
#include "tnrd_fused_tile.hpp"

namespace tnrd {

hipError_t batched_launch_impl(const BatchArgs &a, int ks, int nb, int nw, int rbfm,
                               hipStream_t stream)
{
    const int nmb = (a.Nk + 15) / 16;
    const bool poly = rbfm == RBF_POLY;
    if (ks == 7) {
        if (nmb <= 2) return poly ? batched_nb<7, 2, RBF_POLY>(a, nb, nw, stream)
                                  : batched_nb<7, 2, RBF_HORNER>(a, nb, nw, stream);
        return poly ? batched_nb<7, 3, RBF_POLY>(a, nb, nw, stream)
                    : batched_nb<7, 3, RBF_HORNER>(a, nb, nw, stream);
    }
    if (ks == 5) {
        if (nmb <= 2) return poly ? batched_nb<5, 2, RBF_POLY>(a, nb, nw, stream)
                                  : batched_nb<5, 2, RBF_HORNER>(a, nb, nw, stream);
        return poly ? batched_nb<5, 3, RBF_POLY>(a, nb, nw, stream)
                    : batched_nb<5, 3, RBF_HORNER>(a, nb, nw, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace tnrd
