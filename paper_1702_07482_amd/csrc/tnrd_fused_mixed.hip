// Instantiations of the fused stage kernel: forward, BF16/FP16 filter-bank
// operands (7x7 filters).
#include "tnrd_fused_tile.hpp"

namespace tnrd {

hipError_t fused_launch_fwd_mixed(const StageArgs &s, int th, int tw, int nb, int nw, int rbfm,
                                  hipStream_t stream)
{
    const int nmb = (s.Nk + 15) / 16;
    if (s.ks != 7) return hipErrorInvalidValue;
    if (s.prec == PREC_BF16)
        return nmb <= 2 ? fused_form<7, 2, MODE_FWD, PREC_BF16>(s, th, tw, nb, nw, rbfm, stream)
                        : fused_form<7, 3, MODE_FWD, PREC_BF16>(s, th, tw, nb, nw, rbfm, stream);
    if (s.prec == PREC_F16)
        return nmb <= 2 ? fused_form<7, 2, MODE_FWD, PREC_F16>(s, th, tw, nb, nw, rbfm, stream)
                        : fused_form<7, 3, MODE_FWD, PREC_F16>(s, th, tw, nb, nw, rbfm, stream);
    return hipErrorInvalidValue;
}

}  // namespace tnrd
