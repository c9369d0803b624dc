// Instantiations of the fused stage kernel: input-gradient mode (polynomial
// and Gaussian forms of phi'), FP32 and BF16/FP16 filter-bank operands.
#include "tnrd_fused_tile.hpp"

namespace tnrd {

hipError_t fused_launch_bwd(const StageArgs &s, int th, int tw, int nb, int nw, int rbfm,
                            hipStream_t stream)
{
    const int nmb = (s.Nk + 15) / 16;
    constexpr int M = MODE_BWD_INPUT;
    if (s.prec == PREC_BF16 || s.prec == PREC_F16) {
        if (s.ks != 7) return hipErrorInvalidValue;
        if (s.prec == PREC_BF16)
            return nmb <= 2 ? fused_form<7, 2, M, PREC_BF16>(s, th, tw, nb, nw, rbfm, stream)
                            : fused_form<7, 3, M, PREC_BF16>(s, th, tw, nb, nw, rbfm, stream);
        return nmb <= 2 ? fused_form<7, 2, M, PREC_F16>(s, th, tw, nb, nw, rbfm, stream)
                        : fused_form<7, 3, M, PREC_F16>(s, th, tw, nb, nw, rbfm, stream);
    }
    if (s.ks == 7)
        return nmb <= 2 ? fused_form<7, 2, M, PREC_F32>(s, th, tw, nb, nw, rbfm, stream)
                        : fused_form<7, 3, M, PREC_F32>(s, th, tw, nb, nw, rbfm, stream);
    if (s.ks == 5)
        return nmb <= 2 ? fused_form<5, 2, M, PREC_F32>(s, th, tw, nb, nw, rbfm, stream)
                        : fused_form<5, 3, M, PREC_F32>(s, th, tw, nb, nw, rbfm, stream);
    return hipErrorInvalidValue;
}

hipError_t fused_launch_grad_finish(const StageArgs &s, int th, int tw, hipStream_t stream)
{
    if (s.ks == 7) return launch_grad_finish<7>(s, th, tw, stream);
    if (s.ks == 5) return launch_grad_finish<5>(s, th, tw, stream);
    return hipErrorInvalidValue;
}

}  // namespace tnrd
