// Instantiations of the fused stage kernel: forward, FP32 filter bank; the
// final reaction kernel of the forward.
#include "tnrd_fused_tile.hpp"

namespace tnrd {

hipError_t fused_launch_fwd_f32(const StageArgs &s, int th, int tw, int nb, int nw, int rbfm,
                                hipStream_t stream)
{
    const int nmb = (s.Nk + 15) / 16;
    if (s.ks == 7)
        return nmb <= 2 ? fused_form<7, 2, MODE_FWD, PREC_F32>(s, th, tw, nb, nw, rbfm, stream)
                        : fused_form<7, 3, MODE_FWD, PREC_F32>(s, th, tw, nb, nw, rbfm, stream);
    if (s.ks == 5)
        return nmb <= 2 ? fused_form<5, 2, MODE_FWD, PREC_F32>(s, th, tw, nb, nw, rbfm, stream)
                        : fused_form<5, 3, MODE_FWD, PREC_F32>(s, th, tw, nb, nw, rbfm, stream);
    return hipErrorInvalidValue;
}

hipError_t fused_launch_final(const StageArgs &s, int th, int tw, hipStream_t stream)
{
    if (s.ks == 7) return launch_react_final<7>(s, th, tw, stream);
    if (s.ks == 5) return launch_react_final<5>(s, th, tw, stream);
    return hipErrorInvalidValue;
}

}  // namespace tnrd
