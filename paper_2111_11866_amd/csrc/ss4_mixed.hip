// Mixed-precision solve: FP32 red-black sweeps on BF16-stored coefficients
// inside an FP64 iterative refinement.
#include "ss4_internal.hpp"

namespace ss4 {

int run_mixed_solve(const WsPlan&, double, const double*, const double*, const subsurf4d_step_params&,
                    subsurf4d_result*, void*, hipStream_t)
{
    set_error("mixed precision is not available in this build");
    return SUBSURF4D_EINVAL;
}

}  // namespace ss4
