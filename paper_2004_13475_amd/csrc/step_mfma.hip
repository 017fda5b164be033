// step_mfma.hip -- instantiations of the step kernel for map MAP_MFMA.
#include "step_kernel.hpp"

namespace fractal {

StepFn pick_step_mfma(int rule, int r, int threads, int flags)
{
    return pick_step_kernel<MAP_MFMA>(rule, r, threads, flags);
}

} // namespace fractal
