// step_bb.hip -- instantiations of the step kernel for map MAP_BB.
#include "step_kernel.hpp"

namespace fractal {

StepFn pick_step_bb(int rule, int r, int threads, int flags)
{
    return pick_step_kernel<MAP_BB>(rule, r, threads, flags);
}

} // namespace fractal
