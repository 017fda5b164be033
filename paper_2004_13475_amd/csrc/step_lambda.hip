// step_lambda.hip -- instantiations of the step kernel for map MAP_LAMBDA.
#include "step_kernel.hpp"

namespace fractal {

StepFn pick_step_lambda(int rule, int r, int threads, int flags)
{
    return pick_step_kernel<MAP_LAMBDA>(rule, r, threads, flags);
}

} // namespace fractal
