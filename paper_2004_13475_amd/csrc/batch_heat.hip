// batch_heat.hip -- batched LDS-engine step kernels for rule RULE_HEAT.
#include "batch_kernels.hpp"

namespace fractal {

TileFn pick_batch_heat(int r, int threads, int flags)
{
    return pick_batch_kernel<RULE_HEAT>(r, threads, flags);
}

} // namespace fractal
