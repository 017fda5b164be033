// batch_heat.hip -- batched step kernels for rule RULE_HEAT.
#include "batch_kernels.hpp"

namespace fractal {

void pick_batch_heat(int r, int threads, int flags, TileFn *tf, PersistFn *pf)
{
    pick_batch_kernel<RULE_HEAT>(r, threads, flags, tf, pf);
}

} // namespace fractal
