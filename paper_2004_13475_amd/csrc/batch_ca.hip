// batch_ca.hip -- batched step kernels for rule RULE_CA.
#include "batch_kernels.hpp"

namespace fractal {

void pick_batch_ca(int r, int threads, int flags, TileFn *tf, PersistFn *pf)
{
    pick_batch_kernel<RULE_CA>(r, threads, flags, tf, pf);
}

} // namespace fractal
