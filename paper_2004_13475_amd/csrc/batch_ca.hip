// batch_ca.hip -- batched LDS-engine step kernels for rule RULE_CA.
#include "batch_kernels.hpp"

namespace fractal {

TileFn pick_batch_ca(int r, int threads, int flags)
{
    return pick_batch_kernel<RULE_CA>(r, threads, flags);
}

} // namespace fractal
