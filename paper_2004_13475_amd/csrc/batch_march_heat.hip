// batch_march_heat.hip -- batch march kernels of the heat rule.
#include "batch_march.hpp"

namespace fractal {

BatchMarchFn pick_batch_march_heat(int r, int T, bool nt)
{
    return bm_pick_rule<RULE_HEAT>(r, T, nt);
}

} // namespace fractal
