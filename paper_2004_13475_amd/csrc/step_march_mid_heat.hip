// step_march_mid_heat.hip -- the register-march step kernels of the heat step
// with 10 and 12 steps per launch (lambda map).
#include "march_pick.hpp"

namespace fractal {

MarchFn pick_march_mid_heat(int r, int T, bool nt)
{
    return march_pick_mid_rule<RULE_HEAT>(r, T, nt);
}

} // namespace fractal
