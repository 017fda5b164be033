// step_march_heat.hip -- the register-march step kernels of the heat rule.
#include "march_pick.hpp"

namespace fractal {

MarchFn pick_march_heat(int map, int r, int T, bool nt, bool alt)
{
    return march_pick_rule<RULE_HEAT>(map, r, T, nt, alt);
}

} // namespace fractal
