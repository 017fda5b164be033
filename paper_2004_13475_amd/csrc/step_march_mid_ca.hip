// step_march_mid_ca.hip -- the register-march step kernels of the automaton
// with 10 and 12 steps per launch (lambda map).
#include "march_pick.hpp"

namespace fractal {

MarchFn pick_march_mid_ca(int r, int T, bool nt)
{
    return march_pick_mid_rule<RULE_CA>(r, T, nt);
}

} // namespace fractal
