// step_march_ca.hip -- the register-march step kernels of the automaton.
#include "march_pick.hpp"

namespace fractal {

MarchFn pick_march_ca(int map, int r, int T, bool nt, bool alt)
{
    return march_pick_rule<RULE_CA>(map, r, T, nt, alt);
}

} // namespace fractal
