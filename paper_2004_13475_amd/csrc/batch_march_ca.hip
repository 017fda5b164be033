// batch_march_ca.hip -- batch march kernels of the automaton.
#include "batch_march.hpp"

namespace fractal {

BatchMarchFn pick_batch_march_ca(int r, int T, bool nt)
{
    return bm_pick_rule<RULE_CA>(r, T, nt);
}

} // namespace fractal
