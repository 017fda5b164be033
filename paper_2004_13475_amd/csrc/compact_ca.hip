// compact_ca.hip -- compact-storage march kernels of the automaton.
#include "compact_march.hpp"

namespace fractal {

CompactFn pick_compact_ca(int r, int T, bool nt)
{
    return nt ? compact_pick_rt<RULE_CA, TILE_NT_STORE>(r, T) : compact_pick_rt<RULE_CA, 0>(r, T);
}

} // namespace fractal
