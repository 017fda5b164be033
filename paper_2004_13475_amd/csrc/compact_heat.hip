// compact_heat.hip -- compact-storage march kernels of the heat rule.
#include "compact_march.hpp"

namespace fractal {

CompactFn pick_compact_heat(int r, int T, bool nt)
{
    return nt ? compact_pick_rt<RULE_HEAT, TILE_NT_STORE>(r, T)
              : compact_pick_rt<RULE_HEAT, 0>(r, T);
}

} // namespace fractal
