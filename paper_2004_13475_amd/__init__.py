"""Block-space map lambda(omega) on embedded Sierpinski gaskets for MI355X.

Python face of libfractal.so (hand-written HIP for gfx950).  See
include/fractal.h for the C ABI; every function here forwards to it.
"""
from ._lib import (  # noqa: F401
    E_AGAIN, E_DEVICE, FLAG_FUSE2, FLAG_FUSE4, FLAG_FUSE8, FLAG_FUSE16, FLAG_FUSE24, FLAG_FUSE32, FLAG_FUSE36, FLAG_MARCH, FLAG_STACK2, FLAG_STACK4, FLAG_STACK8, FLAG_OCC_ALT, FLAG_BLOCK, FLAG_NT_STORE, FLAG_PERSISTENT, FLAG_SEGMENTS, E_INVAL, E_NOMEM, EXPORTED, LIB_PATH, MAP_BB, MAP_LAMBDA,
    MAP_MFMA, OK, ORDER_CURVE, ORDER_CURVE_XCD, ORDER_NATURAL, R_AUTO, RULE_CA,
    RULE_HEAT, FractalError, Server, autotune, batch_step, batch_workspace, bb_step, compact_bytes,
    compact_seed_fill, compact_step, pack, unpack, Nbb, NBB_GASKET, NBB_CARPET, NBB_VICSEK,
    NBB_XFRACTAL, NBB_HFRACTAL, NBB_CANTOR, nbb_builtin, nbb_make, nbb_lambda_map,
    nbb_single_write, nbb_reduce_workspace, nbb_reduce, nbb_ca_step,
    exported_symbols, get_tuning, grid_dims, lambda_map, lambda_map_mfma,
    lambda_map_tiles, lambda_step, lambda_step_mfma, load, now, reduce, reduce_noalloc, reduce_workspace,
    seed_fill, set_tuning,
    single_write, step_tuned, tuning_load, tuning_save)
