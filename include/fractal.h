/*
 * fractal.h -- C ABI of libfractal: the block-space map lambda(omega) on an
 * embedded Sierpinski gasket (arXiv 2004.13475, Sections 3-6) and the
 * neighbourhood kernels it drives, for AMD Instinct MI355X (gfx950).
 *
 * Geometry.  A level-k gasket lives in an n x n embedding, n = 2^k.  Cell
 * (x, y) -- x the column, y the row -- is a member iff (x & y) == 0; there are
 * 3^k members (Eq. 2).  This is the vertical mirror of the paper's
 * orientation (its intra-block test in Section 6.1 reads x & (b-1-y) == 0);
 * every lambda value below is given for the (x & y) == 0 orientation.
 * Work is cut into rho x rho tiles (blocks in the paper), rho = 2^r; the
 * block space has side n_b = 2^(k-r) and level r_b = k - r, and exactly
 * 3^r_b tiles hold members.
 *
 * Buffers.  Every state buffer is a caller-owned, row-major n x n array in
 * device memory: cell (x, y) sits at element (size_t)y * n + x.  Cells are
 * uint8 in {0, 1} for the automaton (rule FRACTAL_RULE_CA) and float32 for
 * heat (FRACTAL_RULE_HEAT).  The two buffers of a step call must not overlap,
 * and BOTH must hold 0 in every off-gasket cell on entry: the lambda kernels
 * never visit empty tiles, and every kernel writes only the 16-byte chunks
 * that contain a member, or with FRACTAL_FLAG_SEGMENTS the 16-byte chunks of
 * 64-byte row segments that contain a member (off-gasket cells inside them
 * are written as 0).
 * After `steps` steps the state is in buf[steps & 1] (buf0 when steps is even);
 * steps == 0 does nothing.
 *
 * Asynchrony and errors.  `stream` is a hipStream_t (NULL = the null stream).
 * Calls enqueue work on it and return without waiting.  Every call returns a
 * status; arguments are checked on the host before anything is enqueued, and
 * a call that fails validation has no side effect.  fractal_last_error()
 * returns a message for the calling thread's last failure.  Device buffers
 * are never allocated on the step paths.
 */
#ifndef FRACTAL_H
#define FRACTAL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define FRACTAL_OK 0
#define FRACTAL_E_INVAL 1  /* bad argument; nothing was enqueued */
#define FRACTAL_E_NOMEM 2  /* a request larger than the serving arena */
#define FRACTAL_E_DEVICE 3 /* a HIP runtime call or kernel launch failed */
#define FRACTAL_E_AGAIN 4  /* result not ready yet (serving poll) */

/* neighbourhood rules */
#define FRACTAL_RULE_CA 0   /* uint8 B3/S23 automaton, Moore neighbourhood,
                               only gasket members counted (Section 6.2,
                               test CA) */
#define FRACTAL_RULE_HEAT 1 /* float32 explicit 5-point heat step,
                               u' = (1-4a)u + a(uN+uS+uE+uW) on members,
                               off-gasket neighbours count as 0 */

/* workgroup dispatch orders (a bijection from hardware workgroup id to the
 * tile it handles; results do not depend on it) */
#define FRACTAL_ORDER_NATURAL 0 /* omega = (blockIdx.x, blockIdx.y)         */
#define FRACTAL_ORDER_CURVE 1   /* lambda: omega taken along the gasket's
                                   self-similar order (base-3 digits of the
                                   linear id are the beta_mu); BB: row-major */
#define FRACTAL_ORDER_CURVE_XCD 2 /* as CURVE, with contiguous id ranges per
                                     accelerator die (XCD) so neighbouring
                                     tiles share an L2 */

#define FRACTAL_R_AUTO (-1) /* use the tuned (or default) tile size */

/* flags of a step launch (bitwise or) */
#define FRACTAL_FLAG_SEGMENTS 1 /* move whole 64-byte row segments that hold a
                                   member (their member-free chunks are read
                                   and written as 0) instead of 16-byte chunks */
#define FRACTAL_FLAG_NT_STORE 2 /* non-temporal hint on output stores */
#define FRACTAL_FLAG_FUSE2 8    /* two steps per launch: T = 2 halo rows and
                                   one extra 16-byte chunk column per side are
                                   staged and the intermediate step stays in
                                   LDS, halving state traffic per step.  Needs
                                   FRACTAL_FLAG_SEGMENTS and tile rows of >= 16
                                   bytes.  Launches come in pairs; the last
                                   steps - 2T*floor(steps/2T) steps run one per
                                   launch */
#define FRACTAL_FLAG_FUSE4 16   /* as FUSE2 with four steps per launch */
#define FRACTAL_FLAG_MARCH 32   /* register-march engine (lambda and BB maps):
                                   a wavefront takes several tiles side by
                                   side, one 16-byte chunk column per lane
                                   plus halo lanes, and walks down the tile
                                   rows computing T = 1, 2, 4, 8 or 16 steps
                                   (FUSE2 / 4 / 8 / 16) in registers, with
                                   no LDS.  Needs FRACTAL_FLAG_SEGMENTS and
                                   tile rows of >= 16 bytes.  Steps are
                                   split into launches of T steps, then
                                   smaller powers of two, with a launch count
                                   of the parity of steps */
#define FRACTAL_FLAG_FUSE8 64   /* eight steps per launch (with
                                   FRACTAL_FLAG_MARCH only) */
#define FRACTAL_FLAG_FUSE16 128 /* sixteen steps per launch (with
                                   FRACTAL_FLAG_MARCH; heat on tiles of
                                   side >= 16 only) */
#define FRACTAL_FLAG_PERSISTENT 4 /* batch only: register-march launches run
                                     a persistent grid (as many workgroups as
                                     the chip holds) striding through each
                                     die's share of the tile list, instead of
                                     one workgroup per group of tiles */
#define FRACTAL_FLAG_STACK2 256  /* lambda-map march launches of one gasket:
                                    walk vertical stacks of up to 2 tiles
                                    (the tiles of a column split into runs;
                                    each class of equal runs is a smaller
                                    gasket of stacks mapped by lambda, so the
                                    2T halo rows are paid once per stack;
                                    the classes are interleaved block by
                                    block).  Tiles are then taken in curve
                                    order.  The
                                    BB map, batches and compact states ignore
                                    it.  Needs FRACTAL_FLAG_MARCH; STACK2 / 4
                                    / 8 are exclusive */
#define FRACTAL_FLAG_STACK4 512  /* as STACK2, stacks of up to 4 tiles */
#define FRACTAL_FLAG_STACK8 1024 /* as STACK2, stacks of up to 8 tiles */
#define FRACTAL_FLAG_OCC_ALT 2048 /* lambda-map march launches of 8 or 16
                                     steps on tiles of side 16..64: the kernel
                                     compiled for the other occupancy (heat and
                                     the automaton's 8 steps: 2 wavefronts per
                                     SIMD instead of 3, so more registers per
                                     lane; the automaton's 16 steps: 3 instead
                                     of 2).  Launches of fewer steps, other
                                     tile sizes, the BB map, batches and
                                     compact states ignore it.  Needs
                                     FRACTAL_FLAG_MARCH */
#define FRACTAL_FLAG_FUSE24 8192 /* 24 steps per launch (with
                                    FRACTAL_FLAG_BLOCK only: the halo grows
                                    to 24 cells) */
#define FRACTAL_FLAG_FUSE32 16384 /* as FUSE24, 32 steps per launch */
#define FRACTAL_FLAG_FUSE36 32768 /* as FUSE24, 36 steps per launch */
#define FRACTAL_FLAG_BLOCK 4096 /* 64 x 64 tiles (r = 6) or 128 x 128
                                   tiles (r = 7, two blocks per lane), lambda
                                   or BB map: the block engine -- one
                                   wavefront per tile, one lane per non-empty
                                   8 x 8 block of the tile and of the part of
                                   its halo (16 to 36 cells deep) that can
                                   reach it within a launch (float32 cells in
                                   registers; automaton cells as a 64-bit
                                   board), neighbours exchanged between
                                   lanes; each launch advances up to the
                                   FUSE flag's step count (at most 16, or 24,
                                   32, 36 with FUSE24 / 32 / 36), the steps of
                                   a call shared out evenly over its
                                   launches.  Exclusive with
                                   FRACTAL_FLAG_MARCH, STACK and OCC_ALT.
                                   Batches run instances of levels >= 6 on it
                                   too, with 16 or 32 steps per launch
                                   (smaller levels on the march); compact
                                   states take the march engine */

typedef struct fractal_tuning {
    int r;       /* log2 of the tile side rho, 0..7 (rho <= 128)           */
    int threads; /* threads per workgroup: 64 or 256                        */
    int order;   /* FRACTAL_ORDER_*                                         */
    int flags;   /* FRACTAL_FLAG_*                                          */
} fractal_tuning; /* launch parameters of a step kernel */

/* Lemma 2 / Theorem 1: dimensions of the compact launch grid for a level-k
 * gasket cut into 2^r tiles: gx = 3^ceil(r_b/2), gy = 3^floor(r_b/2),
 * r_b = k - r.  Host only.  0 <= r <= k <= 40.  Returns FRACTAL_E_INVAL on a
 * bad level or a NULL output pointer. */
int fractal_grid_dims(int k, int r, uint32_t *gx, uint32_t *gy);

/* Theorem 1 and Section 6.1: evaluate lambda(omega) for every omega of the
 * compact grid and write d_xy[2*(wy*gx + wx) + 0] = lambda_x,
 * d_xy[... + 1] = lambda_y (block coordinates, (x & y) == 0 orientation).
 * d_xy: device array of 2*gx*gy uint32, caller-owned.  0 <= r <= k,
 * k - r <= 30.  One workgroup per omega; each wavefront computes the base-3
 * digits beta_mu in its lanes and assembles lambda with two ballots. */
int fractal_lambda_map(int k, int r, uint32_t *d_xy, void *stream);

/* Section 6.3, Variant 1: the same map with the sum of offsets done by one
 * matrix-core product per workgroup (row 0 of A holds 2^0..2^(r_b-1) in
 * float16, columns 0 and 1 of B hold tau_x and tau_y; D[0][0..1] is lambda
 * before mirroring).  Exact for k - r <= 16; larger levels give E_INVAL. */
int fractal_lambda_map_mfma(int k, int r, uint32_t *d_xy, void *stream);

/* lambda as the register-march step kernels evaluate it, one tile per lane
 * (their wavefronts hold several tiles side by side, so every lane group
 * computes its own tile's block with a loop over its id's base-3 digits
 * rather than sharing one ballot): for every tile id i in [0, 3^(k-r)),
 * d_xy[2*i + 0] = block x, d_xy[2*i + 1] = block y of the tile that id i
 * stands for in dispatch order `order`.  FRACTAL_ORDER_NATURAL: omega =
 * (i mod gx, i div gx), so the result equals fractal_lambda_map's; the
 * CURVE orders: base-3 digit mu-1 of i is beta_mu (Theorem 1's map taken
 * along the gasket's self-similar order, as compact storage numbers its
 * tiles).  d_xy: device array of 2 * 3^(k-r) uint32, caller-owned.
 * 0 <= r <= k, k - r <= 20. */
int fractal_lambda_map_tiles(int k, int r, int order, uint32_t *d_xy, void *stream);

/* Seeded initial state: writes all n*n cells of d_buf.  Members get
 * SplitMix64 output number i+1 (state 0), i = stream_id * 2^32 + y*n + x:
 * the automaton takes its top bit, heat takes (z >> 40) * 2^-24; other
 * cells get 0.  0 <= k <= 16. */
int fractal_seed_fill(int k, int rule, uint32_t stream_id, void *d_buf,
                      void *stream);

/* Launches of the step entry points below without an explicit tuning use,
 * for an explicit r, the die-aware curve order for lambda and launch order
 * for the bounding box, whole segments, and where tile rows span >= 16 bytes
 * the register-march engine with eight steps per launch (non-temporal
 * stores from level 15), else the LDS engine one step per launch (64 or 256
 * threads); for FRACTAL_R_AUTO, the cached autotuned launch or a built-in
 * default.  The matrix-core map always uses the LDS engine. */

/* Bounding-box step (Section 1; Section 6.2): a grid of all (n/rho)^2
 * workgroups with the identity map omega -> tile; a workgroup whose tile
 * holds no member exits at once.  Runs `steps` synchronous steps of `rule`
 * ping-ponging between d_buf0 (input of step 0) and d_buf1.
 * 0 <= k <= 16, 0 <= r <= min(k, 7) with k - r <= 15, or FRACTAL_R_AUTO;
 * alpha ignored for the
 * automaton and 0 < alpha <= 0.25 for heat, steps >= 0. */
int fractal_bb_step(int k, int r, int rule, float alpha, void *d_buf0,
                    void *d_buf1, int steps, void *stream);

/* lambda step (Theorem 1, Sections 5 and 6.1): a compact grid of exactly
 * 3^(k-r) workgroups, each mapped by lambda(omega) to a non-empty tile; the
 * tile and a 1-cell halo are staged in LDS and the rule is applied to the
 * members (bounding sub-box intra-block mapping).  Arguments as for
 * fractal_bb_step.  Result is bit-identical to fractal_bb_step. */
int fractal_lambda_step(int k, int r, int rule, float alpha, void *d_buf0,
                        void *d_buf1, int steps, void *stream);

/* fractal_lambda_step with lambda computed by the matrix-core product of
 * fractal_lambda_map_mfma.  Same arguments and results; k - r <= 16. */
int fractal_lambda_step_mfma(int k, int r, int rule, float alpha,
                             void *d_buf0, void *d_buf1, int steps,
                             void *stream);

/* lambda step (map 0) or bounding-box step (map 1) or matrix-core lambda
 * step (map 2) with explicit launch parameters.  Same buffer contract. */
int fractal_step_tuned(int map, int k, int rule, float alpha, void *d_buf0,
                       void *d_buf1, int steps, const fractal_tuning *tuning,
                       void *stream);

/* Autotuner: times every supported (r, threads, order, flags) for this level
 * and rule on the given buffers (a few steps each, synchronising `stream`):
 * tile sizes, both engines, dispatch orders, workgroup sizes, steps per
 * launch, stacks, non-temporal stores and, for the long march launches, the
 * occupancy the kernel is compiled for (FRACTAL_FLAG_OCC_ALT) -- and
 * records the fastest lambda launch in a per-process cache keyed by
 * (device, k, rule).  The buffers must satisfy the step contract; they end up
 * holding a state advanced by some number of steps.  `out` may be NULL. */
int fractal_autotune(int k, int rule, float alpha, void *d_buf0, void *d_buf1,
                     void *stream, fractal_tuning *out);

/* Tuning used for FRACTAL_R_AUTO: the cached autotuned entry for
 * (current device, k, rule) if one exists, else a built-in default. */
int fractal_get_tuning(int k, int rule, fractal_tuning *out);

/* Replace the cached entry for (current device, k, rule). */
int fractal_set_tuning(int k, int rule, const fractal_tuning *tuning);

/* Tuning file: one text line per cached entry, "device<TAB>k<TAB>rule<TAB>r
 * <TAB>threads<TAB>order<TAB>flags", where device is the device's product
 * and architecture name (so a file tuned on one MI355X serves every MI355X);
 * lines starting with '#' are comments.  fractal_tuning_save writes every
 * cached entry (replacing the file through a temporary one; E_DEVICE on an
 * I/O error).  fractal_tuning_load adds the entries named for the current
 * device to the cache, replacing entries of the same (k, rule); other
 * devices' lines are skipped; E_DEVICE if the file cannot be read, E_INVAL
 * on a malformed line or an invalid tuning (then nothing is added).  If the
 * environment variable FRACTAL_TUNING_FILE names a file, it is loaded before
 * the first lookup of the process (a missing or malformed file is then
 * ignored) and rewritten after every fractal_autotune. */
int fractal_tuning_save(const char *path);
int fractal_tuning_load(const char *path);

/* Test SW of Section 6.2 (single write): every member cell of the level-k
 * gasket in d_buf (n x n, row-major, uint8 for FRACTAL_RULE_CA, float32 for
 * FRACTAL_RULE_HEAT) is set to `value` (its low byte for uint8 cells, its
 * bit pattern for float32 cells), over tiles of side 2^r reached through
 * lambda (map 0) or the bounding box (map 1).  Cells off the gasket are
 * written 0 where they lie in a non-empty tile and in a 64-byte row segment
 * that holds a member, and are not touched elsewhere, so on a buffer that
 * starts at 0 (as in the paper) the result is value on the gasket and 0 off
 * it.  0 <= k <= 16,
 * 0 <= r <= min(k, 7), k - r <= 15.  d_buf must be 16-byte aligned. */
int fractal_single_write(int map, int k, int r, int rule, uint32_t value,
                         void *d_buf, void *stream);

/* Bytes of device workspace fractal_reduce needs for (k, r): one 8-byte
 * partial per tile plus the partials of the summation tree. */
int fractal_reduce_workspace(int k, int r, size_t *bytes);

/* Test RD of Section 6.2 (reduction): *d_out (8 bytes of device memory) =
 * the sum of the member cells of d_buf: a uint64 for uint8 cells, a float64
 * (the float32 values summed in float64) for float32 cells; cells off the
 * gasket are ignored.  Each tile's cells are summed in a fixed order into
 * slot lambda^-1(tile) of d_work, and the slots are summed by a fixed tree,
 * so the result does not depend on the map, the dispatch or the timing
 * (lambda and BB agree bit for bit).  d_work: caller-owned, at least
 * fractal_reduce_workspace(k, r) bytes, 8-byte aligned; its contents are
 * overwritten.  Same ranges as fractal_single_write; E_INVAL on a short
 * workspace. */
int fractal_reduce(int map, int k, int r, int rule, const void *d_buf,
                   void *d_work, size_t work_bytes, void *d_out, void *stream);

/* fractal_reduce for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and result, bit for bit, with the slots and tree partials
 * in a static scratch array of 16 MiB per device instead of a caller
 * workspace, so k - r <= 13 (larger block levels fail with E_INVAL and a
 * message naming fractal_reduce).  Nothing is allocated and nothing is
 * freed: the scratch is part of the loaded code object, one copy per device,
 * held until the process ends; its address is looked up once per device, on
 * the first call made with that device current.  Every call on a device
 * shares that device's scratch, and each call writes every slot it reads,
 * so nothing carries over from an earlier call; calls that overlap in time
 * on one device (different streams, or different host threads without
 * ordering) race on the scratch and give undefined results -- order them on
 * one stream.  d_out: 8 bytes of device memory, 8-byte aligned.  Other
 * arguments and errors as fractal_reduce. */
int fractal_reduce_noalloc(int map, int k, int r, int rule, const void *d_buf,
                           void *d_out, void *stream);

/* Compact storage through lambda^-1 (the compact manipulation that Section 7
 * names as future work): a state of level k with tiles of side rho = 2^r
 * keeps only its 3^(k-r) non-empty tiles.  Tile L (0 <= L < 3^(k-r)) is the
 * one whose block is lambda(L) in the curve order -- base-3 digit mu-1 of L
 * is beta_mu, block bit mu-1 of x is [beta == 2] and of y is [beta == 0] --
 * and its rho x rho box is stored row-major at cell offset L * rho^2; so
 * cell (x, y) of the gasket lives at
 *   (lambda^-1(x >> r, y >> r) * rho + (y & (rho-1))) * rho + (x & (rho-1)).
 * Box cells off the gasket hold 0.  Size 3^(k-r) * 4^r cells instead of 4^k,
 * which lets one GPU hold levels up to 20.  Tile rows must span >= 16 bytes
 * (r >= 4 for uint8 cells, r >= 2 for float32); 0 <= r <= 7, k - r <= 18. */

/* Bytes of one compact state; k <= 20. */
int fractal_compact_bytes(int k, int r, int rule, size_t *bytes);

/* Copy the tile boxes of an n x n state (k <= 16) into compact storage
 * (pack) or back (unpack; cells of empty tiles are not written).  Buffers
 * device, 16-byte aligned, non-overlapping. */
int fractal_pack(int k, int r, int rule, const void *d_embedded, void *d_compact,
                 void *stream);
int fractal_unpack(int k, int r, int rule, const void *d_compact, void *d_embedded,
                   void *stream);

/* Seeded initial state written directly in compact storage: every box cell
 * gets the value fractal_seed_fill gives the same (x, y) (the SplitMix64
 * counter y * n + x taken modulo 2^64 beyond level 16); k <= 20. */
int fractal_compact_seed_fill(int k, int r, int rule, uint32_t stream_id,
                              void *d_compact, void *stream);

/* `steps` steps of `rule` on a compact state, ping-ponging between d_c0 and
 * d_c1 (result in buf[steps & 1]).  States of 64 x 64 tiles (r = 6) take
 * the block engine (one wavefront per tile in curve order, the neighbouring
 * tiles found by lambda^-1); other tile sizes the register-march engine,
 * each lane finding the tiles around its own through lambda^-1.  Results
 * equal pack(fractal_lambda_step(unpack(state))) bit for bit.  flags: 0 for
 * the default (r = 6: the block engine, up to 36 steps per launch; else the
 * longest march launch the tile allows, up to 16 steps for the automaton
 * from level 15, else 8, non-temporal stores from level 15), or
 * FRACTAL_FLAG_FUSE2/4/8/16 and FRACTAL_FLAG_NT_STORE for the march (MARCH
 * and SEGMENTS are implied and accepted; steps per launch and halo must fit
 * in one tile, T <= rho), or FRACTAL_FLAG_BLOCK (r = 6) with a FUSE flag up
 * to FUSE36 and FRACTAL_FLAG_NT_STORE.  k <= 20; buffers of
 * fractal_compact_bytes each; cells off the gasket must be zero in both. */
int fractal_compact_step(int k, int r, int rule, float alpha, void *d_c0,
                         void *d_c1, int steps, int flags, void *stream);

/* General NBB fractals (Section 3, Table 1): a fractal of the family is
 * given by k replicas per level on an s x s grid, replica beta (0 <= beta <
 * k) at offset H[beta] = (tau_x[beta], tau_y[beta]), distinct cells of
 * [0, s)^2.  The level-R fractal lives in an n x n uint8 array, n = s^R,
 * row-major; cell (x, y) is a member iff every base-s digit pair (x_d, y_d)
 * is a replica offset; it has k^R members (Eq. 2).  Tiles have side s^r;
 * map 0 launches Theorem 1's compact grid of k^ceil(r_b/2) x k^floor(r_b/2)
 * workgroups (r_b = R - r), map 1 the bounding box of (n/s^r)^2.  Limits:
 * 2 <= s <= 8, k <= min(s^2, 32), n <= 65536 with n^2 <= 2^32, s^r <= 128.
 * The paper's Table 1 shows the replica grids only as figures; the built-in
 * tables are the usual definitions of those fractals. */
#define FRACTAL_NBB_MAX_K 32
typedef struct fractal_nbb {
    int k; /* replicas per level */
    int s; /* scale factor per level */
    uint8_t tau_x[FRACTAL_NBB_MAX_K];
    uint8_t tau_y[FRACTAL_NBB_MAX_K];
} fractal_nbb;
#define FRACTAL_NBB_GASKET 0  /* (3, 2), H = {(0,0), (0,1), (1,1)}: x & (n-1-y) == 0 */
#define FRACTAL_NBB_CARPET 1  /* (8, 3): all but the centre                        */
#define FRACTAL_NBB_VICSEK 2  /* (5, 3): centre and the four edge midpoints         */
#define FRACTAL_NBB_XFRACTAL 3 /* (5, 3): centre and the four corners               */
#define FRACTAL_NBB_HFRACTAL 4 /* (7, 3): left and right columns and the centre     */
#define FRACTAL_NBB_CANTOR 5  /* (2, 3): (0,0) and (2,0), a Cantor set on one row   */

/* A built-in table (host only); replicas numbered in row-major order of their
 * grid cells, except the gasket, which keeps the paper's numbering. */
int fractal_nbb_builtin(int which, fractal_nbb *out);

/* Theorem 1 for any NBB table: lambda(omega) for every omega of the
 * k^ceil(rb/2) x k^floor(rb/2) grid into d_xy[2*(wy*gx+wx) + {0,1}]; every
 * wavefront sums the levels' offsets tau * s^(mu-1) by a butterfly over its
 * lanes.  s^rb and k^rb <= 2^31. */
int fractal_nbb_lambda_map(const fractal_nbb *f, int rb, uint32_t *d_xy, void *stream);

/* Test SW on an NBB fractal: value (low byte) on every member of d_buf
 * (n x n uint8); other cells untouched. */
int fractal_nbb_single_write(const fractal_nbb *f, int map, int level, int r,
                             uint32_t value, void *d_buf, void *stream);

/* Test RD on an NBB fractal: *d_out (uint64, device) = sum of the member
 * cells; per-tile sums go to the tile's compact-grid slot (the inverse map
 * for BB) and a fixed tree adds them, so both maps agree bit for bit. */
int fractal_nbb_reduce_workspace(const fractal_nbb *f, int level, int r, size_t *bytes);
int fractal_nbb_reduce(const fractal_nbb *f, int map, int level, int r,
                       const void *d_buf, void *d_work, size_t work_bytes,
                       void *d_out, void *stream);

/* Test CA on an NBB fractal: `steps` synchronous B3/S23 steps counting
 * fractal Moore neighbours (cells off the fractal must hold 0 in both
 * buffers), ping-ponging d_buf0 -> d_buf1; result in buf[steps & 1]. */
int fractal_nbb_ca_step(const fractal_nbb *f, int map, int level, int r,
                        void *d_buf0, void *d_buf1, int steps, void *stream);

/* One gasket of a batch. */
typedef struct fractal_instance {
    int k;       /* level, 0..16                                  */
    int rule;    /* FRACTAL_RULE_*                                */
    int steps;   /* >= 0                                          */
    float alpha; /* heat only                                     */
    void *d_buf0; /* state at step 0; result in buf[steps & 1]    */
    void *d_buf1;
} fractal_instance;

/* Bytes of device workspace fractal_batch_step needs for `count` instances
 * (0 <= count <= 65536): the per-instance offset table. */
int fractal_batch_workspace(int count, size_t *bytes);

/* Advance many gaskets of uneven levels together.  Instances are grouped
 * by their tile launch; each group's tiles form one work list: a tile id is
 * turned into (instance, local id) with a device table of per-instance
 * prefix offsets of 3^(k_i - r_i), then into a tile by that instance's
 * lambda.  Each launch is one kernel per group over its whole list; all
 * max_i steps_i launches are captured once into a HIP graph and the graph
 * is launched on `stream`.  Instances with fewer steps drop out of later
 * launches.  `tuning` may be NULL (per-level defaults or cached tuning);
 * otherwise tuning->r applies to every instance (clamped per level) or
 * FRACTAL_R_AUTO keeps the per-level tile size, tuning->threads 0 keeps the
 * default thread count, and tuning->flags, where any flag besides
 * FRACTAL_FLAG_PERSISTENT is set, applies to every instance (FUSE flags fall
 * back to what narrow tiles allow; the block engine takes 16 or 32 steps per
 * launch here, FUSE24 / 36 becoming FUSE32; STACK flags are ignored).  With
 * FRACTAL_FLAG_PERSISTENT the register-march launches run a persistent grid
 * (as many workgroups as the chip holds at once, the workgroups of each die
 * striding through that die's contiguous share of the list); LDS-engine
 * launches always take one workgroup per tile.
 * d_work: caller-owned device workspace of at least
 * fractal_batch_workspace(count) bytes, 16-byte aligned; the table is
 * copied into it on `stream`, so it must stay allocated and unused by
 * other work until the batch's work on `stream` has completed.  The library
 * allocates no device memory (a pinned host staging copy of the table is
 * kept until the graph has run).  Results are bit-identical to one
 * fractal_lambda_step call per instance.  Instance buffers must not overlap
 * one another.  E_INVAL on a short workspace. */
int fractal_batch_step(const fractal_instance *inst, int count,
                       const fractal_tuning *tuning, void *d_work,
                       size_t work_bytes, void *stream);

/* ---------------------------------------------------------------- serving
 * A request server keeps gasket simulations resident in a caller-provided
 * device arena and advances all admitted ones together (continuous batching
 * at step granularity): each iteration is a group of batched launches over
 * every active slot; requests that arrive meanwhile are admitted, first come
 * first served, as soon as both a slot and arena space are free. */
typedef struct fractal_request {
    int k, rule, steps;
    float alpha;
    uint32_t seed;      /* stream id of the seeded state when h_init == NULL */
    const void *h_init; /* n*n host cells, or NULL for the seeded state; must
                           stay valid until poll returns FRACTAL_OK          */
    void *h_out;        /* n*n host cells receiving the final state, or NULL
                           (then only the checksum is produced)              */
    double t_arrival;   /* caller's arrival stamp (seconds, any origin used
                           consistently with fractal_now); < 0 = now         */
} fractal_request;

typedef struct fractal_result {
    int status;       /* FRACTAL_OK, or the error of this request          */
    int reserved;
    double t_arrival; /* stamps in seconds on the fractal_now() clock      */
    double t_admit;
    double t_done;
    uint64_t checksum; /* sum over cells of the final state's bit patterns
                          (uint8 value or float32 bits), modulo 2^64       */
} fractal_result;

/* Monotonic clock (seconds) used for every serving stamp. */
double fractal_now(void);

/* Create a server over d_arena (arena_bytes of device memory owned by the
 * caller, 256-byte aligned; a small header of it holds the server's device
 * tables, the rest request states) with at most max_slots concurrently
 * admitted requests (1..4096), working on `stream`.  Each admitted request
 * advances 32 steps per scheduling iteration until
 * fractal_serve_set_steps_per_iter changes it.  Host threads are started;
 * the library allocates no device memory.  E_NOMEM if the arena cannot hold
 * the header. */
int fractal_serve_create(void *d_arena, size_t arena_bytes, int max_slots,
                         void *stream, void **server);

/* Steps each admitted request advances per scheduling iteration (1..2^20),
 * from the next iteration on.  They are fused into launches of up to 32
 * steps (block engine, levels from 13 / 14) or 16 (march), so multiples of
 * 32 let every launch take its longest form; smaller values admit arriving
 * requests sooner. */
int fractal_serve_set_steps_per_iter(void *server, int steps_per_iter);

/* Queue a request; never waits for the GPU.  A request whose footprint
 * (2 * 4^k cells, plus alignment) exceeds the arena fails with
 * FRACTAL_E_NOMEM, a malformed one with FRACTAL_E_INVAL. */
int fractal_serve_submit(void *server, const fractal_request *rq,
                         uint64_t *ticket);

/* FRACTAL_OK and *res filled once the ticket is done (then the ticket is
 * forgotten), FRACTAL_E_AGAIN while it is pending, FRACTAL_E_INVAL for an
 * unknown ticket. */
int fractal_serve_poll(void *server, uint64_t ticket, fractal_result *res);

/* Latency and throughput of a server's requests so far.  Latency is
 * t_done - t_arrival of each request that completed with FRACTAL_OK;
 * percentiles are nearest-rank over those requests. */
typedef struct fractal_serve_report {
    uint64_t submitted;  /* requests accepted by fractal_serve_submit       */
    uint64_t completed;  /* finished with FRACTAL_OK                         */
    uint64_t failed;     /* finished with an error status                    */
    uint64_t pending;    /* queued, active or retiring                       */
    uint64_t iterations; /* scheduling iterations run                        */
    double p50_latency;  /* seconds                                          */
    double p99_latency;
    double mean_latency;
    double cell_updates; /* sum over completed requests of 3^k * steps       */
    double t_first_arrival; /* earliest arrival stamp of a completed request */
    double t_last_done;     /* latest completion stamp                        */
} fractal_serve_report;

int fractal_serve_stats(void *server, fractal_serve_report *out);

/* Stop the server thread after the queued work has drained and free its
 * host state.  Outstanding tickets are completed first. */
int fractal_serve_destroy(void *server);

/* Message of the calling thread's last failed call ("" if none). */
const char *fractal_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FRACTAL_H */
