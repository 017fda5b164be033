/*
 * fractal_oracle.c -- plain CPU oracle for the block-space map lambda(omega)
 * on the embedded Sierpinski gasket and for the neighbourhood steps it drives.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this code.  It shares no source, header,
 * table or helper with the GPU library, and the product path never calls it.
 *
 * Everything here is the slow, literal definition:
 *   - gasket membership and cell counts by brute-force scans;
 *   - lambda(omega) by the paper's construction (helper beta, replica table H,
 *     offsets Delta, sum over scale levels), one level at a time;
 *   - the automaton and heat steps cell by cell, every neighbour tested for
 *     bounds and membership, double-buffered (synchronous update);
 *   - heat in float64.
 *
 * Conventions (readings of the paper, each also listed in the design notes):
 *   - Cell (x, y) of the n x n embedding (n = 2^k) is x = column, y = row of a
 *     row-major array, and is a gasket member iff (x & y) == 0.  The paper's
 *     intra-block test (Section 6.1) is x & (b-1-y) == 0, the vertical mirror;
 *     lambda is therefore computed in the paper's orientation and mirrored
 *     (y -> n_b - 1 - y) at the end.
 *   - beta_mu takes omega_x for odd mu and omega_y for even mu, as the formula
 *     for beta in Theorem 1 selects (its prose says the opposite; only the
 *     formula gives a bijection onto Lemma 2's grid), mu runs 1..r_b, and the
 *     division inside beta is integer floor division.
 *   - Replica offsets use s^(mu-1) = 2^(mu-1) (Eq. deltas, Section 6.1).
 *   - The array edge is not periodic: cells outside [0, n)^2 do not exist.
 *   - Automaton rule B3/S23 over the 8-cell Moore neighbourhood, counting only
 *     neighbours that are gasket members (Section 6.2, test CA).
 *   - Heat: u' = (1 - 4 alpha) u + alpha (u_N + u_S + u_E + u_W) on members,
 *     neighbours off the gasket or outside the array contribute 0, and
 *     non-members stay 0.
 *
 * Windows: the steppers run on a window [x0, x0+w) x [y0, y0+h) of the
 * embedding.  Cells outside the window are treated as 0; after T steps the
 * cells farther than T from every window edge that is not also an array edge
 * are exact.  A window equal to the whole array gives the exact full result.
 *
 * Parity pins (tests): member count = 3^k (Eq. 2), lambda image = brute-force
 * set of non-empty blocks (bijection) in both orientations, hand-derived
 * lambda values for r_b <= 3, automaton = textbook Game of Life on the
 * zero-padded array followed by masking, heat uniform-field and total-heat
 * closed forms, linearity and a hand-computed level-1 case.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_RULE_CA 0
#define OR_RULE_HEAT 1

/* Domain predicate: (x & y) == 0 (mirror of the Section 6.1 test). */
int oracle_member(int64_t x, int64_t y, int k)
{
    int64_t n = (int64_t)1 << k;
    if (x < 0 || y < 0 || x >= n || y >= n)
        return 0;
    return (x & y) == 0;
}

/* Brute-force cell count of the level-k gasket (compare with Eq. 2: 3^k). */
uint64_t oracle_count_members(int k)
{
    int64_t n = (int64_t)1 << k;
    uint64_t total = 0;
#pragma omp parallel for reduction(+ : total) schedule(static)
    for (int64_t y = 0; y < n; ++y)
        for (int64_t x = 0; x < n; ++x)
            total += (uint64_t)oracle_member(x, y, k);
    return total;
}

static uint64_t ipow(uint64_t b, int e)
{
    uint64_t p = 1;
    for (int i = 0; i < e; ++i)
        p *= b;
    return p;
}

/* Lemma 2 (packing) with 3 replicas: the compact grid is
 * 3^ceil(r_b/2) columns by 3^floor(r_b/2) rows. */
void oracle_grid_dims(int rb, uint64_t *gx, uint64_t *gy)
{
    *gx = ipow(3, (rb + 1) / 2);
    *gy = ipow(3, rb / 2);
}

/* Replica table H of Section 6.1: H[0] = (0,0), H[1] = (0,1), H[2] = (1,1). */
static const int H_TAU_X[3] = {0, 0, 1};
static const int H_TAU_Y[3] = {0, 1, 1};

/* lambda(omega) in the paper's orientation (Theorem 1 construction,
 * Section 6.1 for the gasket).  For each scale level mu = 1..r_b:
 *   beta_mu  = floor(v / 3^(ceil(mu/2) - 1)) mod 3, v = omega_x (mu odd) or
 *              omega_y (mu even)                      (helper beta)
 *   tau^mu   = H[beta_mu]                              (replica offsets)
 *   Delta^mu = (tau_x 2^(mu-1), tau_y 2^(mu-1))        (Eq. deltas)
 *   lambda  += Delta^mu                                (Eqs. lambda-x, lambda-y)
 */
void oracle_lambda_paper(int rb, uint64_t wx, uint64_t wy, uint64_t *lx,
                         uint64_t *ly)
{
    uint64_t sx = 0, sy = 0;
    for (int mu = 1; mu <= rb; ++mu) {
        uint64_t v = (mu % 2 == 1) ? wx : wy;
        int ce = (mu + 1) / 2; /* ceil(mu / 2) */
        uint64_t beta = (v / ipow(3, ce - 1)) % 3;
        uint64_t dx = (uint64_t)H_TAU_X[beta] << (mu - 1);
        uint64_t dy = (uint64_t)H_TAU_Y[beta] << (mu - 1);
        sx += dx;
        sy += dy;
    }
    *lx = sx;
    *ly = sy;
}

/* lambda(omega) for the (x & y) == 0 embedding: the paper's value mirrored
 * vertically inside the n_b x n_b block space (n_b = 2^r_b). */
void oracle_lambda(int rb, uint64_t wx, uint64_t wy, uint64_t *lx, uint64_t *ly)
{
    uint64_t px, py;
    oracle_lambda_paper(rb, wx, wy, &px, &py);
    uint64_t nb = (uint64_t)1 << rb;
    *lx = px;
    *ly = nb - 1 - py;
}

/* lambda over the whole compact grid, row-major in omega:
 * xy[2*(wy*gx + wx) + 0] = lambda_x, [.. + 1] = lambda_y.
 * paper_orient != 0 selects the paper's orientation. */
void oracle_lambda_grid(int rb, int paper_orient, uint32_t *xy)
{
    uint64_t gx, gy;
    oracle_grid_dims(rb, &gx, &gy);
#pragma omp parallel for schedule(static)
    for (int64_t wy = 0; wy < (int64_t)gy; ++wy)
        for (uint64_t wx = 0; wx < gx; ++wx) {
            uint64_t lx, ly;
            if (paper_orient)
                oracle_lambda_paper(rb, wx, (uint64_t)wy, &lx, &ly);
            else
                oracle_lambda(rb, wx, (uint64_t)wy, &lx, &ly);
            uint64_t i = (uint64_t)wy * gx + wx;
            xy[2 * i + 0] = (uint32_t)lx;
            xy[2 * i + 1] = (uint32_t)ly;
        }
}

/* Bounding-box approach (Section 1; Section 6.2): identity map over the
 * n_b x n_b block grid, a block doing work only if it holds a member.
 * mask[Y * n_b + X] = 1 iff the rho x rho block (X, Y) holds a member cell,
 * found by scanning every cell of the block. */
void oracle_nonempty_blocks(int k, int r, uint8_t *mask)
{
    int64_t rho = (int64_t)1 << r;
    int64_t nb = (int64_t)1 << (k - r);
#pragma omp parallel for schedule(static)
    for (int64_t Y = 0; Y < nb; ++Y)
        for (int64_t X = 0; X < nb; ++X) {
            int any = 0;
            for (int64_t j = 0; j < rho && !any; ++j)
                for (int64_t i = 0; i < rho && !any; ++i)
                    any = oracle_member(X * rho + i, Y * rho + j, k);
            mask[Y * nb + X] = (uint8_t)any;
        }
}

/* Value of window cell (x, y) in global coordinates; 0 outside the window. */
static inline int win_inside(int64_t x, int64_t y, int64_t x0, int64_t y0,
                             int64_t w, int64_t h)
{
    return x >= x0 && y >= y0 && x < x0 + w && y < y0 + h;
}

/* One automaton step (Section 6.2, test CA; rule B3/S23): a member cell
 * counts the members among its 8 Moore neighbours that are alive; it is alive
 * next step iff the count is 3, or it is alive and the count is 2.  Cells
 * that are not members stay 0. */
static void ca_step(int k, int64_t x0, int64_t y0, int64_t w, int64_t h,
                    const uint8_t *in, uint8_t *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < h; ++j)
        for (int64_t i = 0; i < w; ++i) {
            int64_t x = x0 + i, y = y0 + j;
            uint8_t next = 0;
            if (oracle_member(x, y, k)) {
                int count = 0;
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        if (dx == 0 && dy == 0)
                            continue;
                        int64_t xn = x + dx, yn = y + dy;
                        if (!win_inside(xn, yn, x0, y0, w, h))
                            continue;
                        if (!oracle_member(xn, yn, k))
                            continue;
                        if (in[(yn - y0) * w + (xn - x0)] == 1)
                            count += 1;
                    }
                int alive = in[j * w + i] == 1;
                if (count == 3 || (alive && count == 2))
                    next = 1;
            }
            out[j * w + i] = next;
        }
}

/* One heat step in float64 (5-point explicit finite difference,
 * Dirichlet 0 off the gasket):
 *   u'(c) = (1 - 4 alpha) u(c) + alpha (u_N + u_S + u_E + u_W). */
static void heat_step(int k, int64_t x0, int64_t y0, int64_t w, int64_t h,
                      const double *in, double alpha, double *out)
{
    static const int NB[4][2] = {{0, -1}, {0, 1}, {1, 0}, {-1, 0}};
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < h; ++j)
        for (int64_t i = 0; i < w; ++i) {
            int64_t x = x0 + i, y = y0 + j;
            double next = 0.0;
            if (oracle_member(x, y, k)) {
                double s = 0.0;
                for (int q = 0; q < 4; ++q) {
                    int64_t xn = x + NB[q][0], yn = y + NB[q][1];
                    if (!win_inside(xn, yn, x0, y0, w, h))
                        continue;
                    if (!oracle_member(xn, yn, k))
                        continue;
                    s += in[(yn - y0) * w + (xn - x0)];
                }
                next = (1.0 - 4.0 * alpha) * in[j * w + i] + alpha * s;
            }
            out[j * w + i] = next;
        }
}

/* T automaton steps on a window.  Returns 0, or -1 if memory ran out. */
int oracle_ca_run(int k, int64_t x0, int64_t y0, int64_t w, int64_t h,
                  const uint8_t *in, int T, uint8_t *out)
{
    size_t cells = (size_t)w * (size_t)h;
    uint8_t *a = (uint8_t *)malloc(cells), *b = (uint8_t *)malloc(cells);
    if (!a || !b) {
        free(a);
        free(b);
        return -1;
    }
    memcpy(a, in, cells);
    for (int t = 0; t < T; ++t) {
        ca_step(k, x0, y0, w, h, a, b);
        uint8_t *tmp = a;
        a = b;
        b = tmp;
    }
    memcpy(out, a, cells);
    free(a);
    free(b);
    return 0;
}

/* T heat steps on a window in float64.  Returns 0, or -1 on no memory. */
int oracle_heat_run(int k, int64_t x0, int64_t y0, int64_t w, int64_t h,
                    const double *in, double alpha, int T, double *out)
{
    size_t cells = (size_t)w * (size_t)h;
    double *a = (double *)malloc(cells * sizeof(double));
    double *b = (double *)malloc(cells * sizeof(double));
    if (!a || !b) {
        free(a);
        free(b);
        return -1;
    }
    memcpy(a, in, cells * sizeof(double));
    for (int t = 0; t < T; ++t) {
        heat_step(k, x0, y0, w, h, a, alpha, b);
        double *tmp = a;
        a = b;
        b = tmp;
    }
    memcpy(out, a, cells * sizeof(double));
    free(a);
    free(b);
    return 0;
}

/* Number of threads the OpenMP runtime will use (0 when built without it). */
int oracle_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
