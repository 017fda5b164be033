/*
 * oracle_sanitize_test.c -- the CPU oracle's own pins, run as a C program
 * built with AddressSanitizer and UndefinedBehaviorSanitizer (the test suite
 * compiles it with gcc together with oracle/fractal_oracle.c).  Every check
 * compares the oracle with something other than itself:
 *   - member count = 3^k (Eq. 2) for k <= 10;
 *   - lambda is a bijection of Lemma 2's grid onto the non-empty blocks,
 *     found by brute force, in both orientations, r_b <= 8;
 *   - hand-derived lambda values for r_b = 1 and 2 (the mirrored orientation);
 *   - the automaton equals textbook B3/S23 Life on the zero-padded array
 *     (written out here) followed by masking, k <= 6, 12 steps;
 *   - level-1 hand cases: the full 3-cell L lives on, a single cell dies;
 *   - heat on a uniform field: u' = 1 - 4a + a deg4 exactly (closed form);
 *   - a window's exact interior equals the whole-array result.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_member(int64_t x, int64_t y, int k);
uint64_t oracle_count_members(int k);
void oracle_grid_dims(int rb, uint64_t *gx, uint64_t *gy);
void oracle_lambda_paper(int rb, uint64_t wx, uint64_t wy, uint64_t *lx, uint64_t *ly);
void oracle_lambda(int rb, uint64_t wx, uint64_t wy, uint64_t *lx, uint64_t *ly);
void oracle_lambda_grid(int rb, int paper_orient, uint32_t *xy);
void oracle_nonempty_blocks(int k, int r, uint8_t *mask);
int oracle_ca_run(int k, int64_t x0, int64_t y0, int64_t w, int64_t h, const uint8_t *in,
                  int T, uint8_t *out);
int oracle_heat_run(int k, int64_t x0, int64_t y0, int64_t w, int64_t h, const double *in,
                    double alpha, int T, double *out);

static int failures = 0;
#define CHECK(c, ...)                                                                          \
    do {                                                                                       \
        if (!(c)) {                                                                            \
            printf("FAIL %s:%d: ", __FILE__, __LINE__);                                        \
            printf(__VA_ARGS__);                                                               \
            printf("\n");                                                                      \
            ++failures;                                                                        \
        }                                                                                      \
    } while (0)

static uint64_t pow3(int e)
{
    uint64_t p = 1;
    while (e-- > 0)
        p *= 3;
    return p;
}

static void pin_counts(void)
{
    for (int k = 0; k <= 10; ++k)
        CHECK(oracle_count_members(k) == pow3(k), "count k=%d", k);
}

static void pin_lambda_bijection(void)
{
    for (int rb = 0; rb <= 8; ++rb) {
        uint64_t gx, gy;
        oracle_grid_dims(rb, &gx, &gy);
        CHECK(gx * gy == pow3(rb), "grid rb=%d", rb);
        const uint64_t nb = 1ull << rb;
        for (int paper = 0; paper <= 1; ++paper) {
            uint8_t *seen = calloc(nb * nb, 1);
            uint32_t *xy = malloc(sizeof(uint32_t) * 2 * gx * gy);
            oracle_lambda_grid(rb, paper, xy);
            for (uint64_t i = 0; i < gx * gy; ++i) {
                const uint64_t X = xy[2 * i], Y = xy[2 * i + 1];
                CHECK(X < nb && Y < nb, "range rb=%d", rb);
                if (X >= nb || Y >= nb)
                    continue;
                /* the block holds a member: brute force over its one cell */
                const int nonempty = paper ? ((X & (nb - 1 - Y)) == 0) : ((X & Y) == 0);
                CHECK(nonempty, "empty block rb=%d paper=%d (%llu,%llu)", rb, paper,
                      (unsigned long long)X, (unsigned long long)Y);
                CHECK(!seen[Y * nb + X], "repeat rb=%d", rb);
                seen[Y * nb + X] = 1;
            }
            free(seen);
            free(xy);
        }
    }
    /* the image equals the brute-force set of non-empty blocks (k=6, r=2) */
    uint8_t mask[16 * 16];
    oracle_nonempty_blocks(6, 2, mask);
    int count = 0;
    for (int i = 0; i < 256; ++i)
        count += mask[i];
    CHECK(count == 81, "nonempty blocks k=6 r=2: %d", count);
}

static void pin_lambda_values(void)
{
    /* r_b = 1, grid 3 x 1: (0,1) (0,0) (1,0); r_b = 2 row omega_y = 2:
       (2,1) (2,0) (3,0) (hand-derived from Theorem 1's table, mirrored) */
    const uint64_t want1[3][2] = {{0, 1}, {0, 0}, {1, 0}};
    const uint64_t want2[3][2] = {{2, 1}, {2, 0}, {3, 0}};
    for (uint64_t wx = 0; wx < 3; ++wx) {
        uint64_t lx, ly;
        oracle_lambda(1, wx, 0, &lx, &ly);
        CHECK(lx == want1[wx][0] && ly == want1[wx][1], "rb=1 wx=%llu", (unsigned long long)wx);
        oracle_lambda(2, wx, 2, &lx, &ly);
        CHECK(lx == want2[wx][0] && ly == want2[wx][1], "rb=2 wx=%llu", (unsigned long long)wx);
    }
    uint64_t lx = 9, ly = 9;
    oracle_lambda(0, 0, 0, &lx, &ly);
    CHECK(lx == 0 && ly == 0, "rb=0");
}

/* textbook B3/S23 on the zero-padded n x n array, then non-members zeroed */
static void life_masked(int k, const uint8_t *in, uint8_t *out)
{
    const int n = 1 << k;
    for (int y = 0; y < n; ++y)
        for (int x = 0; x < n; ++x) {
            int c = 0;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int xx = x + dx, yy = y + dy;
                    if ((dx || dy) && xx >= 0 && yy >= 0 && xx < n && yy < n)
                        c += in[yy * n + xx];
                }
            const int alive = (c == 3) || (in[y * n + x] && c == 2);
            out[y * n + x] = (uint8_t)(alive && ((x & y) == 0));
        }
}

static void pin_automaton(void)
{
    uint64_t z = 2004;
    for (int k = 1; k <= 6; ++k) {
        const int n = 1 << k;
        uint8_t *a = malloc(n * n), *b = malloc(n * n), *o = malloc(n * n);
        for (int i = 0; i < n * n; ++i) {
            z = z * 6364136223846793005ull + 1442695040888963407ull;
            a[i] = (uint8_t)(((z >> 33) & 1) && (((i % n) & (i / n)) == 0));
        }
        for (int t = 1; t <= 12; ++t) {
            life_masked(k, a, b);
            CHECK(oracle_ca_run(k, 0, 0, n, n, a, 1, o) == 0, "alloc");
            CHECK(memcmp(o, b, n * n) == 0, "automaton k=%d t=%d", k, t);
            memcpy(a, b, n * n);
        }
        free(a);
        free(b);
        free(o);
    }
    const uint8_t l3[4] = {1, 1, 1, 0}, one[4] = {1, 0, 0, 0};
    uint8_t o[4];
    oracle_ca_run(1, 0, 0, 2, 2, l3, 1, o);
    CHECK(memcmp(o, l3, 4) == 0, "L stays live");
    oracle_ca_run(1, 0, 0, 2, 2, one, 1, o);
    CHECK(o[0] == 0 && o[1] == 0 && o[2] == 0 && o[3] == 0, "single cell dies");
}

static void pin_heat(void)
{
    const int k = 5, n = 1 << k;
    const double a = 0.2;
    double *u = malloc(sizeof(double) * n * n), *o = malloc(sizeof(double) * n * n);
    for (int y = 0; y < n; ++y)
        for (int x = 0; x < n; ++x)
            u[y * n + x] = ((x & y) == 0) ? 1.0 : 0.0;
    CHECK(oracle_heat_run(k, 0, 0, n, n, u, a, 1, o) == 0, "alloc");
    for (int y = 0; y < n; ++y)
        for (int x = 0; x < n; ++x) {
            if ((x & y) != 0) {
                CHECK(o[y * n + x] == 0.0, "non-member (%d,%d)", x, y);
                continue;
            }
            int deg = 0;
            const int nx[4] = {x, x, x + 1, x - 1}, ny[4] = {y - 1, y + 1, y, y};
            for (int q = 0; q < 4; ++q)
                deg += nx[q] >= 0 && ny[q] >= 0 && nx[q] < n && ny[q] < n &&
                       (nx[q] & ny[q]) == 0;
            CHECK(fabs(o[y * n + x] - (1.0 - 4.0 * a + a * deg)) < 1e-15, "uniform (%d,%d)", x,
                  y);
        }
    free(u);
    free(o);
}

static void pin_window(void)
{
    const int k = 7, n = 1 << k, T = 5;
    uint8_t *a = calloc(n * n, 1), *full = malloc(n * n);
    uint64_t z = 7;
    for (int i = 0; i < n * n; ++i) {
        z = z * 6364136223846793005ull + 1442695040888963407ull;
        a[i] = (uint8_t)(((z >> 40) & 1) && (((i % n) & (i / n)) == 0));
    }
    oracle_ca_run(k, 0, 0, n, n, a, T, full);
    const int x0 = 20, y0 = 30, w = 50, h = 40;
    uint8_t *win = malloc(w * h), *out = malloc(w * h);
    for (int j = 0; j < h; ++j)
        memcpy(win + j * w, a + (y0 + j) * n + x0, w);
    oracle_ca_run(k, x0, y0, w, h, win, T, out);
    for (int j = T; j < h - T; ++j)
        for (int i = T; i < w - T; ++i)
            CHECK(out[j * w + i] == full[(y0 + j) * n + x0 + i], "window (%d,%d)", i, j);
    free(a);
    free(full);
    free(win);
    free(out);
}

int main(void)
{
    pin_counts();
    pin_lambda_bijection();
    pin_lambda_values();
    pin_automaton();
    pin_heat();
    pin_window();
    if (failures) {
        printf("%d failures\n", failures);
        return 1;
    }
    printf("oracle sanitized pins ok\n");
    return 0;
}
