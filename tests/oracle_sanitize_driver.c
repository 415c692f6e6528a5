/*
 * Drives every entry point of the oracle (oracle/rn_oracle.c, included as one
 * translation unit) over small seeded networks: 2D and 3D, every flow axis,
 * no-flow and periodic sides, undiluted and diluted near the percolation
 * threshold, plus the degenerate shapes (two planes along the flow axis,
 * extent 1 across it). Built with AddressSanitizer and UBSan by
 * tests/test_oracle_sanitizers.py, so an out-of-bounds access, a leak or
 * undefined behaviour in the oracle aborts the run. Exit status 0 when every
 * call returned a valid status and the two mask routes agreed.
 */
#include "../oracle/rn_oracle.c"

#include <stdio.h>

static uint64_t rng_state = 190803301u;
static double uniform01(void)   /* 64-bit LCG (Knuth's MMIX constants), top 53 bits */
{
    rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

static int run_case(int dim, int64_t nx, int64_t ny, int64_t nz, int axis, int periodic, double occupancy)
{
    const int64_t n = nx * ny * nz;
    double *g[3] = {NULL, NULL, NULL};
    for (int k = 0; k < dim; ++k) {
        g[k] = (double *)malloc(sizeof(double) * (size_t)n);
        for (int64_t i = 0; i < n; ++i) {
            const double u = uniform01(), v = uniform01();
            g[k][i] = u < occupancy ? exp(2.0 * (v - 0.5)) : 0.0;
        }
    }
    uint8_t *m1 = (uint8_t *)malloc((size_t)n), *m2 = (uint8_t *)malloc((size_t)n);
    double *P = (double *)malloc(sizeof(double) * (size_t)n);
    int64_t l1 = -1, l2 = -2;
    int bad = 0;
    if (rno_mask_bfs(dim, nx, ny, nz, axis, periodic, g[0], g[1], g[2], m1, &l1) != RNO_OK) bad = 1;
    if (rno_mask_uf(dim, nx, ny, nz, axis, periodic, g[0], g[1], g[2], m2, &l2) != RNO_OK) bad = 1;
    if (!bad && (l1 != l2 || memcmp(m1, m2, (size_t)n) != 0)) bad = 2;
    rno_result res;
    /* x0 = 0 with Jacobi, then the linear initial guess without a preconditioner */
    int st = rno_solve(dim, nx, ny, nz, axis, periodic, g[0], g[1], g[2], 1e-10, 100000, 1, 0, P, m1, &res);
    if (st != RNO_OK && st != RNO_ENOCONV) bad = 3;
    st = rno_solve(dim, nx, ny, nz, axis, periodic, g[0], g[1], g[2], 1e-10, 100000, 0, 1, P, m1, &res);
    if (st != RNO_OK && st != RNO_ENOCONV) bad = 3;
    double out[10];
    if (rno_check_pressure(dim, nx, ny, nz, axis, periodic, g[0], g[1], g[2], P, out) != RNO_OK) bad = 4;
    if (bad)
        fprintf(stderr, "case dim %d %lldx%lldx%lld axis %d periodic %d occ %.2f: failure %d\n", dim, (long long)nx,
                (long long)ny, (long long)nz, axis, periodic, occupancy, bad);
    for (int k = 0; k < dim; ++k) free(g[k]);
    free(m1);
    free(m2);
    free(P);
    return bad;
}

int main(void)
{
    int fails = 0, cases = 0;
    const double occ[3] = {1.0, 0.7, 0.5};
    for (int periodic = 0; periodic <= 1; ++periodic)
        for (int o = 0; o < 3; ++o) {
            for (int axis = 0; axis < 2; ++axis) {
                fails += run_case(2, 13, 9, 1, axis, periodic, occ[o]) != 0; ++cases;
                fails += run_case(2, 2, 7, 1, axis, periodic, occ[o]) != 0; ++cases;
                fails += run_case(2, 6, 1, 1, 0, periodic, occ[o]) != 0; ++cases;
            }
            for (int axis = 0; axis < 3; ++axis) {
                fails += run_case(3, 7, 6, 5, axis, periodic, occ[o] * 0.8) != 0; ++cases;
                fails += run_case(3, 2, 3, 4, axis, periodic, occ[o]) != 0; ++cases;
            }
        }
    /* invalid arguments take the error path */
    /* 2 x 2 lattice: entry 3 of either array is past the edge, entry 0 of the
       x-bonds is the in-lattice bond (0,0) -> (1,0) */
    double g0[4] = {1, 1, 1, 1}, g1[4] = {1, 1, 1, -1}, g2[4] = {-1, 1, 1, 1};
    uint8_t m[4];
    int64_t l;
    if (rno_mask_bfs(2, 2, 2, 1, 0, 0, g0, g1, NULL, m, &l) != RNO_OK) ++fails;   /* edge entry ignored */
    if (rno_mask_bfs(2, 2, 2, 1, 0, 0, g2, g0, NULL, m, &l) == RNO_OK) ++fails;   /* negative in-lattice bond */
    if (rno_mask_bfs(4, 2, 2, 1, 0, 0, g0, g0, NULL, m, &l) == RNO_OK) ++fails;   /* dim 4 */
    cases += 3;
    printf("%d cases, %d failures\n", cases, fails);
    return fails != 0;
}
