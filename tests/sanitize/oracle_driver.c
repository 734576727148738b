/* The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).
 * argv[1]: binary file of the Joe-Kuo primitive polynomials (int64 [ndim]),
 * argv[2]: their initial direction values (int64 [ndim][cols]), argv[3]:
 * ndim, argv[4]: cols.  The direction numbers come from the oracle's own
 * recurrence (or_sobol_directions), run here too.
 * Runs every entry point on small and edge-case shapes; exit 0 and no
 * sanitizer report = pass. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/amq_oracle.h"

static int fails = 0;
#define CHECK(c) do { if (!(c)) { fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); ++fails; } } while (0)

int main(int argc, char **argv)
{
    if (argc < 5) return 2;
    const int ndim = atoi(argv[3]), cols = atoi(argv[4]);
    int64_t *poly = (int64_t *)malloc(sizeof(int64_t) * (size_t)ndim);
    int64_t *vinit = (int64_t *)malloc(sizeof(int64_t) * (size_t)ndim * (size_t)cols);
    uint32_t *V = (uint32_t *)malloc(sizeof(uint32_t) * 32 * (size_t)ndim);
    FILE *f = fopen(argv[1], "rb"), *g = fopen(argv[2], "rb");
    if (!f || !g || !poly || !vinit || !V) return 3;
    if (fread(poly, sizeof(int64_t), (size_t)ndim, f) != (size_t)ndim) return 3;
    if (fread(vinit, sizeof(int64_t), (size_t)ndim * cols, g) != (size_t)ndim * cols) return 3;
    fclose(f);
    fclose(g);
    CHECK(or_sobol_directions(ndim, poly, vinit, cols, V) == 0);
    free(poly);
    free(vinit);

    /* points, normals, bridge */
    uint32_t *blk = (uint32_t *)malloc(sizeof(uint32_t) * 7 * 100);
    or_sobol_block(V, 7, 1, 100, blk);
    for (int i = 0; i < 700; ++i) CHECK(blk[i] == or_sobol_int(V, i % 7, 1 + (uint64_t)(i / 7)));
    free(blk);
    CHECK(or_inv_normal_u32(2147483648u) == 0.0);
    CHECK(isfinite(or_inv_normal_u32(1u)) && isfinite(or_inv_normal_u32(4294967295u)));
    CHECK(isfinite(or_inv_normal_mid_u32(0u)) && isfinite(or_inv_normal_mid_u32(4294967295u)));
    for (int M = 1; M <= ndim; M += (M < 20 ? 1 : 37)) {
        int32_t *m = malloc(sizeof(int32_t) * M), *l = malloc(sizeof(int32_t) * M), *r = malloc(sizeof(int32_t) * M);
        double *z = malloc(sizeof(double) * M), *W = malloc(sizeof(double) * (M + 1));
        CHECK(or_bridge_nodes(M, m, l, r) == 0);
        for (int q = 0; q < M; ++q) z[q] = 0.25 * (q % 5) - 0.5;
        or_bridge_apply(M, 1.5, z, W);
        for (int q = 0; q <= M; ++q) CHECK(isfinite(W[q]));
        free(m); free(l); free(r); free(z); free(W);
    }

    /* pricing on every mode and basis, edge shapes included */
    const or_params put = {36.0, 40.0, 0.06, 0.2, 1.0, 0, 1};
    const or_params call = {100.0, 95.0, 0.03, 0.3, 0.75, 1, 1};
    const or_params euro = {100.0, 100.0, 0.05, 0.25, 1.0, 0, 0};
    const or_params *ps[3] = {&put, &call, &euro};
    const int64_t Ns[] = {1, 2, 3, 7, 64, 1000, 4099};
    const int Ms[] = {1, 2, 3, 10, 50};
    double beta[(50 + 1) * OR_BETA_STRIDE];
    int32_t nitm[51];
    for (int pi = 0; pi < 3; ++pi)
        for (size_t ni = 0; ni < sizeof Ns / sizeof Ns[0]; ++ni)
            for (size_t mi = 0; mi < sizeof Ms / sizeof Ms[0]; ++mi)
                for (int kind = 0; kind < 2; ++kind)
                    for (int deg = 0; deg <= 6; deg += 3)
                        for (int s32 = 0; s32 < 2; ++s32) {
                            const int64_t N = Ns[ni];
                            const int M = Ms[mi];
                            if (M > ndim) continue;
                            or_result res;
                            double *pv = malloc(sizeof(double) * (size_t)N);
                            CHECK(or_price_american_stored(ps[pi], V, N, M, kind, deg, NULL, s32, &res, beta, nitm,
                                                           pv) == 0);
                            CHECK(isfinite(res.price) && isfinite(res.std_err) && res.std_err >= 0.0);
                            free(pv);
                        }
    /* shifted points, the paper's estimator, closed forms, lattice */
    uint32_t sh[50];
    for (int q = 0; q < 50; ++q) sh[q] = 0x9E3779B9u * (uint32_t)(q + 1);
    or_result res;
    CHECK(or_price_american_shifted(&put, V, 1000, 50 <= ndim ? 50 : ndim, 0, 2, sh, &res, NULL, NULL, NULL) == 0);
    for (int m = 0; m <= 10; ++m) {
        CHECK(or_paper_estimator(&call, V, 513, m, &res) == 0);
        CHECK(isfinite(res.price));
    }
    CHECK(isfinite(or_bs_price(36.0, 40.0, 0.06, 0.2, 1.0, 0)));
    CHECK(isfinite(or_crr_price(36.0, 40.0, 0.06, 0.2, 1.0, 0, 500, OR_BERMUDAN, 50)));
    CHECK(isfinite(or_crr_price(36.0, 40.0, 0.06, 0.2, 1.0, 1, 500, OR_AMERICAN, 0)));
    /* rejected shapes */
    CHECK(or_price_american_stored(&put, V, 0, 5, 0, 2, NULL, 0, &res, NULL, NULL, NULL) != 0);
    CHECK(or_price_american_stored(&put, V, 10, 0, 0, 2, NULL, 0, &res, NULL, NULL, NULL) != 0);
    CHECK(or_price_american_stored(&put, V, 10, 5, 0, 9, NULL, 0, &res, NULL, NULL, NULL) != 0);
    free(V);
    if (fails) { fprintf(stderr, "%d checks failed\n", fails); return 1; }
    printf("oracle checks passed\n");
    return 0;
}
