/* oracle_check.c — drives the FP64 oracle (oracle/hexsv_oracle.c) under the
 * address and undefined-behaviour sanitizers on the CPU.  It is test
 * infrastructure: tests/test_sanitizers.py compiles it with the oracle and runs
 * it.
 *
 * Every raster kind the tables handle is built (walls, periodic sides, masked
 * domains whose rim is OUTFLOW, side segments, Dirichlet and given-flux cells),
 * checked for a symmetric neighbour relation, and advanced a few steps with
 * rain, plant drag, the viscous flux and infiltration; the books must close.
 * The hex convolution and its gradient run on the masked raster.  Any
 * sanitizer report aborts the process; a failed check exits with status 1.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "hexsv_oracle.h"

static int failures = 0;

#define CHECK(cond, ...)                      \
    do {                                      \
        if (!(cond)) {                        \
            fprintf(stderr, "FAIL: " __VA_ARGS__); \
            fprintf(stderr, "\n");            \
            ++failures;                       \
        }                                     \
    } while (0)

/* Deterministic values in [lo, hi) (a 64-bit LCG; no library generator). */
static uint64_t lcg = 14933u;
static double urand(double lo, double hi) {
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return lo + (hi - lo) * (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}

typedef struct {
    const char *name;
    int nq, nr;
    int32_t side[4];
    int nseg;
    int32_t seg[8];
    int mask;       /* 0: none, 1: hexagon, 2: hexagon + Dirichlet ring, 3: flux column */
    int32_t mask_code;
    int visc;
    double f_inf;
} Case;

static void run_case(const Case *c) {
    const int N = c->nq * c->nr;
    int32_t *nbr = malloc(sizeof(int32_t) * 6 * (size_t)N);
    uint8_t *code = malloc(6 * (size_t)N);
    uint8_t *act = NULL;
    double *z = malloc(sizeof(double) * N), *th = malloc(sizeof(double) * N);
    double *ap = malloc(sizeof(double) * N), *h = malloc(sizeof(double) * N);
    double *v1 = malloc(sizeof(double) * N), *v2 = malloc(sizeof(double) * N);
    if (c->mask) {
        act = malloc((size_t)N);
        const int qc = c->nq / 2, rc = c->nr / 2, R = (c->nq < c->nr ? c->nq : c->nr) / 2 - 2;
        for (int r = 0; r < c->nr; ++r)
            for (int q = 0; q < c->nq; ++q) {
                const int dq = q - qc, dr = r - rc, ds = dq + dr;
                const int d = abs(dq) > abs(dr) ? (abs(dq) > abs(ds) ? abs(dq) : abs(ds))
                                                : (abs(dr) > abs(ds) ? abs(dr) : abs(ds));
                uint8_t a = d <= R ? 1 : 0;
                if (c->mask == 2 && d == R + 1) a = 2;
                if (c->mask == 3) a = q == 0 ? 3 : 1;
                act[r * c->nq + q] = a;
            }
    }
    const int rc = ref_tables(c->nq, c->nr, c->side, c->nseg, c->nseg ? c->seg : NULL, act,
                              c->mask_code, nbr, code);
    CHECK(rc == 0, "%s: ref_tables returned %d", c->name, rc);
    /* a symmetric neighbour relation: j across edge k of i has i across edge k+3 */
    for (int i = 0; i < N; ++i)
        for (int k = 0; k < 6; ++k) {
            const int32_t j = nbr[i * 6 + k];
            if (code[i * 6 + k] == REF_INTERIOR) {
                CHECK(j >= 0 && j < N, "%s: cell %d edge %d: neighbour %d", c->name, i, k, j);
                if (j >= 0 && j < N)
                    CHECK(nbr[j * 6 + (k + 3) % 6] == i, "%s: %d-%d not symmetric", c->name, i, j);
            }
        }
    /* fields: a tilted, rough bed, vegetation, a wet start with currents */
    for (int i = 0; i < N; ++i) {
        const int q = i % c->nq, r = i / c->nq;
        z[i] = 0.02 * r + 0.01 * q + urand(0.0, 0.01);
        th[i] = urand(0.5, 1.0);
        ap[i] = 73.39;
        h[i] = urand(0.0, 0.05);
        v1[i] = urand(-0.3, 0.3);
        v2[i] = urand(-0.3, 0.3);
        if (act) {
            if (act[i] == 0) th[i] = 0.0;
            else if (act[i] == 2) { th[i] = -th[i]; h[i] = 0.05; v1[i] = 0.0; v2[i] = -0.5; }
            else if (act[i] == 3) { th[i] = -1.0; h[i] = 0.04; v1[i] = 0.5; v2[i] = 0.0; }
        }
    }
    ref_params p = {9.81, 0.5, 1.0, 0.0, 0.00709, 0.0, c->visc, c->f_inf, 0.005, NULL};
    double *soil = NULL;
    if (strcmp(c->name, "walls") == 0) { /* a soil coefficient per cell */
        soil = malloc(sizeof(double) * N);
        for (int i = 0; i < N; ++i) soil[i] = urand(0.001, 0.02);
        p.alpha_s_cell = soil;
    }
    ref_rain rn = {1, 50.0 / 3.6e6, 100.0, 400.0};
    ref_books b;
    ref_books_init(N, 1.0, th, h, 0.0, &b);
    const int64_t taken = ref_run(N, nbr, code, 1.0, z, th, ap, &p, &rn, 1e30, 40, h, v1, v2, &b,
                                  NULL, 1);
    CHECK(taken == 40, "%s: ref_run took %lld steps", c->name, (long long)taken);
    CHECK(b.residual <= 1e-12, "%s: books residual %.3e", c->name, b.residual);
    for (int i = 0; i < N; ++i)
        CHECK(isfinite(h[i]) && h[i] >= 0.0 && isfinite(v1[i]) && isfinite(v2[i]),
              "%s: state of cell %d", c->name, i);
    double out[6], vs[2];
    for (int i = 0; i < N; ++i)
        if (th[i] > 0.0) {
            ref_cell_sums(N, nbr, code, 1.0, 9.81, z, th, h, v1, v2, i, out);
            ref_visc_sums(N, nbr, code, 1.0, 9.81, th, h, v1, v2, i, vs);
        }
    if (c->mask == 1) {
        /* hex convolution on the masked raster: the gradient is the adjoint of the
           forward, <y, dy> = <W, dW> + <b, db> for a linear layer */
        const int cin = 3, cout = 2;
        double *x = malloc(sizeof(double) * cin * N), *y = malloc(sizeof(double) * cout * N);
        double *dy = malloc(sizeof(double) * cout * N), *dx = calloc((size_t)cin * N, sizeof(double));
        double W[2 * 3 * 7], bb[2], dW[2 * 3 * 7], db[2];
        for (int e = 0; e < cin * N; ++e) x[e] = urand(-1.0, 1.0);
        for (int e = 0; e < cout * N; ++e) dy[e] = urand(-1.0, 1.0);
        for (int e = 0; e < 42; ++e) W[e] = urand(-1.0, 1.0);
        bb[0] = 0.25;
        bb[1] = -0.5;
        memset(dW, 0, sizeof dW);
        memset(db, 0, sizeof db);
        ref_hexconv_fwd(N, nbr, cin, cout, x, W, bb, y);
        ref_hexconv_bwd(N, nbr, cin, cout, x, W, dy, dx, dW, db);
        double lhs = 0.0, rhs = 0.0, lx = 0.0;
        for (int e = 0; e < cout * N; ++e) lhs += y[e] * dy[e];
        for (int e = 0; e < 42; ++e) rhs += W[e] * dW[e];
        rhs += bb[0] * db[0] + bb[1] * db[1];
        CHECK(fabs(lhs - rhs) <= 1e-10 * (fabs(lhs) + 1.0), "%s: conv adjoint %.17g vs %.17g",
              c->name, lhs, rhs);
        /* and <y - b, dy> = <x, dx> */
        for (int e = 0; e < cin * N; ++e) lx += x[e] * dx[e];
        double ly = 0.0;
        for (int o = 0; o < cout; ++o)
            for (int i = 0; i < N; ++i) ly += (y[o * N + i] - bb[o]) * dy[o * N + i];
        CHECK(fabs(lx - ly) <= 1e-10 * (fabs(ly) + 1.0), "%s: data adjoint %.17g vs %.17g",
              c->name, lx, ly);
        free(x); free(y); free(dy); free(dx);
    }
    free(nbr); free(code); free(act); free(z); free(th); free(ap); free(h); free(v1); free(v2);
    free(soil);
}

int main(void) {
    const Case cases[] = {
        {"walls", 9, 7, {REF_WALL, REF_WALL, REF_WALL, REF_WALL}, 0, {0}, 0, REF_WALL, 0, 0.0},
        {"outflow-segments", 12, 9, {REF_OUTFLOW, REF_WALL, REF_WALL, REF_WALL}, 2,
         {REF_S, 3, 6, REF_WALL, REF_E, 2, 5, REF_OUTFLOW}, 0, REF_WALL, 0, 0.0},
        {"periodic-q", 10, 8, {REF_OUTFLOW, REF_PERIODIC, REF_WALL, REF_PERIODIC}, 0, {0}, 0,
         REF_WALL, 1, 0.0},
        {"periodic-both", 6, 4, {REF_PERIODIC, REF_PERIODIC, REF_PERIODIC, REF_PERIODIC}, 0, {0},
         0, REF_WALL, 1, 1e-5},
        {"periodic-one-column", 1, 5, {REF_WALL, REF_PERIODIC, REF_WALL, REF_PERIODIC}, 0, {0}, 0,
         REF_WALL, 0, 0.0},
        {"masked-cone", 15, 15, {REF_WALL, REF_WALL, REF_WALL, REF_WALL}, 0, {0}, 1, REF_OUTFLOW,
         0, 0.0},
        {"dirichlet-ring", 17, 17, {REF_WALL, REF_WALL, REF_WALL, REF_WALL}, 0, {0}, 2,
         REF_OUTFLOW, 1, 0.0},
        {"flux-column", 12, 6, {REF_WALL, REF_OUTFLOW, REF_WALL, REF_WALL}, 0, {0}, 3, REF_WALL, 1,
         2e-6},
    };
    for (size_t k = 0; k < sizeof(cases) / sizeof(cases[0]); ++k) {
        run_case(&cases[k]);
        printf("%s done\n", cases[k].name);
    }
    /* malformed descriptions are refused, not read past */
    int32_t nbr[6 * 4];
    uint8_t code[6 * 4];
    const int32_t bad_side[4] = {REF_PERIODIC, REF_WALL, REF_WALL, REF_WALL};
    CHECK(ref_tables(2, 2, bad_side, 0, NULL, NULL, REF_WALL, nbr, code) != 0,
          "unpaired periodic side accepted");
    printf("%s\n", failures ? "FAILED" : "OK");
    return failures ? 1 : 0;
}
