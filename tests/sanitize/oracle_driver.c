/*
 * Drives every entry point of the FP64 oracle (oracle/nf_oracle.c) on small
 * seeded boxes, for an AddressSanitizer + UndefinedBehaviorSanitizer build:
 * empty and one-particle boxes, K = 5 (the block is the whole box), sink
 * subsets with repeats, both laws, both offset modes, positions outside the
 * box and on cell faces, and the error returns (bad eps, bad sink index).
 * Exits non-zero if a call returns an unexpected status; the sanitizers
 * abort on any invalid access or undefined operation.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_cells(int64_t n, const double *pos, int32_t K, double L, int64_t *cell, double *off);
int oracle_bin(int64_t n, const double *pos, int32_t K, double L, int32_t *cell_start,
               int32_t *order, float *off);
int oracle_accel(int64_t n, const double *pos, int32_t K, double L, double eps_s, double gm,
                 int law, int round_offsets, int64_t nsink, const int64_t *sinks, double *acc,
                 int64_t *interactions);
int oracle_jvp(int64_t n, const double *pos, int32_t K, double L, double eps_s, double gm,
               int law, int round_offsets, const double *tvec, int64_t nsink,
               const int64_t *sinks, double *out);
int oracle_vjp(int64_t n, const double *pos, int32_t K, double L, double eps_s, double gm,
               int law, int round_offsets, const double *v, double *out);
int oracle_interactions(int64_t n, const double *pos, int32_t K, double L, int64_t *total);

static uint64_t state = 0x9e3779b97f4a7c15ull;
static double uni(void) { /* xorshift64*, uniform in [0, 1) */
    state ^= state >> 12;
    state ^= state << 25;
    state ^= state >> 27;
    return (double)((state * 0x2545f4914f6cdd1dull) >> 11) * (1.0 / 9007199254740992.0);
}

static int fails = 0;
static void expect(int got, int want, const char *what) {
    if (got != want) {
        fprintf(stderr, "%s: status %d, expected %d\n", what, got, want);
        ++fails;
    }
}

static void run_box(int64_t n, int32_t K, double L, double eps) {
    double *pos = malloc(sizeof(double) * 3 * (n ? n : 1));
    double *t = malloc(sizeof(double) * 3 * (n ? n : 1));
    for (int64_t i = 0; i < 3 * n; ++i) {
        pos[i] = (uni() * 3.0 - 1.0) * L; /* inside and outside the box */
        t[i] = uni() - 0.5;
    }
    if (n > 3) {
        pos[0] = 0.0;          /* on a face */
        pos[4] = L;            /* x = L wraps to 0 */
        pos[8] = -L / K;       /* a whole cell below */
    }
    int64_t ncell = (int64_t)K * K * K;
    int64_t *cell = malloc(sizeof(int64_t) * 3 * (n ? n : 1));
    double *off = malloc(sizeof(double) * 3 * (n ? n : 1));
    int32_t *cs = malloc(sizeof(int32_t) * (ncell + 1));
    int32_t *order = malloc(sizeof(int32_t) * (n ? n : 1));
    float *off4 = malloc(sizeof(float) * 4 * (n ? n : 1));
    double *a = malloc(sizeof(double) * 3 * (n ? n : 1));
    double *g = malloc(sizeof(double) * 3 * (n ? n : 1));
    expect(oracle_cells(n, pos, K, L, cell, off), 0, "cells");
    expect(oracle_bin(n, pos, K, L, cs, order, off4), 0, "bin");
    int64_t cnt = 0, tot = 0;
    for (int law = 0; law < 2; ++law)
        for (int ro = 0; ro < 2; ++ro) {
            expect(oracle_accel(n, pos, K, L, eps, 1.5, law, ro, 0, NULL, a, &cnt), 0, "accel");
            expect(oracle_jvp(n, pos, K, L, eps, 1.5, law, ro, t, 0, NULL, g), 0, "jvp");
            expect(oracle_vjp(n, pos, K, L, eps, 1.5, law, ro, t, g), 0, "vjp");
            if (n > 0) {
                int64_t sinks[5] = {0, n - 1, n / 2, 0, n - 1};
                double as[15], gs[15];
                expect(oracle_accel(n, pos, K, L, eps, 1.0, law, ro, 5, sinks, as, NULL), 0,
                       "accel sinks");
                expect(oracle_jvp(n, pos, K, L, eps, 1.0, law, ro, t, 5, sinks, gs), 0,
                       "jvp sinks");
                int64_t badsink[1] = {n};
                expect(oracle_accel(n, pos, K, L, eps, 1.0, law, ro, 1, badsink, as, NULL), 1,
                       "accel bad sink");
            }
        }
    expect(oracle_interactions(n, pos, K, L, &tot), 0, "interactions");
    if (tot != cnt) {
        fprintf(stderr, "interactions %lld != accel count %lld\n", (long long)tot, (long long)cnt);
        ++fails;
    }
    expect(oracle_accel(n, pos, K, L, 0.0, 1.0, 0, 0, 0, NULL, a, NULL), 1, "eps 0");
    expect(oracle_accel(n, pos, K, L, NAN, 1.0, 0, 0, 0, NULL, a, NULL), 1, "eps nan");
    expect(oracle_accel(n, pos, K, L, eps, 1.0, 2, 0, 0, NULL, a, NULL), 1, "bad law");
    free(pos); free(t); free(cell); free(off); free(cs); free(order); free(off4); free(a);
    free(g);
}

int main(void) {
    run_box(0, 5, 1.0, 0.01);
    run_box(1, 5, 1.0, 0.01);
    run_box(300, 5, 2.0, 0.05);
    run_box(2000, 7, 1.0, 0.004);
    run_box(3000, 11, 3.0, 0.02);
    if (fails) {
        fprintf(stderr, "%d unexpected statuses\n", fails);
        return 1;
    }
    printf("oracle driver ok\n");
    return 0;
}
