/*
 * Drives the host side of libnf.so (include/nf.h) without a GPU, for an
 * AddressSanitizer + UndefinedBehaviorSanitizer build of the library's host
 * code: workspace sizing for one box, many uneven boxes and NF_MAX_BOXES
 * boxes, and every validation failure of every entry point (each must be
 * refused before any device call).  Exits non-zero on an unexpected status;
 * the sanitizers abort on any invalid access or undefined operation.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "nf.h"

static int fails = 0;
static void expect(int got, int want, const char *what) {
    if (got != want) {
        fprintf(stderr, "%s: status %d, expected %d (%s)\n", what, got, want, nf_last_error());
        ++fails;
    }
}

static nf_box box(int64_t n, int32_t K) {
    nf_box b;
    memset(&b, 0, sizeof b);
    b.n = n;
    b.K = K;
    b.L = 1.0;
    b.eps_s = 0.01;
    b.pos = (const double *)0x1000;
    b.off = (float *)0x2000;
    b.cell_start = (int32_t *)0x3000;
    b.order = (int32_t *)0x4000;
    return b;
}

int main(void) {
    char ws_store[64];
    void *ws = (void *)(((uintptr_t)ws_store + 255) & ~(uintptr_t)255); /* never dereferenced */
    if (nf_version() != NF_ABI_VERSION) ++fails;
    for (int c = -1; c < 7; ++c)
        if (!nf_strerror(c) || !nf_strerror(c)[0]) ++fails;
    /* workspace sizing */
    nf_box one = box(100000, 32);
    if (nf_workspace_bytes(1, &one, 0) == 0) ++fails;
    nf_box *many = calloc(NF_MAX_BOXES + 1, sizeof(nf_box));
    for (int b = 0; b <= NF_MAX_BOXES; ++b) many[b] = box(1 + (b * 7919) % 5000, 5 + b % 9);
    if (nf_workspace_bytes(NF_MAX_BOXES, many, 0) == 0) ++fails;
    if (nf_workspace_bytes(NF_MAX_BOXES + 1, many, 0) != 0) ++fails;
    if (nf_workspace_bytes(0, many, 0) != 0) ++fails;
    if (nf_workspace_bytes(1, NULL, 0) != 0) ++fails;
    many[1].light_window = 2048; /* windows must agree across boxes */
    if (nf_workspace_bytes(3, many, 0) != 0) ++fails;
    /* every field out of range */
    nf_box bad[14];
    for (int k = 0; k < 14; ++k) bad[k] = box(10, 8);
    bad[0].n = -1;
    bad[1].K = 4;
    bad[2].L = 0.0;
    bad[3].L = INFINITY;
    bad[4].eps_s = NAN;
    bad[5].dense_min = 1;
    bad[6].narrow_max = 65;
    bad[7].light_window = 768;
    bad[8].narrow_window = 64;
    bad[9].flush = 257;
    bad[10].off = NULL;
    bad[11].cell_start = NULL;
    bad[12].K = 1300;          /* K^3 + 1 over 2^31 - 1 */
    bad[13].n = (int64_t)1 << 31;
    for (int k = 0; k < 14; ++k) {
        if (nf_workspace_bytes(1, &bad[k], 0) != 0) {
            fprintf(stderr, "bad box %d accepted\n", k);
            ++fails;
        }
        if (!nf_last_error()[0]) ++fails;
    }
    /* each entry point refuses before touching a device */
    nf_box good = box(10, 8);
    float *outs[1] = {(float *)0x5000};
    const float *cots[1] = {(const float *)0x6000};
    float *nulls[1] = {NULL};
    expect(nf_bin_particles(1, &bad[1], ws, 1 << 20, NULL), NF_EINVAL, "bin K");
    expect(nf_bin_particles(1, &good, NULL, 1 << 20, NULL), NF_EWORKSPACE, "bin ws");
    expect(nf_bin_particles(1, &good, ws, 16, NULL), NF_EWORKSPACE, "bin ws size");
    expect(nf_bin_particles(1, &good, (char *)ws + 1, (size_t)1 << 30, NULL), NF_EWORKSPACE,
           "bin ws align");
    expect(nf_accel(1, &good, 1.0, 1u << 7, outs, ws, 1 << 20, NULL), NF_EINVAL, "accel flag");
    expect(nf_accel(1, &good, NAN, 0, outs, ws, 1 << 20, NULL), NF_EINVAL, "accel gm");
    expect(nf_accel(1, &good, 1.0, 0, nulls, ws, 1 << 20, NULL), NF_EINVAL, "accel out");
    expect(nf_accel(1, &bad[13], 1.0, 0, outs, ws, 1 << 20, NULL), NF_EUNSUPPORTED, "accel n");
    expect(nf_accel_vjp(1, &good, 1.0, 0, NULL, outs, ws, 1 << 20, NULL), NF_EINVAL, "vjp cot");
    expect(nf_accel_vjp(1, &good, 1.0, 0, cots, NULL, ws, 1 << 20, NULL), NF_EINVAL, "vjp out");
    nf_box big = box(10, 160);
    expect(nf_accel_noalloc(1, &big, 1.0, 0, outs, NULL), NF_EUNSUPPORTED, "noalloc size");
    expect(nf_accel_noalloc(1, &good, 1.0, 1u << 9, outs, NULL), NF_EINVAL, "noalloc flag");
    expect(nf_multipoles(1, &good, 9, outs, ws, 1 << 20, NULL), NF_EINVAL, "multipoles order");
    expect(nf_multipoles(1, &good, 8, nulls, ws, 1 << 20, NULL), NF_EINVAL, "multipoles out");
    expect(nf_step_stats(1, &good, (const float *const *)outs, (const float *const *)outs, outs,
                         outs, NULL, ws, 1 << 20, NULL), NF_EINVAL, "stats glob");
    double *g = (double *)0x7000;
    expect(nf_step_choose(1, &good, (const float *const *)outs, (const float *const *)outs, g,
                          0.0, 1.0, 0.1, g, ws, 1 << 20, NULL), NF_EINVAL, "choose dlna");
    expect(nf_step_choose(1, &good, (const float *const *)outs, (const float *const *)outs, g,
                          0.1, 1.0, 0.1, NULL, ws, 1 << 20, NULL), NF_EINVAL, "choose out");
    double *ps[1] = {g};
    expect(nf_kick_drift(1, &good, (const float *const *)outs, outs, ps, NAN, 0.1, ws, 1 << 20,
                         NULL), NF_EINVAL, "kick nan");
    free(many);
    if (fails) {
        fprintf(stderr, "%d unexpected results\n", fails);
        return 1;
    }
    printf("abi driver ok\n");
    return 0;
}
