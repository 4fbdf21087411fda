/*
 * nf_oracle.c -- plain FP64 CPU oracle for the near-field force.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header or constant with the HIP library: it is written from the paper's
 * definitions so that the GPU path can be checked against it.
 *
 * Definitions followed (Garrison, Eisenstein & Pinto 2019, arXiv:1810.02916):
 *  - Sec. 2.1: the box is split into K^3 cubic cells, each particle belongs to
 *    exactly one cell, and particles in cells at most R = 2 cells apart (per
 *    axis, i.e. the 5x5x5 block of cells around a particle's cell) interact by
 *    direct pairwise summation.  The box is periodic.
 *  - Sec. 2.1: positions are kept as offsets from the centre of their cell.
 *  - Sec. 4.3, Eq. 2: the spline-softened force
 *        F(r) = [10 - 15 (r/e) + 6 (r/e)^2] r / e^3   for r <  e,
 *        F(r) = r / r^3                              for r >= e.
 *  - Sec. 4.5: the near field is an exact sum; the single-precision result is
 *    judged against a double-precision evaluation of the same state.
 *
 * Conventions taken where the paper is silent:
 *  - r = x_source - x_sink, so the force is attractive; accelerations are
 *    a_i = gm * sum_j F(r_ij) with gm = G * m_particle (equal masses).
 *  - a coincident pair (r = 0, including the self pair) contributes 0, the
 *    limit of Eq. 2 as r -> 0.
 *  - cell of a coordinate: s = x * kappa with kappa = K / L, c = floor(s) mod K,
 *    offset o = (s - floor(s)) - 1/2 in cell widths.
 *  - linear cell id = (cx * K + cy) * K + cz; particles sorted by cell id,
 *    ties kept in input order.
 *
 * Everything is evaluated in double precision with the direct (branching)
 * form of Eq. 2, not the single-min form the paper's GPU kernel uses.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EINVAL 1
#define OR_ENOMEM 2

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* Non-negative remainder. */
static int64_t pos_mod(int64_t a, int64_t m) {
    int64_t r = a % m;
    return r < 0 ? r + m : r;
}

/*
 * Cell index and centre offset of every particle (Sec. 2.1).
 *   cell[3*i + a]  in [0, K)
 *   off[3*i + a]   in cell widths, (s - floor(s)) - 1/2
 * Returns OR_EINVAL for a non-finite coordinate or one too large to floor
 * into a 64-bit integer.
 */
int oracle_cells(int64_t n, const double *pos, int32_t K, double L,
                 int64_t *cell, double *off) {
    if (n < 0 || K < 5 || !(L > 0) || !isfinite(L)) return OR_EINVAL;
    const double kappa = (double)K / L;
    for (int64_t i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) {
            volatile double s = pos[3 * i + a] * kappa; /* one rounding, no contraction */
            if (!isfinite(s) || fabs(s) >= 4611686018427387904.0) return OR_EINVAL; /* 2^62 */
            double f = floor(s);
            volatile double frac = s - f;
            volatile double o = frac - 0.5;
            cell[3 * i + a] = pos_mod((int64_t)f, K);
            off[3 * i + a] = o;
        }
    }
    return OR_OK;
}

/*
 * Binning: stable counting sort of particles by linear cell id.
 *   cell_start[K^3 + 1]  first sorted slot of each cell (cell_start[K^3] = n)
 *   order[n]             input index of each sorted slot
 *   off32[n][4]          (ox, oy, oz, cz) of each sorted slot: each offset
 *                        rounded to float with round-to-nearest-even, and
 *                        the z cell index as a float
 */
int oracle_bin(int64_t n, const double *pos, int32_t K, double L,
               int32_t *cell_start, int32_t *order, float *off32) {
    if (n < 0 || K < 5) return OR_EINVAL;
    const int64_t ncell = (int64_t)K * K * K;
    int64_t *cell = (int64_t *)malloc(sizeof(int64_t) * 3 * (size_t)(n > 0 ? n : 1));
    double *off = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    int64_t *count = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    if (!cell || !off || !count) {
        free(cell); free(off); free(count);
        return OR_ENOMEM;
    }
    int rc = oracle_cells(n, pos, K, L, cell, off);
    if (rc != OR_OK) {
        free(cell); free(off); free(count);
        return rc;
    }
    for (int64_t i = 0; i < n; ++i) {
        int64_t id = (cell[3 * i] * K + cell[3 * i + 1]) * K + cell[3 * i + 2];
        count[id + 1] += 1;
    }
    for (int64_t c = 0; c < ncell; ++c) count[c + 1] += count[c];
    for (int64_t c = 0; c <= ncell; ++c) cell_start[c] = (int32_t)count[c];
    /* count[c] is now the next free slot of cell c; walking i upwards keeps
       equal keys in input order. */
    for (int64_t i = 0; i < n; ++i) {
        int64_t id = (cell[3 * i] * K + cell[3 * i + 1]) * K + cell[3 * i + 2];
        int64_t slot = count[id]++;
        order[slot] = (int32_t)i;
        off32[4 * slot + 0] = (float)off[3 * i + 0];
        off32[4 * slot + 1] = (float)off[3 * i + 1];
        off32[4 * slot + 2] = (float)off[3 * i + 2];
        off32[4 * slot + 3] = (float)cell[3 * i + 2];
    }
    free(cell); free(off); free(count);
    return OR_OK;
}

/* Spline-softened pair force in cell units, Eq. 2 (direct piecewise form). */
static void spline_force(const double r[3], double eps, double F[3]) {
    double rho = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    double g;
    if (rho == 0.0) {
        g = 0.0; /* r = 0: the force vector is 0 */
    } else if (rho < eps) {
        double u = rho / eps;
        g = (10.0 - 15.0 * u + 6.0 * u * u) / (eps * eps * eps);
    } else {
        g = 1.0 / (rho * rho * rho);
    }
    F[0] = g * r[0];
    F[1] = g * r[1];
    F[2] = g * r[2];
}

/*
 * Jacobian of the spline force, dF_a/dr_b = g(rho) delta_ab + h(rho) r_a r_b,
 * with g = F/r as in Eq. 2 and h = g'(rho)/rho.  At rho = 0 only the
 * isotropic part 10/e^3 remains.
 */
static void spline_jacobian(const double r[3], double eps, double J[9]) {
    double rho = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    double g, h;
    if (rho < eps) {
        double e3 = eps * eps * eps;
        double u = rho / eps;
        g = (10.0 - 15.0 * u + 6.0 * u * u) / e3;
        /* g'(rho) = (-15/e + 12 rho/e^2) / e^3, h = g'/rho */
        h = (rho == 0.0) ? 0.0 : (-15.0 / eps + 12.0 * rho / (eps * eps)) / (e3 * rho);
    } else {
        double r3 = rho * rho * rho;
        g = 1.0 / r3;
        h = -3.0 / (r3 * rho * rho);
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            J[3 * a + b] = (a == b ? g : 0.0) + h * r[a] * r[b];
}

/* Plummer-softened pair force in cell units (Sec. 4.3, the Plummer law):
   F = r / (rho^2 + eps^2)^(3/2).  Finite at r = 0, where F = 0. */
static void plummer_force(const double r[3], double eps, double F[3]) {
    double w = r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + eps * eps;
    double g = 1.0 / (w * sqrt(w));
    F[0] = g * r[0];
    F[1] = g * r[1];
    F[2] = g * r[2];
}

/* Jacobian of the Plummer force: g = w^(-3/2), h = g'(rho)/rho = -3 w^(-5/2),
   with w = rho^2 + eps^2. */
static void plummer_jacobian(const double r[3], double eps, double J[9]) {
    double w = r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + eps * eps;
    double g = 1.0 / (w * sqrt(w));
    double h = -3.0 * g / w;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            J[3 * a + b] = (a == b ? g : 0.0) + h * r[a] * r[b];
}

/* Softening law: 0 = Eq. 2 spline (eps = spline radius), 1 = Plummer (eps = eps_p). */
static void pair_force(int law, const double r[3], double eps, double F[3]) {
    if (law == 1) plummer_force(r, eps, F); else spline_force(r, eps, F);
}

static void pair_jacobian(int law, const double r[3], double eps, double J[9]) {
    if (law == 1) plummer_jacobian(r, eps, J); else spline_jacobian(r, eps, J);
}

/* Internal binned view built by the force routines below. */
typedef struct {
    int64_t n;
    int32_t K;
    double kappa;
    int64_t *cellv;    /* [n][3] cell coordinates, input order */
    double *off;       /* [n][3] offsets used for the force, input order */
    int64_t *start;    /* [K^3 + 1] */
    int64_t *members;  /* [n] input indices, sorted by cell */
} binned_t;

static void binned_free(binned_t *b) {
    free(b->cellv); free(b->off); free(b->start); free(b->members);
    memset(b, 0, sizeof(*b));
}

/* round_offsets != 0 evaluates on the float-rounded offsets (the GPU's input
   representation) instead of the exact double offsets. */
static int binned_build(binned_t *b, int64_t n, const double *pos, int32_t K,
                        double L, int round_offsets) {
    memset(b, 0, sizeof(*b));
    if (n < 0 || K < 5 || !(L > 0) || !isfinite(L)) return OR_EINVAL;
    const int64_t ncell = (int64_t)K * K * K;
    b->n = n;
    b->K = K;
    b->kappa = (double)K / L;
    size_t nn = (size_t)(n > 0 ? n : 1);
    b->cellv = (int64_t *)malloc(sizeof(int64_t) * 3 * nn);
    b->off = (double *)malloc(sizeof(double) * 3 * nn);
    b->start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    b->members = (int64_t *)malloc(sizeof(int64_t) * nn);
    if (!b->cellv || !b->off || !b->start || !b->members) {
        binned_free(b);
        return OR_ENOMEM;
    }
    int rc = oracle_cells(n, pos, K, L, b->cellv, b->off);
    if (rc != OR_OK) {
        binned_free(b);
        return rc;
    }
    if (round_offsets)
        for (int64_t i = 0; i < 3 * n; ++i) b->off[i] = (double)(float)b->off[i];
    for (int64_t i = 0; i < n; ++i) {
        int64_t id = (b->cellv[3 * i] * K + b->cellv[3 * i + 1]) * K + b->cellv[3 * i + 2];
        b->start[id + 1] += 1;
    }
    for (int64_t c = 0; c < ncell; ++c) b->start[c + 1] += b->start[c];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncell);
    if (!fill) {
        binned_free(b);
        return OR_ENOMEM;
    }
    memcpy(fill, b->start, sizeof(int64_t) * (size_t)ncell);
    for (int64_t i = 0; i < n; ++i) {
        int64_t id = (b->cellv[3 * i] * K + b->cellv[3 * i + 1]) * K + b->cellv[3 * i + 2];
        b->members[fill[id]++] = i;
    }
    free(fill);
    return OR_OK;
}

/* Visit every source j of sink i (5x5x5 cells, each cell once for K >= 5),
   with r = (o_j - o_i) + d in cell widths. */
#define FOR_EACH_NEIGHBOUR(b, i, r, j, BODY)                                        \
    do {                                                                            \
        const int64_t K_ = (b)->K;                                                  \
        const int64_t cx_ = (b)->cellv[3 * (i)], cy_ = (b)->cellv[3 * (i) + 1],     \
                      cz_ = (b)->cellv[3 * (i) + 2];                                \
        for (int dx_ = -2; dx_ <= 2; ++dx_)                                         \
            for (int dy_ = -2; dy_ <= 2; ++dy_)                                     \
                for (int dz_ = -2; dz_ <= 2; ++dz_) {                               \
                    int64_t c_ = (pos_mod(cx_ + dx_, K_) * K_ + pos_mod(cy_ + dy_, K_)) \
                                     * K_ + pos_mod(cz_ + dz_, K_);                 \
                    for (int64_t s_ = (b)->start[c_]; s_ < (b)->start[c_ + 1]; ++s_) { \
                        const int64_t j = (b)->members[s_];                         \
                        double r[3];                                                \
                        r[0] = ((b)->off[3 * j + 0] - (b)->off[3 * (i) + 0]) + dx_; \
                        r[1] = ((b)->off[3 * j + 1] - (b)->off[3 * (i) + 1]) + dy_; \
                        r[2] = ((b)->off[3 * j + 2] - (b)->off[3 * (i) + 2]) + dz_; \
                        BODY                                                        \
                    }                                                               \
                }                                                                   \
    } while (0)

/*
 * Near-field accelerations, FP64.
 *   sinks == NULL: every particle, acc is [n][3] in input order.
 *   otherwise:     acc is [nsink][3] for the listed input indices.
 * round_offsets: 0 = exact double offsets, 1 = float-rounded offsets.
 * Also returns the number of pair evaluations (self pairs included) in
 * *interactions when non-NULL.
 */
int oracle_accel(int64_t n, const double *pos, int32_t K, double L, double eps_s,
                 double gm, int law, int round_offsets, int64_t nsink, const int64_t *sinks,
                 double *acc, int64_t *interactions) {
    if (!(eps_s > 0) || !isfinite(eps_s) || !isfinite(gm) || law < 0 || law > 1)
        return OR_EINVAL;
    binned_t b;
    int rc = binned_build(&b, n, pos, K, L, round_offsets);
    if (rc != OR_OK) return rc;
    const double eps = eps_s * b.kappa; /* softening radius in cell widths */
    const double scale = gm * b.kappa * b.kappa;
    const int64_t m = sinks ? nsink : n;
    int64_t total = 0;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : total) reduction(| : bad)
    for (int64_t t = 0; t < m; ++t) {
        const int64_t i = sinks ? sinks[t] : t;
        if (i < 0 || i >= n) {
            bad = 1;
            continue;
        }
        double ax = 0.0, ay = 0.0, az = 0.0;
        int64_t cnt = 0;
        FOR_EACH_NEIGHBOUR(&b, i, r, j, {
            double F[3];
            pair_force(law, r, eps, F);
            ax += F[0];
            ay += F[1];
            az += F[2];
            ++cnt;
            (void)j;
        });
        acc[3 * t + 0] = scale * ax;
        acc[3 * t + 1] = scale * ay;
        acc[3 * t + 2] = scale * az;
        total += cnt;
    }
    binned_free(&b);
    if (interactions) *interactions = total;
    return bad ? OR_EINVAL : OR_OK;
}

/*
 * Jacobian-vector product, gather form:
 *   (J t)_i = gm kappa^3 sum_{j in N(i)} Jhat(r_ij) (t_j - t_i)
 * where Jhat = dF/dr in cell units and the cell assignment is held fixed.
 * tvec and out are [n][3] in input order (out: [nsink][3] if sinks given).
 * round_offsets as in oracle_accel.
 */
int oracle_jvp(int64_t n, const double *pos, int32_t K, double L, double eps_s,
               double gm, int law, int round_offsets, const double *tvec, int64_t nsink,
               const int64_t *sinks, double *out) {
    if (!(eps_s > 0) || !isfinite(eps_s) || !isfinite(gm) || law < 0 || law > 1)
        return OR_EINVAL;
    binned_t b;
    int rc = binned_build(&b, n, pos, K, L, round_offsets);
    if (rc != OR_OK) return rc;
    const double eps = eps_s * b.kappa;
    const double scale = gm * b.kappa * b.kappa * b.kappa;
    const int64_t m = sinks ? nsink : n;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(| : bad)
    for (int64_t t = 0; t < m; ++t) {
        const int64_t i = sinks ? sinks[t] : t;
        if (i < 0 || i >= n) {
            bad = 1;
            continue;
        }
        double o0 = 0.0, o1 = 0.0, o2 = 0.0;
        FOR_EACH_NEIGHBOUR(&b, i, r, j, {
            double J[9];
            pair_jacobian(law, r, eps, J);
            double d0 = tvec[3 * j] - tvec[3 * i];
            double d1 = tvec[3 * j + 1] - tvec[3 * i + 1];
            double d2 = tvec[3 * j + 2] - tvec[3 * i + 2];
            o0 += J[0] * d0 + J[1] * d1 + J[2] * d2;
            o1 += J[3] * d0 + J[4] * d1 + J[5] * d2;
            o2 += J[6] * d0 + J[7] * d1 + J[8] * d2;
        });
        out[3 * t + 0] = scale * o0;
        out[3 * t + 1] = scale * o1;
        out[3 * t + 2] = scale * o2;
    }
    binned_free(&b);
    return bad ? OR_EINVAL : OR_OK;
}

/*
 * Vector-Jacobian product, scatter form written straight from the chain rule:
 *   xbar_k = sum_i (d a_i / d x_k)^T v_i,
 * with d a_i/d x_j = gm kappa^3 Jhat(r_ij) for j != i and
 *      d a_i/d x_i = -gm kappa^3 sum_j Jhat(r_ij).
 * Serial (it scatters into shared outputs).  v and out are [n][3], input order.
 * round_offsets as in oracle_accel.
 */
int oracle_vjp(int64_t n, const double *pos, int32_t K, double L, double eps_s,
               double gm, int law, int round_offsets, const double *v, double *out) {
    if (!(eps_s > 0) || !isfinite(eps_s) || !isfinite(gm) || law < 0 || law > 1)
        return OR_EINVAL;
    binned_t b;
    int rc = binned_build(&b, n, pos, K, L, round_offsets);
    if (rc != OR_OK) return rc;
    const double eps = eps_s * b.kappa;
    const double scale = gm * b.kappa * b.kappa * b.kappa;
    for (int64_t k = 0; k < 3 * n; ++k) out[k] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        FOR_EACH_NEIGHBOUR(&b, i, r, j, {
            double J[9];
            pair_jacobian(law, r, eps, J);
            /* block (i, j): +J ; block (i, i): -J.  Transpose applied to v_i. */
            for (int a = 0; a < 3; ++a) {
                double col = J[0 + a] * v[3 * i] + J[3 + a] * v[3 * i + 1] + J[6 + a] * v[3 * i + 2];
                out[3 * j + a] += scale * col;
                out[3 * i + a] -= scale * col;
            }
        });
    }
    binned_free(&b);
    return OR_OK;
}

/* Sum over sinks of the 5^3-neighbourhood source count (self pairs included). */
int oracle_interactions(int64_t n, const double *pos, int32_t K, double L, int64_t *total) {
    binned_t b;
    int rc = binned_build(&b, n, pos, K, L, 0);
    if (rc != OR_OK) return rc;
    int64_t acc = 0;
    const int64_t K_ = K;
    for (int64_t cx = 0; cx < K_; ++cx)
        for (int64_t cy = 0; cy < K_; ++cy)
            for (int64_t cz = 0; cz < K_; ++cz) {
                int64_t c = (cx * K_ + cy) * K_ + cz;
                int64_t nc = b.start[c + 1] - b.start[c];
                if (!nc) continue;
                int64_t s = 0;
                for (int dx = -2; dx <= 2; ++dx)
                    for (int dy = -2; dy <= 2; ++dy)
                        for (int dz = -2; dz <= 2; ++dz) {
                            int64_t d = (pos_mod(cx + dx, K_) * K_ + pos_mod(cy + dy, K_)) * K_
                                        + pos_mod(cz + dz, K_);
                            s += b.start[d + 1] - b.start[d];
                        }
                acc += nc * s;
            }
    binned_free(&b);
    *total = acc;
    return OR_OK;
}
