/*
 * nf.h -- C ABI of the MI355X near-field force library (libnf.so).
 *
 * The library computes the near-field part of the compact near/far force
 * split of Garrison, Eisenstein & Pinto (arXiv:1810.02916):
 *
 *   Sec. 2.1  A periodic box of side L is cut into K^3 cubic cells and every
 *             particle belongs to exactly one cell.  Particles whose cells are
 *             at most R = 2 cells apart on every axis (the 5x5x5 block of cells
 *             around a particle's own cell) interact by direct pairwise
 *             summation.  Positions are kept as single-precision offsets from
 *             the centre of their cell.
 *   Sec. 4.3  The pair force is the spline-softened law of Eq. 2,
 *               F(r) = [10 - 15 (r/e) + 6 (r/e)^2] r / e^3   (r <  e)
 *               F(r) = r / |r|^3                            (r >= e)
 *             with e = eps_s, the spline radius.  The paper picks a
 *             Plummer-equivalent length eps_p and uses eps_s = 2.16 eps_p; this
 *             ABI takes eps_s itself.
 *   Sec. 4.5  The near field is an exact sum whose only error is floating-point
 *             round-off.
 *
 * Conventions fixed by this library where the paper is silent:
 *   - a_i = gm * sum_{j in N(i)} F(x_j - x_i), so the force is attractive and
 *     gm = G * m_particle (all particles have equal mass).
 *   - a coincident pair (r = 0, the self pair included) contributes zero.
 *   - cell of a coordinate x: s = x * (K / L) in double precision,
 *     c = floor(s) mod K, offset o = (s - floor(s)) - 1/2 in cell widths,
 *     rounded to float (round to nearest even).  Any finite real x is legal;
 *     it is wrapped into the box.
 *   - linear cell id = (cx * K + cy) * K + cz.
 *
 * Memory: every pointer inside nf_box and every array argument of the compute
 * entry points is a DEVICE pointer owned by the caller.  The library allocates
 * no device memory; temporary storage comes from the caller's workspace, sized
 * by nf_workspace_bytes().  `stream` is a hipStream_t (NULL = null stream).
 * All work is enqueued asynchronously on that stream.
 *
 * Errors: arguments are validated on the host before anything is enqueued.
 * On a non-zero return nothing has been enqueued and no output is touched;
 * nf_last_error() gives a thread-local description.  NF_EHIP reports a HIP
 * launch error (the stream may then hold part of the work).  Faults that
 * happen while kernels run surface at the caller's next synchronisation.
 * No C++ exception crosses this interface.
 *
 * Determinism: for fixed inputs, flags and device the outputs are bitwise
 * reproducible (stable binning, fixed summation order, no float atomics).
 */
#ifndef NF_H
#define NF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NF_ABI_VERSION 2

/* Status codes. */
enum {
    NF_OK = 0,
    NF_EINVAL = 1,        /* an argument is out of range or a pointer is NULL */
    NF_EWORKSPACE = 2,    /* workspace NULL or smaller than nf_workspace_bytes() */
    NF_EHIP = 3,          /* a HIP runtime call failed */
    NF_EUNSUPPORTED = 4   /* sizes beyond the 32-bit index range, or a device
                             that is not gfx950 */
};

/* Flags for nf_accel / nf_accel_vjp. */
enum {
    /* Compensated (Kahan) per-sink accumulation.  Sec. 4.5 names round-off
       in the accumulation of accelerations as the main error source of the
       single-precision near field; this removes it. */
    NF_COMPENSATED = 1u << 0,
    /* Reference kernel: one sink per thread, sources read straight from
       global memory.  Same arithmetic, slower; kept for cross-checks. */
    NF_SIMPLE = 1u << 1,
    /* Plummer softening instead of Eq. 2 (Sec. 4.3, the Plummer law):
       F(r) = r / (r^2 + eps_p^2)^(3/2) for every pair of the block, with the
       box's eps_s field read as the Plummer length eps_p. */
    NF_PLUMMER = 1u << 2,
    /* Evaluate Eq. 2's min form for every pair: the outer-shell shortcut (a
       cell with some |d| = 2 is at r >= 1 cell, so for eps_s <= 1 cell the
       min always selects r^-3 there) is switched off.  Every pair takes the
       same branch as before, so results differ only in the FP32 summation
       order (the light kernel then slices one segment instead of two); the
       point is the cost (for measurement). */
    NF_SPLINE_EVERYWHERE = 1u << 3,
    /* Run the dense, light and narrow kernels one after another on the
       caller's stream instead of side by side on the library's side streams
       (same results, bitwise; for measuring each kernel on its own). */
    NF_SERIAL = 1u << 4,
    /* Newton's third law between dense cells (nf_accel only): every pair lies
       in exactly one of the near and far fields (Sec. 2.1) and the force of
       Eq. 2 is odd in r, so for two cells of 1 to 16 chunks of 64 sinks, all
       summed by the dense kernel, in each other's 5x5x5 block, each pair is
       evaluated once and applied to both particles.  The partial sums are
       combined in a fixed order (bitwise reproducible); the results differ
       from the gather form only in FP32 summation order.  Needs the workspace
       that nf_workspace_bytes reports with this flag (about 520 bytes per
       particle more: room for 16 partial sums per particle); a call whose
       symmetric plan outgrows it runs in the gather form.  At most 2^27
       particles per call (NF_EUNSUPPORTED); not with NF_SIMPLE,
       nf_accel_vjp or nf_accel_noalloc. */
    NF_PAIR_SYMMETRIC = 1u << 5
};

/* Upper bound on boxes per call. */
#define NF_MAX_BOXES 4096

/* Size of the static scratch array of nf_accel_noalloc, per GPU (32 MiB). */
#define NF_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)

/* Highest multipole order of nf_multipoles. */
#define NF_MAX_ORDER 8

/*
 * One periodic box.  Layouts:
 *   pos         [n][3] double, caller (input) order.  Read by nf_bin_particles.
 *   off         [n][4] float, cell-sorted: (ox, oy, oz, cz): the offsets of
 *               Sec. 2.1 in cell widths, each in [-1/2, 1/2], and the
 *               particle's z cell index cz (an integer stored as float).
 *               Written by nf_bin_particles, read by nf_accel / nf_accel_vjp.
 *   cell_start  [K^3 + 1] int32: sorted slots of cell c are
 *               cell_start[c] .. cell_start[c+1]-1; cell_start[K^3] = n.
 *   order       [n] int32: input index of each sorted slot.  Within a cell,
 *               slots are in increasing input index (stable sort).
 *   nbad        optional [1] int32 (may be NULL): nf_bin_particles stores the
 *               number of particles with a non-finite coordinate, or one so
 *               large that s = x K / L has magnitude >= 2^62.  Such particles
 *               are binned into cell 0 at offset 0 and every force computed
 *               for that box is then meaningless; the caller must check it.
 * Requirements: n >= 0, 5 <= K (K = 2R+1 with R = 2; smaller grids would
 * alias the 5x5x5 block), K^3 + 1 <= 2^31 - 1, n <= 2^31 - 1, L and eps_s
 * finite and > 0.  Pointers may be NULL only when n == 0 (cell_start never).
 *
 * Tile choices (dense_min and the four fields after nbad; 0 everywhere picks
 * the library defaults).  The force kernels cut the sinks of a cell into
 * chunks of 64 and sort the chunks into three occupancy classes: a chunk of
 * at least dense_min sinks is dense (one sink per lane, sources broadcast);
 * a smaller last chunk is light (sinks spread over (sink, source-slice) lanes
 * of four waves, sources staged in LDS), or narrow below narrow_max sinks
 * (the same on one wave).  The choices change only speed and the FP32
 * summation order, never which pairs are summed:
 *   dense_min      2..65, default 41
 *   narrow_max     1..64, default 12 (1: no narrow items)
 *   light_window   sources staged per round by a light item: 512, 1024
 *                  (default) or 2048; the VJP stages 512, 768 or 1536
 *   narrow_window  the same for narrow items: 128, 256 (default) or 512; the
 *                  VJP stages 128, 192 or 384
 *   flush          compensated mode: the plain FP32 partial sums folded into
 *                  the compensated sum hold at most this many terms, 1..256,
 *                  default 32 (1 compensates every term)
 * The windows select kernel instances, so all boxes of one call must agree on
 * them (0 and the default are the same choice).  The workspace size depends
 * on dense_min only.
 */
typedef struct nf_box {
    int64_t n;
    int32_t K;
    int32_t dense_min;  /* tile choice: the sinks of a cell are cut into chunks of
                           64; a chunk of at least dense_min sinks is summed one
                           sink per lane (sources broadcast), a smaller one is
                           spread over (sink, source-slice) lanes.  0 picks the
                           library default (41); otherwise 2..65.  The workspace
                           size depends on it (it grows as dense_min falls). */
    double L;
    double eps_s;
    const double *pos;
    float *off;
    int32_t *cell_start;
    int32_t *order;
    int32_t *nbad;
    int32_t narrow_max;
    int32_t light_window;
    int32_t narrow_window;
    int32_t flush;
} nf_box;

/* Library version (NF_ABI_VERSION). */
int nf_version(void);

/* Static text for a status code. */
const char *nf_strerror(int status);

/* Thread-local description of the last failure of this thread ("" if none). */
const char *nf_last_error(void);

/*
 * Bytes of workspace that nf_bin_particles, nf_accel and nf_accel_vjp need
 * for this set of boxes (sizes and dense_min) and flags.  The workspace is
 * scratch only: nothing in it outlives a call, so it may be replaced between
 * calls, e.g. by a larger one after dense_min is lowered.  The same workspace serves all three
 * (calls on one stream run in order; overlapping calls need separate
 * workspaces).  Returns 0 and sets nf_last_error() if the boxes are invalid.
 */
size_t nf_workspace_bytes(int nbox, const nf_box *boxes, uint32_t flags);

/*
 * Binning (Sec. 2.1): for each box, assign every particle to its cell,
 * compute its centre offset, and sort particles by cell (stable).
 * Writes off, cell_start, order (and nbad) of every box.
 * Work: about 40 bytes of HBM traffic per particle per radix pass.
 */
int nf_bin_particles(int nbox, const nf_box *boxes, void *ws, size_t ws_bytes,
                     void *stream);

/*
 * Near-field accelerations (Sec. 2.1 direct sum, Sec. 4.3 Eq. 2):
 *   acc[b][i] = gm * sum_{j in N(i)} F(x_j - x_i)     (length / time^2 units
 *   of gm / L^2), float, [n_b][3] in caller order.
 * Requires the boxes as filled by nf_bin_particles (off, cell_start, order);
 * pos is not read.  acc is an array of nbox device pointers (host array).
 * Arithmetic: FP32 on cell offsets; flags may add NF_COMPENSATED, and
 * NF_PLUMMER selects the Plummer law in place of Eq. 2.
 */
int nf_accel(int nbox, const nf_box *boxes, double gm, uint32_t flags,
             float *const *acc, void *ws, size_t ws_bytes, void *stream);

/*
 * Allocation-free nf_accel, for callers that cannot allocate device memory or
 * hand over a workspace: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments and results as nf_accel,
 * bitwise, without ws / ws_bytes: the call's scratch (descriptor table,
 * planner tables, work items, queue counters) is a static device array of
 * NF_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends.  The first call on a device looks up that device's
 * copy of the array (hipGetSymbolAddress); no call allocates device memory.
 * The dense, light and narrow kernels run one after another on `stream`.
 * Limit: calls whose scratch exceeds NF_NOALLOC_SCRATCH_BYTES return
 * NF_EUNSUPPORTED with nothing enqueued; the scratch is about 20 bytes per
 * cell plus 16 bytes per 41 particles plus 9 KB (a box of 64^3 cells and
 * 2^21 particles needs about 6 MiB; 2^20 cells is the largest grid that fits).
 * Every call on one GPU shares that GPU's array and leaves its contents
 * there (each call clears what it needs zeroed): calls that overlap on one
 * GPU, on other streams or host threads, race and must be ordered by the
 * caller.
 */
int nf_accel_noalloc(int nbox, const nf_box *boxes, double gm, uint32_t flags,
                     float *const *acc, void *stream);

/*
 * Vector-Jacobian product of the accelerations with respect to positions,
 * with the cell assignment held fixed (the derivative is taken inside a cell
 * assignment; it is the derivative of the same sum of Eq. 2 terms):
 *   grad[b][k] = sum_i (d a_i / d x_k)^T cot[b][i]
 *              = gm * kappa^3 * sum_{j in N(k)} J(r_kj) (cot_j - cot_k),
 * where kappa = K/L and J(r) = dF/dr (cell units) is the 3x3 Jacobian of Eq. 2.
 * cot and grad: nbox device pointers each to [n_b][3] float, caller order.
 */
int nf_accel_vjp(int nbox, const nf_box *boxes, double gm, uint32_t flags,
                 const float *const *cot, float *const *grad, void *ws,
                 size_t ws_bytes, void *stream);

/*
 * The work list that nf_accel and nf_accel_vjp build before their force
 * kernels (the near-force work preparation of Sec. 2.2-2.3), without running
 * them: for inspection, and for callers that schedule the work themselves.
 * The sinks of every cell are cut into chunks of 64; a chunk is one item of
 * class 0 (dense: a full chunk, or a last chunk of at least dense_min sinks),
 * 1 (light: a smaller last chunk) or 2 (narrow: a last chunk of fewer than
 * narrow_max sinks), with the boxes' tile choices.
 *   items   device int32 [max_items][4]: (box, cell, chunk, class) of every
 *           item, dense items first, then light, then narrow, each class in
 *           the planner's order (inside one cost bucket or spatial slab that
 *           order may differ between calls; the set of items does not)
 *   counts  device int64 [3]: the number of items of each class (also those
 *           beyond max_items, which are not written)
 * Requires the boxes as filled by nf_bin_particles (cell_start).  ws/ws_bytes
 * as for nf_accel (nf_workspace_bytes with flags 0).  Errors as for nf_accel.
 */
int nf_plan_items(int nbox, const nf_box *boxes, int32_t *items, int64_t max_items,
                  int64_t *counts, void *ws, size_t ws_bytes, void *stream);

/*
 * Per-cell multipole moments of the binned particles (Sec. 2.1: computed for
 * every cell after the binning, double precision inside, float storage;
 * p = 8 is the paper's usual order).  Basis (the paper does not fix one):
 * complete Cartesian moments about the cell centre,
 *   M_abc(cell) = sum_{i in cell} x_i^a y_i^b z_i^c,   a + b + c <= order,
 * of the cell offsets in cell widths (the float offsets of nf_bin_particles,
 * widened to double; products and sums in double, each moment rounded once
 * to float).  mom: nbox device pointers, each to [K_b^3][T] float with
 * T = (order+1)(order+2)(order+3)/6, cells in linear order (cx*K + cy)*K + cz,
 * terms by degree n = a+b+c, then a descending, then b descending.  Every
 * cell is written (0 for an empty cell).  0 <= order <= NF_MAX_ORDER.
 * Requires the boxes as filled by nf_bin_particles (off, cell_start).
 * Work: reads 16 bytes per particle, writes 4 T bytes per cell.
 */
int nf_multipoles(int nbox, const nf_box *boxes, int order, float *const *mom, void *ws,
                  size_t ws_bytes, void *stream);

/*
 * Inputs of the global step choice (Sec. 4.2: the step is bounded by a
 * largest step in ln a, by eta times the per-cell ratio v_rms / a_max and by
 * the step in which the fastest particle moves 80% of a cell).  For every
 * box, from its accelerations and velocities (caller order, [n][3] float) and
 * its binning:
 *   amax[b][c] = max_{i in c} |a_i|, vrms[b][c] = sqrt(mean_{i in c} |v_i|^2)
 *     ([K^3] float each, 0 for an empty cell; the mean velocity is not removed),
 *   glob[3 b + 0..2] = (max_i |a_i|, sqrt(mean_i |v_i|^2), max_i |v_i|)
 *     (device double array of 3 nbox values).
 * Double precision inside, fixed summation order (bitwise reproducible).
 * nf_step_choose turns these values into the step.
 */
int nf_step_stats(int nbox, const nf_box *boxes, const float *const *acc,
                  const float *const *vel, float *const *amax, float *const *vrms,
                  double *glob, void *ws, size_t ws_bytes, void *stream);

/*
 * The global step of Sec. 4.2 from the outputs of nf_step_stats (amax, vrms:
 * nbox device pointers to [K_b^3] float; glob: device [nbox][3] double).
 * The section bounds the one step of all particles by a largest step in ln a,
 * by eta times the ratio v_rms / a_max evaluated within each cell, with the
 * box-wide ratio as a floor against cold cells, and by the step in which the
 * fastest particle moves 80% of a cell.  Per box b, into the device array
 * bounds [nbox][4] double:
 *   bounds[4b+0] = dlna_max / hubble
 *   bounds[4b+1] = eta * max(min over cells with amax > 0 of vrms / amax,
 *                            glob[3b+1] / glob[3b+0])
 *   bounds[4b+2] = (0.8 * L / K) / glob[3b+2]
 *   bounds[4b+3] = the smallest of the three (the step)
 * Each ratio is one double division of the stored values (the per-cell floats
 * widened to double); a ratio whose denominator is zero is +inf; no
 * multiply-add is fused, so the values are bitwise reproducible.  dlna_max,
 * hubble and eta must be finite and > 0 (hubble is the caller's H, giving
 * the ln a bound in time units).
 */
int nf_step_choose(int nbox, const nf_box *boxes, const float *const *amax,
                   const float *const *vrms, const double *glob, double dlna_max, double hubble,
                   double eta, double *bounds, void *ws, size_t ws_bytes, void *stream);

/*
 * The step's Kick and Drift stages, kick then drift, in caller order:
 *   v_i <- float(v_i + kick * a_i)      (evaluated in double, rounded once)
 *   x_i <- x_i + drift * v_i            (double, with the kicked v_i)
 * acc: [n][3] float; vel: [n][3] float, updated in place; pos: [n][3] double,
 * updated in place (it may be the box's pos array; positions are not
 * wrapped, the next nf_bin_particles wraps them).  kick and drift are the
 * caller's step factors (time, or the cosmological kick/drift integrals).
 */
int nf_kick_drift(int nbox, const nf_box *boxes, const float *const *acc, float *const *vel,
                  double *const *pos, double kick, double drift, void *ws, size_t ws_bytes,
                  void *stream);

#ifdef __cplusplus
}
#endif

#endif /* NF_H */
