// nf_multipole.hip -- per-cell multipole moments of the binned particles
// (Sec. 2.1: the step that follows the near-field binning; double precision
// inside, float storage; order p = 8 is the paper's usual choice).
//
// Basis: complete Cartesian moments about the cell centre,
//   M_abc(cell) = sum_{i in cell} x_i^a y_i^b z_i^c,   a + b + c <= p,
// of the float cell offsets (cell widths) widened to double.  Terms are
// stored per cell in degree order n = a + b + c, then a descending, then b
// descending: T = (p+1)(p+2)(p+3)/6 floats per cell, cells in linear order.
//
// One workgroup thread per term.  A workgroup takes a run of consecutive
// cells of bounded cost (particles plus a fixed cost per cell): their
// particles (contiguous in the sorted array) are staged 128 at a time as
// double powers x^k, y^k, z^k in LDS, and each thread sums its term over them
// in sorted order, one cell segment at a time, writing one moment per cell
// as it passes the cell's end.  A thread keeps two partial sums (particles at
// even and odd staged positions) so that consecutive products do not wait on
// each other, and adds them when the cell ends: the order is fixed by the
// partition, so the moments are reproducible.
#include "nf_internal.h"
#include "nf_kernels.h"

namespace nf {
namespace {

constexpr int kMaxOrder = 8;
constexpr int kTermThreads = 192;   // >= (8+1)(8+2)(8+3)/6 = 165
constexpr int kChunk = 128;         // particles staged per round
constexpr int kPow = 3 * (kMaxOrder + 1);   // x^0..8, y^0..8, z^0..8 of one particle
// Work partition: cell c costs its particles plus kCellCost (its T stores);
// workgroup w takes the cells whose cumulative cost
//   cost(c) = cell_start[c] + kCellCost * c
// lies in [w kRange, (w + 1) kRange).  cost is increasing in c, so the first
// cell of every range is found by one pass over the cells.
constexpr int kCellCost = 8;
constexpr int kRange = 512;

// (a, b, c) of each term at the largest order, in storage order; a lower
// order p uses the first (p+1)(p+2)(p+3)/6 entries (the order is by degree).
struct TermTable {
    uint8_t a[kTermThreads], b[kTermThreads], c[kTermThreads];
};
constexpr TermTable make_terms() {
    TermTable t{};
    int k = 0;
    for (int n = 0; n <= kMaxOrder; ++n)
        for (int a = n; a >= 0; --a)
            for (int b = n - a; b >= 0; --b, ++k) {
                t.a[k] = (uint8_t)a;
                t.b[k] = (uint8_t)b;
                t.c[k] = (uint8_t)(n - a - b);
            }
    return t;
}
__constant__ TermTable kTerms = make_terms();

__device__ __forceinline__ int64_t cell_cost(const int32_t *cs, int c) {
    return (int64_t)cs[c] + (int64_t)kCellCost * c;
}

// first[w] = smallest c with cost(c) >= w kRange, for w = 0 .. nrange - 1,
// and first[nrange] = ncell.
__global__ void __launch_bounds__(256)
k_mp_ranges(const DevBox *__restrict__ boxes, const int64_t *__restrict__ range_base,
            int32_t *__restrict__ first) {
    const DevBox &B = boxes[blockIdx.y];
    int32_t *f = first + range_base[blockIdx.y] + blockIdx.y;   // nrange + 1 entries per box
    const int nrange = (int)(range_base[blockIdx.y + 1] - range_base[blockIdx.y]);
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c > B.ncell) return;
    if (c == 0) {
        f[0] = 0;
        f[nrange] = B.ncell;
        return;
    }
    const int64_t lo = cell_cost(B.cell_start, c - 1) / kRange + 1;
    const int64_t hi = cell_cost(B.cell_start, c) / kRange;
    for (int64_t w = lo; w <= hi && w < nrange; ++w) f[w] = c;
}

__global__ void __launch_bounds__(kTermThreads)
k_multipoles(const DevBox *__restrict__ boxes, const int64_t *__restrict__ range_base,
             const int32_t *__restrict__ first, int p, int nterms) {
    // powers of the staged particles, particle-major: the threads of one
    // particle read 27 consecutive doubles (distinct banks)
    __shared__ double pw[kChunk][kPow];
    __shared__ int cst[kRange / kCellCost + 1];   // cell starts of the range (<= 64 cells)
    const int box = blockIdx.y;
    const int w = blockIdx.x;
    if ((int64_t)w >= range_base[box + 1] - range_base[box]) return;   // whole workgroup
    const DevBox &B = boxes[box];
    const int32_t *f = first + range_base[box] + box;
    const int t = threadIdx.x;
    // (a, b, c) of this thread's term, as offsets into a particle's powers
    const bool has_term = t < nterms;
    const int ia = has_term ? kTerms.a[t] : 0;
    const int ib = kMaxOrder + 1 + (has_term ? kTerms.b[t] : 0);
    const int ic = 2 * (kMaxOrder + 1) + (has_term ? kTerms.c[t] : 0);
    const int32_t *__restrict__ cs = B.cell_start;
    const float4 *__restrict__ off = B.off;
    float *__restrict__ out = B.out;
    static_assert(kRange % kCellCost == 0, "range bound");
    const int c0 = f[w], c1 = f[w + 1];
    if (c0 >= c1) return;
    // each cell costs >= kCellCost, so a range holds at most kRange / kCellCost cells
    for (int k = t; k <= c1 - c0; k += kTermThreads) cst[k] = cs[c0 + k];
    __syncthreads();
    const int p0 = cst[0], p1 = cst[c1 - c0];
    int cell = c0;            // current cell (uniform)
    int cend = cst[1];
    double acc0 = 0.0, acc1 = 0.0;
    for (int s = p0; s < p1; s += kChunk) {
        const int e = min(s + kChunk, p1);
        if (s != p0) __syncthreads();   // the previous chunk is consumed
        if (t < e - s) {
            const float4 o = off[s + t];
            const double x = o.x, y = o.y, z = o.z;
            double px = 1.0, py = 1.0, pz = 1.0;
            for (int k = 0; k <= p; ++k) {
                pw[t][k] = px;
                pw[t][kMaxOrder + 1 + k] = py;
                pw[t][2 * (kMaxOrder + 1) + k] = pz;
                px *= x;
                py *= y;
                pz *= z;
            }
        }
        __syncthreads();
        // segments of the chunk that lie in one cell (bounds are uniform)
        for (int i = s; i < e;) {
            while (i >= cend) {   // cells that end at or before particle i
                if (has_term) out[(int64_t)cell * nterms + t] = (float)(acc0 + acc1);
                acc0 = 0.0;
                acc1 = 0.0;
                ++cell;
                cend = cst[cell - c0 + 1];
            }
            const int j = min(e, cend);
            const int lend = j - s;
            int l = i - s;
#pragma unroll 2
            for (; l + 1 < lend; l += 2) {
                acc0 = __fma_rn(pw[l][ia] * pw[l][ib], pw[l][ic], acc0);
                acc1 = __fma_rn(pw[l + 1][ia] * pw[l + 1][ib], pw[l + 1][ic], acc1);
            }
            if (l < lend) acc0 = __fma_rn(pw[l][ia] * pw[l][ib], pw[l][ic], acc0);
            i = j;
        }
    }
    for (; cell < c1; ++cell) {   // the last non-empty cell and trailing empty ones
        if (has_term) out[(int64_t)cell * nterms + t] = (float)(acc0 + acc1);
        acc0 = 0.0;
        acc1 = 0.0;
    }
}

}  // namespace

int multipole_max_order() { return kMaxOrder; }

int multipole_terms(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

int64_t multipole_ranges(int64_t n, int64_t ncell) {
    return (n + (int64_t)kCellCost * ncell) / kRange + 1;
}

hipError_t multipole_launch(const DevBox *d_boxes, int nbox, int64_t max_ncell,
                            int64_t max_ranges, const int64_t *d_range_base, int32_t *d_first,
                            int p, hipStream_t s) {
    hipLaunchKernelGGL(k_mp_ranges, dim3((unsigned)((max_ncell + 1 + 255) / 256), (unsigned)nbox),
                       dim3(256), 0, s, d_boxes, d_range_base, d_first);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_multipoles, dim3((unsigned)max_ranges, (unsigned)nbox), dim3(kTermThreads),
                       0, s, d_boxes, d_range_base, (const int32_t *)d_first, p,
                       multipole_terms(p));
    return hipGetLastError();
}

}  // namespace nf
