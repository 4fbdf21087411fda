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
// One workgroup thread per term.  A workgroup walks batches of kBatch
// consecutive cells: the particles of the batch (contiguous in the sorted
// array) are staged 64 at a time as double powers x^k, y^k, z^k in LDS, and
// each thread sums its term over them in sorted order, writing one moment
// per cell as it passes the cell's end.  Bound by the moment writes.
#include "nf_internal.h"
#include "nf_kernels.h"

namespace nf {
namespace {

constexpr int kMaxOrder = 8;
constexpr int kTermThreads = 192;   // >= (8+1)(8+2)(8+3)/6 = 165
constexpr int kChunk = 64;          // particles staged per round
constexpr int kBatch = 16;          // cells per workgroup pass

__global__ void __launch_bounds__(kTermThreads)
k_multipoles(const DevBox *__restrict__ boxes, int p, int nterms) {
    __shared__ double pw[3][kMaxOrder + 1][kChunk];
    __shared__ int cst[kBatch + 1];
    const DevBox &B = boxes[blockIdx.y];
    const int t = threadIdx.x;
    // (a, b, c) of this thread's term
    int ta = 0, tb = 0, tc = 0;
    {
        int k = 0;
        for (int n = 0; n <= p; ++n)
            for (int a = n; a >= 0; --a)
                for (int b = n - a; b >= 0; --b, ++k)
                    if (k == t) {
                        ta = a;
                        tb = b;
                        tc = n - a - b;
                    }
    }
    const bool has_term = t < nterms;
    const int ncell = B.ncell;
    const float4 *__restrict__ off = B.off;
    float *__restrict__ out = B.out;
    const int nbatch = (ncell + kBatch - 1) / kBatch;
    for (int bi = blockIdx.x; bi < nbatch; bi += gridDim.x) {
        const int c0 = bi * kBatch, nc = min(kBatch, ncell - c0);
        __syncthreads();   // the previous batch is done with cst and pw
        if (t <= nc) cst[t] = B.cell_start[c0 + t];
        __syncthreads();
        const int p0 = cst[0], p1 = cst[nc];
        int cell = 0;            // current cell of the batch (uniform)
        int cend = cst[1];
        double acc = 0.0;
        for (int s = p0; s < p1; s += kChunk) {
            const int e = min(s + kChunk, p1);
            if (s != p0) __syncthreads();   // the previous chunk is consumed
            if (t < e - s) {
                const float4 o = off[s + t];
                const double x = o.x, y = o.y, z = o.z;
                double px = 1.0, py = 1.0, pz = 1.0;
                for (int k = 0; k <= p; ++k) {
                    pw[0][k][t] = px;
                    pw[1][k][t] = py;
                    pw[2][k][t] = pz;
                    px *= x;
                    py *= y;
                    pz *= z;
                }
            }
            __syncthreads();
            for (int i = s; i < e; ++i) {
                while (i >= cend) {   // cells that end before particle i (uniform)
                    if (has_term) out[(int64_t)(c0 + cell) * nterms + t] = (float)acc;
                    acc = 0.0;
                    ++cell;
                    cend = cst[cell + 1];
                }
                const int l = i - s;
                acc = __fma_rn(pw[0][ta][l] * pw[1][tb][l], pw[2][tc][l], acc);
            }
        }
        for (; cell < nc; ++cell) {   // the last non-empty cell and trailing empty ones
            if (has_term) out[(int64_t)(c0 + cell) * nterms + t] = (float)acc;
            acc = 0.0;
        }
    }
}

}  // namespace

int multipole_max_order() { return kMaxOrder; }

int multipole_terms(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

hipError_t multipole_launch(const DevBox *d_boxes, int nbox, int64_t max_ncell, int p,
                            hipStream_t s) {
    const int64_t nb = (max_ncell + kBatch - 1) / kBatch;
    const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>(nb, 4096));
    hipLaunchKernelGGL(k_multipoles, dim3(gx, (unsigned)nbox), dim3(kTermThreads), 0, s, d_boxes,
                       p, multipole_terms(p));
    return hipGetLastError();
}

}  // namespace nf
