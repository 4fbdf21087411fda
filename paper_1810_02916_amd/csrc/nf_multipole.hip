// One wave per workgroup.  Lane u owns a unit: a product x^a y^b and up to
// four consecutive powers z^c0 .. z^(c0+3) of the same (a, b), so its terms
// x^a y^b z^c share one product, each added by one fused multiply-add with a
// staged z power (61 units cover the 165 terms of order 8).  Particles are
// staged 64 at a time as double powers x^k, y^k, z^k in LDS (the next 64
// offsets are loaded while the current ones are summed).
//
//   k_multipoles  a run of consecutive cells of bounded cost (particles plus
//                 a fixed cost per cell) per workgroup; each lane adds its
//                 terms over the run's particles in sorted order, one cell
//                 segment at a time, and writes a cell's moments as it passes
//                 the cell's end.  Cells of more than kBig particles are
//                 skipped: one workgroup summing them alone would set the
//                 kernel's length.
//   k_mp_pieces   those cells, cut into pieces of kBig particles, one piece
//                 per workgroup, moments of the piece in double;
//   k_mp_combine  adds a cell's pieces in piece order and writes its moments.
// Every moment is a fixed sequence of double operations, so the moments are
// reproducible.
#include "nf_internal.h"
#include "nf_kernels.h"

namespace nf {
namespace {

constexpr int kMaxOrder = 8;
constexpr int kUnitTerms = 4;       // consecutive z powers per lane
constexpr int kChunk = 64;          // particles staged per round (one per lane)
// staged powers of one particle: x^0..8, y^0..8, then z^0..11 (a unit starting
// at z^8 reads four; the powers past the order feed terms that are never stored)
constexpr int kZPow = kMaxOrder + kUnitTerms;
constexpr int kPow = 2 * (kMaxOrder + 1) + kZPow;
static_assert(kPow % 2 == 0 && (2 * (kMaxOrder + 1)) % 2 == 0 && kUnitTerms % 2 == 0,
              "z powers of a unit are read as 16-byte pairs");
// Work partition: cell c costs its particles plus kCellCost (its T stores);
// workgroup w takes the cells whose cumulative cost
//   cost(c) = cell_start[c] + kCellCost * c
// lies in [w kRange, (w + 1) kRange).  cost is increasing in c, so the first
// cell of every range is found by one pass over the cells.
constexpr int kCellCost = 8;
constexpr int kRange = 512;
constexpr int kBig = 512;           // larger cells are summed in pieces of kBig
constexpr int kMaxTerms = (kMaxOrder + 1) * (kMaxOrder + 2) * (kMaxOrder + 3) / 6;

__device__ __forceinline__ int64_t cell_cost(const int32_t *cs, int c) {
    return (int64_t)cs[c] + (int64_t)kCellCost * c;
}

// Storage index of term (a, b, c), n = a + b + c: the terms of lower degree,
// then a descending, then b descending within degree n.
constexpr int term_index(int a, int b, int c) {
    const int n = a + b + c;
    return n * (n + 1) * (n + 2) / 6 + (n - a) * (n - a + 1) / 2 + (n - a - b);
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

// The lanes' units for every order p: (a, b) pairs in order, each cut into
// runs of <= 4 z powers of which the first uk are terms.  ia, ib, ic index a
// particle's staged powers; idx are the storage indices of the unit's terms,
// and for j >= uk idx[j] repeats idx[0], so that a lane stores all four slots
// without a branch (the extra stores rewrite term 0 with its own value).
// Lanes without a unit repeat lane 0's: they compute and store the same
// values at the same places.  Built at compile time, read once per workgroup.
struct LaneUnit {
    int16_t ia, ib, ic, uk;
    int16_t idx[kUnitTerms];
};
struct UnitTable {
    LaneUnit u[kMaxOrder + 1][64];
};
constexpr UnitTable make_units() {
    UnitTable T{};
    for (int p = 0; p <= kMaxOrder; ++p) {
        int n = 0;
        for (int a = 0; a <= p; ++a)
            for (int b = 0; a + b <= p; ++b)
                for (int c = 0; a + b + c <= p; c += kUnitTerms, ++n) {
                    LaneUnit L{(int16_t)a, (int16_t)(kMaxOrder + 1 + b),
                               (int16_t)(2 * (kMaxOrder + 1) + c),
                               (int16_t)(p - a - b - c + 1 < kUnitTerms ? p - a - b - c + 1
                                                                        : kUnitTerms),
                               {0, 0, 0, 0}};
                    for (int j = 0; j < kUnitTerms; ++j)
                        L.idx[j] = (int16_t)term_index(a, b, j < L.uk ? c + j : c);
                    T.u[p][n] = L;
                }
        for (int t = n; t < 64; ++t) T.u[p][t] = T.u[p][0];
    }
    return T;
}
constexpr int count_units(int p) {
    int n = 0;
    for (int a = 0; a <= p; ++a)
        for (int b = 0; a + b <= p; ++b)
            for (int c = 0; a + b + c <= p; c += kUnitTerms) ++n;
    return n;
}
static_assert(count_units(kMaxOrder) <= 64, "one unit per lane");
__constant__ UnitTable kUnits = make_units();

__device__ __forceinline__ LaneUnit lane_unit(int p, int t) { return kUnits.u[p][t]; }

// Lane t < cnt writes the powers 0..p of x and y and 0..11 of z of its
// particle's offset o.
__device__ __forceinline__ void stage_powers(double (*pw)[kPow], int t, int cnt, int p, float4 o) {
    if (t < cnt) {
        const double x = o.x, y = o.y, z = o.z;
        double px = 1.0, py = 1.0;
        for (int k = 0; k <= p; ++k) {
            pw[t][k] = px;
            pw[t][kMaxOrder + 1 + k] = py;
            px *= x;
            py *= y;
        }
        double pz = 1.0;
#pragma unroll
        for (int k = 0; k < kZPow; ++k) {
            pw[t][2 * (kMaxOrder + 1) + k] = pz;
            pz *= z;
        }
    }
}

// acc[j] += sum over staged particles l in [l0, l1), in order, of
// x^a y^b z^(c0 + j), each term one fused multiply-add of the product
// x^a y^b and the staged z power.  Terms past the unit's last one are computed
// and never stored.
__device__ __forceinline__ void add_staged(const double (*pw)[kPow], int l0, int l1,
                                           const LaneUnit &U, double acc[kUnitTerms]) {
    // unrolled so that the loads and products of several particles are in
    // flight at once; only the additions into acc chain
#pragma unroll 4
    for (int l = l0; l < l1; ++l) {
        const double m = pw[l][U.ia] * pw[l][U.ib];
        // z^c0 .. z^(c0+3): c0 is a multiple of 4 and rows are 16-byte multiples
        const double2 z01 = *reinterpret_cast<const double2 *>(&pw[l][U.ic]);
        const double2 z23 = *reinterpret_cast<const double2 *>(&pw[l][U.ic + 2]);
        acc[0] = __builtin_fma(m, z01.x, acc[0]);
        acc[1] = __builtin_fma(m, z01.y, acc[1]);
        acc[2] = __builtin_fma(m, z23.x, acc[2]);
        acc[3] = __builtin_fma(m, z23.y, acc[3]);
    }
}

// The offset of sorted slot i (x, y, z) through a global pointer.
__device__ __forceinline__ float4 ld_off(gptr<const float> off, int i) {
    const gptr<const float> q = off + 4 * (int64_t)i;   // 4 i passes 2^31 for i >= 2^29
    return make_float4(q[0], q[1], q[2], 0.f);
}

__global__ void __launch_bounds__(64)
k_multipoles(const DevBox *__restrict__ boxes, const int64_t *__restrict__ range_base,
             const int32_t *__restrict__ first, int p, int nterms) {
    __shared__ __align__(16) double pw[kChunk][kPow];   // powers of the staged particles
    const int box = blockIdx.y;
    const int w = blockIdx.x;
    if ((int64_t)w >= range_base[box + 1] - range_base[box]) return;   // whole workgroup
    const DevBox &B = boxes[box];
    const int32_t *f = first + range_base[box] + box;
    const int t = threadIdx.x;
    const LaneUnit U = lane_unit(p, t);
    const gptr<const int32_t> cs = gp(B.cell_start);
    const gptr<const float> off = gp((const float *)B.off);
    const gptr<float> out = gp(B.out);
    static_assert(kRange % kCellCost == 0, "range bound");
    static_assert(kChunk <= 64, "one staged particle per lane");
    const int c0 = f[w], c1 = f[w + 1];
    if (c0 >= c1) return;
    // each cell costs >= kCellCost, so a range holds at most kRange / kCellCost
    // = 64 cells: lane k holds the start and end of the range's cell k, read
    // back with readlane (uniform index, no memory wait)
    static_assert(kRange / kCellCost <= 64, "one cell of the range per lane");
    const int cbeg_l = t < c1 - c0 ? cs[c0 + t] : 0;
    const int cend_l = t < c1 - c0 ? cs[c0 + t + 1] : 0;
    auto cbeg = [&](int cell) { return __builtin_amdgcn_readlane(cbeg_l, cell - c0); };
    auto cend_of = [&](int cell) { return __builtin_amdgcn_readlane(cend_l, cell - c0); };
    double acc[kUnitTerms] = {0.0, 0.0, 0.0, 0.0};
    auto flush = [&](int cell) {
        const gptr<float> o = out + (int64_t)cell * nterms;
        const float v0 = (float)acc[0];
#pragma unroll
        for (int j = 0; j < kUnitTerms; ++j) {
            o[U.idx[j]] = j < U.uk ? (float)acc[j] : v0;
            acc[j] = 0.0;
        }
    };
    // runs [ca, cb) of cells of at most kBig particles (bounds are uniform)
    for (int ca = c0; ca < c1;) {
        if (cend_of(ca) - cbeg(ca) > kBig) {
            ++ca;
            continue;
        }
        int cb = ca + 1;
        while (cb < c1 && cend_of(cb) - cbeg(cb) <= kBig) ++cb;
        const int p0 = cbeg(ca), p1 = cend_of(cb - 1);
        int cell = ca;
        int cend = cend_of(ca);
        float4 o = make_float4(0.f, 0.f, 0.f, 0.f);
        if (t < kChunk && p0 + t < p1) o = ld_off(off, p0 + t);
        for (int s = p0; s < p1; s += kChunk) {
            const int e = min(s + kChunk, p1);
            __syncthreads();   // the previous chunk is consumed
            stage_powers(pw, t, e - s, p, o);
            if (t < kChunk && e + t < p1) o = ld_off(off, e + t);   // next chunk, in flight
            __syncthreads();
            for (int i = s; i < e;) {   // segments of the chunk that lie in one cell
                while (i >= cend) {     // cells that end at or before particle i
                    flush(cell);
                    ++cell;
                    cend = cend_of(cell);
                }
                const int j = min(e, cend);
                add_staged(pw, i - s, j - s, U, acc);
                i = j;
            }
        }
        for (; cell < cb; ++cell) flush(cell);   // the run's last cells (and empty ones)
        ca = cb;
    }
}

// Pieces per cell (0 for a cell of at most kBig particles).
__global__ void __launch_bounds__(256)
k_mp_count(const DevBox *__restrict__ boxes, uint32_t *__restrict__ npieces) {
    const DevBox &B = boxes[blockIdx.y];
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= B.ncell) return;
    const gptr<const int32_t> cs = gp(B.cell_start);
    const int n = cs[c + 1] - cs[c];
    npieces[B.cellbase + c] = n > kBig ? (uint32_t)((n + kBig - 1) / kBig) : 0u;
}

// The pieces of each big cell at its offset (the exclusive scan of the counts).
__global__ void __launch_bounds__(256)
k_mp_emit(const DevBox *__restrict__ boxes, const uint32_t *__restrict__ offsets,
          MpPiece *__restrict__ pieces, int64_t max_pieces) {
    const DevBox &B = boxes[blockIdx.y];
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= B.ncell) return;
    const gptr<const int32_t> cs = gp(B.cell_start);
    const int q = cs[c], n = cs[c + 1] - q;
    if (n <= kBig) return;
    const int np = (n + kBig - 1) / kBig;
    const int64_t at = offsets[B.cellbase + c];
    for (int k = 0; k < np && at + k < max_pieces; ++k)
        pieces[at + k] = MpPiece{(int32_t)blockIdx.y, c, q + k * kBig, min(q + n, q + (k + 1) * kBig),
                                 k, np};
}

__global__ void __launch_bounds__(64)
k_mp_pieces(const DevBox *__restrict__ boxes, const MpPiece *__restrict__ pieces,
            const uint32_t *__restrict__ total, double *__restrict__ partial, int p) {
    __shared__ __align__(16) double pw[kChunk][kPow];
    const int w = blockIdx.x;
    if (w >= (int64_t)*total) return;   // whole workgroup
    const MpPiece pc = pieces[w];
    const DevBox &B = boxes[pc.box];
    const int t = threadIdx.x;
    const LaneUnit U = lane_unit(p, t);
    const gptr<const float> off = gp((const float *)B.off);
    double acc[kUnitTerms] = {0.0, 0.0, 0.0, 0.0};
    float4 o = make_float4(0.f, 0.f, 0.f, 0.f);
    if (t < kChunk && pc.q0 + t < pc.q1) o = ld_off(off, pc.q0 + t);
    for (int s = pc.q0; s < pc.q1; s += kChunk) {
        const int e = min(s + kChunk, pc.q1);
        __syncthreads();
        stage_powers(pw, t, e - s, p, o);
        if (t < kChunk && e + t < pc.q1) o = ld_off(off, e + t);
        __syncthreads();
        add_staged(pw, 0, e - s, U, acc);
    }
#pragma unroll
    for (int j = 0; j < kUnitTerms; ++j)
        partial[(int64_t)w * kMaxTerms + U.idx[j]] = j < U.uk ? acc[j] : acc[0];
}

// The first piece of each big cell adds the cell's pieces in order.
__global__ void __launch_bounds__(64)
k_mp_combine(const DevBox *__restrict__ boxes, const MpPiece *__restrict__ pieces,
             const uint32_t *__restrict__ total, const double *__restrict__ partial,
             int nterms) {
    const int w = blockIdx.x;
    if (w >= (int64_t)*total) return;
    const MpPiece pc = pieces[w];
    if (pc.k != 0) return;
    const DevBox &B = boxes[pc.box];
    for (int t = threadIdx.x; t < nterms; t += 64) {
        double sum = 0.0;
        for (int k = 0; k < pc.np && w + k < (int)gridDim.x; ++k)
            sum += partial[(int64_t)(w + k) * kMaxTerms + t];
        gp(B.out)[(int64_t)pc.cell * nterms + t] = (float)sum;
    }
}

}  // namespace

int multipole_max_order() { return kMaxOrder; }

int multipole_terms(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

int64_t multipole_ranges(int64_t n, int64_t ncell) {
    return (n + (int64_t)kCellCost * ncell) / kRange + 1;
}

int multipole_big() { return kBig; }

// Sum over big cells of ceil(n_c / kBig) <= n / kBig + (big cells) < 2 n / kBig.
int64_t multipole_max_pieces(int64_t n) { return 2 * (n / kBig) + 1; }

hipError_t multipole_launch(const DevBox *d_boxes, int nbox, const MpPlan &mp, int p,
                            hipStream_t s) {
    const dim3 cells((unsigned)((mp.max_ncell + 255) / 256), (unsigned)nbox);
    hipLaunchKernelGGL(k_mp_ranges, dim3((unsigned)((mp.max_ncell + 1 + 255) / 256), (unsigned)nbox),
                       dim3(256), 0, s, d_boxes, mp.range_base, mp.first);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // big cells: counts, offsets (the last entry becomes the total), pieces
    if ((e = fill_u32(mp.npieces, mp.C + 1, 0u, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_mp_count, cells, dim3(256), 0, s, d_boxes, mp.npieces);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = scan_exclusive(mp.npieces, mp.C + 1, mp.scan, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_mp_emit, cells, dim3(256), 0, s, d_boxes,
                       (const uint32_t *)mp.npieces, mp.pieces, mp.max_pieces);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_multipoles, dim3((unsigned)mp.max_ranges, (unsigned)nbox), dim3(64), 0, s,
                       d_boxes, mp.range_base, (const int32_t *)mp.first, p, multipole_terms(p));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const uint32_t *total = mp.npieces + mp.C;
    const unsigned gp = (unsigned)std::max<int64_t>(1, mp.max_pieces);
    hipLaunchKernelGGL(k_mp_pieces, dim3(gp), dim3(64), 0, s, d_boxes,
                       (const MpPiece *)mp.pieces, total, mp.partial, p);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_mp_combine, dim3(gp), dim3(64), 0, s, d_boxes,
                       (const MpPiece *)mp.pieces, total, (const double *)mp.partial,
                       multipole_terms(p));
    return hipGetLastError();
}

}  // namespace nf
