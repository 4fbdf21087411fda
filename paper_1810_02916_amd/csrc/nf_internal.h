// nf_internal.h -- device-side descriptors and helpers shared by the HIP
// translation units of libnf.so (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nf {

// Global-address-space view of a device pointer.  Pointers read from a
// descriptor are generic, and generic (flat) loads and stores also count
// against the counter that LDS accesses and scalar loads wait on: a kernel
// that mixed them would wait for its global traffic at every such wait.
template <class T>
using gptr = __attribute__((address_space(1))) T *;
template <class T>
__device__ __forceinline__ gptr<T> gp(T *p) {
    return (gptr<T>)p;
}

// Radix sort geometry: 8-bit digits, 256 threads per block, 16 keys per thread.
// Tile defaults (an nf_box field of 0 picks these).
constexpr int kDefaultDenseMin = 41;      // nf_box.dense_min
constexpr int kDefaultNarrowMax = 12;     // nf_box.narrow_max
constexpr int kDefaultFlush = 32;         // nf_box.flush
constexpr int kDefaultLightWindow = 1024; // nf_box.light_window (512 / 1024 / 2048)
constexpr int kDefaultNarrowWindow = 256; // nf_box.narrow_window (128 / 256 / 512)
// Smallest float added to r^2 for Eq. 2: keeps rsq finite for coincident
// pairs, whose force is then min(poly, inf) * 0 = 0, and is far below half an
// ulp of any separation that floats resolve between offsets of order one.
constexpr float kR2Floor = 1.0e-30f;
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;   // 4096 keys per block

// Scan geometry: 256 threads x 16 items per block.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;   // 4096 values per block

// Per-box descriptor as the kernels see it.  Lives in the workspace and is
// written there by a small upload kernel (no host-to-device memcpy), so every
// launch stays capturable in a HIP graph.
struct DevBox {
    // geometry
    int32_t n;            // particles
    int32_t K;            // cells per side
    int32_t ncell;        // K^3
    int32_t plummer;      // 1: Plummer law for every pair (eps = eps_p), 0: Eq. 2
    int64_t base;         // first element of this box in the concatenated arrays
    int64_t cellbase;     // first key of this box in the concatenated key space
    double kappa;         // K / L (cells per length unit), double
    double cellw;         // L / K (cell width in length units), double
    float eps;            // spline radius in cell widths (eps_s * kappa)
    float scale;          // gm * kappa^2 (accel) or gm * kappa^3 (vjp)
    float cA, cB, cC;     // Eq. 2 in cell widths: F/r = cA + cB r + cC r^2 inside eps
                          // (10/eps^3, -15/eps^4, 6/eps^5, rounded from double)
    int32_t dense_min;    // a last chunk of at least this many sinks is dense
    int32_t narrow_max;   // a light item of fewer sinks is narrow
    int32_t flush;        // compensated mode: terms per plain partial sum
    int32_t outer_newton; // 1 when eps <= 1: every pair from the outer shell of
                          // the 5x5x5 block is at r >= 1 >= eps (Newton branch)
    float r2floor;        // added to r^2: 1e-30 for Eq. 2 (a coincident pair then
                          // gives 0), eps_p^2 for the Plummer law
    // caller buffers
    const double *pos;    // [n][3]
    float4 *off;          // [n] sorted offsets
    int32_t *cell_start;  // [K^3 + 1]
    int32_t *order;       // [n]
    int32_t *nbad;        // [1] or null
    float *out;           // acc or grad, [n][3], caller order
    const float *cot;     // [n][3] cotangent (vjp), caller order
    // pair symmetry (NF_PAIR_SYMMETRIC): per-call arrays over all boxes' cells
    // (index cellbase + cell), null when off
    const uint32_t *f4tot;   // [0] 1 when the plan fits (the path is on)
    const int32_t *f4P;      // partial sums per sink (0: not a symmetric cell)
    const int32_t *f4nf;     // partners of higher id
    const uint32_t *f4off;   // first partial slot of the cell
    float4 *f4part;          // partial sums, slot-major per cell
};
static_assert(sizeof(DevBox) % 8 == 0, "DevBox must stay 8-byte aligned");

// Cells whose pairs with each other are evaluated once (NF_PAIR_SYMMETRIC):
// 1 to kF4MaxChunks chunks of 64 sinks, every chunk summed by the dense
// kernel (the count is a multiple of 64 or its last chunk holds at least
// dense_min sinks).
constexpr int kF4MaxChunks = 16;
__device__ __forceinline__ bool f4_symmetric_cell(int n, int dense_min) {
    const int rem = n & 63;
    return n > 0 && n <= 64 * kF4MaxChunks && (rem == 0 || rem >= dense_min);
}

// The offset (x, y, z) and cz of sorted slot i through a global pointer.
__device__ __forceinline__ float4 ld_off4(const float4 *off, int64_t i) {
    const __attribute__((address_space(1))) float *q =
        (const __attribute__((address_space(1))) float *)off + 4 * i;
    return make_float4(q[0], q[1], q[2], q[3]);
}

// Element i of a float4 array through a global-address-space pointer.
typedef float nf_v4f __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void st_g4(float4 *base, uint64_t i, float x, float y, float z) {
    __attribute__((address_space(1))) nf_v4f *p =
        (__attribute__((address_space(1))) nf_v4f *)base + i;
    nf_v4f v = {x, y, z, 0.f};
    *p = v;
}
__device__ __forceinline__ nf_v4f ld_g4(const float4 *base, uint64_t i) {
    const __attribute__((address_space(1))) nf_v4f *p =
        (const __attribute__((address_space(1))) nf_v4f *)base + i;
    return *p;
}

// A symmetric pair item: chunk `chunk` of cell `cell` against every chunk of
// its partner in direction `dir` (rank `rank` among the cell's partners of
// higher id).
struct PairItem {
    int32_t box, cell, chunk, dir, rank, pad;
};

// One work item of the tiled force kernels: the sinks of cell `cell0` of
// box `box`, all of them when the cell holds at most 64 particles, else the
// 64 sinks starting at 64 * chunk.  m is always 1 (reserved).
struct Item {
    int32_t box, cell0, m, chunk;
};

// Global (all boxes) scratch used by the binning kernels.
struct BinScratch {
    uint32_t *keys[2];    // [N] concatenated keys (cellbase_b + cell id)
    uint32_t *vals[2];    // [N] concatenated element index (vals[0] unused: the
                          // first pass takes the identity)
    float4 *offc;         // [N] float offsets and z cell, concatenated caller order
    uint32_t *hist;       // [radix * nblk] digit-major block histograms
    uint32_t *cellcnt;    // [C + 1] first sorted slot of each concatenated cell key
};

// Cell of one coordinate, exactly as the method defines it: s = x * kappa
// (one rounding), c = floor(s) mod K, o = (s - floor(s)) - 1/2.  The
// sequence is evaluated without contraction so that host-side checks can
// reproduce the rounded offset bit for bit.  Returns false when s is not
// finite or |s| >= 2^62.
__device__ __forceinline__ bool cell_coord(double x, double kappa, int K, int &c, double &o) {
#pragma clang fp contract(off)
    double s = x * kappa;
    if (!(fabs(s) < 4.611686018427387904e18)) {   // also catches NaN
        c = 0;
        o = 0.0;
        return false;
    }
    double f = floor(s);
    double frac = s - f;
    o = frac - 0.5;
    long long fi = (long long)f;
    long long r = fi % (long long)K;
    if (r < 0) r += K;
    c = (int)r;
    return true;
}

// Wave-level "match any" on a BITS-bit digit: mask of the active lanes whose
// digit equals this lane's digit.
template <int BITS>
__device__ __forceinline__ uint64_t match_digit(bool valid, uint32_t d) {
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        bool bit = (d >> b) & 1u;
        uint64_t bb = __ballot(valid && bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

}  // namespace nf
