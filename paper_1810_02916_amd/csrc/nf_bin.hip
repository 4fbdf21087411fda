// nf_bin.hip -- binning of particles into the K^3 cell grid (Sec. 2.1):
// cell index + centre offset in double precision, then a stable sort by cell.
//
// All boxes of one call are binned together: box b's keys live in their own
// range [cellbase_b, cellbase_b + K_b^3) of one concatenated key space, so a
// single stable LSD radix sort over the concatenation of all boxes leaves
// every box's particles in its own slice, sorted by cell, ties in input order.
#include "nf_internal.h"
#include "nf_kernels.h"

namespace nf {

// ---------------------------------------------------------------- utilities

__global__ void k_fill_u32(uint32_t *p, int64_t count, uint32_t value) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = value;
}

// Zero each box's bad-particle counter.
__global__ void k_bin_zero_status(const DevBox *boxes, int nbox) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nbox && boxes[b].nbad) boxes[b].nbad[0] = 0;
}

// ------------------------------------------------------------- cell keys

// One thread per particle: linear cell id (in the box's key range), its
// concatenated element index, and its float offsets and z cell in caller
// order (the sort then moves 16 bytes per particle once, in k_bin_finish,
// instead of recomputing them from the double positions).
__global__ void __launch_bounds__(256) k_bin_keys(const DevBox *boxes, BinScratch sc) {
    const DevBox &B = boxes[blockIdx.y];
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= B.n) return;
    int c[3];
    float o[3];
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double od;
        ok &= cell_coord(B.pos[3 * (int64_t)i + a], B.kappa, B.K, c[a], od);
        o[a] = (float)od;
    }
    if (!ok) {
        c[0] = c[1] = c[2] = 0;
        o[0] = o[1] = o[2] = 0.0f;
        if (B.nbad) atomicAdd(B.nbad, 1);
    }
    uint32_t key = (uint32_t)B.cellbase + (uint32_t)((c[0] * B.K + c[1]) * B.K + c[2]);
    int64_t g = B.base + i;
    sc.keys[0][g] = key;
    sc.offc[g] = make_float4(o[0], o[1], o[2], (float)c[2]);
}

// ------------------------------------------------------------- radix sort

static_assert(kSortThreads == kScanThreads, "the sort's digit scan uses block_exclusive");

// Block-wide exclusive scan of 256 thread totals; returns this thread's prefix
// and the block total.
__device__ __forceinline__ uint32_t block_exclusive(uint32_t v, uint32_t &total) {
    __shared__ uint32_t wsum[kScanThreads / 64];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint32_t wpre = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < kScanThreads / 64; ++q) {
        uint32_t s = wsum[q];
        if (q < w) wpre += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return wpre + x - v;
}

// Per-tile digit histogram, written digit-major: hist[d * nblk + tile].  The
// count does not depend on the order within the tile, so a full tile is read
// with 16-byte loads.
template <int BITS>
__global__ void __launch_bounds__(kSortThreads)
k_radix_hist(const uint32_t *__restrict__ keys, int64_t N, int shift, int nblk,
             uint32_t *__restrict__ hist) {
    constexpr int R = 1 << BITS;
    __shared__ uint32_t cnt[R];
    const int t = threadIdx.x;
    for (int d = t; d < R; d += kSortThreads) cnt[d] = 0;
    __syncthreads();
    const int w = t >> 6, lane = t & 63;
    const int64_t base = (int64_t)blockIdx.x * kSortTile + w * (kSortTile / 4);
    auto count = [&](bool valid, uint32_t key) {
        uint32_t d = valid ? ((key >> shift) & (R - 1)) : 0u;
        uint64_t m = match_digit<BITS>(valid, d);
        if (valid && lane == 63 - __clzll(m)) atomicAdd(&cnt[d], (uint32_t)__popcll(m));
    };
    if ((int64_t)(blockIdx.x + 1) * kSortTile <= N) {
        const uint4 *k4 = reinterpret_cast<const uint4 *>(keys + base);
        uint4 q[kSortItems / 4];
#pragma unroll
        for (int k = 0; k < kSortItems / 4; ++k) q[k] = k4[k * 64 + lane];
#pragma unroll
        for (int k = 0; k < kSortItems / 4; ++k) {
            count(true, q[k].x);
            count(true, q[k].y);
            count(true, q[k].z);
            count(true, q[k].w);
        }
    } else {
        for (int k = 0; k < kSortItems; ++k) {
            int64_t idx = base + k * 64 + lane;
            bool valid = idx < N;
            count(valid, valid ? keys[idx] : 0u);
        }
    }
    __syncthreads();
    for (int d = t; d < R; d += kSortThreads) hist[(int64_t)d * nblk + blockIdx.x] = cnt[d];
}

// The tile of workgroup b when each of the 8 XCDs (workgroups are dealt to
// them round-robin by id) takes one contiguous range of the nb tiles.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int x = b % 8, j = b / 8, per = nb / 8, rem = nb % 8;
    return x * per + min(x, rem) + j;
}

// Stable scatter of one tile, workgroup b taking tile xcd_tile(b): the
// neighbouring output runs of a digit (consecutive tiles) then meet whole in
// one XCD's L2 instead of as line fragments in several.  Wave w owns the contiguous quarter
// [w*1024, (w+1)*1024) of the tile and walks it in rounds of 64, so
// "earlier round, then lower lane, then lower wave" is input order; that
// gives every key its rank within the tile's run of its digit.  The tile is
// then reordered by digit in LDS and written out slot by slot, so that the
// lanes of a wave store consecutive addresses of one output run.  The first
// pass (vals_in null) takes the element index as its value.
template <int BITS>
__global__ void __launch_bounds__(kSortThreads)
k_radix_scatter(const uint32_t *__restrict__ keys_in, const uint32_t *__restrict__ vals_in,
                uint32_t *__restrict__ keys_out, uint32_t *__restrict__ vals_out,
                int64_t N, int shift, int nblk, const uint32_t *__restrict__ hist_scan) {
    constexpr int R = 1 << BITS;
    constexpr int DPT = R / kSortThreads;   // digits per thread in the digit scan
    static_assert(R % kSortThreads == 0, "radix must be a multiple of the block size");
    __shared__ uint32_t gshift[R];        // output slot of the tile's local slot 0, per digit
    __shared__ uint32_t wcnt[4][R];
    __shared__ uint32_t skey[kSortTile];
    __shared__ uint32_t sval[kSortTile];
    const int t = threadIdx.x;
    const int w = t >> 6, lane = t & 63;
    for (int d = t; d < R; d += kSortThreads) {
#pragma unroll
        for (int q = 0; q < 4; ++q) wcnt[q][d] = 0;
    }
    __syncthreads();

    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int tile = xcd_tile((int)blockIdx.x, nblk);
    const int64_t tile0 = (int64_t)tile * kSortTile;
    const int64_t base = tile0 + w * (kSortTile / 4);
    uint32_t kk[kSortItems], vv[kSortItems], rk[kSortItems];
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        int64_t idx = base + k * 64 + lane;
        bool valid = idx < N;
        uint32_t key = valid ? keys_in[idx] : 0u;
        uint32_t val = valid ? (vals_in ? vals_in[idx] : (uint32_t)idx) : 0u;
        uint32_t d = (key >> shift) & (R - 1);
        uint64_t m = match_digit<BITS>(valid, d);
        uint32_t before = wcnt[w][d];
        __builtin_amdgcn_wave_barrier();
        rk[k] = before + (uint32_t)__popcll(m & below);
        if (valid && lane == 63 - __clzll(m)) wcnt[w][d] = before + (uint32_t)__popcll(m);
        __builtin_amdgcn_wave_barrier();
        kk[k] = key;
        vv[k] = val;
    }
    __syncthreads();
    {   // per digit: exclusive prefix over the waves, then over the digits
        uint32_t tot[DPT], sum = 0;
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            const int d = t * DPT + j;
            uint32_t s = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint32_t c = wcnt[q][d];
                wcnt[q][d] = s;
                s += c;
            }
            tot[j] = s;
            sum += s;
        }
        uint32_t all;
        uint32_t run = block_exclusive(sum, all);
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            const int d = t * DPT + j;
#pragma unroll
            for (int q = 0; q < 4; ++q) wcnt[q][d] += run;
            gshift[d] = hist_scan[(int64_t)d * nblk + tile] - run;
            run += tot[j];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        if (base + k * 64 + lane < N) {
            uint32_t d = (kk[k] >> shift) & (R - 1);
            uint32_t slot = wcnt[w][d] + rk[k];
            skey[slot] = kk[k];
            sval[slot] = vv[k];
        }
    }
    __syncthreads();
    const int cnt = (int)min<int64_t>(kSortTile, N - tile0);
    for (int j = t; j < cnt; j += kSortThreads) {
        const uint32_t key = skey[j];
        const uint32_t dst = gshift[(key >> shift) & (R - 1)] + (uint32_t)j;
        if (dst < (uint64_t)N) {   // always true for a consistent histogram
            keys_out[dst] = key;
            vals_out[dst] = sval[j];
        }
    }
}

// ------------------------------------------------------------- exclusive scan

// Per-tile sums.
__global__ void __launch_bounds__(kScanThreads)
k_scan_reduce(const uint32_t *__restrict__ in, int64_t M, uint32_t *__restrict__ sums) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        if (i < M) s += in[i];
    }
    uint32_t tot;
    block_exclusive(s, tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Exclusive scan of tile blockIdx.x plus `offset`.  In-place (in == out) is
// allowed.
__device__ __forceinline__ void scan_tile(const uint32_t *in, uint32_t *out, int64_t M,
                                          uint32_t offset) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        v[k] = (i < M) ? in[i] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t run = block_exclusive(s, tot) + offset;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        if (i < M) out[i] = run;
        run += v[k];
    }
}

// Exclusive scan of each tile plus the tile's scanned offset (offsets may be
// null for a single tile).
__global__ void __launch_bounds__(kScanThreads)
k_scan_down(const uint32_t *in, uint32_t *out, int64_t M, const uint32_t *__restrict__ offsets) {
    scan_tile(in, out, M, offsets ? offsets[blockIdx.x] : 0u);
}

// The same with unscanned tile sums: each block adds up the sums of the tiles
// before it (few enough that every block can: at most kScanTile tiles).
__global__ void __launch_bounds__(kScanThreads)
k_scan_down_sums(uint32_t *data, int64_t M, const uint32_t *__restrict__ sums) {
    uint32_t part = 0;
    for (int i = threadIdx.x; i < (int)blockIdx.x; i += kScanThreads) part += sums[i];
    uint32_t before;
    block_exclusive(part, before);
    scan_tile(data, data, M, before);
}

// ------------------------------------------------------------- cell starts

// first[k] = the first sorted slot whose key is >= k, for k = 0 .. C (the
// exclusive scan of the cell counts), from the sorted keys: slot s writes
// the keys in (key[s-1], key[s]], slot N the keys after the last one.  Keys
// are non-decreasing, so every k is written exactly once; no atomics.
__global__ void __launch_bounds__(256)
k_cell_first(const uint32_t *__restrict__ keys, int64_t N, int64_t C,
             uint32_t *__restrict__ first) {
    for (int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x; s <= N;
         s += (int64_t)gridDim.x * 256) {
        const int64_t lo = s == 0 ? 0 : (int64_t)keys[s - 1] + 1;
        const int64_t hi = s == N ? C : (int64_t)keys[s];
        for (int64_t k = lo; k <= hi; ++k) first[k] = (uint32_t)s;
    }
}

// ------------------------------------------------------------- finish

// Per box: cell_start from the first slots of its cells, order from the
// sorted element indices, and the float offsets gathered from caller order.
__global__ void __launch_bounds__(256)
k_bin_finish(const DevBox *boxes, const uint32_t *__restrict__ cellscan,
             const uint32_t *__restrict__ vals_sorted, const float4 *__restrict__ offc) {
    const DevBox &B = boxes[blockIdx.y];
    int t = blockIdx.x * 256 + threadIdx.x;
    if (t <= B.ncell) B.cell_start[t] = (int32_t)((int64_t)cellscan[B.cellbase + t] - B.base);
    if (t < B.n) {
        int64_t gi = (int64_t)vals_sorted[B.base + t] - B.base;
        int i = (gi >= 0 && gi < B.n) ? (int)gi : 0;   // always in range for a valid sort
        B.order[t] = i;
        B.off[t] = offc[B.base + i];
    }
}

// ------------------------------------------------------------- host driver

int64_t scan_scratch_words(int64_t M) {
    // words needed by scan_exclusive(M): the sums of each level, recursively
    int64_t words = 0;
    while (M > kScanTile) {
        int64_t nb = (M + kScanTile - 1) / kScanTile;
        words += nb;
        M = nb;
    }
    return words + 64;
}

hipError_t scan_exclusive(uint32_t *data, int64_t M, uint32_t *scratch, hipStream_t s) {
    if (M <= kScanTile) {
        hipLaunchKernelGGL(k_scan_down, dim3(1), dim3(kScanThreads), 0, s, data, data, M,
                           (const uint32_t *)nullptr);
        return hipGetLastError();
    }
    int64_t nb = (M + kScanTile - 1) / kScanTile;
    uint32_t *sums = scratch;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, M, sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (nb <= kScanTile) {   // two launches: each block adds up its predecessors
        hipLaunchKernelGGL(k_scan_down_sums, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data,
                           M, (const uint32_t *)sums);
        return hipGetLastError();
    }
    e = scan_exclusive(sums, nb, scratch + nb, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, data, M,
                       (const uint32_t *)sums);
    return hipGetLastError();
}

hipError_t fill_u32(uint32_t *p, int64_t count, uint32_t value, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<int64_t>(4096, (count + 255) / 256);
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(256), 0, s, p, count, value);
    return hipGetLastError();
}

template <int BITS>
static hipError_t sort_passes(const BinPlan &p, hipStream_t s) {
    hipError_t e;
    int src = 0;
    for (int pass = 0; pass < p.passes; ++pass) {
        const int shift = pass * BITS;
        hipLaunchKernelGGL(k_radix_hist<BITS>, dim3((unsigned)p.nblk), dim3(kSortThreads), 0, s,
                           p.sc.keys[src], p.N, shift, (int)p.nblk, p.sc.hist);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = scan_exclusive(p.sc.hist, (int64_t)(1 << BITS) * p.nblk, p.scan_scratch, s)) !=
            hipSuccess)
            return e;
        hipLaunchKernelGGL(k_radix_scatter<BITS>, dim3((unsigned)p.nblk), dim3(kSortThreads), 0, s,
                           p.sc.keys[src], pass == 0 ? (const uint32_t *)nullptr : p.sc.vals[src],
                           p.sc.keys[src ^ 1], p.sc.vals[src ^ 1], p.N, shift, (int)p.nblk,
                           p.sc.hist);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        src ^= 1;
    }
    return hipSuccess;
}

hipError_t bin_launch(const DevBox *d_boxes, int nbox, const BinPlan &p, hipStream_t s) {
    hipError_t e;
    hipLaunchKernelGGL(k_bin_zero_status, dim3((nbox + 255) / 256), dim3(256), 0, s, d_boxes, nbox);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (p.N > 0) {
        hipLaunchKernelGGL(k_bin_keys, dim3((unsigned)((p.max_n + 255) / 256), (unsigned)nbox),
                           dim3(256), 0, s, d_boxes, p.sc);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        e = p.radix_bits == 9 ? sort_passes<9>(p, s) : sort_passes<8>(p, s);
        if (e != hipSuccess) return e;
    }
    // with at least one pass the sorted arrays sit in buffer (passes & 1)
    const uint32_t *keys = p.sc.keys[p.passes & 1];
    const uint32_t *vals = p.sc.vals[p.passes & 1];
    const unsigned first_blocks =
        (unsigned)std::max<int64_t>(1, std::min<int64_t>(65535, (p.N + 1 + 255) / 256));
    hipLaunchKernelGGL(k_cell_first, dim3(first_blocks), dim3(256), 0, s, keys, p.N, p.C,
                       p.sc.cellcnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin_finish,
                       dim3((unsigned)((std::max<int64_t>(p.max_n, p.max_ncell + 1) + 255) / 256),
                            (unsigned)nbox),
                       dim3(256), 0, s, d_boxes, (const uint32_t *)p.sc.cellcnt, vals,
                       (const float4 *)p.sc.offc);
    return hipGetLastError();
}

}  // namespace nf
