// nf_tile.hip -- tiled near-field kernels for gfx950: a device-side planner
// that cuts the cell grid into work items, and two persistent kernels that
// sum the pair forces of Eq. 2 (Sec. 4.3) over the 5x5x5 cell block of
// Sec. 2.1.
//
// The sinks of a cell are cut into chunks of 64.  Work items:
//   * dense  -- a full 64-sink chunk, or the last chunk when it holds at
//               least dense_min sinks (41 by default); one wave per item, one
//               sink per lane.  Every lane needs the same source at the same
//               time, so sources are read from the cell-sorted array with
//               scalar loads and enter the arithmetic as SGPR operands, and
//               the sink is shifted into each source cell's frame.  No LDS, so
//               many waves fit on a CU and hide the load latency.  Items run
//               heaviest neighbourhood first.
//   * light  -- a smaller last chunk (all sinks of a cell of fewer than
//               dense_min particles), one item per 4-wave workgroup.  The 125
//               source cells are staged in LDS in the sink cell's own frame,
//               (o_x + dx, o_y + dy, o_z + dz), the 27 cells with |d| <= 1
//               first, then the 98 outer cells, so the sum is two contiguous
//               segments; the g sinks are spread over the 256 threads as
//               (sink a, source slice b), thread = a + g b, P = 256 / g
//               slices, summed at the end by a fixed-order pairwise tree.
//   * narrow -- a light item of fewer than narrow_max sinks (12 by default):
//               the same kernel on one wave per workgroup (P = 64 / g), so the
//               per-item costs that do not shrink with g (item setup, the
//               per-wave header, the slice tree) are paid by one wave instead
//               of four.
// The class boundaries (dense_min, narrow_max), the staging windows of the
// light and narrow kernels and the compensated partial-sum length are tile
// choices of the caller (nf_box), picked by the autotuner.
// In both paths a source of the sink's own cell is used unshifted, so the
// closest pairs are formed from the exact float offsets, and a cell of the
// outer shell of the block (some |d| = 2) is at r >= 1 and takes the Newton
// branch directly when eps <= 1.  The Plummer law is the Newton branch with
// eps_p^2 as the floor on r^2, for every pair.
#include <climits>
#include <mutex>
#include <vector>

#include "nf_internal.h"
#include "nf_kernels.h"

namespace nf {

namespace {

constexpr int kUnit = 64;            // sinks per wave
constexpr int kQueues = 32;          // light-item queues (a multiple of the 8 XCDs)
constexpr int kXcds = 8;             // workgroups are dealt to the XCDs round-robin by id
constexpr int kXcdBlock = 256;       // consecutive light items kept on one XCD
constexpr int kDenseBlock = 16;      // consecutive dense items kept on one XCD
constexpr int kQueueStride = 32;     // words between queue counters (own 128-byte line)
constexpr int kLightWaves = 4;       // waves sharing one light item
constexpr int kLightThreads = 64 * kLightWaves;
constexpr int kNarrowThreads = 64;   // one wave per narrow item
constexpr int kRows = 25;            // (dx, dy) rows of the 5x5x5 block

__device__ __forceinline__ int wrapk(int c, int K) { return c < 0 ? c + K : (c >= K ? c - K : c); }
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Inclusive prefix sums over the lanes of a wave (all 64 lanes active): a
// Kogge-Stone scan inside each row of 16 lanes by DPP row shifts (one
// v_add_u32_dpp per step), then the row totals read back with readlane.
// scan_lanes<32> is exact on lanes 0..31 only.
template <int W>
__device__ __forceinline__ int scan_lanes(int x) {
    static_assert(W == 32 || W == 64, "one or two halves of the wave");
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);   // row_shr:8
    const int row = (threadIdx.x & 63) >> 4;
    const int t15 = __builtin_amdgcn_readlane(x, 15);
    if constexpr (W == 32) return x + ((row & 1) ? t15 : 0);
    const int t31 = __builtin_amdgcn_readlane(x, 31), t47 = __builtin_amdgcn_readlane(x, 47);
    return x + (row >= 1 ? t15 : 0) + (row >= 2 ? t31 : 0) + (row >= 3 ? t47 : 0);
}

// ------------------------------------------------------------------ planner

// Sources in the 5x5x5 block of cell (cx, cy, cz): 25 row ranges of 5 cells.
__device__ int block_sources(gptr<const int32_t> cs, int K, int cx, int cy, int cz) {
    int s = 0;
    for (int r = 0; r < kRows; ++r) {
        const int rb = (wrapk(cx + r / 5 - 2, K) * K + wrapk(cy + r % 5 - 2, K)) * K;
        const int lo = cz - 2, hi = cz + 2;
        if (lo < 0)
            s += (cs[rb + K] - cs[rb + lo + K]) + (cs[rb + hi + 1] - cs[rb]);
        else if (hi >= K)
            s += (cs[rb + K] - cs[rb + lo]) + (cs[rb + hi - K + 1] - cs[rb]);
        else
            s += cs[rb + hi + 1] - cs[rb + lo];
    }
    return s;
}

// Buckets, placed highest first: dense items by cost (quarter octaves of
// their block's source count S, heaviest first); light and narrow items by
// spatial slab (128 slabs of consecutive cells, in cell order).
constexpr int kBuckets = 128;
constexpr int kKinds = 3;                  // 0: dense, 1: light, 2: narrow
__device__ __forceinline__ int cost_bucket(float pairs) {
    const float l = __log2f(fmaxf(pairs, 1.0f));
    return min(kBuckets - 1, (int)(4.0f * l));
}

// Items of a cell of n particles: n / 64 full dense chunks, and the last
// n % 64 sinks as one more dense chunk if they are at least dense_min, else as
// one light item (a narrow one below narrow_max sinks).  cellinfo packs
// (dense bucket + 1) | (light bucket + 1) << 16, 0 for none; the item counts
// per (kind, bucket) are summed in LDS first so that each block adds one value
// per non-empty bucket.
struct CellItems {
    int ndense;     // dense chunks
    int light;      // kind of the remainder's item: 0 none, 1 light, 2 narrow
};
__device__ __forceinline__ CellItems cell_items(int n, int dense_min, int narrow_max) {
    const int full = n / kUnit, rem = n % kUnit;
    const int lk = (rem > 0 && rem < dense_min) ? (rem < narrow_max ? 2 : 1) : 0;
    return CellItems{full + (rem >= dense_min ? 1 : 0), lk};
}

__global__ void __launch_bounds__(256)
k_plan_count(const DevBox *boxes, uint32_t *cellinfo, uint32_t *bucket_cnt) {
    __shared__ uint32_t h[kKinds * kBuckets];
    for (int t = threadIdx.x; t < kKinds * kBuckets; t += 256) h[t] = 0;
    __syncthreads();
    const DevBox &B = boxes[blockIdx.y];
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c < B.ncell) {
        const gptr<const int32_t> cs = gp(B.cell_start);
        const int n = cs[c + 1] - cs[c];
        uint32_t info = 0;
        if (n > 0) {
            const CellItems it = cell_items(n, B.dense_min, B.narrow_max);
            if (it.ndense) {   // S (the block's sources) ranks dense items only
                const int K = B.K;
                const float S = (float)block_sources(cs, K, c / (K * K), (c / K) % K, c % K);
                const int b = cost_bucket(S);
                atomicAdd(&h[b], (uint32_t)it.ndense);
                info |= (uint32_t)(b + 1);
            }
            if (it.light) {
                // light items run in spatial order (slabs of consecutive cells):
                // neighbouring items share their staged sources in L2, and the
                // dense kernel, running alongside, absorbs the tail
                const int b = kBuckets - 1 - (int)((int64_t)c * kBuckets / B.ncell);
                atomicAdd(&h[it.light * kBuckets + b], 1u);
                info |= (uint32_t)(b + 1) << 16;
            }
        }
        cellinfo[B.cellbase + c] = info;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kKinds * kBuckets; t += 256)
        if (h[t]) atomicAdd(&bucket_cnt[t], h[t]);
}

// Bucket offsets per kind, heaviest bucket first; totals[kind] = item count.
__global__ void __launch_bounds__(kKinds * kBuckets)
k_plan_buckets(uint32_t *bucket_cnt, uint32_t *bucket_off, uint32_t *totals) {
    __shared__ uint32_t c[kKinds * kBuckets];
    const int t = threadIdx.x;
    const int kind = t / kBuckets, bk = t % kBuckets;
    c[t] = bucket_cnt[t];
    __syncthreads();
    uint32_t off = 0;
    for (int b = kBuckets - 1; b > bk; --b) off += c[kind * kBuckets + b];
    bucket_off[t] = off;
    bucket_cnt[t] = 0;   // reused as the fill cursor by k_plan_emit
    if (bk == 0) totals[kind] = off + c[t];
}

// Items into their bucket ranges: each block reserves one range per non-empty
// bucket with a global atomic and places its cells by LDS ranks.  The order
// inside a bucket depends on timing; every item's result does not.  Narrow
// items follow the light ones in the same array.
__global__ void __launch_bounds__(256)
k_plan_emit(const DevBox *boxes, const uint32_t *__restrict__ cellinfo,
            const uint32_t *__restrict__ bucket_off, const uint32_t *__restrict__ totals,
            uint32_t *bucket_cur, Item *dense, Item *light) {
    __shared__ uint32_t h[kKinds * kBuckets];
    __shared__ uint32_t base[kKinds * kBuckets];
    for (int t = threadIdx.x; t < kKinds * kBuckets; t += 256) h[t] = 0;
    __syncthreads();
    const DevBox &B = boxes[blockIdx.y];
    const int c = blockIdx.x * 256 + threadIdx.x;
    uint32_t info = 0, rd = 0, rl = 0;
    int n = 0, bd = 0, bl = 0;
    CellItems it{0, 0};
    if (c < B.ncell) {
        info = cellinfo[B.cellbase + c];
        if (info) {
            n = gp(B.cell_start)[c + 1] - gp(B.cell_start)[c];
            it = cell_items(n, B.dense_min, B.narrow_max);
            bd = (int)(info & 0xffffu) - 1;
            bl = (int)(info >> 16) - 1;
            if (it.ndense) rd = atomicAdd(&h[bd], (uint32_t)it.ndense);
            if (it.light) rl = atomicAdd(&h[it.light * kBuckets + bl], 1u);
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kKinds * kBuckets; t += 256)
        if (h[t]) base[t] = bucket_off[t] + atomicAdd(&bucket_cur[t], h[t]);
    __syncthreads();
    if (it.ndense) {
        const uint32_t at = base[bd] + rd;
        for (int k = 0; k < it.ndense; ++k) dense[at + k] = Item{(int)blockIdx.y, c, 1, k};
    }
    if (it.light) {
        const uint32_t at = (it.light == 2 ? totals[1] : 0u) + base[it.light * kBuckets + bl] + rl;
        light[at] = Item{(int)blockIdx.y, c, 1, n / kUnit};
    }
}

// ------------------------------------------------------------------ pair arithmetic

struct Acc {
    float x = 0.f, y = 0.f, z = 0.f;
    float cx = 0.f, cy = 0.f, cz = 0.f;   // Kahan compensation (negated low parts)
};

__device__ __forceinline__ void kahan(float &s, float &c, float v) {
    const float y = v - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

template <bool COMP>
__device__ __forceinline__ void fold(Acc &a, float px, float py, float pz) {
    if constexpr (COMP) {
        kahan(a.x, a.cx, px);
        kahan(a.y, a.cy, py);
        kahan(a.z, a.cz, pz);
    } else {
        a.x += px;
        a.y += py;
        a.z += pz;
    }
}

struct Coef {
    float cA, cB, cC, cC2, eps2;
    float floor;   // added to r^2 (DevBox::r2floor)
};

// One pair of the acceleration sum; SPLINE selects Eq. 2's single-min form,
// otherwise the pair is known to lie outside eps (Newton branch).  Outside
// eps the spline lies above r^-3 (their difference is 10 (r/eps - 1)^3 in
// units of eps^-3), so the min form is evaluated only when some lane of the
// wave has r^2 < eps^2, which few pairs do: a compare per pair instead of
// the polynomial and the min.  (The empty volatile asm keeps the rare branch
// a branch instead of letting the compiler evaluate both sides.)
template <bool SPLINE>
__device__ __forceinline__ void pair_accel(float sx, float sy, float sz, float xi, float yi,
                                           float zi, const Coef &k, float &px, float &py,
                                           float &pz) {
    const float rx = sx - xi, ry = sy - yi, rz = sz - zi;
    float r2 = __builtin_fmaf(rx, rx, k.floor);
    r2 = __builtin_fmaf(ry, ry, r2);
    r2 = __builtin_fmaf(rz, rz, r2);
    const float q = __builtin_amdgcn_rsqf(r2);
    float f = q * q * q;
    if constexpr (SPLINE) {
        const bool in = r2 < k.eps2;
        if (__any(in)) {
            asm volatile("");
            const float rho = r2 * q;
            const float g = fminf(__builtin_fmaf(__builtin_fmaf(k.cC, rho, k.cB), rho, k.cA), f);
            f = in ? g : f;
        }
    }
    px = __builtin_fmaf(f, rx, px);
    py = __builtin_fmaf(f, ry, py);
    pz = __builtin_fmaf(f, rz, pz);
}

// Four pairs of the acceleration sum with the sources' offsets in sx, sy,
// sz, added in order; the spline's branch is taken once for the four.
template <bool SPLINE>
__device__ __forceinline__ void pair_accel4(const float (&sx)[4], const float (&sy)[4],
                                            const float (&sz)[4], float xi, float yi, float zi,
                                            const Coef &k, float &px, float &py, float &pz) {
    float rx[4], ry[4], rz[4], r2[4], q[4], f[4];
    bool in = false;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        rx[u] = sx[u] - xi;
        ry[u] = sy[u] - yi;
        rz[u] = sz[u] - zi;
        r2[u] = __builtin_fmaf(rx[u], rx[u], k.floor);
        r2[u] = __builtin_fmaf(ry[u], ry[u], r2[u]);
        r2[u] = __builtin_fmaf(rz[u], rz[u], r2[u]);
        q[u] = __builtin_amdgcn_rsqf(r2[u]);
        f[u] = q[u] * q[u] * q[u];
        if constexpr (SPLINE) in |= r2[u] < k.eps2;
    }
    if constexpr (SPLINE) {
        if (__any(in)) {
            asm volatile("");
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float rho = r2[u] * q[u];
                const float g =
                    fminf(__builtin_fmaf(__builtin_fmaf(k.cC, rho, k.cB), rho, k.cA), f[u]);
                f[u] = r2[u] < k.eps2 ? g : f[u];
            }
        }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        px = __builtin_fmaf(f[u], rx[u], px);
        py = __builtin_fmaf(f[u], ry[u], py);
        pz = __builtin_fmaf(f[u], rz[u], pz);
    }
}

// N pairs of the VJP, added in order: xbar_i += g (v_j - v_i) + h (r .
// (v_j - v_i)) r, with g = F/r and h = g'(rho)/rho, written as
// xbar_i += A (u + W r) with u = v_j - v_i, A = g and W = h (r . u) / g.
// Outside eps (Newton, or Plummer through the r^2 floor) A = q^3 and
// W = -3 q^2 (r . u): 23 VALU.  Inside eps g = cA + cB rho + cC rho^2 > 0 and
// h = cB / rho + 2 cC = cB q + 2 cC.  With SPLINE the inside coefficients
// replace the Newton ones only when some lane of the wave has one of the N
// pairs inside eps (a compare per pair otherwise), as in pair_accel; the
// branch rewrites A and W only, so the sums are updated outside it.
template <bool SPLINE, int N>
__device__ __forceinline__ void pair_vjpN(const float (&sx)[N], const float (&sy)[N],
                                          const float (&sz)[N], const float (&vx)[N],
                                          const float (&vy)[N], const float (&vz)[N], float xi,
                                          float yi, float zi, float vxi, float vyi, float vzi,
                                          const Coef &k, float &px, float &py, float &pz) {
    float rx[N], ry[N], rz[N], ux[N], uy[N], uz[N], r2[N], q[N], rdu[N], A[N], W[N];
    bool in = false;
#pragma unroll
    for (int u = 0; u < N; ++u) {
        rx[u] = sx[u] - xi;
        ry[u] = sy[u] - yi;
        rz[u] = sz[u] - zi;
        ux[u] = vx[u] - vxi;
        uy[u] = vy[u] - vyi;
        uz[u] = vz[u] - vzi;
        r2[u] = __builtin_fmaf(rx[u], rx[u], k.floor);
        r2[u] = __builtin_fmaf(ry[u], ry[u], r2[u]);
        r2[u] = __builtin_fmaf(rz[u], rz[u], r2[u]);
        q[u] = __builtin_amdgcn_rsqf(r2[u]);
        rdu[u] = rx[u] * ux[u];
        rdu[u] = __builtin_fmaf(ry[u], uy[u], rdu[u]);
        rdu[u] = __builtin_fmaf(rz[u], uz[u], rdu[u]);
        const float q2 = q[u] * q[u];
        A[u] = q2 * q[u];
        W[u] = (-3.0f * q2) * rdu[u];
        if constexpr (SPLINE) in |= r2[u] < k.eps2;
    }
    if constexpr (SPLINE) {
        if (__any(in)) {
            asm volatile("");   // keep the rare branch a branch
#pragma unroll
            for (int u = 0; u < N; ++u) {
                const float rho = r2[u] * q[u];
                const float g = __builtin_fmaf(__builtin_fmaf(k.cC, rho, k.cB), rho, k.cA);
                const float h = __builtin_fmaf(k.cB, q[u], k.cC2);
                const bool inside = r2[u] < k.eps2;
                A[u] = inside ? g : A[u];
                W[u] = inside ? (h * rdu[u]) / g : W[u];
            }
        }
    }
#pragma unroll
    for (int u = 0; u < N; ++u) {
        px = __builtin_fmaf(A[u], __builtin_fmaf(W[u], rx[u], ux[u]), px);
        py = __builtin_fmaf(A[u], __builtin_fmaf(W[u], ry[u], uy[u]), py);
        pz = __builtin_fmaf(A[u], __builtin_fmaf(W[u], rz[u], uz[u]), pz);
    }
}

template <bool SPLINE>
__device__ __forceinline__ void pair_vjp(float sx, float sy, float sz, float vx, float vy,
                                         float vz, float xi, float yi, float zi, float vxi,
                                         float vyi, float vzi, const Coef &k, float &px,
                                         float &py, float &pz) {
    const float ax[1] = {sx}, ay[1] = {sy}, az[1] = {sz}, bx[1] = {vx}, by[1] = {vy},
                bz[1] = {vz};
    pair_vjpN<SPLINE, 1>(ax, ay, az, bx, by, bz, xi, yi, zi, vxi, vyi, vzi, k, px, py, pz);
}

// Final value of a lane's sum (compensation folded in).
template <bool COMP>
__device__ __forceinline__ float3 value(const Acc &a) {
    if constexpr (COMP) return make_float3(a.x - a.cx, a.y - a.cy, a.z - a.cz);
    return make_float3(a.x, a.y, a.z);
}

// Scaled result of sorted slot `slot` to caller index i = order[slot] (read
// by the caller early, so that its latency hides behind the sum).
__device__ __forceinline__ void store(const DevBox &B, int i, float3 f) {
    if (i >= 0 && i < B.n) {   // always true for a consistent binning
        gptr<float> o = gp(B.out) + 3 * (int64_t)i;
        o[0] = f.x * B.scale;
        o[1] = f.y * B.scale;
        o[2] = f.z * B.scale;
    }
}

// ------------------------------------------------------------------ dense path

typedef const __attribute__((address_space(4))) float cfloat;
typedef float rec8 __attribute__((ext_vector_type(8)));
typedef const __attribute__((address_space(4))) rec8 crec8;
typedef const __attribute__((address_space(1))) float gfloat;

// Float4 number i of a global array through a global-address-space pointer
// (plain pointers loaded from a descriptor compile to flat loads).  The index
// is 64-bit: VJP records are addressed by 2 (base + slot), which exceeds 2^31
// once the boxes of a call hold more than 2^30 particles.
__device__ __forceinline__ float4 ld_global4(gfloat *p, int64_t i) {
    gfloat *q = p + 4 * i;
    return make_float4(q[0], q[1], q[2], q[3]);
}

// Sources [j0, j1) of one cell through scalar loads.
template <int MODE, bool SPLINE, bool COMP>
__device__ __forceinline__ void run_scalar(cfloat *__restrict__ src, cfloat *__restrict__ cot,
                                           int j0, int j1, float xs, float ys, float zs,
                                           float4 vi, const Coef &k, int flush, Acc &acc) {
    // the block's first source through a 64-bit address (4 j0 passes 2^31 for
    // j0 >= 2^29); inside a block (at most 256 sources) 32-bit offsets
    constexpr int W = MODE == 0 ? 4 : 8;   // floats per source
    cfloat *p = src + (int64_t)W * j0;
    int j = j0;
    while (j < j1) {
        // compensated: plain partials of at most flush terms; plain: one run
        const int blk = COMP ? min(j1 - j, flush) : j1 - j;
        float px = 0.f, py = 0.f, pz = 0.f;
        if constexpr (!COMP) {
            px = acc.x;
            py = acc.y;
            pz = acc.z;
        }
        if constexpr (MODE == 0) {
            int t = 0;
            for (; t + 4 <= blk; t += 4) {
                float ax[4], ay[4], az[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    ax[u] = p[4 * (t + u)];
                    ay[u] = p[4 * (t + u) + 1];
                    az[u] = p[4 * (t + u) + 2];
                }
                pair_accel4<SPLINE>(ax, ay, az, xs, ys, zs, k, px, py, pz);
            }
            for (; t < blk; ++t)
                pair_accel<SPLINE>(p[4 * t], p[4 * t + 1], p[4 * t + 2], xs, ys, zs, k, px, py,
                                   pz);
        } else {
            // one 32-byte record per source (offset, cotangent), one scalar load
            int t = 0;
            for (; t + 2 <= blk; t += 2) {
                float ax[2], ay[2], az[2], bx[2], by[2], bz[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const rec8 r8 = ((crec8 *)p)[t + u];
                    ax[u] = r8[0];
                    ay[u] = r8[1];
                    az[u] = r8[2];
                    bx[u] = r8[4];
                    by[u] = r8[5];
                    bz[u] = r8[6];
                }
                pair_vjpN<SPLINE, 2>(ax, ay, az, bx, by, bz, xs, ys, zs, vi.x, vi.y, vi.z, k, px,
                                     py, pz);
            }
            for (; t < blk; ++t) {
                const rec8 r8 = ((crec8 *)p)[t];
                pair_vjp<SPLINE>(r8[0], r8[1], r8[2], r8[4], r8[5], r8[6], xs, ys, zs, vi.x,
                                 vi.y, vi.z, k, px, py, pz);
            }
        }
        p += W * blk;
        j += blk;
        if constexpr (COMP) {
            fold<true>(acc, px, py, pz);
        } else {
            acc.x = px;
            acc.y = py;
            acc.z = pz;
        }
    }
}

template <int MODE, bool COMP>
__global__ void __launch_bounds__(kUnit)
k_dense(const DevBox *__restrict__ boxes, const Item *__restrict__ items,
        const uint32_t *__restrict__ totals, uint32_t *counter,
        const float4 *__restrict__ cot_sorted) {
    __shared__ int s_item;
    const int lane = threadIdx.x;
    const int nitems = (int)totals[0];
    // one queue per XCD (workgroup w runs on XCD w % 8): XCD x takes the
    // blocks of kDenseBlock consecutive items c = x, x + 8, ... in order, so
    // the chunks of one cell, which share every source, meet in one L2, and
    // the heaviest items still come first everywhere (the map is one-to-one
    // and increasing, so only the locality depends on the placement)
    const int x = (int)(blockIdx.x % kXcds);
    uint32_t *dq = counter + kQueueStride * x;
    for (;;) {
        if (lane == 0) {
            const int t = (int)__hip_atomic_fetch_add(gp(dq), 1u, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
            s_item = ((t / kDenseBlock) * kXcds + x) * kDenseBlock + t % kDenseBlock;
        }
        __syncthreads();
        const int itx = uni(s_item);
        __syncthreads();
        if (itx >= nitems) break;
        const gptr<const Item> ip = gp(items) + itx;
        const Item I{ip->box, ip->cell0, ip->m, ip->chunk};
        const DevBox &B = boxes[I.box];
        const int K = B.K;
        const int cx = I.cell0 / (K * K), cy = (I.cell0 / K) % K, z = I.cell0 % K;
        const gptr<const int32_t> cs = gp(B.cell_start);
        const int s0 = uni(cs[I.cell0] + kUnit * I.chunk);
        const int g = uni(min(cs[I.cell0 + 1] - s0, kUnit));
        // Lanes beyond the g sinks repeat sink 0 and are dropped at the store:
        // the loop below stays convergent, so every lane holds its row's cell
        // ranges when they are read back with readlane.
        const bool active = lane < g;
        const int slot = s0 + (active ? lane : 0);
        const float4 oi = ld_global4((gfloat *)B.off, slot);
        const int dst = gp(B.order)[slot];
        float4 vi = make_float4(0.f, 0.f, 0.f, 0.f);
        if constexpr (MODE == 1) vi = ld_global4((gfloat *)cot_sorted, 2 * (B.base + slot) + 1);
        const Coef k{B.cA, B.cB, B.cC, 2.0f * B.cC, B.eps * B.eps, B.r2floor};
        const bool fast = B.outer_newton != 0;
        const bool plummer = B.plummer != 0;   // Plummer law: one branch for every pair
        const int flush = uni(B.flush);
        // pair symmetry: the sinks of a symmetric cell skip the sources of
        // their symmetric partner cells (summed once by the pair kernel) and
        // leave their sum in partial slot 0
        const int nX = uni(cs[I.cell0 + 1] - cs[I.cell0]);
        const bool f4sink = MODE == 0 && B.f4tot != nullptr && uni((int)gp(B.f4tot)[0]) != 0 &&
                            f4_symmetric_cell(nX, B.dense_min);
        cfloat *src = (cfloat *)B.off;
        // the VJP reads sources from the 32-byte records (offset, cotangent)
        cfloat *cot = (cfloat *)(cot_sorted + 2 * B.base);
        if constexpr (MODE == 1) src = cot;
        // cell ranges of the 125 source cells: lane r < 25 holds row r's five
        // (start, end) pairs, read back with readlane (uniform, no memory wait)
        int cb[5], ce[5];
        {
            const int r = lane < kRows ? lane : 0;
            const int rb = (wrapk(cx + r / 5 - 2, K) * K + wrapk(cy + r % 5 - 2, K)) * K;
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                const int c = rb + wrapk(z + q - 2, K);
                cb[q] = cs[c];
                ce[q] = cs[c + 1];
            }
        }
        Acc acc;
        {
            for (int r = 0; r < kRows; ++r) {
                const int dx = r / 5 - 2, dy = r % 5 - 2;
                const bool in_row = dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1;
                const float xs = oi.x - (float)dx, ys = oi.y - (float)dy;
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    const int dz = q - 2;
                    const int cbq = __builtin_amdgcn_readlane(cb[q], r);
                    const int ceq = __builtin_amdgcn_readlane(ce[q], r);
                    const int j0 = max(cbq, 0);
                    const int j1 = min(ceq, B.n);
                    if (j0 >= j1) continue;
                    if (f4sink && !(r == 12 && q == 2) && f4_symmetric_cell(ceq - cbq, B.dense_min))
                        continue;
                    const float zs = oi.z - (float)dz;
                    if (!plummer && (!fast || (in_row && dz >= -1 && dz <= 1)))
                        run_scalar<MODE, true, COMP>(src, cot, j0, j1, xs, ys, zs, vi, k, flush,
                                                     acc);
                    else
                        run_scalar<MODE, false, COMP>(src, cot, j0, j1, xs, ys, zs, vi, k, flush,
                                                      acc);
                }
            }
        }
        if (f4sink) {
            if (active) {
                const int64_t gX = B.cellbase + I.cell0;
                const uint64_t idx = (uint64_t)gp(B.f4off)[gX] + (uint64_t)(kUnit * I.chunk + lane);
                if constexpr (COMP) {
                    st_g4(B.f4part, 2 * idx, acc.x, acc.y, acc.z);
                    st_g4(B.f4part, 2 * idx + 1, -acc.cx, -acc.cy, -acc.cz);
                } else {
                    st_g4(B.f4part, idx, acc.x, acc.y, acc.z);
                }
            }
        } else if (active) {
            store(B, dst, value<COMP>(acc));
        }
    }
}

// ------------------------------------------------------------------ light path

// Pieces of the staged union: per row r = (dx+2)*5 + (dy+2) up to four
// contiguous global ranges.  Slots 0-1: the |dz| <= 1 part of an inner row
// (|dx|, |dy| <= 1); slots 2-3: the rest of the row (dz = -2 and +2 for an
// inner row, dz = -2..2 split at the periodic wrap for an outer row).
constexpr int kSlots = 4;
constexpr int kPiece = kRows * kSlots;

template <int MODE, int CAP, int NT>
struct LightSmem {
    union {
        float4 sx[CAP];                  // (o_x + dx, o_y + dy, o_z + dz, v_x)
        float red[6][NT];                // after the sum: slice partials (sum, compensation)
    };
    float2 sv[MODE == 1 ? CAP : 1];  // (v_y, v_z) for the VJP
    int rs[128];                     // staged start of each non-empty piece (run), ascending,
                                     // then INT_MAX
    float4 rd[kPiece];               // per run: (global minus staged index, dx, dy, z bias)
    uint32_t bm[CAP / 32];           // staging window: bit e set when a run starts at u0 + e
    int cum[CAP / 32];               // runs starting before word w of the window
    int item;                        // current item and its (box, cell)
    int ibox, icell, ichunk;
    int inner;                       // staged particles of the 27 inner cells
    int total;
};

// Sum over staged sources [lo, hi) for one lane's sink, the lane taking
// indices lo + b, lo + b + P, ...
template <int MODE, bool SPLINE, bool COMP>
__device__ __forceinline__ void segment(const float4 *__restrict__ sx, const float2 *__restrict__ sv,
                                        int lo, int hi, int b, int P, float xi, float yi,
                                        float zi, float4 vi, const Coef &k, int flush, Acc &acc) {
    const int n = hi - lo;
    const int nfull = n / P;
    int j = lo + b;
    int it = 0;
    while (it < nfull) {
        // compensated: plain partials of at most flush terms; plain: one run
        const int blk = COMP ? min(nfull - it, flush) : nfull - it;
        float px = 0.f, py = 0.f, pz = 0.f;
        if constexpr (!COMP) {
            px = acc.x;
            py = acc.y;
            pz = acc.z;
        }
        if constexpr (MODE == 0) {
            int t = 0;
            for (; t + 4 <= blk; t += 4) {
                float ax[4], ay[4], az[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const float4 s = sx[j + u * P];
                    ax[u] = s.x;
                    ay[u] = s.y;
                    az[u] = s.z;
                }
                pair_accel4<SPLINE>(ax, ay, az, xi, yi, zi, k, px, py, pz);
                j += 4 * P;
            }
            for (; t < blk; ++t) {
                const float4 s = sx[j];
                pair_accel<SPLINE>(s.x, s.y, s.z, xi, yi, zi, k, px, py, pz);
                j += P;
            }
        } else {
            int t = 0;
            for (; t + 2 <= blk; t += 2) {
                float ax[2], ay[2], az[2], bx[2], by[2], bz[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const float4 s = sx[j + u * P];
                    const float2 v = sv[j + u * P];
                    ax[u] = s.x;
                    ay[u] = s.y;
                    az[u] = s.z;
                    bx[u] = s.w;
                    by[u] = v.x;
                    bz[u] = v.y;
                }
                pair_vjpN<SPLINE, 2>(ax, ay, az, bx, by, bz, xi, yi, zi, vi.x, vi.y, vi.z, k, px,
                                     py, pz);
                j += 2 * P;
            }
            for (; t < blk; ++t) {
                const float4 s = sx[j];
                const float2 v = sv[j];
                pair_vjp<SPLINE>(s.x, s.y, s.z, s.w, v.x, v.y, xi, yi, zi, vi.x, vi.y, vi.z, k,
                                 px, py, pz);
                j += P;
            }
        }
        it += blk;
        if constexpr (COMP) {
            fold<true>(acc, px, py, pz);
        } else {
            acc.x = px;
            acc.y = py;
            acc.z = pz;
        }
    }
    if (b < n - nfull * P) {
        float px = 0.f, py = 0.f, pz = 0.f;
        const float4 s = sx[j];
        if constexpr (MODE == 0) {
            pair_accel<SPLINE>(s.x, s.y, s.z, xi, yi, zi, k, px, py, pz);
        } else {
            const float2 v = sv[j];
            pair_vjp<SPLINE>(s.x, s.y, s.z, s.w, v.x, v.y, xi, yi, zi, vi.x, vi.y, vi.z, k, px,
                             py, pz);
        }
        fold<COMP>(acc, px, py, pz);
    }
}

// NT threads share one item (256 for light items, 64 for narrow ones); cls
// selects the item class: 1 light (items from the start of the array), 2
// narrow (after the light ones).
template <int MODE, bool COMP, int CAP, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(MODE == 0 ? 8 : 7)))
k_light(const DevBox *__restrict__ boxes, const Item *__restrict__ all_items,
        const uint32_t *__restrict__ totals, uint32_t *counter,
        const float4 *__restrict__ cot_sorted, int cls) {
    static_assert(CAP % NT == 0, "a staging window is whole rounds of the workgroup");
    static_assert(NT % 64 == 0 && NT <= kLightThreads, "whole waves");
    __shared__ LightSmem<MODE, CAP, NT> sm;
    const int lane = threadIdx.x;   // 0 .. NT-1, all waves share the item
    const int nitems = (int)totals[cls];
    const gptr<const Item> items = gp(all_items) + (cls == 2 ? totals[1] : 0u);

    // kQueues interleaved queues: workgroup w draws from queue q = w % kQueues
    // (a single counter would cap the item rate at what one address sustains
    // for atomics).  The workgroups of queue q run on XCD q % 8, and the
    // queues of one XCD share blocks of kXcdBlock consecutive items (items
    // are in spatial order, so neighbours share their sources in that XCD's
    // L2): XCD x takes the blocks c = x, x + 8, ..., its four queues taking
    // its items in turn.  (q, k) -> item is one-to-one and increasing in k,
    // so the results do not depend on where the workgroups actually run;
    // only the L2 locality does.
    const int q = (int)(blockIdx.x % kQueues);
    uint32_t *qc = counter + kQueueStride * q;
    auto queue_item = [q](int kth) {
        const int t = kth * (kQueues / kXcds) + q / kXcds;   // the XCD's t-th item
        return ((t / kXcdBlock) * kXcds + q % kXcds) * kXcdBlock + t % kXcdBlock;
    };
    if (lane == 0) {
        const int first = queue_item((int)__hip_atomic_fetch_add(gp(qc), 1u, __ATOMIC_RELAXED,
                                                                 __HIP_MEMORY_SCOPE_AGENT));
        sm.item = first;
        if (first < nitems) {
            sm.ibox = items[first].box;
            sm.icell = items[first].cell0;
            sm.ichunk = items[first].chunk;
        }
    }
    for (;;) {
        __syncthreads();
        const int itx = uni(sm.item);
        if (itx >= nitems) break;
        const int ibox = uni(sm.ibox), cell0 = uni(sm.icell), chunk = uni(sm.ichunk);
        // claim the next item now (lane 0); its record is fetched once the setup
        // below is done, and both complete while this item runs
        int nxt = 0;
        if (lane == 0)
            nxt = queue_item((int)__hip_atomic_fetch_add(gp(qc), 1u, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT));
        const DevBox &B = boxes[ibox];
        const int K = B.K;
        const int cx = cell0 / (K * K), cy = (cell0 / K) % K, z = cell0 % K;
        const gptr<const int32_t> cs = gp(B.cell_start);
        gfloat *goff = (gfloat *)B.off;
        gfloat *gcot = (gfloat *)cot_sorted;
        const int s0 = uni(cs[cell0]) + kUnit * chunk;
        const int g = min(uni(cs[cell0 + 1]) - s0, kUnit);

        // ---- this lane's sink (sink a, source slice b), loaded before the setup
        const Coef k{B.cA, B.cB, B.cC, 2.0f * B.cC, B.eps * B.eps, B.r2floor};
        const bool fast = B.outer_newton != 0;
        const int flush = uni(B.flush);
        const int P = NT / g;
        const bool active = lane < g * P;
        const int a = active ? lane % g : 0;
        const int b = active ? lane / g : 0;
        const float4 oi = ld_global4((gfloat *)B.off, s0 + a);
        const int dst = lane < g ? gp(B.order)[s0 + lane] : 0;   // lane < g stores sink lane
        float4 vi = make_float4(0.f, 0.f, 0.f, 0.f);
        if constexpr (MODE == 1) vi = ld_global4((gfloat *)cot_sorted, 2 * (B.base + s0 + a) + 1);

        // ---- pieces and run table: wave 0, one lane per row.  Staged layout: the
        //      inner parts of rows 0..24, then their outer parts; the non-empty
        //      pieces in that order are the runs.
        if (lane < 64) {
            const int r = lane;
            int pg[kSlots] = {0, 0, 0, 0}, pn[kSlots] = {0, 0, 0, 0};
            float pb[kSlots] = {0.f, 0.f, 0.f, 0.f};
            if (r < kRows) {
                const int dx = r / 5 - 2, dy = r % 5 - 2;
                const bool in_row = dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1;
                const int rb = (wrapk(cx + dx, K) * K + wrapk(cy + dy, K)) * K;
                // a run of z cells [za, zb] relative to the sink (za <= zb), split at the wrap
                auto run = [&](int q, int za, int zb) {
                    const int lo = z + za, hi = z + zb;
                    if (lo < 0) {   // [lo+K, K-1] then [0, hi]
                        pg[q] = cs[rb + lo + K];
                        pn[q] = cs[rb + K] - pg[q];
                        pb[q] = -(float)(z + K);
                        pg[q + 1] = cs[rb];
                        pn[q + 1] = cs[rb + hi + 1] - pg[q + 1];
                        pb[q + 1] = -(float)z;
                    } else if (hi >= K) {   // [lo, K-1] then [0, hi-K]
                        pg[q] = cs[rb + lo];
                        pn[q] = cs[rb + K] - pg[q];
                        pb[q] = -(float)z;
                        pg[q + 1] = cs[rb];
                        pn[q + 1] = cs[rb + hi - K + 1] - pg[q + 1];
                        pb[q + 1] = (float)(K - z);
                    } else {
                        pg[q] = cs[rb + lo];
                        pn[q] = cs[rb + hi + 1] - pg[q];
                        pb[q] = -(float)z;
                    }
                };
                if (in_row) {
                    run(0, -1, 1);
                    // the two single cells at dz = -2 and dz = +2
                    const int zm = z - 2, zp = z + 2;
                    const int cm = rb + wrapk(zm, K), cp = rb + wrapk(zp, K);
                    pg[2] = cs[cm];
                    pn[2] = cs[cm + 1] - pg[2];
                    pb[2] = -(float)z + (zm < 0 ? -(float)K : 0.f);
                    pg[3] = cs[cp];
                    pn[3] = cs[cp + 1] - pg[3];
                    pb[3] = -(float)z + (zp >= K ? (float)K : 0.f);
                } else {
                    run(2, -2, 2);
                }
            }
            // exclusive prefixes over rows of the inner and outer counts and of
            // the non-empty piece counts (inner | outer << 16), by a wave scan
            const int ca = pn[0] + pn[1], ce = pn[2] + pn[3];
            const int cn = ((pn[0] > 0) + (pn[1] > 0)) | (((pn[2] > 0) + (pn[3] > 0)) << 16);
            static_assert(kRows <= 32, "the row scans use lanes 0..31");
            const int ia = scan_lanes<32>(ca), ie = scan_lanes<32>(ce), in_ = scan_lanes<32>(cn);
            const int tin = __builtin_amdgcn_readlane(ia, kRows - 1);
            const int tout = __builtin_amdgcn_readlane(ie, kRows - 1);
            const int tn = __builtin_amdgcn_readlane(in_, kRows - 1);
            const int kin = tn & 0xffff, kout = tn >> 16;
            if (r < kRows) {
                const int n0 = in_ - cn;
                int start[kSlots], rank[kSlots];
                start[0] = ia - ca;
                start[1] = start[0] + pn[0];
                start[2] = tin + (ie - ce);
                start[3] = start[2] + pn[2];
                rank[0] = n0 & 0xffff;
                rank[1] = rank[0] + (pn[0] > 0);
                rank[2] = kin + (n0 >> 16);
                rank[3] = rank[2] + (pn[2] > 0);
                const float dxf = (float)(r / 5 - 2), dyf = (float)(r % 5 - 2);
#pragma unroll
                for (int q = 0; q < kSlots; ++q) {
                    if (pn[q] > 0) {
                        sm.rs[rank[q]] = start[q];
                        sm.rd[rank[q]] = make_float4(__int_as_float(pg[q] - start[q]), dxf, dyf,
                                                     pb[q]);
                    }
                }
            }
            // pad the run starts: the search reads any index below 128
            if (r >= kin + kout) sm.rs[r] = INT_MAX;
            if (r + 64 >= kin + kout) sm.rs[r + 64] = INT_MAX;
            if (r == 0) {
                sm.inner = tin;
                sm.total = tin + tout;
            }
        }
        __syncthreads();
        int nbox = 0, ncell = 0, nchunk = 0;
        if (lane == 0 && nxt < nitems) {
            nbox = items[nxt].box;
            ncell = items[nxt].cell0;
            nchunk = items[nxt].chunk;
        }
        const int total = uni(sm.total);
        const int inner = uni(sm.inner);
        const bool single = total <= CAP;

        // stage the union window [u0, u1): thread t takes elements u0 + t + NT i.
        // Wave 0 first marks the run starts inside the window in a bitmap and
        // counts, per 32-element word, the runs that start before it; the run
        // of element d is then (runs starting at or before d) - 1, one word
        // lookup and a popcount.  Every thread issues all its loads before
        // any LDS store.
        auto stage = [&](int u0, int u1) {
            constexpr int kPer = CAP / NT;
            constexpr int kWords = CAP / 32;
            static_assert(CAP % 32 == 0 && kWords <= 64, "one bitmap word per lane of wave 0");
            if (lane < 64) {
                if (lane < kWords) sm.bm[lane] = 0u;
                __builtin_amdgcn_wave_barrier();
                int before = 0;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int v = sm.rs[lane + 64 * h];   // INT_MAX past the last run
                    if (v < u0)
                        ++before;
                    else if (v < u1)
                        atomicOr(&sm.bm[(v - u0) >> 5], 1u << ((v - u0) & 31));
                }
                __builtin_amdgcn_wave_barrier();
                const int kb = (int)__popcll(__ballot(before >= 1)) +
                               (int)__popcll(__ballot(before >= 2));
                const int c = lane < kWords ? __popc(sm.bm[lane]) : 0;
                const int x = scan_lanes<(kWords <= 32 ? 32 : 64)>(c);
                if (lane < kWords) sm.cum[lane] = kb + x - c;
            }
            __syncthreads();
            int pos[kPer], d[kPer];
#pragma unroll
            for (int i = 0; i < kPer; ++i) {
                d[i] = u0 + lane + NT * i;
                const int e = lane + NT * i;   // < CAP
                const uint32_t w = sm.bm[e >> 5];
                pos[i] = sm.cum[e >> 5] + __popc(w & (0xffffffffu >> (31 - (e & 31)))) - 1;
            }
            float4 buf[kPer], cb[kPer];
            float sh[kPer][3];
#pragma unroll
            for (int i = 0; i < kPer; ++i) {
                if (d[i] < u1) {
                    const float4 dsc = sm.rd[pos[i]];
                    const int gsrc = d[i] + __float_as_int(dsc.x);
                    if constexpr (MODE == 1) {   // the source's 32-byte record
                        buf[i] = ld_global4(gcot, 2 * (B.base + gsrc));
                        cb[i] = ld_global4(gcot, 2 * (B.base + gsrc) + 1);
                    } else {
                        buf[i] = ld_global4(goff, gsrc);
                    }
                    sh[i][0] = dsc.y;
                    sh[i][1] = dsc.z;
                    sh[i][2] = dsc.w;
                }
            }
#pragma unroll
            for (int i = 0; i < kPer; ++i) {
                if (d[i] < u1) {
                    const float4 o = buf[i];
                    float4 v = make_float4(o.x + sh[i][0], o.y + sh[i][1], o.z + (o.w + sh[i][2]),
                                           0.f);
                    if constexpr (MODE == 1) {
                        v.w = cb[i].x;
                        sm.sv[d[i] - u0] = make_float2(cb[i].y, cb[i].z);
                    }
                    sm.sx[d[i] - u0] = v;
                }
            }
            __syncthreads();
        };

        if (single) stage(0, total);

        Acc acc;
        for (int u0 = 0; u0 < total; u0 += CAP) {
            const int u1 = min(total, u0 + CAP);
            if (!single) {
                __syncthreads();
                stage(u0, u1);
            }
            if (active) {
                // Eq. 2 branch for [0, split), f = q^3 (Newton, or Plummer
                // through the r^2 floor) for [split, total)
                const int split = B.plummer ? 0 : (fast ? inner : total);
                const int mid = min(max(split, u0), u1) - u0, hi = u1 - u0;
                if (mid > 0)
                    segment<MODE, true, COMP>(sm.sx, sm.sv, 0, mid, b, P, oi.x, oi.y, oi.z, vi, k,
                                              flush, acc);
                if (hi > mid)
                    segment<MODE, false, COMP>(sm.sx, sm.sv, mid, hi, b, P, oi.x, oi.y, oi.z, vi,
                                               k, flush, acc);
            }
        }
        // ---- fixed-order pairwise sum over slices: slice b adds slice b + half
        //      (TwoSum-compensated in the compensated mode); red overlays sx
        __syncthreads();
        if constexpr (COMP) {
            sm.red[0][lane] = acc.x;
            sm.red[1][lane] = acc.y;
            sm.red[2][lane] = acc.z;
            sm.red[3][lane] = -acc.cx;
            sm.red[4][lane] = -acc.cy;
            sm.red[5][lane] = -acc.cz;
        } else {
            sm.red[0][lane] = acc.x;
            sm.red[1][lane] = acc.y;
            sm.red[2][lane] = acc.z;
        }
        __syncthreads();
        for (int span = P; span > 1;) {
            const int half = (span + 1) >> 1;
            if (active && b < span - half) {
                const int o = lane + half * g;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    if constexpr (COMP) {
                        const float x = sm.red[c][lane], y = sm.red[c][o];
                        const float t = x + y;
                        const float yp = t - x;
                        const float e = (x - (t - yp)) + (y - yp);
                        sm.red[c][lane] = t;
                        sm.red[c + 3][lane] = sm.red[c + 3][lane] + sm.red[c + 3][o] + e;
                    } else {
                        sm.red[c][lane] = sm.red[c][lane] + sm.red[c][o];
                    }
                }
            }
            __syncthreads();
            span = half;
        }
        if (lane < g) {
            float3 f;
            if constexpr (COMP)
                f = make_float3(sm.red[0][lane] + sm.red[3][lane], sm.red[1][lane] + sm.red[4][lane],
                                sm.red[2][lane] + sm.red[5][lane]);
            else
                f = make_float3(sm.red[0][lane], sm.red[1][lane], sm.red[2][lane]);
            store(B, dst, f);
        }
        __syncthreads();
        if (lane == 0) {
            sm.item = nxt;
            sm.ibox = nbox;
            sm.icell = ncell;
            sm.ichunk = nchunk;
        }
    }
}

// ------------------------------------------------------------------ launches

template <typename Kern>
int persistent_grid(Kern kern, int threads) {
    int dev = 0, ncu = 0, per = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, threads, 0);
    return std::max(1, ncu) * std::max(1, per);
}

// The dense, light and narrow kernels of one call run concurrently: the
// light and narrow kernels go to two library streams of the same device
// (default priority), forked from and joined back to the caller's stream with
// events, so the kernels share the CUs (the dense kernel uses no LDS and
// waits on scalar loads, the light kernels lean on LDS) and no kernel's tail
// runs alone.  Under graph capture the fork and joins become graph
// dependencies.  The sequence is enqueued under a lock: the events are shared
// by all calls on the device.
struct SideStream {
    hipStream_t s[2] = {nullptr, nullptr};
    hipEvent_t fork = nullptr, join[2] = {nullptr, nullptr};
};
std::mutex g_side_mu;
std::vector<SideStream> g_side;

hipError_t side_stream(SideStream &out) {   // caller holds g_side_mu
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if ((int)g_side.size() <= dev) g_side.resize(dev + 1);
    SideStream &ss = g_side[dev];
    if (!ss.join[1]) {   // created in this order, so the last one marks completion
        if (!ss.fork &&
            (e = hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming)) != hipSuccess)
            return e;
        for (int k = 0; k < 2; ++k) {
            if (!ss.s[k] &&
                (e = hipStreamCreateWithFlags(&ss.s[k], hipStreamNonBlocking)) != hipSuccess)
                return e;
            if (!ss.join[k] &&
                (e = hipEventCreateWithFlags(&ss.join[k], hipEventDisableTiming)) != hipSuccess)
                return e;
        }
    }
    out = ss;
    return hipSuccess;
}

// One light-kernel instance (NT threads per item, CAP staged sources per
// round) on its persistent grid: every queue needs at least one workgroup,
// so the grid is a multiple of kQueues.
template <int MODE, bool COMP, int CAP, int NT>
hipError_t launch_light_inst(const DevBox *d_boxes, const TilePlan &tp, const float4 *cot,
                             uint32_t *counter, int cls, hipStream_t s) {
    static const int grid =
        (persistent_grid(k_light<MODE, COMP, CAP, NT>, NT) + kQueues - 1) / kQueues * kQueues;
    hipLaunchKernelGGL((k_light<MODE, COMP, CAP, NT>), dim3(grid), dim3(NT), 0, s, d_boxes,
                       (const Item *)tp.light, (const uint32_t *)tp.totals, counter, cot, cls);
    return hipGetLastError();
}

// Light items: windows of 512 / 1024 / 2048 sources (the VJP, whose staged
// sources take 24 bytes instead of 16: 512 / 768 / 1536).
template <int MODE, bool COMP>
hipError_t launch_light(const DevBox *d_boxes, const TilePlan &tp, const float4 *cot,
                        hipStream_t s) {
    uint32_t *q = tp.counter + kQueueStride * kXcds;
    switch (tp.light_window) {
        case 512: return launch_light_inst<MODE, COMP, 512, kLightThreads>(d_boxes, tp, cot, q, 1, s);
        case 2048:
            return launch_light_inst<MODE, COMP, MODE == 0 ? 2048 : 1536, kLightThreads>(
                d_boxes, tp, cot, q, 1, s);
        default:
            return launch_light_inst<MODE, COMP, MODE == 0 ? 1024 : 768, kLightThreads>(
                d_boxes, tp, cot, q, 1, s);
    }
}

// Narrow items: windows of 128 / 256 / 512 sources (VJP: 128 / 192 / 384).
template <int MODE, bool COMP>
hipError_t launch_narrow(const DevBox *d_boxes, const TilePlan &tp, const float4 *cot,
                         hipStream_t s) {
    uint32_t *q = tp.counter + kQueueStride * (kXcds + kQueues);
    switch (tp.narrow_window) {
        case 128: return launch_light_inst<MODE, COMP, 128, kNarrowThreads>(d_boxes, tp, cot, q, 2, s);
        case 512:
            return launch_light_inst<MODE, COMP, MODE == 0 ? 512 : 384, kNarrowThreads>(
                d_boxes, tp, cot, q, 2, s);
        default:
            return launch_light_inst<MODE, COMP, MODE == 0 ? 256 : 192, kNarrowThreads>(
                d_boxes, tp, cot, q, 2, s);
    }
}

template <int MODE, bool COMP>
hipError_t launch_dense(const DevBox *d_boxes, const TilePlan &tp, const float4 *cot,
                        hipStream_t s) {
    // every XCD queue needs at least one workgroup: a multiple of kXcds
    static const int grid =
        (persistent_grid(k_dense<MODE, COMP>, kUnit) + kXcds - 1) / kXcds * kXcds;
    hipLaunchKernelGGL((k_dense<MODE, COMP>), dim3(grid), dim3(kUnit), 0, s, d_boxes,
                       (const Item *)tp.dense, (const uint32_t *)tp.totals, tp.counter, cot);
    return hipGetLastError();
}

template <int MODE, bool COMP>
hipError_t launch_force(const DevBox *d_boxes, const TilePlan &tp, const float4 *cot,
                        bool concurrent, hipStream_t s, const F4Plan *f4) {
    hipError_t e;
    if (!concurrent) {   // the kernels in turn on the caller's stream
        if ((e = launch_light<MODE, COMP>(d_boxes, tp, cot, s)) != hipSuccess) return e;
        if ((e = launch_narrow<MODE, COMP>(d_boxes, tp, cot, s)) != hipSuccess) return e;
        if ((e = launch_dense<MODE, COMP>(d_boxes, tp, cot, s)) != hipSuccess) return e;
        if (f4 && (e = f4_ring_launch(d_boxes, *f4, COMP, s)) != hipSuccess) return e;
        return hipSuccess;
    }
    std::lock_guard<std::mutex> lk(g_side_mu);
    SideStream ss;
    if ((e = side_stream(ss)) != hipSuccess) return e;
    if ((e = hipEventRecord(ss.fork, s)) != hipSuccess) return e;
    for (int k = 0; k < 2; ++k)
        if ((e = hipStreamWaitEvent(ss.s[k], ss.fork, 0)) != hipSuccess) return e;
    if ((e = launch_light<MODE, COMP>(d_boxes, tp, cot, ss.s[0])) != hipSuccess) return e;
    if ((e = hipEventRecord(ss.join[0], ss.s[0])) != hipSuccess) return e;
    if ((e = launch_narrow<MODE, COMP>(d_boxes, tp, cot, ss.s[1])) != hipSuccess) return e;
    if ((e = hipEventRecord(ss.join[1], ss.s[1])) != hipSuccess) return e;
    if ((e = launch_dense<MODE, COMP>(d_boxes, tp, cot, s)) != hipSuccess) return e;
    if (f4 && (e = f4_ring_launch(d_boxes, *f4, COMP, s)) != hipSuccess) return e;
    for (int k = 0; k < 2; ++k)
        if ((e = hipStreamWaitEvent(s, ss.join[k], 0)) != hipSuccess) return e;
    return hipSuccess;
}

}  // namespace

int plan_buckets() { return kKinds * kBuckets; }
// dense queue, light and narrow queues, then the pair kernel's queue
// dense queues (one per XCD), light queues, narrow queues, the pair kernel's
int queue_words() { return (kXcds + 2 * kQueues + 1) * kQueueStride; }

namespace {
__global__ void __launch_bounds__(256)
k_plan_export(const uint32_t *__restrict__ totals, const Item *__restrict__ dense,
              const Item *__restrict__ light, int32_t *__restrict__ out, int64_t max_items,
              int64_t *__restrict__ counts) {
    const int64_t nd = totals[0], nl = totals[1], nn = totals[2];
    const int64_t total = min(nd + nl + nn, max_items);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 3) counts[t] = t == 0 ? nd : (t == 1 ? nl : nn);
    for (int64_t i = t; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        // narrow items follow the light ones in the same array
        const Item it = i < nd ? dense[i] : light[i - nd];
        const int32_t cls = i < nd ? 0 : (i < nd + nl ? 1 : 2);
        int32_t *o = out + 4 * i;
        o[0] = it.box;
        o[1] = it.cell0;
        o[2] = it.chunk;
        o[3] = cls;
    }
}
}  // namespace

hipError_t plan_export_launch(const TilePlan &tp, int32_t *items, int64_t max_items,
                              int64_t *counts, hipStream_t s) {
    const unsigned blocks = (unsigned)std::max<int64_t>(
        1, std::min<int64_t>(4096, (max_items + 255) / 256));
    hipLaunchKernelGGL(k_plan_export, dim3(blocks), dim3(256), 0, s,
                       (const uint32_t *)tp.totals, (const Item *)tp.dense,
                       (const Item *)tp.light, items, max_items, counts);
    return hipGetLastError();
}

hipError_t plan_launch(const DevBox *d_boxes, int nbox, const TilePlan &tp, hipStream_t s) {
    hipError_t e;
    dim3 grid((unsigned)((tp.max_cells + 255) / 256), (unsigned)nbox);
    if ((e = fill_u32(tp.bucket_cnt, kKinds * kBuckets, 0u, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_plan_count, grid, dim3(256), 0, s, d_boxes, tp.cellinfo, tp.bucket_cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_plan_buckets, dim3(1), dim3(kKinds * kBuckets), 0, s, tp.bucket_cnt,
                       tp.bucket_off, tp.totals);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_plan_emit, grid, dim3(256), 0, s, d_boxes,
                       (const uint32_t *)tp.cellinfo, (const uint32_t *)tp.bucket_off,
                       (const uint32_t *)tp.totals, tp.bucket_cnt, tp.dense, tp.light);
    return hipGetLastError();
}

hipError_t tile_launch(const DevBox *d_boxes, int mode, bool compensated, const TilePlan &tp,
                       const float4 *cot, bool concurrent, hipStream_t s, const F4Plan *f4) {
    hipError_t e = fill_u32(tp.counter, queue_words(), 0u, s);
    if (e != hipSuccess) return e;
    if (mode == 0)
        return compensated ? launch_force<0, true>(d_boxes, tp, cot, concurrent, s, f4)
                           : launch_force<0, false>(d_boxes, tp, cot, concurrent, s, f4);
    return compensated ? launch_force<1, true>(d_boxes, tp, cot, concurrent, s, nullptr)
                       : launch_force<1, false>(d_boxes, tp, cot, concurrent, s, nullptr);
}

}  // namespace nf
