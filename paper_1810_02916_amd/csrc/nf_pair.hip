// nf_pair.hip -- Newton's third law for dense cell pairs (NF_PAIR_SYMMETRIC).
//
// Every pair of particles belongs to exactly one of the near and far fields
// (Sec. 2.1), and the pair force is odd in r (Eq. 2), so a near pair (i, j)
// can be evaluated once and applied to both: a_i += F(r_ij), a_j -= F(r_ij).
// The gather kernels evaluate every pair twice (once per sink).  This path
// halves the evaluations between symmetric cells: cells of 1 to kF4MaxChunks
// chunks of 64 sinks whose sinks are all summed by the dense kernel (the
// cell count is a multiple of 64, or its last chunk holds at least dense_min
// sinks).  For two such cells X and Y in each other's 5x5x5 block the pairs
// are evaluated once, by the cell of lower linear id; the dense kernel skips
// the other's sources for those sinks.
//
// Deterministic accumulation without float atomics.  Every sink of a
// symmetric cell X owns P_X partial sums, slot-major (slot k of sink i at
// base_X + k n_X + i):
//   k = 0                    the dense kernel's sum over the other sources;
//   k = 1 + r                the r-th partner Y > X (direction order): the
//                            pair kernel's sum over all of Y's sinks;
//   k = 1 + nfwd + c(W) + a  a partner W < X: the reaction from W's chunk a,
//                            c(W) = chunks of X's earlier partners W' < X.
// k_f4_combine adds each sink's partials in slot order (TwoSum-compensated
// in the compensated mode), scales and stores them.  The partial buffer has
// a fixed capacity; a call whose plan exceeds it runs entirely in the gather
// form (a device flag read by every kernel), with the same results as
// without the flag.
//
// The pair kernel k_f4_ring: one wave holds 64 sinks of X (one per lane) and
// 64 sources of Y; the 4096 pairs are visited as 4 phases of 16 steps: in
// step s lane c of a row of 16 lanes pairs its sink with the source in column
// (c + s) mod 16 of the row (a DPP row rotation of the source registers), and
// the reaction accumulators rotate with the sources one column per step; a
// phase ends by moving the sources and their accumulators to the next row.
#include "nf_internal.h"
#include "nf_kernels.h"

namespace nf {
namespace {

__device__ __forceinline__ int wrapk(int c, int K) { return c < 0 ? c + K : (c >= K ? c - K : c); }
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int chunks_of(int n) { return (n + 63) >> 6; }

// Direction t in 0..124 of the 5x5x5 block: t = (dx+2) 25 + (dy+2) 5 + (dz+2);
// t = 62 is the cell itself.
constexpr int kSelf = 62;

__device__ __forceinline__ int neighbour(int cx, int cy, int cz, int t, int K) {
    return (wrapk(cx + t / 25 - 2, K) * K + wrapk(cy + (t / 5) % 5 - 2, K)) * K +
           wrapk(cz + t % 5 - 2, K);
}

// ------------------------------------------------------------------ planner

// Per cell of every box: P (partials per sink, 0 when not symmetric), nfwd,
// the slot count n P and the item count chunks nfwd (one item per chunk of X
// and partner Y > X); each block also leaves its 64-bit totals (the 32-bit
// scans of the counts may wrap before the capacity check sees them).
__global__ void __launch_bounds__(256)
k_f4_count(const DevBox *boxes, int32_t *P, int32_t *nfwd, uint32_t *slotcnt,
           uint32_t *itemcnt, uint64_t *blk) {
    __shared__ uint64_t red[2][256];
    const DevBox &B = boxes[blockIdx.y];
    const int c = blockIdx.x * 256 + threadIdx.x;
    uint64_t my_slots = 0, my_items = 0;
    if (c < B.ncell) {
        const gptr<const int32_t> cs = gp(B.cell_start);
        const int K = B.K, dm = B.dense_min;
        const int n = cs[c + 1] - cs[c];
        int p = 0, nf = 0;
        if (f4_symmetric_cell(n, dm)) {
            const int cx = c / (K * K), cy = (c / K) % K, cz = c % K;
            int nb = 0;
            for (int t = 0; t < 125; ++t) {
                if (t == kSelf) continue;
                const int y = neighbour(cx, cy, cz, t, K);
                const int ny = cs[y + 1] - cs[y];
                if (!f4_symmetric_cell(ny, dm)) continue;
                if (y > c) ++nf;
                else nb += chunks_of(ny);
            }
            p = 1 + nf + nb;
        }
        const int64_t g = B.cellbase + c;
        P[g] = p;
        nfwd[g] = nf;
        my_slots = (uint64_t)n * (uint64_t)p;
        my_items = p ? (uint64_t)chunks_of(n) * (uint64_t)nf : 0;
        slotcnt[g] = (uint32_t)my_slots;
        itemcnt[g] = (uint32_t)my_items;
    }
    red[0][threadIdx.x] = my_slots;
    red[1][threadIdx.x] = my_items;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[0][threadIdx.x] += red[0][threadIdx.x + h];
            red[1][threadIdx.x] += red[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t bi = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
        blk[2 * bi] = red[0][0];
        blk[2 * bi + 1] = red[1][0];
    }
}

// Totals of the block sums; the path is on when the plan fits the
// capacities (then the 32-bit scans did not wrap either).
__global__ void __launch_bounds__(256)
k_f4_check(const uint64_t *blk, int64_t nblk, uint32_t cap_slots, uint32_t cap_items,
           uint32_t *tot) {
    __shared__ uint64_t red[2][256];
    uint64_t s0 = 0, s1 = 0;
    for (int64_t i = threadIdx.x; i < nblk; i += 256) {
        s0 += blk[2 * i];
        s1 += blk[2 * i + 1];
    }
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[0][threadIdx.x] += red[0][threadIdx.x + h];
            red[1][threadIdx.x] += red[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const uint64_t ns = red[0][0], ni = red[1][0];
        tot[0] = (ns <= cap_slots && ni <= cap_items) ? 1u : 0u;
        tot[1] = (uint32_t)(ni <= cap_items ? ni : 0);
        tot[2] = (uint32_t)(ns <= cap_slots ? ns : 0);
    }
}

// Items of each symmetric cell X: for every partner Y > X (rank r in
// direction order) and every chunk a of X.
__global__ void __launch_bounds__(256)
k_f4_emit(const DevBox *boxes, const int32_t *P, const int32_t *nfwd, const uint32_t *itemoff,
          const uint32_t *tot, PairItem *items) {
    const DevBox &B = boxes[blockIdx.y];
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= B.ncell || !tot[0]) return;
    const int64_t g = B.cellbase + c;
    if (!P[g]) return;
    const gptr<const int32_t> cs = gp(B.cell_start);
    const int K = B.K, dm = B.dense_min;
    const int n = cs[c + 1] - cs[c];
    const int cx = c / (K * K), cy = (c / K) % K, cz = c % K;
    const int ch = chunks_of(n), nf = nfwd[g];
    const uint32_t at = itemoff[g];
    int r = 0;
    for (int t = 0; t < 125; ++t) {
        if (t == kSelf) continue;
        const int y = neighbour(cx, cy, cz, t, K);
        if (y <= c) continue;
        if (!f4_symmetric_cell(cs[y + 1] - cs[y], dm)) continue;
        for (int a = 0; a < ch; ++a)
            items[at + (uint32_t)(r * ch + a)] = PairItem{(int)blockIdx.y, c, a, t, r, 0};
        ++r;
    }
    (void)nf;
}

// ------------------------------------------------------------------ pair kernel

// Rotation inside each row of 16 lanes: lane c receives lane (c - N) mod 16
// (N = 0: no move).
template <int N>
__device__ __forceinline__ float ror(float x) {
    if constexpr (N == 0) {
        return x;
    } else {
        return __int_as_float(
            __builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x120 + N, 0xf, 0xf, true));
    }
}

struct Coef4 {
    float cA, cB, cC, floor;
};

// F(r) / |r| for a pair at r (Eq. 2 single-min form, or the Newton branch).
template <bool SPLINE>
__device__ __forceinline__ float pair_f(float rx, float ry, float rz, const Coef4 &k) {
    float r2 = __builtin_fmaf(rx, rx, k.floor);
    r2 = __builtin_fmaf(ry, ry, r2);
    r2 = __builtin_fmaf(rz, rz, r2);
    const float q = __builtin_amdgcn_rsqf(r2);
    const float q3 = q * q * q;
    if constexpr (SPLINE) {
        const float rho = r2 * q;
        return fminf(__builtin_fmaf(__builtin_fmaf(k.cC, rho, k.cB), rho, k.cA), q3);
    } else {
        return q3;
    }
}

struct Ring {
    float ax, ay, az;   // this lane's sink (X frame)
    float bx, by, bz;   // the source this lane holds (shifted into the X frame)
    float mb;           // 1 for a valid source, 0 for a padding lane
    float ma;           // 1 for a valid sink
};

// One step s of a phase: lane c pairs its sink with the source of column
// (c + s) mod 16 of its row; t = F r goes to the sink (pa) and, negated, to
// the reaction accumulator of that source, which rotates with the columns.
template <int S, bool SPLINE, bool MASK>
__device__ __forceinline__ void ring_steps(const Ring &g, const Coef4 &k, float &pax, float &pay,
                                           float &paz, float &rx_, float &ry_, float &rz_) {
    // t = F r is formed once and both updates are plain adds, so the rotation
    // of an accumulator is a DPP operand of its subtraction (no fused forms)
#pragma clang fp contract(off)
    constexpr int N = (16 - S) & 15;   // lane c reads lane (c + S) mod 16
    const float sx = ror<N>(g.bx);
    const float sy = ror<N>(g.by);
    const float sz = ror<N>(g.bz);
    const float rx = sx - g.ax, ry = sy - g.ay, rz = sz - g.az;
    float f = pair_f<SPLINE>(rx, ry, rz, k);
    if constexpr (MASK) f *= g.ma * ror<N>(g.mb);
    const float tx = f * rx, ty = f * ry, tz = f * rz;
    pax += tx;
    pay += ty;
    paz += tz;
    if constexpr (S == 0) {
        rx_ -= tx;
        ry_ -= ty;
        rz_ -= tz;
    } else {   // the accumulator of source (c + S) was at lane c + 1 in step S - 1
        rx_ = ror<15>(rx_) - tx;
        ry_ = ror<15>(ry_) - ty;
        rz_ = ror<15>(rz_) - tz;
    }
    if constexpr (S < 15) ring_steps<S + 1, SPLINE, MASK>(g, k, pax, pay, paz, rx_, ry_, rz_);
}

__device__ __forceinline__ void kahan1(float &s, float &c, float v) {
    const float y = v - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

struct Sum3 {
    float x = 0.f, y = 0.f, z = 0.f, cx = 0.f, cy = 0.f, cz = 0.f;
};
template <bool COMP>
__device__ __forceinline__ void add3(Sum3 &a, float x, float y, float z) {
    if constexpr (COMP) {
        kahan1(a.x, a.cx, x);
        kahan1(a.y, a.cy, y);
        kahan1(a.z, a.cz, z);
    } else {
        a.x += x;
        a.y += y;
        a.z += z;
    }
}

__device__ __forceinline__ float shfl16(float v) {   // lane l receives lane (l + 16) mod 64
    return __shfl(v, (int)((threadIdx.x + 16) & 63), 64);
}

// Slot k of sink i of a cell: float4 (x, y, z, -) per value; two per slot
// (value, compensation) in the compensated mode.
template <bool COMP>
__device__ __forceinline__ void put(float4 *part, uint32_t idx, const Sum3 &v) {
    if constexpr (COMP) {
        st_g4(part, 2 * (uint64_t)idx, v.x, v.y, v.z);
        st_g4(part, 2 * (uint64_t)idx + 1, -v.cx, -v.cy, -v.cz);
    } else {
        st_g4(part, idx, v.x, v.y, v.z);
    }
}

template <bool SPLINE, bool MASK, bool COMP>
__device__ __forceinline__ void ring_chunk(Ring g, const Coef4 &k, Sum3 &A, Sum3 &RB) {
    for (int phase = 0; phase < 4; ++phase) {
        float pax = 0.f, pay = 0.f, paz = 0.f, rx = 0.f, ry = 0.f, rz = 0.f;
        ring_steps<0, SPLINE, MASK>(g, k, pax, pay, paz, rx, ry, rz);
        // after step 15 lane c holds the accumulator of column c - 1: realign
        rx = ror<15>(rx);
        ry = ror<15>(ry);
        rz = ror<15>(rz);
        add3<COMP>(A, pax, pay, paz);
        add3<COMP>(RB, rx, ry, rz);
        // sources and their accumulators move to the next row (the fourth move
        // brings the accumulators home; the sources are not needed after it)
        RB.x = shfl16(RB.x);
        RB.y = shfl16(RB.y);
        RB.z = shfl16(RB.z);
        if constexpr (COMP) {
            RB.cx = shfl16(RB.cx);
            RB.cy = shfl16(RB.cy);
            RB.cz = shfl16(RB.cz);
        }
        if (phase < 3) {
            g.bx = shfl16(g.bx);
            g.by = shfl16(g.by);
            g.bz = shfl16(g.bz);
            if constexpr (MASK) g.mb = shfl16(g.mb);
        }
    }
}

template <bool COMP>
__global__ void __launch_bounds__(64)
k_f4_ring(const DevBox *__restrict__ boxes, const PairItem *__restrict__ items,
          const uint32_t *__restrict__ tot, uint32_t *counter) {
    __shared__ int s_item;
    const int lane = threadIdx.x;
    if (!tot[0]) return;
    const int nitems = (int)tot[1];
    for (;;) {
        if (lane == 0)
            s_item = (int)__hip_atomic_fetch_add(gp(counter), 1u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int itx = uni(s_item);
        __syncthreads();
        if (itx >= nitems) break;
        const gptr<const PairItem> ip = gp(items) + itx;
        const int ib = ip->box, X = ip->cell, a = ip->chunk, t = ip->dir, r = ip->rank;
        const DevBox &B = boxes[ib];
        const int K = B.K, dm = B.dense_min;
        const gptr<const int32_t> cs = gp(B.cell_start);
        const int cx = X / (K * K), cy = (X / K) % K, cz = X % K;
        const int Y = neighbour(cx, cy, cz, t, K);
        const int dx = t / 25 - 2, dy = (t / 5) % 5 - 2, dz = t % 5 - 2;
        const int sX = uni(cs[X]), nX = uni(cs[X + 1]) - sX;
        const int sY = uni(cs[Y]), nY = uni(cs[Y + 1]) - sY;
        const int64_t gX = B.cellbase + X, gY = B.cellbase + Y;
        const int PX = uni(gp(B.f4P)[gX]), PY = uni(gp(B.f4P)[gY]);
        const int nfY = uni(gp(B.f4nf)[gY]);
        const uint32_t baseX = (uint32_t)uni((int)gp(B.f4off)[gX]);
        const uint32_t baseY = (uint32_t)uni((int)gp(B.f4off)[gY]);
        // c(X) for Y: chunks of Y's partners W < Y that come before X in Y's
        // direction order (the direction from Y to X is 124 - t)
        int part = 0;
        for (int u = lane; u < 125; u += 64) {
            if (u == kSelf || u >= 124 - t) continue;
            const int w = neighbour(Y / (K * K), (Y / K) % K, Y % K, u, K);
            if (w >= Y) continue;
            const int nw = cs[w + 1] - cs[w];
            if (f4_symmetric_cell(nw, dm)) part += chunks_of(nw);
        }
        for (int o = 32; o >= 1; o >>= 1) part += __shfl_xor(part, o, 64);
        const int kB = 1 + nfY + uni(part) + a;
        const Coef4 k{B.cA, B.cB, B.cC, B.r2floor};
        const bool spline = !B.plummer && (!B.outer_newton ||
                                          (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 &&
                                           dz >= -1 && dz <= 1));
        const int gA = min(64, nX - 64 * a);
        Ring g;
        {
            const float4 o = ld_off4(B.off, sX + 64 * a + min(lane, gA - 1));
            g.ax = o.x;
            g.ay = o.y;
            g.az = o.z;
            g.ma = lane < gA ? 1.f : 0.f;
        }
        Sum3 A;
        const int chY = chunks_of(nY);
        for (int b = 0; b < chY; ++b) {
            const int gB = min(64, nY - 64 * b);
            const float4 o = ld_off4(B.off, sY + 64 * b + min(lane, gB - 1));
            g.bx = o.x + (float)dx;
            g.by = o.y + (float)dy;
            g.bz = o.z + (float)dz;
            g.mb = lane < gB ? 1.f : 0.f;
            Sum3 RB;
            const bool mask = gA < 64 || gB < 64;
            if (spline) {
                if (mask) ring_chunk<true, true, COMP>(g, k, A, RB);
                else ring_chunk<true, false, COMP>(g, k, A, RB);
            } else {
                if (mask) ring_chunk<false, true, COMP>(g, k, A, RB);
                else ring_chunk<false, false, COMP>(g, k, A, RB);
            }
            if (lane < gB) put<COMP>(B.f4part, baseY + (uint32_t)kB * nY + 64 * b + lane, RB);
        }
        if (lane < gA) put<COMP>(B.f4part, baseX + (uint32_t)(1 + r) * nX + 64 * a + lane, A);
    }
}

// ------------------------------------------------------------------ combine

// One wave per cell: each sink of a symmetric cell adds its partials in slot
// order, scales and stores the result in caller order.
template <bool COMP>
__global__ void __launch_bounds__(256)
k_f4_combine(const DevBox *__restrict__ boxes, const uint32_t *__restrict__ tot) {
    if (!tot[0]) return;
    const DevBox &B = boxes[blockIdx.y];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const gptr<const int32_t> cs = gp(B.cell_start);
    const float4 *part = B.f4part;
    for (int c = blockIdx.x * 4 + wave; c < B.ncell; c += gridDim.x * 4) {
        const int64_t gc = B.cellbase + c;
        const int P = gp(B.f4P)[gc];
        if (!P) continue;
        const int s0 = cs[c], n = cs[c + 1] - s0;
        const uint32_t base = gp(B.f4off)[gc];
        for (int i = lane; i < n; i += 64) {
            float sx = 0.f, sy = 0.f, sz = 0.f, ex = 0.f, ey = 0.f, ez = 0.f;
            for (int kk = 0; kk < P; ++kk) {
                const uint32_t idx = base + (uint32_t)kk * n + i;
                if constexpr (COMP) {
                    const nf_v4f v = ld_g4(part, 2 * (uint64_t)idx);
                    const nf_v4f w = ld_g4(part, 2 * (uint64_t)idx + 1);
                    // TwoSum of the running sum and the value; errors collected
                    auto two = [](float &s, float &e, float x, float lo) {
                        const float t = s + x;
                        const float xp = t - s;
                        e += ((s - (t - xp)) + (x - xp)) + lo;
                        s = t;
                    };
                    two(sx, ex, v.x, w.x);
                    two(sy, ey, v.y, w.y);
                    two(sz, ez, v.z, w.z);
                } else {
                    const nf_v4f v = ld_g4(part, idx);
                    sx += v.x;
                    sy += v.y;
                    sz += v.z;
                }
            }
            const int o = gp(B.order)[s0 + i];
            if (o >= 0 && o < B.n) {
                gptr<float> out = gp(B.out) + 3 * (int64_t)o;
                out[0] = (sx + ex) * B.scale;
                out[1] = (sy + ey) * B.scale;
                out[2] = (sz + ez) * B.scale;
            }
        }
    }
}

}  // namespace

int f4_queue_words() { return 32; }

hipError_t f4_plan_launch(const DevBox *d_boxes, int nbox, const F4Plan &fp, hipStream_t s) {
    hipError_t e;
    dim3 grid((unsigned)((fp.max_cells + 255) / 256), (unsigned)nbox);
    if ((e = fill_u32(fp.slotoff, fp.C + 1, 0u, s)) != hipSuccess) return e;
    if ((e = fill_u32(fp.itemoff, fp.C + 1, 0u, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_f4_count, grid, dim3(256), 0, s, d_boxes, fp.P, fp.nfwd, fp.slotoff,
                       fp.itemoff, fp.blk);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = scan_exclusive(fp.slotoff, fp.C + 1, fp.scan, s)) != hipSuccess) return e;
    if ((e = scan_exclusive(fp.itemoff, fp.C + 1, fp.scan, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_f4_check, dim3(1), dim3(256), 0, s, (const uint64_t *)fp.blk,
                       (int64_t)grid.x * nbox, fp.cap_slots, fp.cap_items, fp.tot);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_f4_emit, grid, dim3(256), 0, s, d_boxes, (const int32_t *)fp.P,
                       (const int32_t *)fp.nfwd, (const uint32_t *)fp.itemoff,
                       (const uint32_t *)fp.tot, fp.items);
    return hipGetLastError();
}

hipError_t f4_ring_launch(const DevBox *d_boxes, const F4Plan &fp, bool compensated,
                          hipStream_t s) {
    int dev = 0, ncu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    const unsigned grid = (unsigned)std::max(1, ncu) * 16;
    if (compensated)
        hipLaunchKernelGGL(k_f4_ring<true>, dim3(grid), dim3(64), 0, s, d_boxes,
                           (const PairItem *)fp.items, (const uint32_t *)fp.tot, fp.counter);
    else
        hipLaunchKernelGGL(k_f4_ring<false>, dim3(grid), dim3(64), 0, s, d_boxes,
                           (const PairItem *)fp.items, (const uint32_t *)fp.tot, fp.counter);
    return hipGetLastError();
}

hipError_t f4_combine_launch(const DevBox *d_boxes, int nbox, const F4Plan &fp, bool compensated,
                             hipStream_t s) {
    const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>((fp.max_cells + 3) / 4, 16384));
    if (compensated)
        hipLaunchKernelGGL(k_f4_combine<true>, dim3(gx, (unsigned)nbox), dim3(256), 0, s, d_boxes,
                           (const uint32_t *)fp.tot);
    else
        hipLaunchKernelGGL(k_f4_combine<false>, dim3(gx, (unsigned)nbox), dim3(256), 0, s,
                           d_boxes, (const uint32_t *)fp.tot);
    return hipGetLastError();
}

}  // namespace nf
