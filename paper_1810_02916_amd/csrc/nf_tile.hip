// nf_tile.hip -- tiled near-field kernels for gfx950: a device-side planner
// that cuts the cell grid into work items, and a persistent one-wave-per-
// workgroup kernel that stages each item's sources in LDS and sums the pair
// forces of Eq. 2 (Sec. 4.3) over the 5x5x5 cell block of Sec. 2.1.
//
// Work items (one wave each): all sinks of a cell with at most 64
// particles, or 64 sinks of a denser cell.  Dense items are queued first; a
// global counter hands items to waves, and every wave leaves once the queue
// is empty.
//
// Staging: the item's 125 source cells are copied into LDS in the sink
// cell's own frame, (o_x + dx, o_y + dy, o_z + dz) for a source cell at
// (dx, dy, dz), the 27 cells with |d| <= 1 first, then the 98 outer cells.
// Sources of the sink's own cell are copied unchanged, so the closest pairs
// are formed from the exact float offsets.  Outer cells are at r >= 1 and
// take the Newton branch directly when eps <= 1.  A union larger than the
// LDS buffer is streamed through it in windows.
//
// Lanes: a unit of g <= 64 sinks is spread over the wave as (sink a, source
// slice b), lane = a + g b, P = 64 / g slices; slices are summed at the end
// in a fixed order.
#include "nf_internal.h"
#include "nf_kernels.h"

namespace nf {

namespace {

constexpr int kUnit = 64;      // sinks per unit (one wave)
constexpr int kRows = 25;      // (dx, dy) rows of the 5x5x5 block
constexpr float kTinyT = 1.0e-30f;   // floor on r^2: a coincident pair gives 0
constexpr int kFlush = 32;     // compensated mode: plain partials of <= 32 terms

__device__ __forceinline__ int wrapk(int c, int K) { return c < 0 ? c + K : (c >= K ? c - K : c); }

// ------------------------------------------------------------------ planner

// Items of one cell: ceil(n / 64) chunks when n > 64 (dense), one item when
// 1 <= n <= 64, none when empty.
__global__ void __launch_bounds__(256)
k_plan_count(const DevBox *boxes, uint32_t *hcnt, uint32_t *lcnt) {
    const DevBox &B = boxes[blockIdx.y];
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= B.ncell) return;
    const int n = B.cell_start[c + 1] - B.cell_start[c];
    hcnt[B.cellbase + c] = n > kUnit ? (uint32_t)((n + kUnit - 1) / kUnit) : 0u;
    lcnt[B.cellbase + c] = (n > 0 && n <= kUnit) ? 1u : 0u;
}

__global__ void __launch_bounds__(256)
k_plan_emit(const DevBox *boxes, const uint32_t *__restrict__ hscan,
            const uint32_t *__restrict__ lscan, int64_t TG, Item *items) {
    const DevBox &B = boxes[blockIdx.y];
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= B.ncell) return;
    const int n = B.cell_start[c + 1] - B.cell_start[c];
    if (n > kUnit) {
        Item *o = items + hscan[B.cellbase + c];
        const int nch = (n + kUnit - 1) / kUnit;
        for (int k = 0; k < nch; ++k) o[k] = Item{(int)blockIdx.y, c, 1, k};
    } else if (n > 0) {
        items[hscan[TG] + lscan[B.cellbase + c]] = Item{(int)blockIdx.y, c, 1, 0};
    }
}

// ------------------------------------------------------------------ tiles

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
};

// One pair of the acceleration sum; SPLINE selects the single-min form of
// Eq. 2, otherwise the pair is known to lie outside eps (Newton branch).
template <bool SPLINE>
__device__ __forceinline__ void pair_accel(const float4 s, float xi, float yi, float zi,
                                           const Coef &k, float &px, float &py, float &pz) {
    const float rx = s.x - xi, ry = s.y - yi, rz = s.z - zi;
    float r2 = __builtin_fmaf(rx, rx, kTinyT);
    r2 = __builtin_fmaf(ry, ry, r2);
    r2 = __builtin_fmaf(rz, rz, r2);
    const float q = __builtin_amdgcn_rsqf(r2);
    const float q3 = q * q * q;
    float f;
    if constexpr (SPLINE) {
        const float rho = r2 * q;
        f = fminf(__builtin_fmaf(__builtin_fmaf(k.cC, rho, k.cB), rho, k.cA), q3);
    } else {
        f = q3;
    }
    px = __builtin_fmaf(f, rx, px);
    py = __builtin_fmaf(f, ry, py);
    pz = __builtin_fmaf(f, rz, pz);
}

// One pair of the VJP: xbar_i += g (v_j - v_i) + h (r . (v_j - v_i)) r.
template <bool SPLINE>
__device__ __forceinline__ void pair_vjp(const float4 s, const float2 v, float xi, float yi,
                                         float zi, float vxi, float vyi, float vzi,
                                         const Coef &k, float &px, float &py, float &pz) {
    const float rx = s.x - xi, ry = s.y - yi, rz = s.z - zi;
    const float ux = s.w - vxi, uy = v.x - vyi, uz = v.y - vzi;
    float r2 = __builtin_fmaf(rx, rx, kTinyT);
    r2 = __builtin_fmaf(ry, ry, r2);
    r2 = __builtin_fmaf(rz, rz, r2);
    const float q = __builtin_amdgcn_rsqf(r2);
    const float q2 = q * q;
    const float q3 = q2 * q;
    float g = q3, h = -3.0f * q3 * q2;
    if constexpr (SPLINE) {
        if (r2 < k.eps2) {
            const float rho = r2 * q;
            g = __builtin_fmaf(__builtin_fmaf(k.cC, rho, k.cB), rho, k.cA);
            h = __builtin_fmaf(k.cB, q, k.cC2);
        }
    }
    float rdu = rx * ux;
    rdu = __builtin_fmaf(ry, uy, rdu);
    rdu = __builtin_fmaf(rz, uz, rdu);
    const float t = h * rdu;
    px = __builtin_fmaf(t, rx, __builtin_fmaf(g, ux, px));
    py = __builtin_fmaf(t, ry, __builtin_fmaf(g, uy, py));
    pz = __builtin_fmaf(t, rz, __builtin_fmaf(g, uz, pz));
}

// Sum over staged sources [lo, hi) (LDS indices) for one lane's sink, the
// lane taking indices lo + b, lo + b + P, ...
template <int MODE, bool SPLINE, bool COMP>
__device__ __forceinline__ void segment(const float4 *__restrict__ sx, const float2 *__restrict__ sv,
                                        int lo, int hi, int b, int P, float xi, float yi,
                                        float zi, float4 vi, const Coef &k, Acc &acc) {
    const int n = hi - lo;
    const int nfull = n / P;
    int j = lo + b;
    int it = 0;
    while (it < nfull) {
        const int blk = min(nfull - it, kFlush);
        float px = 0.f, py = 0.f, pz = 0.f;
        if constexpr (!COMP) {
            px = acc.x;
            py = acc.y;
            pz = acc.z;
        }
#pragma unroll 4
        for (int t = 0; t < blk; ++t) {
            if constexpr (MODE == 0)
                pair_accel<SPLINE>(sx[j], xi, yi, zi, k, px, py, pz);
            else
                pair_vjp<SPLINE>(sx[j], sv[j], xi, yi, zi, vi.x, vi.y, vi.z, k, px, py, pz);
            j += P;
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
        if constexpr (MODE == 0)
            pair_accel<SPLINE>(sx[j], xi, yi, zi, k, px, py, pz);
        else
            pair_vjp<SPLINE>(sx[j], sv[j], xi, yi, zi, vi.x, vi.y, vi.z, k, px, py, pz);
        fold<COMP>(acc, px, py, pz);
    }
}

__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Pieces of the staged union: per row r = (dx+2)*5 + (dy+2) up to four
// contiguous global ranges.  Slots 0-1: the |dz| <= 1 part of an inner row
// (|dx|, |dy| <= 1); slots 2-3: the rest of the row (dz = -2 and +2 for an
// inner row, dz = -2..2 split at the periodic wrap for an outer row).
constexpr int kSlots = 4;
constexpr int kPiece = kRows * kSlots;

template <int MODE, int CAP>
struct TileSmem {
    float4 sx[CAP];                  // (o_x + dx, o_y + dy, o_z + dz, v_x)
    float2 sv[MODE == 1 ? CAP : 1];  // (v_y, v_z) for the VJP
    int pu[kPiece];                  // staged start of each piece
    int pn[kPiece];                  // particles in the piece
    int pg[kPiece];                  // global start of the piece
    float pb[kPiece];                // z shift minus the source's cell index
    int cnt[2][kRows];               // per row: inner-part and outer-part counts
    float red[3][kUnit];
    int item;
    int inner;                       // staged particles of the 27 inner cells
    int total;
};

template <int MODE, bool COMP, int CAP>
__global__ void __launch_bounds__(kUnit)
k_tile(const DevBox *__restrict__ boxes, const Item *__restrict__ items,
       const uint32_t *__restrict__ hscan, const uint32_t *__restrict__ lscan, int64_t TG,
       uint32_t *counter, const float4 *__restrict__ cot_sorted) {
    __shared__ TileSmem<MODE, CAP> sm;
    const int lane = threadIdx.x;
    const int nitems = (int)(hscan[TG] + lscan[TG]);

    for (;;) {
        if (lane == 0) sm.item = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int itx = uni(sm.item);
        if (itx >= nitems) break;
        const Item I = items[itx];
        const DevBox &B = boxes[I.box];
        const int K = B.K;
        const int cx = I.cell0 / (K * K), cy = (I.cell0 / K) % K, z = I.cell0 % K;
        const int32_t *__restrict__ cs = B.cell_start;
        const float4 *__restrict__ off = B.off;

        // ---- pieces, one lane per row
        if (lane < kRows) {
            const int r = lane;
            const int dx = r / 5 - 2, dy = r % 5 - 2;
            const bool in_row = dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1;
            const int rb = (wrapk(cx + dx, K) * K + wrapk(cy + dy, K)) * K;
            int g[kSlots], n[kSlots];
            float bias[kSlots];
            // a run of z cells [za, zb] relative to the sink (za <= zb), split at the wrap
            auto run = [&](int s0, int za, int zb) {
                const int lo = z + za, hi = z + zb;
                if (lo < 0) {                       // [lo+K, K-1] then [0, hi]
                    g[s0] = cs[rb + lo + K];
                    n[s0] = cs[rb + K] - g[s0];
                    bias[s0] = -(float)(z + K);
                    g[s0 + 1] = cs[rb];
                    n[s0 + 1] = cs[rb + hi + 1] - g[s0 + 1];
                    bias[s0 + 1] = -(float)z;
                } else if (hi >= K) {               // [lo, K-1] then [0, hi-K]
                    g[s0] = cs[rb + lo];
                    n[s0] = cs[rb + K] - g[s0];
                    bias[s0] = -(float)z;
                    g[s0 + 1] = cs[rb];
                    n[s0 + 1] = cs[rb + hi - K + 1] - g[s0 + 1];
                    bias[s0 + 1] = (float)(K - z);
                } else {
                    g[s0] = cs[rb + lo];
                    n[s0] = cs[rb + hi + 1] - g[s0];
                    bias[s0] = -(float)z;
                    g[s0 + 1] = 0;
                    n[s0 + 1] = 0;
                    bias[s0 + 1] = 0.f;
                }
            };
            if (in_row) {
                run(0, -1, 1);
                // the two single cells at dz = -2 and dz = +2
                const int zm = z - 2, zp = z + 2;
                const int cm = rb + wrapk(zm, K), cp = rb + wrapk(zp, K);
                g[2] = cs[cm];
                n[2] = cs[cm + 1] - g[2];
                bias[2] = -(float)z + (zm < 0 ? -(float)K : 0.f);
                g[3] = cs[cp];
                n[3] = cs[cp + 1] - g[3];
                bias[3] = -(float)z + (zp >= K ? (float)K : 0.f);
            } else {
                g[0] = g[1] = 0;
                n[0] = n[1] = 0;
                bias[0] = bias[1] = 0.f;
                run(2, -2, 2);
            }
            for (int q = 0; q < kSlots; ++q) {
                sm.pn[r * kSlots + q] = n[q];
                sm.pg[r * kSlots + q] = g[q];
                sm.pb[r * kSlots + q] = bias[q];
            }
            sm.cnt[0][r] = n[0] + n[1];
            sm.cnt[1][r] = n[2] + n[3];
        }
        __syncthreads();
        if (lane < kRows) {
            const int r = lane;
            int in0 = 0, out0 = 0, tin = 0, tout = 0;
            for (int q = 0; q < kRows; ++q) {
                const int a = sm.cnt[0][q], e = sm.cnt[1][q];
                if (q < r) {
                    in0 += a;
                    out0 += e;
                }
                tin += a;
                tout += e;
            }
            out0 += tin;
            sm.pu[r * kSlots + 0] = in0;
            sm.pu[r * kSlots + 1] = in0 + sm.pn[r * kSlots + 0];
            sm.pu[r * kSlots + 2] = out0;
            sm.pu[r * kSlots + 3] = out0 + sm.pn[r * kSlots + 2];
            if (r == 0) {
                sm.inner = tin;
                sm.total = tin + tout;
            }
        }
        __syncthreads();
        const int total = uni(sm.total);
        const int inner = uni(sm.inner);
        const bool single = total <= CAP;

        // stage the union window [u0, u1)
        auto stage = [&](int u0, int u1) {
            for (int pc = 0; pc < kPiece; ++pc) {
                const int pu = uni(sm.pu[pc]);
                const int a = max(pu, u0), e = min(pu + uni(sm.pn[pc]), u1);
                if (a >= e) continue;
                const int gshift = uni(sm.pg[pc]) - pu;
                const int r = pc / kSlots;
                const float dxf = (float)(r / 5 - 2), dyf = (float)(r % 5 - 2);
                const float bias = sm.pb[pc];
                for (int v = a + lane; v < e; v += kUnit) {
                    const float4 o = off[v + gshift];
                    float4 t = make_float4(o.x + dxf, o.y + dyf, o.z + (o.w + bias), 0.f);
                    if constexpr (MODE == 1) {
                        const float4 c = cot_sorted[B.base + v + gshift];
                        t.w = c.x;
                        sm.sv[v - u0] = make_float2(c.y, c.z);
                    }
                    sm.sx[v - u0] = t;
                }
            }
            __syncthreads();
        };

        if (single) stage(0, total);

        const Coef k{B.cA, B.cB, B.cC, 2.0f * B.cC, B.eps * B.eps};
        const bool fast = B.outer_newton != 0;
        int s0 = cs[I.cell0], s1 = cs[I.cell0 + 1];
        if (s1 - s0 > kUnit) {
            s0 += kUnit * I.chunk;
            s1 = min(s1, s0 + kUnit);
        }
        s0 = uni(s0);
        s1 = uni(s1);
        const int g = s1 - s0;
        const int P = kUnit / g;
        const bool active = lane < g * P;
        const int a = active ? lane % g : 0;
        const int b = active ? lane / g : 0;
        const float4 oi = off[s0 + a];
        float4 vi = make_float4(0.f, 0.f, 0.f, 0.f);
        if constexpr (MODE == 1) vi = cot_sorted[B.base + s0 + a];
        Acc acc;
        for (int u0 = 0; u0 < total; u0 += CAP) {
            const int u1 = min(total, u0 + CAP);
            if (!single) {
                __syncthreads();
                stage(u0, u1);
            }
            if (active) {
                const int split = fast ? inner : total;
                const int lo = 0, mid = min(max(split, u0), u1) - u0, hi = u1 - u0;
                if (mid > lo)
                    segment<MODE, true, COMP>(sm.sx, sm.sv, lo, mid, b, P, oi.x, oi.y, oi.z, vi,
                                              k, acc);
                if (hi > mid)
                    segment<MODE, false, COMP>(sm.sx, sm.sv, mid, hi, b, P, oi.x, oi.y, oi.z, vi,
                                               k, acc);
            }
        }
        // ---- fixed-order sum over slices
        float fx, fy, fz;
        if constexpr (COMP) {
            fx = acc.x - acc.cx;
            fy = acc.y - acc.cy;
            fz = acc.z - acc.cz;
        } else {
            fx = acc.x;
            fy = acc.y;
            fz = acc.z;
        }
        if (P > 1) {
            sm.red[0][lane] = fx;
            sm.red[1][lane] = fy;
            sm.red[2][lane] = fz;
            __syncthreads();
            if (lane < g) {
                Acc t;
                for (int sl = 0; sl < P; ++sl)
                    fold<COMP>(t, sm.red[0][lane + sl * g], sm.red[1][lane + sl * g],
                               sm.red[2][lane + sl * g]);
                if constexpr (COMP) {
                    fx = t.x - t.cx;
                    fy = t.y - t.cy;
                    fz = t.z - t.cz;
                } else {
                    fx = t.x;
                    fy = t.y;
                    fz = t.z;
                }
            }
        }
        if (lane < g) {
            const int i = B.order[s0 + lane];
            if (i >= 0 && i < B.n) {
                float *o = B.out + 3 * (int64_t)i;
                o[0] = fx * B.scale;
                o[1] = fy * B.scale;
                o[2] = fz * B.scale;
            }
        }
        __syncthreads();
    }
}

template <int MODE, bool COMP, int CAP>
int tile_grid() {
    static int grid = 0;
    if (grid == 0) {
        int dev = 0, ncu = 0, per = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_tile<MODE, COMP, CAP>, kUnit, 0);
        grid = std::max(1, ncu) * std::max(1, per);
    }
    return grid;
}

template <int MODE, bool COMP>
hipError_t launch_tile(const DevBox *d_boxes, const TilePlan &tp, const float4 *cot, hipStream_t s) {
    constexpr int CAP = MODE == 0 ? 1024 : 768;
    const int grid = tile_grid<MODE, COMP, CAP>();
    hipLaunchKernelGGL((k_tile<MODE, COMP, CAP>), dim3(grid), dim3(kUnit), 0, s, d_boxes,
                       (const Item *)tp.items, (const uint32_t *)tp.hcnt,
                       (const uint32_t *)tp.lcnt, tp.TG, tp.counter, cot);
    return hipGetLastError();
}

}  // namespace

hipError_t plan_launch(const DevBox *d_boxes, int nbox, const TilePlan &tp, hipStream_t s) {
    hipError_t e;
    dim3 grid((unsigned)((tp.max_cells + 255) / 256), (unsigned)nbox);
    if ((e = fill_u32(tp.hcnt + tp.TG, 1, 0u, s)) != hipSuccess) return e;
    if ((e = fill_u32(tp.lcnt + tp.TG, 1, 0u, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_plan_count, grid, dim3(256), 0, s, d_boxes, tp.hcnt, tp.lcnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = scan_exclusive(tp.hcnt, tp.TG + 1, tp.scan_scratch, s)) != hipSuccess) return e;
    if ((e = scan_exclusive(tp.lcnt, tp.TG + 1, tp.scan_scratch, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_plan_emit, grid, dim3(256), 0, s, d_boxes, (const uint32_t *)tp.hcnt,
                       (const uint32_t *)tp.lcnt, tp.TG, tp.items);
    return hipGetLastError();
}

hipError_t tile_launch(const DevBox *d_boxes, int mode, bool compensated, const TilePlan &tp,
                       const float4 *cot, hipStream_t s) {
    hipError_t e = fill_u32(tp.counter, 1, 0u, s);
    if (e != hipSuccess) return e;
    if (mode == 0)
        return compensated ? launch_tile<0, true>(d_boxes, tp, cot, s)
                           : launch_tile<0, false>(d_boxes, tp, cot, s);
    return compensated ? launch_tile<1, true>(d_boxes, tp, cot, s)
                       : launch_tile<1, false>(d_boxes, tp, cot, s);
}

}  // namespace nf
