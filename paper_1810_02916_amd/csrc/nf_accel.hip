// nf_accel.hip -- near-field pair kernels: accelerations (Sec. 2.1 direct sum
// over the 5x5x5 cell block, Eq. 2 spline softening of Sec. 4.3) and their
// vector-Jacobian product.
//
// This file holds the reference ("simple") kernels: one sink per thread,
// sources read from global memory cell by cell.  Arithmetic per pair, in
// cell widths with the sink shifted into the source cell's frame:
//   r   = o_j - (o_i - d)                 (3 sub)
//   r2  = r.r + floor                     (3 fma; floor = 1e-30 makes r = 0 give
//                                          0, or eps_p^2 for the Plummer law)
//   q   = rsq(r2), q3 = q^3               (1 rsq, 2 mul)
//   f   = min(cA + cB rho + cC rho^2, q3) (rho = r2 q; the paper's single-min
//                                          form of Eq. 2, Sec. 4.3 footnote)
//   acc += f r                            (3 fma)
// Pairs from the outer shell of the block (some |d| = 2) are at r >= 1, so
// when eps <= 1 they take f = q3 directly.
#include "nf_internal.h"
#include "nf_kernels.h"

namespace nf {


__device__ __forceinline__ int find_cell(const int32_t *__restrict__ cs, int ncell, int s) {
    int lo = 0, hi = ncell;   // cs[lo] <= s < cs[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (cs[mid] <= s) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int wrap(int c, int K) {
    c = c % K;
    return c < 0 ? c + K : c;
}

struct Acc3 {
    float x = 0.f, y = 0.f, z = 0.f;
    float cx = 0.f, cy = 0.f, cz = 0.f;   // Kahan compensation (negated low parts)
};

template <bool COMP>
__device__ __forceinline__ void acc_add(Acc3 &a, float vx, float vy, float vz) {
    if constexpr (COMP) {
        float y = vx - a.cx; float t = a.x + y; a.cx = (t - a.x) - y; a.x = t;
        y = vy - a.cy; t = a.y + y; a.cy = (t - a.y) - y; a.y = t;
        y = vz - a.cz; t = a.z + y; a.cz = (t - a.z) - y; a.z = t;
    } else {
        a.x += vx; a.y += vy; a.z += vz;
    }
}

template <bool COMP>
__global__ void __launch_bounds__(256) k_accel_simple(const DevBox *boxes) {
    const DevBox &B = boxes[blockIdx.y];
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= B.n) return;
    const int K = B.K;
    const int32_t *__restrict__ cs = B.cell_start;
    const float4 *__restrict__ off = B.off;
    const int c = find_cell(cs, B.ncell, s);
    const int cz = c % K, cy = (c / K) % K, cx = c / (K * K);
    const float4 oi = off[s];
    const float cA = B.cA, cB = B.cB, cC = B.cC;
    const bool fast = B.outer_newton != 0;
    const bool plummer = B.plummer != 0;
    const float floor2 = B.r2floor;
    Acc3 a;
    for (int dx = -2; dx <= 2; ++dx) {
        const int nx = wrap(cx + dx, K);
        for (int dy = -2; dy <= 2; ++dy) {
            const int ny = wrap(cy + dy, K);
            const int row = (nx * K + ny) * K;
            for (int dz = -2; dz <= 2; ++dz) {
                const int nc = row + wrap(cz + dz, K);
                const int j0 = max(cs[nc], 0), j1 = min(cs[nc + 1], B.n);
                const float sx = oi.x - (float)dx, sy = oi.y - (float)dy, sz = oi.z - (float)dz;
                // f = q^3 for the outer shell (eps <= 1) and for every pair of
                // the Plummer law (whose eps_p^2 is in the r^2 floor)
                const bool outer = plummer || (fast && (dx == -2 || dx == 2 || dy == -2 ||
                                                        dy == 2 || dz == -2 || dz == 2));
                for (int j = j0; j < j1; ++j) {
                    const float4 oj = off[j];
                    const float rx = oj.x - sx, ry = oj.y - sy, rz = oj.z - sz;
                    float r2 = __builtin_fmaf(rx, rx, floor2);
                    r2 = __builtin_fmaf(ry, ry, r2);
                    r2 = __builtin_fmaf(rz, rz, r2);
                    const float q = __builtin_amdgcn_rsqf(r2);
                    const float q3 = q * q * q;
                    float f;
                    if (outer) {
                        f = q3;
                    } else {
                        const float rho = r2 * q;
                        const float poly = __builtin_fmaf(__builtin_fmaf(cC, rho, cB), rho, cA);
                        f = fminf(poly, q3);
                    }
                    acc_add<COMP>(a, f * rx, f * ry, f * rz);
                }
            }
        }
    }
    const int i = B.order[s];
    if (i < 0 || i >= B.n) return;   // never taken for a consistent binning
    float *o = B.out + 3 * (int64_t)i;
    const float sc = B.scale;
    if constexpr (COMP) {
        o[0] = (a.x - a.cx) * sc;
        o[1] = (a.y - a.cy) * sc;
        o[2] = (a.z - a.cz) * sc;
    } else {
        o[0] = a.x * sc;
        o[1] = a.y * sc;
        o[2] = a.z * sc;
    }
}

// VJP source records in sorted order, two float4 per slot: the slot's offset
// (ox, oy, oz, cz) and its caller-order cotangent gathered to it (vx, vy, vz, 0),
// so that a source is one 32-byte record.
__global__ void __launch_bounds__(256) k_gather_cot(const DevBox *boxes, float4 *cot_sorted) {
    const DevBox &B = boxes[blockIdx.y];
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= B.n) return;
    const int i = B.order[s];
    if (i < 0 || i >= B.n) return;
    const float *v = B.cot + 3 * (int64_t)i;
    cot_sorted[2 * (B.base + s)] = B.off[s];
    cot_sorted[2 * (B.base + s) + 1] = make_float4(v[0], v[1], v[2], 0.0f);
}

// VJP per pair: with r = x_j - x_i (cell widths), g = F/r and h = g'(rho)/rho,
//   xbar_i += g (v_j - v_i) + h (r . (v_j - v_i)) r.
// Inside eps: g = cA + cB rho + cC rho^2, h = cB / rho + 2 cC = cB q + 2 cC.
// Outside:    g = q^3, h = -3 q^5.
template <bool COMP>
__global__ void __launch_bounds__(256) k_vjp_simple(const DevBox *boxes,
                                                    const float4 *__restrict__ cot_sorted) {
    const DevBox &B = boxes[blockIdx.y];
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= B.n) return;
    const int K = B.K;
    const int32_t *__restrict__ cs = B.cell_start;
    const float4 *__restrict__ off = B.off;
    const float4 *__restrict__ cv = cot_sorted + 2 * B.base;   // records: offset, cotangent
    const int c = find_cell(cs, B.ncell, s);
    const int cz = c % K, cy = (c / K) % K, cx = c / (K * K);
    const float4 oi = off[s];
    const float4 vi = cv[2 * (int64_t)s + 1];
    const float cA = B.cA, cB = B.cB, cC2 = 2.0f * B.cC, cC = B.cC;
    const float eps2 = B.eps * B.eps;
    const bool fast = B.outer_newton != 0;
    const bool plummer = B.plummer != 0;
    const float floor2 = B.r2floor;
    Acc3 a;
    for (int dx = -2; dx <= 2; ++dx) {
        const int nx = wrap(cx + dx, K);
        for (int dy = -2; dy <= 2; ++dy) {
            const int ny = wrap(cy + dy, K);
            const int row = (nx * K + ny) * K;
            for (int dz = -2; dz <= 2; ++dz) {
                const int nc = row + wrap(cz + dz, K);
                const int j0 = max(cs[nc], 0), j1 = min(cs[nc + 1], B.n);
                const float sx = oi.x - (float)dx, sy = oi.y - (float)dy, sz = oi.z - (float)dz;
                // f = q^3 for the outer shell (eps <= 1) and for every pair of
                // the Plummer law (whose eps_p^2 is in the r^2 floor)
                const bool outer = plummer || (fast && (dx == -2 || dx == 2 || dy == -2 ||
                                                        dy == 2 || dz == -2 || dz == 2));
                for (int j = j0; j < j1; ++j) {
                    const float4 oj = off[j];
                    const float4 vj = cv[2 * (int64_t)j + 1];
                    const float rx = oj.x - sx, ry = oj.y - sy, rz = oj.z - sz;
                    const float ux = vj.x - vi.x, uy = vj.y - vi.y, uz = vj.z - vi.z;
                    float r2 = __builtin_fmaf(rx, rx, floor2);
                    r2 = __builtin_fmaf(ry, ry, r2);
                    r2 = __builtin_fmaf(rz, rz, r2);
                    const float q = __builtin_amdgcn_rsqf(r2);
                    const float q2 = q * q;
                    const float q3 = q2 * q;
                    float g = q3, h = -3.0f * q3 * q2;
                    if (!outer && r2 < eps2) {
                        const float rho = r2 * q;
                        g = __builtin_fmaf(__builtin_fmaf(cC, rho, cB), rho, cA);
                        h = __builtin_fmaf(cB, q, cC2);
                    }
                    float rdu = rx * ux;
                    rdu = __builtin_fmaf(ry, uy, rdu);
                    rdu = __builtin_fmaf(rz, uz, rdu);
                    const float t = h * rdu;
                    acc_add<COMP>(a, __builtin_fmaf(t, rx, g * ux), __builtin_fmaf(t, ry, g * uy),
                                  __builtin_fmaf(t, rz, g * uz));
                }
            }
        }
    }
    const int i = B.order[s];
    if (i < 0 || i >= B.n) return;   // never taken for a consistent binning
    float *o = B.out + 3 * (int64_t)i;
    const float sc = B.scale;
    if constexpr (COMP) {
        o[0] = (a.x - a.cx) * sc;
        o[1] = (a.y - a.cy) * sc;
        o[2] = (a.z - a.cz) * sc;
    } else {
        o[0] = a.x * sc;
        o[1] = a.y * sc;
        o[2] = a.z * sc;
    }
}

hipError_t accel_launch(const DevBox *d_boxes, int nbox, const ForcePlan &p, hipStream_t s) {
    if (p.max_n == 0) return hipSuccess;
    dim3 grid((unsigned)((p.max_n + 255) / 256), (unsigned)nbox);
    if (p.compensated)
        hipLaunchKernelGGL(k_accel_simple<true>, grid, dim3(256), 0, s, d_boxes);
    else
        hipLaunchKernelGGL(k_accel_simple<false>, grid, dim3(256), 0, s, d_boxes);
    return hipGetLastError();
}

hipError_t gather_cot_launch(const DevBox *d_boxes, int nbox, const ForcePlan &p, hipStream_t s) {
    if (p.max_n == 0) return hipSuccess;
    dim3 grid((unsigned)((p.max_n + 255) / 256), (unsigned)nbox);
    hipLaunchKernelGGL(k_gather_cot, grid, dim3(256), 0, s, d_boxes, p.cot_sorted);
    return hipGetLastError();
}

hipError_t vjp_launch(const DevBox *d_boxes, int nbox, const ForcePlan &p, hipStream_t s) {
    if (p.max_n == 0) return hipSuccess;
    dim3 grid((unsigned)((p.max_n + 255) / 256), (unsigned)nbox);
    hipError_t e = gather_cot_launch(d_boxes, nbox, p, s);
    if (e != hipSuccess) return e;
    if (p.compensated)
        hipLaunchKernelGGL(k_vjp_simple<true>, grid, dim3(256), 0, s, d_boxes,
                           (const float4 *)p.cot_sorted);
    else
        hipLaunchKernelGGL(k_vjp_simple<false>, grid, dim3(256), 0, s, d_boxes,
                           (const float4 *)p.cot_sorted);
    return hipGetLastError();
}

}  // namespace nf
