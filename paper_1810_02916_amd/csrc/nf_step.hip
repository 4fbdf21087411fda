// nf_step.hip -- inputs of the global time-step choice and the leapfrog
// update (Sec. 4.2: one step for all particles, bounded by a largest step in
// ln a, by eta times a per-cell v_rms / a_max ratio and by the step at which
// the fastest particle crosses 80% of a cell; the step's Kick and Drift
// stages).
//
//   k_step_parts   caller order, streaming: each particle's |a| and |v|^2
//                  (double) into one 16-byte record, so that the cell pass
//                  gathers one record per particle instead of two 12-byte
//                  vectors from two arrays;
//   k_step_cells   a wave per 8 consecutive cells over the cell-sorted
//                  slots: 8 lanes per cell when none of them holds more than
//                  64 particles, else the whole wave for each in turn; a_max
//                  and v_rms of the cell (double inside, float out) and the
//                  cell's (a_max, sum |v|^2, max |v|^2) in double scratch;
//   k_step_partial fixed cell ranges per block -> per-block partials;
//   k_step_final   one block per box -> (a_max, v_rms, v_max) in double.
//   k_choose_partial, k_choose_final
//                  the step itself: the smallest per-cell ratio, then the
//                  three bounds and their minimum, per box.
//   k_kick_drift   v <- v + kick * a (double, rounded once to float),
//                  x <- x + drift * v (double, kicked v), caller order.
// Every sum has a fixed order (lane-strided, then a fixed butterfly or
// tree), so the outputs are bitwise reproducible; no multiply-add is fused
// (contraction is off in these functions, and the products are written as
// plain operators so that the pragma covers them), so each value is the
// plain double sequence.
#include "nf_internal.h"
#include "nf_kernels.h"

namespace nf {
namespace {

constexpr int kStatThreads = 256;
constexpr int kStatWaves = kStatThreads / 64;
constexpr int kGroup = 8;         // lanes per cell (and cells per wave) for small cells
constexpr int kGroupMax = 64;     // the largest cell the 8-lane form takes

__device__ __forceinline__ double dsq3(float x, float y, float z) {
#pragma clang fp contract(off)
    const double a = x, b = y, c = z;
    return (a * a + b * b) + c * c;
}

// Butterfly over groups of W lanes (W a power of two up to 64): every lane
// of a group ends with the same value (the pairwise sums are commutative, so
// each level agrees across the pair).
template <int W>
__device__ __forceinline__ double group_sum(double x) {
    for (int o = W / 2; o >= 1; o >>= 1) x = __dadd_rn(x, __shfl_xor(x, o));
    return x;
}
template <int W>
__device__ __forceinline__ double group_max(double x) {
    for (int o = W / 2; o >= 1; o >>= 1) x = fmax(x, __shfl_xor(x, o));
    return x;
}

// |a| and |v|^2 of every particle of the box, in caller order.
__global__ void __launch_bounds__(256)
k_step_parts(const DevBox *__restrict__ boxes, const StepIO *__restrict__ io,
             PartStat *__restrict__ part) {
#pragma clang fp contract(off)
    const DevBox &B = boxes[blockIdx.y];
    const StepIO &S = io[blockIdx.y];
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= B.n) return;
    const float *a = S.acc + 3 * (int64_t)i;
    const float *v = S.vel + 3 * (int64_t)i;
    part[B.base + i] = PartStat{__dsqrt_rn(dsq3(a[0], a[1], a[2])), dsq3(v[0], v[1], v[2])};
}

// Statistics of cell c over its slots [s0, s1), taken by the W lanes of a
// group lane-strided (q = the lane's index in the group), then reduced by
// the group's butterfly; lane q == 0 writes them.
template <int W>
__device__ __forceinline__ void cell_stats(const DevBox &B, const StepIO &S,
                                           const PartStat *__restrict__ part, CellStat *scratch,
                                           int c, int s0, int s1, int q, bool valid) {
#pragma clang fp contract(off)
    double am = 0.0, v2 = 0.0, vm = 0.0;
    for (int s = s0 + q; s < s1; s += W) {
        const int i = B.order[s];
        if (i < 0 || i >= B.n) continue;   // never taken for a consistent binning
        const PartStat r = part[B.base + i];
        am = fmax(am, r.a);
        v2 = v2 + r.v2;
        vm = fmax(vm, r.v2);
    }
    am = group_max<W>(am);
    v2 = group_sum<W>(v2);
    vm = group_max<W>(vm);
    if (valid && q == 0) {
        const int cnt = s1 - s0;
        S.amax[c] = (float)am;
        S.vrms[c] = cnt > 0 ? (float)__dsqrt_rn(__ddiv_rn(v2, (double)cnt)) : 0.0f;
        scratch[B.cellbase + c] = CellStat{am, v2, vm};
    }
}

__global__ void __launch_bounds__(kStatThreads)
k_step_cells(const DevBox *__restrict__ boxes, const StepIO *__restrict__ io,
             const PartStat *__restrict__ part, CellStat *__restrict__ scratch) {
#pragma clang fp contract(off)
    const DevBox &B = boxes[blockIdx.y];
    const StepIO &S = io[blockIdx.y];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t *__restrict__ cs = B.cell_start;
    for (int cb = (blockIdx.x * kStatWaves + wave) * kGroup; cb < B.ncell;
         cb += gridDim.x * kStatWaves * kGroup) {
        // lane: cell cb + lane / 8, index lane % 8 in its group
        const int c = cb + lane / kGroup;
        const bool valid = c < B.ncell;
        const int s0 = valid ? cs[c] : 0, s1 = valid ? cs[c + 1] : 0;
        if (__all(s1 - s0 <= kGroupMax)) {
            cell_stats<kGroup>(B, S, part, scratch, c, s0, s1, lane % kGroup, valid);
        } else {   // a big cell among the eight: each cell by the whole wave
            for (int k = 0; k < kGroup && cb + k < B.ncell; ++k) {
                const int cc = cb + k;
                cell_stats<64>(B, S, part, scratch, cc, cs[cc], cs[cc + 1], lane, true);
            }
        }
    }
}

// Block b of box y reduces cells [b * chunk, (b + 1) * chunk).
__global__ void __launch_bounds__(kStatThreads)
k_step_partial(const DevBox *__restrict__ boxes, const CellStat *__restrict__ scratch,
               CellStat *__restrict__ partial) {
    __shared__ CellStat red[kStatThreads];
    const DevBox &B = boxes[blockIdx.y];
    const int t = threadIdx.x;
    const int chunk = (B.ncell + kStepBlocks - 1) / kStepBlocks;
    const int c0 = blockIdx.x * chunk, c1 = min(B.ncell, c0 + chunk);
    CellStat r{0.0, 0.0, 0.0};
    for (int c = c0 + t; c < c1; c += kStatThreads) {
        const CellStat x = scratch[B.cellbase + c];
        r.amax = fmax(r.amax, x.amax);
        r.v2sum = __dadd_rn(r.v2sum, x.v2sum);
        r.vmax2 = fmax(r.vmax2, x.vmax2);
    }
    red[t] = r;
    __syncthreads();
    for (int h = kStatThreads / 2; h >= 1; h >>= 1) {
        if (t < h) {
            red[t].amax = fmax(red[t].amax, red[t + h].amax);
            red[t].v2sum = __dadd_rn(red[t].v2sum, red[t + h].v2sum);
            red[t].vmax2 = fmax(red[t].vmax2, red[t + h].vmax2);
        }
        __syncthreads();
    }
    if (t == 0) partial[(int64_t)blockIdx.y * kStepBlocks + blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(kStepBlocks)
k_step_final(const DevBox *__restrict__ boxes, const CellStat *__restrict__ partial,
             double *__restrict__ glob) {
    __shared__ CellStat red[kStepBlocks];
    const DevBox &B = boxes[blockIdx.x];
    const int t = threadIdx.x;
    red[t] = partial[(int64_t)blockIdx.x * kStepBlocks + t];
    __syncthreads();
    for (int h = kStepBlocks / 2; h >= 1; h >>= 1) {
        if (t < h) {
            red[t].amax = fmax(red[t].amax, red[t + h].amax);
            red[t].v2sum = __dadd_rn(red[t].v2sum, red[t + h].v2sum);
            red[t].vmax2 = fmax(red[t].vmax2, red[t + h].vmax2);
        }
        __syncthreads();
    }
    if (t == 0) {
        double *g = glob + 3 * (int64_t)blockIdx.x;
        g[0] = red[0].amax;
        g[1] = B.n > 0 ? __dsqrt_rn(__ddiv_rn(red[0].v2sum, (double)B.n)) : 0.0;
        g[2] = __dsqrt_rn(red[0].vmax2);
    }
}

// Step choice, stage 1: block b of box y takes the smallest v_rms / a_max
// over the cells of its fixed range whose a_max is positive (+inf if none),
// each ratio one double division of the stored float values.
__global__ void __launch_bounds__(kStatThreads)
k_choose_partial(const DevBox *__restrict__ boxes, const StepIO *__restrict__ io,
                 double *__restrict__ partial) {
    __shared__ double red[kStatThreads];
    const DevBox &B = boxes[blockIdx.y];
    const StepIO &S = io[blockIdx.y];
    const int t = threadIdx.x;
    const int chunk = (B.ncell + kStepBlocks - 1) / kStepBlocks;
    const int c0 = blockIdx.x * chunk, c1 = min(B.ncell, c0 + chunk);
    double r = __longlong_as_double(0x7ff0000000000000ll);   // +inf
    for (int c = c0 + t; c < c1; c += kStatThreads) {
        const float am = S.amax_in[c];
        if (am > 0.0f) r = fmin(r, __ddiv_rn((double)S.vrms_in[c], (double)am));
    }
    red[t] = r;
    __syncthreads();
    for (int h = kStatThreads / 2; h >= 1; h >>= 1) {
        if (t < h) red[t] = fmin(red[t], red[t + h]);
        __syncthreads();
    }
    if (t == 0) partial[(int64_t)blockIdx.y * kStepBlocks + blockIdx.x] = red[0];
}

// Step choice, stage 2 (Sec. 4.2), one block per box: the cell ratio is the
// smallest partial; then
//   b0 = dlna_max / hubble                       (largest step in ln a)
//   b1 = eta * max(cell ratio, v_rms / a_max)    (the global ratio protects
//                                                  against cold cells)
//   b2 = (0.8 * cell width) / v_max              (80% of a cell)
//   b3 = min(b0, b1, b2)
// with +inf for a ratio whose denominator is zero.
__global__ void __launch_bounds__(kStepBlocks)
k_choose_final(const DevBox *__restrict__ boxes, const double *__restrict__ partial,
               const double *__restrict__ glob, StepChoice ch, double *__restrict__ bounds) {
#pragma clang fp contract(off)
    __shared__ double red[kStepBlocks];
    const DevBox &B = boxes[blockIdx.x];
    const int t = threadIdx.x;
    red[t] = partial[(int64_t)blockIdx.x * kStepBlocks + t];
    __syncthreads();
    for (int h = kStepBlocks / 2; h >= 1; h >>= 1) {
        if (t < h) red[t] = fmin(red[t], red[t + h]);
        __syncthreads();
    }
    if (t == 0) {
        const double inf = __longlong_as_double(0x7ff0000000000000ll);
        const double *g = glob + 3 * (int64_t)blockIdx.x;
        const double gratio = g[0] > 0.0 ? __ddiv_rn(g[1], g[0]) : inf;
        const double b0 = __ddiv_rn(ch.dlna_max, ch.hubble);
        const double b1 = ch.eta * fmax(red[0], gratio);
        const double b2 = g[2] > 0.0 ? __ddiv_rn(0.8 * B.cellw, g[2]) : inf;
        double *o = bounds + 4 * (int64_t)blockIdx.x;
        o[0] = b0;
        o[1] = b1;
        o[2] = b2;
        o[3] = fmin(fmin(b0, b1), b2);
    }
}

__global__ void __launch_bounds__(256)
k_kick_drift(const DevBox *__restrict__ boxes, const StepIO *__restrict__ io, double kick,
             double drift) {
#pragma clang fp contract(off)   // the update is a multiply then an add, as defined
    const DevBox &B = boxes[blockIdx.y];
    const StepIO &S = io[blockIdx.y];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < B.n;
         i += (int64_t)gridDim.x * 256) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double a = S.acc[3 * i + k];
            const double v = S.vel_rw[3 * i + k];
            const float vn = (float)(v + kick * a);
            S.vel_rw[3 * i + k] = vn;
            S.pos_rw[3 * i + k] = S.pos_rw[3 * i + k] + drift * (double)vn;
        }
    }
}

}  // namespace

hipError_t step_stats_launch(const DevBox *d_boxes, const StepIO *d_io, int nbox,
                             int64_t max_n, int64_t max_ncell, PartStat *part,
                             CellStat *scratch, CellStat *partial, double *glob, hipStream_t s) {
    hipError_t e;
    if (max_n > 0) {
        hipLaunchKernelGGL(k_step_parts, dim3((unsigned)((max_n + 255) / 256), (unsigned)nbox),
                           dim3(256), 0, s, d_boxes, d_io, part);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const int64_t nb = (max_ncell + kStatWaves * kGroup - 1) / (kStatWaves * kGroup);
    const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>(nb, 8192));
    hipLaunchKernelGGL(k_step_cells, dim3(gx, (unsigned)nbox), dim3(kStatThreads), 0, s, d_boxes,
                       d_io, (const PartStat *)part, scratch);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_step_partial, dim3(kStepBlocks, (unsigned)nbox), dim3(kStatThreads), 0, s,
                       d_boxes, (const CellStat *)scratch, partial);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_step_final, dim3((unsigned)nbox), dim3(kStepBlocks), 0, s, d_boxes,
                       (const CellStat *)partial, glob);
    return hipGetLastError();
}

hipError_t step_choose_launch(const DevBox *d_boxes, const StepIO *d_io, int nbox,
                              double *partial, const double *glob, const StepChoice &ch,
                              double *bounds, hipStream_t s) {
    hipLaunchKernelGGL(k_choose_partial, dim3(kStepBlocks, (unsigned)nbox), dim3(kStatThreads), 0,
                       s, d_boxes, d_io, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_choose_final, dim3((unsigned)nbox), dim3(kStepBlocks), 0, s, d_boxes,
                       (const double *)partial, glob, ch, bounds);
    return hipGetLastError();
}

hipError_t kick_drift_launch(const DevBox *d_boxes, const StepIO *d_io, int nbox, int64_t max_n,
                             double kick, double drift, hipStream_t s) {
    const int64_t nb = (max_n + 255) / 256;
    const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>(nb, 16384));
    hipLaunchKernelGGL(k_kick_drift, dim3(gx, (unsigned)nbox), dim3(256), 0, s, d_boxes, d_io,
                       kick, drift);
    return hipGetLastError();
}

}  // namespace nf
