// Internal definitions shared by the HIP translation units of libmaspcg.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace maspcg {

// Host-visible scalars of one PCG solve in device memory.  Only block 0 of
// the kernel that decides a value writes it; the values the iteration itself
// needs (alpha, beta, rho, sigma, ||r||^2) are recomputed by every consumer
// block from per-group partial sums, so no kernel waits on another block.
struct DevState {
    double rr;       // ||r||^2 used by the last convergence test
    double bb;       // ||b||^2
    double tol2;     // tol^2 * ||b||^2
    double rr_true;  // ||b - H x||^2 from the final residual
    double rho[2];   // rho_j = r_j^T z_j in rho[j & 1], written by the SpMV of iteration j + 1
    int32_t done;    // 1: stop; later kernels of the solve return at once
    int32_t iter;    // iterations completed
    int32_t status;  // 0 ok, -2 not SPD, -6 not finite, 2 = converged on the recurrence (FP64 check pending)
    int32_t pad;
};

constexpr int kStatusConvergedRecurrence = 2;

// ------------------------------------------------------------ XCD placement

// The dispatcher deals workgroups to the 8 XCDs round-robin (workgroup b runs
// on XCD b % 8), each XCD behind its own L2.  Groups of slots that exchange
// halo entries are numbered close together by the partition, so each XCD is
// given one contiguous range of the G groups (a bijection of [0, G)) and
// neighbouring groups share that XCD's L2.
constexpr int kXcds = 8;

__host__ __device__ inline int xcd_group(int b, int G) {
    const int x = b % kXcds, i = b / kXcds;
    const int q = G / kXcds, rem = G % kXcds;
    return x * q + (x < rem ? x : rem) + i;
}

// ---------------------------------------------------------------- reductions

// x + x of the lane the DPP control selects (kCtrl: a permutation within
// each row of 16 lanes, so every source lane exists); FP64 moved as two
// 32-bit halves.
template <int kCtrl>
__device__ __forceinline__ double dpp_add(double x) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), kCtrl, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), kCtrl, 0xf, 0xf, false);
    return x + __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_value(double x, int lane) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), lane),
                            __builtin_amdgcn_readlane(__double2loint(x), lane));
}

// row16_sum: the sum over each row of 16 lanes (every lane active) in all
// of its lanes; wave_sum: over the 64 lanes of a wave, the same bits in
// every lane.  Within each row of 16 lanes, partners at distance 1 and 2 (quad
// permutations), then mirrored within each half row and within the row (at
// each step both partners hold equal values, so a + b and b + a agree), then
// the four row sums read out of lanes 0, 16, 32, 48 and added in a fixed
// order.  DPP and readlane instead of shuffles through the LDS crossbar.
__device__ inline double row16_sum(double v) {
    v = dpp_add<0xb1>(v);   // quad_perm [1, 0, 3, 2]
    v = dpp_add<0x4e>(v);   // quad_perm [2, 3, 0, 1]
    v = dpp_add<0x141>(v);  // row_half_mirror
    return dpp_add<0x140>(v);  // row_mirror
}

__device__ inline double wave_sum(double v) {
    v = row16_sum(v);
    return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

// Deterministic sum over the workgroup (whole waves only); the result is
// valid in every thread.  scratch: blockDim.x / 64 doubles of shared memory.
// kReuse = false leaves out the closing barrier, for a caller that does not
// write scratch again.
template <bool kReuse = true>
__device__ inline double block_sum(double v, double* scratch) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) scratch[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += scratch[w];
    if (kReuse) __syncthreads();
    return t;
}

// block_sum as a kernel's last reduction, into thread 0 only (same bits):
// one barrier, for a scratch that no thread has used before in the kernel.
__device__ inline double block_sum_last(double v, double* scratch) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_sum(v);
    if (lane == 0) scratch[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (blockDim.x >> 6); ++w) t += scratch[w];
    return t;
}

// Two block_sum_last reductions at once (same bits as two separate ones):
// the results in thread 0 only; scratch: 2 * blockDim.x / 64 doubles.
__device__ inline void block_sum2_last(double a, double b, double* scratch, double& sa, double& sb) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    a = wave_sum(a);
    b = wave_sum(b);
    if (lane == 0) {
        scratch[wave] = a;
        scratch[nw + wave] = b;
    }
    __syncthreads();
    sa = sb = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < nw; ++w) {
            sa += scratch[w];
            sb += scratch[nw + w];
        }
}

// Sum of n per-group partials in a fixed order that does not depend on the
// workgroup shape, so every kernel that needs the value computes the same
// bits: thread t < 256 adds p[t], p[t + 256], ... (independent loads, issued
// together), then wave 0 folds the 256 bucket sums.  Needs blockDim.x >= 256
// and buf[256] doubles of shared memory; the result is valid in every thread.
__device__ inline double sum_partials(const double* __restrict__ p, int n, double* buf) {
    const int t = threadIdx.x;
    if (t < 256) {
        double s = 0.0;
        int i = t;
        for (; i + 768 < n; i += 1024) s += (p[i] + p[i + 256]) + (p[i + 512] + p[i + 768]);
        for (; i < n; i += 256) s += p[i];
        buf[t] = s;
    }
    __syncthreads();
    if (t < 64) {
        double s = (buf[t] + buf[t + 64]) + (buf[t + 128] + buf[t + 192]);
        s = wave_sum(s);
        if (t == 0) buf[0] = s;
    }
    __syncthreads();
    const double r = buf[0];
    __syncthreads();
    return r;
}

__device__ inline bool finite(double x) { return x - x == 0.0; }

// Ends a kernel's block of early loads: an empty statement that the compiler
// must treat as touching memory, so that it keeps those loads in the order
// written, ahead of this point, instead of sinking each one into the branch
// that first uses it (behind the others).  It emits no instruction.  Uniform
// values (the stop flag) are read before it: after it the compiler no longer
// takes them for unchanged memory and reads them with a vector load, whose
// wait would then cover every load issued before.
__device__ __forceinline__ void keep_loads_issued() { asm volatile("" ::: "memory"); }

// sum_partials split in two, so that the loads can be issued early and their
// latency overlap other loads: partials_load() fetches thread t's bucket
// entries p[t], p[t + 256], ... into registers (n <= 1024), partials_sum()
// adds them in sum_partials' order (same bits) and folds the buckets.  For
// n > 1024 partials_sum() falls back to sum_partials.  Every thread issues
// its four loads unconditionally, at indices clamped to [0, n) (n >= 1), so
// that no branch separates them from the loads issued after them and a wait
// for them need not wait for those too; partials_sum() reads only the
// entries below n.
struct PartialLoads {
    double v[4];
};

__device__ inline PartialLoads partials_load(const double* __restrict__ p, int n) {
    PartialLoads L;
    const int t = threadIdx.x;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        L.v[j] = p[min(t + 256 * j, n - 1)];
    }
    return L;
}

// kReuse = false leaves out the closing barrier, for a caller whose next
// write to buf follows another barrier.
template <bool kReuse = true>
__device__ inline double partials_sum(const PartialLoads& L, const double* __restrict__ p, int n, double* buf) {
    if (n > 1024) return sum_partials(p, n, buf);
    const int t = threadIdx.x;
    if (t < 256) {  // as in partials_load: bucket t holds p[t], p[t + 256], ... below n
        double s = 0.0;
        if (t + 768 < n) {
            s += (L.v[0] + L.v[1]) + (L.v[2] + L.v[3]);
        } else {
            if (t < n) s += L.v[0];
            if (t + 256 < n) s += L.v[1];
            if (t + 512 < n) s += L.v[2];
        }
        buf[t] = s;
    }
    __syncthreads();
    if (t < 64) {
        double s = (buf[t] + buf[t + 64]) + (buf[t + 128] + buf[t + 192]);
        s = wave_sum(s);
        if (t == 0) buf[0] = s;
    }
    __syncthreads();
    const double r = buf[0];
    if (kReuse) __syncthreads();
    return r;
}

inline int ceil_div(long long a, long long b) { return static_cast<int>((a + b - 1) / b); }
inline int round_waves(int threads) { return (threads + 63) / 64 * 64; }

}  // namespace maspcg
