// Internal definitions shared by the HIP translation units of libmaspcg.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace maspcg {

// Scalars of one PCG solve, resident in device memory.  Kernels read alpha /
// beta produced by the previous kernel on the stream; the last workgroup of a
// reducing kernel writes them (see grid_reduce).
struct DevState {
    double rho;      // r^T z of the current iterate
    double sigma;    // p^T H p
    double alpha, beta;
    double rr;       // ||r||^2 (recurrence or replaced)
    double bb;       // ||b||^2
    double tol2;     // tol^2 * ||b||^2
    double rr_true;  // ||b - H x||^2 from the last residual kernel
    int32_t done;    // 1: stop (converged, breakdown or empty rhs); later kernels exit at once
    int32_t iter;    // iterations completed
    int32_t status;  // 0 ok, -2 not SPD, -6 not finite, 2 = converged on the recurrence, needs FP64 check
    int32_t check;   // 1: the convergence test uses rr_true (set by the host before a residual kernel)
    uint32_t counter[8];  // arrival counters of grid_reduce, one per kernel kind
};

enum Counter { kCntSpmv = 0, kCntUpdate = 1, kCntApply = 2, kCntResid = 3, kCntInit = 4, kCntDot = 5 };

constexpr int kStatusConvergedRecurrence = 2;

// ---------------------------------------------------------------- reductions

template <int W = 64>
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
    return v;
}

// Deterministic sum over the workgroup; the result is valid in every thread.
// scratch: at least blockDim.x / 64 doubles of shared memory.
__device__ inline double block_sum(double v, double* scratch) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) scratch[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += scratch[w];
    __syncthreads();
    return t;
}

// Two-stage deterministic grid reduction of K values per workgroup.  Every
// workgroup stores its partials; the workgroup that arrives last adds all
// partials in a fixed order and returns true (with the totals in out[],
// valid in all its threads).  The arrival counter is reset for the next
// launch by that last workgroup.
template <int K>
__device__ inline bool grid_reduce(const double (&v)[K], double* partials, uint32_t* counter, double (&out)[K],
                                   double* scratch) {
    __shared__ int is_last;
    double bs[K];
#pragma unroll
    for (int k = 0; k < K; ++k) bs[k] = block_sum(v[k], scratch);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            __hip_atomic_store(&partials[(size_t)k * gridDim.x + blockIdx.x], bs[k], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        const uint32_t arrived = atomicAdd(counter, 1u);
        is_last = (arrived == gridDim.x - 1);
    }
    __syncthreads();
    if (!is_last) return false;
    __threadfence();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double t = 0.0;
        for (unsigned b = threadIdx.x; b < gridDim.x; b += blockDim.x)
            t += __hip_atomic_load(&partials[(size_t)k * gridDim.x + b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        out[k] = block_sum(t, scratch);
    }
    if (threadIdx.x == 0) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

__device__ inline bool finite(double x) { return x - x == 0.0; }

// ------------------------------------------------------------------ host side

constexpr int kSpmvLanes = 8;           // lanes per block row in the row kernels
constexpr int kSpmvThreads = 256;       // workgroup size of the row kernels
constexpr int kSpmvRows = kSpmvThreads / kSpmvLanes;

inline int ceil_div(long long a, long long b) { return static_cast<int>((a + b - 1) / b); }

}  // namespace maspcg
