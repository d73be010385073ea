// Vector kernels of the PCG iteration (Supp. Eq. 2: T_dot and T_axpby), the
// slot permutation of H and vectors, and the adjoint block scatter.
#include "launch.hpp"

namespace maspcg {
namespace {

constexpr int kVecThreads = 256;
constexpr int kInitGrid = 1024;

__global__ void k_state_reset(DevState* st) {
    if (threadIdx.x == 0) {
        st->rho = st->sigma = st->alpha = st->beta = 0.0;
        st->rr = st->bb = st->tol2 = st->rr_true = 0.0;
        st->done = st->iter = st->status = st->check = 0;
        for (int k = 0; k < 8; ++k) st->counter[k] = 0u;
    }
}

// Caller-ordered FP64 blocks -> slot-ordered planar FP64 (and FP32) copies.
__global__ void __launch_bounds__(kVecThreads) k_permute_H(int nnzb, const int* __restrict__ src,
                                                            const double* __restrict__ Hu, double* __restrict__ H64,
                                                            float* __restrict__ H32) {
    const int k = blockIdx.x * kVecThreads + threadIdx.x;
    if (k >= nnzb) return;
    const double* blk = Hu + 9LL * src[k];
    double val[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) val[c] = blk[c];
#pragma unroll
    for (int c = 0; c < 9; ++c) H64[(long long)c * nnzb + k] = val[c];
    if (H32) {
#pragma unroll
        for (int c = 0; c < 9; ++c) H32[(long long)c * nnzb + k] = static_cast<float>(val[c]);
    }
}

// slot-ordered dst[3s + c] = src[3 remap[s] + c], zero on padded slots
__global__ void __launch_bounds__(kVecThreads) k_perm_in(int NS, const int* __restrict__ remap,
                                                          const double* __restrict__ src, double* __restrict__ dst) {
    const int t = blockIdx.x * kVecThreads + threadIdx.x;
    if (t >= 3 * NS) return;
    const int node = remap[t / 3];
    dst[t] = node >= 0 ? src[3 * node + t % 3] : 0.0;
}

// node-ordered dst[3i + c] = src[3 map[i] + c]
__global__ void __launch_bounds__(kVecThreads) k_perm_out(int V, const int* __restrict__ map,
                                                           const double* __restrict__ src, double* __restrict__ dst) {
    const int t = blockIdx.x * kVecThreads + threadIdx.x;
    if (t >= 3 * V) return;
    dst[t] = src[3 * map[t / 3] + t % 3];
}

// r = b, x = 0, ||b||^2; sets bb, rr, tol2 and stops at once when b = 0.
__global__ void __launch_bounds__(kVecThreads) k_init_rhs(SolverView v, double tol) {
    __shared__ double scratch[kVecThreads / 64];
    const int n = 3 * v.NS;
    double bb = 0.0;
    for (int t = blockIdx.x * kVecThreads + threadIdx.x; t < n; t += gridDim.x * kVecThreads) {
        const double bv = v.b[t];
        v.r[t] = bv;
        v.x[t] = 0.0;
        bb += bv * bv;
    }
    double in[1] = {bb}, out[1];
    if (grid_reduce<1>(in, v.partials, &v.st->counter[kCntInit], out, scratch) && threadIdx.x == 0) {
        DevState* st = v.st;
        st->bb = out[0];
        st->rr = out[0];
        st->rr_true = out[0];
        st->tol2 = tol * tol * out[0];
        if (out[0] == 0.0) st->done = 1;
        if (!finite(out[0])) {
            st->status = -6;
            st->done = 1;
        }
    }
}

// Domains per workgroup of the domain-aligned vector kernels (3 * D * N <= 192 lanes in use).
__host__ __device__ inline int update_domains(int N) { return N >= 64 ? 1 : (64 / N > 0 ? 64 / N : 1); }

// x += alpha p, r -= alpha q, ||r||^2, and the restriction r_1 = C_1 r of the
// updated residual: each level-1 supernode is summed by the lowest slot of
// its level-0 domain that belongs to it (no atomics, fixed order).  With
// kRestrictOnly the vectors are left unchanged and only r_1 is formed.
template <bool kRestrictOnly>
__global__ void k_update(SolverView v, int mixed) {
    extern __shared__ double sm[];
    const int D = update_domains(v.N);
    const int slots = D * v.N;
    double* rs = sm;                                    // [3 * slots]
    int* up = reinterpret_cast<int*>(sm + 3 * slots);   // [slots]
    double* scratch = sm + 3 * slots + (slots + 1) / 2; // [4]
    if (!kRestrictOnly && v.st->done) return;
    const int t = threadIdx.x;
    const int ls = t / 3, c = t % 3;
    const int slot = blockIdx.x * slots + ls;
    const bool valid = ls < slots && slot < v.NS;
    const int dof = 3 * slot + c;
    double rv = 0.0;
    if (valid) {
        if (kRestrictOnly) {
            rv = v.r[dof];
        } else {
            const double alpha = v.st->alpha;
            v.x[dof] += alpha * v.p[dof];
            rv = v.r[dof] - alpha * v.q[dof];
            v.r[dof] = rv;
        }
    }
    if (v.L > 1) {
        if (ls < slots) rs[t] = rv;
        if (c == 0 && ls < slots) up[ls] = valid ? v.anc[slot] : -1;
        __syncthreads();
        if (valid) {
            const int u = v.lead1[slot];
            if (u >= 0) {
                const int first = (ls / v.N) * v.N;
                double s = 0.0;
                for (int a = 0; a < v.N; ++a)
                    if (up[first + a] == u) s += rs[3 * (first + a) + c];
                v.r1[3 * u + c] = s;
            }
        }
    }
    if (kRestrictOnly) return;
    double in[1] = {rv * rv}, out[1];
    if (grid_reduce<1>(in, v.partials, &v.st->counter[kCntUpdate], out, scratch) && threadIdx.x == 0) {
        DevState* st = v.st;
        st->rr = out[0];
        st->iter += 1;
        if (!finite(out[0])) {
            st->status = -6;
            st->done = 1;
        } else if (out[0] <= st->tol2) {
            st->status = mixed ? kStatusConvergedRecurrence : 0;
            st->done = 1;
        }
    }
}

// p = z + beta p (first = 1: p = z, p holds no earlier direction)
__global__ void __launch_bounds__(kVecThreads) k_update_p(SolverView v, int first) {
    if (v.st->done) return;
    const int t = blockIdx.x * kVecThreads + threadIdx.x;
    if (t >= 3 * v.NS) return;
    if (first) {
        v.p[t] = v.z[t];
    } else {
        const double beta = v.st->beta;
        v.p[t] = v.z[t] + beta * v.p[t];
    }
}

// dL/dH_ij = -lambda_i x_j^T on every stored block, caller order and layout.
template <typename T>
__global__ void __launch_bounds__(kSpmvThreads) k_adjoint_scatter(int n_rows, const int* __restrict__ rp,
                                                                   const int* __restrict__ ci,
                                                                   const double* __restrict__ lam,
                                                                   const double* __restrict__ x, T* __restrict__ out) {
    const int row = blockIdx.x * kSpmvRows + threadIdx.x / kSpmvLanes;
    const int sub = threadIdx.x % kSpmvLanes;
    if (row >= n_rows) return;
    const double l0 = lam[3 * row], l1 = lam[3 * row + 1], l2 = lam[3 * row + 2];
    for (int k = rp[row] + sub; k < rp[row + 1]; k += kSpmvLanes) {
        const int j = ci[k];
        const double x0 = x[3 * j], x1 = x[3 * j + 1], x2 = x[3 * j + 2];
        T* o = out + 9LL * k;
        o[0] = static_cast<T>(-l0 * x0);
        o[1] = static_cast<T>(-l0 * x1);
        o[2] = static_cast<T>(-l0 * x2);
        o[3] = static_cast<T>(-l1 * x0);
        o[4] = static_cast<T>(-l1 * x1);
        o[5] = static_cast<T>(-l1 * x2);
        o[6] = static_cast<T>(-l2 * x0);
        o[7] = static_cast<T>(-l2 * x1);
        o[8] = static_cast<T>(-l2 * x2);
    }
}

}  // namespace

int grid_update(int M, int N) { return ceil_div(M, update_domains(N)); }
int grid_vector(int n) { return ceil_div(n, kVecThreads); }

hipError_t launch_state_reset(const SolverView& v, hipStream_t s) {
    hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(64), 0, s, v.st);
    return hipGetLastError();
}

hipError_t launch_permute_H(const SolverView& v, const double* Hu, bool f32, hipStream_t s) {
    hipLaunchKernelGGL(k_permute_H, dim3(grid_vector(v.nnzb)), dim3(kVecThreads), 0, s, v.nnzb, v.perm_src, Hu, v.H64,
                       f32 ? v.H32 : nullptr);
    return hipGetLastError();
}

hipError_t launch_perm_in(const SolverView& v, const double* src, double* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_perm_in, dim3(grid_vector(3 * v.NS)), dim3(kVecThreads), 0, s, v.NS, v.remap, src, dst);
    return hipGetLastError();
}

hipError_t launch_perm_out(const SolverView& v, const double* src, double* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_perm_out, dim3(grid_vector(3 * v.V)), dim3(kVecThreads), 0, s, v.V, v.map, src, dst);
    return hipGetLastError();
}

hipError_t launch_init_rhs(const SolverView& v, double tol, hipStream_t s) {
    int g = grid_vector(3 * v.NS);
    if (g > kInitGrid) g = kInitGrid;
    hipLaunchKernelGGL(k_init_rhs, dim3(g), dim3(kVecThreads), 0, s, v, tol);
    return hipGetLastError();
}

hipError_t launch_update(const SolverView& v, bool restrict_only, bool mixed, hipStream_t s) {
    const int D = update_domains(v.N);
    const int slots = D * v.N;
    const int threads = (3 * slots + 63) / 64 * 64;  // whole waves: shuffle reductions need every lane live
    const size_t shmem = sizeof(double) * (3 * slots + (slots + 1) / 2 + 4);
    dim3 g(grid_update(v.M, v.N)), b(threads);
    if (restrict_only)
        hipLaunchKernelGGL(k_update<true>, g, b, shmem, s, v, mixed ? 1 : 0);
    else
        hipLaunchKernelGGL(k_update<false>, g, b, shmem, s, v, mixed ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_update_p(const SolverView& v, bool first, hipStream_t s) {
    hipLaunchKernelGGL(k_update_p, dim3(grid_vector(3 * v.NS)), dim3(kVecThreads), 0, s, v, first ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_adjoint_scatter(int n_rows, const int* rp, const int* ci, const double* lam, const double* x,
                                  void* out, bool f32, hipStream_t s) {
    if (n_rows <= 0) return hipSuccess;
    dim3 g(grid_spmv_rows(n_rows)), b(kSpmvThreads);
    if (f32)
        hipLaunchKernelGGL(k_adjoint_scatter<float>, g, b, 0, s, n_rows, rp, ci, lam, x, static_cast<float*>(out));
    else
        hipLaunchKernelGGL(k_adjoint_scatter<double>, g, b, 0, s, n_rows, rp, ci, lam, x, static_cast<double*>(out));
    return hipGetLastError();
}

}  // namespace maspcg
