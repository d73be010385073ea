// Vector kernels of the PCG iteration (Supp. Eq. 2: T_dot and T_axpby), the
// slot permutation of H and vectors, and the adjoint block scatter.
//
// The iteration kernels work on groups of D0 consecutive level-0 domains
// (RG slots, one thread per DOF).  Every dot product leaves one partial per
// group; the kernel that needs the scalar sums the partials itself in a
// fixed order, so no kernel waits on other workgroups and no atomics are
// used.
#include "launch.hpp"
#include "restrict.hpp"

namespace maspcg {
namespace {

constexpr int kVecThreads = 256;

__global__ void k_state_reset(DevState* st) {
    if (threadIdx.x == 0) {
        st->rr = st->bb = st->tol2 = st->rr_true = 0.0;
        st->rho[0] = st->rho[1] = 0.0;
        st->done = st->iter = st->status = st->pad = 0;
    }
}

// Resumes the iteration after a stop that the host decided to revisit.
__global__ void k_clear_stop(DevState* st) {
    if (threadIdx.x == 0) {
        st->done = 0;
        st->status = 0;
    }
}

// rr_true = sum of the residual partials (after the final residual kernel).
__global__ void __launch_bounds__(256) k_finalize(SolverView v) {
    __shared__ double buf[256];
    const double rr = sum_partials(v.P_rr, v.G, buf);
    if (threadIdx.x == 0) v.st->rr_true = rr;
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
    if (H64) {
#pragma unroll
        for (int c = 0; c < 9; ++c) H64[(long long)c * nnzb + k] = val[c];
    }
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

// Shared memory of the group kernels: rs[3*RG] + restriction scratch + 256.
inline size_t group_smem(const SolverView& v) {
    return sizeof(double) * (3 * v.RG + restrict_smem_doubles(v.RG, v.W1, v.L) + 256);
}

// r = b, x = 0, partials of ||b||^2 (as both ||r||^2 and ||b||^2), and the
// restriction of r.
__global__ void k_init_rhs(SolverView v) {
    extern __shared__ double sm[];
    double* rs = sm;
    double* scratch = sm + 3 * v.RG + restrict_smem_doubles(v.RG, v.W1, v.L);
    const int g = xcd_group(blockIdx.x, v.G), t = threadIdx.x;
    const long long i = 3LL * g * v.RG + t;
    double bv = 0.0;
    const bool own = t < 3 * v.RG && i < 3LL * v.NS;
    if (own) bv = v.b[i];
    const RestrictLoads<> pl = restrict_load<>(v, g);
    restrict_ready(pl);
    if (own) {
        v.r[i] = bv;
        v.x[i] = 0.0;
    }
    if (t < 3 * v.RG) rs[t] = bv;
    const double bb = block_sum(bv * bv, scratch);  // its barriers also publish rs
    if (t == 0) {
        v.P_rr[g] = bb;
        v.P_bb[g] = bb;
    }
    restrict_group_any(v, g, pl, rs, sm + 3 * v.RG, v.r1, v.cpart);
}

// Iteration k: alpha = rho_{k-1} / sigma_k (sigma summed here from the group
// partials, rho_{k-1} as the SpMV of this iteration recorded it), x += alpha p,
// r -= alpha q, the partial of ||r||^2 and the restriction of the new
// residual.  sigma <= 0 stops the solve (NOT_SPD).
// Writer passes of the restriction whose plan entries k_update loads with
// its other early loads (systems whose groups write many coarse partials,
// such as affine bodies carried through many levels, take several passes).
constexpr int kUpdatePasses = 4;

__global__ void k_update(SolverView v, int k) {
    extern __shared__ double sm[];
    double* rs = sm;
    double* scratch = sm + 3 * v.RG + restrict_smem_doubles(v.RG, v.W1, v.L);
    const int g = xcd_group(blockIdx.x, v.G), t = threadIdx.x;
    // issue every independent load (the stop flag's included) before the
    // first wait, the partials of sigma first (they are needed first, and
    // loads complete in issue order); after a stop nothing is written
    const PartialLoads sig = partials_load(v.P_sigma, v.G);
    const double rho = v.st->rho[(k - 1) & 1];
    const long long i = 3LL * g * v.RG + t;
    const bool own = t < 3 * v.RG && i < 3LL * v.NS;
    const long long ic = own ? i : 0;  // unconditional loads (see partials_load)
    const double* pk = v.p[k & 1];
    const double xv = v.x[ic], pv = pk[ic], rv0 = v.r[ic], qv = v.q[ic];
    const RestrictLoads<kUpdatePasses> pl = restrict_load<kUpdatePasses>(v, g);
    const int stop = v.st->done;
    keep_loads_issued();
    if (stop) return;
    // (block_sum's first barrier orders scratch's reuse)
    const double sigma = partials_sum<false>(sig, v.P_sigma, v.G, scratch);
    if (!(sigma > 0.0) || !finite(sigma) || !finite(rho)) {
        if (g == 0 && t == 0) {
            v.st->status = (finite(sigma) && finite(rho)) ? -2 : -6;
            v.st->done = 1;
            v.st->iter = k - 1;
        }
        return;
    }
    const double alpha = rho / sigma;
    restrict_ready(pl);
    double rv = 0.0;
    if (own) {
        v.x[i] = xv + alpha * pv;
        rv = rv0 - alpha * qv;
        v.r[i] = rv;
    }
    if (t < 3 * v.RG) rs[t] = rv;
    // its barriers also publish rs; scratch is not used again
    const double rr = block_sum<false>(rv * rv, scratch);
    if (t == 0) v.P_rr[g] = rr;
    restrict_group_any(v, g, pl, rs, sm + 3 * v.RG, v.r1, v.cpart);
}

// Restriction of the current r only (preconditioner apply outside PCG).
__global__ void k_restrict(SolverView v) {
    extern __shared__ double sm[];
    double* rs = sm;
    const int g = xcd_group(blockIdx.x, v.G), t = threadIdx.x;
    const long long i = 3LL * g * v.RG + t;
    const double rv = (t < 3 * v.RG && i < 3LL * v.NS) ? v.r[i] : 0.0;
    const RestrictLoads<> pl = restrict_load<>(v, g);
    if (t < 3 * v.RG) rs[t] = rv;
    __syncthreads();
    restrict_group_any(v, g, pl, rs, sm + 3 * v.RG, v.r1, v.cpart);
}

// dL/dH_ij = -lambda_i x_j^T on every stored block, caller order and layout.
// Eight lanes per block row; consecutive lanes write consecutive blocks.
constexpr int kScatterLanes = 8;

template <typename T>
__global__ void __launch_bounds__(kVecThreads) k_adjoint_scatter(int n_rows, const int* __restrict__ rp,
                                                                  const int* __restrict__ ci,
                                                                  const double* __restrict__ lam,
                                                                  const double* __restrict__ x, T* __restrict__ out) {
    const int row = blockIdx.x * (kVecThreads / kScatterLanes) + threadIdx.x / kScatterLanes;
    const int sub = threadIdx.x % kScatterLanes;
    if (row >= n_rows) return;
    const double l0 = lam[3 * row], l1 = lam[3 * row + 1], l2 = lam[3 * row + 2];
    for (int k = rp[row] + sub; k < rp[row + 1]; k += kScatterLanes) {
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

// Group kernels run whole waves and at least 256 threads (sum_partials).
int group_threads(const SolverView& v) { return max(256, round_waves(3 * v.RG)); }

}  // namespace

hipError_t launch_state_reset(const SolverView& v, hipStream_t s) {
    launch_kernel(k_state_reset, dim3(1), dim3(64), 0, s, v.st);
    return hipGetLastError();
}

hipError_t launch_clear_stop(const SolverView& v, hipStream_t s) {
    launch_kernel(k_clear_stop, dim3(1), dim3(64), 0, s, v.st);
    return hipGetLastError();
}

hipError_t launch_finalize(const SolverView& v, hipStream_t s) {
    launch_kernel(k_finalize, dim3(1), dim3(256), 0, s, v);
    return hipGetLastError();
}

hipError_t launch_permute_H(const SolverView& v, const double* Hu, bool f32, hipStream_t s) {
    if (!v.sym || !f32) {
        launch_kernel(k_permute_H, dim3(ceil_div(v.nsb, kVecThreads)), dim3(kVecThreads), 0, s, v.nsb, v.perm_src, Hu,
                      v.H64, f32 ? v.H32 : nullptr);
    } else {  // symmetric FP64 copy, full FP32 copy
        launch_kernel(k_permute_H, dim3(ceil_div(v.nsb, kVecThreads)), dim3(kVecThreads), 0, s, v.nsb, v.perm_src, Hu,
                      v.H64, static_cast<float*>(nullptr));
        launch_kernel(k_permute_H, dim3(ceil_div(v.nnzb, kVecThreads)), dim3(kVecThreads), 0, s, v.nnzb, v.perm_full,
                      Hu, static_cast<double*>(nullptr), v.H32);
    }
    return hipGetLastError();
}

hipError_t launch_perm_in(const SolverView& v, const double* src, double* dst, hipStream_t s) {
    launch_kernel(k_perm_in, dim3(ceil_div(3LL * v.NS, kVecThreads)), dim3(kVecThreads), 0, s, v.NS, v.remap, src,
                       dst);
    return hipGetLastError();
}

hipError_t launch_perm_out(const SolverView& v, const double* src, double* dst, hipStream_t s) {
    launch_kernel(k_perm_out, dim3(ceil_div(3LL * v.V, kVecThreads)), dim3(kVecThreads), 0, s, v.V, v.map, src, dst);
    return hipGetLastError();
}

hipError_t launch_init_rhs(const SolverView& v, hipStream_t s) {
    launch_kernel(k_init_rhs, dim3(v.G), dim3(group_threads(v)), group_smem(v), s, v);
    return hipGetLastError();
}

hipError_t launch_update(const SolverView& v, int k, hipStream_t s) {
    launch_kernel(k_update, dim3(v.G), dim3(group_threads(v)), group_smem(v), s, v, k);
    return hipGetLastError();
}

hipError_t launch_restrict(const SolverView& v, hipStream_t s) {
    if (v.L < 2) return hipSuccess;
    launch_kernel(k_restrict, dim3(v.G), dim3(group_threads(v)), group_smem(v), s, v);
    return hipGetLastError();
}

hipError_t launch_adjoint_scatter(int n_rows, const int* rp, const int* ci, const double* lam, const double* x,
                                  void* out, bool f32, hipStream_t s) {
    if (n_rows <= 0) return hipSuccess;
    dim3 g(ceil_div(n_rows, kVecThreads / kScatterLanes)), b(kVecThreads);
    if (f32)
        launch_kernel(k_adjoint_scatter<float>, g, b, 0, s, n_rows, rp, ci, lam, x, static_cast<float*>(out));
    else
        launch_kernel(k_adjoint_scatter<double>, g, b, 0, s, n_rows, rp, ci, lam, x, static_cast<double*>(out));
    return hipGetLastError();
}

}  // namespace maspcg
