// 3x3-block CSR sparse matrix-vector products (Supp. Eq. 2: T_spmv of a PCG
// iteration).  A group of kSpmvLanes lanes owns one block row: lane k takes
// blocks k, k + L, ... of the row, so the lanes of a group stream adjacent
// blocks; the three row sums are then combined across the group with lane
// shuffles in a fixed order.  Products are accumulated in FP64; FP32-stored
// values are widened on load.
#include "launch.hpp"

namespace maspcg {
namespace {

// Block values: caller layout (9 consecutive values per block) or the
// solver's planar layout (value c of block k at c * stride + k).
template <typename T, bool kPlanar>
struct Blocks {
    const T* __restrict__ v;
    long long stride;
    __device__ __forceinline__ double at(int k, int c) const {
        return kPlanar ? static_cast<double>(v[c * stride + k]) : static_cast<double>(v[9LL * k + c]);
    }
};

// y(row) = sum_k H(row, k) x(col k), valid in lane 0 of the group.
template <typename T, bool kPlanar>
__device__ __forceinline__ void row_product(const int* __restrict__ rp, const int* __restrict__ ci, Blocks<T, kPlanar> H,
                                            const double* __restrict__ x, int row, int sub, double& y0, double& y1,
                                            double& y2) {
    y0 = y1 = y2 = 0.0;
    const int beg = rp[row], end = rp[row + 1];
    for (int k = beg + sub; k < end; k += kSpmvLanes) {
        const int j = ci[k];
        const double x0 = x[3 * j], x1 = x[3 * j + 1], x2 = x[3 * j + 2];
        y0 += H.at(k, 0) * x0 + H.at(k, 1) * x1 + H.at(k, 2) * x2;
        y1 += H.at(k, 3) * x0 + H.at(k, 4) * x1 + H.at(k, 5) * x2;
        y2 += H.at(k, 6) * x0 + H.at(k, 7) * x1 + H.at(k, 8) * x2;
    }
#pragma unroll
    for (int o = kSpmvLanes / 2; o > 0; o >>= 1) {
        y0 += __shfl_xor(y0, o, kSpmvLanes);
        y1 += __shfl_xor(y1, o, kSpmvLanes);
        y2 += __shfl_xor(y2, o, kSpmvLanes);
    }
}

template <typename T>
__global__ void __launch_bounds__(kSpmvThreads) k_spmv_user(int n_rows, const int* __restrict__ rp,
                                                             const int* __restrict__ ci, const T* __restrict__ val,
                                                             const double* __restrict__ x, double* __restrict__ y) {
    const int row = blockIdx.x * kSpmvRows + threadIdx.x / kSpmvLanes;
    const int sub = threadIdx.x % kSpmvLanes;
    if (row >= n_rows) return;
    double y0, y1, y2;
    row_product<T, false>(rp, ci, Blocks<T, false>{val, 0}, x, row, sub, y0, y1, y2);
    if (sub == 0) {
        y[3 * row] = y0;
        y[3 * row + 1] = y1;
        y[3 * row + 2] = y2;
    }
}

// PCG step q = H p with sigma = p^T q; the last workgroup forms
// alpha = rho / sigma (or flags a breakdown when sigma <= 0).
template <typename T>
__global__ void __launch_bounds__(kSpmvThreads) k_spmv_pq(SolverView v, const T* __restrict__ H) {
    __shared__ double scratch[kSpmvThreads / 64];
    if (v.st->done) return;
    const int row = blockIdx.x * kSpmvRows + threadIdx.x / kSpmvLanes;
    const int sub = threadIdx.x % kSpmvLanes;
    double part = 0.0;
    if (row < v.NS) {
        double y0, y1, y2;
        row_product<T, true>(v.rp0, v.ci0, Blocks<T, true>{H, v.nnzb}, v.p, row, sub, y0, y1, y2);
        if (sub == 0) {
            v.q[3 * row] = y0;
            v.q[3 * row + 1] = y1;
            v.q[3 * row + 2] = y2;
            part = v.p[3 * row] * y0 + v.p[3 * row + 1] * y1 + v.p[3 * row + 2] * y2;
        }
    }
    double in[1] = {part}, out[1];
    if (grid_reduce<1>(in, v.partials, &v.st->counter[kCntSpmv], out, scratch) && threadIdx.x == 0) {
        DevState* st = v.st;
        const double sigma = out[0];
        st->sigma = sigma;
        if (!(sigma > 0.0) || !finite(sigma)) {
            st->status = finite(sigma) ? -2 : -6;
            st->done = 1;
        } else {
            st->alpha = st->rho / sigma;
        }
    }
}

// out = b - H x in FP64 (slot order), with ||out||^2 and ||b||^2.
//  init:     out = r; sets rr, bb, tol2 and stops at once if b = 0 or x0 already converged
//  periodic: out = r (residual replacement); skipped after a stop; a stop if converged
//  confirm:  out = r; decides convergence on the FP64 residual (runs even after a stop)
//  final:    out = scratch; records rr_true only
template <int kMode>
__global__ void __launch_bounds__(kSpmvThreads) k_residual(SolverView v, double tol, double* __restrict__ out) {
    __shared__ double scratch[kSpmvThreads / 64];
    if (kMode == kResidPeriodic && v.st->done) return;
    const int row = blockIdx.x * kSpmvRows + threadIdx.x / kSpmvLanes;
    const int sub = threadIdx.x % kSpmvLanes;
    double rr = 0.0, bb = 0.0;
    if (row < v.NS) {
        double y0, y1, y2;
        row_product<double, true>(v.rp0, v.ci0, Blocks<double, true>{v.H64, v.nnzb}, v.x, row, sub, y0, y1, y2);
        if (sub == 0) {
            const double e0 = v.b[3 * row] - y0, e1 = v.b[3 * row + 1] - y1, e2 = v.b[3 * row + 2] - y2;
            out[3 * row] = e0;
            out[3 * row + 1] = e1;
            out[3 * row + 2] = e2;
            rr = e0 * e0 + e1 * e1 + e2 * e2;
            bb = v.b[3 * row] * v.b[3 * row] + v.b[3 * row + 1] * v.b[3 * row + 1] + v.b[3 * row + 2] * v.b[3 * row + 2];
        }
    }
    double in[2] = {rr, bb}, tot[2];
    if (grid_reduce<2>(in, v.partials, &v.st->counter[kCntResid], tot, scratch) && threadIdx.x == 0) {
        DevState* st = v.st;
        st->rr_true = tot[0];
        if (kMode == kResidFinal) return;
        st->rr = tot[0];
        if (kMode == kResidInit) {
            st->bb = tot[1];
            st->tol2 = tol * tol * tot[1];
            if (tot[1] == 0.0 || tot[0] <= st->tol2) st->done = 1;
            if (!finite(tot[0]) || !finite(tot[1])) {
                st->status = -6;
                st->done = 1;
            }
            return;
        }
        if (!finite(tot[0])) {
            st->status = -6;
            st->done = 1;
        } else if (tot[0] <= st->tol2) {
            st->status = 0;
            st->done = 1;
        } else if (kMode == kResidConfirm) {
            st->status = 0;
            st->done = 0;
        }
    }
}

}  // namespace

int grid_spmv_rows(int rows) { return ceil_div(rows, kSpmvRows); }

hipError_t launch_spmv_user(int n_rows, const int* rp, const int* ci, const void* val, bool f32, const double* x,
                            double* y, hipStream_t s) {
    if (n_rows <= 0) return hipSuccess;
    dim3 g(grid_spmv_rows(n_rows)), b(kSpmvThreads);
    if (f32)
        hipLaunchKernelGGL(k_spmv_user<float>, g, b, 0, s, n_rows, rp, ci, static_cast<const float*>(val), x, y);
    else
        hipLaunchKernelGGL(k_spmv_user<double>, g, b, 0, s, n_rows, rp, ci, static_cast<const double*>(val), x, y);
    return hipGetLastError();
}

hipError_t launch_spmv_pq(const SolverView& v, bool f32, hipStream_t s) {
    dim3 g(grid_spmv_rows(v.NS)), b(kSpmvThreads);
    if (f32)
        hipLaunchKernelGGL(k_spmv_pq<float>, g, b, 0, s, v, static_cast<const float*>(v.H32));
    else
        hipLaunchKernelGGL(k_spmv_pq<double>, g, b, 0, s, v, static_cast<const double*>(v.H64));
    return hipGetLastError();
}

hipError_t launch_residual(const SolverView& v, int mode, double tol, double* out, hipStream_t s) {
    dim3 g(grid_spmv_rows(v.NS)), b(kSpmvThreads);
    switch (mode) {
        case kResidInit: hipLaunchKernelGGL(k_residual<kResidInit>, g, b, 0, s, v, tol, out); break;
        case kResidPeriodic: hipLaunchKernelGGL(k_residual<kResidPeriodic>, g, b, 0, s, v, tol, out); break;
        case kResidConfirm: hipLaunchKernelGGL(k_residual<kResidConfirm>, g, b, 0, s, v, tol, out); break;
        default: hipLaunchKernelGGL(k_residual<kResidFinal>, g, b, 0, s, v, tol, out); break;
    }
    return hipGetLastError();
}

}  // namespace maspcg
