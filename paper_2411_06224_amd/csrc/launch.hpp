// Host launchers of the HIP kernels and their argument blocks.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"

namespace maspcg {

constexpr int kMaxLv = 16;

// Device views of the solver's data in the caller's workspace.
struct SolverView {
    int V, N, M, NS, L, nnzb;
    int units[kMaxLv];
    int ndom[kMaxLv];
    // plans
    const int* remap;     // [NS]
    const int* map;       // [V]
    const int* perm_src;  // [nnzb] caller block of each slot-ordered block
    const int* rp0;       // [NS+1]
    const int* ci0;       // [nnzb]
    const int* lead1;     // [NS]
    const int* anc;       // [(L-1)*NS]
    const int* mem_ptr[kMaxLv];
    const int* mem_idx[kMaxLv];
    // slot-ordered matrix (9 planes of nnzb values)
    double* H64;
    float* H32;
    // inverses per level, column-major (3N)^2 per domain
    double* inv64[kMaxLv];
    float* inv32[kMaxLv];
    // vectors in slot order (3*NS doubles)
    double *b, *x, *r, *z, *p, *q;
    // coarse vectors: r1 [3*units[1]], y_l [3*ndom[l]*N] for l >= 1
    double* r1;
    double* y[kMaxLv];
    double* partials;  // 2 * max grid
    DevState* st;
    int* flag;         // inversion status
};

// Build-phase views.
struct BuildView {
    int L, N, nnzb;
    int units[kMaxLv];
    int ndom[kMaxLv];
    int nnzA[kMaxLv];
    const int* red_ptr[kMaxLv];  // level l >= 1
    const int* red_src[kMaxLv];  // level 1: caller block indices
    const int* dom_ptr[kMaxLv];
    const int* dom_blk[kMaxLv];  // level 0: caller block indices
    const int* dom_ab[kMaxLv];
    const int* remap;
    double* A[kMaxLv];           // level l >= 1: 9 planes of nnzA[l]
    double* inv64[kMaxLv];
    float* inv32[kMaxLv];
    int* flag;
};

enum ResidMode { kResidInit = 0, kResidPeriodic = 1, kResidConfirm = 2, kResidFinal = 3 };
enum ApplyMode { kApplyPlain = 0, kApplyInit = 1, kApplyIter = 2 };

// spmv.hip
hipError_t launch_spmv_user(int n_rows, const int* rp, const int* ci, const void* val, bool f32, const double* x,
                            double* y, hipStream_t s);
hipError_t launch_spmv_pq(const SolverView& v, bool f32, hipStream_t s);
hipError_t launch_residual(const SolverView& v, int mode, double tol, double* out, hipStream_t s);

// vectors.hip
hipError_t launch_state_reset(const SolverView& v, hipStream_t s);
hipError_t launch_permute_H(const SolverView& v, const double* Hu, bool f32, hipStream_t s);
hipError_t launch_perm_in(const SolverView& v, const double* src, double* dst, hipStream_t s);
hipError_t launch_perm_out(const SolverView& v, const double* src, double* dst, hipStream_t s);
hipError_t launch_init_rhs(const SolverView& v, double tol, hipStream_t s);
hipError_t launch_update(const SolverView& v, bool restrict_only, bool mixed, hipStream_t s);
hipError_t launch_update_p(const SolverView& v, bool first, hipStream_t s);
hipError_t launch_adjoint_scatter(int n_rows, const int* rp, const int* ci, const double* lam, const double* x,
                                  void* out, bool f32, hipStream_t s);

// mas.hip
hipError_t launch_coarse_sums(const BuildView& b, const double* Hu, hipStream_t s);
hipError_t launch_invert(const BuildView& b, const double* Hu, bool want32, hipStream_t s);
hipError_t launch_apply_coarse(const SolverView& v, bool f32, int mode, hipStream_t s);
hipError_t launch_apply_level0(const SolverView& v, bool f32, int mode, hipStream_t s);

// grid sizes (used for the partials buffer)
int grid_spmv_rows(int rows);
int grid_update(int M, int N);
int grid_apply0(int M, int N);
int grid_vector(int n);

}  // namespace maspcg
