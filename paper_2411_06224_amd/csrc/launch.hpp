// Host launchers of the HIP kernels and their argument blocks.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"

namespace maspcg {

constexpr int kMaxLv = 16;

// Kernel timing: when set, the next launch reports its own start and end to
// these events (the runtime stamps them from the dispatch itself, so the
// elapsed time excludes the gaps between launches); the launch consumes them.
struct DispatchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
inline DispatchEvents& dispatch_events() {
    static thread_local DispatchEvents e;
    return e;
}

template <typename F, typename... Args>
void launch_kernel(F kernel, dim3 grid, dim3 block, uint32_t shmem, hipStream_t s, Args... args) {
    DispatchEvents& e = dispatch_events();
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, e.start, e.stop, 0u, args...);
    e = DispatchEvents{};
}

// Device views of the solver's data in the caller's workspace.
struct SolverView {
    int V, N, M, NS, L, nnzb;
    int D0, RG, G;  // work groups: D0 level-0 domains = RG slots; G groups
    int packed0;    // 1: FP64 level-0 inverses symmetric-packed (N == 16)
    int sym;        // 1: H64 holds the group-symmetric storage (nsb blocks), 0: the full slot-ordered H;
                    // H32 (mixed) always holds the full storage (nnzb blocks)
    int nsb;        // blocks of the stored slot-ordered H (H64 / H32 planes)
    int maxT;       // most transposed entries of one group (symmetric storage)
    const int* gorder;  // [G] SpMV group of each workgroup, or null: xcd_group
    int units[kMaxLv];
    int ndom[kMaxLv];
    // plans
    const int* remap;     // [NS]
    const int* map;       // [V]
    const int* perm_src;  // [nsb] caller block of each stored block (H64)
    const int* perm_full; // [nnzb] caller block of each full slot-ordered block (H32: full storage)
    const int* srp;       // symmetric storage: [NS+1] stored rows
    const int* sci;       // [nsb] column slot of each stored block
    const uint8_t* srow;  // [nsb] local row (slot - group start) of each stored block
    const int* tptr;      // [NS+1] transposed entries of each row
    const int* tidx;      // stored block of each transposed entry
    const int* rp0;       // [NS+1]
    const int* ci0;       // [nnzb]
    const int* lead1;     // [NS]
    const int* anc;       // [(L-1)*NS]
    const int* g_u1;      // [G+1]
    int W1;                       // restriction: most level-1 units in a group
    // levels l >= 2, [G][L-2][W1] (entry (g, l - 2, i) for level-1 unit i of group g, -1 / 0 pad):
    const int* ganc;              // its level-l unit
    const int* gpos;              // its partial position, -1 if it writes none
    const uint64_t* gmask;        // writers: group-local level-1 units below it
    const uint64_t* lmask;        // [NS] leader slots: lanes of the domain in the slot's level-1 unit
    // the restriction by output, padded per group: level-1 unit i of group g
    // at [g * W1 + i] (lowest slot, -1 pad; lane mask), writer e of levels
    // >= 2 at [g * GW + e] (partial position, -1 pad; entry (l - 2) W1 + i of
    // the group's ganc row; member mask over the group's level-1 units)
    const int* gu1_slot;
    const uint64_t* gu1_mask;
    int GW;
    int rfast;  // restrict_fast_ok for the group kernels' block sizes (256 and 384 threads)
    const int* gw_pos;
    const int* gw_li;
    const uint64_t* gw_mask;
    const int* cp_ptr[kMaxLv];    // l >= 2: [S_l + 1]
    // stored slot-ordered matrix (9 planes: H64 of nsb, H32 of nnzb values)
    double* H64;
    float* H32;
    // inverses per level, column-major (3N)^2 per domain
    double* inv64[kMaxLv];
    float* inv32[kMaxLv];
    // vectors in slot order (3*NS doubles)
    double *b, *x, *r, *z, *q;
    double* p[2];  // search direction p_k lives in p[k & 1]
    // coarse vectors: r1 [3*units[1]], y_l [3*ndom[l]*N] for l >= 1, coarse partials [3*n_cpart]
    double* r1;
    double* y[kMaxLv];
    double* cpart;
    // the same restrictions of q = H p (q1, qpart), and the restricted
    // residual C_l r of levels l >= 2 ([3*ndom[l]*N]) that the coarse apply
    // keeps between iterations: C_l r_k = C_l r_{k-1} - alpha_k C_l q_k
    double* q1;
    double* qpart;
    double* rc[kMaxLv];
    // per-group partial sums [G] each
    double *P_sigma, *P_rr, *P_bb, *P_rho[2];
    DevState* st;
    int* flag;  // inversion status
};

// The FP64 level-0 inverses of domain size 16 are stored symmetric-packed:
// the lower triangle of the 48 x 48 inverse column by column (column j holds
// rows j..47, so entry (i, j), i >= j, sits at packed_col(j) + i - j), 1176
// entries per domain.  The FP32 copy, other levels and other domain sizes
// keep the full column-major (3N)^2 block.
constexpr int kPackedN = 48;
constexpr int kPacked = kPackedN * (kPackedN + 1) / 2;
__host__ __device__ constexpr int packed_col(int j) { return j * kPackedN - (j * (j - 1)) / 2; }

// Build-phase views.
struct BuildView {
    int L, N, nnzb;
    int packed0;  // FP64 level-0 inverses symmetric-packed (N == 16)
    int units[kMaxLv];
    int ndom[kMaxLv];
    int nnzA[kMaxLv];
    const int* red_ptr[kMaxLv];  // level l >= 1
    const int* red_src[kMaxLv];  // level 1: caller block indices
    const int* dom_ptr[kMaxLv];
    const int* dom_blk[kMaxLv];  // level 0: caller block indices
    const int* dom_ab[kMaxLv];
    const int* remap;
    double* A[kMaxLv];  // level l >= 1: 9 planes of nnzA[l]
    double* inv64[kMaxLv];
    float* inv32[kMaxLv];
    int* flag;
};

// Residual kernel modes.
enum ResidMode {
    kResidInit = 0,     // r = b - H x0 with ||r||^2, ||b||^2 and the restriction
    kResidReplace = 1,  // r = b - H x with ||r||^2 and the restriction (skipped after a stop)
    kResidConfirm = 2,  // as kResidReplace, run after the host cleared a stop
    kResidFinal = 3     // scratch = b - H x with ||.||^2 only
};
// MAS apply modes.
//  kApplyPlain: z = M^-1 r outside PCG (no decision, no partials).
//  kApplyInit:  the first apply of a solve; decision on r_0 with ||b||.
//  kApplyIter:  iteration k after the x/r update kernel restricted r_k:
//               coarse residuals straight from that restriction (kept for
//               the recurrence), decision on r_k.
//  kApplyRec:   iteration k without the x/r update kernel: the coarse launch
//               forms alpha_k and C_l r_k = C_l r_{k-1} - alpha_k C_l q_k from
//               the restriction of q_k the SpMV left, and takes the decision
//               on r_{k-1}; the level-0 launch performs x += alpha p,
//               r -= alpha q itself and leaves the ||r_k||^2 partials.
enum ApplyMode { kApplyPlain = 0, kApplyInit = 1, kApplyIter = 2, kApplyRec = 3 };

// spmv.hip
hipError_t launch_spmv_user(int n_rows, const int* rp, const int* ci, const void* val, bool f32, const double* x,
                            double* y, hipStream_t s);
// iteration k: p_k = z_{k-1} + beta p_{k-1} (p_1 = z_0) into p[k & 1], q = H p_k, sigma partials;
// restrict_q: also the restriction of q to the coarse levels (q1, qpart)
hipError_t launch_spmv_pq(const SolverView& v, bool f32, int k, bool restrict_q, hipStream_t s);
// Bytes of shared memory the SpMV kernels can lend to the restriction of q
// after their stream (their product planes).
size_t spmv_restrict_capacity();
// Threads per workgroup of the SpMV kernels.
int spmv_threads();
hipError_t launch_residual(const SolverView& v, int mode, double* out, hipStream_t s);

// vectors.hip
hipError_t launch_state_reset(const SolverView& v, hipStream_t s);
hipError_t launch_clear_stop(const SolverView& v, hipStream_t s);
hipError_t launch_finalize(const SolverView& v, hipStream_t s);
hipError_t launch_permute_H(const SolverView& v, const double* Hu, bool f32, hipStream_t s);
hipError_t launch_perm_in(const SolverView& v, const double* src, double* dst, hipStream_t s);
hipError_t launch_perm_out(const SolverView& v, const double* src, double* dst, hipStream_t s);
hipError_t launch_init_rhs(const SolverView& v, hipStream_t s);
hipError_t launch_update(const SolverView& v, int k, hipStream_t s);
hipError_t launch_restrict(const SolverView& v, hipStream_t s);
hipError_t launch_adjoint_scatter(int n_rows, const int* rp, const int* ci, const double* lam, const double* x,
                                  void* out, bool f32, hipStream_t s);

// mas.hip
hipError_t launch_coarse_sums(const BuildView& b, const double* Hu, hipStream_t s);
hipError_t launch_invert(const BuildView& b, const double* Hu, bool want32, hipStream_t s);
// Coarse levels plus the convergence decision (mode as ApplyMode; k = 0:
// the initial apply); rr_true: the residual partials hold b - H x rather
// than the recurrence (residual replacement, FP64 confirmation).
// decision_only: workgroup 0 alone (the decision on r_k, mode kApplyIter).
hipError_t launch_apply_coarse(const SolverView& v, bool f32, int mode, int k, double tol, bool x0_given, bool mixed,
                               bool rr_true, hipStream_t s, bool decision_only = false);
hipError_t launch_apply_level0(const SolverView& v, bool f32, int mode, int k, hipStream_t s);

// assemble.hip: block-list assembly (scratch in the caller's workspace).
struct AsmLayout {
    int cb;                      // index bits: n_rows < 2^cb
    uint64_t *key, *key_sorted;  // (row << cb) | col per listed block
    int *pos, *pos_sorted;       // list position of each listed block
    int *head, *seg;             // segment heads of the sorted list and their exclusive scan
    int *seg_start;              // first sorted entry of each distinct (row, col)
    int* flag;                   // [0]: bit 0 index out of range; [1]: distinct blocks
    void* tmp;                   // radix sort / scan scratch of tmp_bytes
    size_t tmp_bytes;
};
// Layout of the assembly scratch from ws (ws = nullptr: sizes only; *total
// receives the bytes needed).
AsmLayout assemble_layout(char* ws, int n_rows, long long n_in, size_t* total);
// Exclusive scan of n ints into out[0..n] (out[n] = total); n + 1 <= 2^20.
hipError_t launch_scan(const int* in, int n, int* out, int* totals, hipStream_t s);
// Keys, stable sort by (row, col) and segment heads of the listed blocks;
// row_ptr of the result; flag[0] bit 0: index out of range, flag[1]: the
// number of distinct blocks.
hipError_t launch_assemble_sort(const AsmLayout& L, int n_rows, long long n_in, const int* rows, const int* cols,
                                int* row_ptr, hipStream_t s);
// Sums every (row, col) segment in list order into col_idx / val.
hipError_t launch_assemble_reduce(const AsmLayout& L, long long n_in, const double* blocks, int* col_idx, double* val,
                                  int nnzb, hipStream_t s);

// hierarchy.hip: supernode hierarchy on the device, every level queued at
// once; the level state on the device ends it (no host round trip).
struct HierState {
    int n_units;          // units of the current level
    int occupied;         // occupied units of the current level
    int levels;           // levels built so far
    int done;             // 1: no further level
    int bad;              // 1: the node-order pattern had an entry out of range
    int units[kMaxLv];
};
struct HierLayout {
    unsigned long long* mask;
    int *sn, *rep, *up, *cnt, *off, *totals;
    HierState* st;
};
// The pattern the hierarchy is built from: slot-ordered (map = null; rows
// and columns are slots), or in the caller's node order with the node ->
// slot map (nnzb blocks; checked against V).
struct HierPattern {
    const int *rp, *ci, *map;
    long long nnzb;
};
HierLayout hierarchy_layout(char* ws, int NS, int L_max, size_t* total);
// Levels 0 .. L_cap - 1 at most; H.sn + l NS receives the unit of every slot
// at level l, H.st the level count and units.
hipError_t launch_hierarchy(const HierLayout& H, int NS, int V, int N, int L_cap, const int* remap,
                            const HierPattern& pat, hipStream_t s);
// out_units[0] = levels (-1: invalid pattern), out_units[1 + l] = units of
// level l (kMaxLv + 1 entries); out_sn[l V + i] = unit of node i at level l,
// -1 past the last level (kMaxLv V entries).
hipError_t launch_hier_export(const HierLayout& H, int V, int NS, const int* map, int* out_units, int* out_sn,
                              hipStream_t s);

}  // namespace maspcg
