// Two-level reduction of contact Hessians on affine bodies (Sec. 6.1).
//
// A contact Hessian block C(r, c) couples contact nodes r and c.  A node of
// an affine body moves as x = t + A xbar (12 DOFs [t, a1, a2, a3], four
// block rows of the system); its Jacobian is J = [I | xbar1 I | xbar2 I |
// xbar3 I], so J_r^T C J_c has the 3x3 sub-blocks w_a(r) w_b(c) C with
// w = (1, xbar1, xbar2, xbar3).  A node of the deformable mesh has J = I.
//
// First level: the listed blocks of equal node pair (r, c) are summed (the
// block-list assembly over nodes: stable sort by pair, list-order sums);
// each distinct pair is then mapped once to its 16 (body-body), 4 (body-
// mesh) or 1 (mesh-mesh) sub-blocks.  The second level -- the sub-blocks of
// equal DOF block summed, e.g. all node pairs of one body pair -- is the
// block-list assembly of the resulting list together with the system's
// other blocks.  With levels = 1 every listed block is mapped directly (the
// single-level reduction the paper compares against).
#include <rocprim/device/device_scan.hpp>

#include <algorithm>

#include "abd.hpp"
#include "launch.hpp"

namespace maspcg {
namespace {

constexpr int kAbdThreads = 256;

__device__ __forceinline__ int rows_of(const int* __restrict__ is_body, int node) { return is_body[node] ? 4 : 1; }

// Sub-blocks of each pair (r_p, c_p): n_r * n_c; cnt[np] = 0 closes the
// scan that places them.
__global__ void __launch_bounds__(kAbdThreads) k_abd_count(long long np, const int* __restrict__ pr,
                                                           const int* __restrict__ pc, const int* __restrict__ is_body,
                                                           int* __restrict__ cnt) {
    const long long p = static_cast<long long>(blockIdx.x) * kAbdThreads + threadIdx.x;
    if (p < np)
        cnt[p] = rows_of(is_body, pr[p]) * rows_of(is_body, pc[p]);
    else if (p == np)
        cnt[p] = 0;
}

// A node index out of range raises flag[0] (single-level input check).
__global__ void __launch_bounds__(kAbdThreads) k_abd_check(long long m, int n_nodes, const int* __restrict__ r,
                                                           const int* __restrict__ c, int* __restrict__ flag) {
    const long long k = static_cast<long long>(blockIdx.x) * kAbdThreads + threadIdx.x;
    if (k < m && (r[k] < 0 || r[k] >= n_nodes || c[k] < 0 || c[k] >= n_nodes)) atomicOr(flag, 1);
}

__global__ void k_abd_clear(int* flag) {
    if (threadIdx.x == 0) flag[0] = 0;
}

// Pair p's sub-blocks at out[off[p] ...]: (a, b) in row-major order, block
// (w_a(r) * w_b(c)) * C_p entrywise.  One thread per (pair, sub-block slot
// of 16); slots past the pair's count do nothing.
__global__ void __launch_bounds__(kAbdThreads) k_abd_expand(long long np, const int* __restrict__ pr,
                                                            const int* __restrict__ pc, const double* __restrict__ C,
                                                            const int* __restrict__ node_row,
                                                            const int* __restrict__ is_body,
                                                            const double* __restrict__ xbar,
                                                            const int* __restrict__ off, int* __restrict__ out_rows,
                                                            int* __restrict__ out_cols, double* __restrict__ out_blk) {
    const long long t = static_cast<long long>(blockIdx.x) * kAbdThreads + threadIdx.x;
    if (t >= 16 * np) return;
    const long long p = t >> 4;
    const int slot = static_cast<int>(t & 15);
    const int r = pr[p], c = pc[p];
    const int nr = rows_of(is_body, r), nc = rows_of(is_body, c);
    if (slot >= nr * nc) return;
    const int a = slot / nc, b = slot - a * nc;
    const double wa = a == 0 ? 1.0 : xbar[3LL * r + a - 1];
    const double wb = b == 0 ? 1.0 : xbar[3LL * c + b - 1];
    const double w = wa * wb;
    const long long o = off[p] + slot;
    out_rows[o] = node_row[r] + a;
    out_cols[o] = node_row[c] + b;
#pragma unroll
    for (int e = 0; e < 9; ++e) out_blk[9 * o + e] = w * C[9 * p + e];
}

// Row of each distinct pair from the node-level CSR (row_ptr over nodes).
__global__ void __launch_bounds__(kAbdThreads) k_abd_pair_rows(int n_nodes, const int* __restrict__ row_ptr,
                                                               int* __restrict__ pr) {
    const int r = blockIdx.x * kAbdThreads + threadIdx.x;
    if (r >= n_nodes) return;
    for (int p = row_ptr[r]; p < row_ptr[r + 1]; ++p) pr[p] = r;
}

size_t round_up(size_t b) { return (b + 255) / 256 * 256; }

size_t scan_bytes(long long n) {
    size_t b = 0;
    rocprim::exclusive_scan(nullptr, b, static_cast<int*>(nullptr), static_cast<int*>(nullptr), 0,
                            static_cast<int>(std::max<long long>(n, 1)), rocprim::plus<int>());
    return b;
}

}  // namespace

AbdLayout abd_layout(char* ws, int n_nodes, long long m, size_t* total) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = ws ? ws + off : nullptr;
        off += round_up(std::max<size_t>(bytes, 1));
        return p;
    };
    const size_t mm = m > 0 ? static_cast<size_t>(m) : 1;
    AbdLayout L{};
    L.row_ptr = reinterpret_cast<int*>(take(sizeof(int) * (static_cast<size_t>(n_nodes) + 1)));
    L.pair_row = reinterpret_cast<int*>(take(sizeof(int) * mm));
    L.pair_col = reinterpret_cast<int*>(take(sizeof(int) * mm));
    L.pair_val = reinterpret_cast<double*>(take(sizeof(double) * 9 * mm));
    L.cnt = reinterpret_cast<int*>(take(sizeof(int) * (mm + 1)));
    L.off = reinterpret_cast<int*>(take(sizeof(int) * (mm + 1)));
    L.flag = reinterpret_cast<int*>(take(sizeof(int)));
    L.scan_bytes = scan_bytes(static_cast<long long>(mm) + 1);
    L.scan_tmp = take(L.scan_bytes);
    size_t asm_bytes = 0;
    assemble_layout(nullptr, n_nodes, m, &asm_bytes);
    L.asm_ws = take(asm_bytes);
    if (total) *total = off;
    return L;
}

hipError_t launch_abd_check(const AbdLayout& L, long long m, int n_nodes, const int* r, const int* c,
                            hipStream_t s) {
    launch_kernel(k_abd_clear, dim3(1), dim3(64), 0, s, L.flag);
    if (m > 0)
        launch_kernel(k_abd_check, dim3(ceil_div(m, kAbdThreads)), dim3(kAbdThreads), 0, s, m, n_nodes, r, c, L.flag);
    return hipGetLastError();
}

hipError_t launch_abd_pair_rows(const AbdLayout& L, int n_nodes, hipStream_t s) {
    launch_kernel(k_abd_pair_rows, dim3(ceil_div(n_nodes, kAbdThreads)), dim3(kAbdThreads), 0, s, n_nodes,
                  static_cast<const int*>(L.row_ptr), L.pair_row);
    return hipGetLastError();
}

hipError_t launch_abd_count(const AbdLayout& L, long long np, const int* pr, const int* pc, const int* is_body,
                            hipStream_t s) {
    launch_kernel(k_abd_count, dim3(ceil_div(np + 1, kAbdThreads)), dim3(kAbdThreads), 0, s, np, pr, pc, is_body,
                  L.cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    size_t bytes = L.scan_bytes;
    return rocprim::exclusive_scan(L.scan_tmp, bytes, L.cnt, L.off, 0, static_cast<int>(np + 1),
                                   rocprim::plus<int>(), s);
}

hipError_t launch_abd_expand(const AbdLayout& L, long long np, const int* pr, const int* pc, const double* C,
                             const int* node_row, const int* is_body, const double* xbar, int* out_rows,
                             int* out_cols, double* out_blk, hipStream_t s) {
    if (np <= 0) return hipSuccess;
    launch_kernel(k_abd_expand, dim3(ceil_div(16 * np, kAbdThreads)), dim3(kAbdThreads), 0, s, np, pr, pc, C,
                  node_row, is_body, xbar, static_cast<const int*>(L.off), out_rows, out_cols, out_blk);
    return hipGetLastError();
}

}  // namespace maspcg
