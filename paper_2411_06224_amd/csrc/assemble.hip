// Assembly of a list of 3x3 blocks into 3x3-block CSR (what the hash-based
// reduction of Sec. 6.2 computes: the blocks of equal (row, col) key meet
// contiguously after sorting by key and are reduced segment by segment).
//
// Each listed block gets the key (row << cb) | col, cb the bit width of the
// largest index (n_rows < 2^cb); a stable radix sort of
// (key, list position) pairs (rocPRIM) places equal keys together in list
// order; segment heads and their exclusive scan number the distinct blocks;
// each distinct block is summed over its segment in list order, nine
// threads per block.  The sums are those of a sequential pass over the
// list, and no row length is limited.
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include <algorithm>

#include "launch.hpp"
#include "replan.hpp"

namespace maspcg {
namespace {

constexpr int kAsmThreads = 256;
constexpr int kAsmBatch = 4;  // listed blocks loaded together by the segment sums
constexpr int kScanItems = 1024;  // elements per block of the scan

__global__ void k_fill_int(int* __restrict__ p, long long n, int value) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}

// Exclusive scan of n ints: per-block scans with block totals (pass 1), a
// scan of the totals (pass 2, one block, at most kScanItems totals), offsets
// added back (pass 3).  out[n] = the grand total.
__device__ inline int block_exclusive_scan(int v, int* sh, int& total) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int o = 1; o < kAsmThreads; o <<= 1) {
        const int a = t >= o ? sh[t - o] : 0;
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    total = sh[kAsmThreads - 1];
    const int excl = sh[t] - v;
    __syncthreads();
    return excl;
}

__global__ void __launch_bounds__(kAsmThreads) k_scan_blocks(const int* __restrict__ in, int n, int* __restrict__ out,
                                                             int* __restrict__ totals) {
    __shared__ int sh[kAsmThreads];
    const int base = blockIdx.x * kScanItems + threadIdx.x * 4;
    int v[4], s = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        v[j] = base + j < n ? in[base + j] : 0;
        s += v[j];
    }
    int total;
    int run = block_exclusive_scan(s, sh, total);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (base + j < n) out[base + j] = run;
        run += v[j];
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kAsmThreads) k_scan_totals(int* __restrict__ totals, int nb, int* __restrict__ grand) {
    __shared__ int sh[kAsmThreads];
    const int base = threadIdx.x * 4;
    int v[4], s = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        v[j] = base + j < nb ? totals[base + j] : 0;
        s += v[j];
    }
    int total;
    int run = block_exclusive_scan(s, sh, total);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (base + j < nb) totals[base + j] = run;
        run += v[j];
    }
    if (threadIdx.x == 0) *grand = total;
}

__global__ void k_scan_add(int* __restrict__ out, int n, const int* __restrict__ totals) {
    const int i = blockIdx.x * kScanItems + threadIdx.x;
    const int add = totals[blockIdx.x];
    for (int j = i; j < min(n, static_cast<int>(blockIdx.x + 1) * kScanItems); j += blockDim.x) out[j] += add;
}

// Key and list position of every listed block; an index out of range
// raises flag bit 0 (its key sorts last and is never reduced).
__device__ __forceinline__ uint64_t key_sentinel(int cb) { return (1ull << (2 * cb)) - 1; }  // above every valid key

__global__ void __launch_bounds__(kAsmThreads) k_asm_keys(long long n_in, int n_rows, int cb,
                                                          const int* __restrict__ rows, const int* __restrict__ cols,
                                                          uint64_t* __restrict__ key, int* __restrict__ pos,
                                                          int* __restrict__ flag) {
    const long long k = static_cast<long long>(blockIdx.x) * kAsmThreads + threadIdx.x;
    if (k >= n_in) return;
    const int r = rows[k], c = cols[k];
    const bool bad = r < 0 || r >= n_rows || c < 0 || c >= n_rows;
    if (bad) atomicOr(flag, 1);
    key[k] = bad ? key_sentinel(cb) : (static_cast<uint64_t>(r) << cb) | static_cast<uint64_t>(c);
    pos[k] = static_cast<int>(k);
}

__global__ void __launch_bounds__(kAsmThreads) k_asm_heads(long long n_in, const uint64_t* __restrict__ key,
                                                           int* __restrict__ head) {
    const long long k = static_cast<long long>(blockIdx.x) * kAsmThreads + threadIdx.x;
    if (k < n_in) head[k] = (k == 0 || key[k] != key[k - 1]) ? 1 : 0;
}

// Segment starts, row pointers and the number of distinct blocks.  Row r
// begins at the segment of its first sorted entry; rows without blocks take
// the next row's start (every row_ptr entry has one writer).
__global__ void __launch_bounds__(kAsmThreads) k_asm_rows(long long n_in, int n_rows, int cb,
                                                          const uint64_t* __restrict__ key,
                                                          const int* __restrict__ head, const int* __restrict__ seg,
                                                          int* __restrict__ seg_start, int* __restrict__ row_ptr,
                                                          int* __restrict__ flag) {
    const long long k = static_cast<long long>(blockIdx.x) * kAsmThreads + threadIdx.x;
    if (n_in == 0) {
        for (long long r = k; r <= n_rows; r += static_cast<long long>(gridDim.x) * kAsmThreads) row_ptr[r] = 0;
        if (k == 0) flag[1] = 0;
        return;
    }
    if (k >= n_in) return;
    const uint64_t kk = key[k];
    const bool valid = kk < key_sentinel(cb);
    const int r = static_cast<int>(kk >> cb);
    if (head[k] && valid) {
        seg_start[seg[k]] = static_cast<int>(k);
        const int pr = k == 0 ? -1 : static_cast<int>(key[k - 1] >> cb);
        for (int rr = pr + 1; rr <= r; ++rr) row_ptr[rr] = seg[k];
    }
    // the last valid entry closes the remaining rows and counts the blocks
    const bool last = valid && (k + 1 == n_in || key[k + 1] >= key_sentinel(cb));
    if (last) {
        const int total = seg[k] + head[k];
        for (int rr = r + 1; rr <= n_rows; ++rr) row_ptr[rr] = total;
        seg_start[total] = static_cast<int>(k + 1);
        flag[1] = total;
    }
    if (k == 0 && !valid) {  // every index out of range: nothing to assemble
        for (int rr = 0; rr <= n_rows; ++rr) row_ptr[rr] = 0;
        flag[1] = 0;
    }
}

// Distinct block b = t / 9, entry t % 9: the sum over its segment in list
// order (nine consecutive threads read one listed block).  The segment is
// read kAsmBatch entries at a time: their positions, then their values, all
// in flight together, then added in order.
__global__ void __launch_bounds__(kAsmThreads) k_asm_reduce(int nnzb, int cb, const uint64_t* __restrict__ key,
                                                            const int* __restrict__ pos,
                                                            const int* __restrict__ seg_start,
                                                            const double* __restrict__ blocks,
                                                            int* __restrict__ col_idx, double* __restrict__ val) {
    const long long t = static_cast<long long>(blockIdx.x) * kAsmThreads + threadIdx.x;
    if (t >= 9LL * nnzb) return;
    const int b = static_cast<int>(t / 9), c = static_cast<int>(t - 9LL * b);
    const int e0 = seg_start[b], e1 = seg_start[b + 1];
    double acc = 0.0;
    for (int e = e0; e < e1; e += kAsmBatch) {
        int p[kAsmBatch];
#pragma unroll
        for (int j = 0; j < kAsmBatch; ++j) p[j] = pos[min(e + j, e1 - 1)];
        double x[kAsmBatch];
#pragma unroll
        for (int j = 0; j < kAsmBatch; ++j) x[j] = blocks[9LL * p[j] + c];
#pragma unroll
        for (int j = 0; j < kAsmBatch; ++j)
            if (e + j < e1) acc += x[j];
    }
    val[9LL * b + c] = acc;
    if (c == 0) col_idx[b] = static_cast<int>(key[e0] & ((1ull << cb) - 1));
}

size_t tmp_bytes(long long n_in, int key_bits) {
    const int n = static_cast<int>(std::max<long long>(n_in, 1));
    size_t sb = 0, scb = 0;
    rocprim::radix_sort_pairs(nullptr, sb, static_cast<uint64_t*>(nullptr), static_cast<uint64_t*>(nullptr),
                              static_cast<int*>(nullptr), static_cast<int*>(nullptr), n, 0, key_bits);
    rocprim::exclusive_scan(nullptr, scb, static_cast<int*>(nullptr), static_cast<int*>(nullptr), 0, n,
                            rocprim::plus<int>());
    return std::max(sb, scb);
}

// Bit width of the indices of an n_rows system: the smallest cb with
// n_rows < 2^cb, so that every valid key stays below the sentinel.
int index_bits(int n_rows) {
    int cb = 1;
    while (cb < 31 && (1LL << cb) <= n_rows) ++cb;
    return cb;
}

}  // namespace

AsmLayout assemble_layout(char* ws, int n_rows, long long n_in, size_t* total) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = ws ? ws + off : nullptr;
        off += (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
        return p;
    };
    const size_t m = n_in > 0 ? static_cast<size_t>(n_in) : 1;
    AsmLayout L{};
    L.key = reinterpret_cast<uint64_t*>(take(sizeof(uint64_t) * m));
    L.key_sorted = reinterpret_cast<uint64_t*>(take(sizeof(uint64_t) * m));
    L.pos = reinterpret_cast<int*>(take(sizeof(int) * m));
    L.pos_sorted = reinterpret_cast<int*>(take(sizeof(int) * m));
    L.head = reinterpret_cast<int*>(take(sizeof(int) * m));
    L.seg = reinterpret_cast<int*>(take(sizeof(int) * m));
    L.seg_start = reinterpret_cast<int*>(take(sizeof(int) * (m + 1)));
    L.flag = reinterpret_cast<int*>(take(sizeof(int) * 2));
    L.cb = index_bits(n_rows);
    L.tmp_bytes = tmp_bytes(n_in, 2 * L.cb);
    L.tmp = take(L.tmp_bytes);
    if (total) *total = off;
    return L;
}

hipError_t launch_scan(const int* in, int n, int* out, int* totals, hipStream_t s) {
    const int nb = (n + kScanItems - 1) / kScanItems;
    if (nb > 4 * kAsmThreads) return hipErrorInvalidValue;
    launch_kernel(k_scan_blocks, dim3(nb), dim3(kAsmThreads), 0, s, in, n, out, totals);
    launch_kernel(k_scan_totals, dim3(1), dim3(kAsmThreads), 0, s, totals, nb, out + n);
    launch_kernel(k_scan_add, dim3(nb), dim3(kAsmThreads), 0, s, out, n, static_cast<const int*>(totals));
    return hipGetLastError();
}

hipError_t launch_assemble_sort(const AsmLayout& L, int n_rows, long long n_in, const int* rows, const int* cols,
                                int* row_ptr, hipStream_t s) {
    launch_kernel(k_fill_int, dim3(1), dim3(64), 0, s, L.flag, 2LL, 0);
    if (n_in > 0)
        launch_kernel(k_asm_keys, dim3(ceil_div(n_in, kAsmThreads)), dim3(kAsmThreads), 0, s, n_in, n_rows, L.cb, rows,
                      cols, L.key, L.pos, L.flag);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_assemble_sort_keys(L, n_rows, n_in, row_ptr, s, false);
}

hipError_t launch_assemble_sort_keys(const AsmLayout& L, int n_rows, long long n_in, int* row_ptr, hipStream_t s,
                                     bool clear_flag) {
    if (clear_flag) launch_kernel(k_fill_int, dim3(1), dim3(64), 0, s, L.flag, 2LL, 0);
    hipError_t e;
    if (n_in > 0) {
        const int g = ceil_div(n_in, kAsmThreads);
        size_t bytes = L.tmp_bytes;
        if ((e = rocprim::radix_sort_pairs(L.tmp, bytes, L.key, L.key_sorted, L.pos, L.pos_sorted,
                                           static_cast<int>(n_in), 0, 2 * L.cb, s)) != hipSuccess)
            return e;
        launch_kernel(k_asm_heads, dim3(g), dim3(kAsmThreads), 0, s, n_in, static_cast<const uint64_t*>(L.key_sorted),
                      L.head);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        bytes = L.tmp_bytes;
        if ((e = rocprim::exclusive_scan(L.tmp, bytes, L.head, L.seg, 0, static_cast<int>(n_in),
                                         rocprim::plus<int>(), s)) != hipSuccess)
            return e;
        launch_kernel(k_asm_rows, dim3(g), dim3(kAsmThreads), 0, s, n_in, n_rows, L.cb,
                      static_cast<const uint64_t*>(L.key_sorted), static_cast<const int*>(L.head),
                      static_cast<const int*>(L.seg), L.seg_start, row_ptr, L.flag);
    } else {
        launch_kernel(k_asm_rows, dim3(ceil_div(n_rows + 1, kAsmThreads)), dim3(kAsmThreads), 0, s, 0LL, n_rows,
                      L.cb, static_cast<const uint64_t*>(L.key_sorted), static_cast<const int*>(L.head),
                      static_cast<const int*>(L.seg), L.seg_start, row_ptr, L.flag);
    }
    return hipGetLastError();
}

hipError_t launch_assemble_reduce(const AsmLayout& L, long long n_in, const double* blocks, int* col_idx, double* val,
                                  int nnzb, hipStream_t s) {
    (void)n_in;
    if (nnzb <= 0) return hipSuccess;
    launch_kernel(k_asm_reduce, dim3(ceil_div(9LL * nnzb, kAsmThreads)), dim3(kAsmThreads), 0, s, nnzb, L.cb,
                  static_cast<const uint64_t*>(L.key_sorted), static_cast<const int*>(L.pos_sorted),
                  static_cast<const int*>(L.seg_start), blocks, col_idx, val);
    return hipGetLastError();
}

}  // namespace maspcg
