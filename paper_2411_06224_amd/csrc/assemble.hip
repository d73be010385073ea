// Assembly of a list of 3x3 blocks into 3x3-block CSR (what the hash-based
// reduction of Sec. 6.2 computes: the blocks of equal (row, col) key meet
// contiguously after sorting by key and are reduced segment by segment).
//
// Deterministic, without sorting keys globally: the blocks are counted and
// scattered per row (atomic slots, any order), each row's entries are then
// sorted in LDS by (column, position in the list), and every (row, col)
// segment is summed in list order by one thread.  The sums are therefore
// those of a sequential pass over the list.
#include "launch.hpp"

namespace maspcg {
namespace {

constexpr int kAsmThreads = 256;
constexpr int kScanItems = 1024;  // elements per block of the scan

__global__ void k_fill_int(int* __restrict__ p, long long n, int value) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}

// cnt[row]++ for every listed block; an index out of range raises flag bit 0.
__global__ void k_asm_count(long long n_in, int n_rows, const int* __restrict__ rows, const int* __restrict__ cols,
                            int* __restrict__ cnt, int* __restrict__ flag) {
    const long long k = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n_in) return;
    const int r = rows[k], c = cols[k];
    if (r < 0 || r >= n_rows || c < 0 || c >= n_rows) {
        atomicOr(flag, 1);
        return;
    }
    atomicAdd(cnt + r, 1);
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

// Every listed block into a slot of its row (order within the row arbitrary);
// blocks with an index out of range were not counted and are skipped.
__global__ void k_asm_scatter(long long n_in, int n_rows, const int* __restrict__ rows, const int* __restrict__ cols,
                              const int* __restrict__ start, int* __restrict__ fill, int* __restrict__ perm) {
    const long long k = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n_in) return;
    const int r = rows[k], c = cols[k];
    if (r < 0 || r >= n_rows || c < 0 || c >= n_rows) return;
    perm[start[r] + atomicAdd(fill + r, 1)] = static_cast<int>(k);
}

constexpr int kMaxRowEntries = 4096;  // listed blocks per row sorted in LDS

// One workgroup per row: bitonic sort of the row's entries by (column,
// position in the list) in LDS; sorted positions back to perm, sorted
// columns to scol, the number of distinct columns to ucnt[row].  A row with
// more than kMaxRowEntries entries raises flag bit 1.
__global__ void __launch_bounds__(kAsmThreads) k_asm_sort(int n_rows, const int* __restrict__ cols,
                                                          const int* __restrict__ start, int* __restrict__ perm,
                                                          int* __restrict__ scol, int* __restrict__ ucnt,
                                                          int* __restrict__ flag) {
    __shared__ unsigned long long key[kMaxRowEntries];
    __shared__ int heads[kAsmThreads];
    const int row = blockIdx.x, t = threadIdx.x;
    const int s0 = start[row], m = start[row + 1] - s0;
    if (m > kMaxRowEntries) {
        if (t == 0) {
            atomicOr(flag, 2);
            ucnt[row] = 0;
        }
        return;
    }
    int n = 1;
    while (n < m) n <<= 1;
    for (int i = t; i < n; i += kAsmThreads) {
        unsigned long long kv = ~0ull;
        if (i < m) {
            const int p = perm[s0 + i];
            kv = (static_cast<unsigned long long>(static_cast<unsigned int>(cols[p])) << 32) | static_cast<unsigned int>(p);
        }
        key[i] = kv;
    }
    __syncthreads();
    for (int k = 2; k <= n; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = t; i < n; i += kAsmThreads) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const unsigned long long a = key[i], b = key[ixj];
                    const bool up = (i & k) == 0;
                    if ((a > b) == up) {
                        key[i] = b;
                        key[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    int h = 0;
    for (int i = t; i < m; i += kAsmThreads) {
        const unsigned long long kv = key[i];
        perm[s0 + i] = static_cast<int>(kv & 0xffffffffu);
        scol[s0 + i] = static_cast<int>(kv >> 32);
        h += (i == 0 || (key[i - 1] >> 32) != (kv >> 32)) ? 1 : 0;
    }
    heads[t] = h;
    __syncthreads();
    if (t == 0) {
        int s = 0;
        for (int q = 0; q < kAsmThreads; ++q) s += heads[q];
        ucnt[row] = s;
    }
}

// One workgroup per row: thread t owns the sorted entries [t c, (t+1) c) of
// the row (c = ceil(m / threads)); every segment head it owns sums its
// segment in order and writes block row_ptr[row] + rank.
__global__ void __launch_bounds__(kAsmThreads) k_asm_reduce(int n_rows, const int* __restrict__ start,
                                                            const int* __restrict__ perm, const int* __restrict__ scol,
                                                            const double* __restrict__ blocks,
                                                            const int* __restrict__ row_ptr, int* __restrict__ col_idx,
                                                            double* __restrict__ val) {
    __shared__ int sh[kAsmThreads];
    const int row = blockIdx.x, t = threadIdx.x;
    const int s0 = start[row], m = start[row + 1] - s0;
    if (m == 0 || m > kMaxRowEntries) return;
    const int per = (m + kAsmThreads - 1) / kAsmThreads;
    const int e0 = min(m, t * per), e1 = min(m, e0 + per);
    int h = 0;
    for (int e = e0; e < e1; ++e) h += (e == 0 || scol[s0 + e - 1] != scol[s0 + e]) ? 1 : 0;
    int total;
    int rank = block_exclusive_scan(h, sh, total);
    const long long out0 = row_ptr[row];
    for (int e = e0; e < e1; ++e) {
        const int c = scol[s0 + e];
        if (e != 0 && scol[s0 + e - 1] == c) continue;
        double acc[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) acc[q] = 0.0;
        for (int f = e; f < m && scol[s0 + f] == c; ++f) {
            const double* b = blocks + 9LL * perm[s0 + f];
#pragma unroll
            for (int q = 0; q < 9; ++q) acc[q] += b[q];
        }
        const long long o = out0 + rank;
        col_idx[o] = c;
#pragma unroll
        for (int q = 0; q < 9; ++q) val[9 * o + q] = acc[q];
        ++rank;
    }
}

}  // namespace

AsmLayout assemble_layout(char* ws, int n_rows, long long n_in, size_t* total) {
    size_t off = 0;
    auto take = [&](size_t count) {
        int* p = reinterpret_cast<int*>(ws ? ws + off : nullptr);
        off += (sizeof(int) * count + 255) / 256 * 256;
        return p;
    };
    const size_t rows1 = static_cast<size_t>(n_rows) + 1, m = n_in > 0 ? static_cast<size_t>(n_in) : 1;
    AsmLayout L;
    L.cnt = take(rows1);
    L.start = take(rows1);
    L.ucnt = take(rows1);
    L.perm = take(m);
    L.scol = take(m);
    L.totals = take((rows1 + kScanItems - 1) / kScanItems + 1);
    L.flag = take(2);
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

hipError_t launch_assemble_count(const AsmLayout& L, int n_rows, long long n_in, const int* rows, const int* cols,
                                 hipStream_t s) {
    const int fb = ceil_div(n_rows + 1, kAsmThreads);
    launch_kernel(k_fill_int, dim3(fb), dim3(kAsmThreads), 0, s, L.cnt, static_cast<long long>(n_rows + 1), 0);
    launch_kernel(k_fill_int, dim3(1), dim3(kAsmThreads), 0, s, L.flag, 2LL, 0);
    if (n_in > 0)
        launch_kernel(k_asm_count, dim3(ceil_div(n_in, kAsmThreads)), dim3(kAsmThreads), 0, s, n_in, n_rows, rows, cols,
                      L.cnt, L.flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // start = exclusive scan of the counts; cnt is then reused as the fill counters
    if ((e = launch_scan(L.cnt, n_rows, L.start, L.totals, s)) != hipSuccess) return e;
    launch_kernel(k_fill_int, dim3(fb), dim3(kAsmThreads), 0, s, L.cnt, static_cast<long long>(n_rows + 1), 0);
    if (n_in > 0)
        launch_kernel(k_asm_scatter, dim3(ceil_div(n_in, kAsmThreads)), dim3(kAsmThreads), 0, s, n_in, n_rows, rows,
                      cols, static_cast<const int*>(L.start), L.cnt, L.perm);
    launch_kernel(k_asm_sort, dim3(n_rows), dim3(kAsmThreads), 0, s, n_rows, cols, static_cast<const int*>(L.start),
                  L.perm, L.scol, L.ucnt, L.flag);
    return hipGetLastError();
}

hipError_t launch_assemble_reduce(const AsmLayout& L, int n_rows, const double* blocks, int* row_ptr, int* col_idx,
                                  double* val, hipStream_t s) {
    launch_kernel(k_asm_reduce, dim3(n_rows), dim3(kAsmThreads), 0, s, n_rows, static_cast<const int*>(L.start),
                  static_cast<const int*>(L.perm), static_cast<const int*>(L.scol), blocks,
                  static_cast<const int*>(row_ptr), col_idx, val);
    return hipGetLastError();
}

}  // namespace maspcg
