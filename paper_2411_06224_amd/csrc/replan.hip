// Solver plans of a new sparsity pattern on the device (see replan.hpp).
//
// Every plan is a stable sort, a count and scan, or a per-unit scan over a
// few dozen lanes, written so that its output is the one of the host
// analysis for the same pattern and partition:
//   - slot order: keys (map[i] << cb) | map[j], stably sorted, give the rows
//     and columns in slot order and the caller block of each;
//   - coarsening (Supp. Eq. 5): keys (up[s] << cb) | up[t] of the fine
//     blocks, stably sorted, give the coarse pattern, and the sorted fine
//     positions with their segment starts are the reduction plan;
//   - inversion gathers: the upper in-domain blocks of each row, counted,
//     scanned and written in row order;
//   - group-symmetric storage: the kept blocks of each row and, for every
//     row, the stored blocks of its transposed entries, counted and scanned;
//   - restriction: the lowest lane of each level-1 unit in its domain, the
//     level-1 units of each group, and for levels >= 2 the lowest level-1
//     unit of each (group, ancestor) pair, numbered by a stable sort of
//     (ancestor, unit) keys.
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include <algorithm>

#include "replan.hpp"

namespace maspcg {
namespace {

constexpr int kRpThreads = 256;

__device__ __forceinline__ uint64_t sentinel(int cb) { return (1ull << (2 * cb)) - 1; }

__global__ void k_rp_fill(int* __restrict__ p, long long n, int v) {
    const long long i = static_cast<long long>(blockIdx.x) * kRpThreads + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_rp_fill64(uint64_t* __restrict__ p, long long n) {
    const long long i = static_cast<long long>(blockIdx.x) * kRpThreads + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

__global__ void k_rp_counts_init(ReplanCounts* __restrict__ c) {
    if (threadIdx.x != 0) return;
    c->bad = 0;
    c->nnz_distinct = 0;
    for (int l = 0; l < kMaxLv; ++l) {
        c->nnzA[l] = 0;
        c->ndomblk[l] = 0;
    }
    for (int l = 0; l <= kMaxLv; ++l) c->cbase[l] = 0;
    c->gw_max = 0;
}

__global__ void k_rp_store(int* __restrict__ dst, const int* __restrict__ src) {
    if (threadIdx.x == 0) *dst = *src;
}

// Row checks of the caller's pattern: row_ptr from 0 to nnzb and monotone,
// columns in range and strictly ascending, the diagonal present.  A bad
// row range is skipped by every later kernel.
__device__ __forceinline__ bool row_ok(const int* rp, int i, long long nnzb) {
    const int p0 = rp[i], p1 = rp[i + 1];
    return p0 >= 0 && p1 >= p0 && p1 <= nnzb;
}

__global__ void k_rp_check_rows(int V, long long nnzb, const int* __restrict__ rp, const int* __restrict__ ci,
                                ReplanCounts* __restrict__ c) {
    const int i = blockIdx.x * kRpThreads + threadIdx.x;
    if (i >= V) return;
    int bad = 0;
    if (i == 0 && rp[0] != 0) bad |= 1;
    if (i == V - 1 && rp[V] != nnzb) bad |= 1;
    if (!row_ok(rp, i, nnzb)) {
        atomicOr(&c->bad, bad | 1);
        return;
    }
    bool diag = false;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        const int j = ci[p];
        if (j < 0 || j >= V) {
            bad |= 2;
            continue;
        }
        if (p > rp[i] && j <= ci[p - 1]) bad |= 4;
        diag |= j == i;
    }
    if (!diag) bad |= 8;
    if (bad) atomicOr(&c->bad, bad);
}

// Symmetry: every block (i, j) has its transpose (j, i) (binary search in
// row j; rows that failed their own checks are skipped).
__global__ void k_rp_check_sym(int V, long long nnzb, const int* __restrict__ rp, const int* __restrict__ ci,
                               ReplanCounts* __restrict__ c) {
    const int i = blockIdx.x * kRpThreads + threadIdx.x;
    if (i >= V || !row_ok(rp, i, nnzb)) return;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        const int j = ci[p];
        if (j < 0 || j >= V || !row_ok(rp, j, nnzb)) continue;
        int lo = rp[j], hi = rp[j + 1];
        while (lo < hi) {
            const int m = (lo + hi) >> 1;
            if (ci[m] < i)
                lo = m + 1;
            else
                hi = m;
        }
        if (lo == rp[j + 1] || ci[lo] != i) {
            atomicOr(&c->bad, 16);
            return;
        }
    }
}

// Sort input of the slot order: block p of row i -> (map[i], map[j]);
// entries of bad rows keep the -1 of the fill (their keys sort last).
__global__ void k_rp_slot_keys(int V, long long nnzb, const int* __restrict__ rp, const int* __restrict__ ci,
                               const int* __restrict__ map, int* __restrict__ rows, int* __restrict__ cols) {
    const int i = blockIdx.x * kRpThreads + threadIdx.x;
    if (i >= V || !row_ok(rp, i, nnzb)) return;
    const int si = map[i];
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        const int j = ci[p];
        rows[p] = si;
        cols[p] = (j >= 0 && j < V) ? map[j] : -1;
    }
}

// Column of each distinct block from its first sorted key; the caller block
// (list position) of each when every segment is a single block.
__global__ void k_rp_cols(long long n, int cb, const uint64_t* __restrict__ key, const int* __restrict__ seg_start,
                          const int* __restrict__ count, int* __restrict__ col) {
    const long long b = static_cast<long long>(blockIdx.x) * kRpThreads + threadIdx.x;
    if (b >= n || b >= *count) return;
    col[b] = static_cast<int>(key[seg_start[b]] & ((1ull << cb) - 1));
}

// up[u] for the units u of level l: the level-(l+1) unit of any slot of u
// (all of them agree).
__global__ void k_rp_up(int NS, const int* __restrict__ sn_l, const int* __restrict__ sn_next, int* __restrict__ up) {
    const int s = blockIdx.x * kRpThreads + threadIdx.x;
    if (s >= NS) return;
    const int u = sn_l[s];
    if (u >= 0) up[u] = sn_next[s];
}

// Sort keys of one coarsening: fine block p (row r: the last row starting
// at or before p) -> (up[r] << cb) | up[ci[p]] with its position p;
// positions past the fine pattern's blocks get the sentinel (sorted last).
__global__ void k_rp_coarse_keys(long long n, int rowsF, int cb, const int* __restrict__ rp,
                                 const int* __restrict__ ci, const int* __restrict__ up, uint64_t* __restrict__ key,
                                 int* __restrict__ pos) {
    const long long p = static_cast<long long>(blockIdx.x) * kRpThreads + threadIdx.x;
    if (p >= n) return;
    pos[p] = static_cast<int>(p);
    if (p >= rp[rowsF]) {
        key[p] = sentinel(cb);
        return;
    }
    int lo = 0, hi = rowsF;  // largest r with rp[r] <= p
    while (hi - lo > 1) {
        const int m = (lo + hi) >> 1;
        if (rp[m] <= p)
            lo = m;
        else
            hi = m;
    }
    key[p] = (static_cast<uint64_t>(up[lo]) << cb) | static_cast<uint64_t>(up[ci[p]]);
}

// First position in [lo, hi) of the ascending a[] whose value is >= v.
__device__ __forceinline__ int first_at_least(const int* __restrict__ a, int lo, int hi, int v) {
    while (lo < hi) {
        const int m = (lo + hi) >> 1;
        if (a[m] < v)
            lo = m + 1;
        else
            hi = m;
    }
    return lo;
}

// Inversion gathers of one level: per row s the blocks (s, t) with
// s <= t < (domain start) + N, a contiguous range of the row's ascending
// columns (found by binary search: coarse rows can hold thousands of
// blocks).  cnt[rows] = 0 closes the scan.
__global__ void k_rp_dom_count(int rows, int N, const int* __restrict__ rp, const int* __restrict__ ci,
                               int* __restrict__ cnt) {
    const int s = blockIdx.x * kRpThreads + threadIdx.x;
    if (s > rows) return;
    if (s == rows) {
        cnt[s] = 0;
        return;
    }
    const int p0 = first_at_least(ci, rp[s], rp[s + 1], s);
    cnt[s] = first_at_least(ci, p0, rp[s + 1], s / N * N + N) - p0;
}

__global__ void k_rp_dom_fill(int rows, int N, const int* __restrict__ rp, const int* __restrict__ ci,
                              const int* __restrict__ off, const int* __restrict__ perm, int* __restrict__ blk,
                              int* __restrict__ ab) {
    const int s = blockIdx.x * kRpThreads + threadIdx.x;
    if (s >= rows) return;
    const int lo = s / N * N;
    const int p0 = first_at_least(ci, rp[s], rp[s + 1], s);
    const int p1 = first_at_least(ci, p0, rp[s + 1], lo + N);
    int o = off[s];
    for (int p = p0; p < p1; ++p) {
        blk[o] = perm ? perm[p] : p;
        ab[o] = (s - lo) | ((ci[p] - lo) << 8);
        ++o;
    }
}

__global__ void k_rp_dom_ptr(int rows, int N, int nd, const int* __restrict__ off, int* __restrict__ ptr) {
    const int d = blockIdx.x * kRpThreads + threadIdx.x;
    if (d <= nd) ptr[d] = off[min(d * N, rows)];
}

// Group-symmetric storage: row s of group [r0, r1) keeps its blocks whose
// column is outside the group or >= s; its transposed entries are the
// group's blocks (i, s), i < s, that is (by symmetry) its own columns in
// [r0, s).
__global__ void k_rp_sym_keep(int NS, int RG, const int* __restrict__ rp, const int* __restrict__ ci,
                              int* __restrict__ cnt) {
    const int s = blockIdx.x * kRpThreads + threadIdx.x;
    if (s > NS) return;
    if (s == NS) {
        cnt[s] = 0;
        return;
    }
    const int r0 = s / RG * RG, r1 = min(r0 + RG, NS);
    int c = 0;
    for (int p = rp[s]; p < rp[s + 1]; ++p) {
        const int j = ci[p];
        c += (j < r0 || j >= r1 || j >= s) ? 1 : 0;
    }
    cnt[s] = c;
}

__global__ void k_rp_sym_trans(int NS, int RG, const int* __restrict__ rp, const int* __restrict__ ci,
                               int* __restrict__ cnt) {
    const int s = blockIdx.x * kRpThreads + threadIdx.x;
    if (s > NS) return;
    if (s == NS) {
        cnt[s] = 0;
        return;
    }
    const int r0 = s / RG * RG;
    int c = 0;
    for (int p = rp[s]; p < rp[s + 1]; ++p) {
        const int j = ci[p];
        c += (j >= r0 && j < s) ? 1 : 0;
    }
    cnt[s] = c;
}

__global__ void k_rp_sym_fill(int NS, int RG, const int* __restrict__ rp, const int* __restrict__ ci,
                              const int* __restrict__ perm, const int* __restrict__ srp, int* __restrict__ sci,
                              int* __restrict__ sperm, uint8_t* __restrict__ srow) {
    const int s = blockIdx.x * kRpThreads + threadIdx.x;
    if (s >= NS) return;
    const int r0 = s / RG * RG, r1 = min(r0 + RG, NS);
    int o = srp[s];
    for (int p = rp[s]; p < rp[s + 1]; ++p) {
        const int j = ci[p];
        if (j >= r0 && j < r1 && j < s) continue;
        sci[o] = j;
        sperm[o] = perm[p];
        srow[o] = static_cast<uint8_t>(s - r0);
        ++o;
    }
}

// tidx of row j: for its columns i in [r0, j), ascending, the stored index
// of block (i, j) in row i.
__global__ void k_rp_sym_tidx(int NS, int RG, const int* __restrict__ rp, const int* __restrict__ ci,
                              const int* __restrict__ srp, const int* __restrict__ sci, const int* __restrict__ tptr,
                              int* __restrict__ tidx) {
    const int j = blockIdx.x * kRpThreads + threadIdx.x;
    if (j >= NS) return;
    const int r0 = j / RG * RG;
    int o = tptr[j];
    for (int p = rp[j]; p < rp[j + 1]; ++p) {
        const int i = ci[p];
        if (i < r0 || i >= j) continue;
        int lo = srp[i], hi = srp[i + 1];
        while (lo < hi) {
            const int m = (lo + hi) >> 1;
            if (sci[m] < j)
                lo = m + 1;
            else
                hi = m;
        }
        tidx[o++] = lo;
    }
}

// Per group: stored blocks of the full and the symmetric storage and
// transposed entries (the SpMV's group order and the symmetric limit).
__global__ void k_rp_group_sizes(int G, int RG, int NS, const int* __restrict__ rp0, const int* __restrict__ srp,
                                 const int* __restrict__ tptr, int* __restrict__ out) {
    const int g = blockIdx.x * kRpThreads + threadIdx.x;
    if (g >= G) return;
    const int r0 = g * RG, r1 = min(r0 + RG, NS);
    out[g] = rp0[r1] - rp0[r0];
    out[G + g] = srp[r1] - srp[r0];
    out[2 * G + g] = tptr[r1] - tptr[r0];
}

// Level-1 restriction: slot s leads its level-1 unit u if no lower lane of
// its domain belongs to u; its mask holds the domain's lanes in u.
__global__ void k_rp_lead1(int NS, int N, int L, const int* __restrict__ sn1, int* __restrict__ lead1,
                           uint64_t* __restrict__ lmask) {
    const int s = blockIdx.x * kRpThreads + threadIdx.x;
    if (s >= NS) return;
    int lead = -1;
    uint64_t m = 0ull;
    if (L > 1) {
        const int u = sn1[s];
        const int lo = s / N * N, a = s - lo;
        bool first = u >= 0;
        for (int b = 0; b < N && first; ++b)
            if (b < a && sn1[lo + b] == u) first = false;
        if (first) {
            lead = u;
            for (int b = 0; b < N; ++b)
                if (sn1[lo + b] == u) m |= 1ull << b;
        }
    }
    lead1[s] = lead;
    lmask[s] = m;
}

__global__ void k_rp_group_units(int G, int RG, int NS, const int* __restrict__ lead1, int* __restrict__ cnt) {
    const int g = blockIdx.x * kRpThreads + threadIdx.x;
    if (g > G) return;
    if (g == G) {
        cnt[g] = 0;
        return;
    }
    const int r0 = g * RG, r1 = min(r0 + RG, NS);
    int c = 0;
    for (int s = r0; s < r1; ++s) c += lead1[s] >= 0 ? 1 : 0;
    cnt[g] = c;
}

// Level-l ancestor and group of every level-1 unit (through its lowest slot).
__global__ void k_rp_anc1(int NS, int RG, int L, const int* __restrict__ sn, const int* __restrict__ lead1,
                          int* __restrict__ anc1, int* __restrict__ t_grp) {
    const int s = blockIdx.x * kRpThreads + threadIdx.x;
    if (s >= NS) return;
    const int t = lead1[s];
    if (t < 0) return;
    t_grp[t] = s / RG;
    for (int l = 2; l < L; ++l) anc1[static_cast<size_t>(l) * NS + t] = sn[static_cast<size_t>(l) * NS + s];
}

// Writers of level l: the lowest level-1 unit of its group below each
// level-l unit.  Key (ancestor << cb) | unit for writers, the sentinel
// otherwise; partial positions start unset.
__global__ void k_rp_writer_keys(int S1, int NS, int l, int cb, const int* __restrict__ anc1,
                                 const int* __restrict__ t_grp, const int* __restrict__ g_u1,
                                 uint64_t* __restrict__ key, int* __restrict__ pos, int* __restrict__ lpos) {
    const int t = blockIdx.x * kRpThreads + threadIdx.x;
    if (t >= S1) return;
    const int* a = anc1 + static_cast<size_t>(l) * NS;
    const int u = a[t];
    bool writer = true;
    for (int q = g_u1[t_grp[t]]; q < t && writer; ++q) writer = a[q] != u;
    key[t] = writer ? (static_cast<uint64_t>(u) << cb) | static_cast<uint64_t>(t) : sentinel(cb);
    pos[t] = t;
    lpos[static_cast<size_t>(l) * NS + t] = -1;
}

// Sorted writer k of level l holds partial position cbase[l] + k; the last
// writer closes the level (cbase[l + 1]).
__global__ void k_rp_writer_place(int S1, int NS, int l, int cb, const uint64_t* __restrict__ key,
                                  const int* __restrict__ pos, ReplanCounts* __restrict__ c, int* __restrict__ lpos) {
    const int k = blockIdx.x * kRpThreads + threadIdx.x;
    if (k >= S1) return;
    const int base = c->cbase[l];
    const bool valid = key[k] < sentinel(cb);
    if (valid) lpos[static_cast<size_t>(l) * NS + pos[k]] = base + k;
    if (valid && (k + 1 == S1 || key[k + 1] >= sentinel(cb))) c->cbase[l + 1] = base + k + 1;
    if (k == 0 && !valid) c->cbase[l + 1] = base;
}

// cp_ptr of level l: unit u's partials start at its first sorted writer.
__global__ void k_rp_writer_ptr(int units, int NS, int l, int cb, const uint64_t* __restrict__ key,
                                const ReplanCounts* __restrict__ c, int* __restrict__ cpp) {
    const int u = blockIdx.x * kRpThreads + threadIdx.x;
    if (u > units) return;
    const int base = c->cbase[l], nw = c->cbase[l + 1] - base;
    const uint64_t want = static_cast<uint64_t>(u) << cb;
    int lo = 0, hi = nw;
    while (lo < hi) {
        const int m = (lo + hi) >> 1;
        if (key[m] < want)
            lo = m + 1;
        else
            hi = m;
    }
    cpp[static_cast<size_t>(l) * (NS + 1) + u] = base + lo;
}

// Writers of each group over all levels (the widest group sizes the
// writer tables).
__global__ void k_rp_group_writers(int G, int NS, int L, const int* __restrict__ g_u1, const int* __restrict__ lpos,
                                   ReplanCounts* __restrict__ c) {
    const int g = blockIdx.x * kRpThreads + threadIdx.x;
    if (g >= G) return;
    int n = 0;
    for (int l = 2; l < L; ++l)
        for (int t = g_u1[g]; t < g_u1[g + 1]; ++t) n += lpos[static_cast<size_t>(l) * NS + t] >= 0 ? 1 : 0;
    atomicMax(&c->gw_max, n);
}

// ---- placement into the solver workspace

__global__ void k_rp_gather(long long n, const int* __restrict__ perm, const int* __restrict__ idx,
                            int* __restrict__ out) {
    const long long k = static_cast<long long>(blockIdx.x) * kRpThreads + threadIdx.x;
    if (k < n) out[k] = perm[idx[k]];
}

// Level-1 unit i of group g at [g W1 + i]: its lowest slot and lane mask.
__global__ void k_rp_gu1(int NS, int RG, int W1, const int* __restrict__ lead1, const uint64_t* __restrict__ lmask,
                         const int* __restrict__ g_u1, int* __restrict__ slot, uint64_t* __restrict__ mask) {
    const int s = blockIdx.x * kRpThreads + threadIdx.x;
    if (s >= NS) return;
    const int u = lead1[s];
    if (u < 0) return;
    const int g = s / RG;
    const size_t o = static_cast<size_t>(g) * W1 + (u - g_u1[g]);
    slot[o] = s;
    mask[o] = lmask[s];
}

__device__ __forceinline__ uint64_t writer_mask(const int* a, int lo, int n1, int i) {
    uint64_t m = 0ull;
    for (int j = 0; j < n1; ++j)
        if (a[lo + j] == a[lo + i]) m |= 1ull << j;
    return m;
}

// Restriction tables of levels >= 2, [G][L-2][W1]: ancestor and partial
// position of the group's level-1 units (-1 past them); member masks of
// the writers when W1 <= 64.
__global__ void k_rp_gtab(int G, int L, int W1, int NS, const int* __restrict__ g_u1, const int* __restrict__ anc1,
                          const int* __restrict__ lpos, int* __restrict__ ganc, int* __restrict__ gpos,
                          uint64_t* __restrict__ gmask) {
    const long long e = static_cast<long long>(blockIdx.x) * kRpThreads + threadIdx.x;
    const int nl = L - 2;
    if (e >= static_cast<long long>(G) * nl * W1) return;
    const int i = static_cast<int>(e % W1);
    const int l = 2 + static_cast<int>((e / W1) % nl);
    const int g = static_cast<int>(e / (static_cast<long long>(W1) * nl));
    const int lo = g_u1[g], n1 = g_u1[g + 1] - lo;
    const int* a = anc1 + static_cast<size_t>(l) * NS;
    const int* w = lpos + static_cast<size_t>(l) * NS;
    int an = -1, ps = -1;
    uint64_t m = 0ull;
    if (i < n1) {
        an = a[lo + i];
        ps = w[lo + i];
        if (W1 <= 64 && ps >= 0) m = writer_mask(a, lo, n1, i);
    }
    ganc[e] = an;
    gpos[e] = ps;
    gmask[e] = m;
}

// Writer tables [G][GW], levels then units in order: partial position,
// entry (l - 2) W1 + i of the group's table row, member mask.  One wave per
// group: the writers of 64 units at a time are ranked by a ballot.
__global__ void __launch_bounds__(64) k_rp_gw(int L, int W1, int GW, int NS, const int* __restrict__ g_u1,
                                              const int* __restrict__ anc1, const int* __restrict__ lpos,
                                              int* __restrict__ gw_pos, int* __restrict__ gw_li,
                                              uint64_t* __restrict__ gw_mask) {
    const int g = blockIdx.x, lane = threadIdx.x;
    const int lo = g_u1[g], n1 = g_u1[g + 1] - lo;
    const size_t base = static_cast<size_t>(g) * GW;
    int e = 0;
    for (int l = 2; l < L; ++l) {
        const int* a = anc1 + static_cast<size_t>(l) * NS;
        const int* w = lpos + static_cast<size_t>(l) * NS;
        for (int i0 = 0; i0 < n1; i0 += 64) {
            const int i = i0 + lane;
            const int ps = i < n1 ? w[lo + i] : -1;
            const uint64_t writers = __ballot(ps >= 0);
            if (ps >= 0) {
                const size_t o = base + e + __popcll(writers & ((1ull << lane) - 1ull));
                gw_pos[o] = ps;
                gw_li[o] = (l - 2) * W1 + i;
                gw_mask[o] = W1 <= 64 ? writer_mask(a, lo, n1, i) : 0ull;
            }
            e += __popcll(writers);
        }
    }
    for (int k = e + lane; k < GW; k += 64) {
        gw_pos[base + k] = -1;
        gw_li[base + k] = 0;
        gw_mask[base + k] = 0ull;
    }
}

size_t round_up(size_t b) { return (b + 255) / 256 * 256; }

int grid(long long n) { return static_cast<int>(std::max<long long>(1, (n + kRpThreads - 1) / kRpThreads)); }

hipError_t scan(const ReplanLayout& R, const int* in, int* out, int n_plus_1, hipStream_t s) {
    size_t bytes = R.scan_bytes;
    return rocprim::exclusive_scan(R.scan_tmp, bytes, in, out, 0, n_plus_1, rocprim::plus<int>(), s);
}

hipError_t copy_ints(int* dst, const int* src, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    return hipMemcpyAsync(dst, src, sizeof(int) * n, hipMemcpyDeviceToDevice, s);
}

// Coarsens level l - 1 (rowsF rows, at most nF blocks, pattern rpF / ciF)
// into level l (rowsC rows): pattern rpC / ciC; the sorted fine positions
// (R.A.pos_sorted) and segment starts (R.A.seg_start) are the reduction
// plan, R.A.flag[1] the coarse block count.
hipError_t coarsen_level(const ReplanLayout& R, int NS, int l, int rowsF, int rowsC, long long nF, const int* rpF,
                         const int* ciF, int* rpC, int* ciC, hipStream_t s) {
    launch_kernel(k_rp_up, dim3(grid(NS)), dim3(kRpThreads), 0, s, NS,
                  static_cast<const int*>(R.H.sn + static_cast<size_t>(l - 1) * NS),
                  static_cast<const int*>(R.H.sn + static_cast<size_t>(l) * NS), R.up);
    launch_kernel(k_rp_coarse_keys, dim3(grid(nF)), dim3(kRpThreads), 0, s, nF, rowsF, R.A.cb, rpF, ciF,
                  static_cast<const int*>(R.up), R.A.key, R.A.pos);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = launch_assemble_sort_keys(R.A, rowsC, nF, rpC, s, true)) != hipSuccess) return e;
    launch_kernel(k_rp_cols, dim3(grid(nF)), dim3(kRpThreads), 0, s, nF, R.A.cb,
                  static_cast<const uint64_t*>(R.A.key_sorted), static_cast<const int*>(R.A.seg_start),
                  static_cast<const int*>(R.A.flag + 1), ciC);
    return hipGetLastError();
}

// Gather counts of one level into R.off (R.off[rows] = total).
hipError_t dom_counts(const ReplanLayout& R, int rows, int N, const int* rp, const int* ci, hipStream_t s) {
    launch_kernel(k_rp_dom_count, dim3(grid(rows + 1)), dim3(kRpThreads), 0, s, rows, N, rp, ci, R.cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return scan(R, R.cnt, R.off, rows + 1, s);
}

hipError_t dom_place(const ReplanLayout& R, int rows, int N, int nd, const int* rp, const int* ci, const int* perm,
                     int* ptr, int* blk, int* ab, hipStream_t s) {
    hipError_t e = dom_counts(R, rows, N, rp, ci, s);
    if (e != hipSuccess) return e;
    launch_kernel(k_rp_dom_fill, dim3(grid(rows)), dim3(kRpThreads), 0, s, rows, N, rp, ci,
                  static_cast<const int*>(R.off), perm, blk, ab);
    launch_kernel(k_rp_dom_ptr, dim3(grid(nd + 1)), dim3(kRpThreads), 0, s, rows, N, nd,
                  static_cast<const int*>(R.off), ptr);
    return hipGetLastError();
}

}  // namespace

ReplanLayout replan_layout(char* ws, int V, int NS, int G, long long nnzb, size_t* total) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = ws ? ws + off : nullptr;
        off += round_up(std::max<size_t>(bytes, 1));
        return p;
    };
    const size_t I = sizeof(int), m = static_cast<size_t>(std::max<long long>(nnzb, 1));
    const size_t ns = static_cast<size_t>(NS);
    ReplanLayout R{};
    size_t hb = 0;
    hierarchy_layout(nullptr, NS, kMaxLv, &hb);
    R.H = hierarchy_layout(take(hb), NS, kMaxLv, nullptr);
    size_t ab = 0;
    assemble_layout(nullptr, NS, static_cast<long long>(m), &ab);
    R.A = assemble_layout(take(ab), NS, static_cast<long long>(m), nullptr);
    R.rows = reinterpret_cast<int*>(take(I * m));
    R.cols = reinterpret_cast<int*>(take(I * m));
    R.rp0 = reinterpret_cast<int*>(take(I * (ns + 1)));
    R.ci0 = reinterpret_cast<int*>(take(I * m));
    R.perm = reinterpret_cast<int*>(take(I * m));
    for (int k = 0; k < 2; ++k) {
        R.rpX[k] = reinterpret_cast<int*>(take(I * (ns + 1)));
        R.ciX[k] = reinterpret_cast<int*>(take(I * m));
    }
    R.up = reinterpret_cast<int*>(take(I * ns));
    R.cnt = reinterpret_cast<int*>(take(I * (ns + 2)));
    R.off = reinterpret_cast<int*>(take(I * (ns + 2)));
    R.srp = reinterpret_cast<int*>(take(I * (ns + 1)));
    R.tptr = reinterpret_cast<int*>(take(I * (ns + 1)));
    R.lead1 = reinterpret_cast<int*>(take(I * ns));
    R.lmask = reinterpret_cast<uint64_t*>(take(sizeof(uint64_t) * ns));
    R.gcnt = reinterpret_cast<int*>(take(I * (G + 1)));
    R.g_u1 = reinterpret_cast<int*>(take(I * (G + 1)));
    R.gstore = reinterpret_cast<int*>(take(I * 3 * G));
    R.t_grp = reinterpret_cast<int*>(take(I * ns));
    R.anc1 = reinterpret_cast<int*>(take(I * kMaxLv * ns));
    R.lpos = reinterpret_cast<int*>(take(I * kMaxLv * ns));
    R.cpp = reinterpret_cast<int*>(take(I * kMaxLv * (ns + 1)));
    R.map = reinterpret_cast<int*>(take(I * static_cast<size_t>(V)));
    R.remap = reinterpret_cast<int*>(take(I * ns));
    R.counts = reinterpret_cast<ReplanCounts*>(take(sizeof(ReplanCounts)));
    size_t sb = 0;
    const int n_scan = std::max(NS + 2, G + 2);
    rocprim::exclusive_scan(nullptr, sb, static_cast<int*>(nullptr), static_cast<int*>(nullptr), 0, n_scan,
                            rocprim::plus<int>());
    R.scan_bytes = sb;
    R.scan_tmp = take(sb);
    if (total) *total = off;
    return R;
}

hipError_t replan_validate_order_hierarchy(const ReplanLayout& R, int V, int NS, int N, int L_cap, long long nnzb,
                                           const int* row_ptr, const int* col_idx, const int* map, const int* remap,
                                           hipStream_t s) {
    launch_kernel(k_rp_counts_init, dim3(1), dim3(64), 0, s, R.counts);
    launch_kernel(k_rp_check_rows, dim3(grid(V)), dim3(kRpThreads), 0, s, V, nnzb, row_ptr, col_idx, R.counts);
    launch_kernel(k_rp_check_sym, dim3(grid(V)), dim3(kRpThreads), 0, s, V, nnzb, row_ptr, col_idx, R.counts);
    launch_kernel(k_rp_fill, dim3(grid(nnzb)), dim3(kRpThreads), 0, s, R.rows, nnzb, -1);
    launch_kernel(k_rp_slot_keys, dim3(grid(V)), dim3(kRpThreads), 0, s, V, nnzb, row_ptr, col_idx, map, R.rows,
                  R.cols);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // slot order: the rows of H permuted to slots, columns ascending
    if ((e = launch_assemble_sort(R.A, NS, nnzb, R.rows, R.cols, R.rp0, s)) != hipSuccess) return e;
    launch_kernel(k_rp_store, dim3(1), dim3(64), 0, s, &R.counts->nnz_distinct,
                  static_cast<const int*>(R.A.flag + 1));
    launch_kernel(k_rp_cols, dim3(grid(nnzb)), dim3(kRpThreads), 0, s, nnzb, R.A.cb,
                  static_cast<const uint64_t*>(R.A.key_sorted), static_cast<const int*>(R.A.seg_start),
                  static_cast<const int*>(R.A.flag + 1), R.ci0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = copy_ints(R.perm, R.A.pos_sorted, static_cast<size_t>(nnzb), s)) != hipSuccess) return e;
    const HierPattern pat{R.rp0, R.ci0, nullptr, nnzb};
    return launch_hierarchy(R.H, NS, V, N, L_cap, remap, pat, s);
}

hipError_t replan_sizes(const ReplanLayout& R, const ReplanShape& S, hipStream_t s) {
    const int NS = S.NS, G = S.G, RG = S.RG, L = S.L;
    hipError_t e;
    // level 0: inversion gathers and the two SpMV storages
    if ((e = dom_counts(R, NS, S.N, R.rp0, R.ci0, s)) != hipSuccess) return e;
    launch_kernel(k_rp_store, dim3(1), dim3(64), 0, s, &R.counts->ndomblk[0], static_cast<const int*>(R.off + NS));
    launch_kernel(k_rp_sym_keep, dim3(grid(NS + 1)), dim3(kRpThreads), 0, s, NS, RG,
                  static_cast<const int*>(R.rp0), static_cast<const int*>(R.ci0), R.cnt);
    if ((e = scan(R, R.cnt, R.srp, NS + 1, s)) != hipSuccess) return e;
    launch_kernel(k_rp_sym_trans, dim3(grid(NS + 1)), dim3(kRpThreads), 0, s, NS, RG,
                  static_cast<const int*>(R.rp0), static_cast<const int*>(R.ci0), R.cnt);
    if ((e = scan(R, R.cnt, R.tptr, NS + 1, s)) != hipSuccess) return e;
    launch_kernel(k_rp_group_sizes, dim3(grid(G)), dim3(kRpThreads), 0, s, G, RG, NS, static_cast<const int*>(R.rp0),
                  static_cast<const int*>(R.srp), static_cast<const int*>(R.tptr), R.gstore);
    // level-1 restriction
    launch_kernel(k_rp_lead1, dim3(grid(NS)), dim3(kRpThreads), 0, s, NS, S.N, L,
                  static_cast<const int*>(R.H.sn + NS), R.lead1, R.lmask);
    launch_kernel(k_rp_group_units, dim3(grid(G + 1)), dim3(kRpThreads), 0, s, G, RG, NS,
                  static_cast<const int*>(R.lead1), R.gcnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = scan(R, R.gcnt, R.g_u1, G + 1, s)) != hipSuccess) return e;
    // coarse levels; each level's block count is read back to size the next
    // level's sort (sorting a bound instead costs a full-length sort per
    // level: 4-5 ms over the 16 levels of the membrane with bodies)
    long long nF = S.nnzb;
    for (int l = 1; l < L; ++l) {
        const int* rpF = l == 1 ? R.rp0 : R.rpX[(l - 1) & 1];
        const int* ciF = l == 1 ? R.ci0 : R.ciX[(l - 1) & 1];
        if ((e = coarsen_level(R, NS, l, S.units[l - 1], S.units[l], nF, rpF, ciF, R.rpX[l & 1], R.ciX[l & 1], s)) !=
            hipSuccess)
            return e;
        launch_kernel(k_rp_store, dim3(1), dim3(64), 0, s, &R.counts->nnzA[l], static_cast<const int*>(R.A.flag + 1));
        if ((e = dom_counts(R, S.units[l], S.N, R.rpX[l & 1], R.ciX[l & 1], s)) != hipSuccess) return e;
        launch_kernel(k_rp_store, dim3(1), dim3(64), 0, s, &R.counts->ndomblk[l],
                      static_cast<const int*>(R.off + S.units[l]));
        if (l + 1 < L) {  // queued behind the gather counts, which run meanwhile
            int nC = 0;
            if ((e = hipMemcpyAsync(&nC, R.A.flag + 1, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
            if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
            nF = nC;
        }
    }
    // writers of levels >= 2
    if (L > 2) {
        const int S1 = S.units[1], cb = R.A.cb;
        launch_kernel(k_rp_anc1, dim3(grid(NS)), dim3(kRpThreads), 0, s, NS, RG, L, static_cast<const int*>(R.H.sn),
                      static_cast<const int*>(R.lead1), R.anc1, R.t_grp);
        for (int l = 2; l < L; ++l) {
            launch_kernel(k_rp_writer_keys, dim3(grid(S1)), dim3(kRpThreads), 0, s, S1, NS, l, cb,
                          static_cast<const int*>(R.anc1), static_cast<const int*>(R.t_grp),
                          static_cast<const int*>(R.g_u1), R.A.key, R.A.pos, R.lpos);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            size_t bytes = R.A.tmp_bytes;
            if ((e = rocprim::radix_sort_pairs(R.A.tmp, bytes, R.A.key, R.A.key_sorted, R.A.pos, R.A.pos_sorted, S1,
                                               0, 2 * cb, s)) != hipSuccess)
                return e;
            launch_kernel(k_rp_writer_place, dim3(grid(S1)), dim3(kRpThreads), 0, s, S1, NS, l, cb,
                          static_cast<const uint64_t*>(R.A.key_sorted), static_cast<const int*>(R.A.pos_sorted),
                          R.counts, R.lpos);
            launch_kernel(k_rp_writer_ptr, dim3(grid(S.units[l] + 1)), dim3(kRpThreads), 0, s, S.units[l], NS, l, cb,
                          static_cast<const uint64_t*>(R.A.key_sorted), static_cast<const ReplanCounts*>(R.counts),
                          R.cpp);
        }
        launch_kernel(k_rp_group_writers, dim3(grid(G)), dim3(kRpThreads), 0, s, G, NS, L,
                      static_cast<const int*>(R.g_u1), static_cast<const int*>(R.lpos), R.counts);
    }
    return hipGetLastError();
}

hipError_t replan_place(const ReplanLayout& R, const PlacedShape& P, const PlanDest& D, hipStream_t s) {
    const ReplanShape& S = P.S;
    const int NS = S.NS, G = S.G, RG = S.RG, L = S.L, W1 = P.W1;
    const size_t nnzb = static_cast<size_t>(S.nnzb);
    hipError_t e;
    // slot-ordered pattern and the SpMV storage
    if ((e = copy_ints(D.rp0, R.rp0, NS + 1, s)) != hipSuccess) return e;
    if ((e = copy_ints(D.ci0, R.ci0, nnzb, s)) != hipSuccess) return e;
    if (P.sym) {
        launch_kernel(k_rp_sym_fill, dim3(grid(NS)), dim3(kRpThreads), 0, s, NS, RG, static_cast<const int*>(R.rp0),
                      static_cast<const int*>(R.ci0), static_cast<const int*>(R.perm),
                      static_cast<const int*>(R.srp), D.sci, D.perm_src, D.srow);
        launch_kernel(k_rp_sym_tidx, dim3(grid(NS)), dim3(kRpThreads), 0, s, NS, RG, static_cast<const int*>(R.rp0),
                      static_cast<const int*>(R.ci0), static_cast<const int*>(R.srp),
                      static_cast<const int*>(D.sci), static_cast<const int*>(R.tptr), D.tidx);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = copy_ints(D.srp, R.srp, NS + 1, s)) != hipSuccess) return e;
        if ((e = copy_ints(D.tptr, R.tptr, NS + 1, s)) != hipSuccess) return e;
        if (D.perm_full != D.perm_src && (e = copy_ints(D.perm_full, R.perm, nnzb, s)) != hipSuccess) return e;
    } else if ((e = copy_ints(D.perm_src, R.perm, nnzb, s)) != hipSuccess) {
        return e;
    }
    // restriction and prolongation
    if ((e = copy_ints(D.lead1, R.lead1, NS, s)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(D.lmask, R.lmask, sizeof(uint64_t) * NS, hipMemcpyDeviceToDevice, s)) != hipSuccess)
        return e;
    if (L > 1 && (e = copy_ints(D.anc, R.H.sn + NS, static_cast<size_t>(L - 1) * NS, s)) != hipSuccess) return e;
    if ((e = copy_ints(D.g_u1, R.g_u1, G + 1, s)) != hipSuccess) return e;
    const long long gw1 = static_cast<long long>(G) * W1;
    launch_kernel(k_rp_fill, dim3(grid(gw1)), dim3(kRpThreads), 0, s, D.gu1_slot, gw1, -1);
    launch_kernel(k_rp_fill64, dim3(grid(gw1)), dim3(kRpThreads), 0, s, D.gu1_mask, gw1);
    if (L > 1)
        launch_kernel(k_rp_gu1, dim3(grid(NS)), dim3(kRpThreads), 0, s, NS, RG, W1, static_cast<const int*>(R.lead1),
                      static_cast<const uint64_t*>(R.lmask), static_cast<const int*>(R.g_u1), D.gu1_slot,
                      D.gu1_mask);
    launch_kernel(k_rp_gw, dim3(G), dim3(64), 0, s, L, W1, P.GW, NS, static_cast<const int*>(R.g_u1),
                  static_cast<const int*>(R.anc1), static_cast<const int*>(R.lpos), D.gw_pos, D.gw_li, D.gw_mask);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (L > 2) {
        const long long n = static_cast<long long>(G) * (L - 2) * W1;
        launch_kernel(k_rp_gtab, dim3(grid(n)), dim3(kRpThreads), 0, s, G, L, W1, NS, static_cast<const int*>(R.g_u1),
                      static_cast<const int*>(R.anc1), static_cast<const int*>(R.lpos), D.ganc, D.gpos, D.gmask);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        for (int l = 2; l < L; ++l)
            if ((e = copy_ints(D.cp_ptr[l], R.cpp + static_cast<size_t>(l) * (NS + 1), S.units[l] + 1, s)) !=
                hipSuccess)
                return e;
    }
    // inversion gathers of level 0 (caller block order)
    if ((e = dom_place(R, NS, S.N, S.ndom[0], R.rp0, R.ci0, R.perm, D.dom_ptr[0], D.dom_blk[0], D.dom_ab[0], s)) !=
        hipSuccess)
        return e;
    // coarse levels: pattern, reduction plan, inversion gathers
    for (int l = 1; l < L; ++l) {
        const int* rpF = l == 1 ? R.rp0 : R.rpX[(l - 1) & 1];
        const int* ciF = l == 1 ? R.ci0 : R.ciX[(l - 1) & 1];
        const long long nF = P.nnzA[l - 1];
        if ((e = coarsen_level(R, NS, l, S.units[l - 1], S.units[l], nF, rpF, ciF, R.rpX[l & 1], R.ciX[l & 1], s)) !=
            hipSuccess)
            return e;
        if ((e = copy_ints(D.red_ptr[l], R.A.seg_start, static_cast<size_t>(P.nnzA[l]) + 1, s)) != hipSuccess)
            return e;
        if (l == 1) {  // sources in caller block order
            launch_kernel(k_rp_gather, dim3(grid(nF)), dim3(kRpThreads), 0, s, nF, static_cast<const int*>(R.perm),
                          static_cast<const int*>(R.A.pos_sorted), D.red_src[1]);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        } else if ((e = copy_ints(D.red_src[l], R.A.pos_sorted, static_cast<size_t>(nF), s)) != hipSuccess) {
            return e;
        }
        if ((e = dom_place(R, S.units[l], S.N, S.ndom[l], R.rpX[l & 1], R.ciX[l & 1], nullptr, D.dom_ptr[l],
                           D.dom_blk[l], D.dom_ab[l], s)) != hipSuccess)
            return e;
    }
    return hipGetLastError();
}

}  // namespace maspcg
