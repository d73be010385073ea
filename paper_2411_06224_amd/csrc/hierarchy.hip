// Supernode hierarchy on the device (Sec. 4.1; Supp. Alg. 2-5): at every
// level the units of a domain coupled by stored blocks form connected
// components, each a supernode of the next level, numbered inside its domain
// by its lowest lane and globally in domain order.
//
// One level:
//   1. adjacency masks: for every stored block (s, t) of the slot-ordered
//      pattern, with units u = sn(s), w = sn(t) of the current level in the
//      same domain, bit lane(w) is OR-ed into mask[u] (the coarse pattern is
//      the image of the fine one, so no coarse matrix is needed);
//   2. one wave per domain: Warshall closure of the lane masks (for every
//      lane k, a lane whose mask holds k takes k's mask), so each occupied
//      lane ends with the lane set of its component; the lowest set lane is
//      its representative; a ballot gives the domain's representatives and
//      their count;
//   3. an exclusive scan of the counts numbers the domains' supernodes; a
//      unit's next-level id is its domain's offset plus the number of
//      representatives below its own;
//   4. every slot's unit is mapped to the next level.
#include <algorithm>

#include "launch.hpp"

namespace maspcg {
namespace {

constexpr int kHThreads = 256;

// Level 0: slot s is its own unit if occupied; the level state starts with
// NS units (occupied slots: V) and is finished at once for a single domain.
__global__ void k_h_init(int NS, int V, int N, int L_cap, const int* __restrict__ remap, int* __restrict__ sn,
                         HierState* __restrict__ st) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < NS) sn[s] = remap[s] >= 0 ? s : -1;
    if (s == 0) {
        st->n_units = NS;
        st->occupied = V;
        st->levels = 1;
        st->bad = 0;
        st->units[0] = NS;
        for (int l = 1; l < kMaxLv; ++l) st->units[l] = 0;
        st->done = (NS + N - 1) / N == 1 || L_cap <= 1;
    }
}

__global__ void k_h_clear_masks(int NS, const HierState* __restrict__ st, unsigned long long* __restrict__ mask) {
    if (st->done) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < st->n_units) mask[i] = 0ull;
}

__device__ __forceinline__ void or_mask(int u, int w, int N, unsigned long long& m) {
    const int du = u / N;
    if (w >= 0 && w != u && w / N == du) m |= 1ull << (w - du * N);
}

// Adjacency masks from the slot-ordered pattern (rows and columns are slots;
// the analysed pattern is symmetric).
__global__ void k_h_masks(int NS, int N, const int* __restrict__ rp, const int* __restrict__ ci,
                          const int* __restrict__ sn, const HierState* __restrict__ st,
                          unsigned long long* __restrict__ mask) {
    if (st->done) return;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= NS) return;
    const int u = sn[s];
    if (u < 0) return;
    unsigned long long m = 0ull;
    for (int p = rp[s]; p < rp[s + 1]; ++p) or_mask(u, sn[ci[p]], N, m);
    if (m) atomicOr(mask + u, m);
}

// The same from a pattern in the caller's node order (row i is slot map[i]),
// symmetrised: block (i, c) links both units.  A row range or column outside
// the pattern raises st->bad and is skipped.
__global__ void k_h_masks_nodes(int V, int N, long long nnzb, const int* __restrict__ rp, const int* __restrict__ ci,
                                const int* __restrict__ map, const int* __restrict__ sn, HierState* __restrict__ st,
                                unsigned long long* __restrict__ mask) {
    if (st->done) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V) return;
    const int p0 = rp[i], p1 = rp[i + 1];
    if (p0 < 0 || p1 < p0 || p1 > nnzb) {
        atomicOr(&st->bad, 1);
        return;
    }
    const int u = sn[map[i]];
    if (u < 0) return;
    const int du = u / N;
    unsigned long long m = 0ull;
    for (int p = p0; p < p1; ++p) {
        const int c = ci[p];
        if (c < 0 || c >= V) {
            atomicOr(&st->bad, 1);
            continue;
        }
        const int w = sn[map[c]];
        if (w >= 0 && w != u && w / N == du) {
            m |= 1ull << (w - du * N);
            atomicOr(mask + w, 1ull << (u - du * N));
        }
    }
    if (m) atomicOr(mask + u, m);
}

// One wave per domain of the current level: lane a < N holds unit d N + a.
// occ0 (level 0): units are occupied where the remap says so.  Domains past
// the current count write a zero count (the scan runs over the largest
// domain count).
__global__ void k_h_components(int N, int max_dom, const unsigned long long* __restrict__ mask,
                               const int* __restrict__ occ0, const HierState* __restrict__ st, int* __restrict__ rep,
                               int* __restrict__ cnt) {
    if (st->done) return;
    const int d = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int a = threadIdx.x & 63;
    if (d >= max_dom) return;  // whole wave
    const int n_units = st->n_units;
    const int n_dom = (n_units + N - 1) / N;
    if (d >= n_dom) {
        if (a == 0) cnt[d] = 0;
        return;
    }
    const int u = d * N + a;
    const bool live = a < N && u < n_units && (occ0 == nullptr || occ0[u] >= 0);
    unsigned long long m = live ? (mask[u] | (1ull << a)) : 0ull;
    for (int k = 0; k < N; ++k) {
        const unsigned long long mk = __shfl(m, k, 64);
        if ((m >> k) & 1ull) m |= mk;
    }
    const int r = live ? __ffsll(static_cast<unsigned long long>(m)) - 1 : -1;
    const unsigned long long reps = __ballot(live && r == a);
    if (a == 0) cnt[d] = __popcll(reps);
    // lowest lane of the component | rank of that lane among the domain's representatives
    if (live) rep[u] = r | (__popcll(reps & ((1ull << r) - 1ull)) << 8);
}

// up[u] = offset of the unit's domain + rank of its representative.
__global__ void k_h_number(int N, const int* __restrict__ rep, const int* __restrict__ off,
                           const int* __restrict__ occ0, const HierState* __restrict__ st, int* __restrict__ up) {
    if (st->done) return;
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= st->n_units) return;
    const bool live = occ0 == nullptr || occ0[u] >= 0;
    up[u] = live ? off[u / N] + (rep[u] >> 8) : -1;
}

__global__ void k_h_lift(int NS, const int* __restrict__ up, const int* __restrict__ sn,
                         const HierState* __restrict__ st, int* __restrict__ snext) {
    if (st->done) return;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= NS) return;
    const int u = sn[s];
    snext[s] = u >= 0 ? up[u] : -1;
}

// Closes a level: total = the number of next-level units.  Nothing merged:
// the hierarchy ends without this level; otherwise it is kept, and a single
// domain or the level cap ends the hierarchy after it.
__global__ void k_h_advance(int N, int L_cap, const int* __restrict__ total, HierState* __restrict__ st) {
    if (threadIdx.x != 0 || st->done) return;
    const int S = *total;
    if (S == st->occupied) {
        st->done = 1;
        return;
    }
    const int l = st->levels;
    st->units[l] = S;
    st->levels = l + 1;
    st->n_units = S;
    st->occupied = S;
    if ((S + N - 1) / N == 1 || l + 1 >= L_cap) st->done = 1;
}

// Units of every node at every level in node order (-1 past the last level),
// and [levels, units...] (levels = -1 for an invalid pattern).
__global__ void k_h_export(int V, int NS, const int* __restrict__ map, const int* __restrict__ sn,
                           const HierState* __restrict__ st, int* __restrict__ out_units, int* __restrict__ out_sn) {
    const long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int L = st->levels;
    if (t < static_cast<long long>(kMaxLv) * V) {
        const int l = static_cast<int>(t / V), i = static_cast<int>(t - static_cast<long long>(l) * V);
        out_sn[t] = l < L ? sn[static_cast<size_t>(l) * NS + map[i]] : -1;
    }
    if (t <= kMaxLv) out_units[t] = t == 0 ? (st->bad ? -1 : L) : (t - 1 < L ? st->units[t - 1] : 0);
}

}  // namespace

HierLayout hierarchy_layout(char* ws, int NS, int L_max, size_t* total) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = ws ? ws + off : nullptr;
        off += (bytes + 255) / 256 * 256;
        return p;
    };
    HierLayout H;
    const int max_dom = NS;  // domain counts are at most NS / N; NS bounds every N
    H.mask = reinterpret_cast<unsigned long long*>(take(sizeof(unsigned long long) * NS));
    H.sn = reinterpret_cast<int*>(take(sizeof(int) * static_cast<size_t>(NS) * L_max));
    H.rep = reinterpret_cast<int*>(take(sizeof(int) * NS));
    H.up = reinterpret_cast<int*>(take(sizeof(int) * NS));
    H.cnt = reinterpret_cast<int*>(take(sizeof(int) * (max_dom + 1)));
    H.off = reinterpret_cast<int*>(take(sizeof(int) * (max_dom + 1)));
    H.totals = reinterpret_cast<int*>(take(sizeof(int) * ((max_dom + 1 + 1023) / 1024 + 1)));
    H.st = reinterpret_cast<HierState*>(take(sizeof(HierState)));
    if (total) *total = off;
    return H;
}

hipError_t launch_hierarchy(const HierLayout& H, int NS, int V, int N, int L_cap, const int* remap,
                            const HierPattern& pat, hipStream_t s) {
    const int max_dom = (NS + N - 1) / N;
    launch_kernel(k_h_init, dim3(ceil_div(NS, kHThreads)), dim3(kHThreads), 0, s, NS, V, N, L_cap, remap, H.sn, H.st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // every level is queued; once the state says done, the rest return at once
    for (int l = 0; l + 1 < L_cap; ++l) {
        const int* sn = H.sn + static_cast<size_t>(l) * NS;
        int* snext = H.sn + static_cast<size_t>(l + 1) * NS;
        const int* occ0 = l == 0 ? remap : nullptr;
        launch_kernel(k_h_clear_masks, dim3(ceil_div(NS, kHThreads)), dim3(kHThreads), 0, s, NS,
                      static_cast<const HierState*>(H.st), H.mask);
        if (pat.map)
            launch_kernel(k_h_masks_nodes, dim3(ceil_div(V, kHThreads)), dim3(kHThreads), 0, s, V, N, pat.nnzb,
                          pat.rp, pat.ci, pat.map, sn, H.st, H.mask);
        else
            launch_kernel(k_h_masks, dim3(ceil_div(NS, kHThreads)), dim3(kHThreads), 0, s, NS, N, pat.rp, pat.ci, sn,
                          static_cast<const HierState*>(H.st), H.mask);
        launch_kernel(k_h_components, dim3(ceil_div(max_dom, kHThreads / 64)), dim3(kHThreads), 0, s, N, max_dom,
                      static_cast<const unsigned long long*>(H.mask), occ0, static_cast<const HierState*>(H.st),
                      H.rep, H.cnt);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = launch_scan(H.cnt, max_dom, H.off, H.totals, s)) != hipSuccess) return e;
        launch_kernel(k_h_number, dim3(ceil_div(NS, kHThreads)), dim3(kHThreads), 0, s, N,
                      static_cast<const int*>(H.rep), static_cast<const int*>(H.off), occ0,
                      static_cast<const HierState*>(H.st), H.up);
        launch_kernel(k_h_lift, dim3(ceil_div(NS, kHThreads)), dim3(kHThreads), 0, s, NS, static_cast<const int*>(H.up),
                      sn, static_cast<const HierState*>(H.st), snext);
        launch_kernel(k_h_advance, dim3(1), dim3(64), 0, s, N, L_cap, static_cast<const int*>(H.off + max_dom), H.st);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_hier_export(const HierLayout& H, int V, int NS, const int* map, int* out_units, int* out_sn,
                              hipStream_t s) {
    const long long n = std::max<long long>(static_cast<long long>(kMaxLv) * V, kMaxLv + 1);
    launch_kernel(k_h_export, dim3(ceil_div(n, kHThreads)), dim3(kHThreads), 0, s, V, NS, map,
                  static_cast<const int*>(H.sn), static_cast<const HierState*>(H.st), out_units, out_sn);
    return hipGetLastError();
}

}  // namespace maspcg
