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
#include "launch.hpp"

namespace maspcg {
namespace {

constexpr int kHThreads = 256;

__global__ void k_h_fill64(unsigned long long* __restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// Level 0: slot s is its own unit if occupied.
__global__ void k_h_init(int NS, const int* __restrict__ remap, int* __restrict__ sn) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < NS) sn[s] = remap[s] >= 0 ? s : -1;
}

__global__ void k_h_masks(int NS, int N, const int* __restrict__ rp, const int* __restrict__ ci,
                          const int* __restrict__ sn, unsigned long long* __restrict__ mask) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= NS) return;
    const int u = sn[s];
    if (u < 0) return;
    const int du = u / N;
    unsigned long long m = 0ull;
    for (int p = rp[s]; p < rp[s + 1]; ++p) {
        const int w = sn[ci[p]];
        if (w >= 0 && w != u && w / N == du) m |= 1ull << (w - du * N);
    }
    if (m) atomicOr(mask + u, m);
}

// One wave per domain of the current level: lane a < N holds unit d N + a.
// occ: units < n_units are occupied unless the level-0 remap says otherwise.
__global__ void k_h_components(int n_units, int N, int n_dom, const unsigned long long* __restrict__ mask,
                               const int* __restrict__ occ0, int* __restrict__ rep, int* __restrict__ cnt) {
    const int d = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int a = threadIdx.x & 63;
    if (d >= n_dom) return;  // whole wave
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
__global__ void k_h_number(int n_units, int N, const int* __restrict__ rep, const int* __restrict__ off,
                           const int* __restrict__ occ0, int* __restrict__ up) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n_units) return;
    const bool live = occ0 == nullptr || occ0[u] >= 0;
    up[u] = live ? off[u / N] + (rep[u] >> 8) : -1;
}

__global__ void k_h_lift(int NS, const int* __restrict__ up, const int* __restrict__ sn, int* __restrict__ snext) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= NS) return;
    const int u = sn[s];
    snext[s] = u >= 0 ? up[u] : -1;
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
    H.mask = reinterpret_cast<unsigned long long*>(take(sizeof(unsigned long long) * NS));
    H.sn = reinterpret_cast<int*>(take(sizeof(int) * static_cast<size_t>(NS) * L_max));
    H.rep = reinterpret_cast<int*>(take(sizeof(int) * NS));
    H.up = reinterpret_cast<int*>(take(sizeof(int) * NS));
    H.cnt = reinterpret_cast<int*>(take(sizeof(int) * (NS + 1)));
    H.off = reinterpret_cast<int*>(take(sizeof(int) * (NS + 1)));
    H.totals = reinterpret_cast<int*>(take(sizeof(int) * ((NS + 1 + 1023) / 1024 + 1)));
    if (total) *total = off;
    return H;
}

hipError_t launch_hier_init(const HierLayout& H, int NS, const int* remap, hipStream_t s) {
    launch_kernel(k_h_init, dim3(ceil_div(NS, kHThreads)), dim3(kHThreads), 0, s, NS, remap, H.sn);
    return hipGetLastError();
}

hipError_t launch_hier_level(const HierLayout& H, int l, int NS, int N, int n_units, const int* rp, const int* ci,
                             const int* remap, hipStream_t s) {
    const int n_dom = (n_units + N - 1) / N;
    const int* sn = H.sn + static_cast<size_t>(l) * NS;
    int* snext = H.sn + static_cast<size_t>(l + 1) * NS;
    const int* occ0 = l == 0 ? remap : nullptr;
    launch_kernel(k_h_fill64, dim3(ceil_div(n_units, kHThreads)), dim3(kHThreads), 0, s, H.mask, n_units);
    launch_kernel(k_h_masks, dim3(ceil_div(NS, kHThreads)), dim3(kHThreads), 0, s, NS, N, rp, ci, sn, H.mask);
    launch_kernel(k_h_components, dim3(ceil_div(n_dom, kHThreads / 64)), dim3(kHThreads), 0, s, n_units, N, n_dom,
                  static_cast<const unsigned long long*>(H.mask), occ0, H.rep, H.cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = launch_scan(H.cnt, n_dom, H.off, H.totals, s)) != hipSuccess) return e;
    launch_kernel(k_h_number, dim3(ceil_div(n_units, kHThreads)), dim3(kHThreads), 0, s, n_units, N,
                  static_cast<const int*>(H.rep), static_cast<const int*>(H.off), occ0, H.up);
    launch_kernel(k_h_lift, dim3(ceil_div(NS, kHThreads)), dim3(kHThreads), 0, s, NS, static_cast<const int*>(H.up),
                  sn, snext);
    return hipGetLastError();
}

}  // namespace maspcg
