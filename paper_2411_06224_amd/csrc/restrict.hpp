// Restriction of a residual (or of q = H p) to the coarse levels (C_l r of
// Supp. Eq. 6), computed by the workgroup that owns a group of level-0
// domains.
//
// restrict_load() issues every plan load of the group at once into
// registers, early in a kernel, so that no wait for them sits on the
// kernel's path; restrict_group() then works from those registers and the
// vector staged in shared memory.  Each sum reads its terms from shared
// memory as independent loads, several at a time, and adds them in
// ascending order, non-members as +0.0 (which leaves every partial sum's
// bits unchanged: a sum that starts at +0.0 never becomes -0.0), so the
// result is the member-only sum in lane order.
#pragma once

#include "launch.hpp"

namespace maspcg {

// Shared memory of the restriction, in doubles, for a group with at most W1
// level-1 units: the group's level-1 sums r1s[3 W1].
__host__ __device__ inline int restrict_smem_doubles(int RG, int W1, int L) {
    (void)RG;
    (void)L;
    return 3 * W1;
}

// The group's range of level-1 units: first unit and count.
struct GroupUnits {
    int lo, n;
};

// Plan entries a thread holds in registers: thread t takes component t % 3
// of the group's level-1 unit t / 3 and, in pass p < kWP of the writers of
// levels >= 2, of writer (t + p blockDim) / 3 (the common case,
// restrict_fast_ok, needs one pass; entries of later passes are loaded
// where they are used).
template <int kWP = 1>
struct RestrictLoads {
    GroupUnits gu;
    int u1_slot;          // lowest slot of the thread's level-1 unit (-1 pad)
    uint64_t u1_mask;     // lanes of its domain in that unit
    int w_pos[kWP];       // the thread's writers: partial position (-1 pad), table entry
    int w_li[kWP];
    uint64_t w_mask[kWP]; // the writer's members among the group's level-1 units
};

// Issues the loads of the group's plan, all at once and unconditionally (at
// clamped indices), so that no branch separates them from the loads issued
// before them and a wait for those need not wait for these too.
template <int kWP = 1>
__device__ inline RestrictLoads<kWP> restrict_load(const SolverView& v, int g) {
    RestrictLoads<kWP> R;
    const int t = threadIdx.x;
    const int u1_lo = v.g_u1[g];
    R.gu = v.L >= 2 ? GroupUnits{u1_lo, v.g_u1[g + 1] - u1_lo} : GroupUnits{0, 0};
    const long long i1 = static_cast<long long>(g) * v.W1 + min(t / 3, v.W1 - 1);
    R.u1_slot = v.gu1_slot[i1];
    R.u1_mask = v.gu1_mask[i1];
#pragma unroll
    for (int p = 0; p < kWP; ++p) {
        const long long iw = static_cast<long long>(g) * v.GW + min((t + p * static_cast<int>(blockDim.x)) / 3, v.GW - 1);
        R.w_pos[p] = v.gw_pos[iw];
        R.w_li[p] = v.gw_li[iw];
        R.w_mask[p] = v.gw_mask[iw];
    }
    return R;
}

// Makes the plan registers ready now (their loads completed long before):
// called before a kernel's last stores, so that using them afterwards waits
// for nothing.  Loads and stores share one counter, and after a loop whose
// loads the compiler cannot count, a first use of an early-loaded register
// waits for every outstanding access -- the stores just issued included.
template <int kWP>
__device__ __forceinline__ void restrict_ready(const RestrictLoads<kWP>& R) {
    asm volatile("" ::"v"(R.u1_slot), "v"(R.u1_mask));
#pragma unroll
    for (int p = 0; p < kWP; ++p) asm volatile("" ::"v"(R.w_pos[p]), "v"(R.w_li[p]), "v"(R.w_mask[p]));
}

// sum over the members m < n of mask, in ascending m, of x[3 m] (x in shared
// memory): eight independent loads per round, each round's members added as
// a balanced tree (non-members as +0.0) and the round's sum to the total
__device__ __forceinline__ double masked_sum_tree(const double* x, uint64_t mask, int n) {
    double s = 0.0;
    for (int m0 = 0; m0 < n; m0 += 8) {
        double a[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const double e = x[3 * min(m0 + j, n - 1)];
            a[j] = (m0 + j < n && ((mask >> (m0 + j)) & 1u)) ? e : 0.0;
        }
        s += ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    }
    return s;
}

// rs[3*RG]: the group's vector in slot order (zero on slots >= NS), visible
// to the workgroup (barrier done by the caller); R: restrict_load(v, g);
// sm: restrict_smem_doubles of shared memory.  Writes out1 (level 1: the
// residual r_1, or q_1 of q = H p) for the level-1 supernodes of the group
// (lanes of the unit in ascending order) and, for every level l >= 2, one
// partial sum per (group, level-l supernode) into outpart at the position
// the plan assigns (the group's level-1 supernodes below it, ascending).
// No atomics: every output has exactly one writer.  Contains a barrier when
// L > 2 (every thread must call it).  kFast: the caller guarantees
// GW <= blockDim.x and W1 <= 64 (restrict_fast_ok), and the restriction then
// reads no global memory -- a load here would make the stores before it
// wait too.
__host__ __device__ inline bool restrict_fast_ok(int W1, int GW, int threads) {
    return W1 <= 64 && 3 * W1 <= threads && 3 * GW <= threads;
}

template <bool kFast = false, int kWP = 1>
__device__ inline void restrict_group(const SolverView& v, int g, const RestrictLoads<kWP>& R, const double* rs,
                                      double* sm, double* __restrict__ out1, double* __restrict__ outpart) {
    if (v.L < 2) return;
    const int t = threadIdx.x, N = v.N;
    const int u1_lo = R.gu.lo, n1 = R.gu.n;
    double* r1s = sm;
    // one thread per (level-1 unit, component); passes after the first
    // (not in the fast case) load their entries here
    for (int o = t; o < 3 * n1; o += blockDim.x) {
        const int i = o / 3, c = o - 3 * i;
        int slot = R.u1_slot;
        uint64_t m = R.u1_mask;
        if (!kFast && o != t) {
            slot = v.gu1_slot[static_cast<long long>(g) * v.W1 + i];
            m = v.gu1_mask[static_cast<long long>(g) * v.W1 + i];
        }
        const int first = (slot - g * v.RG) / N * N;  // the unit's domain, local slots
        const double s1 = masked_sum_tree(rs + 3 * first + c, m, N);
        out1[3 * u1_lo + o] = s1;
        r1s[o] = s1;
        if (kFast) break;
    }
    if (v.L <= 2) return;
    __syncthreads();
    // one thread per (writer of levels >= 2, component): the first kWP
    // passes from the preloaded entries, later ones (not in the fast case)
    // load theirs; a group's writers come first in its table, then pads, so
    // a thread stops at its first pad
    auto write = [&](int e, int c, int pos, int li, uint64_t m) {
        double s2;
        if (kFast || v.W1 <= 64) {
            s2 = masked_sum_tree(r1s + c, m, n1);
        } else {  // more level-1 units in the group than mask bits: compare ancestors
            const int* anc = v.ganc + static_cast<long long>(g) * (v.L - 2) * v.W1 + (li / v.W1) * v.W1;
            const int a = anc[li % v.W1];
            s2 = 0.0;
            for (int j = 0; j < n1; ++j)
                if (anc[j] == a) s2 += r1s[3 * j + c];
        }
        (void)e;
        outpart[3 * pos + c] = s2;
    };
    int o = t;
#pragma unroll
    for (int p = 0; p < kWP; ++p) {
        if (o >= 3 * v.GW) return;
        const int e = o / 3, c = o - 3 * e;
        if (R.w_pos[p] < 0) return;
        write(e, c, R.w_pos[p], R.w_li[p], R.w_mask[p]);
        if (kFast) return;
        o += blockDim.x;
    }
    for (; o < 3 * v.GW; o += blockDim.x) {
        const int e = o / 3, c = o - 3 * e;
        const long long k = static_cast<long long>(g) * v.GW + e;
        const int pos = v.gw_pos[k];
        if (pos < 0) return;
        write(e, c, pos, v.gw_li[k], v.gw_mask[k]);
    }
}

// restrict_group with the fast path when the host found it applicable
// (v.rfast: tables that fit blocks of 256 threads and more).
template <int kWP>
__device__ inline void restrict_group_any(const SolverView& v, int g, const RestrictLoads<kWP>& R, const double* rs,
                                          double* sm, double* __restrict__ out1, double* __restrict__ outpart) {
    if (v.rfast)
        restrict_group<true, kWP>(v, g, R, rs, sm, out1, outpart);
    else
        restrict_group<false, kWP>(v, g, R, rs, sm, out1, outpart);
}

}  // namespace maspcg
