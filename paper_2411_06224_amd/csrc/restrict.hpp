// Restriction of a residual to the coarse levels (C_l r of Supp. Eq. 6),
// computed by the workgroup that owns a group of level-0 domains.
//
// restrict_prefetch() issues every plan load of the group at once (no
// barrier), so its latency overlaps whatever the kernel does next;
// restrict_group() then works from shared memory only.
#pragma once

#include "launch.hpp"

namespace maspcg {

// Shared memory of the restriction, in doubles, for a group of RG slots with
// at most W1 level-1 units and L levels: r1s[3 W1] doubles, lmask[RG] and
// gmask[(L-2) W1] 64-bit masks, then up0[RG], lead[RG], anc[(L-2) W1],
// pos[(L-2) W1] ints.
__host__ __device__ inline int restrict_smem_doubles(int RG, int W1, int L) {
    const int lv = L > 2 ? L - 2 : 0;
    const int ints = 2 * RG + 2 * lv * W1;
    return 3 * W1 + RG + lv * W1 + (ints + 1) / 2;
}

struct RestrictSmem {
    double* r1s;
    uint64_t *lmask, *gmask;
    int *up0, *lead, *anc, *pos;
};

__device__ inline RestrictSmem restrict_layout(const SolverView& v, double* sm) {
    const int lv = v.L > 2 ? v.L - 2 : 0;
    RestrictSmem r;
    r.r1s = sm;
    r.lmask = reinterpret_cast<uint64_t*>(sm + 3 * v.W1);
    r.gmask = r.lmask + v.RG;
    r.up0 = reinterpret_cast<int*>(r.gmask + lv * v.W1);
    r.lead = r.up0 + v.RG;
    r.anc = r.lead + v.RG;
    r.pos = r.anc + lv * v.W1;
    return r;
}

// The group's range of level-1 units: first unit and count.
struct GroupUnits {
    int lo, n;
};

// Loads the group's plan (level-1 unit and writer flag of every slot, and
// for every level l >= 2 the ancestor and writer position of every level-1
// unit of the group, from the per-group padded tables, so that no load
// waits for another) into shared memory.  Needs a barrier before use.
// Returns the group's level-1 unit range for restrict_group.
__device__ inline GroupUnits restrict_prefetch(const SolverView& v, int g, double* sm) {
    if (v.L < 2) return GroupUnits{0, 0};
    const RestrictSmem S = restrict_layout(v, sm);
    const int RG = v.RG, W = v.W1, slot0 = g * RG;
    const int u1_lo = v.g_u1[g], n1 = v.g_u1[g + 1] - u1_lo;
    for (int i = threadIdx.x; i < RG; i += blockDim.x) {
        const int slot = slot0 + i;
        const bool in = slot < v.NS;
        S.up0[i] = in ? v.anc[slot] : -1;
        S.lead[i] = in ? v.lead1[slot] : -1;
        S.lmask[i] = in ? v.lmask[slot] : 0;
    }
    if (v.L > 2) {
        const int tot = (v.L - 2) * W;
        for (int o = threadIdx.x; o < tot; o += blockDim.x) {
            const int l = 2 + o / W, i = o - (l - 2) * W;
            S.anc[o] = v.ganc[l][static_cast<long long>(g) * W + i];
            S.pos[o] = v.gpos[l][static_cast<long long>(g) * W + i];
            S.gmask[o] = v.gmask[l][static_cast<long long>(g) * W + i];
        }
    }
    return GroupUnits{u1_lo, n1};
}

// rs[3*RG]: the group's residual in slot order (zero on slots >= NS), and
// the prefetched plan, both visible to the workgroup (barrier done by the
// caller).  Writes r_1 for the level-1 supernodes of the group (each summed
// by its lowest slot, lanes in ascending order) and, for every level l >= 2,
// one partial sum per (group, level-l supernode) at the position the plan
// assigns (summed over the group's level-1 supernodes below it, ascending).
// No atomics: every output has exactly one writer.
__device__ inline void restrict_group(const SolverView& v, GroupUnits gu, const double* rs, double* sm) {
    if (v.L < 2) return;
    const RestrictSmem S = restrict_layout(v, sm);
    const int RG = v.RG, N = v.N;
    const int u1_lo = gu.lo, n1 = gu.n;
    for (int o = threadIdx.x; o < 3 * RG; o += blockDim.x) {
        const int ls = o / 3, c = o - 3 * ls;
        const int u = S.lead[ls];
        if (u < 0) continue;
        const int first = (ls / N) * N;
        double s = 0.0;
        if (v.W1 <= 64) {
            // the unit's lanes from the precomputed mask, ascending
            for (uint64_t m = S.lmask[ls]; m; m &= m - 1) s += rs[3 * (first + __ffsll(static_cast<unsigned long long>(m)) - 1) + c];
        } else {
            for (int a = 0; a < N; ++a)
                if (S.up0[first + a] == u) s += rs[3 * (first + a) + c];
        }
        v.r1[3 * u + c] = s;
        S.r1s[3 * (u - u1_lo) + c] = s;
    }
    if (v.L > 2) {
        __syncthreads();
        const int tot = 3 * (v.L - 2) * n1;
        for (int o = threadIdx.x; o < tot; o += blockDim.x) {
            const int li = o / 3, c = o - 3 * li;
            const int l = li / n1, i = li - l * n1;
            const int pos = S.pos[l * v.W1 + i];
            if (pos < 0) continue;
            double s = 0.0;
            if (v.W1 <= 64) {
                for (uint64_t m = S.gmask[l * v.W1 + i]; m; m &= m - 1) s += S.r1s[3 * (__ffsll(static_cast<unsigned long long>(m)) - 1) + c];
            } else {
                const int* anc = S.anc + l * v.W1;
                const int a = anc[i];
                for (int j = 0; j < n1; ++j)
                    if (anc[j] == a) s += S.r1s[3 * j + c];
            }
            v.cpart[3 * pos + c] = s;
        }
    }
}

}  // namespace maspcg
