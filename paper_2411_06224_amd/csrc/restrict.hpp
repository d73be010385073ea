// Restriction of a residual to the coarse levels (C_l r of Supp. Eq. 6),
// computed by the workgroup that owns a group of level-0 domains.
//
// restrict_load() issues every plan load of the group at once into
// registers, and restrict_stage() writes them to shared memory later, just
// before the barrier that publishes the residual: the loads' latency overlaps
// whatever the kernel does in between, and no wait for them sits on the
// kernel's early path.  restrict_group() then works from shared memory only.
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

// Plan entries a thread holds in registers between restrict_load and
// restrict_stage: its slot's entries and kPlanRegs entries of the group's
// level >= 2 table; a larger table's remainder is loaded by restrict_stage.
constexpr int kPlanRegs = 1;

struct RestrictLoads {
    GroupUnits gu;
    int up0, lead;  // raw loads at clamped indices: restrict_stage drops the
    uint64_t lmask; // ones outside the group's slots and table row
    int anc[kPlanRegs], pos[kPlanRegs];
    uint64_t gm[kPlanRegs];
};

// Issues the loads of the group's plan: level-1 unit, writer flag and member
// mask of every slot, and for every level l >= 2 the ancestor, writer
// position and writer mask of every level-1 unit of the group (entry
// (l - 2) W1 + i of the group's row of the level-major tables, so that the
// whole row is one coalesced range and no load waits for another).  One
// slot per thread: RG = D0 N <= 128 and every kernel that restricts runs at
// least 256 threads.  The loads are issued unconditionally, at clamped
// indices (arrays of NS entries stand in for tables a shallow hierarchy does
// not have), so that no branch separates them from the loads issued before
// them and a wait for those need not wait for these too.
__device__ inline RestrictLoads restrict_load(const SolverView& v, int g) {
    RestrictLoads R;
    const int t = threadIdx.x;
    const bool lv1 = v.L >= 2, lv2 = v.L > 2;
    const int u1_lo = v.g_u1[g];
    R.gu = lv1 ? GroupUnits{u1_lo, v.g_u1[g + 1] - u1_lo} : GroupUnits{0, 0};
    const int sc = min(g * v.RG + t, v.NS - 1);
    R.up0 = (lv1 ? v.anc : v.lead1)[sc];
    R.lead = v.lead1[sc];
    R.lmask = v.lmask[sc];
    const int tot = lv2 ? (v.L - 2) * v.W1 : 0;
    const long long row = static_cast<long long>(g) * tot;
    const long long last = lv2 ? static_cast<long long>(v.G) * tot - 1 : 0;
#pragma unroll
    for (int j = 0; j < kPlanRegs; ++j) {
        const long long e = min(row + t + j * static_cast<int>(blockDim.x), last);
        R.anc[j] = (lv2 ? v.ganc : v.lead1)[e];
        R.pos[j] = (lv2 ? v.gpos : v.lead1)[e];
        R.gm[j] = (lv2 ? v.gmask : v.lmask)[e];
    }
    return R;
}

// Writes the loaded plan to shared memory (needs a barrier before
// restrict_group) and returns the group's level-1 unit range.
__device__ inline GroupUnits restrict_stage(const SolverView& v, int g, const RestrictLoads& R, double* sm) {
    if (v.L < 2) return R.gu;
    const RestrictSmem S = restrict_layout(v, sm);
    const int t = threadIdx.x;
    if (t < v.RG) {
        const bool in = g * v.RG + t < v.NS;
        S.up0[t] = in ? R.up0 : -1;
        S.lead[t] = in ? R.lead : -1;
        S.lmask[t] = in ? R.lmask : 0;
    }
    const int tot = (v.L - 2) * v.W1;
#pragma unroll
    for (int j = 0; j < kPlanRegs; ++j) {
        const int o = t + j * static_cast<int>(blockDim.x);
        if (o < tot) {
            S.anc[o] = R.anc[j];
            S.pos[o] = R.pos[j];
            S.gmask[o] = R.gm[j];
        }
    }
    const long long row = static_cast<long long>(g) * tot;
    for (int o = t + kPlanRegs * static_cast<int>(blockDim.x); o < tot; o += blockDim.x) {
        S.anc[o] = v.ganc[row + o];
        S.pos[o] = v.gpos[row + o];
        S.gmask[o] = v.gmask[row + o];
    }
    return R.gu;
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
