// Host-side symbolic analysis for the MAS preconditioner: ordering, hierarchy
// and every gather / reduction plan the device phases consume.  Runs once per
// sparsity pattern (the paper reorders once at load, Sec. 4.2).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace maspcg {

constexpr int kMaxLevels = 16;
// The symmetric storage keeps a group's transposed-entry list in LDS; groups
// with more entries than this use the full storage.
constexpr int kMaxTransposed = 4096;
// The group kernels deal workgroup b to XCD b % kXcdCount, each XCD taking a
// contiguous range of groups (xcd_group on the device).
constexpr int kXcdCount = 8;

struct Plan {
    int V = 0;      // nodes (block rows of H)
    int N = 0;      // domain size
    int M = 0;      // level-0 domains (partition parts)
    int No = 0;     // slack of Eq. num_subdomains
    int NS = 0;     // level-0 slots = M * N
    int L = 0;      // levels
    int nnzb = 0;

    std::vector<int> part, map, remap;  // map[V] node -> slot, remap[NS] slot -> node or -1

    // H permuted into slot order (rows and columns are slots):
    // block k of the permuted matrix is block perm_src[k] of the caller's H.
    std::vector<int> rp0, ci0, perm_src;

    std::vector<int> units;  // per level: level 0 -> NS slots, l >= 1 -> supernodes
    std::vector<int> ndom;   // per level
    std::vector<std::vector<int>> up;  // up[l][unit of level l] -> unit of level l+1 (-1: empty slot)

    // Coarse matrices A_l = C H C^T over level-l units, l = 1..L-1 (index l).
    // A_l[t] = sum over k in [red_ptr[l][t], red_ptr[l][t+1]) of A_{l-1}[red_src[l][k]]
    // with A_0 the permuted H.
    std::vector<std::vector<int>> rpA, ciA, red_ptr, red_src;

    // Inversion gather plan per level: the upper (a <= b) in-domain blocks of
    // each domain: block index into A_l (or the permuted H at level 0), and
    // the lane pair packed as a | (b << 8).
    std::vector<std::vector<int>> dom_ptr, dom_blk, dom_ab;

    // Restriction to level 1, per slot: the level-1 unit if this slot is the
    // lowest lane of that unit in its domain (it sums the unit), else -1.
    std::vector<int> lead1;

    // Work groups of the vector kernels: D0 consecutive level-0 domains
    // (RG = D0 * N slots); G groups.  Every reduction produces one partial
    // per group.
    int D0 = 0, RG = 0, G = 0;
    std::vector<int> g_u1;  // [G+1] first level-1 unit of each group
    // Coarse restriction for l >= 2 through per-group partial sums: the
    // level-1 units of a group are summed per level-l ancestor; the partial
    // of (group, ancestor) is written by the lowest such level-1 unit of the
    // group to position lead_pos[l][t] (-1: not a writer).  The partials of
    // level-l unit u occupy [cp_ptr[l][u], cp_ptr[l][u+1]) of one array.
    std::vector<std::vector<int>> anc1;      // [l][S_1]: level-l unit of each level-1 unit
    std::vector<std::vector<int>> lead_pos;  // [l][S_1]
    std::vector<std::vector<int>> cp_ptr;    // [l][S_l + 1]
    int n_cpart = 0;                         // partial positions over all levels
    // The same per group, padded so that a group's entries sit at a fixed
    // place: ganc[l] / gpos[l] hold anc1[l] / lead_pos[l] of the group's
    // level-1 units at [g * W1 + i] (i < W1 = the most level-1 units in a
    // group; -1 past the group's own).
    int W1 = 1;
    std::vector<std::vector<int>> ganc, gpos;
    // Member masks of the same sums: lmask[slot] (leader slots): the lanes of
    // its domain in its level-1 unit; gmask[l][g * W1 + i] (writers): the
    // group's level-1 units (local index) below the same level-l unit.
    // Used when W1 <= 64.
    std::vector<uint64_t> lmask;
    std::vector<std::vector<uint64_t>> gmask;
    // The same restriction by output, padded per group so that thread t of a
    // group's workgroup finds its entry at a fixed place: level-1 unit i of
    // group g at [g * W1 + i]: its lowest slot (-1 pad) and lane mask; the
    // writers of levels >= 2 at [g * GW + e] (GW = the most writers of one
    // group): partial position (-1 pad), entry (l - 2) * W1 + i of the
    // group's ganc / gpos row, and member mask (W1 <= 64).
    std::vector<int> gu1_slot;
    std::vector<uint64_t> gu1_mask;
    int GW = 1;
    std::vector<int> gw_pos, gw_li;
    std::vector<uint64_t> gw_mask;
    // Prolongation: unit of every slot at levels 1..L-1, [(l-1) * NS + slot], -1 = empty.
    std::vector<int> anc;

    // Group-symmetric storage of the slot-ordered H used by the solver's SpMV
    // kernels (sym = true).  Within a group of RG rows a row keeps its blocks
    // whose column lies outside the group and, of the group's own columns,
    // only those >= the row (diagonal and upper part): an internal
    // off-diagonal block (i, j), j > i, also stands for H_ji = H_ij^T, so each
    // group-internal block pair is stored once.  srp[NS + 1] / sci / sperm:
    // stored rows, columns (slots) and source blocks (caller order); srow:
    // local row of each stored block; tptr[NS + 1] / tidx: for every row j
    // the stored blocks (i, j), i < j, of its group, ascending.  maxT: the
    // most transposed entries of one group.
    bool sym = false;
    std::vector<int> srp, sci, sperm, tptr, tidx;
    std::vector<uint8_t> srow;
    int maxT = 0;

    // SpMV group of each workgroup when the groups' stored blocks are
    // uneven (empty: the contiguous per-XCD mapping of the group kernels)
    std::vector<int> gorder;

    std::vector<int> sn;  // [L * V] unit of each node per level (level 0 = slot), for reports
};

// Workgroup order of the SpMV from the stored blocks of each group (empty:
// the contiguous per-XCD mapping).
std::vector<int> spmv_group_order(const std::vector<long long>& cnt);

// Returns "" on success or a message describing the invalid input.
// part / n_parts (optional): a caller-given level-0 partition, used instead
// of the recursive bisection of the node graph.
std::string analyze(int n_rows, int nnzb, const int32_t* row_ptr, const int32_t* col_idx, const int32_t* g_ptr,
                    const int32_t* g_adj, int N, int max_levels, Plan& out, const int32_t* part = nullptr,
                    int n_parts = 0);

}  // namespace maspcg
