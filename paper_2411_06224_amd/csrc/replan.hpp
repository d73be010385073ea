// Solver plans of a new sparsity pattern derived on the device (Sec. 4.2;
// Supp. Alg. 2-5): the contacts of a Newton step change the pattern of H,
// the level-0 partition stays.  Every array is the one the host analysis
// computes for the same pattern and partition, bit for bit.
//
// Pass 1 (replan_validate_order_hierarchy, then replan_sizes): the pattern
// is checked, put in slot order by a stable sort of (slot row, slot column)
// keys, the hierarchy is built, and every level is coarsened far enough to
// count the blocks, gather entries, coarse partials and writers that size
// the solver workspace; the slot-ordered pattern, the symmetric-storage row
// pointers and the restriction tables indexed by level-1 unit stay in the
// replan workspace.  Pass 2 (replan_place) writes the plans into the solver
// workspace, coarsening every level again with the exact sizes.
#pragma once

#include <cstdint>

#include "launch.hpp"

namespace maspcg {

// assemble.hip: launch_assemble_sort from keys and list positions already in
// L.key / L.pos (keys of entries to leave out: (1 << 2 cb) - 1);
// clear_flag: reset L.flag first.
hipError_t launch_assemble_sort_keys(const AsmLayout& L, int n_rows, long long n_in, int* row_ptr, hipStream_t s,
                                     bool clear_flag);

// Counts read back between the passes (one struct in the replan workspace).
struct ReplanCounts {
    int bad;                 // bit 0: row_ptr, 1: column range, 2: column order, 3: diagonal, 4: symmetry
    int nnz_distinct;        // distinct blocks of the slot-ordered pattern
    int nnzA[kMaxLv];        // blocks of A_l (level 0: the pattern)
    int ndomblk[kMaxLv];     // inversion gather entries of each level
    int cbase[kMaxLv + 1];   // first coarse-partial position of each level >= 2; cbase[L] = n_cpart
    int gw_max;              // most writers of one group
};

struct ReplanLayout {
    HierLayout H;            // hierarchy: sn[l NS + slot], level state
    AsmLayout A;             // sort scratch over nnzb entries, keys over NS indices
    int *rows, *cols;        // slot-order sort input [nnzb]
    int *rp0, *ci0, *perm;   // slot-ordered pattern [NS + 1], [nnzb], [nnzb] (perm: caller block of each)
    int *rpX[2], *ciX[2];    // coarse patterns of consecutive levels [NS + 1], [nnzb]
    int* up;                 // level-l unit -> level-(l+1) unit [NS]
    int *cnt, *off;          // per-row counts and their scan [NS + 2]
    int *srp, *tptr;         // symmetric storage row pointers [NS + 1]
    int* lead1;              // [NS]
    uint64_t* lmask;         // [NS]
    int *gcnt, *g_u1;        // per-group level-1 units and their scan [G + 1]
    int* gstore;             // per group: stored blocks of the full and symmetric storage, transposed entries [3 G]
    int* t_grp;              // group of each level-1 unit [NS]
    int *anc1, *lpos;        // [kMaxLv NS]: level-l unit / partial position of each level-1 unit
    int* cpp;                // [kMaxLv (NS + 1)]: cp_ptr of each level
    int *map, *remap;        // the partition's node -> slot map [V] and its inverse [NS]
    ReplanCounts* counts;
    void* scan_tmp;
    size_t scan_bytes;
};

ReplanLayout replan_layout(char* ws, int V, int NS, int G, long long nnzb, size_t* total);

// Pass 1a: checks of the caller's pattern (node order), the slot-ordered
// pattern and the hierarchy (level cap L_cap).
hipError_t replan_validate_order_hierarchy(const ReplanLayout& R, int V, int NS, int N, int L_cap, long long nnzb,
                                           const int* row_ptr, const int* col_idx, const int* map, const int* remap,
                                           hipStream_t s);

struct ReplanShape {
    int V, N, NS, M, L, G, RG;
    long long nnzb;
    int units[kMaxLv], ndom[kMaxLv];
};

// Pass 1b, after the level count is known: counts of every level (each
// coarse level's block count is read back to size the next level's sort),
// the level-1 restriction tables and the writers of levels >= 2.
hipError_t replan_sizes(const ReplanLayout& R, const ReplanShape& S, hipStream_t s);

// Destinations in the solver workspace.
struct PlanDest {
    int *perm_src, *perm_full, *rp0, *ci0, *lead1, *anc, *g_u1, *gu1_slot, *gw_pos, *gw_li;
    uint64_t *lmask, *gu1_mask, *gw_mask, *gmask;
    int *ganc, *gpos;
    int *srp, *sci, *tptr, *tidx;
    uint8_t* srow;
    int *red_ptr[kMaxLv], *red_src[kMaxLv], *dom_ptr[kMaxLv], *dom_blk[kMaxLv], *dom_ab[kMaxLv], *cp_ptr[kMaxLv];
};

struct PlacedShape {
    ReplanShape S;
    int sym, W1, GW;
    int nnzA[kMaxLv];  // exact, from pass 1
};

// Pass 2: every plan array of the solver workspace.
hipError_t replan_place(const ReplanLayout& R, const PlacedShape& P, const PlanDest& D, hipStream_t s);

}  // namespace maspcg
