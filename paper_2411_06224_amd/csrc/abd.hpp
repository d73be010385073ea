// Two-level reduction of affine-body contact Hessians (abd.hip): scratch
// layout and launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace maspcg {

struct AbdLayout {
    int* row_ptr;      // [n_nodes + 1] node pairs of each row node (first level)
    int* pair_row;     // [m] row node of each distinct pair
    int* pair_col;     // [m] column node
    double* pair_val;  // [9 m] summed 3x3 block of each pair
    int *cnt, *off;    // [m + 1] sub-blocks per pair and their exclusive scan
    int* flag;         // input check
    void* scan_tmp;
    size_t scan_bytes;
    void* asm_ws;      // scratch of the first level's block-list assembly
};

AbdLayout abd_layout(char* ws, int n_nodes, long long m, size_t* total);
hipError_t launch_abd_check(const AbdLayout& L, long long m, int n_nodes, const int* r, const int* c, hipStream_t s);
hipError_t launch_abd_pair_rows(const AbdLayout& L, int n_nodes, hipStream_t s);
// cnt and off (exclusive scan, off[np] = total) of pairs (pr, pc).
hipError_t launch_abd_count(const AbdLayout& L, long long np, const int* pr, const int* pc, const int* is_body,
                            hipStream_t s);
hipError_t launch_abd_expand(const AbdLayout& L, long long np, const int* pr, const int* pc, const double* C,
                             const int* node_row, const int* is_body, const double* xbar, int* out_rows,
                             int* out_cols, double* out_blk, hipStream_t s);

}  // namespace maspcg
