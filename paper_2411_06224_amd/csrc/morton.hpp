// Device Morton-order partition (morton.hip): scratch layout and launcher.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace maspcg {

struct MortonLayout {
    double* part;            // bounding-box partials
    double* box;             // lo[3], extent[3]
    uint64_t* code;          // [n]
    uint64_t* code_sorted;   // [n]
    int* id;                 // [n]
    int* id_sorted;          // [n]
    void* sort_tmp;          // radix sort scratch of sort_bytes
    size_t sort_bytes;
};

// Layout of the scratch from ws (ws = nullptr: sizes only; *total receives
// the bytes needed).
MortonLayout morton_layout(char* ws, int n, size_t* total);
// part[i] = domain of node i: nodes in Morton order of pos (3 n doubles),
// ties by node id, N per domain.
hipError_t launch_morton_partition(const MortonLayout& L, int n, int N, const double* pos, int* part,
                                   hipStream_t s);

}  // namespace maspcg
