// Level-0 domains in Morton (Z-order) of the node positions: the domain
// ordering of the earlier MAS preconditioner that the connectivity-aware
// partition replaces (Sec. 4.1), for the ordering comparison.
//
// Bounding box by a two-pass min/max reduction (exact in any order), 63-bit
// codes (each coordinate scaled to 21 bits over the box, bits interleaved
// x, y, z), a stable radix sort of (code, node) pairs -- equal codes keep
// ascending node ids -- and node k-th in that order goes to domain k / N.
#include <rocprim/device/device_radix_sort.hpp>

#include <algorithm>

#include "launch.hpp"
#include "morton.hpp"

namespace maspcg {
namespace {

constexpr int kMortonThreads = 256;
constexpr int kBoxBlocks = 256;  // workgroups of the first bounding-box pass

// Per-workgroup min and max of each coordinate over a grid-stride range.
__global__ void __launch_bounds__(kMortonThreads) k_box_partial(int n, const double* __restrict__ pos,
                                                                 double* __restrict__ part) {
    __shared__ double sm[6][kMortonThreads];
    const int t = threadIdx.x;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = blockIdx.x * kMortonThreads + t; i < n; i += gridDim.x * kMortonThreads)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double x = pos[3LL * i + c];
            lo[c] = fmin(lo[c], x);
            hi[c] = fmax(hi[c], x);
        }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        sm[c][t] = lo[c];
        sm[3 + c][t] = hi[c];
    }
    __syncthreads();
    for (int o = kMortonThreads / 2; o > 0; o >>= 1) {
        if (t < o)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                sm[c][t] = fmin(sm[c][t], sm[c][t + o]);
                sm[3 + c][t] = fmax(sm[3 + c][t], sm[3 + c][t + o]);
            }
        __syncthreads();
    }
    if (t < 6) part[6 * blockIdx.x + t] = sm[t][0];
}

// The box from the partials; box[0..2] = lo, box[3..5] = extent (at least
// the smallest positive double, as for a flat set of points).
__global__ void __launch_bounds__(64) k_box_final(int nparts, const double* __restrict__ part,
                                                   double* __restrict__ box) {
    if (threadIdx.x != 0) return;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int b = 0; b < nparts; ++b)
        for (int c = 0; c < 3; ++c) {
            lo[c] = fmin(lo[c], part[6 * b + c]);
            hi[c] = fmax(hi[c], part[6 * b + 3 + c]);
        }
    for (int c = 0; c < 3; ++c) {
        box[c] = lo[c];
        box[3 + c] = fmax(hi[c] - lo[c], 2.2250738585072014e-308);
    }
}

// Spreads the low 21 bits of v so that bit i lands on bit 3 i.
__device__ inline uint64_t spread3(uint64_t v) {
    v &= 0x1FFFFFull;
    v = (v | (v << 32)) & 0x1F00000000FFFFull;
    v = (v | (v << 16)) & 0x1F0000FF0000FFull;
    v = (v | (v << 8)) & 0x100F00F00F00F00Full;
    v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

// Code and node id of every node.  The scaled coordinate is computed as
// ((x - lo) / extent) * (2^21 - 1), rounded down and clamped.
__global__ void __launch_bounds__(kMortonThreads) k_codes(int n, const double* __restrict__ pos,
                                                           const double* __restrict__ box,
                                                           uint64_t* __restrict__ code, int* __restrict__ id) {
    const int i = blockIdx.x * kMortonThreads + threadIdx.x;
    if (i >= n) return;
    uint64_t q[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double s = __dmul_rn(__ddiv_rn(pos[3LL * i + c] - box[c], box[3 + c]), 2097151.0);
        const double f = fmin(fmax(floor(s), 0.0), 2097151.0);
        q[c] = static_cast<uint64_t>(f);
    }
    code[i] = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
    id[i] = i;
}

__global__ void __launch_bounds__(kMortonThreads) k_domains(int n, int N, const int* __restrict__ sorted_id,
                                                             int* __restrict__ part) {
    const int k = blockIdx.x * kMortonThreads + threadIdx.x;
    if (k < n) part[sorted_id[k]] = k / N;
}

size_t sort_bytes(int n) {
    size_t bytes = 0;
    rocprim::radix_sort_pairs(nullptr, bytes, static_cast<uint64_t*>(nullptr), static_cast<uint64_t*>(nullptr),
                              static_cast<int*>(nullptr), static_cast<int*>(nullptr), n, 0, 63);
    return bytes;
}

size_t round_up(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

MortonLayout morton_layout(char* ws, int n, size_t* total) {
    MortonLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = ws ? ws + off : nullptr;
        off += round_up(bytes > 0 ? bytes : 1);
        return p;
    };
    L.part = reinterpret_cast<double*>(take(sizeof(double) * 6 * kBoxBlocks));
    L.box = reinterpret_cast<double*>(take(sizeof(double) * 6));
    L.code = reinterpret_cast<uint64_t*>(take(sizeof(uint64_t) * n));
    L.code_sorted = reinterpret_cast<uint64_t*>(take(sizeof(uint64_t) * n));
    L.id = reinterpret_cast<int*>(take(sizeof(int) * n));
    L.id_sorted = reinterpret_cast<int*>(take(sizeof(int) * n));
    L.sort_bytes = sort_bytes(n);
    L.sort_tmp = take(L.sort_bytes);
    if (total) *total = off;
    return L;
}

hipError_t launch_morton_partition(const MortonLayout& L, int n, int N, const double* pos, int* part,
                                   hipStream_t s) {
    const int nb = std::min(kBoxBlocks, ceil_div(n, kMortonThreads));
    launch_kernel(k_box_partial, dim3(nb), dim3(kMortonThreads), 0, s, n, pos, L.part);
    launch_kernel(k_box_final, dim3(1), dim3(64), 0, s, nb, static_cast<const double*>(L.part), L.box);
    const int g = ceil_div(n, kMortonThreads);
    launch_kernel(k_codes, dim3(g), dim3(kMortonThreads), 0, s, n, pos, static_cast<const double*>(L.box), L.code,
                  L.id);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    size_t bytes = L.sort_bytes;
    e = rocprim::radix_sort_pairs(L.sort_tmp, bytes, L.code, L.code_sorted, L.id, L.id_sorted, n, 0, 63, s);
    if (e != hipSuccess) return e;
    launch_kernel(k_domains, dim3(g), dim3(kMortonThreads), 0, s, n, N, static_cast<const int*>(L.id_sorted), part);
    return hipGetLastError();
}

}  // namespace maspcg
