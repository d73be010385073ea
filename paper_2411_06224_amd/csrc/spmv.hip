// 3x3-block CSR sparse matrix-vector products (Supp. Eq. 2: T_spmv of a PCG
// iteration).
//
// A workgroup owns a group of consecutive block rows and streams the
// group's blocks, which are contiguous in memory, in chunks: thread t takes
// blocks t, t + 256, ... of the chunk (consecutive threads read consecutive
// values of each plane), multiplies each 3x3 block by its x entry and parks
// the three products in LDS.  Every (row, component) pair of the group has
// one owner thread that then adds its row's products in column order.  The
// load is balanced by blocks, not rows, so rows of 7 and 19 blocks (the two
// node classes of the tet cube) or long contact / affine rows cost the same
// per block.  Products and sums are FP64; FP32-stored values are widened on
// load.
#include "launch.hpp"
#include "restrict.hpp"

namespace maspcg {
namespace {

constexpr int kThreads = 256;
constexpr int kChunk = 1024;       // blocks staged in LDS per pass
constexpr int kUserRows = 128;     // rows per workgroup for caller matrices
// LDS planes of products are kPad doubles longer than a chunk, so that the
// three components of one row, read by neighbouring lanes at the same
// offset of consecutive planes, fall in different banks
constexpr int kPad = 1;
constexpr int kPlane = kChunk + kPad;

// acc + p[lo] + p[lo + 1] + ... + p[hi - 1], added in this order; four
// entries are loaded at a time so that their LDS latencies overlap
__device__ __forceinline__ double sum_run(double acc, const double* p, int lo, int hi) {
    int k = lo;
    for (; k + 4 <= hi; k += 4) {
        const double a0 = p[k], a1 = p[k + 1], a2 = p[k + 2], a3 = p[k + 3];
        acc = (((acc + a0) + a1) + a2) + a3;
    }
    for (; k < hi; ++k) acc += p[k];
    return acc;
}

// acc plus p[tl[tp] - cs], p[tl[tp + 1] - cs], ... in list order for the
// entries of tl[tp, te) below ce (the lists ascend); tp advances past them.
__device__ __forceinline__ double sum_listed(double acc, const double* p, const int* tl, int& tp, int te, int cs,
                                             int ce) {
    while (tp < te) {
        int kk[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) kk[j] = tp + j < te ? tl[tp + j] : ce;
        double v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = kk[j] < ce ? p[kk[j] - cs] : 0.0;
        int n = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (kk[j] < ce) {
                acc += v[j];
                ++n;
            }
        tp += n;
        if (n < 4) break;
    }
    return acc;
}

// Block values: caller layout (9 consecutive values per block) or the
// solver's planar layout (value c of block k at c * stride + k).
template <typename T, bool kPlanar>
struct Blocks {
    const T* __restrict__ v;
    long long stride;
    __device__ __forceinline__ double at(int k, int c) const {
        return kPlanar ? static_cast<double>(v[c * stride + k]) : static_cast<double>(v[9LL * k + c]);
    }
};

// The vector H multiplies: x itself, or the new search direction
// z + beta p formed on the fly from the previous one.
struct XVec {
    const double* __restrict__ x;
    __device__ __forceinline__ double at(int i) const { return x[i]; }
};
struct XDir {
    const double* __restrict__ z;
    const double* __restrict__ p;
    double beta;
    __device__ __forceinline__ double at(int i) const { return __fma_rn(beta, p[i], z[i]); }
};

// Column indices of this thread's blocks t, t + 256, ... of the chunk
// starting at cs, loaded one chunk ahead of their use so that a chunk's
// gathers need not wait for them.  The loads are unconditional, at indices
// clamped to the range's last block (none for an empty range).
constexpr int kRowPer = kChunk / kThreads;

struct ChunkCols {
    int j[kRowPer];
};

__device__ __forceinline__ ChunkCols chunk_cols(const int* __restrict__ ci, int cs, int ke) {
    ChunkCols c;
#pragma unroll
    for (int kk = 0; kk < kRowPer; ++kk) c.j[kk] = 0;
    if (cs < ke) {
#pragma unroll
        for (int kk = 0; kk < kRowPer; ++kk) c.j[kk] = ci[min(cs + static_cast<int>(threadIdx.x) + kk * kThreads, ke - 1)];
    }
    return c;
}

// The group a workgroup of the matrix-streaming kernels takes: the
// planner's order when the groups' stored blocks are uneven, else the
// contiguous per-XCD mapping of every group kernel.
__device__ __forceinline__ int spmv_group(const SolverView& v) {
    return v.gorder ? v.gorder[blockIdx.x] : xcd_group(blockIdx.x, v.G);
}

// Row sums of rows [r0, r1) of H x.  Owner o = 3 (row - r0) + c is thread
// o (acc[0]) or o - 256 (acc[1]); 3 (r1 - r0) <= 512.  prod: 3 * kPlane LDS.
// kLds: x of the columns r0 .. r1 - 1 is read from xs (LDS), the others
// through X.  first: chunk_cols(ci, rp[r0], rp[r1]), which the caller may
// load early.
template <typename T, bool kPlanar, typename X, bool kLds = false>
__device__ __forceinline__ void stream_rows(const int* __restrict__ rp, const int* __restrict__ ci,
                                            Blocks<T, kPlanar> H, X x, int r0, int r1, double* prod,
                                            double (&acc)[2], const ChunkCols& first, const double* xs = nullptr) {
    const int t = threadIdx.x;
    const int nown = 3 * (r1 - r0);
    int rb[2], re[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int o = t + q * kThreads;
        acc[q] = 0.0;
        rb[q] = re[q] = 0;
        if (o < nown) {
            const int row = r0 + o / 3;
            rb[q] = rp[row];
            re[q] = rp[row + 1];
        }
    }
    const int kb = rp[r0], ke = rp[r1];
    ChunkCols nc = first;
    for (int cs = kb; cs < ke; cs += kChunk) {
        const int ce = min(cs + kChunk, ke);
        const ChunkCols cc = nc;
#pragma unroll
        for (int kk = 0; kk < kRowPer; ++kk) {
            const int k = cs + t + kk * kThreads;
            if (k >= ce) break;
            const int j = cc.j[kk];
            double x0, x1, x2;
            const int jl = j - r0;
            if (kLds && jl >= 0 && jl < r1 - r0) {
                x0 = xs[3 * jl];
                x1 = xs[3 * jl + 1];
                x2 = xs[3 * jl + 2];
            } else {
                x0 = x.at(3 * j);
                x1 = x.at(3 * j + 1);
                x2 = x.at(3 * j + 2);
            }
            const int e = k - cs;
            prod[e] = H.at(k, 0) * x0 + H.at(k, 1) * x1 + H.at(k, 2) * x2;
            prod[kPlane + e] = H.at(k, 3) * x0 + H.at(k, 4) * x1 + H.at(k, 5) * x2;
            prod[2 * kPlane + e] = H.at(k, 6) * x0 + H.at(k, 7) * x1 + H.at(k, 8) * x2;
        }
        nc = chunk_cols(ci, cs + kChunk, ke);  // the next chunk's columns, in flight through the sums
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int o = t + q * kThreads;
            if (o < nown) {
                const int c = o % 3;
                const int lo = max(rb[q], cs), hi = min(re[q], ce);
                acc[q] = sum_run(acc[q], prod + c * kPlane, lo - cs, hi - cs);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------- symmetric storage
// Group-symmetric storage: a group keeps one copy of each internal block
// pair (the block with column >= row), used for both H_ij and H_ji = H_ij^T,
// and its blocks with a column outside the group.  Per chunk of stored blocks
// thread t multiplies block t, t + 256, ... by x of its column (to its row,
// prod planes 0..2) and, for an internal off-diagonal block, its transpose by
// x of its row (to its column, planes 3..5).  Owner o = 3 (row - r0) + c then
// adds its row's direct products in column order and its transposed entries
// in stored order.  xs: x on the group's own slots (LDS); external columns
// are gathered through X; tl: the group's transposed entries (LDS).
constexpr int kSymChunk = 512;
constexpr int kSymPlane = kSymChunk + kPad;
constexpr int kTlRegs = 4;  // transposed-list entries a thread loads ahead (a longer list's rest is loaded late)
constexpr int kSymPer = kSymChunk / kThreads;

// Column slot and local row of this thread's stored blocks t, t + 256, ...
// of the chunk starting at cs, loaded one chunk ahead (as chunk_cols).
struct SymCols {
    int j[kSymPer];
    int r[kSymPer];
};

__device__ __forceinline__ SymCols sym_cols(const SolverView& v, int cs, int ke) {
    SymCols c;
#pragma unroll
    for (int kk = 0; kk < kSymPer; ++kk) c.j[kk] = c.r[kk] = 0;
    if (cs < ke) {
#pragma unroll
        for (int kk = 0; kk < kSymPer; ++kk) {
            const int k = min(cs + static_cast<int>(threadIdx.x) + kk * kThreads, ke - 1);
            c.j[kk] = v.sci[k];
            c.r[kk] = v.srow[k];
        }
    }
    return c;
}

template <typename T, typename X>
__device__ __forceinline__ void stream_sym(const SolverView& v, const T* __restrict__ H, X xg, const double* xs,
                                           const int* tl, int tb0, int r0, int r1, double* prod, double (&acc)[2],
                                           const SymCols& first) {
    const int t = threadIdx.x;
    const int nown = 3 * (r1 - r0), rows = r1 - r0;
    const long long st = v.nsb;
    int rb[2], re[2], tp[2], te[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int o = t + q * kThreads;
        acc[q] = 0.0;
        rb[q] = re[q] = tp[q] = te[q] = 0;
        if (o < nown) {
            const int row = r0 + o / 3;
            rb[q] = v.srp[row];
            re[q] = v.srp[row + 1];
            tp[q] = v.tptr[row] - tb0;
            te[q] = v.tptr[row + 1] - tb0;
        }
    }
    const int kb = v.srp[r0], ke = v.srp[r1];
    SymCols nc = first;
    for (int cs = kb; cs < ke; cs += kSymChunk) {
        const int ce = min(cs + kSymChunk, ke);
        const SymCols cc = nc;
#pragma unroll
        for (int kk = 0; kk < kSymPer; ++kk) {
            const int k = cs + t + kk * kThreads;
            if (k >= ce) break;
            const int j = cc.j[kk];
            const int r = cc.r[kk];
            const int jl = j - r0;
            const bool internal = jl >= 0 && jl < rows;
            double x0, x1, x2;
            if (internal) {
                x0 = xs[3 * jl];
                x1 = xs[3 * jl + 1];
                x2 = xs[3 * jl + 2];
            } else {
                x0 = xg.at(3 * j);
                x1 = xg.at(3 * j + 1);
                x2 = xg.at(3 * j + 2);
            }
            const double h0 = static_cast<double>(H[k]), h1 = static_cast<double>(H[st + k]),
                         h2 = static_cast<double>(H[2 * st + k]), h3 = static_cast<double>(H[3 * st + k]),
                         h4 = static_cast<double>(H[4 * st + k]), h5 = static_cast<double>(H[5 * st + k]),
                         h6 = static_cast<double>(H[6 * st + k]), h7 = static_cast<double>(H[7 * st + k]),
                         h8 = static_cast<double>(H[8 * st + k]);
            const int e = k - cs;
            prod[e] = h0 * x0 + h1 * x1 + h2 * x2;
            prod[kSymPlane + e] = h3 * x0 + h4 * x1 + h5 * x2;
            prod[2 * kSymPlane + e] = h6 * x0 + h7 * x1 + h8 * x2;
            if (internal && jl != r) {
                const double y0 = xs[3 * r], y1 = xs[3 * r + 1], y2 = xs[3 * r + 2];
                prod[3 * kSymPlane + e] = h0 * y0 + h3 * y1 + h6 * y2;
                prod[4 * kSymPlane + e] = h1 * y0 + h4 * y1 + h7 * y2;
                prod[5 * kSymPlane + e] = h2 * y0 + h5 * y1 + h8 * y2;
            }
        }
        nc = sym_cols(v, cs + kSymChunk, ke);  // the next chunk's columns, in flight through the sums
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int o = t + q * kThreads;
            if (o < nown) {
                const int c = o % 3;
                const int lo = max(rb[q], cs), hi = min(re[q], ce);
                acc[q] = sum_run(acc[q], prod + c * kSymPlane, lo - cs, hi - cs);
                acc[q] = sum_listed(acc[q], prod + (3 + c) * kSymPlane, tl, tp[q], te[q], cs, ce);
            }
        }
        __syncthreads();
    }
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_spmv_user(int n_rows, const int* __restrict__ rp,
                                                         const int* __restrict__ ci, const T* __restrict__ val,
                                                         const double* __restrict__ x, double* __restrict__ y) {
    __shared__ double prod[3 * kPlane];
    const int r0 = blockIdx.x * kUserRows;
    const int r1 = min(r0 + kUserRows, n_rows);
    double acc[2];
    stream_rows<T, false>(rp, ci, Blocks<T, false>{val, 0}, XVec{x}, r0, r1, prod, acc,
                          chunk_cols(ci, rp[r0], rp[r1]));
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int o = threadIdx.x + q * kThreads;
        if (o < 3 * (r1 - r0)) y[3 * r0 + o] = acc[q];
    }
}

// Products per launch after the stream: q of the group's rows, the partial
// of p_k^T q and, with kRQ = 1, the restriction of q to
// the coarse levels (q1 and qpart, as restrict_group computes C_l r) from
// the plan pl loaded at the kernel's start, staged in the product planes
// (free once the stream's last barrier has passed; the host checks that
// they hold it, spmv_restrict_capacity).
template <int kRQ>
__device__ __forceinline__ void finish_pq(const SolverView& v, int g, int nown, int r0, const double (&acc)[2],
                                          const double (&pv)[2], double* prod, double* buf, const RestrictLoads<>& pl) {
    const int t = threadIdx.x;
    if constexpr (kRQ) restrict_ready(pl);
    double part = 0.0;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int o = t + q * kThreads;
        if (o < nown) {
            v.q[3LL * r0 + o] = acc[q];
            part += pv[q] * acc[q];
        }
    }
    if constexpr (kRQ) {
        double* rs = prod;
        double* rsm = prod + 3 * v.RG;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int o = t + q * kThreads;
            if (o < 3 * v.RG) rs[o] = o < nown ? acc[q] : 0.0;
        }
        part = block_sum<false>(part, buf);  // its barriers also publish rs
        if (t == 0) v.P_sigma[g] = part;
        restrict_group<true>(v, g, pl, rs, rsm, v.q1, v.qpart);  // the host checked restrict_fast_ok
    } else {
        part = block_sum<false>(part, buf);  // the kernel's last use of buf
        if (t == 0) v.P_sigma[g] = part;
    }
}

// PCG iteration k over the solver's group of slots: the new direction
// p_k = z_{k-1} + beta_{k-1} p_{k-1} (beta = rho_{k-1} / rho_{k-2} summed from
// the group partials; p_1 = z_0) is formed first on the group's own slots
// (into LDS and p_k) and, for columns outside the group, wherever H gathers
// it; q = H p_k and the partial of p_k^T q.  Every workgroup forms the same
// beta and the same fused multiply-add, so a direction entry has the same
// bits in every workgroup that reads it.
template <typename T, int kRQ>
__global__ void __launch_bounds__(kThreads) k_spmv_pq(SolverView v, const T* __restrict__ H, int k) {
    __shared__ double prod[3 * kPlane];
    __shared__ double buf[256];
    __shared__ double xs[384];
    const int t = threadIdx.x;
    const int g = spmv_group(v);
    const int r0 = g * v.RG, r1 = min(r0 + v.RG, v.NS);
    const int nown = 3 * (r1 - r0);
    // every independent load before the first wait: the rho partials first
    // (needed first; loads complete in issue order), then the group's own
    // entries of z and p_{k-1}, unconditionally at clamped indices (see
    // partials_load)
    const double* Prho = v.P_rho[(k - 1) & 1];
    const PartialLoads rl = partials_load(Prho, v.G);
    const double* pold = k > 1 ? v.p[(k - 1) & 1] : v.z;  // k = 1: p_1 = z_0 (+ 0 * z_0)
    double zo[2], po[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const long long e = 3LL * r0 + min(t + q * kThreads, nown - 1);
        zo[q] = v.z[e];
        po[q] = pold[e];
    }
    const ChunkCols c0 = chunk_cols(v.ci0, v.rp0[r0], v.rp0[r1]);
    RestrictLoads<> pl{};
    if constexpr (kRQ) pl = restrict_load(v, g);
    const int stop = v.st->done;
    keep_loads_issued();
    if (stop) return;  // after a stop nothing is written
    // rho_{k-1} from the group partials; rho_{k-2} as the previous SpMV recorded it
    const double rk2 = v.st->rho[k & 1];
    const double rk1 = partials_sum<false>(rl, Prho, v.G, buf);  // buf is next written after later barriers
    if (g == 0 && t == 0) v.st->rho[(k - 1) & 1] = rk1;
    const double beta = k > 1 ? rk1 / rk2 : 0.0;
    double* pk = v.p[k & 1];
    double pv[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int o = t + q * kThreads;
        pv[q] = 0.0;
        if (o < nown) {
            pv[q] = __fma_rn(beta, po[q], zo[q]);
            pk[3LL * r0 + o] = pv[q];
            xs[o] = pv[q];
        }
    }
    __syncthreads();
    double acc[2];
    stream_rows<T, true, XDir, true>(v.rp0, v.ci0, Blocks<T, true>{H, v.nnzb}, XDir{v.z, pold, beta}, r0, r1, prod,
                                     acc, c0, xs);
    finish_pq<kRQ>(v, g, nown, r0, acc, pv, prod, buf, pl);
}

// k_spmv_pq on the group-symmetric storage: the group forms the new
// direction on its own slots first (into LDS and p_k) and gathers it only for
// columns outside the group.
template <typename T, int kRQ>
__global__ void __launch_bounds__(kThreads) k_spmv_pq_sym(SolverView v, const T* __restrict__ H, int k) {
    __shared__ double prod[6 * kSymPlane];
    __shared__ double buf[256];
    extern __shared__ double dyn[];  // xs[3 RG] doubles + tl[maxT] ints
    const int t = threadIdx.x;
    const int g = spmv_group(v);
    const int r0 = g * v.RG, r1 = min(r0 + v.RG, v.NS);
    const int nown = 3 * (r1 - r0);
    double* xs = dyn;
    int* tl = reinterpret_cast<int*>(dyn + 3 * v.RG);
    // every independent load before the first wait: the rho partials first
    // (needed first; loads complete in issue order), then the group's own
    // entries of z and p_{k-1} and its transposed-entry list, all
    // unconditionally at clamped indices (see partials_load); the list goes
    // to LDS only after the rho sum
    const double* Prho = v.P_rho[(k - 1) & 1];
    const PartialLoads rl = partials_load(Prho, v.G);
    const double* pold = k > 1 ? v.p[(k - 1) & 1] : v.z;  // k = 1: p_1 = z_0 (+ 0 * z_0)
    double zo[2], po[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const long long e = 3LL * r0 + min(t + q * kThreads, nown - 1);
        zo[q] = v.z[e];
        po[q] = pold[e];
    }
    const int tb0 = v.tptr[r0], tn = v.tptr[r1] - tb0;
    const int* tsrc = tn > 0 ? v.tidx + tb0 : v.srp;  // srp: a stand-in with entries when the list is empty
    int tlr[kTlRegs];
#pragma unroll
    for (int j = 0; j < kTlRegs; ++j) tlr[j] = tsrc[min(t + j * kThreads, max(tn - 1, 0))];
    const SymCols c0 = sym_cols(v, v.srp[r0], v.srp[r1]);
    RestrictLoads<> pl{};
    if constexpr (kRQ) pl = restrict_load(v, g);
    const int stop = v.st->done;
    keep_loads_issued();
    if (stop) return;  // after a stop nothing is written
    const double rk2 = v.st->rho[k & 1];
    // rho_{k-1} from the group partials; rho_{k-2} as the previous SpMV recorded it
    const double rk1 = partials_sum<false>(rl, Prho, v.G, buf);  // buf is next written after later barriers
    if (g == 0 && t == 0) v.st->rho[(k - 1) & 1] = rk1;
#pragma unroll
    for (int j = 0; j < kTlRegs; ++j)
        if (t + j * kThreads < tn) tl[t + j * kThreads] = tlr[j];
    for (int e = t + kTlRegs * kThreads; e < tn; e += kThreads) tl[e] = v.tidx[tb0 + e];
    const double beta = k > 1 ? rk1 / rk2 : 0.0;
    double* pk = v.p[k & 1];
    double pv[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int o = t + q * kThreads;
        pv[q] = 0.0;
        if (o < nown) {
            pv[q] = __fma_rn(beta, po[q], zo[q]);
            pk[3LL * r0 + o] = pv[q];
        }
        if (o < 3 * v.RG) xs[o] = pv[q];
    }
    __syncthreads();
    double acc[2];
    stream_sym<T>(v, H, XDir{v.z, pold, beta}, xs, tl, tb0, r0, r1, prod, acc, c0);
    finish_pq<kRQ>(v, g, nown, r0, acc, pv, prod, buf, pl);
}

// out = b - H x in FP64 over a group, with the partials of ||out||^2 (and
// ||b||^2 for the initial residual) and, except for the final check, the
// restriction of the new residual to the coarse levels.
template <int kMode, bool kSym>
__global__ void __launch_bounds__(kThreads) k_residual(SolverView v, double* __restrict__ out) {
    __shared__ double prod[(kSym ? 6 * kSymPlane : 3 * kPlane)];
    __shared__ double scratch[kThreads / 64];
    extern __shared__ double dyn[];  // rs[3*RG] + restriction scratch (+ xs[3*RG] + tl[maxT] ints)
    if (kMode == kResidReplace && v.st->done) return;
    const int g = spmv_group(v);
    const int r0 = g * v.RG, r1 = min(r0 + v.RG, v.NS);
    double acc[2];
    const RestrictLoads<> pl = restrict_load(v, g);
    if constexpr (kSym) {
        double* xs = dyn + 3 * v.RG + restrict_smem_doubles(v.RG, v.W1, v.L);
        int* tl = reinterpret_cast<int*>(xs + 3 * v.RG);
        const int nown = 3 * (r1 - r0);
        for (int o = threadIdx.x; o < 3 * v.RG; o += kThreads) xs[o] = o < nown ? v.x[3LL * r0 + o] : 0.0;
        const int tb0 = v.tptr[r0], tn = v.tptr[r1] - tb0;
        for (int e = threadIdx.x; e < tn; e += kThreads) tl[e] = v.tidx[tb0 + e];
        __syncthreads();
        stream_sym<double>(v, v.H64, XVec{v.x}, xs, tl, tb0, r0, r1, prod, acc, sym_cols(v, v.srp[r0], v.srp[r1]));
    } else {
        stream_rows<double, true>(v.rp0, v.ci0, Blocks<double, true>{v.H64, v.nnzb}, XVec{v.x}, r0, r1, prod, acc,
                                  chunk_cols(v.ci0, v.rp0[r0], v.rp0[r1]));
    }
    restrict_ready(pl);
    double rr = 0.0, bb = 0.0;
    double* rs = dyn;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int o = threadIdx.x + q * kThreads;
        if (o < 3 * v.RG) {
            double e = 0.0;
            if (o < 3 * (r1 - r0)) {
                const long long i = 3LL * r0 + o;
                const double bv = v.b[i];
                e = bv - acc[q];
                out[i] = e;
                rr += e * e;
                bb += bv * bv;
            }
            rs[o] = e;
        }
    }
    rr = block_sum(rr, scratch);  // its barriers also publish rs
    if (kMode == kResidInit) bb = block_sum(bb, scratch);
    if (threadIdx.x == 0) {
        v.P_rr[g] = rr;
        if (kMode == kResidInit) v.P_bb[g] = bb;
    }
    if (kMode != kResidFinal) restrict_group_any(v, g, pl, rs, dyn + 3 * v.RG, v.r1, v.cpart);
}

}  // namespace

hipError_t launch_spmv_user(int n_rows, const int* rp, const int* ci, const void* val, bool f32, const double* x,
                            double* y, hipStream_t s) {
    if (n_rows <= 0) return hipSuccess;
    dim3 g(ceil_div(n_rows, kUserRows)), b(kThreads);
    if (f32)
        launch_kernel(k_spmv_user<float>, g, b, 0, s, n_rows, rp, ci, static_cast<const float*>(val), x, y);
    else
        launch_kernel(k_spmv_user<double>, g, b, 0, s, n_rows, rp, ci, static_cast<const double*>(val), x, y);
    return hipGetLastError();
}

template <int kRQ>
void launch_spmv_pq_t(const SolverView& v, bool f32, int k, hipStream_t s) {
    dim3 g(v.G), b(kThreads);
    if (v.sym && !f32) {
        const size_t shmem = sizeof(double) * 3 * v.RG + sizeof(int) * v.maxT;
        launch_kernel(k_spmv_pq_sym<double, kRQ>, g, b, shmem, s, v, static_cast<const double*>(v.H64), k);
    } else if (f32) {
        launch_kernel(k_spmv_pq<float, kRQ>, g, b, 0, s, v, static_cast<const float*>(v.H32), k);
    } else {
        launch_kernel(k_spmv_pq<double, kRQ>, g, b, 0, s, v, static_cast<const double*>(v.H64), k);
    }
}

hipError_t launch_spmv_pq(const SolverView& v, bool f32, int k, bool restrict_q, hipStream_t s) {
    if (!restrict_q)
        launch_spmv_pq_t<0>(v, f32, k, s);
    else if (v.rfast)
        launch_spmv_pq_t<1>(v, f32, k, s);
    else
        return hipErrorInvalidValue;  // the solver restricts q in the SpMV only where restrict_fast_ok holds
    return hipGetLastError();
}

int spmv_threads() { return kThreads; }

size_t spmv_restrict_capacity() { return sizeof(double) * static_cast<size_t>(min(3 * kPlane, 6 * kSymPlane)); }

template <bool kSym>
void launch_residual_t(const SolverView& v, int mode, double* out, hipStream_t s) {
    dim3 g(v.G), b(kThreads);
    size_t shmem = sizeof(double) * (3 * v.RG + restrict_smem_doubles(v.RG, v.W1, v.L));
    if (kSym) shmem += sizeof(double) * 3 * v.RG + sizeof(int) * v.maxT;
    switch (mode) {
        case kResidInit: launch_kernel(k_residual<kResidInit, kSym>, g, b, shmem, s, v, out); break;
        case kResidReplace: launch_kernel(k_residual<kResidReplace, kSym>, g, b, shmem, s, v, out); break;
        case kResidConfirm: launch_kernel(k_residual<kResidConfirm, kSym>, g, b, shmem, s, v, out); break;
        default: launch_kernel(k_residual<kResidFinal, kSym>, g, b, shmem, s, v, out); break;
    }
}

hipError_t launch_residual(const SolverView& v, int mode, double* out, hipStream_t s) {
    if (v.sym)
        launch_residual_t<true>(v, mode, out, s);
    else
        launch_residual_t<false>(v, mode, out, s);
    return hipGetLastError();
}

}  // namespace maspcg
