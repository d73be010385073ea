// MAS preconditioner on the device: coarse matrices, batched domain
// inversion and the apply (Supp. Eq. 4-6; algorithm "Compute MAS
// preconditioner" in Sec. 4.3).
#include <algorithm>

#include "launch.hpp"

namespace maspcg {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

// Inverse entries in the apply.  Full-layout level-0 FP64 inverses (136 MB
// at the 48^3 cube) do not fit the 256 MB MALL next to H, so they are
// streamed with non-temporal loads that leave the caches to H, the vectors
// and the coarse inverses (kStream); the symmetric-packed FP64 set (69 MB),
// the FP32 set of the mixed solve and the coarse levels (16 MB) fit and are
// read through the caches.
template <typename TI, bool kStream = true>
__device__ __forceinline__ double inv_load(const TI* p) {
    if constexpr (sizeof(TI) == 8 && kStream)
        return __builtin_nontemporal_load(p);
    else
        return static_cast<double>(*p);
}

// ------------------------------------------------------------ coarse sums
// A_l = C H C^T by levels (Supp. Eq. 5: A_(l) = C A C^T with unit 3x3
// weights).  Each coarse block owns a list of fine blocks and sums it in a
// fixed order: no atomics, bitwise reproducible.  Nine consecutive threads
// take one coarse block, thread c summing entry c over the list in order,
// four list entries loaded at a time (their indices, then their values), so
// that the list's loads overlap instead of following one another.
constexpr int kSumRound = 4;

__global__ void __launch_bounds__(256) k_coarse_sum_first(int nnzA, const int* __restrict__ ptr,
                                                           const int* __restrict__ src, const double* __restrict__ Hu,
                                                           double* __restrict__ A) {
    const long long gt = static_cast<long long>(blockIdx.x) * 256 + threadIdx.x;
    if (gt >= 9LL * nnzA) return;
    const int t = static_cast<int>(gt / 9), c = static_cast<int>(gt % 9);
    const int qe = ptr[t + 1];
    int q = ptr[t];
    double s = 0.0;
    for (; q + kSumRound <= qe; q += kSumRound) {
        int i[kSumRound];
#pragma unroll
        for (int j = 0; j < kSumRound; ++j) i[j] = src[q + j];
        double a[kSumRound];
#pragma unroll
        for (int j = 0; j < kSumRound; ++j) a[j] = Hu[9LL * i[j] + c];
#pragma unroll
        for (int j = 0; j < kSumRound; ++j) s += a[j];
    }
    for (; q < qe; ++q) s += Hu[9LL * src[q] + c];
    A[static_cast<long long>(c) * nnzA + t] = s;
}

__global__ void __launch_bounds__(256) k_coarse_sum_next(int nnzA, int nnzPrev, const int* __restrict__ ptr,
                                                          const int* __restrict__ src, const double* __restrict__ Ap,
                                                          double* __restrict__ A) {
    const long long gt = static_cast<long long>(blockIdx.x) * 256 + threadIdx.x;
    if (gt >= 9LL * nnzA) return;
    const int t = static_cast<int>(gt / 9), c = static_cast<int>(gt % 9);
    const double* Apc = Ap + static_cast<long long>(c) * nnzPrev;
    const int qe = ptr[t + 1];
    int q = ptr[t];
    double s = 0.0;
    for (; q + kSumRound <= qe; q += kSumRound) {
        int i[kSumRound];
#pragma unroll
        for (int j = 0; j < kSumRound; ++j) i[j] = src[q + j];
        double a[kSumRound];
#pragma unroll
        for (int j = 0; j < kSumRound; ++j) a[j] = Apc[i[j]];
#pragma unroll
        for (int j = 0; j < kSumRound; ++j) s += a[j];
    }
    for (; q < qe; ++q) s += Apc[src[q]];
    A[static_cast<long long>(c) * nnzA + t] = s;
}

// ------------------------------------------------------- domain inversion
// One workgroup of four waves per domain (all levels in one launch).  The
// domain matrix (3N x 3N, padded to 16T with identity rows on empty lanes so
// that the inverse of the occupied part comes out directly) sits in LDS and
// is inverted in place by block Gauss-Jordan over 16x16 tiles:
//   P = inv(A_kk) (register-resident scalar Gauss-Jordan, 16 pivots, wave 0),
//   A_kj <- P A_kj, A_ij <- A_ij - A_ik A_kj, A_ik <- -A_ik P, A_kk <- P,
// with the tile products on v_mfma_f64_16x16x4f64, the tiles of each phase
// dealt round-robin to the four waves.  Pivots are Schur complement
// diagonals of an SPD matrix; a pivot <= 0 flags NOT_SPD.
//
// MFMA f64 16x16x4 lane layout on gfx950: lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; result register v of lane l is D[l / 16 + 4 v][l % 16].

struct DomTable {
    int off[kMaxLv + 1];  // first workgroup of each level
};

__device__ __forceinline__ int level_of(const DomTable& tab, int L, int g) {
    int l = 0;
    while (l + 1 < L && g >= tab.off[l + 1]) ++l;
    return l;
}

constexpr int kInvWaves = 4;
constexpr int kInvThreads = 64 * kInvWaves;

template <int T>
__global__ void __launch_bounds__(kInvThreads) k_invert(BuildView B, const double* __restrict__ Hu, int want32,
                                                        DomTable tab) {
    constexpr int NP = 16 * T;
    constexpr int LD = NP + 1;  // odd stride: a 16-row column read hits 16 distinct bank pairs
    __shared__ double A[NP * LD];
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index, uniform in the wave
    const int l = level_of(tab, B.L, blockIdx.x);
    const int d = blockIdx.x - tab.off[l];
    const int N = B.N, n = 3 * N;

    for (int e = tid; e < NP * LD; e += kInvThreads) A[e] = 0.0;
    __syncthreads();

    // gather the upper in-domain blocks and mirror them
    const int* dptr = B.dom_ptr[l];
    for (int q = dptr[d] + tid; q < dptr[d + 1]; q += kInvThreads) {
        const int k = B.dom_blk[l][q];
        const int ab = B.dom_ab[l][q];
        const int a = ab & 255, b = ab >> 8;
        double v[9];
        if (l == 0) {
#pragma unroll
            for (int c = 0; c < 9; ++c) v[c] = Hu[9LL * k + c];
        } else {
#pragma unroll
            for (int c = 0; c < 9; ++c) v[c] = B.A[l][(long long)c * B.nnzA[l] + k];
        }
        if (a == b) {
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = r; c < 3; ++c) {
                    A[(3 * a + r) * LD + 3 * a + c] = v[3 * r + c];
                    A[(3 * a + c) * LD + 3 * a + r] = v[3 * r + c];
                }
        } else {
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    A[(3 * a + r) * LD + 3 * b + c] = v[3 * r + c];
                    A[(3 * b + c) * LD + 3 * a + r] = v[3 * r + c];
                }
        }
    }
    // occupied lanes of this domain as a bit mask (every wave forms the same)
    bool occ_lane = false;
    if (lane < N) {
        const int u = d * N + lane;
        occ_lane = (l == 0) ? (B.remap[u] >= 0) : (u < B.units[l]);
    }
    const unsigned long long occ = __ballot(occ_lane);
    __syncthreads();
    for (int p = tid; p < NP; p += kInvThreads) {
        const bool live = p < n && ((occ >> (p / 3)) & 1ull);
        if (!live) A[p * LD + p] = 1.0;
    }
    __syncthreads();

    const int c16 = lane & 15, g4 = lane >> 4;
    bool ok = true;
#pragma unroll
    for (int k = 0; k < T; ++k) {
        const int base = 16 * k;
        // ---- P = inv(A_kk) by wave 0: lane holds column c16, rows 4 g4 + v
        if (w == 0) {
            double a[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) a[v] = A[(base + 4 * g4 + v) * LD + base + c16];
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int jg = j >> 2, jv = j & 3;
                const double aj = a[jv];
                const double piv = __shfl(aj, jg * 16 + j);
                const double rowj = __shfl(aj, jg * 16 + c16);
                double colj[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) colj[v] = __shfl(a[v], g4 * 16 + j);
                ok = ok && (piv > 0.0) && finite(piv);
                const double inv = 1.0 / piv;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = 4 * g4 + v;
                    if (i == j)
                        a[v] = (c16 == j) ? inv : a[v] * inv;
                    else
                        a[v] = (c16 == j) ? -colj[v] * inv : a[v] - colj[v] * rowj * inv;
                }
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) A[(base + 4 * g4 + v) * LD + base + c16] = a[v];
        }
        __syncthreads();
        // ---- row panel: A_kj <- P A_kj, tile j (j != k) to wave (its rank) % 4
#pragma unroll
        for (int j = 0; j < T; ++j) {
            if (j == k || (j - (j > k)) % kInvWaves != w) continue;
            v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const double av = A[(base + c16) * LD + base + 4 * kk + g4];
                const double bv = A[(base + 4 * kk + g4) * LD + 16 * j + c16];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) A[(base + g4 + 4 * v) * LD + 16 * j + c16] = acc[v];
        }
        __syncthreads();
        // ---- trailing update: A_ij <- A_ij - A_ik A_kj, tile (i, j) to wave (its rank) % 4
#pragma unroll
        for (int i = 0; i < T; ++i) {
            if (i == k) continue;
#pragma unroll
            for (int j = 0; j < T; ++j) {
                if (j == k || ((i - (i > k)) * (T - 1) + (j - (j > k))) % kInvWaves != w) continue;
                v4d acc;
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[v] = A[(16 * i + g4 + 4 * v) * LD + 16 * j + c16];
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const double av = -A[(16 * i + c16) * LD + base + 4 * kk + g4];
                    const double bv = A[(base + 4 * kk + g4) * LD + 16 * j + c16];
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) A[(16 * i + g4 + 4 * v) * LD + 16 * j + c16] = acc[v];
            }
        }
        __syncthreads();
        // ---- column panel: A_ik <- -A_ik P, tile i (i != k) to wave (its rank) % 4;
        // a tile's wave reads it whole before writing it (one wave, in order)
#pragma unroll
        for (int i = 0; i < T; ++i) {
            if (i == k || (i - (i > k)) % kInvWaves != w) continue;
            v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const double av = -A[(16 * i + c16) * LD + base + 4 * kk + g4];
                const double bv = A[(base + 4 * kk + g4) * LD + base + c16];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) A[(16 * i + g4 + 4 * v) * LD + base + c16] = acc[v];
        }
        __syncthreads();
    }
    if (w == 0 && !ok && lane == 0) atomicOr(B.flag, 1);

    const bool packed = l == 0 && B.packed0;
    if (packed) {
        // FP64: symmetric-packed lower triangle (the mean of the two
        // triangles of the computed inverse), zero on empty lanes
        double* o64 = B.inv64[0] + (long long)d * kPacked;
        for (int j = w; j < kPackedN; j += kInvWaves)  // column j (rows j..47) by wave j % 4
            for (int i = j + lane; i < kPackedN; i += 64) {
                const bool live = ((occ >> (i / 3)) & 1ull) && ((occ >> (j / 3)) & 1ull);
                o64[packed_col(j) + i - j] = live ? 0.5 * (A[i * LD + j] + A[j * LD + i]) : 0.0;
            }
    }
    // column-major n x n, zero rows/columns on empty lanes
    const long long off = (long long)d * n * n;
    double* o64 = packed ? nullptr : B.inv64[l] + off;
    float* o32 = want32 ? B.inv32[l] + off : nullptr;
    if (o64 || o32)
        for (int e = tid; e < n * n; e += kInvThreads) {
            const int col = e / n, row = e - col * n;
            const bool live = ((occ >> (row / 3)) & 1ull) && ((occ >> (col / 3)) & 1ull);
            const double val = live ? A[row * LD + col] : 0.0;
            if (o64) o64[e] = val;
            if (o32) o32[e] = static_cast<float>(val);
        }
}

// ------------------------------------------------------------------ apply
constexpr int kFlagX0 = 1, kFlagMixed = 2, kFlagRrTrue = 4;
constexpr int kRound = 8;  // coarse partials loaded per round by one lane

// Workgroup 0 of the coarse launch takes the convergence decision of the
// iteration: it sums the ||r||^2 partials (and ||b||^2 for the first
// apply) and records rr, the iteration count and, when ||r|| <= tol ||b||,
// the stop for the host and every later kernel.  In mixed precision a stop
// on the recurrence is marked for confirmation on the FP64 residual.
__device__ void convergence_decision(const SolverView& v, int mode, int k, double tol, int flags, double* buf) {
    DevState* st = v.st;
    if (st->done) return;
    const double rr = sum_partials(v.P_rr, v.G, buf);
    if (mode == kApplyInit) {
        const double bb = sum_partials(v.P_bb, v.G, buf);
        const double tol2 = tol * tol * bb;
        const bool bad = !finite(bb) || !finite(rr);
        const bool stop = bad || bb == 0.0 || ((flags & kFlagX0) && rr <= tol2);
        if (threadIdx.x == 0) {
            st->bb = bb;
            st->tol2 = tol2;
            st->rr = rr;
            st->iter = 0;
            if (stop) {
                st->status = bad ? -6 : 0;
                st->done = 1;
            }
        }
    } else {
        const bool bad = !finite(rr);
        const bool conv = rr <= st->tol2;
        if (threadIdx.x == 0) {
            st->rr = rr;
            st->iter = k;
            if (bad || conv) {
                st->status = bad ? -6 : (((flags & kFlagMixed) && !(flags & kFlagRrTrue)) ? kStatusConvergedRecurrence : 0);
                st->done = 1;
            }
        }
    }
}

// Coarse levels l >= 1 (workgroups 1.. of the launch, one per domain, all
// levels at once): r_l for the domain's N units, then y_l = Inv_{l,d} r_l.
// Straight from the residual's restriction (kApplyInit, kApplyIter,
// kApplyPlain): level 1 from r_1, higher levels as sums of the per-group
// partials the restriction left for each unit (a contiguous range per unit;
// for N = 16 sixteen lanes per unit, all units at once, else one wave per
// unit); levels >= 2 keep that r_l in rc_l.  By recurrence (kApplyRec,
// iteration k): alpha_k = rho_{k-1} / sigma_k from the partials, and
// r_l <- r_l - alpha_k (C_l q_k) with C_l q_k gathered in the same way from
// the restriction of q_k the SpMV left (q_1, qpart); the unit's r_l (r_1 or
// rc_l) is updated in place, each unit by the one workgroup of its domain.
template <typename TI, int kN>
__global__ void __launch_bounds__(256) k_apply_coarse(SolverView v, DomTable tab, int mode, int k, double tol,
                                                      int flags) {
    __shared__ double rl[128];
    __shared__ double buf[256];
    if (blockIdx.x == 0) {
        if (mode != kApplyPlain) convergence_decision(v, mode, mode == kApplyRec ? k - 1 : k, tol, flags, buf);
        return;
    }
    const int gb = blockIdx.x - 1;
    int l = 1;
    while (l + 1 < v.L && gb >= tab.off[l + 1]) ++l;
    const int d = gb - tab.off[l];
    const int N = kN > 0 ? kN : v.N, n = 3 * N;
    const int u0 = d * N;
    const int nu = min(N, v.units[l] - u0);
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    const bool rec = mode == kApplyRec;
    const TI* inv;
    if constexpr (sizeof(TI) == 8)
        inv = v.inv64[l];
    else
        inv = v.inv32[l];
    inv += static_cast<long long>(d) * n * n;
    // N = 16: four threads per row, each holding a quarter of the row's
    // inverse entries, loaded before the gather so that both are in flight
    constexpr int kParts = 4;
    constexpr int kCols = kN > 0 ? (3 * kN + kParts - 1) / kParts : 1;
    double pre[kCols];
    const int prow = t % n, ppart = t / n;
    if constexpr (kN > 0) {
        if (t < kParts * n) {
#pragma unroll
            for (int j = 0; j < kCols; ++j) {
                const int kk = ppart * kCols + j;
                pre[j] = kk < n ? inv_load<TI, false>(inv + static_cast<long long>(kk) * n + prow) : 0.0;
            }
        }
    }
    // recurrence: the sigma partials and the unit's previous r_l, issued
    // with the inverse loads (N = 16: lane 0 of each unit's 16-lane segment
    // holds the unit's three components; level 1: thread t < 3 nu holds
    // entry t of the domain's r_1 and q_1)
    PartialLoads sig{};
    double rho = 0.0, prev0 = 0.0, prev1 = 0.0, prev2 = 0.0, q1v = 0.0;
    if (rec) {
        sig = partials_load(v.P_sigma, v.G);
        rho = v.st->rho[(k - 1) & 1];
        if (l == 1) {
            const int e = 3 * u0 + min(t, 3 * nu - 1);
            prev0 = v.r1[e];
            q1v = v.q1[e];
        } else if (kN == 16) {
            const int e = 3 * (u0 + min(t >> 4, nu - 1));
            prev0 = v.rc[l][e];
            prev1 = v.rc[l][e + 1];
            prev2 = v.rc[l][e + 2];
        }
    }
    // the stop flag is read once these loads are in flight; after a stop
    // nothing is written
    const int stop = v.st->done;
    keep_loads_issued();
    if ((mode == kApplyIter || rec) && stop) return;
    double alpha = 0.0;
    if (rec) {
        const double sigma = partials_sum(sig, v.P_sigma, v.G, buf);
        if (!(sigma > 0.0) || !finite(sigma) || !finite(rho)) return;  // the level-0 launch reports it
        alpha = rho / sigma;
    }
    const bool keep = mode != kApplyPlain;  // r_l of levels >= 2 kept for the recurrence
    if (l == 1) {
        if (t < n) {
            double val = 0.0;
            if (t < 3 * nu) {
                if (rec) {
                    val = prev0 - alpha * q1v;
                    v.r1[3 * u0 + t] = val;
                } else {
                    val = v.r1[3 * u0 + t];
                }
            }
            rl[t] = val;
        }
    } else if constexpr (kN == 16) {
        // all 16 units at once: 16 lanes per unit stride over its partials,
        // then fold within the 16-lane segment
        const int* cp = v.cp_ptr[l];
        const double* part = rec ? v.qpart : v.cpart;
        const int a = t >> 4, sub = t & 15;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        if (a < nu) {
            // the lane's partials m0 + sub, + 16, + 32, ... in this order;
            // kRound are loaded per round (at clamped indices, the ones past
            // the range not added) so that their latencies overlap: a unit of
            // the top levels has partials from about a hundred groups, which
            // one round then covers
            const int m0 = cp[u0 + a], m1 = cp[u0 + a + 1];
            for (int m = m0 + sub; m < m1; m += 16 * kRound) {
                double a0[kRound], a1[kRound], a2[kRound];
#pragma unroll
                for (int j = 0; j < kRound; ++j) {
                    const int mj = min(m + 16 * j, m1 - 1);
                    a0[j] = part[3 * mj];
                    a1[j] = part[3 * mj + 1];
                    a2[j] = part[3 * mj + 2];
                }
#pragma unroll
                for (int j = 0; j < kRound; ++j)
                    if (m + 16 * j < m1) {
                        s0 += a0[j];
                        s1 += a1[j];
                        s2 += a2[j];
                    }
            }
        }
        s0 = row16_sum(s0);  // a unit's 16 lanes are one DPP row of the wave
        s1 = row16_sum(s1);
        s2 = row16_sum(s2);
        if (sub == 0) {
            if (rec && a < nu) {
                s0 = prev0 - alpha * s0;
                s1 = prev1 - alpha * s1;
                s2 = prev2 - alpha * s2;
            }
            if (keep && a < nu) {
                double* rc = v.rc[l] + 3 * (u0 + a);
                rc[0] = s0;
                rc[1] = s1;
                rc[2] = s2;
            }
            rl[3 * a] = s0;
            rl[3 * a + 1] = s1;
            rl[3 * a + 2] = s2;
        }
    } else {
        const int* cp = v.cp_ptr[l];
        const double* part = rec ? v.qpart : v.cpart;
        for (int a = w; a < N; a += 4) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
            if (a < nu) {
                const int m0 = cp[u0 + a], m1 = cp[u0 + a + 1];
                for (int m = m0 + lane; m < m1; m += 128) {
                    const int mb = m + 64;  // two independent loads in flight per lane
                    s0 += part[3 * m];
                    s1 += part[3 * m + 1];
                    s2 += part[3 * m + 2];
                    if (mb < m1) {
                        s0 += part[3 * mb];
                        s1 += part[3 * mb + 1];
                        s2 += part[3 * mb + 2];
                    }
                }
            }
            s0 = wave_sum(s0);
            s1 = wave_sum(s1);
            s2 = wave_sum(s2);
            if (lane == 0) {
                if (a < nu) {
                    double* rc = v.rc[l] + 3 * (u0 + a);
                    if (rec) {
                        s0 = rc[0] - alpha * s0;
                        s1 = rc[1] - alpha * s1;
                        s2 = rc[2] - alpha * s2;
                    }
                    if (keep) {
                        rc[0] = s0;
                        rc[1] = s1;
                        rc[2] = s2;
                    }
                }
                rl[3 * a] = s0;
                rl[3 * a + 1] = s1;
                rl[3 * a + 2] = s2;
            }
        }
    }
    __syncthreads();
    if constexpr (kN > 0) {
        __shared__ double quarter[kParts][3 * kN];
        if (t < kParts * n) {
            double a = 0.0;
#pragma unroll
            for (int j = 0; j < kCols; ++j) {
                const int kk = ppart * kCols + j;
                if (kk < n) a += pre[j] * rl[kk];
            }
            quarter[ppart][prow] = a;
        }
        __syncthreads();
        if (t < n) v.y[l][3 * u0 + t] = ((quarter[0][t] + quarter[1][t]) + quarter[2][t]) + quarter[3][t];
    } else if (t < n) {
        double acc = 0.0;
#pragma unroll 8
        for (int kk = 0; kk < n; ++kk) acc += inv_load<TI, false>(inv + static_cast<long long>(kk) * n + t) * rl[kk];
        v.y[l][3 * u0 + t] = acc;
    }
}

constexpr int kPreLevels = 8;  // coarse levels whose corrections are prefetched

// The x/r update of iteration k fused into the level-0 apply (kApplyRec):
// alpha_k = rho_{k-1} / sigma_k from the partials, x += alpha p_k and
// r -= alpha q_k on the thread's DOF (one per thread, slots of the group;
// the vectors are padded to whole groups).  The loads are issued by
// fused_load with the kernel's other early loads; fused_update returns
// false, after flagging NOT_SPD (or NOT_FINITE) from group 0, when
// sigma <= 0 or a value is not finite: every workgroup sees the same sigma
// and returns without writing.  buf: 256 doubles of shared memory.
struct FusedLoads {
    PartialLoads sig;
    double rho, x, p, r, q;
};

__device__ __forceinline__ FusedLoads fused_load(const SolverView& v, int k, long long i) {
    FusedLoads F;
    F.sig = partials_load(v.P_sigma, v.G);
    F.rho = v.st->rho[(k - 1) & 1];
    F.x = v.x[i];
    F.p = v.p[k & 1][i];
    F.r = v.r[i];
    F.q = v.q[i];
    return F;
}

__device__ __forceinline__ bool fused_update(const SolverView& v, int k, int g, long long i, bool live,
                                             const FusedLoads& F, double* buf, double& rv) {
    const double sigma = partials_sum(F.sig, v.P_sigma, v.G, buf);
    if (!(sigma > 0.0) || !finite(sigma) || !finite(F.rho)) {
        if (g == 0 && threadIdx.x == 0) {
            v.st->status = (finite(sigma) && finite(F.rho)) ? -2 : -6;
            v.st->done = 1;
            v.st->iter = k - 1;
        }
        return false;
    }
    const double alpha = F.rho / sigma;
    rv = 0.0;
    if (live) {
        v.x[i] = F.x + alpha * F.p;
        rv = F.r - alpha * F.q;
        v.r[i] = rv;
    }
    return true;
}

// Level 0 over a group of D0 domains, one thread per DOF:
//   z = Inv_{0,d} r_d + sum_{l >= 1} y_l[unit of the slot at level l]
// (prolongation of every coarse level, Supp. Eq. 6) and the partial of
// rho = r^T z; kApplyRec first performs the x/r update of iteration k and
// also leaves the partial of ||r_k||^2.  Returns at once after a stop.
template <typename TI, int kN, int kMode>
__global__ void __launch_bounds__(384) k_apply_level0(SolverView v, int k) {
    constexpr bool kFused = kMode == kApplyRec;
    __shared__ double rs[384];
    __shared__ double red[16];
    __shared__ double pbuf[kFused ? 256 : 1];
    const int N = kN > 0 ? kN : v.N;
    const int n = 3 * N;
    const int g = xcd_group(blockIdx.x, v.G), t = threadIdx.x;
    const int nd = min(v.D0, v.M - g * v.D0);  // domains of this group
    const bool live = t < nd * n;
    const long long base = 3LL * g * v.RG;
    const int slot = g * v.RG + t / 3, c = t % 3;
    // coarse corrections of the slot (prolongation), loaded with r so that
    // their latency ends before the inverse stream starts
    int u[kPreLevels];
#pragma unroll
    for (int j = 0; j < kPreLevels; ++j)
        u[j] = (live && j + 1 < v.L) ? v.anc[static_cast<long long>(j) * v.NS + slot] : -1;
    FusedLoads F{};
    double rv = 0.0;
    if constexpr (kFused)
        F = fused_load(v, k, base + t);
    else
        rv = live ? v.r[base + t] : 0.0;
    // the stop flag is read once these loads are in flight; after a stop
    // nothing is written
    const int stop = v.st->done;
    keep_loads_issued();
    if (kMode != kApplyPlain && stop) return;
    if constexpr (kFused) {
        if (!fused_update(v, k, g, base + t, live, F, pbuf, rv)) return;
    }
    double ycor[kPreLevels];
#pragma unroll
    for (int j = 0; j < kPreLevels; ++j) ycor[j] = u[j] >= 0 ? v.y[j + 1][3 * u[j] + c] : 0.0;
    if (t < 384) rs[t] = rv;
    __syncthreads();
    double zv = 0.0;
    if (live) {
        const int dl = t / n, row = t - dl * n;
        const int d = g * v.D0 + dl;
        const TI* inv;
        if constexpr (sizeof(TI) == 8)
            inv = v.inv64[0];
        else
            inv = v.inv32[0];
        inv += (long long)d * n * n + row;
        const double* rd = rs + dl * n;
        double acc = 0.0;
        if constexpr (kN > 0) {
#pragma unroll
            for (int kk = 0; kk < 3 * kN; ++kk) acc += inv_load(inv + kk * 3 * kN) * rd[kk];
        } else {
#pragma unroll 8
            for (int kk = 0; kk < n; ++kk) acc += inv_load(inv + kk * n) * rd[kk];
        }
#pragma unroll
        for (int j = 0; j < kPreLevels; ++j)
            if (u[j] >= 0) acc += ycor[j];
        if (v.L > kPreLevels + 1) {
            // deeper hierarchies: the remaining levels' unit ids at once, then
            // their corrections at once
            constexpr int kRest = kMaxLv - 1 - kPreLevels;
            int ur[kRest];
#pragma unroll
            for (int j = 0; j < kRest; ++j)
                ur[j] = kPreLevels + 1 + j < v.L ? v.anc[static_cast<long long>(kPreLevels + j) * v.NS + slot] : -1;
            double yr[kRest];
#pragma unroll
            for (int j = 0; j < kRest; ++j) yr[j] = ur[j] >= 0 ? v.y[kPreLevels + 1 + j][3 * ur[j] + c] : 0.0;
#pragma unroll
            for (int j = 0; j < kRest; ++j)
                if (ur[j] >= 0) acc += yr[j];
        }
        zv = acc;
        v.z[base + t] = zv;
    }
    if (kMode == kApplyPlain) return;
    if constexpr (kFused) {
        double prho, prr;
        block_sum2_last(rv * zv, rv * rv, red, prho, prr);
        if (t == 0) {
            v.P_rho[k & 1][g] = prho;
            v.P_rr[g] = prr;
        }
    } else {
        const double part = block_sum_last(rv * zv, red);
        if (t == 0) v.P_rho[k & 1][g] = part;
    }
}

// Level 0 with the symmetric-packed FP64 inverses (domain size 16), over a
// group of D0 domains: the packed inverses of two domains at a time
// (18.8 KB, contiguous) are staged in LDS with coalesced loads, the next
// pair's loads in flight (in registers) while the current pair is
// multiplied.  (With FP32 inverses the full layout streams faster: the
// staging rounds, not the bytes, then bound the kernel.)  Four
// threads per row each take twelve columns: entry (i, kk) of the inverse is
// (kk, i) of the stored lower triangle when kk > i.  The rows' sums go to
// LDS; then, one thread per DOF as in k_apply_level0,
//   z = Inv_{0,d} r_d + sum_{l >= 1} y_l[unit of the slot at level l]
// and the partial of rho = r^T z.  Returns at once after a stop.
constexpr int kPairs = 2;                                // domains staged per round
constexpr int kStageLoads = (kPairs * kPacked + 383) / 384;  // entries per thread and round

template <typename TI, int kMode>
__global__ void __launch_bounds__(384) k_apply_level0_packed(SolverView v, int k) {
    constexpr bool kFused = kMode == kApplyRec;
    __shared__ double rs[384];
    __shared__ double zs[384];
    __shared__ TI stage[kPairs * kPacked];
    __shared__ double red[16];
    const int g = xcd_group(blockIdx.x, v.G), t = threadIdx.x;
    const int nd = min(v.D0, v.M - g * v.D0);  // domains of this group
    const bool live = t < nd * 48;
    const long long base = 3LL * g * v.RG;
    const int slot = g * v.RG + t / 3, c = t % 3;
    const TI* inv;
    if constexpr (sizeof(TI) == 8)
        inv = v.inv64[0];
    else
        inv = v.inv32[0];
    inv += static_cast<long long>(g) * v.D0 * kPacked;
    const int rounds = (nd + kPairs - 1) / kPairs;
    // the first pair, then the corrections of the slot (prolongation) and r
    TI nxt[kStageLoads];
    auto fetch = [&](int p) {
        const int cnt = min(kPairs, nd - kPairs * p) * kPacked;
        const TI* src = inv + static_cast<long long>(kPairs * p) * kPacked;
#pragma unroll
        for (int j = 0; j < kStageLoads; ++j) {
            const int e = t + 384 * j;
            nxt[j] = e < cnt ? inv_load<TI, false>(src + e) : TI(0);
        }
    };
    fetch(0);
    FusedLoads F{};
    double rv = 0.0;
    if constexpr (kFused)
        F = fused_load(v, k, base + t);
    else
        rv = live ? v.r[base + t] : 0.0;
    // the stop flag is read once these loads are in flight; after a stop
    // nothing is written
    const int stop = v.st->done;
    keep_loads_issued();
    if (kMode != kApplyPlain && stop) return;
    if constexpr (kFused) {
        // zs is first written after the first round's barrier
        if (!fused_update(v, k, g, base + t, live, F, zs, rv)) return;
    }
    if (t < 384) rs[t] = rv;
    const int row = t >> 2, q = t & 3;  // 96 rows of a pair, four quarters each
    const int dl = row / 48, i = row - 48 * dl;
    for (int p = 0; p < rounds; ++p) {
        const int cnt = min(kPairs, nd - kPairs * p) * kPacked;
#pragma unroll
        for (int j = 0; j < kStageLoads; ++j) {
            const int e = t + 384 * j;
            if (e < cnt) stage[e] = nxt[j];
        }
        __syncthreads();  // the pair (and, the first time, r) are visible
        if (p + 1 < rounds) fetch(p + 1);
        const int d = kPairs * p + dl;
        double s = 0.0;
        if (d < nd) {
            const TI* Ad = stage + dl * kPacked;
            const double* rd = rs + 48 * d;
#pragma unroll
            for (int m = 0; m < 12; ++m) {
                const int kk = 12 * q + m;
                const int idx = kk <= i ? packed_col(kk) + i - kk : packed_col(i) + kk - i;
                s += static_cast<double>(Ad[idx]) * rd[kk];
            }
        }
        // the row's four quarters, added as (q0 + q1) + (q2 + q3)
        s = dpp_add<0xb1>(s);  // quad_perm [1, 0, 3, 2]
        s = dpp_add<0x4e>(s);  // quad_perm [2, 3, 0, 1]
        if (q == 0 && d < nd) zs[48 * d + i] = s;
        __syncthreads();  // stage free for the next pair
    }
    // the corrections of the slot (prolongation) at every coarse level,
    // loaded after the rounds (registers held through them would cost a
    // workgroup per CU): all unit ids at once, then all corrections at once
    int u[kMaxLv - 1];
#pragma unroll
    for (int j = 0; j < kMaxLv - 1; ++j)
        u[j] = (live && j + 1 < v.L) ? v.anc[static_cast<long long>(j) * v.NS + slot] : -1;
    double ycor[kMaxLv - 1];
#pragma unroll
    for (int j = 0; j < kMaxLv - 1; ++j) ycor[j] = u[j] >= 0 ? v.y[j + 1][3 * u[j] + c] : 0.0;
    double zv = 0.0;
    if (live) {
        double acc = zs[t];
#pragma unroll
        for (int j = 0; j < kMaxLv - 1; ++j)
            if (u[j] >= 0) acc += ycor[j];
        zv = acc;
        v.z[base + t] = zv;
    }
    if (kMode == kApplyPlain) return;
    if constexpr (kFused) {
        double prho, prr;
        block_sum2_last(rv * zv, rv * rv, red, prho, prr);
        if (t == 0) {
            v.P_rho[k & 1][g] = prho;
            v.P_rr[g] = prr;
        }
    } else {
        const double part = block_sum_last(rv * zv, red);
        if (t == 0) v.P_rho[k & 1][g] = part;
    }
}

DomTable make_table(const int* ndom, int first, int L) {
    DomTable t{};
    int acc = 0;
    for (int l = 0; l <= kMaxLv; ++l) t.off[l] = 0;
    for (int l = first; l < L; ++l) {
        t.off[l] = acc;
        acc += ndom[l];
    }
    for (int l = L; l <= kMaxLv; ++l) t.off[l] = acc;
    return t;
}

template <int T>
void launch_invert_t(const BuildView& b, const double* Hu, bool want32, int total, const DomTable& tab, hipStream_t s) {
    launch_kernel(k_invert<T>, dim3(total), dim3(kInvThreads), 0, s, b, Hu, want32 ? 1 : 0, tab);
}

}  // namespace

hipError_t launch_coarse_sums(const BuildView& b, const double* Hu, hipStream_t s) {
    for (int l = 1; l < b.L; ++l) {
        const int g = ceil_div(9LL * b.nnzA[l], 256);  // nine threads per coarse block
        if (g == 0) continue;
        if (l == 1)
            launch_kernel(k_coarse_sum_first, dim3(g), dim3(256), 0, s, b.nnzA[1], b.red_ptr[1], b.red_src[1], Hu,
                               b.A[1]);
        else
            launch_kernel(k_coarse_sum_next, dim3(g), dim3(256), 0, s, b.nnzA[l], b.nnzA[l - 1], b.red_ptr[l],
                               b.red_src[l], b.A[l - 1], b.A[l]);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_invert(const BuildView& b, const double* Hu, bool want32, hipStream_t s) {
    const DomTable tab = make_table(b.ndom, 0, b.L);
    const int total = tab.off[kMaxLv];
    const int T = ceil_div(3 * b.N, 16);
    switch (T) {
        case 1: launch_invert_t<1>(b, Hu, want32, total, tab, s); break;
        case 2: launch_invert_t<2>(b, Hu, want32, total, tab, s); break;
        case 3: launch_invert_t<3>(b, Hu, want32, total, tab, s); break;
        case 4: launch_invert_t<4>(b, Hu, want32, total, tab, s); break;
        case 5: launch_invert_t<5>(b, Hu, want32, total, tab, s); break;
        case 6: launch_invert_t<6>(b, Hu, want32, total, tab, s); break;
        case 7: launch_invert_t<7>(b, Hu, want32, total, tab, s); break;
        case 8: launch_invert_t<8>(b, Hu, want32, total, tab, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_apply_coarse(const SolverView& v, bool f32, int mode, int k, double tol, bool x0_given, bool mixed,
                               bool rr_true, hipStream_t s, bool decision_only) {
    const DomTable tab = make_table(v.ndom, 1, v.L);
    const int total = decision_only ? 1 : 1 + tab.off[kMaxLv];  // workgroup 0 decides convergence
    const int flags = (x0_given ? kFlagX0 : 0) | (mixed ? kFlagMixed : 0) | (rr_true ? kFlagRrTrue : 0);
    if (v.N == 16) {
        if (f32) launch_kernel((k_apply_coarse<float, 16>), dim3(total), dim3(256), 0, s, v, tab, mode, k, tol, flags);
        else launch_kernel((k_apply_coarse<double, 16>), dim3(total), dim3(256), 0, s, v, tab, mode, k, tol, flags);
    } else {
        if (f32) launch_kernel((k_apply_coarse<float, 0>), dim3(total), dim3(256), 0, s, v, tab, mode, k, tol, flags);
        else launch_kernel((k_apply_coarse<double, 0>), dim3(total), dim3(256), 0, s, v, tab, mode, k, tol, flags);
    }
    return hipGetLastError();
}

template <typename TI, int kN>
void launch_level0_t(const SolverView& v, int mode, int k, hipStream_t s) {
    dim3 g(v.G), b(round_waves(3 * v.RG));
    if (kN == 16 && v.packed0 && sizeof(TI) == 8) {
        if (mode == kApplyPlain)
            launch_kernel((k_apply_level0_packed<TI, kApplyPlain>), g, b, 0, s, v, k);
        else if (mode == kApplyInit)
            launch_kernel((k_apply_level0_packed<TI, kApplyInit>), g, b, 0, s, v, k);
        else if (mode == kApplyIter)
            launch_kernel((k_apply_level0_packed<TI, kApplyIter>), g, b, 0, s, v, k);
        else
            launch_kernel((k_apply_level0_packed<TI, kApplyRec>), g, b, 0, s, v, k);
        return;
    }
    if (mode == kApplyPlain)
        launch_kernel((k_apply_level0<TI, kN, kApplyPlain>), g, b, 0, s, v, k);
    else if (mode == kApplyInit)
        launch_kernel((k_apply_level0<TI, kN, kApplyInit>), g, b, 0, s, v, k);
    else if (mode == kApplyIter)
        launch_kernel((k_apply_level0<TI, kN, kApplyIter>), g, b, 0, s, v, k);
    else
        launch_kernel((k_apply_level0<TI, kN, kApplyRec>), g, b, 0, s, v, k);
}

hipError_t launch_apply_level0(const SolverView& v, bool f32, int mode, int k, hipStream_t s) {
    if (v.N == 16) {
        if (f32) launch_level0_t<float, 16>(v, mode, k, s);
        else launch_level0_t<double, 16>(v, mode, k, s);
    } else {
        if (f32) launch_level0_t<float, 0>(v, mode, k, s);
        else launch_level0_t<double, 0>(v, mode, k, s);
    }
    return hipGetLastError();
}

}  // namespace maspcg
