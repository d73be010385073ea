// C ABI of libmaspcg (declared in include/mas_pcg.h): handle, workspace
// layout and the host-side driver of the PCG iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/mas_pcg.h"
#include "abd.hpp"
#include "launch.hpp"
#include "morton.hpp"
#include "planner.hpp"
#include "replan.hpp"
#include "restrict.hpp"

using namespace maspcg;

namespace {

constexpr size_t kAlign = 256;

struct Layout {
    size_t total = 0;
    size_t remap, map, perm_src, perm_full, rp0, ci0, lead1, anc, g_u1, srp, sci, srow, tptr, tidx;
    size_t red_ptr[kMaxLv], red_src[kMaxLv], dom_ptr[kMaxLv], dom_blk[kMaxLv], dom_ab[kMaxLv];
    size_t ganc, gpos, gmask, cp_ptr[kMaxLv], lmask, gorder, gu1_slot, gu1_mask, gw_pos, gw_li, gw_mask;
    size_t H64, H32, A[kMaxLv], inv64[kMaxLv], inv32[kMaxLv];
    size_t b, x, r, z, p0, p1, q, r1, q1, y[kMaxLv], rc[kMaxLv], cpart, qpart, P_sigma, P_rr, P_bb, P_rho0, P_rho1, st, flag;
    size_t inverse_bytes = 0;

    size_t take(size_t bytes) {
        const size_t o = (total + kAlign - 1) / kAlign * kAlign;
        total = o + std::max<size_t>(bytes, 1);
        return o;
    }
};

enum { kEvBuild0 = 0, kEvBuild1, kEvBuild2, kEvSolve0, kEvSolve1, kEvSolve2, kEvPoll0, kEvPoll1, kEvCount };

// Kernel slots of the optional per-launch timing (mas_set_kernel_timing).
enum { kKSpmv = 0, kKUpdate, kKCoarse, kKLevel0, kKLevel0Upd, kKResidual, kKPermute, kKRestrict, kKSlots };

// Per-launch timing entries: the kernel slot and a tag that orders the
// launch against the convergence decisions: 2k for the launches of
// iteration k up to the decision on r_k, 2k + 1 after it, -1 outside the
// iteration.  Launches tagged above 2K, K the iteration the solve stopped
// at, were queued past the stop and returned at once; they are left out.
struct TimedLaunch {
    int slot, tag;
};

struct KernelTimer {
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<TimedLaunch> pending;  // one per started pair
    double total_ms[kKSlots] = {0};
    int launches[kKSlots] = {0};
};

// Array sizes of a plan that the host does not hold when the plan was
// derived on the device (mas_replan); a host analysis takes them from its
// vectors.
struct Shape {
    size_t nsb = 0;               // stored blocks of the FP64 SpMV copy
    size_t n_tidx = 0;            // transposed entries of the symmetric storage
    size_t nnzA[kMaxLv] = {};     // blocks of A_l (level 0: nnzb)
    size_t n_domblk[kMaxLv] = {}; // inversion gather entries of each level
};

Shape shape_of(const Plan& P) {
    Shape S;
    S.nsb = P.sym ? P.sci.size() : static_cast<size_t>(P.nnzb);
    S.n_tidx = P.tidx.size();
    for (int l = 0; l < P.L; ++l) {
        S.nnzA[l] = l == 0 ? static_cast<size_t>(P.nnzb) : P.ciA[l].size();
        S.n_domblk[l] = P.dom_blk[l].size();
    }
    return S;
}

// A plan derived on the device: its arrays stay in the replan workspace
// until mas_build places them in the solver workspace.
struct DevicePlan {
    bool active = false;
    ReplanLayout R{};
    PlacedShape ps{};
};

}  // namespace

struct mas_handle {
    mas_options opts{};
    bool analyzed = false;
    Plan plan;
    Shape shape;
    DevicePlan dev;
    Layout lay;
    std::vector<std::vector<int>> translated;  // level-1 reduction sources and level-0 domain blocks in caller order
    std::vector<int> gtab_i;                   // restriction tables of levels >= 2 as uploaded ([G][L-2][W1]):
    std::vector<uint64_t> gtab_m;              // ancestors then writer positions; writer masks
    char* ws = nullptr;
    size_t ws_size = 0;
    char* uploaded_to = nullptr;
    bool built = false;
    bool fuse_ok = false;  // the SpMV kernels can stage the restriction of q (three launches per iteration)
    DevState* st_host = nullptr;  // pinned: [0] last blocking read, [1..2] per-batch copies
    int* flag_host = nullptr;     // pinned
    hipEvent_t ev[kEvCount]{};
    bool events = false;
    double timings[4] = {0, 0, 0, 0};
    KernelTimer kt;
};

namespace {

#define HIP_TRY(expr)                                \
    do {                                             \
        if ((expr) != hipSuccess) return MAS_HIP_ERROR; \
    } while (0)

// Runs one launch; with kernel timing on, hands it a pair of HIP events that
// the runtime stamps with that dispatch's own start and end (resolved at the
// next synchronisation).
template <typename F>
hipError_t timed(mas_handle* h, int slot, hipStream_t s, F&& launch, int tag = -1) {
    (void)s;
    KernelTimer& t = h->kt;
    if (!t.on) return launch();
    if (t.used + 2 > t.pool.size()) {
        for (int k = 0; k < 64; ++k) {
            hipEvent_t e;
            hipError_t err = hipEventCreate(&e);
            if (err != hipSuccess) return err;
            t.pool.push_back(e);
        }
    }
    DispatchEvents& de = dispatch_events();
    de = DispatchEvents{t.pool[t.used], t.pool[t.used + 1]};
    const hipError_t err = launch();
    const bool launched = de.start == nullptr;  // a launcher with nothing to do leaves them
    de = DispatchEvents{};
    if (err != hipSuccess) return err;
    if (launched) {
        t.used += 2;
        t.pending.push_back(TimedLaunch{slot, tag});
    }
    return hipSuccess;
}

// Called after the stream has been synchronised; last_iter: the iteration
// count of the device state just read.
void collect_timing(mas_handle* h, int last_iter) {
    KernelTimer& t = h->kt;
    for (size_t k = 0; k < t.pending.size(); ++k) {
        const TimedLaunch& e = t.pending[k];
        if (e.tag > 2 * last_iter) continue;  // queued past the stop: returned at once
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, t.pool[2 * k], t.pool[2 * k + 1]) == hipSuccess) {
            t.total_ms[e.slot] += ms;
            t.launches[e.slot] += 1;
        }
    }
    t.pending.clear();
    t.used = 0;
}

template <typename T>
T* at(const mas_handle* h, size_t off) {
    return reinterpret_cast<T*>(h->ws + off);
}

void make_layout(mas_handle* h) {
    const Plan& P = h->plan;
    Layout& Y = h->lay;
    Y = Layout();
    const bool mixed = h->opts.precision == MAS_PRECISION_MIXED;
    const size_t I = sizeof(int), Dd = sizeof(double), F = sizeof(float);
    const int n = 3 * P.N;
    Y.remap = Y.take(I * P.NS);
    Y.map = Y.take(I * P.V);
    const Shape& Z = h->shape;
    const size_t nsb = Z.nsb;
    Y.perm_src = Y.take(I * nsb);
    // the FP32 copy of the mixed solve keeps the full storage (its SpMV is
    // faster there), with its own permutation when the FP64 copy is symmetric
    Y.perm_full = (mixed && P.sym) ? Y.take(I * P.nnzb) : Y.perm_src;
    Y.rp0 = Y.take(I * (P.NS + 1));
    Y.ci0 = Y.take(I * P.nnzb);
    Y.lead1 = Y.take(I * P.NS);
    Y.lmask = Y.take(sizeof(uint64_t) * P.NS);
    Y.anc = Y.take(I * static_cast<size_t>(std::max(P.L - 1, 0)) * P.NS);
    Y.g_u1 = Y.take(I * (static_cast<size_t>(P.G) + 1));
    const size_t gw1 = static_cast<size_t>(P.G) * P.W1, ggw = static_cast<size_t>(P.G) * P.GW;
    Y.gu1_slot = Y.take(I * gw1);
    Y.gu1_mask = Y.take(sizeof(uint64_t) * gw1);
    Y.gw_pos = Y.take(I * ggw);
    Y.gw_li = Y.take(I * ggw);
    Y.gw_mask = Y.take(sizeof(uint64_t) * ggw);
    Y.gorder = Y.take(I * P.gorder.size());
    const size_t gtab = P.L > 2 ? static_cast<size_t>(P.G) * (P.L - 2) * P.W1 : 0;  // [G][L-2][W1]
    Y.ganc = Y.take(I * gtab);
    Y.gpos = Y.take(I * gtab);
    Y.gmask = Y.take(sizeof(uint64_t) * gtab);
    if (P.sym) {
        Y.srp = Y.take(I * (static_cast<size_t>(P.NS) + 1));
        Y.sci = Y.take(I * nsb);
        Y.srow = Y.take(nsb);
        Y.tptr = Y.take(I * (static_cast<size_t>(P.NS) + 1));
        Y.tidx = Y.take(I * Z.n_tidx);
    }
    for (int l = 0; l < P.L; ++l) {
        if (l >= 1) {
            Y.red_ptr[l] = Y.take(I * (Z.nnzA[l] + 1));
            Y.red_src[l] = Y.take(I * Z.nnzA[l - 1]);
        }
        Y.dom_ptr[l] = Y.take(I * (static_cast<size_t>(P.ndom[l]) + 1));
        Y.dom_blk[l] = Y.take(I * Z.n_domblk[l]);
        Y.dom_ab[l] = Y.take(I * Z.n_domblk[l]);
        if (l >= 2) Y.cp_ptr[l] = Y.take(I * (static_cast<size_t>(P.units[l]) + 1));
    }
    Y.H64 = Y.take(Dd * 9 * nsb);
    Y.H32 = mixed ? Y.take(F * 9 * static_cast<size_t>(P.nnzb)) : 0;
    for (int l = 1; l < P.L; ++l) Y.A[l] = Y.take(Dd * 9 * Z.nnzA[l]);
    for (int l = 0; l < P.L; ++l) {
        const size_t cnt = static_cast<size_t>(P.ndom[l]) * n * n;
        const size_t cnt64 = (l == 0 && P.N == 16) ? static_cast<size_t>(P.ndom[l]) * kPacked : cnt;
        Y.inv64[l] = Y.take(Dd * cnt64);
        Y.inverse_bytes += mixed ? F * cnt : Dd * cnt64;
        if (mixed) Y.inv32[l] = Y.take(F * cnt);
    }
    // slot vectors padded to whole groups so group kernels never branch on the tail
    const size_t vec = Dd * 3 * static_cast<size_t>(P.G) * P.RG;
    Y.b = Y.take(vec);
    Y.x = Y.take(vec);
    Y.r = Y.take(vec);
    Y.z = Y.take(vec);
    Y.p0 = Y.take(vec);
    Y.p1 = Y.take(vec);
    Y.q = Y.take(vec);
    Y.r1 = Y.take(Dd * 3 * (P.L > 1 ? P.units[1] : 1));
    Y.q1 = Y.take(Dd * 3 * (P.L > 1 ? P.units[1] : 1));
    for (int l = 1; l < P.L; ++l) Y.y[l] = Y.take(Dd * 3 * static_cast<size_t>(P.ndom[l]) * P.N);
    for (int l = 2; l < P.L; ++l) Y.rc[l] = Y.take(Dd * 3 * static_cast<size_t>(P.ndom[l]) * P.N);
    Y.cpart = Y.take(Dd * 3 * std::max(P.n_cpart, 1));
    Y.qpart = Y.take(Dd * 3 * std::max(P.n_cpart, 1));
    Y.P_sigma = Y.take(Dd * P.G);
    Y.P_rr = Y.take(Dd * P.G);
    Y.P_bb = Y.take(Dd * P.G);
    Y.P_rho0 = Y.take(Dd * P.G);
    Y.P_rho1 = Y.take(Dd * P.G);
    Y.st = Y.take(sizeof(DevState));
    Y.flag = Y.take(I);
}

SolverView view(const mas_handle* h) {
    const Plan& P = h->plan;
    const Layout& Y = h->lay;
    SolverView v{};
    v.V = P.V;
    v.N = P.N;
    v.packed0 = P.N == 16 ? 1 : 0;
    v.M = P.M;
    v.NS = P.NS;
    v.L = P.L;
    v.nnzb = P.nnzb;
    v.D0 = P.D0;
    v.RG = P.RG;
    v.G = P.G;
    v.sym = P.sym ? 1 : 0;
    v.nsb = static_cast<int>(h->shape.nsb);
    v.maxT = P.maxT;
    if (P.sym) {
        v.srp = at<int>(h, Y.srp);
        v.sci = at<int>(h, Y.sci);
        v.srow = at<uint8_t>(h, Y.srow);
        v.tptr = at<int>(h, Y.tptr);
        v.tidx = at<int>(h, Y.tidx);
    }
    v.W1 = P.W1;
    for (int l = 0; l < P.L; ++l) {
        v.units[l] = P.units[l];
        v.ndom[l] = P.ndom[l];
        v.inv64[l] = at<double>(h, Y.inv64[l]);
        v.inv32[l] = h->opts.precision == MAS_PRECISION_MIXED ? at<float>(h, Y.inv32[l]) : nullptr;
        if (l >= 2) v.cp_ptr[l] = at<int>(h, Y.cp_ptr[l]);
        if (l >= 1) v.y[l] = at<double>(h, Y.y[l]);
        if (l >= 2) v.rc[l] = at<double>(h, Y.rc[l]);
    }
    v.g_u1 = at<int>(h, Y.g_u1);
    v.gu1_slot = at<int>(h, Y.gu1_slot);
    v.gu1_mask = at<uint64_t>(h, Y.gu1_mask);
    v.GW = P.GW;
    v.rfast = restrict_fast_ok(P.W1, P.GW, spmv_threads()) ? 1 : 0;
    v.gw_pos = at<int>(h, Y.gw_pos);
    v.gw_li = at<int>(h, Y.gw_li);
    v.gw_mask = at<uint64_t>(h, Y.gw_mask);
    v.gorder = P.gorder.empty() ? nullptr : at<int>(h, Y.gorder);
    v.ganc = at<int>(h, Y.ganc);
    v.gpos = at<int>(h, Y.gpos);
    v.gmask = at<uint64_t>(h, Y.gmask);
    v.cpart = at<double>(h, Y.cpart);
    v.qpart = at<double>(h, Y.qpart);
    v.P_sigma = at<double>(h, Y.P_sigma);
    v.P_rr = at<double>(h, Y.P_rr);
    v.P_bb = at<double>(h, Y.P_bb);
    v.P_rho[0] = at<double>(h, Y.P_rho0);
    v.P_rho[1] = at<double>(h, Y.P_rho1);
    v.remap = at<int>(h, Y.remap);
    v.map = at<int>(h, Y.map);
    v.perm_src = at<int>(h, Y.perm_src);
    v.perm_full = at<int>(h, Y.perm_full);
    v.rp0 = at<int>(h, Y.rp0);
    v.ci0 = at<int>(h, Y.ci0);
    v.lead1 = at<int>(h, Y.lead1);
    v.lmask = at<uint64_t>(h, Y.lmask);
    v.anc = at<int>(h, Y.anc);
    v.H64 = at<double>(h, Y.H64);
    v.H32 = h->opts.precision == MAS_PRECISION_MIXED ? at<float>(h, Y.H32) : nullptr;
    v.b = at<double>(h, Y.b);
    v.x = at<double>(h, Y.x);
    v.r = at<double>(h, Y.r);
    v.z = at<double>(h, Y.z);
    v.p[0] = at<double>(h, Y.p0);
    v.p[1] = at<double>(h, Y.p1);
    v.q = at<double>(h, Y.q);
    v.r1 = at<double>(h, Y.r1);
    v.q1 = at<double>(h, Y.q1);
    v.st = at<DevState>(h, Y.st);
    v.flag = at<int>(h, Y.flag);
    return v;
}

BuildView build_view(const mas_handle* h) {
    const Plan& P = h->plan;
    const Layout& Y = h->lay;
    BuildView b{};
    b.L = P.L;
    b.N = P.N;
    b.packed0 = P.N == 16 ? 1 : 0;
    b.nnzb = P.nnzb;
    for (int l = 0; l < P.L; ++l) {
        b.units[l] = P.units[l];
        b.ndom[l] = P.ndom[l];
        b.nnzA[l] = static_cast<int>(h->shape.nnzA[l]);
        if (l >= 1) {
            b.red_ptr[l] = at<int>(h, Y.red_ptr[l]);
            b.red_src[l] = at<int>(h, Y.red_src[l]);
            b.A[l] = at<double>(h, Y.A[l]);
        }
        b.dom_ptr[l] = at<int>(h, Y.dom_ptr[l]);
        b.dom_blk[l] = at<int>(h, Y.dom_blk[l]);
        b.dom_ab[l] = at<int>(h, Y.dom_ab[l]);
        b.inv64[l] = at<double>(h, Y.inv64[l]);
        b.inv32[l] = h->opts.precision == MAS_PRECISION_MIXED ? at<float>(h, Y.inv32[l]) : nullptr;
    }
    b.remap = at<int>(h, Y.remap);
    b.flag = at<int>(h, Y.flag);
    return b;
}

int upload_plan(mas_handle* h, hipStream_t s) {
    const Plan& P = h->plan;
    const Layout& Y = h->lay;
    auto put = [&](size_t off, const std::vector<int>& v) -> hipError_t {
        if (v.empty()) return hipSuccess;
        return hipMemcpyAsync(h->ws + off, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice, s);
    };
    HIP_TRY(put(Y.remap, P.remap));
    HIP_TRY(put(Y.map, P.map));
    HIP_TRY(put(Y.perm_src, P.sym ? P.sperm : P.perm_src));
    if (Y.perm_full != Y.perm_src) HIP_TRY(put(Y.perm_full, P.perm_src));
    if (P.sym) {
        HIP_TRY(put(Y.srp, P.srp));
        HIP_TRY(put(Y.sci, P.sci));
        HIP_TRY(hipMemcpyAsync(h->ws + Y.srow, P.srow.data(), P.srow.size(), hipMemcpyHostToDevice, s));
        HIP_TRY(put(Y.tptr, P.tptr));
        HIP_TRY(put(Y.tidx, P.tidx));
    }
    HIP_TRY(put(Y.rp0, P.rp0));
    HIP_TRY(put(Y.ci0, P.ci0));
    HIP_TRY(put(Y.lead1, P.lead1));
    HIP_TRY(hipMemcpyAsync(h->ws + Y.lmask, P.lmask.data(), sizeof(uint64_t) * P.lmask.size(), hipMemcpyHostToDevice,
                           s));
    HIP_TRY(put(Y.anc, P.anc));
    HIP_TRY(put(Y.g_u1, P.g_u1));
    HIP_TRY(put(Y.gu1_slot, P.gu1_slot));
    HIP_TRY(hipMemcpyAsync(h->ws + Y.gu1_mask, P.gu1_mask.data(), sizeof(uint64_t) * P.gu1_mask.size(),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(put(Y.gw_pos, P.gw_pos));
    HIP_TRY(put(Y.gw_li, P.gw_li));
    HIP_TRY(hipMemcpyAsync(h->ws + Y.gw_mask, P.gw_mask.data(), sizeof(uint64_t) * P.gw_mask.size(),
                           hipMemcpyHostToDevice, s));
    if (!P.gorder.empty()) HIP_TRY(put(Y.gorder, P.gorder));
    for (int l = 0; l < P.L; ++l) {
        if (l >= 1) {
            HIP_TRY(put(Y.red_ptr[l], P.red_ptr[l]));
            HIP_TRY(put(Y.red_src[l], l == 1 ? h->translated[0] : P.red_src[l]));
        }
        HIP_TRY(put(Y.dom_ptr[l], P.dom_ptr[l]));
        HIP_TRY(put(Y.dom_blk[l], l == 0 ? h->translated[1] : P.dom_blk[l]));
        HIP_TRY(put(Y.dom_ab[l], P.dom_ab[l]));
        if (l >= 2) HIP_TRY(put(Y.cp_ptr[l], P.cp_ptr[l]));
    }
    if (P.L > 2) {
        // the per-level [G][W1] tables interleaved to [G][L-2][W1]: one
        // contiguous row per group
        const int W = P.W1, nl = P.L - 2;
        const size_t gtab = static_cast<size_t>(P.G) * nl * W;
        h->gtab_i.assign(2 * gtab, -1);
        h->gtab_m.assign(gtab, 0);
        for (int g = 0; g < P.G; ++g)
            for (int l = 2; l < P.L; ++l)
                for (int i = 0; i < W; ++i) {
                    const size_t src = static_cast<size_t>(g) * W + i;
                    const size_t dst = (static_cast<size_t>(g) * nl + (l - 2)) * W + i;
                    h->gtab_i[dst] = P.ganc[l][src];
                    h->gtab_i[gtab + dst] = P.gpos[l][src];
                    h->gtab_m[dst] = P.gmask[l][src];
                }
        HIP_TRY(hipMemcpyAsync(h->ws + Y.ganc, h->gtab_i.data(), sizeof(int) * gtab, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(h->ws + Y.gpos, h->gtab_i.data() + gtab, sizeof(int) * gtab, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(h->ws + Y.gmask, h->gtab_m.data(), sizeof(uint64_t) * gtab, hipMemcpyHostToDevice, s));
    }
    HIP_TRY(hipStreamSynchronize(s));  // the host vectors are pageable
    return MAS_OK;
}

// A device-derived plan (mas_replan) into the solver workspace: the
// partition's maps and the SpMV group order from the host, every other
// array written on the device from the replan workspace.
int place_device_plan(mas_handle* h, hipStream_t s) {
    const Plan& P = h->plan;
    const Layout& Y = h->lay;
    auto put = [&](size_t off, const std::vector<int>& v) -> hipError_t {
        if (v.empty()) return hipSuccess;
        return hipMemcpyAsync(h->ws + off, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice, s);
    };
    HIP_TRY(put(Y.remap, P.remap));
    HIP_TRY(put(Y.map, P.map));
    if (!P.gorder.empty()) HIP_TRY(put(Y.gorder, P.gorder));
    PlanDest D{};
    D.perm_src = at<int>(h, Y.perm_src);
    D.perm_full = at<int>(h, Y.perm_full);
    D.rp0 = at<int>(h, Y.rp0);
    D.ci0 = at<int>(h, Y.ci0);
    D.lead1 = at<int>(h, Y.lead1);
    D.lmask = at<uint64_t>(h, Y.lmask);
    D.anc = at<int>(h, Y.anc);
    D.g_u1 = at<int>(h, Y.g_u1);
    D.gu1_slot = at<int>(h, Y.gu1_slot);
    D.gu1_mask = at<uint64_t>(h, Y.gu1_mask);
    D.gw_pos = at<int>(h, Y.gw_pos);
    D.gw_li = at<int>(h, Y.gw_li);
    D.gw_mask = at<uint64_t>(h, Y.gw_mask);
    D.ganc = at<int>(h, Y.ganc);
    D.gpos = at<int>(h, Y.gpos);
    D.gmask = at<uint64_t>(h, Y.gmask);
    if (P.sym) {
        D.srp = at<int>(h, Y.srp);
        D.sci = at<int>(h, Y.sci);
        D.srow = at<uint8_t>(h, Y.srow);
        D.tptr = at<int>(h, Y.tptr);
        D.tidx = at<int>(h, Y.tidx);
    }
    for (int l = 0; l < P.L; ++l) {
        if (l >= 1) {
            D.red_ptr[l] = at<int>(h, Y.red_ptr[l]);
            D.red_src[l] = at<int>(h, Y.red_src[l]);
        }
        D.dom_ptr[l] = at<int>(h, Y.dom_ptr[l]);
        D.dom_blk[l] = at<int>(h, Y.dom_blk[l]);
        D.dom_ab[l] = at<int>(h, Y.dom_ab[l]);
        if (l >= 2) D.cp_ptr[l] = at<int>(h, Y.cp_ptr[l]);
    }
    HIP_TRY(replan_place(h->dev.R, h->dev.ps, D, s));
    HIP_TRY(hipStreamSynchronize(s));  // the host vectors are pageable
    return MAS_OK;
}

bool bcsr_ok(const mas_handle* h, const mas_bcsr* H) {
    return H && H->row_ptr && H->col_idx && H->val && H->n_rows == h->plan.V && H->nnzb == h->plan.nnzb &&
           H->dtype == MAS_F64;
}

int finish_status(const DevState& st) {
    if (st.status == -2) return MAS_NOT_SPD;
    if (st.status == -6) return MAS_NOT_FINITE;
    if (st.done && st.status == 0) return MAS_OK;
    return MAS_NOT_CONVERGED;
}

// The MAS apply of iteration k after the residual's direct restriction:
// coarse levels with the decision on r_k, then level 0.
hipError_t apply_iter(mas_handle* h, const SolverView& v, bool mixed, int k, bool rr_true, hipStream_t s) {
    hipError_t e;
    if ((e = timed(
             h, kKCoarse, s,
             [&] { return launch_apply_coarse(v, mixed, kApplyIter, k, 0.0, false, mixed, rr_true, s); },
             2 * k)) != hipSuccess)
        return e;
    return timed(h, kKLevel0, s, [&] { return launch_apply_level0(v, mixed, kApplyIter, k, s); }, 2 * k + 1);
}

int read_state(mas_handle* h, const SolverView& v, hipStream_t s) {
    HIP_TRY(hipMemcpyAsync(h->st_host, v.st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    collect_timing(h, h->st_host[0].iter);
    return MAS_OK;
}

// The PCG driver shared by pcg_solve and pcg_adjoint.  Iteration k takes
// three launches:
//   p = z + beta p, q = H p (sigma partials) and the restriction of q ->
//   convergence test on r_{k-1}, alpha, C_l r_k = C_l r_{k-1} - alpha C_l q_k
//   and the coarse apply -> x += alpha p, r -= alpha q (||r||^2 partials),
//   level-0 apply and prolongation (rho partials);
// every replace_every-th iteration (and every iteration when the SpMV cannot
// lend shared memory to the restriction) restricts r_k itself instead:
//   SpMV -> x/r update with the restriction of r_k -> [mixed: FP64 residual
//   replacement] -> convergence test on r_k and coarse apply -> level-0
//   apply, which also bounds the rounding the recurrence accumulates.
// The host reads the state every check_every iterations; iterations queued
// after a stop return at once.
int solve_impl(mas_handle* h, const mas_bcsr* H, const double* b, double* x, const pcg_options* o, pcg_result* res,
               hipStream_t s) {
    if (!h || !h->analyzed) return MAS_NOT_READY;
    if (!h->built) return MAS_NOT_READY;
    if (!bcsr_ok(h, H) || !b || !x || b == x) return MAS_INVALID_ARG;
    pcg_options opt{1e-4, 10000, 0, 50, 8};
    if (o) opt = *o;
    if (!(opt.tol >= 0.0) || opt.max_iter < 0) return MAS_INVALID_ARG;
    if (opt.replace_every <= 0) opt.replace_every = 50;
    if (opt.check_every <= 0) opt.check_every = 8;
    const bool mixed = h->opts.precision == MAS_PRECISION_MIXED;
    const bool x0 = opt.x0_given != 0;
    const SolverView v = view(h);

    HIP_TRY(hipEventRecord(h->ev[kEvSolve0], s));
    HIP_TRY(timed(h, kKPermute, s, [&] { return launch_permute_H(v, static_cast<const double*>(H->val), mixed, s); }));
    HIP_TRY(hipEventRecord(h->ev[kEvSolve1], s));
    HIP_TRY(launch_state_reset(v, s));
    HIP_TRY(launch_perm_in(v, b, v.b, s));
    if (x0) {
        HIP_TRY(launch_perm_in(v, x, v.x, s));
        HIP_TRY(launch_residual(v, kResidInit, v.r, s));
    } else {
        HIP_TRY(launch_init_rhs(v, s));
    }
    HIP_TRY(launch_apply_coarse(v, mixed, kApplyInit, 0, opt.tol, x0, mixed, false, s));
    HIP_TRY(launch_apply_level0(v, mixed, kApplyInit, 0, s));

    int k = 0;
    int rc = MAS_OK;
    DevState& st = *h->st_host;
    // Iterations run in batches of check_every.  After each batch the device
    // state is copied into a pinned slot; the host looks at a batch's copy
    // only once the next batch is queued, so the device never waits for the
    // host.  Kernels queued after a stop return at once.
    auto direct = [&](int kk) { return !h->fuse_ok || kk % opt.replace_every == 0; };
    auto batch = [&](int nb) -> int {
        for (int i = 0; i < nb; ++i) {
            ++k;
            if (!direct(k)) {
                HIP_TRY(timed(h, kKSpmv, s, [&] { return launch_spmv_pq(v, mixed, k, true, s); }, 2 * k));
                HIP_TRY(timed(
                    h, kKCoarse, s,
                    [&] { return launch_apply_coarse(v, mixed, kApplyRec, k, 0.0, false, mixed, false, s); },
                    2 * k));
                HIP_TRY(timed(h, kKLevel0Upd, s, [&] { return launch_apply_level0(v, mixed, kApplyRec, k, s); },
                              2 * k));
                continue;
            }
            HIP_TRY(timed(h, kKSpmv, s, [&] { return launch_spmv_pq(v, mixed, k, false, s); }, 2 * k));
            HIP_TRY(timed(h, kKUpdate, s, [&] { return launch_update(v, k, s); }, 2 * k));
            bool replaced = false;
            if (mixed && k % opt.replace_every == 0) {
                HIP_TRY(timed(h, kKResidual, s, [&] { return launch_residual(v, kResidReplace, v.r, s); }, 2 * k));
                replaced = true;
            }
            HIP_TRY(apply_iter(h, v, mixed, k, replaced, s));
        }
        // a last iteration by recurrence leaves its decision to the next
        // coarse launch: at max_iter, take it here
        if (k == opt.max_iter && k > 0 && !direct(k))
            HIP_TRY(launch_apply_coarse(v, mixed, kApplyIter, k, 0.0, false, mixed, false, s, true));
        return MAS_OK;
    };
    int inflight = 0, head = 0, next = 0;  // batch copies not yet looked at; ring slots 1 + (0|1)
    for (;;) {
        while (inflight < 2 && k < opt.max_iter) {
            if ((rc = batch(std::min(opt.check_every, opt.max_iter - k))) != MAS_OK) return rc;
            HIP_TRY(hipMemcpyAsync(h->st_host + 1 + next, v.st, sizeof(DevState), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipEventRecord(h->ev[kEvPoll0 + next], s));
            next ^= 1;
            ++inflight;
        }
        if (inflight == 0) break;  // max_iter reached, every batch looked at
        HIP_TRY(hipEventSynchronize(h->ev[kEvPoll0 + head]));
        const DevState seen = h->st_host[1 + head];
        head ^= 1;
        --inflight;
        if (seen.status >= 0 && !seen.done) continue;
        // stopped: let the batch still queued run out (no-ops) and read the state
        if ((rc = read_state(h, v, s)) != MAS_OK) return rc;
        inflight = 0;
        head = next;
        if (st.status != kStatusConvergedRecurrence) break;
        // stopped on the recurrence: confirm on the FP64 residual b - H x,
        // which also replaces r; if it is not small enough, finish iteration
        // st.iter with it and go on
        k = st.iter;
        HIP_TRY(launch_clear_stop(v, s));
        HIP_TRY(timed(h, kKResidual, s, [&] { return launch_residual(v, kResidConfirm, v.r, s); }, 2 * k));
        HIP_TRY(apply_iter(h, v, mixed, k, true, s));
        if ((rc = read_state(h, v, s)) != MAS_OK) return rc;
        if (st.done || st.status < 0) break;
    }
    if ((rc = read_state(h, v, s)) != MAS_OK) return rc;
    if (st.bb == 0.0)  // b = 0: the solution is x = b = 0 (also when an x0 was given)
        HIP_TRY(hipMemcpyAsync(v.x, v.b, sizeof(double) * 3 * v.NS, hipMemcpyDeviceToDevice, s));
    HIP_TRY(launch_residual(v, kResidFinal, v.q, s));
    HIP_TRY(launch_finalize(v, s));
    HIP_TRY(launch_perm_out(v, v.x, x, s));
    HIP_TRY(hipEventRecord(h->ev[kEvSolve2], s));
    if ((rc = read_state(h, v, s)) != MAS_OK) return rc;

    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->ev[kEvSolve0], h->ev[kEvSolve1]) == hipSuccess) h->timings[2] = ms;
    if (hipEventElapsedTime(&ms, h->ev[kEvSolve1], h->ev[kEvSolve2]) == hipSuccess) h->timings[3] = ms;

    rc = finish_status(st);
    if (st.bb == 0.0 && st.status == 0) rc = MAS_OK;
    if (res) {
        res->status = rc;
        res->iterations = st.iter;
        res->rel_residual = st.bb > 0 ? std::sqrt(st.rr / st.bb) : 0.0;
        res->true_rel_residual = st.bb > 0 ? std::sqrt(st.rr_true / st.bb) : 0.0;
    }
    return rc;
}

}  // namespace

extern "C" {

int mas_create(const mas_options* opts, mas_handle** out) {
    if (!out) return MAS_INVALID_ARG;
    *out = nullptr;
    mas_options o{16, 0, MAS_PRECISION_F64, 0};
    if (opts) o = *opts;
    if (o.domain_size < 1 || o.domain_size > MAS_MAX_DOMAIN_SIZE) return MAS_INVALID_ARG;
    if (o.precision != MAS_PRECISION_F64 && o.precision != MAS_PRECISION_MIXED) return MAS_INVALID_ARG;
    if (o.reserved != 0 || o.max_levels > MAS_MAX_LEVELS) return MAS_INVALID_ARG;
    mas_handle* h = new (std::nothrow) mas_handle();
    if (!h) return MAS_HIP_ERROR;
    h->opts = o;
    *out = h;
    return MAS_OK;
}

void mas_destroy(mas_handle* h) {
    if (!h) return;
    if (h->st_host) (void)hipHostFree(h->st_host);
    if (h->flag_host) (void)hipHostFree(h->flag_host);
    if (h->events)
        for (auto& e : h->ev) (void)hipEventDestroy(e);
    for (auto& e : h->kt.pool) (void)hipEventDestroy(e);
    delete h;
}

namespace {

void set_fusion(mas_handle* h) {
    const Plan& R = h->plan;
    // three launches per iteration where the SpMV's restriction of q takes
    // one pass of its threads (restrict_fast_ok): on systems whose groups
    // have many more coarse units (a group of the membrane + bodies system
    // has up to 448 writers), the longer restriction in the SpMV costs more
    // than the x/r update launch it saves, and every iteration restricts r
    // directly
    h->fuse_ok = sizeof(double) * (3 * static_cast<size_t>(R.RG) + restrict_smem_doubles(R.RG, R.W1, R.L)) <=
                     spmv_restrict_capacity() &&
                 restrict_fast_ok(R.W1, R.GW, spmv_threads());
}

int analyze_impl(mas_handle* h, int32_t n_rows, int32_t nnzb, const int32_t* row_ptr, const int32_t* col_idx,
                 const int32_t* g_ptr, const int32_t* g_adj, const int32_t* part, int32_t n_parts) {
    if (!h) return MAS_INVALID_ARG;
    Plan P;
    const std::string err = analyze(n_rows, nnzb, row_ptr, col_idx, g_ptr, g_adj, h->opts.domain_size,
                                    h->opts.max_levels, P, part, n_parts);
    if (!err.empty()) return MAS_INVALID_ARG;
    h->plan = std::move(P);
    h->analyzed = true;
    h->built = false;
    h->uploaded_to = nullptr;
    h->dev = DevicePlan{};
    // level-1 reduction sources and level-0 inversion blocks in caller block order
    h->translated.assign(2, {});
    const Plan& Q = h->plan;
    if (Q.L > 1) {
        h->translated[0].resize(Q.red_src[1].size());
        for (size_t k = 0; k < Q.red_src[1].size(); ++k) h->translated[0][k] = Q.perm_src[Q.red_src[1][k]];
    }
    h->translated[1].resize(Q.dom_blk[0].size());
    for (size_t k = 0; k < Q.dom_blk[0].size(); ++k) h->translated[1][k] = Q.perm_src[Q.dom_blk[0][k]];
    h->shape = shape_of(h->plan);
    make_layout(h);
    set_fusion(h);
    return MAS_OK;
}

}  // namespace

int mas_analyze(mas_handle* h, int32_t n_rows, int32_t nnzb, const int32_t* row_ptr, const int32_t* col_idx,
                const int32_t* g_ptr, const int32_t* g_adj) {
    return analyze_impl(h, n_rows, nnzb, row_ptr, col_idx, g_ptr, g_adj, nullptr, 0);
}

int mas_analyze_partition(mas_handle* h, int32_t n_rows, int32_t nnzb, const int32_t* row_ptr,
                          const int32_t* col_idx, const int32_t* part, int32_t n_parts) {
    if (!part) return MAS_INVALID_ARG;
    return analyze_impl(h, n_rows, nnzb, row_ptr, col_idx, nullptr, nullptr, part, n_parts);
}

size_t mas_workspace_size(const mas_handle* h) { return (h && h->analyzed) ? h->lay.total : 0; }

int mas_build(mas_handle* h, const mas_bcsr* H, void* workspace, size_t ws_bytes, void* stream) {
    if (!h) return MAS_INVALID_ARG;
    if (!h->analyzed) return MAS_NOT_READY;
    if (!bcsr_ok(h, H) || !workspace) return MAS_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return MAS_INVALID_ARG;
    if (ws_bytes < h->lay.total) return MAS_WORKSPACE_TOO_SMALL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!h->st_host) {
        HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&h->st_host), 3 * sizeof(DevState), hipHostMallocDefault));
        HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&h->flag_host), sizeof(int), hipHostMallocDefault));
    }
    if (!h->events) {
        for (int i = 0; i < kEvCount; ++i)
            HIP_TRY(hipEventCreateWithFlags(&h->ev[i], i >= kEvPoll0 ? hipEventDisableTiming : hipEventDefault));
        h->events = true;
    }
    h->ws = static_cast<char*>(workspace);
    h->ws_size = ws_bytes;
    h->built = false;
    if (h->uploaded_to != h->ws) {
        int rc = h->dev.active ? place_device_plan(h, s) : upload_plan(h, s);
        if (rc != MAS_OK) return rc;
        h->uploaded_to = h->ws;
    }
    const SolverView v = view(h);
    const BuildView bv = build_view(h);
    const bool mixed = h->opts.precision == MAS_PRECISION_MIXED;
    const double* Hu = static_cast<const double*>(H->val);
    *h->flag_host = 0;
    HIP_TRY(hipMemcpyAsync(v.flag, h->flag_host, sizeof(int), hipMemcpyHostToDevice, s));
    HIP_TRY(launch_state_reset(v, s));
    HIP_TRY(hipEventRecord(h->ev[kEvBuild0], s));
    HIP_TRY(launch_coarse_sums(bv, Hu, s));
    HIP_TRY(hipEventRecord(h->ev[kEvBuild1], s));
    HIP_TRY(launch_invert(bv, Hu, mixed, s));
    HIP_TRY(hipEventRecord(h->ev[kEvBuild2], s));
    HIP_TRY(hipMemcpyAsync(h->flag_host, v.flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->ev[kEvBuild0], h->ev[kEvBuild1]) == hipSuccess) h->timings[0] = ms;
    if (hipEventElapsedTime(&ms, h->ev[kEvBuild1], h->ev[kEvBuild2]) == hipSuccess) h->timings[1] = ms;
    if (*h->flag_host) return MAS_NOT_SPD;
    h->built = true;
    return MAS_OK;
}

int mas_apply(mas_handle* h, const double* r, double* z, void* stream) {
    if (!h || !h->analyzed || !h->built) return MAS_NOT_READY;
    if (!r || !z || r == z) return MAS_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const SolverView v = view(h);
    const bool mixed = h->opts.precision == MAS_PRECISION_MIXED;
    HIP_TRY(launch_perm_in(v, r, v.r, s));
    HIP_TRY(timed(h, kKRestrict, s, [&] { return launch_restrict(v, s); }));
    HIP_TRY(launch_apply_coarse(v, mixed, kApplyPlain, 0, 0.0, false, mixed, false, s));
    HIP_TRY(launch_apply_level0(v, mixed, kApplyPlain, 0, s));
    HIP_TRY(launch_perm_out(v, v.z, z, s));
    return MAS_OK;
}

int bcsr_spmv(const mas_bcsr* H, const double* x, double* y, void* stream) {
    if (!H || !x || !y || x == y) return MAS_INVALID_ARG;
    if (H->n_rows < 0 || H->nnzb < 0 || (H->dtype != MAS_F64 && H->dtype != MAS_F32)) return MAS_INVALID_ARG;
    if (H->n_rows == 0) return MAS_OK;
    if (!H->row_ptr || !H->col_idx || (H->nnzb > 0 && !H->val)) return MAS_INVALID_ARG;
    HIP_TRY(launch_spmv_user(H->n_rows, H->row_ptr, H->col_idx, H->val, H->dtype == MAS_F32, x, y,
                             static_cast<hipStream_t>(stream)));
    return MAS_OK;
}

int pcg_solve(mas_handle* h, const mas_bcsr* H, const double* b, double* x, const pcg_options* opts, pcg_result* res,
              void* stream) {
    const int rc = solve_impl(h, H, b, x, opts, res, static_cast<hipStream_t>(stream));
    if (res && rc != res->status) res->status = rc;
    return rc;
}

int pcg_adjoint(mas_handle* h, const mas_bcsr* H, const double* x, const double* dLdx, double* lambda, void* dLdH,
                int32_t dLdH_dtype, const pcg_options* opts, pcg_result* res, void* stream) {
    if (!x || !dLdx || !lambda || x == lambda || dLdx == lambda) return MAS_INVALID_ARG;
    if (dLdH && dLdH_dtype != MAS_F64 && dLdH_dtype != MAS_F32) return MAS_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int rc = solve_impl(h, H, dLdx, lambda, opts, res, s);
    if (rc < 0) return rc;
    if (dLdH) {
        HIP_TRY(launch_adjoint_scatter(H->n_rows, H->row_ptr, H->col_idx, lambda, x, dLdH, dLdH_dtype == MAS_F32, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    return rc;
}

size_t bcsr_assemble_workspace_size(int32_t n_rows, int64_t n_in) {
    if (n_rows < 1 || n_in < 0) return 0;
    size_t total = 0;
    assemble_layout(nullptr, n_rows, n_in, &total);
    return total;
}

}  // extern "C"

namespace {

// bcsr_assemble on scratch memory ws (256-byte aligned, at least
// bcsr_assemble_workspace_size bytes: checked by the callers).
int assemble_impl(int32_t n_rows, int64_t n_in, const int32_t* rows, const int32_t* cols, const double* blocks,
                  int32_t* row_ptr, int32_t* col_idx, double* val, int64_t capacity, int64_t* nnzb, char* ws,
                  hipStream_t s) {
    const AsmLayout L = assemble_layout(ws, n_rows, n_in, nullptr);
    HIP_TRY(launch_assemble_sort(L, n_rows, n_in, rows, cols, row_ptr, s));
    int host[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(host, L.flag, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (host[0]) return MAS_INVALID_ARG;  // an index out of range
    *nnzb = host[1];
    if (host[1] > capacity || (host[1] > 0 && (!col_idx || !val))) return MAS_INVALID_ARG;
    HIP_TRY(launch_assemble_reduce(L, n_in, blocks, col_idx, val, host[1], s));
    HIP_TRY(hipStreamSynchronize(s));
    return MAS_OK;
}

bool assemble_args_ok(int32_t n_rows, int64_t n_in, const int32_t* rows, const int32_t* cols, const double* blocks,
                      int32_t* row_ptr, int64_t capacity, int64_t* nnzb) {
    if (n_rows < 1 || n_rows > 0x7ffffffe || n_in < 0 || n_in > 0x7fffffffLL || capacity < 0 || !nnzb ||
        !row_ptr)
        return false;
    return n_in == 0 || (rows && cols && blocks);
}

// Scratch of bcsr_assemble_noalloc.  Each device the library runs on holds
// its own copy from the code object's load until the process ends.  Host
// code never passes the array's name to a kernel or a copy (on the host it
// only stands for the symbol): it looks up the device address once per
// device and uses that.
__device__ __align__(256) char scratch[MAS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch (looked up on the first
// call on that device, with it current).
int noalloc_scratch(char** out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return MAS_HIP_ERROR;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MAS_HIP_ERROR;
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<char*>(g_scratch_ptr[dev]);
    return MAS_OK;
}

}  // namespace

extern "C" {

int bcsr_assemble(int32_t n_rows, int64_t n_in, const int32_t* rows, const int32_t* cols, const double* blocks,
                  int32_t* row_ptr, int32_t* col_idx, double* val, int64_t capacity, int64_t* nnzb,
                  void* workspace, size_t ws_bytes, void* stream) {
    if (!assemble_args_ok(n_rows, n_in, rows, cols, blocks, row_ptr, capacity, nnzb) || !workspace)
        return MAS_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return MAS_INVALID_ARG;
    if (ws_bytes < bcsr_assemble_workspace_size(n_rows, n_in)) return MAS_WORKSPACE_TOO_SMALL;
    return assemble_impl(n_rows, n_in, rows, cols, blocks, row_ptr, col_idx, val, capacity, nnzb,
                         static_cast<char*>(workspace), static_cast<hipStream_t>(stream));
}

size_t abd_contact_workspace_size(int32_t n_nodes, int64_t m) {
    if (n_nodes < 1 || m < 0) return 0;
    size_t total = 0;
    abd_layout(nullptr, n_nodes, m, &total);
    return total;
}

int abd_contact_blocks(int32_t n_nodes, const int32_t* node_row, const int32_t* node_is_body,
                       const double* node_xbar, int64_t m, const int32_t* r, const int32_t* c, const double* C,
                       int32_t levels, int32_t* out_rows, int32_t* out_cols, double* out_blocks, int64_t capacity,
                       int64_t* n_out, void* workspace, size_t ws_bytes, void* stream) {
    if (n_nodes < 1 || n_nodes > 0x7ffffffe || m < 0 || m > 0x7fffffffLL / 16 || capacity < 0 || !n_out ||
        !node_row || !node_is_body || !node_xbar || !workspace || (levels != 1 && levels != 2))
        return MAS_INVALID_ARG;
    if (m > 0 && (!r || !c || !C)) return MAS_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return MAS_INVALID_ARG;
    if (ws_bytes < abd_contact_workspace_size(n_nodes, m)) return MAS_WORKSPACE_TOO_SMALL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const AbdLayout L = abd_layout(static_cast<char*>(workspace), n_nodes, m, nullptr);
    const int *pr = r, *pc = c;
    const double* pv = C;
    long long np = m;
    if (levels == 2) {
        // first level: equal node pairs summed in list order (block-list
        // assembly over the contact nodes)
        int64_t pairs = 0;
        const int rc = assemble_impl(n_nodes, m, r, c, C, L.row_ptr, L.pair_col, L.pair_val, m, &pairs,
                                     static_cast<char*>(L.asm_ws), s);
        if (rc != MAS_OK) return rc;
        HIP_TRY(launch_abd_pair_rows(L, n_nodes, s));
        pr = L.pair_row;
        pc = L.pair_col;
        pv = L.pair_val;
        np = pairs;
    } else {
        HIP_TRY(launch_abd_check(L, m, n_nodes, r, c, s));
        int bad = 0;
        HIP_TRY(hipMemcpyAsync(&bad, L.flag, sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (bad) return MAS_INVALID_ARG;
    }
    HIP_TRY(launch_abd_count(L, np, pr, pc, node_is_body, s));
    int total = 0;
    HIP_TRY(hipMemcpyAsync(&total, L.off + np, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *n_out = total;
    if (total > capacity || (total > 0 && (!out_rows || !out_cols || !out_blocks))) return MAS_INVALID_ARG;
    HIP_TRY(launch_abd_expand(L, np, pr, pc, pv, node_row, node_is_body, node_xbar, out_rows, out_cols, out_blocks,
                              s));
    HIP_TRY(hipStreamSynchronize(s));
    return MAS_OK;
}

size_t mas_morton_workspace_size(int32_t n_rows) {
    if (n_rows < 1) return 0;
    size_t total = 0;
    morton_layout(nullptr, n_rows, &total);
    return total;
}

int mas_morton_partition(int32_t n_rows, const double* positions, int32_t domain_size, int32_t* part,
                         void* workspace, size_t ws_bytes, void* stream) {
    if (n_rows < 1 || domain_size < 1 || !positions || !part || !workspace) return MAS_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return MAS_INVALID_ARG;
    if (ws_bytes < mas_morton_workspace_size(n_rows)) return MAS_WORKSPACE_TOO_SMALL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const MortonLayout L = morton_layout(static_cast<char*>(workspace), n_rows, nullptr);
    HIP_TRY(launch_morton_partition(L, n_rows, domain_size, positions, part, s));
    return MAS_OK;
}

int bcsr_assemble_noalloc(int32_t n_rows, int64_t n_in, const int32_t* rows, const int32_t* cols,
                          const double* blocks, int32_t* row_ptr, int32_t* col_idx, double* val, int64_t capacity,
                          int64_t* nnzb, void* stream) {
    if (!assemble_args_ok(n_rows, n_in, rows, cols, blocks, row_ptr, capacity, nnzb)) return MAS_INVALID_ARG;
    if (bcsr_assemble_workspace_size(n_rows, n_in) > MAS_NOALLOC_SCRATCH_BYTES) return MAS_WORKSPACE_TOO_SMALL;
    char* ws = nullptr;
    const int rc = noalloc_scratch(&ws);
    if (rc != MAS_OK) return rc;
    return assemble_impl(n_rows, n_in, rows, cols, blocks, row_ptr, col_idx, val, capacity, nnzb, ws,
                         static_cast<hipStream_t>(stream));
}

namespace {

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

size_t mas_hierarchy_workspace_size(const mas_handle* h) {
    if (!h || !h->analyzed) return 0;
    const Plan& P = h->plan;
    size_t t = 0;
    hierarchy_layout(nullptr, P.NS, kMaxLv, &t);
    return t + round256(sizeof(int) * (P.NS + 1)) + round256(sizeof(int) * P.nnzb) + round256(sizeof(int) * P.NS) +
           round256(sizeof(int) * P.V);
}

namespace {

struct HierWs {
    HierLayout H;
    int *rp, *ci, *remap, *map;
};

HierWs hier_ws(const Plan& P, char* ws) {
    HierWs W;
    size_t off = 0;
    W.H = hierarchy_layout(ws, P.NS, kMaxLv, &off);
    W.rp = reinterpret_cast<int*>(ws + off);
    off += round256(sizeof(int) * (P.NS + 1));
    W.ci = reinterpret_cast<int*>(ws + off);
    off += round256(sizeof(int) * P.nnzb);
    W.remap = reinterpret_cast<int*>(ws + off);
    off += round256(sizeof(int) * P.NS);
    W.map = reinterpret_cast<int*>(ws + off);
    return W;
}

int hier_level_cap(const mas_handle* h) {
    const int m = h->opts.max_levels;
    return m > 0 ? std::min(m, kMaxLv) : kMaxLv;
}

}  // namespace

int mas_hierarchy_device(mas_handle* h, int32_t* levels, int32_t* units, int32_t* sn, void* workspace,
                         size_t ws_bytes, void* stream) {
    if (!h) return MAS_INVALID_ARG;
    if (!h->analyzed) return MAS_NOT_READY;
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % kAlign) return MAS_INVALID_ARG;
    if (ws_bytes < mas_hierarchy_workspace_size(h)) return MAS_WORKSPACE_TOO_SMALL;
    const Plan& P = h->plan;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const HierWs W = hier_ws(P, static_cast<char*>(workspace));
    if (h->dev.active) {  // the slot-ordered pattern of the replan
        HIP_TRY(hipMemcpyAsync(W.rp, h->dev.R.rp0, sizeof(int) * (P.NS + 1), hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(W.ci, h->dev.R.ci0, sizeof(int) * P.nnzb, hipMemcpyDeviceToDevice, s));
    } else {
        HIP_TRY(hipMemcpyAsync(W.rp, P.rp0.data(), sizeof(int) * (P.NS + 1), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(W.ci, P.ci0.data(), sizeof(int) * P.nnzb, hipMemcpyHostToDevice, s));
    }
    HIP_TRY(hipMemcpyAsync(W.remap, P.remap.data(), sizeof(int) * P.NS, hipMemcpyHostToDevice, s));
    const HierPattern pat{W.rp, W.ci, nullptr, P.nnzb};
    HIP_TRY(launch_hierarchy(W.H, P.NS, P.V, P.N, hier_level_cap(h), W.remap, pat, s));
    HierState st{};
    HIP_TRY(hipMemcpyAsync(&st, W.H.st, sizeof(st), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const int L = st.levels;
    if (levels) *levels = L;
    if (units)
        for (int l = 0; l < L; ++l) units[l] = st.units[l];
    if (sn) {
        std::vector<int> slot_sn(static_cast<size_t>(L) * P.NS);
        HIP_TRY(hipMemcpyAsync(slot_sn.data(), W.H.sn, sizeof(int) * slot_sn.size(), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        for (int l = 0; l < L; ++l)
            for (int i = 0; i < P.V; ++i)
                sn[static_cast<size_t>(l) * P.V + i] = slot_sn[static_cast<size_t>(l) * P.NS + P.map[i]];
    }
    return MAS_OK;
}

int mas_hierarchy_rebuild(mas_handle* h, int64_t nnzb, const int32_t* row_ptr, const int32_t* col_idx,
                          int32_t* out_units, int32_t* out_sn, void* workspace, size_t ws_bytes, void* stream) {
    if (!h) return MAS_INVALID_ARG;
    if (!h->analyzed) return MAS_NOT_READY;
    if (nnzb < 0 || nnzb > 0x7fffffffLL || !row_ptr || (nnzb > 0 && !col_idx) || !out_units || !out_sn)
        return MAS_INVALID_ARG;
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % kAlign) return MAS_INVALID_ARG;
    if (ws_bytes < mas_hierarchy_workspace_size(h)) return MAS_WORKSPACE_TOO_SMALL;
    const Plan& P = h->plan;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const HierWs W = hier_ws(P, static_cast<char*>(workspace));
    // the node -> slot map: from the solver's workspace once mas_build has
    // placed the plans there, else copied from the handle
    const int* remap = W.remap;
    const int* map = W.map;
    if (h->uploaded_to) {
        remap = at<int>(h, h->lay.remap);
        map = at<int>(h, h->lay.map);
    } else {
        HIP_TRY(hipMemcpyAsync(W.remap, P.remap.data(), sizeof(int) * P.NS, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(W.map, P.map.data(), sizeof(int) * P.V, hipMemcpyHostToDevice, s));
    }
    const HierPattern pat{row_ptr, col_idx, map, nnzb};
    HIP_TRY(launch_hierarchy(W.H, P.NS, P.V, P.N, hier_level_cap(h), remap, pat, s));
    HIP_TRY(launch_hier_export(W.H, P.V, P.NS, map, out_units, out_sn, s));
    return MAS_OK;
}

size_t mas_replan_workspace_size(const mas_handle* h, int64_t nnzb) {
    if (!h || !h->analyzed || nnzb < 1 || nnzb > 0x7fffffffLL) return 0;
    const Plan& P = h->plan;
    size_t t = 0;
    replan_layout(nullptr, P.V, P.NS, P.G, nnzb, &t);
    return t;
}

int mas_replan(mas_handle* h, int64_t nnzb, const int32_t* row_ptr, const int32_t* col_idx, void* workspace,
               size_t ws_bytes, void* stream) {
    if (!h) return MAS_INVALID_ARG;
    if (!h->analyzed) return MAS_NOT_READY;
    const Plan& P0 = h->plan;
    if (nnzb < P0.V || nnzb > 0x7fffffffLL || !row_ptr || !col_idx) return MAS_INVALID_ARG;
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % kAlign) return MAS_INVALID_ARG;
    if (ws_bytes < mas_replan_workspace_size(h, nnzb)) return MAS_WORKSPACE_TOO_SMALL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const ReplanLayout R = replan_layout(static_cast<char*>(workspace), P0.V, P0.NS, P0.G, nnzb, nullptr);
    HIP_TRY(hipMemcpyAsync(R.map, P0.map.data(), sizeof(int) * P0.V, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(R.remap, P0.remap.data(), sizeof(int) * P0.NS, hipMemcpyHostToDevice, s));
    HIP_TRY(replan_validate_order_hierarchy(R, P0.V, P0.NS, P0.N, hier_level_cap(h), nnzb, row_ptr, col_idx, R.map,
                                            R.remap, s));
    ReplanCounts c{};
    HierState st{};
    HIP_TRY(hipMemcpyAsync(&c, R.counts, sizeof(c), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&st, R.H.st, sizeof(st), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (c.bad || c.nnz_distinct != nnzb) return MAS_INVALID_ARG;
    ReplanShape S{};
    S.V = P0.V;
    S.N = P0.N;
    S.NS = P0.NS;
    S.M = P0.M;
    S.L = st.levels;
    S.G = P0.G;
    S.RG = P0.RG;
    S.nnzb = nnzb;
    for (int l = 0; l < S.L; ++l) {
        S.units[l] = st.units[l];
        S.ndom[l] = (st.units[l] + S.N - 1) / S.N;
    }
    HIP_TRY(replan_sizes(R, S, s));
    const int G = S.G;
    std::vector<int> g_u1(static_cast<size_t>(G) + 1), gsz(3 * static_cast<size_t>(G));
    HIP_TRY(hipMemcpyAsync(&c, R.counts, sizeof(c), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(g_u1.data(), R.g_u1, sizeof(int) * g_u1.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(gsz.data(), R.gstore, sizeof(int) * gsz.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));

    // the new plan: the partition and its maps stay, every size is new
    Plan Q;
    Q.V = P0.V;
    Q.N = P0.N;
    Q.M = P0.M;
    Q.No = P0.No;
    Q.NS = P0.NS;
    Q.L = S.L;
    Q.nnzb = static_cast<int>(nnzb);
    Q.part = P0.part;
    Q.map = P0.map;
    Q.remap = P0.remap;
    Q.units.assign(S.units, S.units + S.L);
    Q.ndom.assign(S.ndom, S.ndom + S.L);
    Q.D0 = P0.D0;
    Q.RG = P0.RG;
    Q.G = P0.G;
    Q.W1 = 1;
    for (int g = 0; g < G; ++g) Q.W1 = std::max(Q.W1, g_u1[g + 1] - g_u1[g]);
    Q.GW = S.L > 2 ? std::max(1, c.gw_max) : 1;
    Q.n_cpart = S.L > 2 ? c.cbase[S.L] : 0;
    long long n_sym = 0, n_tidx = 0;
    Q.maxT = 0;
    for (int g = 0; g < G; ++g) {
        n_sym += gsz[G + g];
        n_tidx += gsz[2 * static_cast<size_t>(G) + g];
        Q.maxT = std::max(Q.maxT, gsz[2 * static_cast<size_t>(G) + g]);
    }
    Q.sym = Q.RG <= 256 && Q.maxT <= kMaxTransposed;
    std::vector<long long> cnt(G);
    for (int g = 0; g < G; ++g) cnt[g] = Q.sym ? gsz[G + g] : gsz[g];
    Q.gorder = spmv_group_order(cnt);
    Shape Z;
    Z.nsb = Q.sym ? static_cast<size_t>(n_sym) : static_cast<size_t>(nnzb);
    Z.n_tidx = static_cast<size_t>(n_tidx);
    PlacedShape ps{};
    ps.S = S;
    ps.sym = Q.sym ? 1 : 0;
    ps.W1 = Q.W1;
    ps.GW = Q.GW;
    for (int l = 0; l < S.L; ++l) {
        const int nA = l == 0 ? static_cast<int>(nnzb) : c.nnzA[l];
        Z.nnzA[l] = static_cast<size_t>(nA);
        Z.n_domblk[l] = static_cast<size_t>(c.ndomblk[l]);
        ps.nnzA[l] = nA;
    }
    h->plan = std::move(Q);
    h->shape = Z;
    h->translated.clear();
    h->dev.active = true;
    h->dev.R = R;
    h->dev.ps = ps;
    h->built = false;
    h->uploaded_to = nullptr;
    make_layout(h);
    set_fusion(h);
    return MAS_OK;
}

int mas_get_info(const mas_handle* h, mas_info* out) {
    if (!h || !out) return MAS_INVALID_ARG;
    if (!h->analyzed) return MAS_NOT_READY;
    const Plan& P = h->plan;
    std::memset(out, 0, sizeof(*out));
    out->n_rows = P.V;
    out->nnzb = P.nnzb;
    out->domain_size = P.N;
    out->parts = P.M;
    out->slack = P.No;
    out->levels = P.L;
    for (int l = 0; l < P.L; ++l) {
        out->units[l] = P.units[l];
        out->domains[l] = P.ndom[l];
        out->coarse_nnzb[l] = static_cast<int>(h->shape.nnzA[l]);
    }
    out->workspace_bytes = static_cast<int64_t>(h->lay.total);
    out->inverse_bytes = static_cast<int64_t>(h->lay.inverse_bytes);
    out->stored_blocks = static_cast<int32_t>(h->shape.nsb);
    return MAS_OK;
}

int mas_get_ordering(const mas_handle* h, int32_t* map, int32_t* remap, int32_t* sn) {
    if (!h) return MAS_INVALID_ARG;
    if (!h->analyzed) return MAS_NOT_READY;
    const Plan& P = h->plan;
    if (map) std::memcpy(map, P.map.data(), sizeof(int) * P.map.size());
    if (remap) std::memcpy(remap, P.remap.data(), sizeof(int) * P.remap.size());
    if (sn && !h->dev.active) std::memcpy(sn, P.sn.data(), sizeof(int) * P.sn.size());
    if (sn && h->dev.active) {  // from the hierarchy in the replan workspace (unchanged since mas_replan)
        std::vector<int> slot_sn(static_cast<size_t>(P.L) * P.NS);
        HIP_TRY(hipMemcpy(slot_sn.data(), h->dev.R.H.sn, sizeof(int) * slot_sn.size(), hipMemcpyDeviceToHost));
        for (int l = 0; l < P.L; ++l)
            for (int i = 0; i < P.V; ++i)
                sn[static_cast<size_t>(l) * P.V + i] = slot_sn[static_cast<size_t>(l) * P.NS + P.map[i]];
    }
    return MAS_OK;
}

int mas_get_inverses(const mas_handle* h, int32_t level, int32_t precision, double* out, void* stream) {
    if (!h || !out) return MAS_INVALID_ARG;
    if (!h->analyzed || !h->built) return MAS_NOT_READY;
    const Plan& P = h->plan;
    if (level < 0 || level >= P.L) return MAS_INVALID_ARG;
    const bool want32 = precision == MAS_PRECISION_MIXED;
    if (!want32 && precision != MAS_PRECISION_F64) return MAS_INVALID_ARG;
    if (want32 && h->opts.precision != MAS_PRECISION_MIXED) return MAS_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int n = 3 * P.N;
    const size_t nd = static_cast<size_t>(P.ndom[level]), full = nd * n * n;
    if (want32) {
        std::vector<float> tmp(full);
        HIP_TRY(hipMemcpyAsync(tmp.data(), h->ws + h->lay.inv32[level], sizeof(float) * full, hipMemcpyDeviceToHost,
                               s));
        HIP_TRY(hipStreamSynchronize(s));
        for (size_t e = 0; e < full; ++e) out[e] = static_cast<double>(tmp[e]);
        return MAS_OK;
    }
    if (level == 0 && P.N == 16) {  // symmetric-packed: lower triangle column by column
        std::vector<double> tmp(nd * kPacked);
        HIP_TRY(hipMemcpyAsync(tmp.data(), h->ws + h->lay.inv64[0], sizeof(double) * tmp.size(),
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        for (size_t d = 0; d < nd; ++d) {
            const double* src = tmp.data() + d * kPacked;
            double* dst = out + d * n * n;
            for (int j = 0; j < n; ++j)
                for (int i = j; i < n; ++i) {
                    const double val = src[packed_col(j) + i - j];
                    dst[static_cast<size_t>(j) * n + i] = val;
                    dst[static_cast<size_t>(i) * n + j] = val;
                }
        }
        return MAS_OK;
    }
    HIP_TRY(hipMemcpyAsync(out, h->ws + h->lay.inv64[level], sizeof(double) * full, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return MAS_OK;
}

int mas_get_timings(const mas_handle* h, double* ms4) {
    if (!h || !ms4) return MAS_INVALID_ARG;
    for (int k = 0; k < 4; ++k) ms4[k] = h->timings[k];
    return MAS_OK;
}

int mas_set_kernel_timing(mas_handle* h, int enable) {
    if (!h) return MAS_INVALID_ARG;
    h->kt.on = enable != 0;
    for (int k = 0; k < kKSlots; ++k) {
        h->kt.total_ms[k] = 0.0;
        h->kt.launches[k] = 0;
    }
    h->kt.pending.clear();
    h->kt.used = 0;
    return MAS_OK;
}

int mas_get_kernel_timing(const mas_handle* h, double* total_ms, int32_t* launches) {
    if (!h || !total_ms || !launches) return MAS_INVALID_ARG;
    for (int k = 0; k < kKSlots; ++k) {
        total_ms[k] = h->kt.total_ms[k];
        launches[k] = h->kt.launches[k];
    }
    return MAS_OK;
}

const char* mas_status_string(int status) {
    switch (status) {
        case MAS_OK: return "ok";
        case MAS_NOT_CONVERGED: return "not converged (max_iter reached)";
        case MAS_INVALID_ARG: return "invalid argument";
        case MAS_NOT_SPD: return "matrix not symmetric positive definite";
        case MAS_HIP_ERROR: return "HIP runtime error";
        case MAS_WORKSPACE_TOO_SMALL: return "workspace too small";
        case MAS_NOT_READY: return "handle not ready (analyze, then build)";
        case MAS_NOT_FINITE: return "non-finite residual";
        default: return "unknown status";
    }
}

}  // extern "C"
