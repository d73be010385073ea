// Host-side symbolic analysis (see planner.hpp).
//
// Ordering (Sec. 4.2): the node graph is partitioned into
// M = ceil(V / (N - N_o)) parts of at most N nodes, the slack N_o searched
// upward from 0 (Eq. num_subdomains).  The paper uses METIS; here the
// partitioner is a recursive BFS bisection with fully specified tie-breaks
// so that an independent implementation reproduces it bit for bit:
//   split(S, k): k == 1 -> S is the next part; otherwise kL = k/2,
//   nL = floor(|S| kL / k) and S is cut after its first nL nodes in
//   pseudo-peripheral BFS order (start at the smallest id, twice jump to the
//   smallest id on the deepest BFS level, then the BFS visit order with
//   ascending neighbours, restarting at the smallest unvisited id).
// Part p occupies slots [pN, pN + N) in ascending node order; the rest of
// its slots are padding (-1), one part per MAS domain (Fig. mapping).
//
// Hierarchy (Sec. 4.1, Supp. Alg. 2-5): at each level the units of a domain
// that are coupled by stored blocks form connected components; each
// component is a supernode of the next level, numbered inside its domain by
// its lowest lane and globally by domain order.  N consecutive supernodes
// form a domain of the next level.  Construction stops at a single domain,
// at max_levels, or when no component merges two units.
#include "planner.hpp"

#include <algorithm>
#include <array>
#include <cstring>
#include <numeric>
#include <thread>

namespace maspcg {
namespace {

struct Graph {
    std::vector<int> off, nbr;
};

// Both directions of every edge (self loops and out-of-range ends
// dropped), each node's neighbours ascending and distinct: the edge list
// bucketed by node, then each bucket sorted.
Graph symmetrize(int V, const int32_t* ptr, const int32_t* adj) {
    std::vector<int> start(V + 1, 0);
    for (int i = 0; i < V; ++i)
        for (int p = ptr[i]; p < ptr[i + 1]; ++p) {
            const int j = adj[p];
            if (j < 0 || j >= V || j == i) continue;
            start[i + 1]++;
            start[j + 1]++;
        }
    for (int i = 0; i < V; ++i) start[i + 1] += start[i];
    std::vector<int> fill(start.begin(), start.end() - 1), nb(start[V]);
    for (int i = 0; i < V; ++i)
        for (int p = ptr[i]; p < ptr[i + 1]; ++p) {
            const int j = adj[p];
            if (j < 0 || j >= V || j == i) continue;
            nb[fill[i]++] = j;
            nb[fill[j]++] = i;
        }
    Graph g;
    g.off.assign(V + 1, 0);
    g.nbr.reserve(nb.size());
    for (int i = 0; i < V; ++i) {
        std::sort(nb.begin() + start[i], nb.begin() + start[i + 1]);
        for (int q = start[i]; q < start[i + 1]; ++q)
            if (q == start[i] || nb[q] != nb[q - 1]) g.nbr.push_back(nb[q]);
        g.off[i + 1] = static_cast<int>(g.nbr.size());
    }
    return g;
}

// A set of the recursion: nodes[lo, hi) (in the parent's BFS order), to be
// cut into k parts numbered from p0.
struct BisectTask {
    int lo, hi, k, p0;
};

// One worker of the recursive bisection.  nodes[] and asc[] are shared by
// all workers, each task owning its range: asc[lo, hi) holds the task's set
// ascending (split from the parent's ascending list, not sorted again).
// Each worker has its own membership tags, so workers on disjoint tasks do
// not interact, and a task's split depends on its set alone: the parts do
// not depend on how the tasks are spread over workers.
class Bisection {
  public:
    Bisection(const Graph& g, int* nodes, int* asc)
        : g_(g), nodes_(nodes), asc_(asc), in_(g.off.size() - 1, -1), seen_(g.off.size() - 1, -1),
          depth_(g.off.size() - 1, 0), tmp_(g.off.size() - 1) {}

    // Splits t (k >= 2) into its left and right tasks.
    void split(const BisectTask& t, BisectTask& left, BisectTask& right) {
        const int kl = t.k / 2;
        const int n = t.hi - t.lo;
        const int nl = static_cast<int>(static_cast<long long>(n) * kl / t.k);
        if (n > 0) {
            reorder(nodes_ + t.lo, asc_ + t.lo, n);
            split_ascending(nodes_ + t.lo, asc_ + t.lo, n, nl);
        }
        left = {t.lo, t.lo + nl, kl, t.p0};
        right = {t.lo + nl, t.hi, t.k - kl, t.p0 + kl};
    }

    // The whole subtree of t: part[node] for its nodes.
    void finish(const BisectTask& root, int* part) {
        std::vector<BisectTask> stack{root};
        while (!stack.empty()) {
            const BisectTask t = stack.back();
            stack.pop_back();
            if (t.k == 1) {
                for (int q = t.lo; q < t.hi; ++q) part[nodes_[q]] = t.p0;
                continue;
            }
            BisectTask left, right;
            split(t, left, right);
            stack.push_back(right);
            stack.push_back(left);
        }
    }

  private:
    // BFS inside the current set from root; appends visit order to out and
    // records depths.  Returns the deepest level reached.
    int bfs(int root, std::vector<int>& out) {
        size_t head = out.size();
        out.push_back(root);
        seen_[root] = mark_;
        depth_[root] = 0;
        int deepest = 0;
        while (head < out.size()) {
            const int u = out[head++];
            for (int p = g_.off[u]; p < g_.off[u + 1]; ++p) {
                const int v = g_.nbr[p];
                if (in_[v] != set_ || seen_[v] == mark_) continue;
                seen_[v] = mark_;
                depth_[v] = depth_[u] + 1;
                deepest = std::max(deepest, depth_[v]);
                out.push_back(v);
            }
        }
        return deepest;
    }

    // asc: the set ascending.
    void reorder(int* S, const int* asc, int n) {
        set_ = ++tag_;
        for (int q = 0; q < n; ++q) in_[S[q]] = set_;
        int root = asc[0];
        std::vector<int> visit;
        visit.reserve(n);
        for (int rep = 0; rep < 2; ++rep) {
            mark_ = ++tag_;
            visit.clear();
            const int deepest = bfs(root, visit);
            int best = -1;
            for (int v : visit)
                if (depth_[v] == deepest && (best < 0 || v < best)) best = v;
            root = best;
        }
        mark_ = ++tag_;
        visit.clear();
        bfs(root, visit);
        size_t scan = 0;
        while (static_cast<int>(visit.size()) < n) {
            while (seen_[asc[scan]] == mark_) ++scan;
            bfs(asc[scan], visit);
        }
        std::copy(visit.begin(), visit.end(), S);
    }

    // asc (the set ascending) reordered into the ascending lists of the
    // first nl nodes of S and of the rest.
    void split_ascending(const int* S, int* asc, int n, int nl) {
        const int left = ++tag_;
        for (int q = 0; q < nl; ++q) in_[S[q]] = left;
        int a = 0, b = nl;
        for (int q = 0; q < n; ++q) {
            const int v = asc[q];
            tmp_[in_[v] == left ? a++ : b++] = v;
        }
        std::copy(tmp_.begin(), tmp_.begin() + n, asc);
    }

    const Graph& g_;
    int *nodes_, *asc_;
    std::vector<int> in_, seen_, depth_, tmp_;
    int tag_ = 0, set_ = -1, mark_ = -1;
};

// Recursive bisection of all V nodes into k parts (see the file comment):
// the top of the recursion is split level by level, the tasks of a level
// on threads of their own, until there are enough subtrees for the
// threads; each subtree is then finished on a thread.
void bisect(const Graph& g, int k, std::vector<int>& part) {
    const int V = static_cast<int>(g.off.size()) - 1;
    std::vector<int> nodes(V), asc(V);
    std::iota(nodes.begin(), nodes.end(), 0);
    std::iota(asc.begin(), asc.end(), 0);
    const int hw = static_cast<int>(std::thread::hardware_concurrency());
    const int T = std::max(1, std::min(hw, 8));
    auto run_all = [&](int n_tasks, const auto& work) {
        if (n_tasks == 1 || T == 1) {
            for (int i = 0; i < n_tasks; ++i) work(i);
            return;
        }
        std::vector<std::thread> th;
        th.reserve(n_tasks);
        for (int i = 0; i < n_tasks; ++i) th.emplace_back(work, i);
        for (auto& x : th) x.join();
    };
    std::vector<BisectTask> level{{0, V, k, 0}};
    while (static_cast<int>(level.size()) < T) {
        std::vector<BisectTask> next(2 * level.size());
        bool any = false;
        for (const BisectTask& t : level) any |= t.k > 1;
        if (!any) break;
        run_all(static_cast<int>(level.size()), [&](int i) {
            const BisectTask& t = level[i];
            if (t.k <= 1) {  // a finished part (k = 1) or a placeholder (k = 0) moves down as it is
                next[2 * i] = t;
                next[2 * i + 1] = {t.hi, t.hi, 0, t.p0};  // placeholder: nothing to do
                return;
            }
            Bisection b(g, nodes.data(), asc.data());
            b.split(t, next[2 * i], next[2 * i + 1]);
        });
        level.swap(next);
    }
    run_all(static_cast<int>(level.size()), [&](int i) {
        if (level[i].k < 1) return;
        Bisection b(g, nodes.data(), asc.data());
        b.finish(level[i], part.data());
    });
}

// Components of the units of each domain under the block pattern (rp, ci)
// over units.  Returns the next-level id of every unit (-1 if empty) and the
// number of components.
int components(int units, int N, const std::vector<int>& rp, const std::vector<int>& ci,
               const std::vector<char>& occupied, std::vector<int>& comp) {
    comp.assign(units, -1);
    int next = 0;
    std::vector<int> stack;
    for (int d = 0; d * N < units; ++d) {
        const int lo = d * N, hi = std::min(units, lo + N);
        for (int u = lo; u < hi; ++u) {
            if (!occupied[u] || comp[u] >= 0) continue;
            const int id = next++;
            comp[u] = id;
            stack.assign(1, u);
            while (!stack.empty()) {
                const int s = stack.back();
                stack.pop_back();
                for (int p = rp[s]; p < rp[s + 1]; ++p) {
                    const int t = ci[p];
                    if (t < lo || t >= hi || comp[t] >= 0) continue;
                    comp[t] = id;
                    stack.push_back(t);
                }
            }
        }
    }
    return next;
}

// Galerkin pattern and reduction plan: block (s, t) of the fine matrix goes
// to block (up[s], up[t]) of the coarse one.  The fine blocks are ordered
// by (up[s], up[t]), equal pairs in block order: a stable counting sort by
// up[t], then one by up[s].
void coarsen(const std::vector<int>& rp, const std::vector<int>& ci, const std::vector<int>& up, int coarse_units,
             std::vector<int>& rpC, std::vector<int>& ciC, std::vector<int>& red_ptr, std::vector<int>& red_src) {
    const int fine_units = static_cast<int>(rp.size()) - 1;
    const int nnz = rp.back();
    std::vector<long long> key(nnz);
    std::vector<int> row(nnz);
    for (int s = 0; s < fine_units; ++s)
        for (int p = rp[s]; p < rp[s + 1]; ++p) {
            key[p] = static_cast<long long>(up[s]) * coarse_units + up[ci[p]];
            row[p] = up[s];
        }
    std::vector<int> by_col(nnz), cnt(coarse_units + 1);
    for (int p = 0; p < nnz; ++p) cnt[up[ci[p]] + 1]++;
    for (int c = 0; c < coarse_units; ++c) cnt[c + 1] += cnt[c];
    for (int p = 0; p < nnz; ++p) by_col[cnt[up[ci[p]]]++] = p;
    std::fill(cnt.begin(), cnt.end(), 0);
    for (int p = 0; p < nnz; ++p) cnt[row[p] + 1]++;
    for (int c = 0; c < coarse_units; ++c) cnt[c + 1] += cnt[c];
    red_src.resize(nnz);
    for (int q = 0; q < nnz; ++q) red_src[cnt[row[by_col[q]]]++] = by_col[q];
    rpC.assign(coarse_units + 1, 0);
    ciC.clear();
    red_ptr.assign(1, 0);
    for (int q = 0; q < nnz; ++q) {
        const long long k = key[red_src[q]];
        if (q == 0 || k != key[red_src[q - 1]]) {
            if (q) red_ptr.push_back(q);
            ciC.push_back(static_cast<int>(k % coarse_units));
            rpC[k / coarse_units + 1]++;
        }
    }
    red_ptr.push_back(nnz);
    for (int s = 0; s < coarse_units; ++s) rpC[s + 1] += rpC[s];
}

void domain_plan(const std::vector<int>& rp, const std::vector<int>& ci, int units, int N, std::vector<int>& ptr,
                 std::vector<int>& blk, std::vector<int>& ab) {
    const int nd = (units + N - 1) / N;
    ptr.assign(1, 0);
    blk.clear();
    ab.clear();
    for (int d = 0; d < nd; ++d) {
        const int lo = d * N, hi = std::min(units, lo + N);
        for (int s = lo; s < hi; ++s)
            for (int p = rp[s]; p < rp[s + 1]; ++p) {
                const int t = ci[p];
                if (t < s || t >= lo + N) continue;
                blk.push_back(p);
                ab.push_back((s - lo) | ((t - lo) << 8));
            }
        ptr.push_back(static_cast<int>(blk.size()));
    }
}

// Group-symmetric storage (see Plan::srp).
void symmetric_storage(Plan& P) {
    const int NS = P.NS, RG = P.RG;
    P.srp.assign(NS + 1, 0);
    P.sci.clear();
    P.sperm.clear();
    P.srow.clear();
    P.sci.reserve(P.ci0.size());
    P.sperm.reserve(P.ci0.size());
    P.srow.reserve(P.ci0.size());
    std::vector<int> cnt(NS + 1, 0);
    for (int s = 0; s < NS; ++s) {
        const int r0 = s / RG * RG, r1 = std::min(r0 + RG, NS);
        for (int k = P.rp0[s]; k < P.rp0[s + 1]; ++k) {
            const int j = P.ci0[k];
            if (j < r0 || j >= r1 || j >= s) {
                P.sci.push_back(j);
                P.sperm.push_back(P.perm_src[k]);
                P.srow.push_back(static_cast<uint8_t>(s - r0));
                if (j >= r0 && j < r1 && j > s) cnt[j + 1]++;
            }
        }
        P.srp[s + 1] = static_cast<int>(P.sci.size());
    }
    P.tptr.assign(NS + 1, 0);
    for (int s = 0; s < NS; ++s) P.tptr[s + 1] = P.tptr[s] + cnt[s + 1];
    P.tidx.assign(P.tptr[NS], 0);
    std::vector<int> fill(P.tptr.begin(), P.tptr.end() - 1);
    for (int s = 0; s < NS; ++s) {
        const int r0 = s / RG * RG, r1 = std::min(r0 + RG, NS);
        for (int k = P.srp[s]; k < P.srp[s + 1]; ++k) {
            const int j = P.sci[k];
            if (j >= r0 && j < r1 && j > s) P.tidx[fill[j]++] = k;  // ascending k within row j
        }
    }
    P.maxT = 0;
    for (int g = 0; g < P.G; ++g) {
        const int r0 = g * RG, r1 = std::min(r0 + RG, NS);
        P.maxT = std::max(P.maxT, P.tptr[r1] - P.tptr[r0]);
    }
    P.sym = P.RG <= 256 && P.maxT <= kMaxTransposed;
}

// Workgroup order of the SpMV.  The group kernels give each XCD a
// contiguous range of groups, dispatched in order.  Groups with far more
// stored blocks than the mean (rows coupled to many distant columns, such as
// the rows of bodies attached to a sheet) tend to sit together at one end of
// the numbering, so one XCD gets all of them and starts them last.  When a
// group holds more than 1.5x the mean, the heavy groups are dealt
// round-robin over the XCDs, heaviest first, at the head of each XCD's
// order, and each XCD is then filled with a contiguous run of the other
// groups (keeping neighbouring groups, which share halo entries, on one
// XCD).  Otherwise gorder stays empty.
void spmv_order(Plan& P) {
    const int G = P.G, NS = P.NS, RG = P.RG;
    const std::vector<int>& rp = P.sym ? P.srp : P.rp0;
    std::vector<long long> cnt(std::max(G, 0));
    for (int g = 0; g < G; ++g) {
        const int r0 = g * RG, r1 = std::min(r0 + RG, NS);
        cnt[g] = rp[r1] - rp[r0];
    }
    P.gorder = spmv_group_order(cnt);
}

}  // namespace

std::vector<int> spmv_group_order(const std::vector<long long>& cnt) {
    const int G = static_cast<int>(cnt.size());
    std::vector<int> gorder;
    if (G <= 0) return gorder;
    double mean = 0.0;
    for (int g = 0; g < G; ++g) mean += static_cast<double>(cnt[g]);
    mean /= G;
    std::vector<int> heavy, light;
    for (int g = 0; g < G; ++g) (static_cast<double>(cnt[g]) > 1.5 * mean ? heavy : light).push_back(g);
    if (heavy.empty()) return gorder;
    std::stable_sort(heavy.begin(), heavy.end(), [&](int a, int b) { return cnt[a] > cnt[b]; });
    const int q = G / kXcdCount, rem = G % kXcdCount;
    std::array<std::vector<int>, kXcdCount> lists;
    auto cap = [&](int x) { return static_cast<size_t>(q + (x < rem ? 1 : 0)); };
    int x = 0;
    for (const int g : heavy) {
        while (lists[x].size() == cap(x)) x = (x + 1) % kXcdCount;
        lists[x].push_back(g);
        x = (x + 1) % kXcdCount;
    }
    size_t li = 0;
    for (x = 0; x < kXcdCount; ++x)
        while (lists[x].size() < cap(x)) lists[x].push_back(light[li++]);
    // workgroup b = i kXcdCount + x runs the i-th group of XCD x's list
    gorder.assign(G, -1);
    for (x = 0; x < kXcdCount; ++x)
        for (size_t i = 0; i < lists[x].size(); ++i) gorder[i * kXcdCount + x] = lists[x][i];
    return gorder;
}

std::string analyze(int V, int nnzb, const int32_t* row_ptr, const int32_t* col_idx, const int32_t* g_ptr,
                    const int32_t* g_adj, int N, int max_levels, Plan& P, const int32_t* part, int n_parts) {
    if (V <= 0 || nnzb < V || !row_ptr || !col_idx) return "empty matrix or null pattern";
    if (N < 1 || N > 40) return "domain_size must be in [1, 40]";
    if ((g_ptr == nullptr) != (g_adj == nullptr)) return "graph needs both g_ptr and g_adj";
    if (row_ptr[0] != 0 || row_ptr[V] != nnzb) return "row_ptr must start at 0 and end at nnzb";
    for (int i = 0; i < V; ++i) {
        if (row_ptr[i + 1] < row_ptr[i]) return "row_ptr not monotone";
        bool diag = false;
        for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            const int j = col_idx[p];
            if (j < 0 || j >= V) return "column index out of range";
            if (p > row_ptr[i] && j <= col_idx[p - 1]) return "columns must be strictly ascending in a row";
            diag |= (j == i);
        }
        if (!diag) return "every row needs its diagonal block";
    }
    for (int i = 0; i < V; ++i)
        for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            const int j = col_idx[p];
            if (!std::binary_search(col_idx + row_ptr[j], col_idx + row_ptr[j + 1], i)) return "pattern is not symmetric";
        }
    if (g_ptr) {
        if (g_ptr[0] != 0) return "g_ptr must start at 0";
        for (int i = 0; i < V; ++i)
            if (g_ptr[i + 1] < g_ptr[i]) return "g_ptr not monotone";
    }

    P = Plan();
    P.V = V;
    P.N = N;
    P.nnzb = nnzb;

    // ---- partition with the slack search of Eq. num_subdomains, or the
    // caller's (every part 1..N nodes)
    if (part) {
        if (n_parts < 1 || n_parts > V) return "n_parts must be in [1, n_rows]";
        std::vector<int> size(n_parts, 0);
        for (int i = 0; i < V; ++i) {
            if (part[i] < 0 || part[i] >= n_parts) return "part id out of range";
            if (++size[part[i]] > N) return "a part holds more than domain_size nodes";
        }
        for (int q = 0; q < n_parts; ++q)
            if (size[q] == 0) return "empty part";
    }
    const Graph g = part ? Graph() : (g_ptr ? symmetrize(V, g_ptr, g_adj) : symmetrize(V, row_ptr, col_idx));
    P.part.assign(V, 0);
    bool found = false;
    if (part) {
        P.part.assign(part, part + V);
        P.M = n_parts;
        P.No = 0;
        found = true;
    }
    for (int No = 0; No < N && !found; ++No) {
        const int M = (V + (N - No) - 1) / (N - No);
        bisect(g, M, P.part);
        std::vector<int> size(M, 0);
        bool fits = true;
        for (int i = 0; i < V; ++i) fits &= (++size[P.part[i]] <= N);
        if (fits) {
            P.M = M;
            P.No = No;
            found = true;
        }
    }
    if (!found) return "partition failed";

    // ---- slots (one part per domain, ascending node ids, -1 padding)
    P.NS = P.M * N;
    P.map.assign(V, -1);
    P.remap.assign(P.NS, -1);
    {
        std::vector<int> fill(P.M, 0);
        for (int i = 0; i < V; ++i) {
            const int s = P.part[i] * N + fill[P.part[i]]++;
            P.map[i] = s;
            P.remap[s] = i;
        }
    }

    // ---- H in slot order
    P.rp0.assign(P.NS + 1, 0);
    P.ci0.resize(nnzb);
    P.perm_src.resize(nnzb);
    for (int s = 0; s < P.NS; ++s) {
        const int i = P.remap[s];
        P.rp0[s + 1] = P.rp0[s] + (i >= 0 ? row_ptr[i + 1] - row_ptr[i] : 0);
    }
    {
        // rows are independent: ranges of slots on up to eight threads
        auto rows = [&](int s0, int s1) {
            std::vector<std::pair<int, int>> row;
            for (int s = s0; s < s1; ++s) {
                const int i = P.remap[s];
                if (i < 0) continue;
                row.clear();
                for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p) row.emplace_back(P.map[col_idx[p]], p);
                std::sort(row.begin(), row.end());
                for (size_t q = 0; q < row.size(); ++q) {
                    P.ci0[P.rp0[s] + q] = row[q].first;
                    P.perm_src[P.rp0[s] + q] = row[q].second;
                }
            }
        };
        const int T = nnzb >= (1 << 16) ? std::max(1, std::min(static_cast<int>(std::thread::hardware_concurrency()), 8)) : 1;
        std::vector<std::thread> th;
        for (int w = 1; w < T; ++w)
            th.emplace_back(rows, static_cast<int>(static_cast<long long>(P.NS) * w / T),
                            static_cast<int>(static_cast<long long>(P.NS) * (w + 1) / T));
        rows(0, static_cast<int>(static_cast<long long>(P.NS) / T));
        for (auto& x : th) x.join();
    }

    // ---- hierarchy
    P.units.push_back(P.NS);
    P.ndom.push_back(P.M);
    // room for every level up front: the loop holds references into rpA /
    // ciA while it appends the next level
    P.rpA.reserve(kMaxLevels);
    P.ciA.reserve(kMaxLevels);
    P.red_ptr.reserve(kMaxLevels);
    P.red_src.reserve(kMaxLevels);
    P.rpA.emplace_back();  // level 0 uses rp0 / ci0
    P.ciA.emplace_back();
    P.red_ptr.emplace_back();
    P.red_src.emplace_back();
    int occupied_count = V;
    for (int l = 0;; ++l) {
        if (P.ndom[l] == 1) break;
        if (max_levels > 0 && l + 1 >= max_levels) break;
        if (l + 1 >= kMaxLevels) break;
        const std::vector<int>& rp = l == 0 ? P.rp0 : P.rpA[l];
        const std::vector<int>& ci = l == 0 ? P.ci0 : P.ciA[l];
        std::vector<char> occ(P.units[l], 1);
        if (l == 0)
            for (int s = 0; s < P.NS; ++s) occ[s] = P.remap[s] >= 0;
        std::vector<int> comp;
        const int S = components(P.units[l], N, rp, ci, occ, comp);
        if (S == occupied_count) break;  // nothing merged
        P.up.push_back(comp);
        P.units.push_back(S);
        P.ndom.push_back((S + N - 1) / N);
        P.rpA.emplace_back();
        P.ciA.emplace_back();
        P.red_ptr.emplace_back();
        P.red_src.emplace_back();
        coarsen(rp, ci, comp, S, P.rpA[l + 1], P.ciA[l + 1], P.red_ptr[l + 1], P.red_src[l + 1]);
        occupied_count = S;
    }
    P.L = static_cast<int>(P.units.size());

    // ---- inversion plans
    P.dom_ptr.resize(P.L);
    P.dom_blk.resize(P.L);
    P.dom_ab.resize(P.L);
    for (int l = 0; l < P.L; ++l)
        domain_plan(l == 0 ? P.rp0 : P.rpA[l], l == 0 ? P.ci0 : P.ciA[l], P.units[l], N, P.dom_ptr[l], P.dom_blk[l],
                    P.dom_ab[l]);

    // ---- restriction / prolongation plans
    P.lead1.assign(P.NS, -1);
    if (P.L > 1) {
        for (int d = 0; d < P.M; ++d) {
            int last = -1;  // ids inside a domain appear in increasing order of lowest lane
            for (int a = 0; a < N; ++a) {
                const int u = P.up[0][d * N + a];
                if (u > last) {
                    P.lead1[d * N + a] = u;
                    last = u;
                }
            }
        }
    }
    P.lmask.assign(P.NS, 0);
    if (P.L > 1)
        for (int d = 0; d < P.M; ++d)
            for (int a = 0; a < N; ++a) {
                const int u = P.lead1[d * N + a];
                if (u < 0) continue;
                uint64_t m = 0;
                for (int b = 0; b < N; ++b)
                    if (P.up[0][d * N + b] == u) m |= uint64_t(1) << b;
                P.lmask[d * N + a] = m;
            }
    P.anc.assign(static_cast<size_t>(std::max(P.L - 1, 0)) * P.NS, -1);
    for (int l = 1; l < P.L; ++l)
        for (int s = 0; s < P.NS; ++s) {
            const int below = l == 1 ? s : P.anc[static_cast<size_t>(l - 2) * P.NS + s];
            P.anc[static_cast<size_t>(l - 1) * P.NS + s] = below < 0 ? -1 : P.up[l - 1][below];
        }
    // ---- work groups and per-group coarse partials
    P.D0 = std::max(1, 128 / N);
    P.RG = P.D0 * N;
    P.G = (P.M + P.D0 - 1) / P.D0;
    P.g_u1.assign(P.G + 1, 0);
    if (P.L > 1) {
        // level-1 ids follow domain order: count the units of each group
        for (int s = 0; s < P.NS; ++s)
            if (P.lead1[s] >= 0) P.g_u1[s / P.RG + 1]++;
        for (int g = 0; g < P.G; ++g) P.g_u1[g + 1] += P.g_u1[g];
    }
    P.anc1.assign(P.L, {});
    P.lead_pos.assign(P.L, {});
    P.cp_ptr.assign(P.L, {});
    P.n_cpart = 0;
    if (P.L > 2) {
        const int S1 = P.units[1];
        std::vector<int> a(S1);
        std::iota(a.begin(), a.end(), 0);
        for (int l = 2; l < P.L; ++l) {
            for (int& v : a) v = P.up[l - 1][v];
            P.anc1[l] = a;
            // (unit, group, writer) of every distinct (group, unit) pair
            std::vector<std::array<int, 3>> pairs;
            std::vector<int> seen(P.units[l], -1);
            for (int g = 0; g < P.G; ++g)
                for (int t = P.g_u1[g]; t < P.g_u1[g + 1]; ++t)
                    if (seen[a[t]] != g) {
                        seen[a[t]] = g;
                        pairs.push_back({a[t], g, t});
                    }
            std::sort(pairs.begin(), pairs.end());
            P.lead_pos[l].assign(S1, -1);
            P.cp_ptr[l].assign(P.units[l] + 1, 0);
            for (size_t k = 0; k < pairs.size(); ++k) {
                P.lead_pos[l][pairs[k][2]] = P.n_cpart + static_cast<int>(k);
                P.cp_ptr[l][pairs[k][0] + 1]++;
            }
            P.cp_ptr[l][0] = P.n_cpart;
            for (int u = 0; u < P.units[l]; ++u) P.cp_ptr[l][u + 1] += P.cp_ptr[l][u];
            P.n_cpart += static_cast<int>(pairs.size());
        }
    }

    P.W1 = 1;
    for (int g = 0; g < P.G; ++g) P.W1 = std::max(P.W1, P.g_u1[g + 1] - P.g_u1[g]);
    P.ganc.assign(P.L, {});
    P.gpos.assign(P.L, {});
    P.gmask.assign(P.L, {});
    for (int l = 2; l < P.L; ++l) {
        P.ganc[l].assign(static_cast<size_t>(P.G) * P.W1, -1);
        P.gpos[l].assign(static_cast<size_t>(P.G) * P.W1, -1);
        for (int g = 0; g < P.G; ++g)
            for (int t = P.g_u1[g]; t < P.g_u1[g + 1]; ++t) {
                const size_t o = static_cast<size_t>(g) * P.W1 + (t - P.g_u1[g]);
                P.ganc[l][o] = P.anc1[l][t];
                P.gpos[l][o] = P.lead_pos[l][t];
            }
        P.gmask[l].assign(static_cast<size_t>(P.G) * P.W1, 0);
        if (P.W1 <= 64)
            for (int g = 0; g < P.G; ++g) {
                const int lo = P.g_u1[g], n1 = P.g_u1[g + 1] - lo;
                for (int i = 0; i < n1; ++i) {
                    if (P.lead_pos[l][lo + i] < 0) continue;
                    uint64_t m = 0;
                    for (int j = 0; j < n1; ++j)
                        if (P.anc1[l][lo + j] == P.anc1[l][lo + i]) m |= uint64_t(1) << j;
                    P.gmask[l][static_cast<size_t>(g) * P.W1 + i] = m;
                }
            }
    }

    // the restriction tables by output (see Plan)
    P.gu1_slot.assign(static_cast<size_t>(P.G) * P.W1, -1);
    P.gu1_mask.assign(static_cast<size_t>(P.G) * P.W1, 0);
    if (P.L > 1)
        for (int s = 0; s < P.NS; ++s) {
            const int u = P.lead1[s];
            if (u < 0) continue;
            const int g = s / P.RG;
            const size_t o = static_cast<size_t>(g) * P.W1 + (u - P.g_u1[g]);
            P.gu1_slot[o] = s;
            P.gu1_mask[o] = P.lmask[s];
        }
    P.GW = 1;
    std::vector<std::vector<std::array<long long, 3>>> writers(P.G);
    for (int l = 2; l < P.L; ++l)
        for (int g = 0; g < P.G; ++g)
            for (int i = 0; i < P.W1; ++i) {
                const size_t o = static_cast<size_t>(g) * P.W1 + i;
                if (P.gpos[l][o] < 0) continue;
                writers[g].push_back({P.gpos[l][o], static_cast<long long>(l - 2) * P.W1 + i,
                                      static_cast<long long>(o)});
            }
    for (int g = 0; g < P.G; ++g) P.GW = std::max(P.GW, static_cast<int>(writers[g].size()));
    P.gw_pos.assign(static_cast<size_t>(P.G) * P.GW, -1);
    P.gw_li.assign(static_cast<size_t>(P.G) * P.GW, 0);
    P.gw_mask.assign(static_cast<size_t>(P.G) * P.GW, 0);
    for (int g = 0; g < P.G; ++g)
        for (size_t e = 0; e < writers[g].size(); ++e) {
            const size_t o = static_cast<size_t>(g) * P.GW + e;
            P.gw_pos[o] = static_cast<int>(writers[g][e][0]);
            P.gw_li[o] = static_cast<int>(writers[g][e][1]);
            const int l = 2 + static_cast<int>(writers[g][e][1] / P.W1);
            P.gw_mask[o] = P.gmask[l][static_cast<size_t>(writers[g][e][2])];
        }

    symmetric_storage(P);
    spmv_order(P);

    // ---- per-node units for reports
    P.sn.assign(static_cast<size_t>(P.L) * V, -1);
    for (int i = 0; i < V; ++i) {
        P.sn[i] = P.map[i];
        for (int l = 1; l < P.L; ++l) P.sn[static_cast<size_t>(l) * V + i] = P.anc[static_cast<size_t>(l - 1) * P.NS + P.map[i]];
    }
    return "";
}

}  // namespace maspcg
