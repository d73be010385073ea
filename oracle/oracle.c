/*
 * CPU oracle for the connectivity-enhanced MAS-preconditioned PCG solve.
 * TEST INFRASTRUCTURE ONLY -- see oracle.h for scope and conventions.
 *
 * Readings of points the paper leaves open (each also listed in the design
 * notes of the repository):
 *  - Partitioner (Sec. 4.2 uses METIS, unavailable here): recursive BFS
 *    bisection.  RB(S, k): k == 1 emits S as the next part; otherwise
 *    kL = k/2, kR = k - kL, nL = floor(|S| kL / k), order = BFS_ORDER(S),
 *    RB(order[0:nL], kL), RB(order[nL:], kR).  BFS_ORDER on the subgraph
 *    induced by S: start at the smallest id, twice move to the smallest id
 *    on the last BFS level (pseudo-peripheral node), then the BFS visit order
 *    from there (neighbours ascending; restart at the smallest unvisited id).
 *  - Slots: nodes of a part sorted by id (Supp. Alg. 1 sorts by part index).
 *  - Hierarchy: at level l the units of domain d are [dN, dN+N); unit s and t
 *    of the same domain are connected when a stored block (i, j), i != j,
 *    has sn_l(i) = s, sn_l(j) = t.  Components are the next level's
 *    supernodes, numbered per domain by lowest lane, domains in order
 *    (Sec. 4.1 case-study figure: a merged supernode takes the position of
 *    its lowest member; Supp. Alg. 5 elects the lowest lane).  Stop when a
 *    level has one domain, max_levels is reached or nothing merged.
 *  - Coarse weights: unit 3x3 identities (plain sums of blocks).
 *  - Domain matrices: summed in (row, column) order, then the upper scalar
 *    triangle is copied onto the lower one (exact symmetry).
 *  - Inverse of the occupied principal submatrix through Cholesky:
 *    Inv = L^-T L^-1; unoccupied lanes stay zero.
 *  - PCG: x0 = 0, stop when ||r||_2 <= tol ||b||_2 after the x/r update.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* graph helpers                                                            */
/* ------------------------------------------------------------------------ */

static int cmp_int(const void* a, const void* b) {
    int x = *(const int*)a, y = *(const int*)b;
    return (x > y) - (x < y);
}

/* Symmetric adjacency with ascending, unique neighbours and no self loops. */
static void canonical_graph(int V, const int* gptr, const int* gadj, int** out_ptr, int** out_adj) {
    int* deg = (int*)calloc((size_t)V + 1, sizeof(int));
    for (int i = 0; i < V; ++i)
        for (int p = gptr[i]; p < gptr[i + 1]; ++p) {
            int j = gadj[p];
            if (j == i || j < 0 || j >= V) continue;
            deg[i]++;
            deg[j]++;
        }
    int* ptr = (int*)malloc(((size_t)V + 1) * sizeof(int));
    ptr[0] = 0;
    for (int i = 0; i < V; ++i) ptr[i + 1] = ptr[i] + deg[i];
    int* fill = (int*)calloc((size_t)V + 1, sizeof(int));
    int* adj = (int*)malloc(((size_t)ptr[V] + 1) * sizeof(int));
    for (int i = 0; i < V; ++i)
        for (int p = gptr[i]; p < gptr[i + 1]; ++p) {
            int j = gadj[p];
            if (j == i || j < 0 || j >= V) continue;
            adj[ptr[i] + fill[i]++] = j;
            adj[ptr[j] + fill[j]++] = i;
        }
    /* sort and remove duplicates, compacting in place */
    int w = 0;
    int* nptr = (int*)malloc(((size_t)V + 1) * sizeof(int));
    nptr[0] = 0;
    for (int i = 0; i < V; ++i) {
        int s = ptr[i], e = ptr[i + 1];
        qsort(adj + s, (size_t)(e - s), sizeof(int), cmp_int);
        for (int p = s; p < e; ++p)
            if (p == s || adj[p] != adj[p - 1]) adj[w++] = adj[p];
        nptr[i + 1] = w;
    }
    free(deg);
    free(fill);
    free(ptr);
    *out_ptr = nptr;
    *out_adj = adj;
}

/* ------------------------------------------------------------------------ */
/* recursive BFS bisection                                                  */
/* ------------------------------------------------------------------------ */

typedef struct {
    int V;
    const int* ptr;
    const int* adj;
    int* in_set;   /* stamp of the set a node currently belongs to */
    int* seen;     /* stamp of the BFS run that reached the node */
    int* level;
    int* queue;
    int* sorted;   /* scratch: the set in ascending order */
    int stamp;
    int* part;
    int next_part;
} rb_ctx;

/* BFS over the subgraph induced by the set with stamp `set`, from `seed`.
 * Writes the visit order into ctx->queue (returns its length) and levels. */
static int bfs_from(rb_ctx* c, int set, int seed, int run) {
    int head = 0, tail = 0;
    c->queue[tail++] = seed;
    c->seen[seed] = run;
    c->level[seed] = 0;
    while (head < tail) {
        int u = c->queue[head++];
        for (int p = c->ptr[u]; p < c->ptr[u + 1]; ++p) {
            int v = c->adj[p];
            if (c->in_set[v] != set || c->seen[v] == run) continue;
            c->seen[v] = run;
            c->level[v] = c->level[u] + 1;
            c->queue[tail++] = v;
        }
    }
    return tail;
}

/* BFS_ORDER(S): reorders S[0..n) in place. */
static void bfs_order(rb_ctx* c, int* S, int n) {
    int set = ++c->stamp;
    for (int i = 0; i < n; ++i) c->in_set[S[i]] = set;
    memcpy(c->sorted, S, (size_t)n * sizeof(int));
    qsort(c->sorted, (size_t)n, sizeof(int), cmp_int);

    int seed = c->sorted[0];
    for (int rep = 0; rep < 2; ++rep) {
        int run = ++c->stamp;
        int cnt = bfs_from(c, set, seed, run);
        int maxlev = 0;
        for (int q = 0; q < cnt; ++q)
            if (c->level[c->queue[q]] > maxlev) maxlev = c->level[c->queue[q]];
        int best = -1;
        for (int q = 0; q < cnt; ++q) {
            int v = c->queue[q];
            if (c->level[v] == maxlev && (best < 0 || v < best)) best = v;
        }
        seed = best;
    }

    /* final BFS with restarts at the smallest unvisited id */
    int run = ++c->stamp;
    int out = 0, scan = 0;
    int* order = (int*)malloc((size_t)n * sizeof(int));
    while (out < n) {
        int start;
        if (out == 0) {
            start = seed;
        } else {
            while (c->seen[c->sorted[scan]] == run) ++scan;
            start = c->sorted[scan];
        }
        int cnt = bfs_from(c, set, start, run);
        memcpy(order + out, c->queue, (size_t)cnt * sizeof(int));
        out += cnt;
    }
    memcpy(S, order, (size_t)n * sizeof(int));
    free(order);
}

static void rb(rb_ctx* c, int* S, int n, int k) {
    if (k == 1) {
        for (int i = 0; i < n; ++i) c->part[S[i]] = c->next_part;
        c->next_part++;
        return;
    }
    int kL = k / 2, kR = k - kL;
    int nL = (int)(((long long)n * kL) / k);
    if (n > 0) bfs_order(c, S, n);
    rb(c, S, nL, kL);
    rb(c, S + nL, n - nL, kR);
}

int orc_partition(int V, const int* gptr, const int* gadj, int N, int* part, int* M_out, int* No_out) {
    if (V <= 0 || N <= 0) return ORC_INVALID;
    int *ptr, *adj;
    canonical_graph(V, gptr, gadj, &ptr, &adj);
    rb_ctx c;
    c.V = V;
    c.ptr = ptr;
    c.adj = adj;
    c.in_set = (int*)calloc((size_t)V, sizeof(int));
    c.seen = (int*)calloc((size_t)V, sizeof(int));
    c.level = (int*)calloc((size_t)V, sizeof(int));
    c.queue = (int*)malloc((size_t)V * sizeof(int));
    c.sorted = (int*)malloc((size_t)V * sizeof(int));
    c.part = part;
    int* S = (int*)malloc((size_t)V * sizeof(int));
    int status = ORC_INVALID;
    for (int No = 0; No < N; ++No) {
        int M = (V + (N - No) - 1) / (N - No); /* ceil(V / (N - N_o)) */
        for (int i = 0; i < V; ++i) S[i] = i;
        c.stamp = 0;
        memset(c.in_set, 0, (size_t)V * sizeof(int));
        memset(c.seen, 0, (size_t)V * sizeof(int));
        c.next_part = 0;
        rb(&c, S, V, M);
        int* size = (int*)calloc((size_t)M, sizeof(int));
        int ok = 1;
        for (int i = 0; i < V; ++i)
            if (++size[part[i]] > N) ok = 0;
        free(size);
        if (ok) {
            *M_out = M;
            *No_out = No;
            status = ORC_OK;
            break;
        }
    }
    free(S);
    free(c.in_set);
    free(c.seen);
    free(c.level);
    free(c.queue);
    free(c.sorted);
    free(ptr);
    free(adj);
    return status;
}

int orc_slots(int V, const int* part, int M, int N, int* map, int* remap) {
    int* fill = (int*)calloc((size_t)M, sizeof(int));
    for (int s = 0; s < M * N; ++s) remap[s] = -1;
    for (int i = 0; i < V; ++i) { /* ascending id inside each part */
        int p = part[i];
        if (p < 0 || p >= M || fill[p] >= N) {
            free(fill);
            return ORC_INVALID;
        }
        int slot = p * N + fill[p]++;
        map[i] = slot;
        remap[slot] = i;
    }
    free(fill);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* MAS hierarchy, domain matrices and inverses                              */
/* ------------------------------------------------------------------------ */

struct orc_mas {
    int V, N, M, No, L;
    int* map;                      /* [V] */
    int* remap;                    /* [M*N] */
    int* sn[ORC_MAX_LEVELS];       /* [V] unit of each node per level */
    int units[ORC_MAX_LEVELS];     /* level 0: M*N, else S_l */
    int ndom[ORC_MAX_LEVELS];
    double* K[ORC_MAX_LEVELS];     /* ndom * (3N)^2 */
    double* Inv[ORC_MAX_LEVELS];
};

static int find_root(int* par, int a) {
    while (par[a] != a) a = par[a];
    return a;
}

/* Lane a of level-l domain d holds a unit (a node or a supernode)? */
static int lane_occupied(const orc_mas* P, int l, int d, int a) {
    int u = d * P->N + a;
    if (l == 0) return P->remap[u] >= 0;
    return u < P->units[l];
}

static void build_hierarchy(orc_mas* P, const int* rp, const int* ci, int max_levels) {
    int V = P->V, N = P->N;
    P->sn[0] = (int*)malloc((size_t)V * sizeof(int));
    for (int i = 0; i < V; ++i) P->sn[0][i] = P->map[i];
    P->units[0] = P->M * N;
    P->ndom[0] = P->M;
    int occupied = V; /* number of occupied units at the current level */
    int l = 0;
    for (;;) {
        if (P->ndom[l] == 1) break;
        if (max_levels > 0 && l + 1 >= max_levels) break;
        if (l + 1 >= ORC_MAX_LEVELS) break;
        int U = P->units[l];
        int* par = (int*)malloc((size_t)U * sizeof(int));
        for (int u = 0; u < U; ++u) par[u] = u;
        const int* sl = P->sn[l];
        for (int i = 0; i < V; ++i)
            for (int p = rp[i]; p < rp[i + 1]; ++p) {
                int j = ci[p];
                if (j == i) continue;
                int s = sl[i], t = sl[j];
                if (s == t || s / N != t / N) continue;
                int rs = find_root(par, s), rt = find_root(par, t);
                if (rs != rt) {
                    if (rs < rt) par[rt] = rs;
                    else par[rs] = rt;
                }
            }
        /* number components by lowest lane, domains in order */
        int* id = (int*)malloc((size_t)U * sizeof(int));
        for (int u = 0; u < U; ++u) id[u] = -1;
        int next = 0;
        for (int d = 0; d < P->ndom[l]; ++d)
            for (int a = 0; a < N; ++a) {
                if (!lane_occupied(P, l, d, a)) continue;
                int r = find_root(par, d * N + a);
                if (id[r] < 0) id[r] = next++;
            }
        if (next == occupied) { /* nothing merged anywhere */
            free(par);
            free(id);
            break;
        }
        P->sn[l + 1] = (int*)malloc((size_t)V * sizeof(int));
        for (int i = 0; i < V; ++i) P->sn[l + 1][i] = id[find_root(par, sl[i])];
        P->units[l + 1] = next;
        P->ndom[l + 1] = (next + N - 1) / N;
        occupied = next;
        free(par);
        free(id);
        ++l;
    }
    P->L = l + 1;
}

static void build_domain_matrices(orc_mas* P, const int* rp, const int* ci, const double* val) {
    int V = P->V, N = P->N, n3 = 3 * N;
    for (int l = 0; l < P->L; ++l) {
        size_t sz = (size_t)P->ndom[l] * n3 * n3;
        double* K = (double*)calloc(sz, sizeof(double));
        const int* sl = P->sn[l];
        for (int i = 0; i < V; ++i)
            for (int p = rp[i]; p < rp[i + 1]; ++p) {
                int j = ci[p];
                int s = sl[i], t = sl[j];
                if (s / N != t / N) continue;
                int d = s / N, a = s - d * N, b = t - d * N;
                double* Kd = K + (size_t)d * n3 * n3;
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) Kd[(3 * a + r) * n3 + (3 * b + c)] += val[(size_t)p * 9 + 3 * r + c];
            }
        for (int d = 0; d < P->ndom[l]; ++d) { /* upper scalar triangle -> lower */
            double* Kd = K + (size_t)d * n3 * n3;
            for (int r = 0; r < n3; ++r)
                for (int c = r + 1; c < n3; ++c) Kd[c * n3 + r] = Kd[r * n3 + c];
        }
        P->K[l] = K;
    }
}

/* Inverse of the occupied principal submatrix via Cholesky. */
static int invert_domain(const orc_mas* P, int l, int d, const double* K, double* Inv) {
    int N = P->N, n3 = 3 * N;
    int* occ = (int*)malloc((size_t)n3 * sizeof(int));
    int m = 0;
    for (int a = 0; a < N; ++a)
        if (lane_occupied(P, l, d, a))
            for (int c = 0; c < 3; ++c) occ[m++] = 3 * a + c;
    double* A = (double*)malloc((size_t)m * m * sizeof(double) + 1);
    double* Lf = (double*)calloc((size_t)m * m + 1, sizeof(double));
    double* W = (double*)calloc((size_t)m * m + 1, sizeof(double));
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) A[i * m + j] = K[occ[i] * n3 + occ[j]];
    int status = ORC_OK;
    for (int j = 0; j < m && status == ORC_OK; ++j) {
        double s = A[j * m + j];
        for (int k = 0; k < j; ++k) s -= Lf[j * m + k] * Lf[j * m + k];
        if (!(s > 0.0)) {
            status = ORC_NOT_SPD;
            break;
        }
        Lf[j * m + j] = sqrt(s);
        for (int i = j + 1; i < m; ++i) {
            double t = A[i * m + j];
            for (int k = 0; k < j; ++k) t -= Lf[i * m + k] * Lf[j * m + k];
            Lf[i * m + j] = t / Lf[j * m + j];
        }
    }
    memset(Inv, 0, (size_t)n3 * n3 * sizeof(double));
    if (status == ORC_OK) {
        for (int j = 0; j < m; ++j) { /* W = L^-1 by forward substitution */
            W[j * m + j] = 1.0 / Lf[j * m + j];
            for (int i = j + 1; i < m; ++i) {
                double t = 0.0;
                for (int k = j; k < i; ++k) t += Lf[i * m + k] * W[k * m + j];
                W[i * m + j] = -t / Lf[i * m + i];
            }
        }
        for (int p = 0; p < m; ++p) /* Inv = W^T W, upper then mirrored */
            for (int q = p; q < m; ++q) {
                double t = 0.0;
                for (int k = q; k < m; ++k) t += W[k * m + p] * W[k * m + q];
                Inv[occ[p] * n3 + occ[q]] = t;
                Inv[occ[q] * n3 + occ[p]] = t;
            }
    }
    free(occ);
    free(A);
    free(Lf);
    free(W);
    return status;
}

static orc_mas* mas_alloc(int V, int N, int M) {
    orc_mas* P = (orc_mas*)calloc(1, sizeof(orc_mas));
    P->V = V;
    P->N = N;
    P->M = M;
    P->map = (int*)malloc((size_t)V * sizeof(int));
    P->remap = (int*)malloc((size_t)M * N * sizeof(int));
    return P;
}

orc_mas* orc_mas_build_parts(int V, const int* rp, const int* ci, const double* val, const int* part, int M,
                             int N, int max_levels, int* status) {
    if (V <= 0 || N <= 0 || M <= 0) {
        *status = ORC_INVALID;
        return NULL;
    }
    orc_mas* P = mas_alloc(V, N, M);
    if (orc_slots(V, part, M, N, P->map, P->remap) != ORC_OK) {
        orc_mas_free(P);
        *status = ORC_INVALID;
        return NULL;
    }
    build_hierarchy(P, rp, ci, max_levels);
    build_domain_matrices(P, rp, ci, val);
    int n3 = 3 * N;
    *status = ORC_OK;
    for (int l = 0; l < P->L; ++l) {
        P->Inv[l] = (double*)calloc((size_t)P->ndom[l] * n3 * n3, sizeof(double));
        for (int d = 0; d < P->ndom[l]; ++d) {
            int s = invert_domain(P, l, d, P->K[l] + (size_t)d * n3 * n3, P->Inv[l] + (size_t)d * n3 * n3);
            if (s != ORC_OK) *status = s;
        }
    }
    return P;
}

orc_mas* orc_mas_build(int V, const int* rp, const int* ci, const double* val, const int* gptr, const int* gadj,
                       int N, int max_levels, int* status) {
    int* part = (int*)malloc((size_t)(V > 0 ? V : 1) * sizeof(int));
    int M = 0, No = 0, s;
    if (gptr && gadj) s = orc_partition(V, gptr, gadj, N, part, &M, &No);
    else s = orc_partition(V, rp, ci, N, part, &M, &No); /* the pattern of H as the graph */
    if (s != ORC_OK) {
        free(part);
        *status = s;
        return NULL;
    }
    orc_mas* P = orc_mas_build_parts(V, rp, ci, val, part, M, N, max_levels, status);
    if (P) P->No = No;
    free(part);
    return P;
}

void orc_mas_free(orc_mas* P) {
    if (!P) return;
    for (int l = 0; l < ORC_MAX_LEVELS; ++l) {
        free(P->sn[l]);
        free(P->K[l]);
        free(P->Inv[l]);
    }
    free(P->map);
    free(P->remap);
    free(P);
}

int orc_mas_levels(const orc_mas* P) { return P->L; }
int orc_mas_parts(const orc_mas* P) { return P->M; }
int orc_mas_slack(const orc_mas* P) { return P->No; }
int orc_mas_units(const orc_mas* P, int l) { return (l >= 0 && l < P->L) ? P->units[l] : 0; }
int orc_mas_domains(const orc_mas* P, int l) { return (l >= 0 && l < P->L) ? P->ndom[l] : 0; }

void orc_mas_get_map(const orc_mas* P, int* map, int* remap) {
    memcpy(map, P->map, (size_t)P->V * sizeof(int));
    memcpy(remap, P->remap, (size_t)P->M * P->N * sizeof(int));
}

void orc_mas_get_sn(const orc_mas* P, int l, int* sn) { memcpy(sn, P->sn[l], (size_t)P->V * sizeof(int)); }

void orc_mas_get_domain_matrix(const orc_mas* P, int l, int d, double* K) {
    size_t n2 = (size_t)9 * P->N * P->N;
    memcpy(K, P->K[l] + (size_t)d * n2, n2 * sizeof(double));
}

void orc_mas_get_inverse(const orc_mas* P, int l, int d, double* Inv) {
    size_t n2 = (size_t)9 * P->N * P->N;
    memcpy(Inv, P->Inv[l] + (size_t)d * n2, n2 * sizeof(double));
}

/* Rounding-level perturbation of the preconditioner, for deriving how far two
 * correct FP64 implementations of the same MAS operator may drift apart in
 * their PCG iteration counts (test infrastructure, no part of the method).
 * Every stored inverse entry (p <= q) of every level and domain is scaled by
 * (1 + eps * u) with u uniform in [-1, 1), and mirrored, so each inverse
 * stays exactly symmetric.  u comes from SplitMix64 (Steele, Lea and Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014) evaluated
 * at counter (seed, running entry index): state = seed + (index + 1) * gamma
 * with gamma = 0x9e3779b97f4a7c15, then the published 64-bit finaliser. */
static unsigned long long splitmix64_at(unsigned long long seed, unsigned long long index) {
    unsigned long long z = seed + (index + 1ULL) * 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

void orc_mas_perturb(orc_mas* P, double eps, unsigned long long seed) {
    int n3 = 3 * P->N;
    unsigned long long idx = 0;
    for (int l = 0; l < P->L; ++l)
        for (int d = 0; d < P->ndom[l]; ++d) {
            double* A = P->Inv[l] + (size_t)d * n3 * n3;
            for (int p = 0; p < n3; ++p)
                for (int q = p; q < n3; ++q) {
                    /* top 53 bits -> [0, 1) -> [-1, 1) */
                    double u = (double)(splitmix64_at(seed, idx++) >> 11) * (1.0 / 9007199254740992.0);
                    double v = A[p * n3 + q] * (1.0 + eps * (2.0 * u - 1.0));
                    A[p * n3 + q] = v;
                    A[q * n3 + p] = v;
                }
        }
}

/* ------------------------------------------------------------------------ */
/* MAS apply (Supp. Eq. 4-6)                                                */
/* ------------------------------------------------------------------------ */

void orc_mas_apply(const orc_mas* P, const double* r, double* z) {
    int V = P->V, N = P->N, n3 = 3 * N;
    for (int i = 0; i < 3 * V; ++i) z[i] = 0.0;
    for (int l = 0; l < P->L; ++l) {
        size_t len = (size_t)P->ndom[l] * N * 3;
        double* rl = (double*)calloc(len, sizeof(double));
        double* yl = (double*)calloc(len, sizeof(double));
        const int* sl = P->sn[l];
        for (int i = 0; i < V; ++i) /* restriction: C_l r */
            for (int c = 0; c < 3; ++c) rl[(size_t)3 * sl[i] + c] += r[3 * i + c];
        for (int d = 0; d < P->ndom[l]; ++d) { /* blockdiag_d(Inv) */
            const double* A = P->Inv[l] + (size_t)d * n3 * n3;
            const double* x = rl + (size_t)d * n3;
            double* y = yl + (size_t)d * n3;
            for (int p = 0; p < n3; ++p) {
                double t = 0.0;
                for (int q = 0; q < n3; ++q) t += A[p * n3 + q] * x[q];
                y[p] = t;
            }
        }
        for (int i = 0; i < V; ++i) /* prolongation: C_l^T y, levels summed */
            for (int c = 0; c < 3; ++c) z[3 * i + c] += yl[(size_t)3 * sl[i] + c];
        free(rl);
        free(yl);
    }
}

/* ------------------------------------------------------------------------ */
/* SpMV, PCG, adjoint scatter                                               */
/* ------------------------------------------------------------------------ */

void orc_spmv(int n, const int* rp, const int* ci, const double* val, const double* x, double* y) {
    for (int i = 0; i < n; ++i) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            const double* B = val + (size_t)p * 9;
            const double* xj = x + 3 * ci[p];
            a0 += B[0] * xj[0] + B[1] * xj[1] + B[2] * xj[2];
            a1 += B[3] * xj[0] + B[4] * xj[1] + B[5] * xj[2];
            a2 += B[6] * xj[0] + B[7] * xj[1] + B[8] * xj[2];
        }
        y[3 * i] = a0;
        y[3 * i + 1] = a1;
        y[3 * i + 2] = a2;
    }
}

static double dot_seq(int m, const double* a, const double* b) {
    double s = 0.0;
    for (int i = 0; i < m; ++i) s += a[i] * b[i];
    return s;
}

/* Compensated dot product, algorithm Dot2 of Ogita, Rump and Oishi
 * ("Accurate sum and dot product", SIAM J. Sci. Comput. 26(6), 2005): the
 * result is as accurate as if the sum were accumulated in twice the working
 * precision and rounded once.  Error-free transformations: TwoProduct with an
 * explicit fused multiply-add, TwoSum by Knuth's branch-free form. */
static double dot_comp(int m, const double* a, const double* b) {
    double s = 0.0, c = 0.0;
    for (int i = 0; i < m; ++i) {
        double p = a[i] * b[i];
        double ep = fma(a[i], b[i], -p);
        double t = s + p;
        double z = t - s;
        double es = (s - (t - z)) + (p - z);
        s = t;
        c += es + ep;
    }
    return s + c;
}

double orc_dot(int m, const double* a, const double* b, int dot_mode) {
    return dot_mode == ORC_DOT_COMPENSATED ? dot_comp(m, a, b) : dot_seq(m, a, b);
}

int orc_pcg(int n, const int* rp, const int* ci, const double* val, const orc_mas* P, const double* b, double* x,
            double tol, int max_iter, int* iters, double* relres, double* true_relres) {
    return orc_pcg_dots(n, rp, ci, val, P, b, x, tol, max_iter, ORC_DOT_SEQUENTIAL, iters, relres, true_relres);
}

int orc_pcg_dots(int n, const int* rp, const int* ci, const double* val, const orc_mas* P, const double* b,
                 double* x, double tol, int max_iter, int dot_mode, int* iters, double* relres, double* true_relres) {
#define dot(m_, a_, b_) orc_dot((m_), (a_), (b_), dot_mode)
    int m = 3 * n;
    for (int i = 0; i < m; ++i) x[i] = 0.0;
    *iters = 0;
    double bn = sqrt(dot(m, b, b));
    if (bn == 0.0) {
        *relres = 0.0;
        *true_relres = 0.0;
        return ORC_OK;
    }
    double* r = (double*)malloc((size_t)m * sizeof(double));
    double* z = (double*)malloc((size_t)m * sizeof(double));
    double* p = (double*)malloc((size_t)m * sizeof(double));
    double* q = (double*)malloc((size_t)m * sizeof(double));
    memcpy(r, b, (size_t)m * sizeof(double));
    orc_mas_apply(P, r, z);
    memcpy(p, z, (size_t)m * sizeof(double));
    double rho = dot(m, r, z);
    int status = ORC_NOT_CONVERGED;
    double rn = bn;
    for (int k = 1; k <= max_iter; ++k) {
        orc_spmv(n, rp, ci, val, p, q);
        double sigma = dot(m, p, q);
        if (!(sigma > 0.0)) {
            status = ORC_NOT_SPD;
            break;
        }
        double alpha = rho / sigma;
        for (int i = 0; i < m; ++i) x[i] += alpha * p[i];
        for (int i = 0; i < m; ++i) r[i] -= alpha * q[i];
        *iters = k;
        rn = sqrt(dot(m, r, r));
        if (rn <= tol * bn) {
            status = ORC_OK;
            break;
        }
        orc_mas_apply(P, r, z);
        double rho_new = dot(m, r, z);
        double beta = rho_new / rho;
        for (int i = 0; i < m; ++i) p[i] = z[i] + beta * p[i];
        rho = rho_new;
    }
    *relres = rn / bn;
    orc_spmv(n, rp, ci, val, x, q);
    for (int i = 0; i < m; ++i) q[i] = b[i] - q[i];
    *true_relres = sqrt(dot(m, q, q)) / bn;
    free(r);
    free(z);
    free(p);
    free(q);
    return status;
#undef dot
}

/* dL/dH_ij = -lambda_i x_j^T on every stored block (from dx = -H^-1 dH x). */
void orc_adjoint_scatter(int n, const int* rp, const int* ci, const double* lambda, const double* x, double* dLdH) {
    for (int i = 0; i < n; ++i)
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            int j = ci[p];
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) dLdH[(size_t)p * 9 + 3 * r + c] = -lambda[3 * i + r] * x[3 * j + c];
        }
}

/* ------------------------------------------------------------- assembly */

typedef struct {
    int row, col;
    long idx;
} orc_entry;

static int orc_entry_cmp(const void* a, const void* b) {
    const orc_entry* x = (const orc_entry*)a;
    const orc_entry* y = (const orc_entry*)b;
    if (x->row != y->row) return x->row < y->row ? -1 : 1;
    if (x->col != y->col) return x->col < y->col ? -1 : 1;
    if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
    return 0;
}

long orc_assemble(int n, long n_in, const int* rows, const int* cols, const double* blocks, int* row_ptr,
                  int* col_idx, double* val) {
    for (long k = 0; k < n_in; ++k)
        if (rows[k] < 0 || rows[k] >= n || cols[k] < 0 || cols[k] >= n) return -1;
    orc_entry* e = (orc_entry*)malloc(sizeof(orc_entry) * (size_t)(n_in > 0 ? n_in : 1));
    for (long k = 0; k < n_in; ++k) {
        e[k].row = rows[k];
        e[k].col = cols[k];
        e[k].idx = k;
    }
    /* order by (row, col, position in the list): equal blocks meet in list order */
    qsort(e, (size_t)n_in, sizeof(orc_entry), orc_entry_cmp);
    long nb = 0;
    for (int i = 0; i <= n; ++i) row_ptr[i] = 0;
    for (long k = 0; k < n_in; ++k) {
        if (k == 0 || e[k].row != e[k - 1].row || e[k].col != e[k - 1].col) {
            col_idx[nb] = e[k].col;
            for (int c = 0; c < 9; ++c) val[9 * nb + c] = 0.0;
            row_ptr[e[k].row + 1]++;
            ++nb;
        }
        for (int c = 0; c < 9; ++c) val[9 * (nb - 1) + c] += blocks[9 * e[k].idx + c];
    }
    for (int i = 0; i < n; ++i) row_ptr[i + 1] += row_ptr[i];
    free(e);
    return nb;
}

/* Contact Hessian blocks on affine bodies in DOF-block coordinates, the plain
 * definition behind the two-level reduction of Sec. 6.1: listed block C_k
 * between contact nodes r_k and c_k contributes J_r^T C_k J_c, where a node
 * of an affine body (is_body) has J = [I | xbar1 I | xbar2 I | xbar3 I]
 * (x = t + A xbar; its body's 12 DOFs are block rows row .. row + 3) and a
 * mesh node has J = I (block row row).  Sub-block (a, b) of the product is
 * (w_a(r) w_b(c)) C_k with w = (1, xbar1, xbar2, xbar3).  Writes the
 * sub-blocks of every listed block in list order, (a, b) row-major, and
 * returns their number, or -1 for a node index out of range. */
long orc_abd_expand(int n_nodes, const int* node_row, const int* is_body, const double* xbar, long m, const int* r,
                    const int* c, const double* C, int* out_rows, int* out_cols, double* out_blocks) {
    long o = 0;
    for (long k = 0; k < m; ++k) {
        if (r[k] < 0 || r[k] >= n_nodes || c[k] < 0 || c[k] >= n_nodes) return -1;
        const int nr = is_body[r[k]] ? 4 : 1, nc = is_body[c[k]] ? 4 : 1;
        for (int a = 0; a < nr; ++a)
            for (int b = 0; b < nc; ++b) {
                const double wa = a == 0 ? 1.0 : xbar[3L * r[k] + a - 1];
                const double wb = b == 0 ? 1.0 : xbar[3L * c[k] + b - 1];
                const double w = wa * wb;
                out_rows[o] = node_row[r[k]] + a;
                out_cols[o] = node_row[c[k]] + b;
                for (int e = 0; e < 9; ++e) out_blocks[9 * o + e] = w * C[9 * k + e];
                ++o;
            }
    }
    return o;
}
