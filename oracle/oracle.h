/*
 * CPU oracle for the connectivity-enhanced MAS-preconditioned PCG solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain single-threaded C, FP64 throughout, every
 * loop in ascending index order, built without FMA contraction.  Only the
 * test-suite, the smoke check and the benchmark's CPU-baseline leg may load
 * this library.  It shares no code, header, table or helper with the HIP
 * library it checks.
 *
 * What it computes (StiffGIPC, arXiv 2411.06224):
 *   - partition of the node graph into M = ceil(V / (N - N_o)) parts of at
 *     most N nodes, smallest slack N_o first (Sec. 4.2, Eq. num_subdomains);
 *     METIS is replaced by a specified recursive BFS bisection (see below);
 *   - map / remap with -1 padding, one part per level-0 domain (Sec. 4.2,
 *     Fig. mapping; Supp. Alg. 1 map/remap construction);
 *   - the supernode hierarchy: connected components inside each domain,
 *     numbered by their lowest lane, N consecutive supernodes per coarser
 *     domain (Sec. 4.1 case study, Supp. Alg. 2-5 semantics);
 *   - per level and domain the matrix S_d C_l H C_l^T S_d^T and its inverse
 *     over occupied lanes (Alg. "Compute MAS preconditioner"; Supp. Eq. 5);
 *   - the MAS operator  z = sum_l C_l^T blockdiag_d(Inv_{l,d}) C_l r
 *     (Supp. Eq. 4-6);
 *   - 3x3-block CSR SpMV, textbook PCG (Sec. 3.2 "IP Minimization and Linear
 *     Solves": P d = -grad E solved by PCG) and the adjoint block scatter
 *     dL/dH_ij = -lambda_i x_j^T;
 *   - assembly of a list of 3x3 blocks into BCSR, equal (row, col) blocks
 *     summed in list order (what the hash-based reduction of Sec. 6.2
 *     produces).
 *
 * Conventions.  H is 3x3-block CSR: row_ptr[n+1], col_idx[nnzb] ascending per
 * row, val[nnzb*9] row-major blocks; both triangles stored.  Vectors are
 * 3n doubles, node-major.  Domain matrices are (3N)x(3N) row-major with
 * lane-major, component-minor scalar index 3*lane + c.
 */
#ifndef MAS_ORACLE_H
#define MAS_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_INVALID (-1)
#define ORC_NOT_SPD (-2)
#define ORC_MAX_LEVELS 16

/* Recursive BFS bisection partition (the METIS replacement), with the slack
 * search of Eq. num_subdomains.  part[V] receives part ids in emission order. */
int orc_partition(int V, const int* gptr, const int* gadj, int N, int* part, int* M_out, int* No_out);

/* Node k (ascending id) of part p goes to slot p*N + k.  remap[M*N]. */
int orc_slots(int V, const int* part, int M, int N, int* map, int* remap);

typedef struct orc_mas orc_mas;

/* Full build: partition (graph NULL = off-diagonal pattern of H), slots,
 * hierarchy, domain matrices, inverses.  max_levels <= 0 means unlimited. */
orc_mas* orc_mas_build(int V, const int* rp, const int* ci, const double* val, const int* gptr,
                       const int* gadj, int N, int max_levels, int* status);
/* Same from a given partition part[V] into M parts (each of <= N nodes). */
orc_mas* orc_mas_build_parts(int V, const int* rp, const int* ci, const double* val, const int* part,
                             int M, int N, int max_levels, int* status);
void orc_mas_free(orc_mas* P);

int orc_mas_levels(const orc_mas* P);
int orc_mas_parts(const orc_mas* P);
int orc_mas_slack(const orc_mas* P);
int orc_mas_units(const orc_mas* P, int l);   /* level 0: M*N slots; l >= 1: S_l */
int orc_mas_domains(const orc_mas* P, int l);
void orc_mas_get_map(const orc_mas* P, int* map, int* remap);
void orc_mas_get_sn(const orc_mas* P, int l, int* sn); /* sn[V]: unit of each node */
void orc_mas_get_domain_matrix(const orc_mas* P, int l, int d, double* K);
void orc_mas_get_inverse(const orc_mas* P, int l, int d, double* Inv);

/* Test infrastructure: scales every inverse entry (p <= q, mirrored) by
 * (1 + eps u), u uniform in [-1, 1) from SplitMix64 at (seed, entry index).
 * Used only to measure how PCG iteration counts spread under rounding-level
 * changes of the preconditioner; eps = 0 leaves the inverses unchanged. */
void orc_mas_perturb(orc_mas* P, double eps, unsigned long long seed);
void orc_mas_apply(const orc_mas* P, const double* r, double* z);
void orc_spmv(int n, const int* rp, const int* ci, const double* val, const double* x, double* y);
int orc_pcg(int n, const int* rp, const int* ci, const double* val, const orc_mas* P, const double* b,
            double* x, double tol, int max_iter, int* iters, double* relres, double* true_relres);
/* Dot products of orc_pcg_dots: ORC_DOT_SEQUENTIAL sums the products in
 * ascending order in working precision (what orc_pcg does);
 * ORC_DOT_COMPENSATED uses the compensated algorithm Dot2 (Ogita, Rump and
 * Oishi 2005), as accurate as a sum in twice the working precision.  Both are
 * evaluations of the same definition; PCG iteration counts depend on which. */
#define ORC_DOT_SEQUENTIAL 0
#define ORC_DOT_COMPENSATED 1
double orc_dot(int m, const double* a, const double* b, int dot_mode);
int orc_pcg_dots(int n, const int* rp, const int* ci, const double* val, const orc_mas* P, const double* b,
                 double* x, double tol, int max_iter, int dot_mode, int* iters, double* relres, double* true_relres);
void orc_adjoint_scatter(int n, const int* rp, const int* ci, const double* lambda, const double* x,
                         double* dLdH);

/* Assembly of 3x3 blocks given as a list (row[k], col[k], blocks[9k..9k+8],
 * row-major) into BCSR (the hash-based reduction of Sec. 6.2 computes the
 * same sums): blocks with the same (row, col) are added in list order, rows
 * ascending, columns ascending within a row.  row_ptr[n+1]; col_idx and val
 * hold up to n_in blocks.  Returns the number of distinct blocks, or -1 if
 * an index is out of range. */
long orc_assemble(int n, long n_in, const int* rows, const int* cols, const double* blocks, int* row_ptr,
                  int* col_idx, double* val);

/* Contact blocks on affine bodies in DOF-block coordinates (Sec. 6.1):
 * every listed block's J_r^T C J_c sub-blocks, in list order. */
long orc_abd_expand(int n_nodes, const int* node_row, const int* is_body, const double* xbar, long m, const int* r,
                    const int* c, const double* C, int* out_rows, int* out_cols, double* out_blocks);

#ifdef __cplusplus
}
#endif
#endif
