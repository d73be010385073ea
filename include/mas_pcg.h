/*
 * mas_pcg.h -- C ABI of the MI355X MAS-preconditioned PCG library
 * (libmaspcg.so).
 *
 * The library solves the SPD Newton system  H dx = -grad E  of an IPC
 * time step (StiffGIPC, arXiv 2411.06224, Sec. 3.2 "IP Minimization and
 * Linear Solves": P(u) d = -grad E(u) with P symmetric positive definite) by
 * preconditioned conjugate gradients, preconditioned with the
 * connectivity-enhanced multilevel additive Schwarz (MAS) operator
 *
 *     M^-1 = sum_l C_l^T blockdiag_d( (S_d C_l H C_l^T S_d^T)^-1 ) C_l
 *
 * (Supp. Eq. 4-6; domains from a connectivity-aware partition with padding,
 * Sec. 4.2 and Fig. mapping; coarse levels from connected components inside
 * each domain, Sec. 4.1 and Supp. Alg. 2-5; per-domain matrices from the
 * algorithm "Compute MAS preconditioner" and inverted over unpadded lanes).
 *
 * Conventions
 *  - H is 3x3-block CSR (the block rows/columns of the paper's matrix AG):
 *    row_ptr[n_rows+1] and col_idx[nnzb] are int32 with columns ascending in
 *    each row; val holds nnzb row-major 3x3 blocks (9 values each).  Both
 *    triangles are stored, every row holds its diagonal block, and H must be
 *    symmetric (val(j,i) = val(i,j)^T).  One block row per mesh node.
 *  - Vectors are 3*n_rows doubles, node-major (x[3*i + c]).
 *  - "device" pointers are HIP device memory on the current device; "host"
 *    pointers are ordinary CPU memory.  The library never frees or keeps
 *    ownership of caller memory.  All device memory the library needs comes
 *    from the caller's workspace (see mas_workspace_size); the library itself
 *    allocates only small pinned host buffers inside the handle.
 *  - stream is a hipStream_t passed as void* (NULL = the null stream).  Work
 *    is enqueued on that stream; calls that report results (mas_build,
 *    pcg_solve, pcg_adjoint) synchronise it before returning.
 *  - Every call returns a mas_status; no call throws or aborts.
 *  - Thread safety: a handle may be used by one stream at a time.
 */
#ifndef MAS_PCG_H
#define MAS_PCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
typedef enum {
    MAS_OK = 0,
    MAS_NOT_CONVERGED = 1,       /* max_iter reached; outputs hold the last iterate */
    MAS_INVALID_ARG = -1,        /* bad size, pointer, option or pattern */
    MAS_NOT_SPD = -2,            /* a domain pivot <= 0, or p^T H p <= 0 in PCG */
    MAS_HIP_ERROR = -3,          /* a HIP runtime call failed */
    MAS_WORKSPACE_TOO_SMALL = -4,/* ws_bytes < mas_workspace_size() */
    MAS_NOT_READY = -5,          /* call order: analyze -> build -> apply/solve */
    MAS_NOT_FINITE = -6          /* NaN/Inf met in a residual norm */
} mas_status;

/* Value types of a BCSR matrix. */
enum { MAS_F64 = 0, MAS_F32 = 1 };

/* Solver precision modes. */
enum {
    MAS_PRECISION_F64 = 0,   /* everything FP64 */
    MAS_PRECISION_MIXED = 1  /* H values and domain inverses stored and applied in FP32;
                                domain inversion, dot products, alpha/beta and the x/r
                                updates in FP64; FP64 residual replacement */
};

#define MAS_MAX_LEVELS 16
/* The batched inversion keeps a domain's 3N x 3N FP64 matrix, padded to
 * 16 x 16 tiles, in one workgroup's LDS (160 KB per CU): 3N <= 128, so
 * N <= 42; 40 is the largest size the tests cover.  The paper's N = 16
 * (Sec. 4.2) is the default; 64 would need a 192 x 192 matrix (288 KB). */
#define MAS_MAX_DOMAIN_SIZE 40

/* A 3x3-block CSR matrix in device memory (layout above). */
typedef struct {
    int32_t n_rows;          /* number of block rows (nodes) */
    int32_t nnzb;            /* number of stored 3x3 blocks */
    const int32_t* row_ptr;  /* device, n_rows + 1 */
    const int32_t* col_idx;  /* device, nnzb */
    const void* val;         /* device, nnzb * 9 values of type dtype */
    int32_t dtype;           /* MAS_F64 or MAS_F32 */
} mas_bcsr;

typedef struct {
    int32_t domain_size;     /* N: nodes per level-0 domain, 1..MAS_MAX_DOMAIN_SIZE (paper: 16) */
    int32_t max_levels;      /* <= 0: build levels until one domain or no merge */
    int32_t precision;       /* MAS_PRECISION_F64 or MAS_PRECISION_MIXED */
    int32_t reserved;        /* must be 0 */
} mas_options;

typedef struct {
    double tol;              /* stop when ||r||_2 <= tol * ||b||_2 */
    int32_t max_iter;        /* >= 0 */
    int32_t x0_given;        /* 1: x holds the initial guess, else x0 = 0 */
    int32_t replace_every;   /* period of the iterations that restrict the residual itself rather
                                than updating its coarse restriction by recurrence, and in mixed
                                mode of the FP64 residual replacement (0 -> 50) */
    int32_t check_every;     /* iterations between host convergence checks (0 -> 8) */
} pcg_options;

typedef struct {
    int32_t status;          /* same as the return value */
    int32_t iterations;      /* CG iterations performed */
    double rel_residual;     /* ||r||/||b|| of the recurrence at exit */
    double true_rel_residual;/* ||b - H x||/||b|| recomputed with FP64 H */
} pcg_result;

/* Static description of an analysed handle (host copy). */
typedef struct {
    int32_t n_rows, nnzb, domain_size, parts, slack, levels;
    int32_t units[MAS_MAX_LEVELS];    /* level 0: parts*domain_size slots; l >= 1: supernodes */
    int32_t domains[MAS_MAX_LEVELS];  /* domains per level */
    int32_t coarse_nnzb[MAS_MAX_LEVELS]; /* stored blocks of the level-l coarse matrix (l >= 1) */
    int64_t workspace_bytes;
    int64_t inverse_bytes;            /* bytes of domain inverses (all levels, as stored) */
    int32_t stored_blocks;            /* blocks of H the solver keeps in domain order: fewer than
                                         nnzb when each pair of blocks inside a work group of
                                         domains is stored once (symmetric storage) */
    int32_t reserved;
} mas_info;

typedef struct mas_handle mas_handle;

/* Creates an empty handle.  opts may be NULL (N = 16, all levels, FP64).
 * Errors: MAS_INVALID_ARG for out-of-range options. */
int mas_create(const mas_options* opts, mas_handle** out);

/* Frees the handle and its pinned host buffers (never the workspace). */
void mas_destroy(mas_handle* h);

/* Symbolic phase, on the host, once per sparsity pattern (the paper runs its
 * METIS reordering once at load, Sec. 4.2): partition of the node graph into
 * M = ceil(V/(N - N_o)) parts of at most N nodes with the smallest slack N_o
 * (Eq. num_subdomains), map/remap with -1 padding, supernode hierarchy from
 * the block pattern of H (contact couplings included), and every gather /
 * reduction plan the device phases use.  When contacts later change the
 * pattern, mas_replan derives the plans again on the device under this
 * partition.
 *   row_ptr, col_idx: host copies of H's pattern (conventions above).
 *   g_ptr, g_adj: host CSR node graph to partition (e.g. mesh edges); both
 *                 NULL = the off-diagonal pattern of H.  Self loops and
 *                 duplicates are ignored; the graph is symmetrised.
 * Errors: MAS_INVALID_ARG (sizes, unsorted or out-of-range columns, missing
 * diagonal block, asymmetric pattern). */
int mas_analyze(mas_handle* h, int32_t n_rows, int32_t nnzb, const int32_t* row_ptr, const int32_t* col_idx,
                const int32_t* g_ptr, const int32_t* g_adj);

/* mas_analyze with a caller-given level-0 partition instead of the
 * connectivity-aware bisection, e.g. consecutive nodes in Morton (Z-order)
 * of their positions, the domain ordering of the earlier MAS preconditioner
 * that Sec. 4.1 compares against.  part[n_rows] (host) puts node i in
 * level-0 domain part[i], 0 <= part[i] < n_parts; every domain must hold
 * 1..domain_size nodes.  Slots, hierarchy and plans then follow as in
 * mas_analyze (slack reported as 0).
 * Errors: MAS_INVALID_ARG (as mas_analyze, plus a part id out of range, an
 * empty part or one with more than domain_size nodes). */
int mas_analyze_partition(mas_handle* h, int32_t n_rows, int32_t nnzb, const int32_t* row_ptr,
                          const int32_t* col_idx, const int32_t* part, int32_t n_parts);

/* Device bytes of the scratch abd_contact_blocks needs. */
size_t abd_contact_workspace_size(int32_t n_nodes, int64_t m);

/* Contact Hessian blocks on affine bodies mapped to the system's DOF blocks
 * with the two-level reduction of Sec. 6.1 ("Two-Level Reduction for ABD
 * Hessian Assembly"; sub-block decomposition of Sec. 6.2).  A contact node
 * i either belongs to an affine body (node_is_body[i] != 0), whose 12 DOFs
 * [t, a1, a2, a3] are the four block rows node_row[i] .. node_row[i] + 3 and
 * which moves the node as x = t + A xbar_i (xbar_i = node_xbar[3i..3i+2],
 * the rest position in the body frame), or is a node of the deformable mesh
 * with block row node_row[i].  Block C_k couples nodes r[k] (rows) and c[k]
 * (columns) and contributes J_r^T C_k J_c with J = [I | xbar1 I | xbar2 I |
 * xbar3 I] for a body node and J = I for a mesh node, i.e. the 3x3
 * sub-blocks (a, b) = (w_a(r) w_b(c)) C_k with w = (1, xbar1, xbar2, xbar3):
 * 16 for a body-body pair, 4 for body-mesh or mesh-body, 1 for mesh-mesh.
 *   levels = 2: the blocks of equal node pair (r, c) are first summed in
 *     list order, and each distinct pair is mapped once; levels = 1: every
 *     listed block is mapped (single-level).
 * Output: the sub-block list (rows, cols, row-major 3x3 blocks), pairs in
 * (r, c) order (levels = 2) or list order (levels = 1), sub-blocks (a, b)
 * row-major within a pair; *n_out receives their number (also when it
 * exceeds capacity).  The second level -- equal DOF blocks summed, e.g. all
 * node pairs of one body pair -- is bcsr_assemble of this list together with
 * the system's other blocks.
 *   node_row, node_is_body: device int32[n_nodes]; node_xbar: device
 *   double[3 n_nodes]; r, c: device int32[m], 0 <= index < n_nodes;
 *   C: device double[9 m]; out_rows, out_cols: device int32[capacity];
 *   out_blocks: device double[9 capacity].
 *   workspace: device scratch of ws_bytes >= abd_contact_workspace_size,
 *              256-byte aligned.
 * node_row entries are not checked here (the DOF rows they produce are, by
 * bcsr_assemble).
 * Limits: n_nodes < 2^31 - 1, 16 m < 2^31.  Synchronises the stream.
 * Errors: MAS_INVALID_ARG (an index out of range, n_out > capacity: then
 * nothing is written), MAS_WORKSPACE_TOO_SMALL, MAS_HIP_ERROR. */
int abd_contact_blocks(int32_t n_nodes, const int32_t* node_row, const int32_t* node_is_body,
                       const double* node_xbar, int64_t m, const int32_t* r, const int32_t* c, const double* C,
                       int32_t levels, int32_t* out_rows, int32_t* out_cols, double* out_blocks, int64_t capacity,
                       int64_t* n_out, void* workspace, size_t ws_bytes, void* stream);

/* Device bytes of the scratch mas_morton_partition needs for n_rows nodes. */
size_t mas_morton_workspace_size(int32_t n_rows);

/* Level-0 domains of domain_size consecutive nodes in Morton (Z-order) of
 * the node positions: the domain ordering of the earlier MAS preconditioner
 * that the connectivity-aware partition replaces (Sec. 4.1), for
 * mas_analyze_partition.  Each coordinate is scaled to 21 bits over the
 * bounding box, ((x - lo) / extent) * (2^21 - 1) rounded down (extent at
 * least the smallest positive double), and the bits are interleaved x, y, z
 * (x most significant) into a 63-bit code; nodes are ordered by code, equal
 * codes by node id, and the k-th node goes to domain k / domain_size.
 *   positions: device, 3*n_rows doubles (node-major).
 *   part: device, n_rows int32 (output).
 *   workspace: device scratch of ws_bytes >= mas_morton_workspace_size,
 *              256-byte aligned.
 * Asynchronous.  Errors: MAS_INVALID_ARG, MAS_WORKSPACE_TOO_SMALL,
 * MAS_HIP_ERROR. */
int mas_morton_partition(int32_t n_rows, const double* positions, int32_t domain_size, int32_t* part,
                         void* workspace, size_t ws_bytes, void* stream);

/* Device bytes the handle needs (valid after mas_analyze; 0 before). */
size_t mas_workspace_size(const mas_handle* h);

/* Numeric phase on the device (algorithm "Compute MAS preconditioner"):
 * sums the coarse matrices C_l H C_l^T level by level, gathers every domain
 * matrix S_d C_l H C_l^T S_d^T and inverts it over its occupied lanes in FP64
 * (batched, LDS-resident, MFMA tiles); in mixed mode also stores FP32 copies
 * of the inverses.
 *   H: device matrix with the analysed pattern, dtype MAS_F64.
 *   workspace: device buffer of ws_bytes >= mas_workspace_size(h), 256-byte
 *              aligned, owned by the caller and kept alive while the handle
 *              is used; it holds plans, values, inverses and solver vectors.
 * Synchronises the stream.  Errors: MAS_NOT_READY (no analyze),
 * MAS_WORKSPACE_TOO_SMALL, MAS_INVALID_ARG, MAS_NOT_SPD (a domain matrix is
 * not positive definite), MAS_HIP_ERROR. */
int mas_build(mas_handle* h, const mas_bcsr* H, void* workspace, size_t ws_bytes, void* stream);

/* z = M^-1 r (Supp. Eq. 6): restrict r to every level, multiply each domain
 * by its inverse, prolong and sum over levels.  r, z: device, 3*n_rows
 * doubles, node order; may not alias.  Uses the precision chosen at create.
 * Asynchronous.  Errors: MAS_NOT_READY, MAS_INVALID_ARG, MAS_HIP_ERROR. */
int mas_apply(mas_handle* h, const double* r, double* z, void* stream);

/* y = H x for a 3x3-block CSR matrix (FP64 or FP32 values, FP64 vectors).
 * x, y: device, 3*n_rows doubles; may not alias.  Needs no handle.
 * Asynchronous.  Errors: MAS_INVALID_ARG, MAS_HIP_ERROR. */
int bcsr_spmv(const mas_bcsr* H, const double* x, double* y, void* stream);

/* Solves H x = b by PCG with the handle's MAS preconditioner.
 *   H: device, FP64, the analysed pattern.  Its current values are permuted
 *      into domain order (plus an FP32 copy in mixed mode) at the start of
 *      every call; the preconditioner is the one built by the last mas_build.
 *   b, x: device, 3*n_rows doubles (x may hold x0 when opts->x0_given).
 *   opts: NULL = tol 1e-4, max_iter 10000.  res: host, may be NULL.
 * Stops when ||r||_2 <= tol ||b||_2; in mixed mode the stop is confirmed on
 * the FP64 residual b - H x.  b = 0 gives x = 0 after 0 iterations.
 * Synchronises the stream.  Returns MAS_OK, MAS_NOT_CONVERGED (x holds the
 * last iterate), MAS_NOT_SPD, MAS_NOT_FINITE, MAS_INVALID_ARG, MAS_NOT_READY
 * or MAS_HIP_ERROR. */
int pcg_solve(mas_handle* h, const mas_bcsr* H, const double* b, double* x, const pcg_options* opts,
              pcg_result* res, void* stream);

/* Backward of x = H^-1 b for a loss L(x): solves H lambda = dL/dx with the
 * same MAS (H is symmetric, so the forward preconditioner serves the adjoint
 * system), then writes dL/db = lambda and dL/dH_ij = -lambda_i x_j^T on every
 * stored block (from dx = -H^-1 dH x).
 *   x: device, the forward solution; dLdx: device, 3*n_rows doubles.
 *   lambda: device, 3*n_rows doubles (= dL/db).
 *   dLdH: device, nnzb*9 values of type dLdH_dtype (MAS_F64 or MAS_F32), in
 *         H's block order, row-major 3x3; NULL skips the scatter.
 * Synchronises the stream.  Errors as pcg_solve. */
int pcg_adjoint(mas_handle* h, const mas_bcsr* H, const double* x, const double* dLdx, double* lambda, void* dLdH,
                int32_t dLdH_dtype, const pcg_options* opts, pcg_result* res, void* stream);

/* Device bytes of scratch bcsr_assemble needs for n_rows block rows and a
 * list of n_in blocks. */
size_t bcsr_assemble_workspace_size(int32_t n_rows, int64_t n_in);

/* Assembles a list of 3x3 blocks into 3x3-block CSR on the device: the
 * operation the hash-based parallel reduction of Sec. 6.2 performs (blocks
 * with the same (row, col) summed; rows ascending, columns ascending within
 * a row), here deterministic: a stable radix sort of (row, col) keys keeps
 * equal blocks in list order and each is summed in that order, so the
 * result is that of a sequential pass over the list.
 *   rows, cols: device int32[n_in], 0 <= index < n_rows.
 *   blocks: device double[9 n_in], row-major 3x3 blocks.
 *   row_ptr: device int32[n_rows + 1]; col_idx: device int32[capacity];
 *   val: device double[9 capacity]  (outputs, caller-owned).
 *   nnzb: host, receives the number of distinct blocks (also when it
 *         exceeds capacity, so the caller can size the outputs).
 *   workspace: device scratch of ws_bytes >= bcsr_assemble_workspace_size,
 *              256-byte aligned.
 * Limits: n_in < 2^31, n_rows < 2^31 - 1 (the sort runs over 2 ceil(log2
 * (n_rows + 1)) key bits: 34 for a 110,592-row system).  Synchronises the
 * stream.
 * Errors: MAS_INVALID_ARG (an index out of range, a limit exceeded,
 * nnzb > capacity: then col_idx and val are not written),
 * MAS_WORKSPACE_TOO_SMALL, MAS_HIP_ERROR. */
int bcsr_assemble(int32_t n_rows, int64_t n_in, const int32_t* rows, const int32_t* cols, const double* blocks,
                  int32_t* row_ptr, int32_t* col_idx, double* val, int64_t capacity, int64_t* nnzb,
                  void* workspace, size_t ws_bytes, void* stream);

/* Scratch bytes held by bcsr_assemble_noalloc on each device it runs on. */
#define MAS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* bcsr_assemble for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same operation, arguments and results, with the scratch
 * taken from a static device array of MAS_NOALLOC_SCRATCH_BYTES that each
 * device the library runs on holds from the library's load until the
 * process ends.  The call allocates no device memory (no hipMalloc or
 * hipFree, no allocating library routine); the caller still provides rows,
 * cols, blocks and the outputs.  The stream must belong to the current
 * device.  Every call on one device shares that device's array and leaves
 * its contents behind (each call clears what it needs cleared): calls that
 * overlap on one device, e.g. on two streams, race and must be serialised
 * by the caller.  Limits: as bcsr_assemble, and
 * bcsr_assemble_workspace_size(n_rows, n_in) <= MAS_NOALLOC_SCRATCH_BYTES
 * (MAS_WORKSPACE_TOO_SMALL otherwise; nothing is launched).  Synchronises
 * the stream.  Errors: as bcsr_assemble. */
int bcsr_assemble_noalloc(int32_t n_rows, int64_t n_in, const int32_t* rows, const int32_t* cols,
                          const double* blocks, int32_t* row_ptr, int32_t* col_idx, double* val, int64_t capacity,
                          int64_t* nnzb, void* stream);

/* Device bytes of scratch mas_hierarchy_device and mas_hierarchy_rebuild
 * need (after mas_analyze). */
size_t mas_hierarchy_workspace_size(const mas_handle* h);

/* The supernode hierarchy computed on the device (Supp. Alg. 2-5, with
 * 64-lane masks: per level, adjacency masks of each domain's units from the
 * slot-ordered pattern, connected components by a wave-level closure of the
 * masks, supernodes numbered by their lowest lane through a ballot and a
 * scan over domains), from the pattern and level-0 partition of the last
 * mas_analyze.  It gives the same hierarchy as the host analysis, which
 * still builds the solver's plans; the device construction is what the
 * paper repeats each Newton step when contacts change the pattern.
 *   levels, units: host, receive the level count and the units per level
 *                  (units[MAS_MAX_LEVELS]), as mas_get_info;
 *   sn: host, [levels * n_rows] unit of each node per level, as
 *       mas_get_ordering; any output may be NULL.
 *   workspace: device scratch, ws_bytes >= mas_hierarchy_workspace_size,
 *              256-byte aligned.
 * After mas_replan the pattern is the replan's (its slot-ordered copy in
 * the replan workspace).
 * Synchronises the stream.  Errors: MAS_NOT_READY, MAS_INVALID_ARG,
 * MAS_WORKSPACE_TOO_SMALL, MAS_HIP_ERROR. */
int mas_hierarchy_device(mas_handle* h, int32_t* levels, int32_t* units, int32_t* sn, void* workspace,
                         size_t ws_bytes, void* stream);

/* The supernode hierarchy of a new block pattern under the analysed level-0
 * partition, built and left on the device: what Sec. 4.2 repeats every
 * Newton iteration, when contacts change H's pattern while the partition
 * computed at load stays (the construction of mas_hierarchy_device; every
 * level is queued at once and a level state on the device ends the
 * hierarchy, so nothing is read back to the host).
 *   nnzb, row_ptr, col_idx: device, the new pattern in the caller's node
 *       order (n_rows of the analysis; row_ptr[n_rows + 1], col_idx[nnzb]);
 *       it is symmetrised (block (i, j) links both nodes), so one triangle
 *       suffices; the diagonal is not needed.
 *   out_units: device int32[MAS_MAX_LEVELS + 1]: [0] = the level count, or
 *       -1 when a row range or a column index lies outside the pattern;
 *       [1 + l] = units of level l (0 past the last level).
 *   out_sn: device int32[MAS_MAX_LEVELS * n_rows]: unit of node i at level
 *       l at [l * n_rows + i], -1 past the last level.
 *   workspace: device scratch, ws_bytes >= mas_hierarchy_workspace_size,
 *       256-byte aligned (not shared with a running call).
 * The node -> slot map of the analysis is read from the solver's workspace
 * once mas_build has placed the plans there (nothing is copied; that
 * workspace must then still be allocated and unchanged); before the
 * first mas_build it is copied from the handle into this workspace on each
 * call.  Does not synchronise the stream.  Errors:
 * MAS_NOT_READY, MAS_INVALID_ARG, MAS_WORKSPACE_TOO_SMALL, MAS_HIP_ERROR. */
int mas_hierarchy_rebuild(mas_handle* h, int64_t nnzb, const int32_t* row_ptr, const int32_t* col_idx,
                          int32_t* out_units, int32_t* out_sn, void* workspace, size_t ws_bytes, void* stream);

/* Device bytes of scratch mas_replan needs for a new pattern of nnzb
 * blocks (0 before mas_analyze or for nnzb outside [1, 2^31 - 1]). */
size_t mas_replan_workspace_size(const mas_handle* h, int64_t nnzb);

/* Every solver plan of a new block pattern of H, derived on the device
 * under the analysed level-0 partition: what Sec. 4.2 repeats each Newton
 * iteration when contacts change H's pattern (Supp. Alg. 2-5 for the
 * hierarchy, Supp. Eq. 5 for the coarse patterns and their reduction
 * plans).  The pattern is checked and put in slot order by a stable sort;
 * the hierarchy, the coarse patterns, the inversion gathers, the
 * restriction and prolongation tables and the group-symmetric SpMV storage
 * are built by sorts, scans and per-domain kernels, each equal bit for bit
 * to what mas_analyze_partition computes on the host for the same pattern
 * and partition.  The host reads back counts (the level count, each coarse
 * level's block count to size the next level's sort, then the array sizes)
 * and orders the SpMV's work groups from their block counts; it analyses
 * nothing.
 *   nnzb, row_ptr, col_idx: device, the new pattern in the caller's node
 *       order, with the rules of mas_analyze (n_rows of the analysis,
 *       row_ptr[n_rows + 1] from 0 to nnzb, columns strictly ascending,
 *       every diagonal block, a symmetric pattern); nnzb >= n_rows.
 *   workspace: device scratch, ws_bytes >= mas_replan_workspace_size(h,
 *       nnzb), 256-byte aligned.  It holds the new plans until mas_build
 *       places them in the solver workspace, so it must stay allocated and
 *       unchanged as long as the handle uses them (until the next
 *       mas_analyze*, mas_replan or mas_destroy).
 * On success the handle describes the new pattern: mas_get_info and
 * mas_workspace_size give its sizes, and the next mas_build (on a matrix of
 * the new pattern) places the plans and builds the preconditioner.  On an
 * error the handle keeps its previous plans.  Synchronises the stream.
 * Errors: MAS_NOT_READY, MAS_INVALID_ARG (also for a pattern that breaks
 * the rules above), MAS_WORKSPACE_TOO_SMALL, MAS_HIP_ERROR. */
int mas_replan(mas_handle* h, int64_t nnzb, const int32_t* row_ptr, const int32_t* col_idx, void* workspace,
               size_t ws_bytes, void* stream);

/* Host copy of the handle's static description (after mas_analyze). */
int mas_get_info(const mas_handle* h, mas_info* out);

/* Host copies of the ordering: map[n_rows] (node -> level-0 slot),
 * remap[parts*domain_size] (slot -> node or -1), sn[levels*n_rows]
 * (unit of each node at each level; level 0 = slot).  Any pointer may be
 * NULL.  After mas_replan, sn is read from the replan workspace (a
 * synchronous device copy).  Errors: MAS_NOT_READY, MAS_HIP_ERROR. */
int mas_get_ordering(const mas_handle* h, int32_t* map, int32_t* remap, int32_t* sn);

/* Host copy of the domain inverses Inv_{l,d} = (S_d C_l H C_l^T S_d^T)^-1 of
 * level l as the last mas_build left them (the per-domain inverses of
 * Supp. Eq. 6; inverted over the occupied lanes, Sec. 4.2), for checking them
 * against a reference.
 *   level: 0 <= level < levels.
 *   precision: MAS_PRECISION_F64 for the FP64 inverses, MAS_PRECISION_MIXED
 *              for the FP32 copy of a mixed-precision handle (widened).
 *   out: host, ndom[level] * (3N)^2 doubles; domain d at d (3N)^2, entry
 *        (i, j) at d (3N)^2 + j 3N + i (column-major; the inverses are
 *        symmetric), DOF 3 a + c of lane a.  Unoccupied lanes are zero rows
 *        and columns.  Inverses kept symmetric-packed on the device are
 *        expanded.
 * Synchronises the stream.  Errors: MAS_NOT_READY (no successful
 * mas_build), MAS_INVALID_ARG (level out of range, FP32 copy asked of an FP64
 * handle), MAS_HIP_ERROR. */
int mas_get_inverses(const mas_handle* h, int32_t level, int32_t precision, double* out, void* stream);

/* Device time in milliseconds of the phases of the last mas_build and
 * pcg_solve / pcg_adjoint call on this handle, measured with HIP events on
 * the call's stream: [0] coarse sums and [1] batched inversion (mas_build),
 * [2] permutation of H into domain order and [3] the PCG iterations with
 * their setup and final residual check (pcg_solve). */
int mas_get_timings(const mas_handle* h, double* ms4);

/* Per-launch kernel timing for measurement.  With enable != 0 every later
 * pcg_solve / pcg_adjoint launches its iteration kernels with a pair of HIP
 * events that the runtime stamps with that dispatch's own start and end, and
 * accumulates the elapsed times (the event bookkeeping adds host work per
 * launch, so leave it off for timed runs).  Enabling or disabling clears the
 * totals. */
int mas_set_kernel_timing(mas_handle* h, int enable);

/* Totals since the last mas_set_kernel_timing: total_ms[8] and launches[8]
 * for the kernel slots [0] direction update and SpMV q = H p with p^T q
 * (and the restriction of q), [1] x/r update with ||r||^2 and the
 * restriction of r, [2] coarse-level MAS apply, [3] level-0 MAS apply with
 * prolongation and r^T z, [4] the same fused with the x/r update,
 * [5] FP64 residual replacement, [6] permutation of H, [7] restriction only.
 * Launches queued after the solve had stopped, which return at once, are
 * not counted.  Host arrays. */
int mas_get_kernel_timing(const mas_handle* h, double* total_ms, int32_t* launches);

/* Short English description of a status code (static string). */
const char* mas_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif
