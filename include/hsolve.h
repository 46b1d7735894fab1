/*
 * hsolve: hierarchical (LoRaSp / GC) factorization of a sparse SPD matrix on one
 * MI355X (gfx950) GPU, used as a preconditioner inside PCG.
 *
 * The operation is the one of arXiv:1611.03189 (Yang, Pouransari, Darve, "Sparse
 * hierarchical solvers with guaranteed convergence"):
 *   - §2-§3: the problem A x = b with A sparse SPD (eq. Axb), block partition into
 *     2^L red nodes by recursive bisection, pairwise merge into super nodes;
 *   - §3.2 and Algorithm "Setup": for each super node, compression of its
 *     well-separated block (eq. local_compression / compression_sw), extension
 *     (eq. extended) and elimination (eq. extended_rearranged), level by level up
 *     to an exact root;
 *   - §6: the GC variant, which keeps the action of A on chosen vectors exact
 *     (eq. compression_xy, eq. preserve);
 *   - §3.3 and Algorithm "Solve" (Appendix A): z = A_H^{-1} r with P_ss and M_ss.
 *
 * Conventions for every call:
 *   - Every function returns an hsolve_status and never throws or aborts.
 *   - "host" pointers are ordinary CPU memory, "device" pointers are GPU memory of
 *     the current HIP device (e.g. torch.cuda tensors' data_ptr()).
 *   - The caller keeps ownership of every array it passes. hsolve_analyze copies the
 *     pattern (and coordinates / preserved vectors); hsolve_factor copies the values.
 *   - Dense vectors are column-major n x nrhs with a leading dimension >= n.
 *   - All GPU work of a plan runs on the stream given in the options (NULL = the
 *     default stream); calls return after that work has finished.
 *   - A plan is not reentrant: calls on one plan must not overlap. Separate plans may
 *     be used from separate host threads.
 *   - Device memory comes from the caller: hsolve_analyze reports an upper bound, and
 *     hsolve_factor takes an arena of that size (or of the size an earlier factorization
 *     of the same values used). The library allocates only pinned host staging.
 */
#ifndef HSOLVE_H
#define HSOLVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hsolve_plan_s* hsolve_plan;

typedef enum {
    HSOLVE_OK = 0,
    HSOLVE_NOT_CONVERGED = 1,      /* warning: x holds the last iterate, stats are filled */
    HSOLVE_ERR_INVALID = -1,       /* bad sizes, unsorted / out-of-range CSR, NaN, bad options */
    HSOLVE_ERR_NOT_SYMMETRIC = -2, /* the sparsity pattern is not symmetric */
    HSOLVE_ERR_NOT_SPD = -3,       /* a pivot block (or S = U^T A_ss^-1 U) failed Cholesky;
                                      stats.fail_level / fail_node name it */
    HSOLVE_ERR_OOM = -4,           /* the arena given to hsolve_factor is too small */
    HSOLVE_ERR_DEVICE = -5,        /* a HIP runtime call failed */
    HSOLVE_ERR_STATE = -6,         /* call out of order (e.g. apply before factor) */
    HSOLVE_ERR_TOO_LARGE = -7      /* a merged super node grew beyond opt.max_super unknowns (the
                                      ranks below it were larger than the plan was sized for);
                                      stats.fail_level / fail_node name it */
} hsolve_status;

/* compression: LoRaSp (truncated SVD of A_sw, §3.2); GC (keeps the given vectors exactly, §6);
   GC_PROJ1 (keeps them approximately: the first-order one-sided projection of Appendix B, where
   U1 holds the singular directions of [X_s, A_sw X_w] above eps1 times the largest, X = phi) */
enum { HSOLVE_LORASP = 0, HSOLVE_GC = 1, HSOLVE_GC_PROJ1 = 2 };
/* outer iteration of hsolve_solve (§7): conjugate gradients with the standard or the
   flexible beta, right-preconditioned restarted GMRES, or the stationary iteration
   x <- x + A_H^{-1} (b - A x) of §7.1 */
enum { HSOLVE_PCG = 0, HSOLVE_FPCG = 1, HSOLVE_GMRES = 2, HSOLVE_STATIONARY = 3 };
/* compression tolerance per level (§7.1 "3D cases", Table 3); lmax = L - 1 is the depth of the
   first super nodes and d the depth of the node compressed:
   CONSTANT  eps everywhere;
   SHRINK    eps 2^{(d - lmax)/3}: eps at the leaves, smaller toward the root (the paper's
             adaptive choice for GC);
   GROW      eps h 2^{(lmax - d)/3}, h = n^{-1/dim}: small at the leaves, larger toward the root
             (the paper's adaptive choice for LoRaSp) */
enum { HSOLVE_EPS_CONSTANT = 0, HSOLVE_EPS_SHRINK = 1, HSOLVE_EPS_GROW = 2 };
/* which clusters are neighbours (their interaction is never compressed):
   FOOTPRINT  clusters joined by a nonzero of A (§3.1: the original graph's adjacency);
   GEOMETRIC  the rule of §7's experiments: with every unknown a unit cell at its coordinates,
              clusters (boxes of their cells) are well separated when the Euclidean gap
              between the boxes exceeds the larger box side, and neighbours otherwise */
enum { HSOLVE_NEIGHBOURS_FOOTPRINT = 0, HSOLVE_NEIGHBOURS_GEOMETRIC = 1 };
/* order in which the super nodes of a level are eliminated (§3.2 leaves it open); both rules
   eliminate colour by colour, a colour being a set of nodes without blocks between them, built
   by one greedy pass over the nodes not yet eliminated and then eliminated in index order:
   INDEX    the pass visits the nodes in index order;
   WAITING  the pass visits first the nodes with the most partners (nodes with a block to
            them) not yet eliminated at the level, ties by index. It packs the colours
            tighter: fewer colours per level, so fewer batched steps in the factorization */
enum { HSOLVE_ORDER_INDEX = 0, HSOLVE_ORDER_WAITING = 1 };

typedef struct {
    int leaf_size;          /* target unknowns per leaf red node (default 16); the tree
                               depth L is the integer nearest log2(n / leaf_size) */
    double eps;             /* relative compression tolerance (>= 0; 0 = no truncation):
                               keep singular values > eps * ||A_sw||_2 */
    int variant;            /* HSOLVE_LORASP, HSOLVE_GC (default) or HSOLVE_GC_PROJ1 */
    int nvec;               /* GC: number of preserved vectors in phi (<= 8) */
    const double* phi;      /* GC, host: n x nvec column-major, or NULL for the constant
                               vector (GC-constant); for GC_PROJ1 the vectors X of Appendix B
                               (low-frequency eigenvectors divided by their eigenvalues) */
    int dim;                /* coordinate dimension 0..3 */
    const double* coords;   /* host: n x dim, row-major (coords[i*dim + t]); NULL = use
                               the unknown index as a 1-D coordinate */
    double tol;             /* hsolve_solve: stop at ||b - A x||_2 <= tol ||b||_2 (1e-10) */
    int max_iter;           /* hsolve_solve: iteration cap (1000) */
    int krylov;             /* HSOLVE_PCG (default), HSOLVE_FPCG, HSOLVE_GMRES, HSOLVE_STATIONARY */
    void* stream;           /* hipStream_t or NULL */
    int apply_prec;         /* 64 (default) or 32: precision of the solve phase. With 32 the
                               factor is computed in FP64 and its solve-phase blocks are rounded
                               once to FP32; the sweeps read and accumulate in FP32 (vectors
                               enter and leave in FP64). Pair it with HSOLVE_FPCG or GMRES. */
    int restart;            /* HSOLVE_GMRES: Krylov vectors per cycle (200) */
    int overlap_pivots;     /* 1 (default): the pivot blocks of a colour are factored on a
                               second stream of the plan while the colour is compressed, and the
                               compression of its nodes above 128 unknowns runs on a third one
                               beside that of the smaller nodes; 0: all in order on opt.stream
                               (for callers that run many plans at once). The results are the
                               same bits either way */
    int factor_prec;        /* 64 (default) or 32: storage and arithmetic of the factorization. With
                               32 the blocks, pivots (Cholesky and inverse), Schur updates, Gram
                               matrices and the products of the elimination run in FP32 on the
                               matrix cores; the symmetric eigen-solver of the compression reads the
                               FP32 Gram matrix in FP64 and its basis is rounded back to FP32. The
                               solve phase then runs in FP32 (apply_prec is 32); pair it with
                               HSOLVE_FPCG or HSOLVE_GMRES, whose FP64 loop refines to opt.tol. */
    int max_super;          /* largest super node, in unknowns, the plan admits (1..512, default
                               512); it caps the ranks the arena bound of hsolve_analyze assumes */
    int max_nrhs;           /* right-hand sides per batch the arena bound covers (default 32);
                               hsolve_solve / hsolve_apply with more run in batches */
    int eps_schedule;       /* HSOLVE_EPS_CONSTANT (default), HSOLVE_EPS_SHRINK, HSOLVE_EPS_GROW */
    int cmp_lpe;            /* launch shape of the eigenvalue multisection: lanes per eigenvalue
                               (1, 2, 4, ..., 64), 0 = chosen from the launch size (default) */
    int cmp_vectors;        /* inverse iteration: 0 = chosen from the launch size (default),
                               1 = one lane per eigenvalue, 2 = one wave per eigenvalue */
    int apply_graph;        /* 1 (default): the forward and backward sweeps of an apply are
                               captured once per workspace as a HIP graph and replayed; 0: the
                               launches are issued one by one */
    int neighbours;         /* HSOLVE_NEIGHBOURS_FOOTPRINT (default) or HSOLVE_NEIGHBOURS_GEOMETRIC */
    double eps1;            /* HSOLVE_GC_PROJ1: relative truncation of [X_s, A_sw X_w] (0 <= eps1 < 1;
                               0 keeps its whole range, as GC) */
    int cmp_ritz;           /* 1 (default): the last kept directions of each compression are
                               refined by Rayleigh-Ritz on A_sw itself (FP64 factorization, eps > 0):
                               the eigen-solver also returns up to 8 eigenvectors past the
                               threshold, and the window of up to 8 kept plus those is rotated by
                               the eigenvectors of (W^T A_sw)(W^T A_sw)^T; 0: the Gram matrix's
                               eigenvectors as they are */
    int order;              /* HSOLVE_ORDER_WAITING (default) or HSOLVE_ORDER_INDEX */
} hsolve_options;

typedef struct {
    int iterations;             /* outer iterations of the last hsolve_solve (max over rhs) */
    double rel_residual;        /* largest true ||b - A x||_2 / ||b||_2 over the rhs */
    double t_analyze;           /* seconds, host wall clock */
    double t_factor;
    double t_solve;
    int levels;                 /* tree depth L */
    int colours;                /* elimination colours summed over levels */
    int max_rank;               /* largest red-node size */
    int64_t factor_bytes;       /* device bytes of the stored factors (apply data) */
    double factor_flops;        /* counted algorithmic flops of the last factorization */
    double apply_bytes;         /* algorithmic bytes read+written by one apply (1 rhs) */
    int fail_level;             /* for HSOLVE_ERR_NOT_SPD: depth and node of the failure */
    int fail_node;
    int64_t device_bytes;       /* arena bytes in use: pattern, values, factors, and the larger of
                                   the factorization's transient regions and the solve workspace */
    int64_t arena_bound;        /* the upper bound hsolve_analyze reported */
} hsolve_stats;

/* Fill *opt with the defaults listed above. */
void hsolve_default_options(hsolve_options* opt);

/* Symbolic analysis (§2.1, §3, §3.1): clustering into 2^L leaves by recursive bisection,
 * footprint adjacency per level, simulated elimination (block fill, neighbour and
 * well-separated sets, colour order per level), and the device memory a factorization of
 * this pattern can need. Host only: no GPU work, no device memory.
 *   n        number of unknowns (>= 1)
 *   row_ptr  host, n+1 entries, row_ptr[0] = 0, nondecreasing
 *   col_idx  host, row_ptr[n] entries, each row sorted ascending, in [0, n), and the
 *            pattern structurally symmetric (HSOLVE_ERR_NOT_SYMMETRIC otherwise)
 *   opt      host, may be NULL for defaults
 *   out      receives the new plan (NULL on error)
 *   arena_bytes_upper_bound  may be NULL; receives the arena size that holds any
 *            factorization of this pattern whose super nodes stay within opt.max_super,
 *            together with the solve phase of opt.max_nrhs right-hand sides. It is found by
 *            replaying the factorization's allocations with every rank at its largest
 *            possible value, min(m_s, 2p + |W(s)|) (p preserved vectors, §6). */
hsolve_status hsolve_analyze(int n, const int64_t* row_ptr, const int32_t* col_idx,
                             const hsolve_options* opt, hsolve_plan* out,
                             size_t* arena_bytes_upper_bound);

/* Numeric factorization (Algorithm "Setup"; §3.2 compression, extension, elimination;
 * §6 GC compression).
 *   values   host or device, row_ptr[n] doubles in the pattern given to hsolve_analyze;
 *            A must be symmetric positive definite; NaN or Inf gives HSOLVE_ERR_INVALID
 *   d_arena  device memory owned by the caller, 256-byte aligned (e.g. a torch.uint8 tensor
 *            of the bound reported by hsolve_analyze); the plan keeps the pattern, values,
 *            factors and solve-phase vectors in it and uses it until hsolve_destroy or the
 *            next hsolve_factor. The library never allocates or frees device memory.
 *   arena_bytes  its size; HSOLVE_ERR_OOM (nothing computed) when the factorization does not
 *            fit. The analysis bound always fits; stats.device_bytes tells what one
 *            factorization used, which also fits a refactorization of the same values.
 * Replaces any previous factorization of the plan. HSOLVE_ERR_NOT_SPD if a pivot block is
 * not positive definite, HSOLVE_ERR_TOO_LARGE if a super node exceeds opt.max_super (the
 * plan then has no factorization). */
hsolve_status hsolve_factor(hsolve_plan plan, const double* values, void* d_arena, size_t arena_bytes);

/* Preconditioner application z = A_H^{-1} r (Algorithm "Solve"): forward
 * substitution, restriction, parent-level solve, prolongation and backward substitution
 * in reverse elimination order, level by level. r, z: device, n x nrhs column-major;
 * r and z may not overlap. The solve vectors come from the arena (batches of columns when
 * it does not hold all of them at once). */
hsolve_status hsolve_apply(hsolve_plan plan, int nrhs, const double* r, int ldr, double* z,
                           int ldz);

/* hsolve_apply for callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): the same z = A_H^{-1} r, bitwise, with the two
 * solve vectors in a static device scratch of the library (64 MiB per GPU, held until the
 * process ends) instead of the arena. No device or host allocation, no kernel timing.
 * HSOLVE_ERR_OOM when 2 * (n + sum of ranks) * nrhs values (8 bytes each, 4 with
 * apply_prec = 32) exceed the scratch. All plans on one GPU share its scratch, which keeps the
 * last call's contents: calls that overlap on one GPU (any plans, any host threads) race. */
hsolve_status hsolve_apply_static(hsolve_plan plan, int nrhs, const double* r, int ldr, double* z,
                                  int ldz);

/* Solve A x = b preconditioned with A_H^{-1} (x0 = 0) to the relative residual opt.tol, with
 * the outer iteration opt.krylov. b, x: device, n x nrhs column-major. A column of b with a
 * NaN or Inf gives HSOLVE_ERR_INVALID.
 * PCG / FPCG: the columns advance together (one batched SpMV and apply per iteration), each
 * with its own scalars, and a column stops changing once it has converged, so every column
 * equals its own single-column solve. FPCG takes beta = r_{k+1}^T (z_{k+1} - z_k) / r_k^T z_k.
 * GMRES: right-preconditioned, restarted every opt.restart steps, modified Gram-Schmidt; the
 * columns are solved one after the other. Needs (2 restart + 4) n doubles of the arena.
 * STATIONARY: x_{k+1} = x_k + A_H^{-1} (b - A x_k) from x_0 = 0, all columns together, until
 * the true residual ||b - A x_k|| <= tol ||b|| (iterations counted as applies).
 * stats may be NULL; stats.iterations is the largest count over the columns and
 * stats.rel_residual the largest final relative residual (PCG: of the recursion; GMRES:
 * recomputed as ||b - A x|| / ||b||). HSOLVE_NOT_CONVERGED if max_iter is reached first
 * (x = last iterate). */
hsolve_status hsolve_solve(hsolve_plan plan, int nrhs, const double* b, int ldb, double* x,
                           int ldx, hsolve_stats* stats);

/* y = A x with the matrix of the last hsolve_factor. x, y: device, n entries. */
hsolve_status hsolve_spmv(hsolve_plan plan, const double* x, double* y);

/* Change the stream the plan's GPU work runs on (hipStream_t or NULL), e.g. when a request
 * loop hands an analysed plan to the slot that runs it. Not while a call on the plan runs. */
hsolve_status hsolve_set_stream(hsolve_plan plan, void* stream);

/* ---- Autotuning of the grouped GEMM (Schur updates, Gram matrices, pivot products) ----
 * The GEMM runs in one of HSOLVE_GEMM_VARIANTS output-tile shapes (0: 64x64 with K steps of
 * 16, 1: 64x64/32, 2: 128x64/16, 3: 128x128/16, 4: 32x32/64, 5: 32x32/128, 6: 64x64/16 and
 * 7: 32x32/64 persistent, i.e. a grid of resident workgroups looping over the tiles); every
 * shape gives the same bits. A launch
 * falls into one of HSOLVE_GEMM_BUCKETS buckets: its number of 64x64 output tiles (< 32,
 * < 256, < 2048, more) times its mean inner dimension (<= 64, <= 256, more), bucket =
 * 3 * tile_class + k_class; FP64 and FP32 GEMMs are tuned apart. hsolve_tune_gemm times every
 * shape on a synthetic launch of each bucket and type and keeps the fastest for the process:
 * d_work is caller device memory of at least hsolve_tune_workspace_bytes(); choice
 * (2 x HSOLVE_GEMM_BUCKETS entries: FP64 buckets, then FP32) and ms (2 x HSOLVE_GEMM_BUCKETS x
 * HSOLVE_GEMM_VARIANTS, best of three) may be NULL. Untuned, every bucket uses shape 0.
 * hsolve_set_gemm_choice installs a saved choice (2 x HSOLVE_GEMM_BUCKETS entries). Neither
 * may run while a factorization is in flight. */
#define HSOLVE_GEMM_VARIANTS 8
#define HSOLVE_GEMM_BUCKETS 12
size_t hsolve_tune_workspace_bytes(void);
hsolve_status hsolve_tune_gemm(void* d_work, size_t work_bytes, void* stream, int32_t* choice, double* ms);
hsolve_status hsolve_set_gemm_choice(const int32_t* choice);

/* Counters of the plan (levels, colours, ranks, bytes, flops, timings). */
hsolve_status hsolve_get_stats(hsolve_plan plan, hsolve_stats* stats);

/* Release the plan (host memory; the arena stays the caller's). NULL is accepted. */
hsolve_status hsolve_destroy(hsolve_plan plan);

/* Static, human-readable name of a status code. */
const char* hsolve_status_string(hsolve_status s);

/* Message of the last failed call on this plan ("" if none); valid until the next call. */
const char* hsolve_last_error(hsolve_plan plan);

/* ---- Kernel timing (HIP events on the plan's stream around every launch) ----
 * hsolve_profile_begin clears and starts recording for calls on this plan from the calling
 * thread; hsolve_profile_end stops, waits for the device and aggregates by kernel name
 * (*nkernels entries); hsolve_profile_entry reads entry i: name, summed milliseconds,
 * launches, and summed algorithmic work (flops for k_gemm, k_chol_inv*, k_comp_reduce*; bytes
 * for k_copy, k_fwd, k_bwd, k_spmv). */
hsolve_status hsolve_profile_begin(hsolve_plan plan);
/* Record only the launches of the kernel named `kernel` (as hsolve_profile_entry reports
 * it), so that the events of the others cost nothing; NULL or "" records every kernel. */
hsolve_status hsolve_profile_only(hsolve_plan plan, const char* kernel);
hsolve_status hsolve_profile_end(hsolve_plan plan, int32_t* nkernels);
hsolve_status hsolve_profile_entry(hsolve_plan plan, int i, char* name, int cap, double* ms,
                                   int64_t* launches, double* work);

/* ---- Introspection of the symbolic schedule (host arrays, caller-allocated) ---- */

/* Tree depth L of the plan. */
int hsolve_depth(hsolve_plan plan);

/* Leaf order: perm[p] = original index of the unknown at position p (n entries), and
 * leaf_off[i] = first position of leaf i (2^L + 1 entries). */
hsolve_status hsolve_leaf_order(hsolve_plan plan, int32_t* perm, int32_t* leaf_off);

/* Colour of every super node of level `depth` (2^depth entries; -1 = empty node) and
 * the number of colours in *ncolours. Colours are processed in increasing order, nodes
 * of one colour in increasing index. */
hsolve_status hsolve_level_colours(hsolve_plan plan, int depth, int32_t* colour_of,
                                   int32_t* ncolours);

/* Neighbour set N(s) and well-separated set W(s) of super node `node` of level `depth`
 * when it is eliminated, as ascending indices. Each list entry is 2*index + (1 if the
 * partner was already a red node at that time, else 0). At most `cap` entries are
 * written per list; *nn / *nw receive the full lengths. */
hsolve_status hsolve_node_sets(hsolve_plan plan, int depth, int node, int32_t* nbrs,
                               int32_t* nn, int32_t* ws, int32_t* nw, int cap);

/* Stored factor of super node `node` of level `depth` after the last factorization:
 * dims[0] = m (super-node size), dims[1] = ntot (rows of all neighbour blocks), dims[2] = k.
 * If G is not NULL, copies the (m + ntot + k) x m column-major matrix [M_ss; A_Ns M_ss; P_ss]
 * (Appendix A) to the host array G of `cap` doubles. Empty nodes report m = 0. */
hsolve_status hsolve_node_factor(hsolve_plan plan, int depth, int node, int32_t* dims,
                                 double* G, int64_t cap);

/* Red-node sizes (ranks k) of level `depth` after the last factorization
 * (2^depth entries, 0 for empty nodes). */
hsolve_status hsolve_ranks(hsolve_plan plan, int depth, int32_t* ranks);

#ifdef __cplusplus
}
#endif
#endif /* HSOLVE_H */
