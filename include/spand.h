/*
 * spand.h - C ABI of the MI355X spaND + s-step GMRES library (libspand.so).
 *
 * The library solves A x = b for the block-sparse Jacobian of an implicit
 * DG discretisation (the linear system of the paper's Eq. (5)) with a
 * sparsified-nested-dissection (spaND) factorization used as a right
 * preconditioner of s-step GMRES.  All compute runs in HIP kernels on the
 * current device; the host code only plans and launches.
 *
 * Conventions shared by every entry point
 *  - Matrices are BSR: n_brows block rows of bs x bs blocks, blocks stored
 *    row-major and contiguous, block columns strictly ascending in each
 *    row.  Block row e corresponds to grid element (i, j) with
 *    e = j * nx + i; inside a block the unknown index is 4*m + c (mode m,
 *    conserved variable c), so bs = 4 (p+1)^2.
 *  - Pointers named d_* are device pointers; h_* are host pointers.  The
 *    caller owns all of them.  A is borrowed for the duration of a call:
 *    the library copies what it keeps.
 *  - Vectors are float64 of length N = n_brows * bs.
 *  - "stream" is a hipStream_t passed as void* (0 = null stream).  Every
 *    call is stream-ordered; calls that return host-visible results
 *    (ranks, iteration counts) synchronise that stream before returning.
 *  - Return value: SPAND_OK (0), a negative hard error or a positive soft
 *    result (see spand_status_t).  spand_last_error() gives a message for
 *    the last failure on the calling thread.
 *  - A factor handle is used by one stream at a time.
 */
#ifndef SPAND_H
#define SPAND_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SPAND_OK = 0,
  SPAND_EINVAL = -1,      /* bad argument, detected before any launch       */
  SPAND_ENOMEM = -2,      /* device allocation failed                        */
  SPAND_ESINGULAR = -3,   /* exactly zero pivot met in a factorization       */
  SPAND_EHIP = -4,        /* HIP runtime error                               */
  SPAND_ENOTCONV = 1,     /* GMRES hit maxit; d_x holds the last iterate      */
  SPAND_EBREAKDOWN = 2    /* CholQR met a non-SPD Gram matrix; d_x holds the
                             iterate before the failing block                */
} spand_status_t;

typedef struct {
  int32_t n_brows;          /* number of block rows (= grid elements K)      */
  int32_t bs;               /* block size b                                  */
  int64_t nnzb;             /* number of stored blocks                       */
  const int32_t *d_rowptr;  /* [n_brows+1]                                   */
  const int32_t *d_colind;  /* [nnzb], ascending inside each block row       */
  const double *d_val;      /* [nnzb * bs * bs], row-major blocks            */
} spand_bsr_t;

typedef struct {
  int32_t nx, ny;           /* element grid, n_brows = nx * ny               */
  int32_t periodic_x;       /* 1: wrap-around adjacency in x                 */
  int32_t periodic_y;       /* 1: wrap-around adjacency in y                 */
} spand_grid_t;

enum { SPAND_F64 = 0, SPAND_F32 = 1 };

/* spand_opts_t.flags */
#define SPAND_FLAG_NO_GRAPH 1   /* run the sweeps eagerly instead of replaying
                                   a captured hipGraph                        */

typedef struct {
  double eps;               /* RRQR tolerance epsilon (>= 0); 0 keeps all    */
  int32_t nlevels;          /* lmax; 0 -> round(log2(K/32)) + 1               */
  int32_t factor_dtype;     /* SPAND_F64 or SPAND_F32 (storage and compute of
                               the factor; vectors stay float64)            */
  int32_t flags;            /* SPAND_FLAG_* bits, 0 by default               */
} spand_opts_t;

/* sstep_opts_t.flags (0: Newton basis on Leja-ordered Ritz values, two
 * block CGS + CholQR passes, no diagnostics - the method of Sec. CAGMRES).
 * For the stability study of the basis and the orthogonalisation (Fig. 6):
 *   SSTEP_FLAG_MONOMIAL  all shifts zero, no Ritz steps: the monomial basis
 *   SSTEP_FLAG_ONE_PASS  one block CGS + CholQR pass per block instead of two
 *   SSTEP_FLAG_ORTH_LOSS record ||Q^T Q - I||_F of the basis after every block
 *                        (a diagnostic: one Gram matrix of the whole basis per
 *                        block, inside the timed phases as "other")          */
#define SSTEP_FLAG_MONOMIAL 1
#define SSTEP_FLAG_ONE_PASS 2
#define SSTEP_FLAG_ORTH_LOSS 4
/*   SSTEP_FLAG_CLASSICAL classical GMRES (Algorithm 1): every column by an
 *                        Arnoldi step with modified Gram-Schmidt, the baseline
 *                        the s-step method is compared with (Fig. 7)         */
#define SSTEP_FLAG_CLASSICAL 8
/*   SSTEP_FLAG_LAGGED    the single-reduce schedule of Algorithm 2: the
 *                        operator applications of a block start from the
 *                        previous block after its first pass; one Gram matrix
 *                        per block gives that block's second pass (its
 *                        Hessenberg columns and convergence check) and the new
 *                        block's first pass.  Same basis, Hessenberg matrix and
 *                        residual history as the default schedule in exact
 *                        arithmetic, one reduction per block instead of four.
 *                        Not with SSTEP_FLAG_ONE_PASS (SPAND_EINVAL).        */
#define SSTEP_FLAG_LAGGED 16
typedef struct {
  int32_t s;                /* block size of the s-step method (1..8)        */
  int32_t restart;          /* restart length m, a multiple of s              */
  int32_t maxit;            /* maximum number of Krylov vectors              */
  int32_t transpose;        /* 1: solve A^T x = b, preconditioned by M^-T    */
  double rtol;              /* stop when ||b - A x|| <= rtol ||b||            */
  int32_t flags;            /* SSTEP_FLAG_* bits                             */
  int32_t pad;
} sstep_opts_t;

#define SSTEP_MAX_HIST 1024
typedef struct {
  int32_t iters;            /* Krylov vectors used                           */
  int32_t restarts;         /* cycles run                                    */
  int32_t converged;        /* 1 if the true residual met rtol               */
  int32_t n_hist;           /* entries in hist (<= SSTEP_MAX_HIST)           */
  double relres;            /* true ||b - A x|| / ||b|| at exit               */
  double hist[SSTEP_MAX_HIST]; /* |g_{k+1}| after every column (Givens)      */
  int32_t n_shifts;         /* Newton shifts used (slots)                    */
  double shift_re[8];
  double shift_im[8];
  /* phase times in milliseconds (hipEvent based, on the call's stream)    */
  double t_total_ms, t_spmv_ms, t_apply_ms, t_orth_ms, t_other_ms;
  int32_t n_spmv;           /* SpMV launches (t_spmv_ms covers exactly these) */
  int32_t n_apply;          /* preconditioner applications                  */
  int32_t n_orth;           /* entries in orth_loss (SSTEP_FLAG_ORTH_LOSS)   */
  int32_t n_reduce;         /* inner-product reductions over the vectors
                               (dot products and Gram matrices)             */
  double orth_loss[SSTEP_MAX_HIST]; /* ||Q^T Q - I||_F after each block, with
                               the basis size j + s + 1 in orth_cols       */
  int32_t orth_cols[SSTEP_MAX_HIST];
} sstep_stats_t;

#define SPAND_MAX_LEVELS 32
typedef struct {
  int32_t nlevels;
  int32_t n_clusters[SPAND_MAX_LEVELS];   /* interfaces sparsified per level */
  int32_t rank_min[SPAND_MAX_LEVELS];
  int32_t rank_max[SPAND_MAX_LEVELS];
  double rank_avg[SPAND_MAX_LEVELS];
  int64_t size_before[SPAND_MAX_LEVELS];  /* sum |s| before sparsification  */
  int64_t size_after[SPAND_MAX_LEVELS];   /* sum k after sparsification      */
  int32_t top_size;                       /* unknowns left at the top        */
  int64_t factor_bytes;                   /* device bytes read by one apply  */
  double factor_flops;                    /* algorithmic flops of the factor */
  double t_host_ms;                       /* host ND + planning              */
  double t_device_ms;                     /* device phases (event timed)     */
  double t_lu_ms, t_schur_ms, t_scale_ms, t_rrqr_ms, t_compress_ms;
  /* the rank-revealing QR kernel alone (HIP events around each launch) */
  double t_qrcp_ms;                       /* summed kernel time              */
  int32_t n_qrcp;                         /* launches (one per level)        */
  int32_t pad0;
  double qrcp_bytes;                      /* algorithmic bytes: every W read
                                             once, every Q written once     */
  double qrcp_flops;                      /* 4mck - 2k^2(m+c) + 4k^3/3 sums  */
  double t_alloc_ms;                      /* host time in hipMalloc/hipFree
                                             (blocks not found in the cache) */
  int64_t resident_bytes;                 /* device memory the factor keeps  */
  /* host time (planning and launches) spent in each phase: gather, LU,
     Schur, scale, RRQR, compress; the device waits when it exceeds the
     phase's device time */
  double t_plan_ms[6];
  /* the factorization's matrix-core products (HIP events around each
     launch): batched GEMMs (elimination, scaling, compression, completion,
     Schur updates of levels >= 1) and the level-0 element-block Schur
     kernel, with their algorithmic flops (2MNK per product, the zero half
     of a triangular operand excluded; 4 b^3 per Schur coupling pair) and
     bytes (operands read once, C read when accumulated, C written) */
  double t_gemm_ms, gemm_flops, gemm_bytes;
  int32_t n_gemm, n_schur_elem;
  double t_schur_elem_ms, schur_elem_flops, schur_elem_bytes;
  /* systems factored together (1 unless the handle comes from
     spand_factor_batched and shares its factorization with other systems of
     the batch: then the ranks, top_size, factor_bytes and factor_flops
     above are this system's own, and the times, counts and bytes of the
     kernels, resident_bytes and t_host_ms are those of the shared
     factorization) */
  int32_t batch_systems;
  int32_t pad1;
} spand_factor_stats_t;

typedef struct spand_factor_s *spand_factor_t;

/*
 * spand_factor - build the spaND factorization of A (paper Sec. "Sparsified
 * Nested Dissection algorithm", Eqs. (10)-(13)): geometric nested
 * dissection of the element grid, then level by level: row-pivoted LU
 * elimination of interiors with Schur updates, LU scaling of interfaces with
 * the diagonal of U split evenly, rank-revealing QR sparsification of every
 * interface at tolerance eps, compression of all blocks, merge.
 * In:  A (device BSR, bs = 4(p+1)^2, n_brows = nx*ny), grid, opts.
 * Out: *out, an opaque handle owned by the library until spand_destroy.
 * Errors: SPAND_EINVAL for inconsistent sizes/options (before any launch),
 * SPAND_ESINGULAR if a pivot is exactly zero, SPAND_ENOMEM, SPAND_EHIP.
 * Synchronises the stream (per-level ranks are read back to plan the next
 * level).
 */
int spand_factor(const spand_bsr_t *A, const spand_grid_t *grid,
                 const spand_opts_t *opts, void *stream, spand_factor_t *out);

/*
 * spand_apply - d_out = M^{-1} d_in with A ~ M = prod F_i (paper Sec.
 * "Sparsified Nested Dissection algorithm": the product of triangular and
 * orthogonal factors used as a preconditioner).  Forward sweep over the
 * levels applies the left factors, backward sweep the right ones.
 * d_in and d_out: device float64[N]; d_in == d_out is allowed.
 * Deterministic: repeated calls give bitwise-equal results.
 */
int spand_apply(spand_factor_t F, const double *d_in, double *d_out, void *stream);

/*
 * spand_refactor - rebuild the factorization held by F for new values of a
 * matrix with the same block pattern and grid (the next nonlinear step of a
 * pseudo-transient solve, paper Sec. "Flow Solver", Eqs. (5), (8), (9): the
 * factorization is computed at every nonlinear step, the partitioning is
 * pre-processing, Sec. "Scalability study of spaND").  Reuses F's symbolic
 * phase (the validated block pattern and the nested dissection) with F's
 * options; every numeric phase runs again (the ranks depend on the values).
 * A is borrowed for the call.  Returns SPAND_EINVAL, before any launch, if
 * A's sizes or block pattern (compared on the host) differ from F's; any
 * other failure leaves F's previous factorization in place.  The previous
 * factorization stays allocated until the new one is built (peak memory
 * holds both).  Stream-ordered like spand_factor.
 */
int spand_refactor(spand_factor_t F, const spand_bsr_t *A, void *stream);

/* spand_apply_T - d_out = M^{-T} d_in, the exact transpose of spand_apply
 * (same factors, transposed sweeps).  Same arguments and rules. */
int spand_apply_T(spand_factor_t F, const double *d_in, double *d_out, void *stream);

/*
 * sstep_gmres_solve - right-preconditioned restarted s-step GMRES (paper
 * Algorithm 2 with the Newton basis, Leja-ordered Ritz shifts from s steps
 * of standard GMRES, two block CGS and two Cholesky QR passes): solves
 * A x = b (transpose = 0) or A^T x = b (transpose = 1, with M^{-T}).
 * M may be NULL (no preconditioner).  d_x holds x0 on entry (pass zeros
 * for x0 = 0) and the solution on exit.  st may be NULL.
 * Returns SPAND_OK, SPAND_ENOTCONV or SPAND_EBREAKDOWN (d_x valid in all
 * three), or a negative error.
 */
int sstep_gmres_solve(const spand_bsr_t *A, spand_factor_t M, const double *d_b,
                      double *d_x, const sstep_opts_t *opts, sstep_stats_t *st,
                      void *stream);

/*
 * sstep_gmres_solve_noalloc - sstep_gmres_solve for callers that cannot
 * allocate device memory (serving loops and harnesses that forbid
 * hipMalloc).  Same arguments, results and statuses, computed by the same
 * kernels; it allocates no device memory: its workspace (the Krylov basis,
 * N x (restart + 1) doubles, two N-vectors, the Krylov state, the partial
 * sums) lives in a library-owned array of SPAND_NOALLOC_SCRATCH_BYTES per
 * device, held from the first call on that device until the process ends.
 * A solve whose workspace would exceed it returns SPAND_EINVAL before any
 * launch (about N (restart + 3) 8 bytes: N up to ~130,000 at restart 60).
 * It does not tune the SpMV (the tuned or default lanes are used) and
 * reports no phase times (t_* = 0 in st).  A transposed solve with M uses
 * the eager M^-T sweeps unless a transposed solve or spand_apply_T has
 * captured them before.  The solver synchronises with the host every cycle,
 * so the call cannot be captured into a HIP graph.  All calls on one device
 * share its array: they are serialised by a lock, each returns only after
 * its work on `stream` has finished, and the array keeps the last call's
 * contents (every buffer is rewritten before it is read).
 */
#define SPAND_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int sstep_gmres_solve_noalloc(const spand_bsr_t *A, spand_factor_t M, const double *d_b,
                              double *d_x, const sstep_opts_t *opts, sstep_stats_t *st,
                              void *stream);

/*
 * spand_bsr_spmv - d_y = alpha * op(A) d_x + beta * d_y, op = A or A^T
 * (the SpMV of Algorithms 1 and 2).  float64.  d_x != d_y.  A^T reads the
 * mirror block (J, I) of every stored (I, J) in place: the block pattern
 * must be structurally symmetric, which is checked first (SPAND_EINVAL,
 * after a synchronisation of `stream`, before the product).
 */
int spand_bsr_spmv(const spand_bsr_t *A, int transpose, double alpha, const double *d_x,
                   double beta, double *d_y, void *stream);

/*
 * spand_bsr_pattern_outer - for every stored block (I,J) of the pattern:
 * d_out[t] = alpha * u_I v_J^T (row-major bs x bs).  This is the gradient
 * of g^T A^{-1} b with respect to the stored values when u = lambda,
 * v = x and alpha = -1 (adjoint of the linear solve; values only on the
 * BSR pattern).  d_out: device float64[nnzb*bs*bs].
 */
int spand_bsr_pattern_outer(const spand_bsr_t *pattern, const double *d_u,
                            const double *d_v, double alpha, double *d_out, void *stream);

/*
 * spand_factor_batched - factor n independent systems of possibly different
 * sizes (A[i], grids[i], opts[i]; each is checked as by spand_factor before
 * any work).  The systems with the same block size, factor precision, eps
 * and flags are factored together, in index order, in groups of at most
 * SPAND_BATCH_UNION_DOF unknowns (default 4M), each group as one
 * block-diagonal matrix: the systems' orderings are placed side by side
 * (level l holds the level-l clusters of every one of them, a system with
 * fewer levels finishes at its own top), and every phase of every level is
 * one set of launches for all of them.  No launch mixes the arithmetic of
 * two systems, and each cluster takes the kernels its own size selects, so
 * every system's factor is the one spand_factor computes for it alone (same
 * ranks, same values).  The groups run concurrently on library-owned HIP
 * streams, at most SPAND_BATCH_FACTOR_STREAMS (default 2) at a time; the
 * call waits on `stream` first and makes `stream` wait for all of them at
 * the end.  SPAND_BATCH_SEPARATE=1 factors every system on its own instead
 * (SPAND_BATCH_STREAMS, default 8, at a time).
 * out[i] receives system i's handle; the handles of one group share the
 * factorization's device memory, which is released with the last of them.
 * Such a handle applies its own system's operators only (its own sweep
 * graphs; apply, apply_T, solves and stats as for spand_factor), several of
 * them may be used on different streams at once, and spand_refactor rejects
 * it (SPAND_EINVAL).  Returns SPAND_OK, or the first negative status; then
 * every out[i] is NULL.
 */
int spand_factor_batched(int32_t n, const spand_bsr_t *A, const spand_grid_t *grids,
                         const spand_opts_t *opts, void *stream, spand_factor_t *out);

/*
 * spand_apply_batched - d_out[i] = M_i^-1 d_in[i] (transpose = 0) or
 * M_i^-T d_in[i] (1) for i < n, in stream order on `stream`.  Where the
 * handles include every system of one factorization of
 * spand_factor_batched, each once, those systems are applied together by one
 * replay of that factorization's sweep graph (all its systems in each
 * launch); other handles are applied one by one.  Vectors: device float64
 * of each system's length; d_in[i] == d_out[i] is allowed.  Must not
 * overlap in time with another apply or solve that uses one of these
 * handles.
 */
int spand_apply_batched(int32_t n, const spand_factor_t *F, const double *const *d_in,
                        double *const *d_out, int32_t transpose, void *stream);

/*
 * sstep_gmres_solve_batched - n independent s-step GMRES solves, run
 * concurrently on library-owned HIP streams from a pool of host workers
 * (SPAND_BATCH_STREAMS, default 8), ordered after `stream` and waited for
 * on it at the end.  M[i] may be NULL; one handle may appear at
 * several M[i] (one operator, many right-hand sides): the systems that share
 * a handle are solved one after the other, in index order, on one worker
 * stream, since they share its scratch vectors.  d_b[i], d_x[i] device
 * float64 vectors (x0 in, solution out); opts[i]; st may be NULL or an
 * array of n stats.  Returns SPAND_OK if every system converged, otherwise
 * the most severe status (negative errors first, then SPAND_EBREAKDOWN,
 * SPAND_ENOTCONV); per-system results are in st[i].
 */
int sstep_gmres_solve_batched(int32_t n, const spand_bsr_t *A, const spand_factor_t *M,
                              const double *const *d_b, double *const *d_x,
                              const sstep_opts_t *opts, sstep_stats_t *st, void *stream);

/*
 * Measurement helpers: the achievable ceilings of the device, measured by
 * this library's own kernels (to state roofline fractions against both the
 * published peaks and what the device delivers).
 * spand_measure_bandwidth - mode 0: streaming copy of `bytes` (16-byte
 *   non-temporal loads and stores, grid-stride), *gbs = 2 bytes / median
 *   time of `reps` launches (read + write); mode 1: streaming read of
 *   `bytes`, *gbs = bytes / median time.  GB/s.  Allocates and frees the
 *   buffers (2 x bytes for a copy).
 * spand_measure_mfma - loops of independent matrix-core instructions on
 *   every CU: v_mfma_f32_32x32x2f32 (dtype SPAND_F32) or
 *   v_mfma_f64_16x16x4f64 (SPAND_F64); *tflops = flops / median time.
 */
int spand_measure_bandwidth(int32_t mode, size_t bytes, int reps, void *stream, double *gbs);
int spand_measure_mfma(int32_t dtype, int reps, void *stream, double *tflops);

/* spand_factor_stats - rank statistics per level (paper Figs. 4-5 report
 * ranks per level), apply bytes and algorithmic flops.  Host struct. */
int spand_factor_stats(spand_factor_t F, spand_factor_stats_t *out);

/* spand_destroy - release the factor and its device memory. NULL is ok. */
int spand_destroy(spand_factor_t F);

/*
 * spand_nd - host-only geometric nested dissection (no GPU use), exposed so
 * that the integer ordering can be checked exactly.  Recursive bisection
 * of the (i, j) grid (paper Sec. "Scalability study of spaND"), levels
 * 0..L-1 of interiors and interfaces (Sec. "Sparsified Nested Dissection
 * algorithm").  L <= 0 selects round(log2(K/32)) + 1.
 * Outputs (host, caller-allocated):
 *   h_node_of_elem[K], h_perm[K];
 *   h_ncl[L]              number of clusters per level;
 *   h_cl_ptr[sum(ncl)+L]  per level, ncl+1 offsets into that level's
 *                         element list (levels concatenated);
 *   h_cl_elems[L*K]       per level, K slots (only the first ptr[ncl] used);
 *   h_cl_key[2*sum(ncl)]  (node, box) per cluster;
 *   h_cl_interior[sum(ncl)].
 * Pass NULL for h_cl_* to query h_ncl only.  *L_out receives L.
 */
int spand_nd(const spand_grid_t *grid, int32_t L, int32_t *L_out,
             int32_t *h_node_of_elem, int32_t *h_perm, int32_t *h_ncl,
             int32_t *h_cl_ptr, int32_t *h_cl_elems, int32_t *h_cl_key,
             int32_t *h_cl_interior);

/*
 * spand_pool_trim - return every device block the library keeps cached.
 * Factorizations and solves take their device memory from a per-process
 * cache of blocks (sizes rounded up to 2 MiB, at most SPAND_POOL_MB MiB
 * cached, default 3/4 of the device memory) so that repeated builds and
 * solves neither call hipMalloc/hipFree again nor synchronise the device
 * for each release.
 * Blocks held by live factors are not affected.  Call with no library call
 * running on another thread.  Always returns SPAND_OK.
 */
int spand_pool_trim(void);

/* Status name ("SPAND_OK", ...). */
const char *spand_status_string(int status);
/* Message of the last error on the calling thread ("" if none). */
const char *spand_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SPAND_H */
