/*
 * pipesafe.h -- C ABI of the MI355X (gfx950) solver library libpipesafe.so.
 *
 * The library solves a nonsymmetric sparse system A x = b (Huynh & Suito,
 * "Communication-hiding pipelined BiCGSafe methods for solving large linear
 * systems", arXiv 2108.10591, Section 2) with one of four Krylov iterations:
 *
 *   PS_SSBICGSAFE2   ssBiCGSafe2, Algorithm 3: one reduction phase of nine
 *                    inner products per iteration, two sparse products.
 *   PS_PBICGSAFE     p-BiCGSafe, Algorithm 4: the products A r and A u of
 *                    Algorithm 3 are replaced by the recurrences of Section 3
 *                    (Eqs. (s), (q), (w), (l), (g)); the nine inner products
 *                    are independent of the product A s_i and are reduced
 *                    concurrently with it.
 *   PS_PBICGSAFE_RR  p-BiCGSafe-rr, Algorithm 5: p-BiCGSafe with the
 *                    recursively updated vectors reset to their true values
 *                    every m iterations while i < M (Section 4).
 *   PS_PBICGSTAB     pipelined BiCGStab (Cools & Vanroose), cited in the
 *                    paper's introduction and Table 1: two reduction phases,
 *                    each concurrent with one sparse product.
 *
 * All arithmetic is IEEE binary64 (the paper's experiments are in double
 * precision, Section 5).  Matrices are CSR with int32 column indices.
 *
 * Conventions shared by every entry point
 *   - Return value: PS_OK (0) or a negative ps_error.  On error, outputs are
 *     left untouched unless stated otherwise.  Not converging is NOT an error:
 *     the call returns PS_OK and reports it in *status.
 *   - The caller owns every pointer it passes; the library never frees or
 *     retains caller memory past the call.
 *   - A handle is not thread-safe: a call that finds the handle in use by
 *     another thread returns PS_EBUSY.
 *   - "host" pointers point to ordinary CPU memory, "device" pointers to GPU
 *     memory of the device the handle was created on.
 */
#ifndef PIPESAFE_H
#define PIPESAFE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ps_matrix ps_matrix; /* opaque: device CSR, workspace, streams */

enum ps_variant {
  PS_SSBICGSAFE2 = 0,
  PS_PBICGSAFE = 1,
  PS_PBICGSAFE_RR = 2,
  PS_PBICGSTAB = 3
};

/* outcome of a solve (Section 5: converged, or stopped at the iteration limit) */
enum ps_status {
  PS_CONVERGED = 0, /* ||r_i|| <= tol * ||r_ref||                                     */
  PS_MAXIT = 1,     /* reached i = maxit without converging                           */
  PS_BREAKDOWN = 2, /* a coefficient denominator was exactly zero or not finite       */
  PS_NONFINITE = 3  /* an inner product was NaN or infinite (e.g. NaN in b)           */
};

enum ps_error {
  PS_OK = 0,
  PS_EINVAL = -1, /* invalid argument (sizes, CSR structure, variant, options)        */
  PS_ENOMEM = -2, /* device or host allocation failed                                 */
  PS_EHIP = -3,   /* a HIP runtime call failed                                        */
  PS_EBUSY = -4,  /* the handle is in use by another thread                           */
  PS_ENODEV = -5, /* no usable gfx950 device                                          */
  PS_ETOOBIG = -6 /* the solve does not fit the static workspace (ps_solve_dev_static)   */
};

typedef struct {
  int32_t rr_m;        /* replacement period m of Algorithm 5 (default 100; Section 5.2).
                          <= 0 disables replacement. Ignored by other variants.          */
  int32_t rr_M;        /* no replacement at i >= M (Algorithm 5); <= 0 means maxit.     */
  int32_t norm_ref;    /* stop-test scale: 0 = ||r_0|| (the paper's criterion, default),
                          1 = ||b||.                                                     */
  int32_t batch_iters; /* iterations enqueued between host checks of the device stop
                          flag; 0 = automatic.  Iterations enqueued after the stop are
                          no-ops, so the result does not depend on this value.           */
  int32_t overlap;     /* 1: the reduction phase runs on a second stream concurrently
                          with the sparse product it is independent of; 0: everything
                          on one stream; -1 (default): on when one product streams at
                          least 128 MiB (shorter products cannot hide the cross-stream
                          waits); ps_info.auto_overlap tells.  Results are
                          bit-identical in every case.                                 */
  int32_t profile;     /* bit mask of ps_kernel classes to time with HIP events on the
                          stream each kernel runs on; 0 (default) = none.               */
  int32_t resume;      /* 0 (default): initialise from b and x0.  1: skip initialisation
                          and continue from the state loaded by ps_set_state /
                          ps_set_scalars, starting at iteration resume_iter.            */
  int32_t resume_iter;
  int32_t graph;       /* 1 (default): replay batches of identical iterations as cached
                          HIP graphs; 0: launch every kernel directly.  Results are
                          bit-identical either way.  Ignored while profiling.          */
  int32_t schedule;    /* Where the reduction phases run: p-BiCGSafe, p-BiCGSafe-rr and
                          (0 and 3 only) p-BiCGStab.  -1 (default): automatic --
                          sliced layout: 4 up to 1024 rows (p-BiCGSafe in FP64 from
                          x0; otherwise 3), else 3; CSR: 3 below 2^18 rows, else 0;
                          batches: 4 on the sliced layout when no system has more
                          than 1600 rows (same conditions; otherwise 2), else 2
                          (ps_info.auto_schedule tells); p-BiCGStab: 3 for one
                          system, 0 for batches; ssBiCGSafe2 ignores -1.
                          With -rr, a replacement step and the iteration after it form
                          their inner products in their own pass.
                          0: the reduction phase of Algorithm 4
                          as its own multi-inner-product pass, concurrent with A s_i.
                          1: fused inner products -- pass A and the epilogue of A w_i of
                          iteration i also form the per-block partial sums of the nine
                          inner products of iteration i+1 (Algorithms 3-5: (y,y), (y,r),
                          (r0*,r), (r0*,t), (r,r) from pass A; (s,s), (s,y), (s,r),
                          (r0*,s) from the epilogue), so that only their final sums and
                          the coefficients remain, concurrent with A s_{i+1}.  Reads
                          32n bytes more and skips the 40n-byte pass.
                          2: fused epilogue -- as 1, but a pass forms only w_i (Eqs.
                          (q), (w)) and the epilogue of A w_i makes every other update
                          of the iteration and all nine partial sums: 24n bytes fewer
                          than 1 (measured: equal to 1 within 1% up to 112^3 stencils,
                          5.5% faster at 128^3; slower than 0 on uneven CSR rows).
                          Batches: each system's partial sums are added by a workgroup
                          of its own.
                          3: as 2 on one stream: the product A s_i also performs the
                          reduction phase -- its first workgroups fold the partial
                          sums before their rows, and the last of them to finish
                          adds the folded sums and forms the stop test and the
                          coefficients -- so no fold or finish launch and no
                          cross-stream wait remain (overlap is then unused).  One
                          system only (batches: PS_EINVAL).  Measured: 7-14% faster
                          than 2 on stencils from 24^3 to 128^3 rows and on banded
                          CSR matrices up to 2*10^5 rows.
                          p-BiCGStab, 3: pass 1 also forms the partial sums of
                          (q,y), (y,y), (r0*,s), (r0*,z) and pass 2 those of
                          (r0*,r), (r0*,w), (r,r); the products A z_i and A w_{i+1}
                          fold and finish the two reduction phases the same way:
                          four launches per iteration on one stream, 40n bytes fewer
                          than the separate passes (0).
                          4: the whole solve in one workgroup per system (64-512
                          threads, by the rows per system and how many systems run;
                          Algorithm 4 with schedule 3's reduction phase; one launch
                          per solve, barriers between the phases that gather):
                          p-BiCGSafe only, FP64, sliced layout with one row per lane,
                          no resume or profiling, at most 2^20 rows per system, one
                          system or a batch; otherwise PS_EINVAL.  Systems of at
                          most two rows per thread and at most 8 entries per row keep
                          their rows in registers and s, w in LDS.  Measured: faster
                          than 3 up to about 1000 rows (256 rows: 5.7 against 16.1
                          us per iteration; 1024: 11.5 against 17.6), far slower
                          above (4096 rows: 43.3 against 17.9), where one CU's
                          bandwidth bounds it; batches of systems up to 40^2 rows:
                          1.4-3.5x the solves/s of 2.
                          Results are bit-identical to schedule 0.  ssBiCGSafe2: 1, 2,
                          3 and 4 are PS_EINVAL; p-BiCGStab: 1, 2 and 4.               */
  int32_t x0_fallback; /* What to do with a given x0 (per system for a batch).
                          0 (default): use it as given.
                          1: if ||b - A x0|| > ||b|| (or is not finite), start from
                          x0 = 0 instead: a guess that is worse than zero costs nothing.
                          2: first replace x0 by c x0, c = (A x0, b) / (A x0, A x0), the
                          multiple with the least residual ||b - c A x0|| (<= ||b|| in
                          exact arithmetic; x0 = 0 when c cannot be formed), then the
                          rule of 1.  The inner products are rounded once from their
                          exact values.  The set-up's residual statements (x0 of
                          Algorithms 3-5) decide; r_0 = b - A x0 of the guess used.
                          Other values: PS_EINVAL.                                     */
  int32_t precision;   /* ps_precision: the matrix values the products read.
                          PS_PREC_FP64 (default): the FP64 values.  PS_PREC_FP32_MATRIX:
                          every product reads the values rounded to the nearest FP32
                          number (ties to even), so the system solved is that rounded
                          matrix.  PS_PREC_FP32_KRYLOV: the residual statements
                          (r_0 = b - A x_0, the x0_fallback test and the true residual of
                          p-BiCGSafe-rr's replacement steps, Algorithm 5) read the FP64
                          values, every other product the rounded ones; with
                          PS_PBICGSAFE_RR the replacement steps re-anchor the iteration
                          to the FP64 system (a solve that stops before its first
                          replacement is only as accurate as the rounded matrix).
                          Vectors, inner products, coefficients and x are FP64 in these
                          modes (PS_PREC_FP32_VECTORS below also stores p, u, z in FP32).
                          The FP32 copy is made on the device at the first such
                          solve (4 bytes per stored value) and kept; a value beyond the
                          FP32 range makes these modes PS_EINVAL.                      */
  void *stream;        /* hipStream_t on which the solve orders its work (e.g. the
                          caller's current stream).  NULL: ps_solve_dev uses the null
                          stream, ps_solve the library's own stream.                   */
} ps_options;

/* ps_options.precision */
enum ps_precision {
  PS_PREC_FP64 = 0,
  PS_PREC_FP32_MATRIX = 1,
  PS_PREC_FP32_KRYLOV = 2,
  PS_PREC_FP32_VECTORS = 3 /* PS_PREC_FP32_KRYLOV, and the search directions p, u and the
                              vector z of p-BiCGSafe(-rr) held as FP32 numbers: each rounded
                              to the nearest FP32 number when formed and widened exactly
                              when read (all arithmetic FP64); other variants: PS_EINVAL.
                              Only the replacement steps bring the iterate back to the FP64
                              system, so the replacement period bounds the accuracy.  The
                              state functions convert p, u, z to and from FP64.          */
};

/* device layout of the matrix, chosen by ps_create (ps_info.format) */
enum ps_format {
  PS_FMT_CSR = 0,  /* the caller's CSR (int32 row pointer and columns, FP64 values),
                      cut into row blocks whose products fit the LDS                  */
  PS_FMT_SELL = 1  /* sliced ELLPACK: slices of 64 consecutive rows stored column by
                      column, each row in its CSR order and padded to the slice's
                      longest row (padding is skipped, never multiplied).  Chosen when
                      the padded size is at most 1.10 nnz (stencil-like matrices).
                      Same products, same summation order, same results as CSR.      */
};

/* what ps_create built, for ps_matrix_info */
typedef struct {
  int32_t format;        /* ps_format                                                   */
  int32_t spmv_shape;    /* CSR product shape 0..4 (lanes per row, LDS budget); -1 SELL */
  int64_t n, nnz;         /* as given to ps_create / ps_create_batch                     */
  int64_t slots;         /* stored matrix entries including padding (= nnz for CSR)     */
  int32_t spmv_blocks;   /* workgroups of one sparse product                            */
  int32_t dot_grid;      /* workgroups of the multi-inner-product kernel                */
  int64_t matrix_bytes;  /* bytes one sparse product must stream from the matrix arrays:
                            CSR (8 + index_bits/8 + 2 gather_sort) nnz + 4 (n+1);
                            SELL (8 + index_bits/8) slots + 4 (slices+1)               */
  int32_t auto_overlap;  /* what ps_options.overlap = -1 resolves to on this matrix     */
  int32_t auto_schedule; /* what ps_options.schedule = -1 resolves to for p-BiCGSafe (4 is
                            3, for batches 2, with p-BiCGSafe-rr and with the options
                            schedule 4 excludes) */
  int32_t nsys;          /* systems (1 unless created by ps_create_batch)              */
  int32_t streaming;     /* 1: p-BiCGSafe(-rr)'s update passes load and store the vectors that
                            no kernel reads before the next iteration with streaming
                            (nontemporal) hints -- when an iteration moves at least
                            512 MiB (two products plus 272 bytes per row), or as
                            PIPESAFE_STREAM=0|1 sets; the results are the same.
                            p-BiCGStab's passes and ssBiCGSafe2's epilogue do the same
                            from 640 MiB by that count (not reported here).            */
  int64_t n_padded;      /* rows on the device: n, or for a batch the systems padded to
                            multiples of 512 rows                                      */
  int32_t index_bits;    /* stored column index: 32, or 16 when every entry fits --
                            sliced layout: column - row within 32767; CSR: column -
                            the first row of its row block within 32767 -- 10 instead
                            of 12 bytes per FP64 entry (PIPESAFE_INDEX=32 keeps 32)    */
  int32_t gather_sort;    /* CSR: 1 when row blocks are stored in column order
                            (ps_layout.gather_sort; +2 bytes per entry)              */
} ps_info;

/* classes of kernels, for ps_options.profile and ps_kernel_stats */
enum ps_kernel {
  PS_K_SPMV = 0,        /* sparse product with no fused work (A s_i, A z_i, and the
                           products A o, A u, A t, A y, A r of a replacement step)       */
  PS_K_DOTS = 1,        /* multi-inner-product kernel (per-block partial sums)          */
  PS_K_UPDATE = 2,      /* fused vector-update pass                                      */
  PS_K_SPMV_FUSED = 3,  /* sparse product with a fused update epilogue (A w_i, A u_i,
                           and b - A x of a replacement step)                            */
  PS_K_OTHER = 4,       /* set-up, replacement and bookkeeping kernels                   */
  PS_K_DOTS_FINISH = 5, /* one-block finish: final sums, coefficients, stop test         */
  PS_K_COUNT = 6
};

/* state vectors, for ps_get_state / ps_set_state (names follow Algorithms 3-5;
   for PS_PBICGSTAB: s = A p, z = A s, w = A r, t = A w, v = A z, q = r - alpha s,
   y = A q).  Each is double[n].  p-BiCGSafe keeps q_i and o_i in registers (q_i
   is formed in pass A and again in the epilogue of A w_i), so their slots hold
   values only after a replacement step (A o_i, o_i) or in the other variants. */
enum ps_vec {
  PS_V_X = 0, PS_V_R, PS_V_RS /* r0* */, PS_V_S, PS_V_Y, PS_V_T, PS_V_P, PS_V_U, PS_V_Z,
  PS_V_W, PS_V_L, PS_V_G, PS_V_Q, PS_V_O, PS_V_AS, PS_V_V, PS_V_B, PS_V_COUNT
};

/* scalar state, for ps_get_scalars / ps_set_scalars (double[PS_S_COUNT]) */
enum ps_scalar {
  PS_S_ALPHA = 0,  /* alpha of the last coefficient update (p-BiCGStab: alpha_i)         */
  PS_S_BETA,       /* beta used in p_i                                                   */
  PS_S_ZETA,
  PS_S_ETA,
  PS_S_OMEGA,      /* p-BiCGStab: omega_{i-1}                                            */
  PS_S_F,          /* (r0*, r) of the last coefficient update                           */
  PS_S_RHOREF,     /* squared stop-test scale (||r_0||^2 or ||b||^2)                      */
  PS_S_RHO,        /* (r_i, r_i) of the last reduction phase                             */
  PS_S_PENDING,    /* p-BiCGStab: 1 if alpha_i/beta_{i-1} could not be formed            */
  PS_S_GS,         /* p-BiCGStab: (r0*, s), (r0*, w), (r0*, z) of the last phase          */
  PS_S_GW,
  PS_S_GZ,
  PS_S_COUNT
};

/* Fill *opt with the defaults documented above. */
void ps_default_options(ps_options *opt);

/*
 * Create a solver handle for the n x n CSR matrix (rowptr, col, val), all HOST
 * pointers: rowptr int64[n+1], col int32[nnz], val double[nnz].  The matrix is
 * copied to the current HIP device; the caller may free its arrays on return.
 * Validation: n >= 1, nnz = rowptr[n] < 2^31, rowptr[0] = 0, rowptr
 * non-decreasing, 0 <= col < n, val finite; otherwise PS_EINVAL.  Columns need
 * not be sorted; duplicate (row, col) entries are summed; empty rows are
 * allowed (they make A singular).  The device layout (ps_format) and the
 * product's launch shape are chosen here from the row lengths; the
 * environment variables PIPESAFE_FORMAT (0 CSR, 1 SELL), PIPESAFE_SELL_RPL
 * (rows per lane of the sliced layout: 1, the default, or 2 with 128-row
 * slices), PIPESAFE_INDEX (32: no 16-bit column offsets), PIPESAFE_CSR_SORT
 * (0 or 1: the CSR gather order),
 * PIPESAFE_SPMV_SHAPE (0..4), PIPESAFE_DOT_GRID (1..8192 workgroups) and
 * PIPESAFE_STREAM (0 or 1, ps_info.streaming) override the choices, for
 * tuning and tests.  Every choice gives
 * the same results.
 */
int ps_create(ps_matrix **out, int64_t n, int64_t nnz, const int64_t *rowptr, const int32_t *col,
              const double *val);

/* An explicit device layout (ps_create_ex, ps_create_batch_ex); -1 in a field
   keeps the automatic choice for it. */
typedef struct ps_layout {
  int32_t format;             /* PS_FMT_CSR or PS_FMT_SELL (any padding)            */
  int32_t sell_rows_per_lane; /* sliced layout: 1 (64-row slices) or 2 (128-row)    */
  int32_t spmv_shape;         /* CSR launch shape 0..4: (nonzeros per thread, lanes
                                 per row) = (4,1) (8,1) (16,4) (16,8) (16,16)        */
  int32_t index_bits;         /* 32 keeps 32-bit columns; 16 (or -1) stores 16-bit
                                 offsets where every entry fits (sliced: column -
                                 row; CSR: column - first row of its row block)      */
  int32_t gather_sort;        /* CSR: 1 stores each row block's entries in column
                                 order (with each one's place in the block's row
                                 order, 2 bytes), so that a wave's gathers of x touch
                                 few cache lines; 0 row order; -1 automatic: 1 when a
                                 typical block's columns span more than 4096       */
} ps_layout;

/* ps_create / ps_create_batch with an explicit layout (NULL: automatic, as
   they are); the layout overrides the environment variables above.  Results
   do not depend on the layout.  PS_EINVAL also for a field out of range. */
int ps_create_ex(ps_matrix **out, int64_t n, int64_t nnz, const int64_t *rowptr,
                 const int32_t *col, const double *val, const ps_layout *layout);
int ps_create_batch_ex(ps_matrix **out, int32_t nsys, const int64_t *sys_ptr, int64_t n,
                       int64_t nnz, const int64_t *rowptr, const int32_t *col, const double *val,
                       const ps_layout *layout);

/*
 * Autotuner.  Every layout, launch shape and schedule computes the same
 * iterates (inner products rounded once from their exact value), so the
 * tuner picks by measured time only.
 */
#define PS_TUNE_MAX 48
typedef struct ps_tune_entry {
  ps_layout layout;     /* the layout timed (ps_autotune_layout), else all -1            */
  int32_t schedule;     /* the options timed (ps_tune_options), else -1                  */
  int32_t overlap;
  int32_t streaming;
  int32_t batch_iters;
  double us;            /* microseconds per iteration                                   */
} ps_tune_entry;
typedef struct ps_tune_report {
  int32_t count;        /* entries filled                                               */
  int32_t best;         /* index of the chosen entry                                    */
  ps_tune_entry entry[PS_TUNE_MAX];
} ps_tune_report;

/* Create the matrix in every candidate layout -- the sliced layout with 1 and 2
   rows per lane and 16- and 32-bit columns (where its padding stays within
   1.5x the nonzeros), CSR with each of the 5 launch shapes in row order and in
   gather order -- time `reps` iterations of p-BiCGSafe on each (b = 1, x0 = 0,
   tol = 0, default options, so the automatic schedule of that layout; run
   once to capture the graphs, then timed with the host clock around the
   call), and keep the fastest: *out receives that handle, the others are
   destroyed.  Every layout computes the same iterates, so a system that
   stops early (a breakdown at b = 1) stops at the same iteration in each.
   nsys = 1 (sys_ptr ignored) for one system, else the batch arguments of
   ps_create_batch.  report: NULL or HOST, filled with every timed layout.
   Costs one creation per candidate (host layout build and upload). */
int ps_autotune_layout(ps_matrix **out, int32_t nsys, const int64_t *sys_ptr, int64_t n,
                       int64_t nnz, const int64_t *rowptr, const int32_t *col, const double *val,
                       int32_t reps, ps_tune_report *report);

/* Time `iters` iterations of `variant` from b_dev (DEVICE, the caller's row
   order, as ps_solve_batch_dev; x0 = 0, tol = 0) for every combination of
   schedule (p-BiCGSafe(-rr): 0, 1, 2, and 3 for one system; p-BiCGStab: 0,
   and 3 for one system; 4 where the options allow it), overlap (0, 1;
   ssBiCGSafe2, schedules 3 and 4: 0), streaming update passes (p-BiCGSafe(-rr):
   off, on; schedule 4: as the handle has it) and graph batch (8, 16, 32
   iterations; schedule 4: one launch), each run once to capture its graphs and once timed (host
   clock around the call), and write the fastest into opt->schedule,
   opt->overlap and opt->batch_iters (the other fields of *opt are the base
   of every run and stay as given).  The streaming choice is stored in the
   handle and applies to its later solves.  report: NULL or HOST. */
int ps_tune_options(ps_matrix *A, const double *b_dev, int32_t variant, int32_t iters,
                    ps_options *opt, ps_tune_report *report);

/*
 * Solve A x = b from HOST buffers.  b: double[n]; x0: double[n] or NULL (zero,
 * the paper's x_0); x: double[n] output, x_{iters}.  tol: the run stops when
 * ||r_i|| <= tol * ||r_ref|| (Section 5 uses 1e-8 and ||r_0||).  maxit >= 0: at
 * i = maxit the run stops with PS_MAXIT.  variant: ps_variant.  opt: NULL for
 * defaults.  hist: NULL or double[maxit+1]; receives hist[k] = ||r_k||/||r_ref||
 * for k = 0..iters from the recursively updated residual (the quantity
 * Algorithms 3-5 test).  iters: the number of x updates made.  status:
 * ps_status.  PS_EINVAL for a bad variant, negative maxit, negative or NaN tol.
 */
int ps_solve(ps_matrix *A, const double *b, const double *x0, double tol, int32_t maxit,
             int32_t variant, const ps_options *opt, double *x, int32_t *iters, double *hist,
             int32_t *status);

/*
 * As ps_solve, with b, x0 (or NULL) and x in DEVICE memory; hist, iters and
 * status are HOST pointers.  Work is ordered on opt->stream (or the library's
 * stream); the call returns after the solve has finished on the device.
 */
int ps_solve_dev(ps_matrix *A, const double *b_dev, const double *x0_dev, double tol, int32_t maxit,
                 int32_t variant, const ps_options *opt, double *x_dev, int32_t *iters,
                 double *hist, int32_t *status);

/*
 * ps_solve_dev for callers that cannot allocate device memory (serving loops,
 * harnesses that forbid hipMalloc): same arguments and results, bit for bit,
 * but the call allocates nothing.  The solve's scalar and control blocks,
 * inner-product partial sums and residual history live in a static device
 * workspace of 4 MiB (524,288 doubles) that each GPU holds for the life of the
 * process; the handle's vectors and matrix were allocated by ps_create.
 * Limits: it needs 32 + 32 + 27 (G + ceil(G/256)) + 3 (5 max(ceil(n/512), P) + 4 P + 9 F) +
 * maxit + 2 doubles (each term rounded up to a multiple of 32), where G, P, F
 * are ps_info.dot_grid, ps_info.spmv_blocks and ceil(max(ceil(n/512), P)/256)
 * -- about 0.11 n + maxit doubles on the sliced layout (2.1M rows with maxit =
 * 10000 fit); beyond that PS_ETOOBIG.  PS_EINVAL also for a batch handle, for
 * opt->resume or opt->profile set, and for a mixed precision before the handle's
 * FP32 values exist (the first mixed-precision ps_solve* makes them).  Batches
 * of iterations are launched directly (opt->graph is ignored).  Every call on a
 * GPU uses that GPU's one workspace: calls that overlap in time on one GPU (from
 * several threads, or on streams that run concurrently) race and must not be
 * made.  ps_get_scalars after this call returns the scalars of the handle's last
 * other solve, not this one's.
 */
int ps_solve_dev_static(ps_matrix *A, const double *b_dev, const double *x0_dev, double tol,
                        int32_t maxit, int32_t variant, const ps_options *opt, double *x_dev,
                        int32_t *iters, double *hist, int32_t *status);

/*
 * Batched systems: nsys independent systems A_k x_k = b_k given as one
 * block-diagonal CSR (HOST pointers as in ps_create, global column indices);
 * sys_ptr int64[nsys+1]: the rows of system k are sys_ptr[k] .. sys_ptr[k+1]-1
 * (sys_ptr[0] = 0, strictly increasing, sys_ptr[nsys] = n), and every column of
 * those rows lies in the same range; otherwise PS_EINVAL.  Each system is
 * solved exactly as ps_solve would solve it alone (same iterations, residual
 * history and solution bits), but all systems share every kernel launch: each
 * is padded on the device to a multiple of 512 rows with empty rows, each has
 * its own coefficients, stop test and iteration count, and a system that has
 * stopped makes its share of every later launch a no-op.  ps_solve,
 * ps_solve_dev, ps_spmv_dev and the state functions return PS_EINVAL on a
 * batch handle (nsys > 1); nsys = 1 gives an ordinary handle.
 */
int ps_create_batch(ps_matrix **out, int32_t nsys, const int64_t *sys_ptr, int64_t n, int64_t nnz,
                    const int64_t *rowptr, const int32_t *col, const double *val);

/*
 * Solve every system of a batch handle (or the one system of a handle).
 * b, x0 (NULL: zero), x: HOST double[n] in the caller's row order; iters,
 * status: HOST int32[nsys] per system (as in ps_solve); hist: NULL or HOST
 * double[nsys * (maxit+1)], row k holding system k's history (entries past
 * iters[k] are undefined).  opt as in ps_solve, except: resume is not
 * supported (PS_EINVAL) and schedule -1 means 2 for nsys > 1.
 * The solve runs until every system has stopped.
 */
int ps_solve_batch(ps_matrix *A, const double *b, const double *x0, double tol, int32_t maxit,
                   int32_t variant, const ps_options *opt, double *x, int32_t *iters, double *hist,
                   int32_t *status);
/* ps_solve_batch with b, x0, x DEVICE double[n] (iters, status, hist on the host),
   ordered on opt->stream as ps_solve_dev. */
int ps_solve_batch_dev(ps_matrix *A, const double *b_dev, const double *x0_dev, double tol,
                       int32_t maxit, int32_t variant, const ps_options *opt, double *x_dev,
                       int32_t *iters, double *hist, int32_t *status);

/* y = A x with x, y DEVICE double[n] (x and y must not overlap), ordered on
   `stream` (hipStream_t, NULL = the null stream); returns after completion. */
int ps_spmv_dev(ps_matrix *A, const double *x_dev, double *y_dev, void *stream);

/* Copy state vector `which` (ps_vec) of the last solve into HOST double[n]. */
int ps_get_state(ps_matrix *A, int32_t which, double *host_out);
/* Load state vector `which` from HOST double[n] (for opt.resume). */
int ps_set_state(ps_matrix *A, int32_t which, const double *host_in);
/* Copy / load the scalar state, HOST double[PS_S_COUNT]. */
int ps_get_scalars(ps_matrix *A, double *host_out);
int ps_set_scalars(ps_matrix *A, const double *host_in);

/* Describe the handle's device layout (HOST *info).  PS_EINVAL on NULL. */
int ps_matrix_info(ps_matrix *A, ps_info *info);

/* Kernel timing of the last solve run with opt.profile != 0: total milliseconds
   and launch count of class `cls` (ps_kernel), measured with HIP events around
   each launch on its own stream.  Only launches of iterations before the
   stopping one are counted (later launches may be no-ops). */
int ps_kernel_stats(ps_matrix *A, int32_t cls, double *total_ms, int64_t *launches);

/* Of the launches ps_kernel_stats counts for class `cls`, how many were enqueued
   on the library's second stream (the reduction phases that run concurrently
   with a sparse product, Section 3; ps_options.overlap).  HOST *aux_launches. */
int ps_kernel_streams(ps_matrix *A, int32_t cls, int64_t *aux_launches);

/* Device copy dst = src of `bytes` bytes (DEVICE pointers, 16-byte aligned,
   bytes a multiple of 16) with a plain streaming kernel of the library's own;
   used to calibrate bandwidth counters and the copy ceiling.  Ordered on
   `stream`; returns after completion. */
int ps_stream_copy(void *dst, const void *src, int64_t bytes, void *stream);

/* Release the handle and all device memory it owns.  NULL is accepted. */
int ps_destroy(ps_matrix *A);

/* Static description of a ps_error or ps_status code. */
const char *ps_strerror(int code);

/* Library version string. */
const char *ps_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PIPESAFE_H */
