/*
 * ckkt.h -- condensed-space KKT solves on one MI355X (gfx950).
 *
 * The library computes the Newton direction of the condensed KKT system of
 * an interior-point method (Pacaud, Shin, Montoison, Schanen, Anitescu,
 * "Condensed interior-point methods for scalable nonlinear programming on
 * GPUs", arXiv 2405.14236) in its two Cholesky-based forms:
 *
 *   LiftedKKT (Sec. 3.2, eq:liftedkkt): equalities are relaxed into tight
 *     inequality rows, J = [G; H], and
 *         K_tau d_x = b,   K_tau = W + diag(sigma_x) + J^T diag(sigma_s) J.
 *
 *   HyKKT (Sec. 3.1, eq:kkt:hykkt and eq:kkt:schurcomplhykkt):
 *         K1 = [[K, G^T], [G, 0]] (d_x, d_y) = (rbar1, rbar2),
 *         K  = W + diag(sigma_x) + H^T diag(sigma_s) H,
 *     solved through the Cholesky factor of K_gamma = K + gamma G^T G and
 *     conjugate gradient on S_gamma = G K_gamma^{-1} G^T.
 *
 * sigma_x plays the role of delta_w I (any nonnegative diagonal) and
 * sigma_s the role of D_H = (D_s + delta_w I) C with delta_c = 0
 * (Sec. 2.2, K1; Remark 1).
 *
 * Call sequence:  ckkt_analyze (host symbolic analysis, once per pattern)
 *              -> ckkt_bind_workspace (caller-allocated device memory)
 *              -> { ckkt_factorize (values, sigma, gamma)
 *                   -> ckkt_solve (rhs) ... } repeated for every new system.
 *
 * Conventions for every entry point:
 *  - All functions return a ckkt_status (0 = success, < 0 = error); none
 *    aborts, throws or prints.
 *  - Pattern arrays (ckkt_pattern) are HOST memory, read during
 *    ckkt_analyze only; the library keeps its own copies.
 *  - Value, diagonal, right-hand-side and solution pointers are DEVICE
 *    memory owned by the caller.  They are used by work enqueued on the
 *    caller's stream; factor values must stay unchanged until the last
 *    ckkt_solve that uses the factor has returned (the refinement applies
 *    K unassembled from them).
 *  - After ckkt_bind_workspace the library allocates no device memory; it
 *    writes only into the bound workspace and the caller's output arrays.
 *  - Matrices are CSR with int32 indices, column indices strictly
 *    increasing inside each row; W is given by its lower triangle
 *    (column <= row) and must hold every diagonal entry it has.
 *  - One handle is used by one host thread / one stream at a time.
 */
#ifndef CKKT_H
#define CKKT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ckkt_status;
#define CKKT_OK                  0
#define CKKT_ERR_ARG            -1  /* bad argument (null pointer, negative size, bad enum) */
#define CKKT_ERR_PATTERN        -2  /* malformed CSR: unsorted, duplicate, out of range, W upper entry */
#define CKKT_ERR_NOT_SPD        -3  /* a Cholesky pivot was not positive; see ckkt_info.failed_column
                                       (n: the capacitance matrix of the split dense rows) */
#define CKKT_ERR_NO_CONVERGENCE -4  /* refinement or CG did not reach the tolerance within its limit */
#define CKKT_ERR_BREAKDOWN      -5  /* CG breakdown (p^T S p <= 0 or not finite) */
#define CKKT_ERR_STATE          -6  /* call out of order (solve before factorize, no workspace, ...) */
#define CKKT_ERR_HIP            -7  /* a HIP runtime call failed */
#define CKKT_ERR_WORKSPACE      -8  /* workspace missing, too small or misaligned */
#define CKKT_ERR_NONFINITE      -9  /* NaN or Inf in an input that reaches the assembled matrix
                                       (ckkt_factor_status and the solves report it) or in a
                                       right-hand side (the solves) */
#define CKKT_ERR_TIMEOUT       -10  /* a dependency wait inside a triangular sweep exceeded its time
                                       limit (seconds); the results of that solve are invalid.  Reported
                                       by the next call that synchronizes (ckkt_solve, ckkt_pcg_solve,
                                       ckkt_factor_status) and cleared by ckkt_factorize. */
#define CKKT_ERR_HOST_MEMORY   -11  /* host memory or another host resource (a thread) ran out during
                                       analysis, plan I/O or the host factor-solve */

/* Formulations (Sec. 3). */
#define CKKT_LIFTED 0
#define CKKT_HYKKT  1

/* Precision of the Cholesky factor.  Residuals, refinement updates, CG
 * vectors, dot products and the gamma-scaled terms are FP64 in both.
 * CKKT_FP32_IR factors the Jacobi-scaled matrix in FP32 (static pivoting)
 * and refines in FP64; the solve gives the FP32 factor up for an FP64
 * refactorization when it cannot reach opt.tol: at once when a pivot was
 * floored or the first FP32 solve has omega > 0.1 (the FP32 error grows
 * with the largest diagonal weights, Sec. 4), else after Richardson and PCG
 * around it stagnate.  After such a system the next 4 factorizations of the
 * handle are FP64 from the start (8, 16, .. 64 while failures repeat;
 * info->fallback = 8 on their solves), then FP32 is tried again. */
#define CKKT_FP64    0
#define CKKT_FP32_IR 1

/* Fill-reducing orderings (host analysis). */
#define CKKT_ORDER_AMD     0  /* approximate minimum degree */
#define CKKT_ORDER_NATURAL 1  /* identity (tests and tiny inputs) */

typedef struct {
    int64_t n;            /* primal variables */
    int64_t m_eq;         /* equality rows (G) */
    int64_t m_ineq;       /* inequality rows (H) */
    const int32_t *w_ptr, *w_idx;   /* W lower triangle, n+1 / nnz(W) */
    const int32_t *g_ptr, *g_idx;   /* G, m_eq+1 / nnz(G); may be NULL when m_eq == 0 */
    const int32_t *h_ptr, *h_idx;   /* H, m_ineq+1 / nnz(H); may be NULL when m_ineq == 0 */
    int32_t formulation;            /* CKKT_LIFTED or CKKT_HYKKT */
} ckkt_pattern;

typedef struct {
    int32_t precision;    /* CKKT_FP64 (default) or CKKT_FP32_IR */
    int32_t ordering;     /* CKKT_ORDER_AMD (default) */
    double  tol;          /* residual gate: componentwise relative backward
                             error (see ckkt_solve); default 1e-10 */
    int32_t ir_maxit;     /* refinement steps after the first solve; default 10 */
    double  cg_tol;       /* HyKKT CG: stop when ||r_k||_2 <= cg_tol ||r_0||_2; default 1e-10 */
    int32_t cg_maxit;     /* HyKKT CG iteration limit; default min(m_eq, 1000) when <= 0 */
    int32_t relax;        /* supernode amalgamation: 0 off, 1 default */
    int32_t lds_front_max;/* largest front order factored entirely in LDS by one
                             workgroup; larger fronts take the tiled
                             multi-workgroup path.  0 = what 160 KiB of LDS
                             holds in FP64 (140), in both precisions. */
    int32_t learned;      /* 1: reserve workspace for the learned preconditioner
                             (features, MLP cache, stale-system references) */
    int32_t dense_row_min;/* rows of J = [G; H] with at least this many nonzeros
                             are kept out of the condensed matrix, whose pattern
                             one dense row would fill (Sec. 1, Sec. 2.2): the factor is
                             that of K_s = K - J_d^T D_d J_d, and every
                             application of K^{-1} adds the Woodbury correction
                             of the k split rows (K_s^{-1} J_d^T and the k x k
                             capacitance D_d^{-1} + J_d K_s^{-1} J_d^T, formed
                             on the device by each factorization).  Needs
                             K_s positive definite (it is when W + sigma_x is).
                             0 (default) = no split.  FP64 single-system
                             handles only (else CKKT_ERR_ARG from
                             ckkt_analyze), at most 64 split rows. */
} ckkt_options;

typedef struct {
    int64_t n, m_eq, m_ineq;
    int64_t nnz_k;            /* lower triangle of K (incl. diagonal) */
    int64_t nnz_l;            /* structural nonzeros of the Cholesky factor */
    int64_t nnz_l_stored;     /* stored entries (supernode panels incl. explicit zeros) */
    double  factor_flops;     /* algorithmic flops of the factorization (true structure) */
    double  assembly_products;/* J products summed by the assembly */
    int32_t n_supernodes;
    int32_t n_levels;         /* height of the supernodal assembly tree */
    int32_t max_front;        /* largest frontal matrix order */
    int32_t n_big_fronts;     /* fronts factored by the tiled (multi-workgroup) path */
    int64_t workspace_bytes;
    double  analyze_seconds;
    int32_t failed_column;    /* a column with a non-positive pivot (original
                                 numbering; an FP64 factorization stops after the
                                 level of fronts that meets the first one), -1 if
                                 none; valid after a solve or ckkt_factor_status */
    int32_t n_dense_rows;     /* rows split off by opt.dense_row_min */
    int32_t n_instances;      /* instances of a batch (1 for a single pattern) */
    int32_t pad;
    double  order_seconds;    /* part of analyze_seconds up to the ordering (pattern, AMD) */
    double  symbolic_seconds; /* part spent in the steps ckkt_analyze_device runs on the GPU
                                 (0 for a plan from ckkt_plan_load) */
} ckkt_info;

typedef struct {
    int32_t status;           /* same as the return value */
    int32_t refine_steps;     /* refinement steps taken after the first solve (outer steps for HyKKT) */
    int32_t cg_iters;         /* total CG iterations (HyKKT) */
    int32_t pcg_iters;        /* total PCG iterations (FP32 fallback path) */
    int32_t fallback;         /* 0 none, 1 PCG around the FP32 factor, 2 FP64 refactorization,
                                 8 factorized in FP64 from the start after an earlier FP32
                                 failure (FP32_IR handles); ckkt_batch_factorize_solve adds 4
                                 when its device steps did not reach opt.tol and the
                                 refinement of ckkt_solve took over */
    int32_t pad;
    double  omega;            /* final componentwise relative backward error */
    double  rho;              /* final unscaled ||r||_inf / ||rhs||_inf */
} ckkt_solve_info;

typedef struct ckkt_handle ckkt_handle;

/* Fills *opt with the defaults listed above. */
void ckkt_default_options(ckkt_options* opt);

/* Host symbolic analysis (Sec. 2.2 K1 / Sec. 3: the condensed pattern is
 * pattern(W) U diag U pattern(J^T J) for LiftedKKT and the same union with
 * G^T G for HyKKT, so both formulations share one analysis).  Computes the
 * fill-reducing ordering, elimination tree, supernodes, assembly maps and
 * level schedule, and the device workspace size.
 *   pat, opt : host; opt may be NULL for defaults.
 *   out      : receives a new handle (free with ckkt_destroy).
 *   workspace_bytes : receives the size ckkt_bind_workspace needs.
 * Errors: CKKT_ERR_ARG, CKKT_ERR_PATTERN (nothing is allocated then). */
ckkt_status ckkt_analyze(const ckkt_pattern* pat, const ckkt_options* opt,
                         ckkt_handle** out, size_t* workspace_bytes);

/* Checkpoint and resume of the symbolic phase (the analysis is done once
 * per pattern and reused across factorizations, the reuse Sec. 6.1.1 counts
 * on).  ckkt_plan_size gives the bytes of a serialized plan
 * of handle h (single system or batch); ckkt_plan_save writes it into a
 * HOST buffer of at least that size; ckkt_plan_load builds a new handle from
 * such a buffer without analysing the pattern again (same meaning of opt,
 * out and workspace_bytes as ckkt_analyze).  The options that shaped the
 * plan (ordering, relax, LDS front limit, dense_row_min) and the
 * formulation are taken from the plan; the others (precision, tolerances,
 * learned) from opt.  The buffer carries a magic word, a format version and
 * an FNV-1a checksum: a truncated, corrupted or foreign buffer gives
 * CKKT_ERR_ARG.  A plan is tied to this library's format version, and its
 * contents are trusted: load only buffers written by ckkt_plan_save (the
 * checksum catches corruption, not tampering). */
ckkt_status ckkt_plan_size(const ckkt_handle* h, size_t* bytes);
ckkt_status ckkt_plan_save(const ckkt_handle* h, void* buf, size_t bytes);
ckkt_status ckkt_plan_load(const void* buf, size_t bytes, const ckkt_options* opt, ckkt_handle** out,
                           size_t* workspace_bytes);

/* The same analysis with the symbolic factorization on the GPU (Sec. 1:
 * the solver orders on the host and factors symbolically on the device).
 * The host builds the pattern and the AMD ordering; kernels on `stream`
 * compute the elimination tree (atomic-minimum climb of the pattern's
 * entries to a fixed point), its postorder (Euler tour ranked by pointer
 * jumping), the K lower CSC, the column counts of L (row-subtree counting
 * with nearest common ancestors), the front row lists, the child-to-parent
 * and K-to-front positions and the K slots of the assembly products; the
 * host keeps the supernode amalgamation, the arena layout and the level
 * schedule.  The plan equals ckkt_analyze's element by element.  The call
 * allocates and frees device memory (about 8 bytes per K entry and per
 * product, plus 4 * ceil(log2 n) bytes per variable for the ancestor
 * table) and returns after `stream` is idle.  Same arguments and errors as
 * ckkt_analyze (ckkt_batch_analyze for the batched form), plus
 * CKKT_ERR_HIP when a HIP call fails. */
ckkt_status ckkt_analyze_device(const ckkt_pattern* pat, const ckkt_options* opt, void* stream,
                                ckkt_handle** out, size_t* workspace_bytes);
ckkt_status ckkt_batch_analyze_device(int32_t count, const ckkt_pattern* pats, const ckkt_options* opt,
                                      void* stream, ckkt_handle** out, size_t* workspace_bytes);

/* Batched analysis: `count` independent systems analysed as one
 * block-diagonal system.  Value arrays passed to ckkt_factorize and
 * ckkt_solve are the per-instance arrays concatenated in instance order
 * (W values, G values, H values, sigma_x, sigma_s, rhs, sol), and every
 * instance must reach the tolerance on its own. All patterns must have the
 * same formulation. */
ckkt_status ckkt_batch_analyze(int32_t count, const ckkt_pattern* pats,
                               const ckkt_options* opt, ckkt_handle** out,
                               size_t* workspace_bytes);

/* Binds `bytes` of caller-owned device memory at `dev_ptr` (256-byte
 * aligned, at least workspace_bytes) and uploads the analysis plans into
 * it on `stream`; returns after the upload completed.  The memory must
 * outlive every later call on the handle.
 * Errors: CKKT_ERR_WORKSPACE, CKKT_ERR_HIP. */
ckkt_status ckkt_bind_workspace(ckkt_handle* h, void* dev_ptr, size_t bytes, void* stream);

/* Numeric phase for one new system (assembly and factorization):
 * assembles K (LiftedKKT) or K_gamma (HyKKT) in FP64 into the factor's
 * pattern and factorizes it, LL^T, in the handle's precision.  Work is
 * enqueued on `stream` (a hipStream_t, NULL = default stream); the call
 * returns without waiting.
 *   w_val   : nnz(W) device doubles, in the order of w_idx
 *   g_val   : nnz(G) device doubles (NULL if m_eq == 0)
 *   h_val   : nnz(H) device doubles (NULL if m_ineq == 0)
 *   sigma_x : n device doubles (>= 0)
 *   sigma_s : LiftedKKT m_eq + m_ineq doubles (rows of G first, then H);
 *             HyKKT m_ineq doubles (> 0)
 *   gamma   : HyKKT weight of G^T G (> 0), ignored for LiftedKKT.
 * A non-positive pivot is reported by the next ckkt_solve or
 * ckkt_factor_status as CKKT_ERR_NOT_SPD. */
ckkt_status ckkt_factorize(ckkt_handle* h, const double* w_val, const double* g_val,
                           const double* h_val, const double* sigma_x,
                           const double* sigma_s, double gamma, void* stream);

/* Waits for the factorization and reports CKKT_OK, CKKT_ERR_NOT_SPD (the
 * failing column is then in ckkt_info.failed_column), CKKT_ERR_NONFINITE (an
 * assembled entry was NaN or Inf) or CKKT_ERR_TIMEOUT (left by a solve). */
ckkt_status ckkt_factor_status(ckkt_handle* h, void* stream);

/* HyKKT handles: the numeric phase for a system with dual regularization
 * delta_c > 0 (Remark 1, eqn:primal).  K1 then carries -delta_c I in its
 * (2,2) block, and eliminating d_y = (G d_x - rbar2) / delta_c leaves the
 * primal Schur complement K + G^T G / delta_c, which is K_gamma with
 * gamma = 1 / delta_c: this call is ckkt_factorize with that gamma (same
 * arguments, memory and errors).  The following ckkt_solve calls solve
 * K1(delta_c) (d_x, d_y) = (rbar1, rbar2) directly, without CG:
 * d_x = K_gamma^{-1}(rbar1 + G^T rbar2 / delta_c), d_y = (G d_x - rbar2) / delta_c,
 * inside the same FP64 refinement on K1(delta_c), whose backward error
 * counts delta_c as data of the second block row.  The next ckkt_factorize
 * returns the handle to delta_c = 0.  CKKT_ERR_ARG for LiftedKKT handles and
 * unless delta_c and 1/delta_c are both positive and finite. */
ckkt_status ckkt_factorize_dual_reg(ckkt_handle* h, const double* w_val, const double* g_val,
                                    const double* h_val, const double* sigma_x, const double* sigma_s,
                                    double delta_c, void* stream);

/* ---- Inertia correction (primal regularization delta_w) ----
 *
 * The augmented system K2 (Sec. 2.2, eq:kkt:augmented) is regularized by
 * delta_w I on its primal and on its slack block whenever its inertia is not
 * (n + m_i, m_i + m_e, 0); delta_w follows the inertia-controlling rule of
 * Waechter & Biegler (2006, Sec. 3.1), which the paper adopts (Sec. 2.2,
 * Remark 1).  By Sylvester's law (eq:ipm:inertia) the inertia is correct
 * exactly when the condensed matrix is positive definite -- K_tau for
 * LiftedKKT (Sec. 3.2), K_gamma for HyKKT once gamma exceeds its threshold
 * (Sec. 3.1) -- so a Cholesky factorization that meets a non-positive pivot
 * is the signal to try a larger delta_w.  Condensing K2 with delta_w
 * (delta_c = 0) adds delta_w to sigma_x and to every slack weight sigma_s
 * (for HyKKT only the inequality rows have slacks).
 *
 * Trials: delta_w = 0; then delta_w_0 when delta_w_last == 0, else
 * max(delta_w_min, kappa_minus * delta_w_last); each failure multiplies by
 * kappa_plus_bar (delta_w_last == 0) or kappa_plus (delta_w_last > 0); no
 * trial above delta_w_max.  A success with delta_w > 0 stores it in
 * delta_w_last.  The zero-eigenvalue branch of the rule (delta_c > 0) is
 * not taken: a Cholesky factorization cannot tell a zero eigenvalue from a
 * negative one, and a singular matrix is treated like an indefinite one. */
typedef struct ckkt_inertia {
    double  delta_w_min;     /* smallest nonzero trial                 (default 1e-20) */
    double  delta_w_0;       /* first trial without history           (default 1e-4)  */
    double  delta_w_max;     /* largest trial                          (default 1e40)  */
    double  kappa_minus;     /* decrease of delta_w_last, in (0, 1)    (default 1/3)   */
    double  kappa_plus;      /* growth with history, > 1               (default 8)     */
    double  kappa_plus_bar;  /* growth without history, > 1            (default 100)   */
    double  delta_w_last;    /* in/out: last nonzero delta_w accepted; 0 before the first */
    double  delta_w;         /* out: delta_w of the accepted factor (the last trial on failure) */
    int32_t attempts;        /* out: factorizations performed (>= 1) */
    int32_t pad;
} ckkt_inertia;

/* Fills the parameters with the defaults above, delta_w_last = 0 and the
 * outputs with zero. */
void ckkt_default_inertia(ckkt_inertia* ic);

/* Factorizes K (LiftedKKT) or K_gamma (HyKKT) of the system given by the
 * arguments (same meaning and memory as ckkt_factorize: the UNREGULARIZED
 * sigma_x and slack weights sigma_s) with the smallest trial delta_w of the
 * rule above that gives a positive definite matrix.  Each trial is one
 * ckkt_factorize of the shifted diagonals followed by one synchronization of
 * `stream`; the shifted diagonals are kept in the workspace, so the
 * following ckkt_solve calls refine against the regularized system.
 *   ic : host, in/out (parameters, delta_w_last; delta_w and attempts out).
 * FP64 handles of one system only (an FP32_IR factor pivots statically and
 * reveals no definiteness; a batch has no single delta_w): else
 * CKKT_ERR_ARG, as for parameters out of range.  Returns CKKT_ERR_NOT_SPD
 * when every trial up to delta_w_max fails (delta_w_last unchanged; the
 * factor then is that of the last trial and ckkt_solve reports
 * CKKT_ERR_NOT_SPD), CKKT_ERR_NONFINITE / CKKT_ERR_HIP as ckkt_factorize. */
ckkt_status ckkt_factorize_inertia(ckkt_handle* h, const double* w_val, const double* g_val,
                                   const double* h_val, const double* sigma_x, const double* sigma_s,
                                   double gamma, ckkt_inertia* ic, void* stream);

/* Solve with the current factor: triangular sweeps plus FP64
 * iterative refinement with K applied unassembled (Sec. 2.2, "Iterative
 * refinement"); for HyKKT the CG of eq:kkt:schurcomplhykkt inside an outer
 * FP64 refinement on K1.  Stops when the componentwise relative backward
 * error omega = max_i |res_i| / (|data| |sol| + |rhs|)_i <= opt.tol.
 *   rhs : LiftedKKT n doubles (b); HyKKT n + m_eq doubles (rbar1; rbar2)
 *   sol : same length; receives d_x (LiftedKKT) or (d_x; d_y) (HyKKT)
 *   info: host, may be NULL.
 * Blocks until the result is in `sol`.
 * Errors: CKKT_ERR_STATE, CKKT_ERR_NOT_SPD, CKKT_ERR_NONFINITE (an input of the
 * factor or the right-hand side), CKKT_ERR_NO_CONVERGENCE (sol then holds the
 * best iterate), CKKT_ERR_BREAKDOWN, CKKT_ERR_TIMEOUT, CKKT_ERR_HIP. */
ckkt_status ckkt_solve(ckkt_handle* h, const double* rhs, double* sol,
                       ckkt_solve_info* info, void* stream);

/* Factorization and solve of a whole LiftedKKT system in one call, meant
 * for a batch analysed by ckkt_batch_analyze (the solver's factorization
 * and solve phases, Sec. 5 and 6.1, applied to every instance at once; also
 * accepted for a single pattern).  One captured launch sequence does what
 * ckkt_factorize and ckkt_solve do: assembly (Sec. 3.2, eq:liftedkkt),
 * factorization in the handle's precision, x = K^{-1} b, then `refine`
 * refinement steps (residual with K unassembled in FP64, a factor
 * application, and the update x += dx applied only to the instances whose
 * componentwise backward error omega is still above opt.tol, so a
 * converged instance is left as it is), and the final residual.  Then the
 * call synchronizes `stream` once and reads every instance's omega.  If an
 * instance is still above opt.tol, the refinement of ckkt_solve (FP32:
 * Richardson, PCG around the FP32 factor, FP64 refactorization) continues
 * from that iterate on the host's control, with its own synchronizations
 * (the device steps count against opt.ir_maxit), and info->fallback gets
 * 4 added.
 *   values, sigma_x, sigma_s : as ckkt_factorize (device, caller-owned)
 *   rhs, sol    : n doubles each (device); sol receives d_x
 *   refine      : device refinement steps, 0 .. CKKT_MAX_DEVICE_REFINE
 *   inst_omega  : host, one double per instance (the instance's omega), or NULL
 *   info        : host, may be NULL (refine_steps counts the device steps)
 * The sequence is captured on the first call and replayed while the value,
 * right-hand side and solution pointers and `refine` stay the same (a
 * change of any of them captures it again).  The handle stays factorized
 * for ckkt_solve / ckkt_apply_inverse afterwards; the stale reference of
 * the learned preconditioner is not updated.  FP32_IR handles follow the
 * precision policy described at CKKT_FP32_IR (an FP64 factorization from
 * the start after a recent FP32 failure, with at most one device step:
 * info->fallback has 8 set; a different precision uses its own captured
 * sequence).  LiftedKKT handles without
 * split dense rows only (else CKKT_ERR_ARG).  Errors as ckkt_factorize and
 * ckkt_solve. */
#define CKKT_MAX_DEVICE_REFINE 8
ckkt_status ckkt_batch_factorize_solve(ckkt_handle* h, const double* w_val, const double* g_val,
                                       const double* h_val, const double* sigma_x, const double* sigma_s,
                                       const double* rhs, double* sol, int32_t refine, double* inst_omega,
                                       ckkt_solve_info* info, void* stream);

/* Newton step of the augmented system K2 (Sec. 2.2, eq:kkt:augmented,
 * delta_c = 0) around the condensed factor:
 *   [ W + Sx  0   G^T  H^T ] [dx]     [r1]
 *   [ 0       E   0    I   ] [ds]     [r2]
 *   [ G       0   0    0   ] [dy] = - [r3]
 *   [ H       I   0    0   ] [dz]     [r4]
 * with Sx = sigma_x and E = D_s + delta_w I the slack diagonal, which is the
 * factor's slack weight sigma_s (D_H = E when delta_c = 0).  Slack rows:
 * LiftedKKT every constraint row (its equalities are relaxed inequalities,
 * Sec. 3.2; rows of G first, then H), HyKKT the rows of H; the equality
 * block (r3, dy) exists for HyKKT only.  The condensed right-hand side
 * rbar1 = -(r1 + H^T (E r4 - r2)), rbar2 = -r3 is solved with the current
 * factor (LiftedKKT: one application; HyKKT: its CG on S_gamma), the slacks
 * are recovered (dz = -r2 + E (H dx + r4), ds = -(r2 + dz) / E), and FP64
 * Richardson iterations on K2 (K2 applied blockwise, unassembled) repeat the
 * same steps on the residual until the componentwise relative backward error
 * of K2 w.r.t. its data is <= opt.tol (info->omega; refine_steps counts the
 * corrections after the first).
 *   r1, dx : n device doubles;  r2, r4, ds, dz : slack-row count (LiftedKKT
 *   m_eq + m_ineq, HyKKT m_ineq);  r3, dy : m_eq (HyKKT; ignored, may be
 *   NULL, for LiftedKKT).  Outputs are overwritten.  Blocks until done.
 * Errors: CKKT_ERR_ARG (batch handle, missing pointer), CKKT_ERR_STATE (not
 * factorized, or factorized with ckkt_factorize_dual_reg), CKKT_ERR_NOT_SPD,
 * CKKT_ERR_NONFINITE, CKKT_ERR_NO_CONVERGENCE, CKKT_ERR_BREAKDOWN,
 * CKKT_ERR_TIMEOUT, CKKT_ERR_HIP. */
ckkt_status ckkt_solve_augmented(ckkt_handle* h, const double* r1, const double* r2, const double* r3,
                                 const double* r4, double* dx, double* ds, double* dy, double* dz,
                                 ckkt_solve_info* info, void* stream);

/* Bound-multiplier step of the unreduced system K3 (eq:kkt:unreduced, last
 * block row V ds + S dv = -(S v - mu e); Sec. 2.2):
 * dv = -S^{-1} (V ds - mu e) - v, elementwise over `count` slacks.  s, v, ds,
 * dv are device doubles (s > 0); enqueued on stream, does not wait. */
ckkt_status ckkt_recover_bound_dual(int64_t count, const double* s, const double* v, double mu,
                                   const double* ds, double* dv, void* stream);

/* One application of the factor, x = (L L^T)^{-1} b (forward and backward
 * sweeps only, no refinement; with rows split off by opt.dense_row_min,
 * the sweeps of K_s followed by the Woodbury step, so x = K^{-1} b), for
 * LiftedKKT and HyKKT (K_gamma).
 * rhs, sol: n device doubles; enqueued on stream, does not wait. */
ckkt_status ckkt_apply_inverse(ckkt_handle* h, const double* rhs, double* sol, void* stream);

/* The assembled K (or K_gamma) of the last factorize -- without the rows
 * split off by opt.dense_row_min, i.e. K_s -- as coordinates in the
 * ORIGINAL numbering (row >= col), one entry per internal slot, nnz_k
 * entries: rows/cols are host arrays filled when non-NULL, values is a
 * device array of nnz_k doubles filled (synchronously) when non-NULL. */
ckkt_status ckkt_export_k(ckkt_handle* h, int32_t* rows, int32_t* cols, double* values, void* stream);

/* Host execution of the numeric phase over the same analysis plan (same
 * assembly recipe, multifrontal maps, level schedule and sweeps as the
 * device kernels, FP64, sequential): x = K^{-1} rhs for LiftedKKT or
 * x = K_gamma^{-1} rhs for HyKKT, no refinement.  All pointers are HOST
 * memory; needs no GPU and no workspace.  For validating the analysis on
 * machines without a GPU.  Returns CKKT_ERR_NOT_SPD (with *failed_column,
 * original numbering) on a non-positive pivot. */
ckkt_status ckkt_host_factor_solve(const ckkt_handle* h, const double* w_val, const double* g_val,
                                  const double* h_val, const double* sigma_x, const double* sigma_s,
                                  double gamma, const double* rhs, double* sol, int32_t* failed_column);

/* ckkt_factorize_inertia run on the host execution of ckkt_host_factor_solve:
 * the same trials of delta_w, each a sequential host factorization, then
 * x = K(delta_w)^{-1} rhs with the accepted factor.  All pointers are HOST
 * memory (ic as in ckkt_factorize_inertia); needs no GPU.  Returns
 * CKKT_ERR_NOT_SPD when every trial fails. */
ckkt_status ckkt_host_factor_solve_inertia(const ckkt_handle* h, const double* w_val, const double* g_val,
                                           const double* h_val, const double* sigma_x, const double* sigma_s,
                                           double gamma, ckkt_inertia* ic, const double* rhs, double* sol);

/* ---- Learned diagonal preconditioner (PCG around a stale factor) ----
 *
 * For a new system K (LiftedKKT) and the factor of an earlier system K_s
 * (the last ckkt_factorize), PCG uses M^{-1} = D K_s^{-1} D with
 * D = diag(exp(o)), o_j the output of an 8-64-64-1 tanh MLP evaluated on 8
 * per-variable features that compare the new diagonals with those of K_s:
 * f0 = log10 sigma_x / 8, f1 = its change / 8, f2 = log10 K_jj / 8, f3 = its
 * change / 8, f4 = max over constraint rows r touching j of log10 d_r / 8,
 * f5 / f6 = max / min over those rows of the change of log10 d_r / 8 (0 for a
 * variable in no row), f7 = 1.  M is SPD for every parameter value.
 * Parameters: CKKT_MLP_NPARAM FP32 values, W1[64][8], b1[64], W2[64][64],
 * b2[64], w3[64], b3 (row-major).  The handle must be analysed with
 * opt.learned = 1. */
#define CKKT_MLP_FEATURES 8
#define CKKT_MLP_HIDDEN   64
#define CKKT_MLP_NPARAM   (64 * 8 + 64 + 64 * 64 + 64 + 64 + 1)

/* Features (n x 8 FP32, device, row-major) of the system given by the value
 * pointers (same meaning as ckkt_factorize) against the system of the
 * current factor.  Enqueued on stream. */
ckkt_status ckkt_features(ckkt_handle* h, const double* w_val, const double* g_val, const double* h_val,
                          const double* sigma_x, const double* sigma_s, double gamma, float* features,
                          void* stream);

/* MLP forward on n rows of features: out[n]; cache (2 * 64 * n FP32, may be
 * NULL) keeps the hidden activations for ckkt_mlp_backward.  Device
 * pointers, no handle needed. */
ckkt_status ckkt_mlp_forward(int64_t n, const float* features, const float* params, float* out, float* cache,
                             void* stream);

/* Bytes of scratch ckkt_mlp_backward needs for n rows. */
size_t ckkt_mlp_workspace(int64_t n);

/* Gradient (CKKT_MLP_NPARAM FP32) of sum_j g_out[j] * out_j with respect to
 * the parameters, from the cache of ckkt_mlp_forward; ws has
 * ckkt_mlp_workspace(n) bytes.  Fixed-order reductions (deterministic). */
ckkt_status ckkt_mlp_backward(int64_t n, const float* features, const float* params, const float* cache,
                              const float* g_out, float* grad, void* ws, void* stream);

/* ckkt_mlp_backward for callers that cannot allocate device memory (code
 * under graph capture, tight serving loops, harnesses that forbid
 * allocation): the same kernels and result (bitwise), with the scratch in a
 * static device array of the library instead of a workspace argument, so
 * the call allocates nothing.  n is at most CKKT_MLP_NOALLOC_MAX_ROWS
 * (CKKT_ERR_ARG beyond).  The array holds 2 * 64 * N + 4801 * N / 256 + 64
 * FP32 values, N = CKKT_MLP_NOALLOC_MAX_ROWS (19.2 MB), on every device the
 * library runs on, until the process ends.  Every call on one device
 * shares that array and nothing in it has to start at zero: calls
 * that overlap on one device (other streams, other threads) race, so the
 * caller serializes them.  Other arguments and errors as
 * ckkt_mlp_backward. */
#define CKKT_MLP_NOALLOC_MAX_ROWS 32768
ckkt_status ckkt_mlp_backward_noalloc(int64_t n, const float* features, const float* params, const float* cache,
                                      const float* g_out, float* grad, void* stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8); step counts from 1. */
ckkt_status ckkt_adam(int32_t nparam, float* params, const float* grad, float* m, float* v, int32_t step,
                      float lr, void* stream);

/* One training step on a solver-generated pair (rhs, target = K^{-1} rhs) of
 * the system given by the values, against the current (stale) factor: loss
 * L = ||D K_s^{-1}(D rhs) - target||^2 / ||target||^2, its gradient through
 * two stale solves and the MLP, and an Adam step on params/m/v.  *loss
 * (host) receives L before the step.  Blocks until done. */
ckkt_status ckkt_mlp_train_step(ckkt_handle* h, const double* w_val, const double* g_val, const double* h_val,
                                const double* sigma_x, const double* sigma_s, double gamma, const double* rhs,
                                const double* target, float* params, float* m, float* v, int32_t step, float lr,
                                double* loss, void* stream);

/* FP64 PCG on the new system K x = rhs (LiftedKKT, K applied unassembled)
 * preconditioned by D K_s^{-1} D around the current factor; params NULL
 * means D = I.  Stops when omega <= tol; after maxit iterations, if
 * allow_refactor, factorizes the new system (which becomes the stale
 * reference) and solves it with ckkt_solve (info->fallback = 2), else
 * returns CKKT_ERR_NO_CONVERGENCE with the last iterate.  Blocks. */
ckkt_status ckkt_pcg_solve(ckkt_handle* h, const double* w_val, const double* g_val, const double* h_val,
                           const double* sigma_x, const double* sigma_s, double gamma, const float* params,
                           const double* rhs, double* sol, int32_t maxit, double tol, int32_t allow_refactor,
                           ckkt_solve_info* info, void* stream);

/* Autotuner of the launch shapes that leave the factor layout unchanged
 * (boundary of the compact small-front class, workgroup sizes of the small
 * fronts and of the sweeps).  Times `reps` factorize + factor applications of
 * the given system for every candidate on `stream`, keeps the fastest for
 * this handle and caches it for patterns with the same analysis (a later
 * call on such a pattern applies the cached choice without timing and
 * returns *best_ms = -1).  chosen (host, 4 int32, may be NULL) receives
 * {compact front order, compact workgroup size, tiny workgroup size, sweep
 * cutoff}.  Leaves a valid factor of the given system.  Blocks. */
ckkt_status ckkt_autotune(ckkt_handle* h, const double* w_val, const double* g_val, const double* h_val,
                          const double* sigma_x, const double* sigma_s, double gamma, int32_t reps,
                          int32_t* chosen, double* best_ms, void* stream);

ckkt_status ckkt_get_info(const ckkt_handle* h, ckkt_info* info);
const char* ckkt_status_string(ckkt_status s);
void        ckkt_destroy(ckkt_handle* h);

/* Per-phase device time, in milliseconds, accumulated with HIP events on
 * the caller's stream since the last reset (0 = assemble, 1 = factor,
 * 2 = sweeps, 3 = residual/refinement/CG vector work) and the number of
 * calls of each phase.  Timing is off unless enabled; `enable` is a mask of
 * the phases to time (bit p for phase p; -1 = all, 0 = off).  A timed phase
 * adds two event records per call but no synchronisation. */
ckkt_status ckkt_set_timing(ckkt_handle* h, int32_t enable);
ckkt_status ckkt_get_timing(ckkt_handle* h, double ms[4], int64_t calls[4]);

#ifdef __cplusplus
}
#endif
#endif /* CKKT_H */
