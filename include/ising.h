/*
 * ising.h -- C ABI of the MI355X (gfx950) pruning + domain-selection Ising solver.
 *
 * Problem (paper, Sec. II, scalar energy form and primal problem):
 *     minimise E(s) = s^T J s + h^T s   over s in {-1,+1}^n,
 * with J real symmetric, J_ii = 0.  J is the matrix of that form (each pair is
 * counted twice); a Hamiltonian given with J-hat (sum over i > j) is passed as
 * J = J-hat / 2.
 *
 * Pipeline (paper, Fig. 1): pruning (Sec. III-A, Algorithm 1) -> domain
 * selection (Sec. III-B, loss-function equation, optimised by GD or ADAM as in
 * Sec. IV-B) over many independent replicas -> selection of the best replica
 * -> retrieval of the full spin vector from the pruning record (Fig. 1c).
 *
 * Conventions for every entry point:
 *  - Return value: ISING_OK or an error code; no exception crosses the ABI.
 *    A one-line message for the last failure of a context is available from
 *    ising_last_error().  A context is used by one host thread at a time,
 *    except ising_submit / ising_wait / ising_cancel, which are thread-safe.
 *  - Ownership: the caller owns every buffer it passes.  Host inputs are
 *    read (and copied) before the call returns.  Outputs go to caller-
 *    allocated buffers.  The library owns the memory behind handles it
 *    returns (ising_ctx, ising_pruned) until the matching destroy/free call.
 *  - "_dev" entry points take device pointers (memory on the context's
 *    device) and a hipStream_t passed as void*; they enqueue work on that
 *    stream, borrow the buffers only for the duration of the call, and return
 *    after the work is enqueued unless stated otherwise.  NULL stream = the
 *    legacy default stream.
 *  - Layouts: dense J is row-major n x n (row stride n).  CSR holds both
 *    directions of every coupling, column indices strictly ascending within a
 *    row, no diagonal entries, int32 row_ptr[n+1] and col[nnz].  Spin arrays
 *    are int8 values -1/+1; a block of R spin vectors is replica-major
 *    (vector r occupies [r*n, (r+1)*n)).
 */
#ifndef ISING_H
#define ISING_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ising_status {
    ISING_OK = 0,
    ISING_EINVAL = 1,     /* malformed problem or parameters (asymmetric J, diagonal, bad CSR, n <= 0 ...) */
    ISING_ENOMEM = 2,     /* device or host allocation failed, or over the serving memory budget */
    ISING_EDEVICE = 3,    /* a HIP runtime call failed */
    ISING_EBUSY = 4,      /* request not finished yet / queue full */
    ISING_ETIMEDOUT = 5,  /* ising_wait timed out */
    ISING_ECANCELED = 6,  /* request was cancelled */
    ISING_ENOTSUP = 7     /* combination of format / value type / precision not supported */
} ising_status;

enum { ISING_DENSE = 0, ISING_CSR = 1 };

/* Value type of J (dense entries or CSR values) and of h. */
enum { ISING_I32 = 0, ISING_F32 = 1, ISING_F64 = 2 };

enum { ISING_OPT_GD = 0, ISING_OPT_ADAM = 1 };

/* The local optimum s~* of the loss (Sec. III-B, loss-function equation).
 * VERTEX: the current vertex sgn(sin theta), piecewise constant, so the step
 * uses dL/dtheta = cos(theta) ((J - mu I) s~* + h).  RELAXED: the relaxed flip
 * pattern sin(theta) itself, L = x^T (J - mu I) x + h^T x with x = sin(theta),
 * dL/dtheta = cos(theta) (2 (J - mu I) x + h); the energy of the vertex
 * sgn(sin theta) is still tracked every step.  RELAXED runs on the persistent
 * engine only (not the matrix-core engine, the staged +-w image, the streaming
 * form or the serving form): other requests for it fail with ISING_ENOTSUP. */
enum { ISING_LOSS_VERTEX = 0, ISING_LOSS_RELAXED = 1 };

/* Arithmetic of domain selection.  FP64 and FP32: iterates (angles, moments,
 * gradient) and coupling product in that precision.  BF16X2 and BF16 (dense
 * couplings on the matrix cores only): FP32 iterates, coupling product with J
 * split into two BF16 parts (J = J_hi + J_lo) or rounded to one BF16, the
 * vertex (+-1) exact in BF16, FP32 accumulation.  FP8 (dense couplings whose
 * nonzero values are integers of one magnitude w, with n w < 2^24, e.g. +-1;
 * ENOTSUP otherwise): J / w and the vertex exact in FP8 (E4M3) on the matrix
 * cores, FP32 accumulation, FP32 iterates; every product and sum is exact, so
 * the results equal the FP32 form's bit for bit, and an FP32 request on such
 * couplings runs this form.  I8X3 and I8X2 (dense couplings, n <= 65536;
 * ENOTSUP otherwise): J held as 2^e Jq, one power-of-two scale for the whole
 * matrix and Jq an integer of three (two) balanced INT8 digits, the vertex +-1
 * in INT8; the product Jq S~ is exact in int32 on the matrix cores and y =
 * 2^e float(Jq S~) is rounded once.  e is the smallest exponent with
 * max|J_ij| <= 2^e qmax (qmax = 8355711 for three digits, 32639 for two) and
 * max_i sum_j |J_ij| + 2^e 257 n <= 2^e (2^31 - 1), so each entry carries an
 * absolute error of at most 2^(e-1) (none when J / 2^e is an integer, e.g.
 * +-1 couplings); FP32 iterates.  An FP32 request that runs on the matrix
 * cores (dense, n > 256) with integer couplings |J| <= 127 of several
 * magnitudes (and n max|J| < 2^24) runs the same form with one digit: exact,
 * with the FP32 form's results.  The energy of the returned vector is always
 * recomputed in FP64 (or exactly for integer J). */
enum {
    ISING_PREC_FP64 = 0,
    ISING_PREC_FP32 = 1,
    ISING_PREC_BF16X2 = 2,
    ISING_PREC_BF16 = 3,
    ISING_PREC_FP8 = 4,
    ISING_PREC_I8X3 = 5,
    ISING_PREC_I8X2 = 6
};

typedef struct ising_problem {
    int32_t n;           /* spin count, > 0 */
    int32_t format;      /* ISING_DENSE or ISING_CSR */
    int32_t value_type;  /* ISING_I32, ISING_F32 or ISING_F64: type of J values and of h */
    int32_t reserved0;
    int64_t nnz;         /* CSR: number of stored couplings (both directions) */
    const void *J;       /* DENSE: n*n values, row-major */
    const int32_t *row_ptr; /* CSR: n+1 offsets */
    const int32_t *col;  /* CSR: nnz column indices */
    const void *val;     /* CSR: nnz values */
    const void *h;       /* n values, or NULL for h = 0 */
} ising_problem;

typedef struct ising_params {
    int32_t replicas;    /* R >= 1 independent trajectories */
    int32_t steps;       /* T >= 0 iterations (T = 0 scores no vertex: every best record keeps
                            its start, +1 on every spin, and replica 0 is selected) */
    int32_t optimizer;   /* ISING_OPT_GD or ISING_OPT_ADAM */
    int32_t precision;   /* ISING_PREC_* (BF16X2, BF16, FP8, I8X3, I8X2: dense couplings only) */
    double lr;           /* learning rate, finite and > 0 (the paper uses 6.0 with ADAM) */
    double mu;           /* augmented-Lagrangian weight of the L1-norm form, finite and > 0 */
    double beta1, beta2, eps;  /* ADAM constants (Kingma-Ba defaults 0.9, 0.999, 1e-8): 0 <= beta < 1,
                                  eps finite and > 0.  lr, mu or (ADAM) these outside their
                                  ranges: ISING_EINVAL before any work */
    uint64_t seed;       /* key of the counter-based initial draws */
    int32_t prune;       /* nonzero: run Algorithm 1 before domain selection */
    int32_t loss;        /* ISING_LOSS_VERTEX (0) or ISING_LOSS_RELAXED */
    /* Convergence test (Sec. IV-B), off when conv_tol <= 0: a replica stops after the
     * first step t >= conv_window at which the spread (maximum minus minimum) of its
     * last conv_window losses is <= conv_tol * |L_t - L_1| (the paper: 5 and 0.005).
     * Its angles, moments and best vertex are then final; the launch ends when every
     * replica has stopped.  Persistent engine (register-resident form) and the
     * serving form, where a request whose replicas have all stopped finishes at the
     * end of that chunk; ising_ds_dev continues the test across calls through the
     * state's conv_step and conv_state (not the matrix-core or streaming forms: ENOTSUP
     * there).  1 <= conv_window <= 8. */
    int32_t conv_window;
    int32_t reserved1;
    double conv_tol;
} ising_params;

typedef struct ising_stats {
    int32_t n;               /* original spin count */
    int32_t n_G;             /* spins left after pruning */
    int32_t rounds;          /* pruning rounds executed */
    int32_t best_replica;    /* replica whose vertex was returned */
    int64_t steps;           /* domain-selection steps per replica */
    int32_t best_step;       /* step at which the returned vertex was first seen */
    int32_t converged;       /* replicas that met the convergence test (0 when it is off) */
    double eta;              /* pruning rate 1 - n_G / n */
    double constant_C;       /* constant of the reduced problem */
    double t_upload_ms, t_prune_ms, t_ds_ms, t_finish_ms, t_total_ms;
    double replica_spin_updates_per_s;  /* n_G * R * T / t_ds */
    double t_ds_kernel_ms;   /* the domain-selection kernel alone (HIP events around its launch) */
    double mean_steps_run;   /* mean over replicas of the steps run (the convergence step or T) */
} ising_stats;

typedef struct ising_ctx ising_ctx;
typedef struct ising_pruned ising_pruned;

/* ---- context ----------------------------------------------------------- */

/* Create a context on HIP device `device`.  *out receives the handle. */
ising_status ising_create(int device, ising_ctx **out);
/* Destroy a context; waits for its outstanding work.  NULL is allowed. */
ising_status ising_destroy(ising_ctx *ctx);
/* Message of the last failed call on ctx ("" if none; with serving, also the last
 * failure of a served request collected by ising_wait).  A copy owned by the
 * calling thread, valid until that thread calls ising_last_error again. */
const char *ising_last_error(const ising_ctx *ctx);

/* ---- whole solve (host buffers) ---------------------------------------- */

/* Solve the problem of Sec. II with the pipeline of Fig. 1.
 * problem: host buffers.  spins_out: n int8 (host).  energy_out: E(s) of the
 * returned vector on the full instance, recomputed exactly on the device
 * (FP64 for real J, exact integer for ISING_I32).  energy_int_out (nullable):
 * the same as int64 for ISING_I32 problems.  stats_out nullable.
 * Blocking.  Errors: EINVAL for a malformed problem or parameters, ENOTSUP,
 * ENOMEM, EDEVICE. */
ising_status ising_solve(ising_ctx *ctx, const ising_problem *problem, const ising_params *params,
                         int8_t *spins_out, double *energy_out, int64_t *energy_int_out,
                         ising_stats *stats_out);

/* The same pipeline on device buffers: problem, spins_out (n int8),
 * energy_out (1 double, nullable) and energy_int_out (1 int64, nullable) are
 * device pointers; stats_out is host memory (nullable).  Work is enqueued on
 * `stream`; the call returns after it has completed (pruning reads a counter
 * per round and the stats need the event timings). */
ising_status ising_solve_dev(ising_ctx *ctx, const ising_problem *problem, const ising_params *params,
                             int8_t *spins_out, double *energy_out, int64_t *energy_int_out,
                             ising_stats *stats_out, void *stream);

/* Name of the domain-selection kernel form launched by the last ising_ds_dev,
 * ising_ds_dense_dev or ising_solve(_dev) call on ctx, e.g. "k_ds_split<adam>",
 * "k_ds<float, PME, rg=1, ept=28, no loss, unit>" or "k_dense_step<bf16x2>" ("" before the
 * first launch).  A diagnostic: the engine picks its form from the problem and the requested
 * outputs (traces, the convergence test); the forms compute the same method and agree with
 * each other to rounding (the loss-free forms evaluate cos(theta) alone), and tests use the
 * name to know which one they checked.  Valid until the next call on ctx. */
const char *ising_last_kernel(const ising_ctx *ctx);

/* ---- exact energy (scalar energy form, Sec. II) ------------------------- */

/* E(s_r) = s_r^T J s_r + h^T s_r for `count` spin vectors on host buffers:
 * problem and spins (count * n int8, replica-major) are host memory, copied to
 * the device before the call returns; E_out (nullable): count doubles (host);
 * E_int_out (nullable, ISING_I32 problems only): count int64 (host), exact.
 * Same kernels and summation order as ising_energy_dev.  Blocking.  Errors:
 * EINVAL for a malformed problem or count < 0, ENOMEM, EDEVICE.  The problem is
 * not checked for symmetry here (the energy is defined for any J). */
ising_status ising_energy(ising_ctx *ctx, const ising_problem *problem, const int8_t *spins, int32_t count,
                          double *E_out, int64_t *E_int_out);

/* E(s_r) = s_r^T J s_r + h^T s_r for `count` spin vectors (replica-major).
 * problem and spins are device pointers.  E_out (nullable): count doubles.
 * E_int_out (nullable, ISING_I32 problems only): count int64, exact.
 * Real J: FP64, each row summed as 64 strided partials combined by an xor
 * butterfly, rows and blocks combined in a fixed order, so results are
 * reproducible run to run. */
ising_status ising_energy_dev(ising_ctx *ctx, const ising_problem *problem, const int8_t *spins,
                              int32_t count, double *E_out, int64_t *E_int_out, void *stream);

/* ising_energy_dev for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and results, with the per-block partial sums kept in a static device
 * array of the library (8 MiB per GPU, held until the process ends) instead of a
 * buffer allocated on demand.  The call allocates nothing.  Limit: count *
 * ceil(n / 4) * 8 bytes <= 8 MiB (e.g. 1024 vectors of n = 4096, 104 of
 * n = 20000); larger requests fail with EINVAL before any work is enqueued.
 * Every call on one GPU shares that GPU's array, so calls that overlap on one
 * GPU (concurrent streams or threads) race and must be serialised by the
 * caller; the array needs no clearing (every partial is written before it is
 * read).  Arguments, layouts and errors as ising_energy_dev. */
ising_status ising_energy_dev_noalloc(ising_ctx *ctx, const ising_problem *problem, const int8_t *spins,
                                      int32_t count, double *E_out, int64_t *E_int_out, void *stream);

/* ---- pruning (Sec. III-A, Algorithm 1) and retrieval (Fig. 1c) --------- */

/* Algorithm 1 on host buffers: the problem (host memory) is copied to the
 * device, validated (EINVAL as for ising_solve) and pruned there; the handle
 * owns that copy, the record and the reduced problem.  Blocking: the handle is
 * complete when the call returns.  Read it with ising_pruned_info,
 * ising_pruned_record, ising_pruned_copy (host) or the _dev readers; free it
 * with ising_pruned_free.  Pruning as ising_prune_dev below. */
ising_status ising_prune(ising_ctx *ctx, const ising_problem *problem, ising_pruned **out);

/* Run Algorithm 1 on the device.  problem: device pointers.  Each round takes
 * the determined spins D (|h_i| > 2 sum_{j active}|J_ij|, strict), folds them
 * into h and C, then the semi-determined spins S (exactly one active
 * neighbour k, 2|J_ik| >= |h_i|; of a mutual pair only the larger index),
 * folds them, and repeats until a round removes nothing.  Row sums of real J
 * (which decide D) use 64 strided partials combined by an xor butterfly
 * (32,16,8,4,2,1), a fixed order any implementation can reproduce; the folds
 * into h and C use the same per-row reduction, which differs from a plain
 * ascending sum only by rounding, within gamma_k times the sum of the terms'
 * magnitudes.  Integer problems are exact.  Synchronises the stream once per
 * round.  *out receives a handle owning the device-resident reduced problem
 * and record; free it with ising_pruned_free. */
ising_status ising_prune_dev(ising_ctx *ctx, const ising_problem *problem, ising_pruned **out,
                             void *stream);
void ising_pruned_free(ising_pruned *pruned);

/* Sizes of a pruning result: n, n_G, rounds, nnz of the reduced CSR (0 for
 * dense) and the constant C of the reduced problem. */
ising_status ising_pruned_info(const ising_pruned *pruned, int32_t *n, int32_t *n_G,
                               int32_t *rounds, int64_t *nnz_G, double *C);
/* Copy the record to device buffers (each nullable; n entries unless noted):
 * kind (int8: 0 kept, 1 determined, 2 semi-determined), round_of (int32, -1
 * for kept), fixed (int8 value of determined spins), partner (int32 n(k) of
 * semi-determined spins, -1 otherwise), sigma (int8 sgn J_k,n(k)), G (int32,
 * n_G original indices ascending), h_G (n_G values of the reduced problem's
 * value type, see ising_pruned_problem). */
ising_status ising_pruned_record_dev(ising_ctx *ctx, const ising_pruned *pruned, int8_t *kind,
                                     int32_t *round_of, int8_t *fixed, int32_t *partner,
                                     int8_t *sigma, int32_t *G, void *h_G, void *stream);
/* The reduced problem (device pointers owned by the handle, valid until
 * ising_pruned_free).  When nothing was pruned it aliases the input problem
 * (same pointers and value type); otherwise its value type is ISING_I32 for
 * integer problems and ISING_F64 otherwise. */
ising_status ising_pruned_problem(const ising_pruned *pruned, ising_problem *reduced);
/* Copy the reduced problem into caller device buffers (each nullable): dense
 * J_G (n_G*n_G) or CSR values, row_ptr (n_G+1), col (nnz_G), and h (n_G; left
 * untouched when the reduced problem has no field).  Value type as reported
 * by ising_pruned_problem. */
ising_status ising_pruned_copy_dev(ising_ctx *ctx, const ising_pruned *pruned, void *J_or_val,
                                   int32_t *row_ptr, int32_t *col, void *h, void *stream);
/* Retrieval: s[G] = s_G, then rounds in reverse: s_k = -sigma s_n(k) for
 * semi-determined spins, the recorded value for determined ones.  s_G: n_G
 * int8 (device), s_out: n int8 (device). */
ising_status ising_unprune_dev(ising_ctx *ctx, const ising_pruned *pruned, const int8_t *s_G,
                               int8_t *s_out, void *stream);
/* Retrieval (Fig. 1c) on host buffers, without a context: s_G (n_G int8 values
 * -1/+1, host; ignored when n_G = 0) gives s_out (n int8, host).  Runs the same
 * kernel as ising_unprune_dev on the handle's device (which becomes the calling
 * thread's current device) on its default stream, with a transient device
 * buffer of n + n_G bytes; blocking.  Errors: EINVAL (NULL handle or buffer),
 * ENOMEM, EDEVICE (no message: there is no context to hold one). */
ising_status ising_unprune(const ising_pruned *pruned, const int8_t *s_G, int8_t *s_out);
/* The record and h_G in host buffers (each nullable; layouts and value types as
 * ising_pruned_record_dev).  No context; the handle's device becomes current.
 * Blocking.  Errors: EINVAL, ENOMEM, EDEVICE. */
ising_status ising_pruned_record(const ising_pruned *pruned, int8_t *kind, int32_t *round_of, int8_t *fixed,
                                 int32_t *partner, int8_t *sigma, int32_t *G, void *h_G);
/* The reduced problem in host buffers (each nullable; layouts and value type as
 * ising_pruned_copy_dev).  No context; blocking.  Errors: EINVAL, EDEVICE. */
ising_status ising_pruned_copy(const ising_pruned *pruned, void *J_or_val, int32_t *row_ptr, int32_t *col,
                               void *h);

/* ---- domain selection (Sec. III-B), persistent replica-parallel engine -- */

/* Device-resident state of R replicas of an n-spin problem.  Angles and
 * moments are replica-major (element (r,i) at r*n+i) in the precision chosen
 * by params->precision (double for FP64, float for FP32). */
typedef struct ising_ds_state {
    void *theta;          /* R*n angles */
    void *m;              /* R*n ADAM first moments (may be NULL for GD) */
    void *v;              /* R*n ADAM second moments (may be NULL for GD) */
    int8_t *s_best;       /* R*n vertex with the lowest energy seen */
    double *e_best;       /* R lowest energy seen (+inf before the first step) */
    int32_t *best_step;   /* R step index (1-based) of e_best */
    double *energy_trace; /* nullable: steps*R energies E_t, row t-1-t0 holds step t */
    double *loss_trace;   /* nullable: steps*R losses L_t */
    int32_t *conv_step;   /* nullable: R steps at which the convergence test held (0: never) */
    void *conv_state;     /* nullable: R*9 values of the state precision, the convergence test's
                             window of losses and L_1, written by every call and read by a call
                             with t0 > 0 (needed, with conv_step, to continue the test) */
} ising_ds_state;

/* Run steps t0+1 .. t0+steps of domain selection on the problem (device
 * pointers) for params->replicas replicas.  Each step, per replica:
 * x = sin theta, s = sgn x (sgn 0 = +1), y = J s, E = s^T (y + h),
 * L = x^T (y - mu s + h), best-vertex update if E < e_best (strict),
 * g = cos theta (y - mu s + h), GD or ADAM update (bias corrections use the
 * global step index), theta <- theta - 2 pi rint(theta / 2 pi).
 * If t0 == 0 the state is initialised first: theta = asin(U) with U from
 * `uniform` (R*n values of the state precision, nullable) or, when NULL, from
 * the counter-based SplitMix64 draws U = 2 (top24(splitmix64(seed,
 * (r << 32) | i)) / 2^24) - 1; m = v = 0; e_best = +inf.  If t0 > 0 the
 * state is read from `state` and continued.
 * Energies of integer problems are exact.  One kernel launch per call; every
 * replica is handled by one workgroup, whose angles and moments stay in
 * registers across all steps: up to 4 spins per thread (n <= 4096), and for
 * sparse FP32 problems with one replica per workgroup up to 32 spins per
 * thread (n <= 24576); larger sparse problems up to ising_ds_max_n stream the
 * angles and moments through device memory each step (FP64 above 2048 spins
 * too).  The relaxed loss and the convergence test need the register-resident
 * form.  ENOTSUP if n is beyond the on-chip limit (ising_ds_max_n). */
ising_status ising_ds_dev(ising_ctx *ctx, const ising_problem *problem, const ising_params *params,
                          const void *uniform, int32_t t0, int32_t steps, ising_ds_state *state,
                          void *stream);
/* Largest n the persistent engine accepts for a given precision. */
int32_t ising_ds_max_n(int32_t precision);

/* The same steps for a dense problem on the matrix cores: each step is one
 * launch computing Y = J S~ in tiles of 128 spins x 128 replicas (x 256 replicas
 * for BF16X2, I8X3 and I8X2) with MFMA (precision FP32: v_mfma_f32_32x32x2_f32;
 * BF16X2 / BF16: v_mfma_f32_32x32x16_bf16 on J_hi (+ J_lo); FP8, and FP32 on
 * couplings of one integer magnitude: v_mfma_f32_32x32x64_f8f6f4 on J / w;
 * I8X3 / I8X2, and FP32 on integer couplings of several magnitudes up to 127:
 * v_mfma_i32_32x32x32_i8 on each digit plane of Jq), with the elementwise update
 * fused into the tile epilogue; each launch also keeps the previous step's best
 * energies, and a small launch after the last step keeps the final one's.
 * State arrays are float (theta, m, v), traces and e_best double; energies
 * tracked during the run are those of the chosen form (FP32 accumulation, int32
 * for the INT8 digit planes).  Any R >= 1; n up to the device memory (65536 for
 * the INT8 forms).  Errors: ENOTSUP for FP64 precision, a CSR problem, or the
 * conditions the precision states. */
ising_status ising_ds_dense_dev(ising_ctx *ctx, const ising_problem *problem, const ising_params *params,
                                const void *uniform, int32_t t0, int32_t steps, ising_ds_state *state,
                                void *stream);

/* ---- best replica (argmin) ---------------------------------------------- */

/* *best = argmin_r e_best[r] (lowest index on ties), written to device memory. */
ising_status ising_select_dev(ising_ctx *ctx, const double *e_best, int32_t replicas, int32_t *best,
                              void *stream);

/* ---- serving: continuous batching of many solves --------------------------
 * Callers: request loops that submit independent problems over time.  A
 * scheduler thread admits queued requests in arrival order while their device
 * footprint fits `hbm_budget_bytes` and fewer than `max_resident` are resident,
 * keeps their state on the device, and advances all resident requests by
 * `chunk_steps` steps per iteration: sparse requests with the same launch shape
 * share one launch of the persistent engine (one workgroup per request x
 * replica group), dense requests run the matrix-core engine on `dense_streams`
 * streams, its launches replayed from HIP graphs.  Finished requests are harvested (best replica, retrieval, exact
 * energy) and their memory is freed, so newly arrived requests are admitted
 * while others run.  A request's result depends only on its own problem and
 * parameters: it is bit-identical alone and in any mix. */
typedef struct ising_serve_config {
    size_t hbm_budget_bytes;  /* device memory resident requests may hold (0: 16 GiB) */
    int32_t max_resident;     /* requests resident at once (0: 64) */
    int32_t chunk_steps;      /* steps per scheduling iteration (0: 100) */
    int32_t dense_streams;    /* streams for dense requests (0: 4) */
    /* 0: each dense group's chunk of launches (two per step) is captured once into a HIP
     * graph and replayed while the group's shape and step count stay the same (the
     * per-problem descriptors are re-uploaded before every replay); nonzero: launched one
     * by one.  Results are the same either way. */
    int32_t no_graphs;
} ising_serve_config;

typedef struct ising_serve_info {
    uint64_t submitted, admitted, completed, canceled, failed;
    uint64_t chunks;          /* scheduling iterations with device work */
    uint64_t launches;        /* kernel launches issued by those iterations */
    int32_t resident, queued;
    size_t bytes_in_use;      /* device memory held by resident requests */
    double busy_ms;           /* wall time spent in device chunks */
} ising_serve_info;

/* Start the scheduler of ctx (one per context).  cfg nullable (defaults). */
ising_status ising_serve_start(ising_ctx *ctx, const ising_serve_config *cfg);
/* Finish every queued and resident request, then stop the scheduler.  ising_wait
 * calls blocked on requests when it is called return their results before the
 * server is released; no other call on the context may run concurrently with it,
 * and results not collected before it returns are discarded. */
ising_status ising_serve_stop(ising_ctx *ctx);
/* Queue a solve.  problem: host buffers, copied before the call returns.
 * params as for ising_solve; sparse requests run in FP32.  *ticket identifies
 * the request.  Thread-safe.  With the convergence test on, a request runs on the
 * persistent engine in FP32 and finishes at the end of the chunk in which its last
 * replica stopped (its result as from ising_solve with the same params).  Errors:
 * EINVAL (no server, malformed shape, step parameters out of range), ENOTSUP
 * (params->loss other than ISING_LOSS_VERTEX; the convergence test with a
 * precision other than FP32), EBUSY (the server is stopping). */
ising_status ising_submit(ising_ctx *ctx, const ising_problem *problem, const ising_params *params,
                          uint64_t *ticket);
/* Wait up to timeout_ms (negative: forever) for a request and copy its result
 * (spins_out: n int8, energy_out, stats_out; each nullable).  A wait that
 * returns anything but ETIMEDOUT consumes the ticket: of two waits on one
 * ticket, one returns the result and the other EINVAL.  For served requests the
 * stats hold: t_upload_ms = time queued, t_prune_ms = admission (upload,
 * checks, pruning, formats), t_ds_ms = time resident, t_total_ms = submit to
 * completion.  Returns the request's status: OK, EINVAL / ENOTSUP (rejected at
 * admission), ENOMEM (larger than the budget), ECANCELED, ETIMEDOUT. */
ising_status ising_wait(ising_ctx *ctx, uint64_t ticket, int32_t timeout_ms, int8_t *spins_out,
                        double *energy_out, ising_stats *stats_out);
/* Cancel a request (queued: never admitted; resident: dropped at the next
 * chunk boundary).  Its wait returns ECANCELED.  Thread-safe. */
ising_status ising_cancel(ising_ctx *ctx, uint64_t ticket);
/* Counters of the scheduler. */
ising_status ising_serve_query(ising_ctx *ctx, ising_serve_info *out);


/* ---- problem front-ends (host buffers, no device work, no context) ------ */

/* QUBO (the primal problem's binary form, Sec. II): minimise
 * f(x) = x^T Q x + c^T x over x in {0,1}^n.  With x = (1 + s) / 2 and Q
 * symmetrised as (Q + Q^T) / 2, f(x) = E(s) + *offset_out for the Ising
 * problem J_ij = Q_ij / 4 (i != j), J_ii = 0, h_i = (sum_j Q_ij + c_i) / 2.
 * Q: n*n row-major; c: n values or NULL (0).  J_out: n*n (dense, row-major),
 * h_out: n; all caller-owned.  Errors: EINVAL for n <= 0, NULL buffers or
 * non-finite entries. */
ising_status ising_from_qubo(int32_t n, const double *Q, const double *c, double *J_out, double *h_out,
                             double *offset_out);

/* MaxCut (Sec. IV-D, MaxCut-3 / MaxCut-D): edges (2*m vertex indices, pairs
 * a != b) with weights w (m values, NULL = 1).  The Ising problem is J = W,
 * h = 0 (the convention of Table 3, E = 2 (m - 2 cut) for unit weights), so
 * cut(s) = (2 *total_weight - E(s)) / 4.  Output CSR with both directions,
 * duplicate edges summed, ascending columns.  Call once with row_ptr == NULL
 * to get *nnz_out, then with row_ptr (n+1), col (nnz) and val (nnz).
 * Errors: EINVAL for bad indices, self-loops or non-finite weights. */
ising_status ising_from_maxcut(int32_t n, int64_t m, const int32_t *edges, const double *w, int32_t *row_ptr,
                               int32_t *col, double *val, int64_t *nnz_out, double *total_weight);

/* NAE-3SAT (Sec. IV-D): m clauses of three literals, +(v+1) for variable v
 * true (spin +1) and -(v+1) for false.  A clause is violated when its three
 * literal values are equal.  J_ab = sum of sign_a sign_b over the literal pairs
 * of all clauses (integers, as in Table 3), h = 0; the number of violated
 * clauses is U(s) = (E(s) + *base_out) / 8.  Output CSR with int32 values;
 * sizing call with row_ptr == NULL as for MaxCut.  Errors: EINVAL for a zero
 * or out-of-range literal. */
ising_status ising_from_nae3sat(int32_t n, int64_t m, const int32_t *lits, int32_t *row_ptr, int32_t *col,
                                int32_t *val, int64_t *nnz_out, int64_t *base_out);

#ifdef __cplusplus
}
#endif
#endif /* ISING_H */
