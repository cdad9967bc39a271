/*
 * hsrq.h -- batched robust solves of shifted Hessenberg systems on MI355X.
 *
 * Computes, for an unreduced real upper Hessenberg matrix H and many distinct
 * shifts lambda_l (real, or complex given by one member of a conjugate pair),
 * the solutions of (H - lambda_l I) x_l = b_l of arXiv 2101.05063 ("Robust
 * level-3 BLAS inverse iteration from the Hessenberg matrix"): Henry's RQ
 * sweep (Sec. 2.2, Algorithm 1) rearranged into tiles so that the
 * back-substitution updates drawn from tiles of H shared by all shifts become
 * matrix-matrix products (Sec. 3.1, eq. update; Algorithms 6 and 10), with
 * power-of-two segment scale factors that keep every intermediate below the
 * overflow threshold (Sec. 4.1, eq. robust-update), complex Givens rotations
 * for complex shifts (Sec. 4.3, eq. cgivens), and the normalisation and
 * back-transform of Algorithm 11.  It returns unit 2-norm vectors together
 * with the binary scale of the true solution and a convergence flag
 * (Sec. 4.2).  With b_l a starting vector and lambda_l an eigenvalue estimate,
 * this is one step of inverse iteration and the outputs are eigenvectors.
 *
 * Conventions
 *   - All matrices are FP64, column-major with a leading dimension (LAPACK).
 *   - "device" pointers are HIP device memory of the handle's device;
 *     "host" pointers are ordinary host memory.
 *   - Column layout of X (Sec. 4.3): one column per real shift, two adjacent
 *     columns [re im] per complex shift, in the order of the shift list.
 *   - Calls are asynchronous on the handle's stream (hsrq_set_stream); device
 *     outputs are valid once that stream has been synchronised.  Host inputs
 *     (shift lists, problem descriptors) are consumed before the call returns.
 *   - Return value: HSRQ_OK, or a negative status.  A status of -k from the
 *     single-problem call means that its k-th argument is invalid (LAPACK
 *     convention).  Per-shift outcomes are reported in info[], never by the
 *     return value.
 *   - The library allocates no device memory inside a solve: the caller passes
 *     a workspace whose size is returned by the matching *_workspace_size
 *     call.  The handle owns a small pinned host staging buffer for the plan.
 *
 * Per-shift info codes
 *   0  converged: ||x_true||_2 / ||b||_2 >= 1 / (10 n eps ||H||_inf), the
 *      paper's convergence test (Sec. 4.2) without assuming b = ||H|| eps e
 *   1  not converged (the vector is still returned)
 *   2  exactly singular: R(1,1) = 0; the vector is the null vector Q^H e_1,
 *      scale_exp = INT32_MAX, scale_mant = 0
 *   3  non-finite entry in H (Hessenberg part) or in the shift
 *   4  H is not unreduced (a zero subdiagonal entry), which the method
 *      assumes (Sec. 1)
 */
#ifndef HSRQ_H
#define HSRQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    HSRQ_OK = 0,
    HSRQ_ERR_HIP = -1001,        /* a HIP runtime call failed */
    HSRQ_ERR_WORKSPACE = -1002,  /* workspace missing, too small or misaligned */
    HSRQ_ERR_ALLOC = -1003,      /* host staging allocation failed */
    HSRQ_ERR_ARG = -1004,        /* invalid argument in a batched/serving call */
    HSRQ_ERR_BUSY = -1005,       /* serving: the request does not fit the budget */
    HSRQ_ERR_TOO_LARGE = -1006   /* hsrq_dhsrq3_noalloc: the problem needs more
                                    than HSRQ_NOALLOC_SCRATCH_BYTES of workspace
                                    (or its plan more than the handle's 2 MiB
                                    staging buffer) */
};

typedef struct hsrq_handle_s* hsrq_handle_t;

/*
 * Options.  Zero-initialised options select the defaults.
 *   nb            tile size b_r of Sec. 3.2 (rows and columns of an H tile):
 *                 64 or 128; 0 = the choice of hsrq_autotune for this problem
 *                 set if it ran on the handle, else 128 when the largest
 *                 order is >= 2048 and 64 otherwise.
 *   Any other value of nb, precision (0, 1), residual (0, 1), graph
 *   (-1, 0, 1), rotations (0, 1), share_min_far (>= -1) or cols_per_block
 *   (0, 64; 32 with rotations 1 and precision 0) makes the call
 *   fail with the position of opts (LAPACK style: -16 for hsrq_dhsrq3, -5
 *   for hsrq_workspace_size) or HSRQ_ERR_ARG for the batched, tuning and
 *   debug calls; nothing is substituted silently.
 *   cols_per_block columns (shifts) per far-tile block, the b_c of Sec. 3.2:
 *                 64, or 32 in the level-3 form (rotations 1, precision 0);
 *                 0 = the tuner's choice for this problem set if it ran,
 *                 else 32 in the level-3 form and 64 otherwise.  Critical
 *                 blocks always take 8 columns.
 *   precision     0 = all FP64; 1 = tile-update products in FP32 on the
 *                 matrix cores, then a residual check per shift with a fall
 *                 back to the all-FP64 solve for shifts that fail it.
 *   residual      1 = also compute the FP64 normalised residual
 *                 ||H y - lambda y||_2 / (||H||_F ||y||_2) into resid[].
 *   graph         1 = replay the launch sequence as a HIP graph (captured on
 *                 the first call with the same plan shape, workspace and
 *                 residual option; up to 8 cached per handle); -1 = launch
 *                 kernel by kernel; 0 = default (graph for batched calls,
 *                 kernel by kernel for single calls).  Profiling forces
 *                 kernel-by-kernel launches.
 *   share_min_far the critical kernel of a tile-column step comes in two
 *                 variants that compute the same bits: one that takes a
 *                 compute unit to itself and one that leaves room on it for
 *                 one far-tile block.  Steps with at least share_min_far
 *                 far-tile blocks of 64 columns (two blocks of 32 columns
 *                 count as one) use the second.  0 = the library's default
 *                 (512), -1 = never; any value >= -1 is accepted.
 *   rotations     how the rotations of a tile column reach the cross-over
 *                 columns of the tile rows above its superdiagonal tile
 *                 (ReduceOffdiag, Sec. 3.1): 0 = one rotation at a time in
 *                 the order of Alg. 1 (default), so that every rotation,
 *                 R(k,k) and working column is bit-identical to that order;
 *                 1 = the NB rotations of a tile column folded into one
 *                 matrix W and applied as the product H(I, J-) W on the
 *                 matrix cores.  Form 1 agrees with form 0 to rounding: the
 *                 rotations, and the scale exponent of a shift whose system
 *                 is nearly singular, can then differ as far as the
 *                 conditioning allows.  The FP32 tile products of
 *                 precision 1 always use form 0.
 */
typedef struct {
    int nb;
    int cols_per_block;
    int precision;
    int residual;
    int graph;
    int rotations;
    int share_min_far;
    int reserved;
} hsrq_opts_t;

/* One problem of a batched call.  H, X, scale_exp, scale_mant, info and
   resid are device pointers; wr and wi are host arrays of length m. */
typedef struct {
    int n;
    const double* H;
    int ldh;
    int m;
    const double* wr;
    const double* wi;
    double* X;
    int ldx;
    int32_t* scale_exp;
    double* scale_mant;
    int32_t* info;
    double* resid;
} hsrq_problem_t;

/* Create a handle on HIP device `device` (the device is made current for the
   call).  Ownership of *out passes to the caller; release with hsrq_destroy. */
int hsrq_create(hsrq_handle_t* out, int device);

/* Release the handle, its pinned staging buffer and cached plans. */
int hsrq_destroy(hsrq_handle_t h);

/* Set the HIP stream (a hipStream_t, e.g. torch.cuda.current_stream()) that
   subsequent calls enqueue on.  NULL selects the null stream. */
int hsrq_set_stream(hsrq_handle_t h, void* stream);

/*
 * Workspace query for hsrq_dhsrq3: bytes of device workspace for a problem
 * of order n with the m shifts whose imaginary parts are wi (host, length m;
 * only wi != 0 matters).  Returns HSRQ_OK and writes *bytes.
 */
int hsrq_workspace_size(hsrq_handle_t h, int n, int m, const double* wi,
                        const hsrq_opts_t* opts, size_t* bytes);

/*
 * Solve (H - lambda_l I) x_l = b_l, l = 1..m, robustly (DHSRQ3, Algorithm 13,
 * generalised to complex shifts as in Algorithm 15), and normalise.
 *
 *   n            order of H (n >= 1)                                    arg 2
 *   H, ldh       device, n x n upper Hessenberg, ldh >= n; only the
 *                Hessenberg part is read; H is not modified             3, 4
 *   m            number of shifts (m >= 0)                              5
 *   wr, wi       host, shift l = wr[l] + i wi[l]; a complex shift stands
 *                for its conjugate pair; wi < 0 is accepted (the
 *                conjugate is solved and the result conjugated back)    6, 7
 *   X, ldx       device, n x ncols (ncols = #real + 2 #complex), in: the
 *                right-hand sides / starting vectors b_l, out: the unit
 *                2-norm vectors y_l = x_l / ||x_l||_2 in the same columns 8, 9
 *   scale_exp,   device, length m: ||x_l||_2 = scale_mant[l] * 2^scale_exp[l]
 *   scale_mant   with scale_mant in [0.5, 1) (exact binary exponent of the
 *                true, unscaled solution, which may exceed the double range) 10, 11
 *   info         device, length m, per-shift codes above                12
 *   resid        device, length m, or NULL (see opts.residual)           13
 *   work, work_bytes  device workspace, 256-byte aligned                14, 15
 *   opts         options or NULL                                         16
 */
int hsrq_dhsrq3(hsrq_handle_t h, int n, const double* H, int ldh,
                int m, const double* wr, const double* wi,
                double* X, int ldx,
                int32_t* scale_exp, double* scale_mant, int32_t* info,
                double* resid, void* work, size_t work_bytes,
                const hsrq_opts_t* opts);

/*
 * For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): hsrq_dhsrq3 with the
 * workspace taken from a fixed device array of HSRQ_NOALLOC_SCRATCH_BYTES
 * (64 MiB) inside the library.  Each device the library runs on holds its
 * own copy of the array from the first hsrq_create on it until the process
 * ends; the call itself allocates and creates nothing (no device, pinned or
 * graph memory, no events or streams), launches kernel by kernel on the
 * handle's stream and stages the plan through the handle's pinned buffer.
 *   Arguments 1-13 as for hsrq_dhsrq3 (the same statuses -1 .. -13);
 *   opts (arg 14) as for hsrq_dhsrq3 except that precision must be 0 and
 *   graph must not be 1 (status -14 otherwise).
 *   Returns HSRQ_ERR_TOO_LARGE, before anything is enqueued, when the
 *   problem's workspace (hsrq_workspace_size) exceeds the array or its plan
 *   exceeds the handle's staging buffer.
 * Every call on a device uses the same array, which keeps the last call's
 * contents (each call clears what must start at zero): calls that overlap
 * on one device, on any handles or streams, race and give wrong results;
 * serialise them (one stream, or synchronise between calls).
 */
#define HSRQ_NOALLOC_SCRATCH_BYTES (64u << 20)
int hsrq_dhsrq3_noalloc(hsrq_handle_t h, int n, const double* H, int ldh,
                        int m, const double* wr, const double* wi,
                        double* X, int ldx,
                        int32_t* scale_exp, double* scale_mant, int32_t* info,
                        double* resid, const hsrq_opts_t* opts);

/*
 * Inverse iteration with restarts (HSRQ3IN, Sec. 4.2, Algorithm 14, with
 * the grouping of Algorithm 15): every shift is solved from the starting
 * vector S(:, 0); the shifts that fail the convergence test are solved again
 * from S(:, 1), those that fail again from S(:, 2), and so on up to S(:,
 * ntries - 1), each try one hsrq_dhsrq3 of the shifts still open.  A complex
 * shift starts from the real vector S(:, t) (imaginary part zero).  The paper
 * takes each new starting vector orthogonal to the previous ones; the caller
 * supplies them, so that the same vectors can be given to any other
 * implementation.  Shifts are processed in groups of consecutive shifts
 * (a complex shift's two columns never split) with as many columns as the
 * workspace holds (Algorithm 15's w_max is work_bytes), so a small workspace
 * bounds the memory at the cost of more launches.
 *
 *   n, H, ldh, m, wr, wi   as for hsrq_dhsrq3                        2-7
 *   S, lds       device, n x ntries starting vectors, lds >= n         8, 9
 *   ntries       tries per shift (>= 1)                                10
 *   X, ldx       device, n x ncols, out only: the unit vectors of the last
 *                try of each shift, caller column layout               11, 12
 *   scale_exp, scale_mant, info   device, length m, as for hsrq_dhsrq3,
 *                of the returned try (info 1: no try converged)        13-15
 *   tries        device, length m, or NULL: the 0-based try whose result
 *                is returned                                           16
 *   resid        device, length m, or NULL (opts.residual)             17
 *   work, work_bytes  device workspace, 256-byte aligned; at least the
 *                bytes of a group of one shift (two columns if any shift
 *                is complex), at most hsrq_hsrq3in_workspace_size      18, 19
 *   opts         as for hsrq_dhsrq3; precision must be 0               20
 * The call synchronises the handle's stream once per try and group (the
 * flags decide the next try) and returns when the last try has been
 * enqueued.
 */
int hsrq_hsrq3in_workspace_size(hsrq_handle_t h, int n, int m, const double* wi,
                                const hsrq_opts_t* opts, size_t* bytes);
int hsrq_hsrq3in(hsrq_handle_t h, int n, const double* H, int ldh,
                 int m, const double* wr, const double* wi,
                 const double* S, int lds, int ntries,
                 double* X, int ldx,
                 int32_t* scale_exp, double* scale_mant, int32_t* info,
                 int32_t* tries, double* resid, void* work, size_t work_bytes,
                 const hsrq_opts_t* opts);

/*
 * The steps around the solve (Sec. 1): a general real matrix A is reduced to
 * upper Hessenberg form H = Q0^T A Q0, and an eigenvector x of H becomes the
 * eigenvector z = Q0 x of A.  Q0 = H_0 H_1 ... H_{n-3}, H_k = I - tau_k u_k
 * u_k^T, u_k zero above row k+1, u_k(k+1) = 1; the layout is LAPACK's DGEHRD
 * one, with H_k A(k+1:n, k) = beta e_1 and beta = -sign(A(k+1, k)) times the
 * norm of A(k+1:n, k).  The reduction is unblocked (one reflector at a
 * time; each step is one read and one write of the trailing matrix, which
 * also forms the products the next reflector needs); the back-transform is
 * blocked (panels of 128 reflectors applied as Z -= V T V^T Z, compact WY,
 * the products on rocBLAS DGEMM on the handle's stream; a rocBLAS handle is
 * created on the first call).  Both are asynchronous on the handle's stream,
 * workspace from the caller (256-byte aligned).  Run-to-run deterministic.
 *
 * hsrq_gehrd: A (device, n x n, lda >= n) in: general; out: H on and above
 *   the first subdiagonal, u_k(k+2:n) below it in column k.  tau (device,
 *   n - 1 entries; tau[n-2] = 0).  The result can be passed as the H of
 *   hsrq_dhsrq3 as it is (only the Hessenberg part is read there).
 *   Statuses -1 .. -6 for an invalid h, n, A, lda, tau, work.
 * hsrq_ormhr: Z (device, n x ncols, ldz >= n) <- Q0 Z, with A and tau as
 *   hsrq_gehrd left them.  Statuses -1 .. -9 for an invalid h, n, A, lda,
 *   tau, ncols, Z, ldz, work; HSRQ_ERR_HIP if rocBLAS cannot be set up or a
 *   product fails.
 */
int hsrq_gehrd_workspace_size(hsrq_handle_t h, int n, size_t* bytes);
int hsrq_gehrd(hsrq_handle_t h, int n, double* A, int lda, double* tau, void* work, size_t work_bytes);
int hsrq_ormhr_workspace_size(hsrq_handle_t h, int n, int ncols, size_t* bytes);
int hsrq_ormhr(hsrq_handle_t h, int n, const double* A, int lda, const double* tau, int ncols, double* Z, int ldz,
               void* work, size_t work_bytes);

/* Workspace query for hsrq_dhsrq3_batched (problems: host array of count
   descriptors; only n, m and wi are read). */
int hsrq_workspace_size_batched(hsrq_handle_t h, int count, const hsrq_problem_t* problems,
                                const hsrq_opts_t* opts, size_t* bytes);

/*
 * Many independent problems of uneven order in one launch sequence: every
 * tile-column step of every problem runs in the same kernel launch as the
 * steps of the others (one tile size for the whole set), and by default the
 * whole sequence is replayed as one HIP graph launch (opts->graph).
 * problems: host array of count descriptors (device data pointers inside).
 * Returns HSRQ_ERR_ARG if any descriptor is invalid.
 */
int hsrq_dhsrq3_batched(hsrq_handle_t h, int count, const hsrq_problem_t* problems,
                        void* work, size_t work_bytes, const hsrq_opts_t* opts);

/*
 * Mixed precision (opts->precision == 1).  The call runs in three phases on
 * the handle's stream: (1) the whole solve with the tile-update products in
 * FP32 on the matrix cores (operands scaled by powers of two into FP32 range,
 * FP32 accumulation over a tile; rotations, scale factors, small solves and
 * normalisation stay FP64) and the check value of every shift: the FP64
 * normalised residual when residuals are requested (resid[] given), else a
 * sketch of it, ||R^T (H y - lambda y)||_2 / ||H||_F with a fixed n x 8
 * matrix R of entries +-1/sqrt(8) (an unbiased estimate of the squared
 * residual, O(8 n) work per shift once R^T H is formed); (2) one host
 * synchronisation; a shift passes when it converged and its residual is at
 * most 10 n eps (eps = 2^-52), its sketch at most a quarter of that;
 * (3) the shifts that fail are
 * solved again from their starting vectors entirely in FP64 and their outputs
 * replace the first pass's.  Shifts flagged singular (2) or with invalid input
 * (3, 4) are final after phase 1.  The call therefore returns only after
 * phase 2; phase 3 is asynchronous.  Workspace: query with the same opts.
 * hsrq_fallback_count writes the number of shifts re-solved by the last such
 * call on the handle.
 */
int hsrq_fallback_count(hsrq_handle_t h, int64_t* count);

/*
 * Autotuner (tile size b_r and far-block width b_c, Sec. 3.2).  Runs the
 * solve of the given problem set once per candidate pair (b_r in {64, 128},
 * b_c in {32, 64} for the level-3 form, b_c = 64 otherwise) that fits the
 * workspace, timed with HIP events on the handle's stream, and records the
 * fastest for this problem set (keyed by the orders and column counts of its
 * problems) in the handle: later calls with opts->nb == 0 use its b_r, and
 * with opts->cols_per_block == 0 its b_c.  The caller's X, residuals and
 * starting vectors are left untouched; scale_exp, scale_mant and info
 * receive the results of a candidate run.  Synchronises the handle's stream.
 * *best_nb and *best_cb (host; best_cb may be NULL) receive the choice; ms
 * (host, length 4, may be NULL) the measured milliseconds per candidate at
 * index 2 (b_r == 128) + (b_c == 64) (0 for a candidate not run).  work as
 * for hsrq_dhsrq3_batched, sized with opts->nb == 0; opts (may be NULL) as
 * for the solve (its nb, cols_per_block and graph fields are ignored).
 * Returns HSRQ_ERR_WORKSPACE if no candidate fits.
 */
int hsrq_autotune(hsrq_handle_t h, int count, const hsrq_problem_t* problems, void* work, size_t work_bytes,
                  const hsrq_opts_t* opts, int* best_nb, int* best_cb, double* ms);

/*
 * Tuner cache.  hsrq_autotune_save writes the handle's tuned choices (one per
 * problem-set signature) to the text file at path (host string);
 * hsrq_autotune_load merges a file written by hsrq_autotune_save into the
 * handle (an entry replaces one with the same signature), so that a later
 * process skips the timing runs.  HSRQ_ERR_ARG if the file cannot be opened
 * or is malformed (then nothing is merged).
 */
int hsrq_autotune_save(hsrq_handle_t h, const char* path);
int hsrq_autotune_load(hsrq_handle_t h, const char* path);

/*
 * Debug/parity view of the workspace after a single-problem call: device
 * pointers to the recorded rotations (c, s and the diagonal of R; row k,
 * column c at [k * ld + c], internal column order) and the final working
 * columns (cross-overs entering each diagonal tile).  col_of[l] (host out,
 * length m) gives the internal column of shift l.  Valid until the workspace
 * is reused.
 */
int hsrq_debug_view(hsrq_handle_t h, int n, int m, const double* wi, const hsrq_opts_t* opts,
                    void* work, const double** C, const double** S, const double** PHI,
                    const double** V, int* ld, int* nb, int32_t* col_of);

/*
 * Profiling (for benchmarks; off by default).  While enabled, every kernel
 * launch of subsequent calls is bracketed by a pair of HIP events recorded
 * on the handle's stream.  hsrq_profile_read synchronises the recorded
 * events, writes per kernel family k (HSRQ_K_*) the accumulated milliseconds
 * ms[k] and the number of launches launches[k] (host arrays of nkinds
 * entries), and clears the accumulators.  Events are created by the library
 * (host-side handles; no device memory).  The far-tile kernels of a call run
 * on a second stream owned by the handle, forked from and joined back into
 * the handle's stream with events, so that they overlap the critical chain.
 */
enum {
    HSRQ_K_PREP = 0,    /* validity flags, norms of H and of its tiles */
    HSRQ_K_INIT = 1,    /* working columns and right-hand sides */
    HSRQ_K_CRIT = 2,    /* superdiagonal tile + diagonal Givens/solve chain */
    HSRQ_K_FAR = 3,     /* off-diagonal tile updates (MFMA) and rotations */
    HSRQ_K_FINAL = 4,   /* consistency scaling, norm, back-transform */
    HSRQ_K_OUTPUT = 5,  /* copy-out in the caller's column layout */
    HSRQ_K_RESID = 6,   /* optional FP64 residual */
    HSRQ_K_COUNT = 7
};
int hsrq_profile_enable(hsrq_handle_t h, int on);
int hsrq_profile_read(hsrq_handle_t h, int nkinds, double* ms, int64_t* launches);

/*
 * Serving: a request loop with continuous batching (one worker thread per
 * server, on HIP device `device`).
 *
 * hsrq_server_submit queues one problem (H and X device-resident, owned by
 * the caller and kept alive until its completion is polled; wr and wi are
 * copied).  stream (a hipStream_t; NULL is the null stream) is the stream on
 * which the caller produced H and X: the server's kernels for the request
 * wait for every piece of work enqueued on it before the call (an event
 * recorded on it at submission).  Requests are admitted in arrival order
 * while the sum of their
 * device bytes (workspace, which the server allocates from its own pool, plus
 * H and X) stays within hbm_budget_bytes.  Every admitted request advances one
 * tile-column step per tick; a tick is one critical and one far-tile launch
 * covering every admitted request at whatever step it is, so requests that
 * arrive while others run join at the next tick.  opts: nb (0 = 128),
 * precision (0 all FP64; 1 FP32 tile products with the FP64 residual check and
 * an FP64 re-solve of the failing shifts, see hsrq_fallback_count), residual
 * (write resid[] when the problem gives it), rotations (as for hsrq_dhsrq3).
 * Graph replay does not apply.
 * Returns HSRQ_ERR_BUSY from submit when the request can never fit (its bytes
 * exceed the budget or its task lists exceed a tick), HSRQ_ERR_ARG for an
 * invalid problem (n < 1, m < 1, missing pointers) or a stopped server.
 *
 * hsrq_server_poll moves up to `max` completion records (host array) out of
 * the server, waiting up to wait_ms milliseconds when none is ready; *count
 * receives how many.  Times are seconds on the server's steady clock
 * (hsrq_server_clock); latency = t_done - t_submit, where t_done is when the
 * worker observed the request's last kernel complete.  The return value is a
 * device error that stopped the server, else HSRQ_OK.
 * hsrq_server_destroy finishes every queued request, then releases the pool.
 */
typedef struct hsrq_server_s* hsrq_server_t;
typedef struct {
    uint64_t tag;
    int status;      /* HSRQ_OK or the error that failed the request */
    int fallback;    /* shifts re-solved in FP64 (precision 1) */
    double t_submit;
    double t_start;  /* admitted */
    double t_done;
} hsrq_completion_t;

int hsrq_server_create(hsrq_server_t* out, int device, size_t hbm_budget_bytes, const hsrq_opts_t* opts);
int hsrq_server_submit(hsrq_server_t server, const hsrq_problem_t* problem, uint64_t tag, void* stream);
int hsrq_server_poll(hsrq_server_t server, hsrq_completion_t* out, int max, int* count, int wait_ms);
int hsrq_server_clock(hsrq_server_t server, double* seconds);
int hsrq_server_destroy(hsrq_server_t server);

#ifdef __cplusplus
}
#endif

#endif /* HSRQ_H */
