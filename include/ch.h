/*
 * ch.h -- C ABI of the MI355X (gfx950) library for the explicit time steps of
 * the space-discretised Cahn-Hilliard equation
 *
 *     y' = -A (F'(y) + eps^2 A y),   F'(y) = y^3 - y        (Section 2, eq. IVP, eq. F)
 *
 * on a grid of n^dim points over [0,L]^dim (h = L/n; periodic, or with the
 * homogeneous Neumann conditions of the paper on a cell-centred grid), where
 * -A is the standard (2 dim + 1)-point Laplacian.  Two schemes of Botchev (arXiv
 * 2502.14589) are provided:
 *
 *   EE2  exponential Euler of order 2 (Section 4): the Jacobian is frozen at
 *        y^n, giving y' = -Ahat_n y + ghat^n (eq. IVPlin) with
 *        Ahat_n = A (J_n + eps^2 A), ghat^n = A (J_n y^n - F'(y^n)) (eq. A_g);
 *        its solution y^n + tau phi(-tau Ahat_n)(ghat^n - Ahat_n y^n) (eq. yt) is
 *        evaluated by the Arnoldi process with the residual-time (RT) restart
 *        of the Krylov algorithm (Fig. 3) -- by default with classical
 *        Gram-Schmidt applied twice and its second projection delayed
 *        (CH_ORTH_DCGS2), or with the modified Gram-Schmidt that Fig. 3
 *        prints (CH_ORTH_MGS); adaptive steps follow Fig. 4 (eqs. tol_phi,
 *        LIMest, EEdt).
 *   LIM  the Chebyshev local-iteration scheme (Fig. 1), 2p-1 explicit-Euler-like
 *        stages with p from eq. p and lambda_max = ||Ahat_n||_1; adaptive steps
 *        follow Fig. 2 (eqs. LIMest, LIMdt).
 *
 * With eyre != 0 both use the Eyre splitting (eq. A_g_cs).
 *
 * Memory and streams.  Every field argument is a DEVICE pointer to a
 * contiguous FP64 array of n^dim values, row-major with x fastest
 * (index = (z n + y) n + x), owned by the caller.  The library owns all
 * scratch (Krylov basis, state ping-pong buffers, reduction partials, control
 * block); it is sized lazily to the largest problem seen and freed by
 * ch_destroy.  All work is issued on the stream given to ch_create; every
 * call below returns after that stream has drained the call's work (host and
 * device agree on the result when the call returns).
 *
 * Errors.  Every call returns a ch_status; nothing aborts or throws across
 * the ABI.  When a call fails, the caller's field holds the last state that
 * was fully accepted (for a one-step call: its input, unchanged).
 *
 * Threading.  A context is used by one host thread at a time.
 */
#ifndef CH_H
#define CH_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ch_ctx ch_ctx;

enum ch_status {
    CH_OK = 0,
    CH_EINVAL = -1,          /* bad argument: dim not 2/3, n < 5, eps <= 0, tau <= 0, m_max out of range, NULL */
    CH_ENOMEM = -2,          /* device allocation failed */
    CH_ENONFINITE = -3,      /* a NaN/Inf appeared in the input or in a step */
    CH_ETAU_UNDERFLOW = -4,  /* the residual-time trace found no admissible step >= tau_min */
    CH_EBUSY = -5,           /* serving queue full */
    CH_ENOENT = -6,          /* unknown ticket */
    CH_EDEVICE = -7          /* HIP runtime error (see ch_last_error_message) */
};

enum ch_precision {
    CH_FP64 = 0,        /* every vector and stencil in FP64 */
    CH_FP32_MIXED = 1   /* Krylov basis, matvecs and MGS axpys in FP32; state, reductions,
                           Hessenberg phi, solution update and error estimate in FP64 */
};

/* Largest Krylov dimension m_max: the paper's EE2(100) of Table 1.  The phi
 * of H_{m,m} runs in one workgroup: in its LDS up to order 48 (Krylov
 * dimension 47), beyond that in a device scratch of 0.6 MB per instance. */
#define CH_MMAX 100
/* Largest Chebyshev order p of one LIM step. */
#define CH_PMAX 4096
/* Largest grid (points) of ch_step_lim_noalloc. */
#define CH_NOALLOC_MAX_POINTS (1 << 20)

/*
 * Boundary conditions of the grid (Section 2, eq. CH; Section 5.1).
 *   CH_BC_PERIODIC: nodes x_i = i h on the torus [0, L)^dim.
 *   CH_BC_NEUMANN: homogeneous Neumann conditions for c and mu on the
 *     cell-centred grid x_i = (i + 1/2) h of (0, L)^dim (the paper's test
 *     problem): a mirror ghost cell y_{-1} = y_0, y_n = y_{n-1}, so the
 *     boundary rows of A have (number of neighbours) / h^2 on the diagonal,
 *     A is symmetric positive semidefinite and A 1 = 0.  2-D only.
 */
enum ch_bc { CH_BC_PERIODIC = 0, CH_BC_NEUMANN = 1 };

typedef struct {
    int dim;        /* 2 or 3 */
    int n;          /* grid points per direction, >= 5; h = length / n */
    double eps;     /* interface parameter epsilon > 0 */
    int eyre;       /* 0: eq. A_g; 1: Eyre splitting eq. A_g_cs */
    int prec;       /* ch_precision (EE2 only; LIM always runs in FP64) */
    int bc;         /* ch_bc (0, the zero-initialised default: periodic) */
    double length;  /* side L of the domain (<= 0: 1, the unit cube) */
    /* Variable mobility (Section 2, Remark 1): with mobility != 0 the equation is
     * c_t = div(M(c) grad mu), M(c) = max(mob0 + mob1 (1 - c^2), 0), discretised as
     * y' = -A_M(y) (F'(y) + eps^2 A y), (A_M v)_i = h^-2 sum over the neighbours k of
     * (M_i + M_k)/2 (v_i - v_k); A_M is frozen at y^n within a step:
     * Ahat_n = A_M(y^n) (J_n + eps^2 A [+ I]).  Single 2-D periodic grids only: with
     * dim 3, Neumann boundaries, negative or non-finite coefficients or mob0 + mob1 = 0
     * the calls return CH_EINVAL.  mobility = 0 (zero-initialised) is M = 1. */
    int mobility;
    double mob0, mob1;
} ch_problem;

/*
 * Orthogonalisation of the Arnoldi process (Fig. 3 of Section 4.1).  Both give
 * the same basis and Hessenberg matrix in exact arithmetic; they differ in
 * rounding and in cost.
 *   CH_ORTH_DCGS2 (default): classical Gram-Schmidt applied twice -- twice is
 *     enough for orthogonality to working precision (Giraud, Langou,
 *     Rozloznik, Comput. Math. Appl. 50 (2005)) -- with the second projection
 *     of each vector delayed into the next iteration (the low-synchronisation
 *     Gram-Schmidt idea of Swirydowicz et al., Numer. Linear Algebra Appl.,
 *     2021): one reduction and two streaming passes over the basis per
 *     iteration, whatever j.  The test of dimension j waits for the matvec of
 *     the (j+1)-th vector, so each Krylov cycle makes one matvec more than it
 *     reports (the paper's count).
 *   CH_ORTH_MGS: modified Gram-Schmidt as printed in Fig. 3, one streaming
 *     pass per basis vector (j + 1 passes in iteration j).
 */
enum ch_orth { CH_ORTH_DCGS2 = 0, CH_ORTH_MGS = 1 };

typedef struct {
    int m_max;              /* Krylov dimension, 1..CH_MMAX */
    double tol;             /* accuracy tolerance of eq. EEdt and eq. tol_phi */
    double tol_phi_fixed;   /* > 0: use this tol_phi instead of eq. tol_phi */
    double tau_min;         /* trace underflow threshold (>= 0) */
    int constant_step;      /* 1: constant tau with linear RT restarts (no controller) */
    int orth;               /* ch_orth (0, the zero-initialised default: CH_ORTH_DCGS2) */
    /* DCGS2 only: > 0 issues the Arnoldi iterations of a cycle as HIP graphs of
     * graph_chunk iterations each (1..CH_MMAX + 1), captured once per context,
     * instance table and buffers and then replayed; 0 launches every kernel
     * directly.  The launches and their results are the same either way. */
    int graph_chunk;
} ch_ee_opts;

/* Per-step record (one per accepted step). */
typedef struct {
    double t;           /* time after the step */
    double tau;         /* accepted step */
    double tau_next;    /* proposal for the next step */
    double est;         /* eq. LIMest estimate */
    double tol_phi;     /* Krylov tolerance used (EE2) */
    double beta;        /* ||ghat - Ahat y^n|| (EE2) */
    double resnorm;     /* final ||r||/beta of the last Krylov cycle (EE2) */
    double lambda_max;  /* ||Ahat||_1 (LIM) */
    int j;              /* Krylov dimension of the last cycle (EE2) / Chebyshev order p (LIM) */
    int cycles;         /* Krylov cycles in the step (EE2; > 1 only with constant_step) */
    int traced;         /* the RT trace shortened the step (EE2) */
    int matvecs;        /* matvecs with Ahat_n in the step, counted as the paper does */
} ch_step_record;

typedef struct {
    double t;               /* time reached */
    double tau_next;        /* proposed next step */
    int steps;              /* accepted steps */
    long long matvecs;      /* total matvecs with Ahat_n */
    int restarts;           /* Krylov cycles beyond the first, summed over steps */
    int traces;             /* steps shortened by the RT trace */
    int status;             /* ch_status of the run */
} ch_run_stats;

/* Create a context on HIP device `device`; `hip_stream` is a hipStream_t (NULL: the null stream). */
int ch_create(ch_ctx **ctx, int device, void *hip_stream);
int ch_destroy(ch_ctx *ctx);
const char *ch_strerror(int status);
/* Text of the last HIP runtime error seen by this context ("" if none). */
const char *ch_last_error_message(ch_ctx *ctx);

/*
 * Adaptive (Fig. 4) or constant-step EE2 run on the field y (in/out).
 * Starts at time t0 with proposed step tau0 and advances until t >= T or
 * max_steps steps were accepted (T may be INFINITY; max_steps <= 0: no limit,
 * then T must be finite).  Every step clips tau to T - t (Fig. 4).
 * records: NULL or an array of max_steps ch_step_record (host memory).
 */
int ch_run_ee(ch_ctx *ctx, const ch_problem *prob, double *y, double tau0, double t0, double T,
              int max_steps, const ch_ee_opts *opts, ch_run_stats *stats, ch_step_record *records);

/* One EE2 step (Fig. 3 with the controller of Fig. 4): ch_run_ee with max_steps = 1. */
int ch_step_ee(ch_ctx *ctx, const ch_problem *prob, double *y, double tau, double t, double T,
               const ch_ee_opts *opts, ch_step_record *out);

/* One instance of a batched run: a periodic grid of n^dim points. */
typedef struct {
    int n;          /* points per direction, >= 5 */
    double eps;     /* interface parameter epsilon > 0 */
    double *y;      /* DEVICE field, in/out, FP64, n^dim values (x fastest) */
    double tau0;    /* first proposed step > 0 */
    double T;       /* final time (INFINITY: limited by max_steps) */
    int max_steps;  /* accepted steps to take (<= 0: until T) */
} ch_batch_item;

/*
 * Adaptive EE2 (Fig. 4) on `count` independent instances at once: every
 * kernel launch covers all instances (ragged sizes, each with its own eps,
 * step sizes, Krylov convergence, final time and step limit), so the small
 * per-instance launches of separate runs become one launch per kernel.  dim,
 * eyre, precision, Krylov dimension and tolerances (opts) are common;
 * opts->constant_step must be 0.  Each instance's result equals that of a
 * separate ch_run_ee call up to the order of floating-point sums, and does not
 * depend on the other members of the batch.  stats: NULL or `count` entries.
 * Returns the first failing instance's status; the other instances complete.
 */
int ch_run_ee_batch(ch_ctx *ctx, int count, ch_batch_item *items, int dim, int eyre, int prec,
                    const ch_ee_opts *opts, ch_run_stats *stats);

/*
 * Adaptive (Fig. 2, tol > 0) or constant-step (tol <= 0) LIM run on y (in/out),
 * same conventions as ch_run_ee.
 */
int ch_run_lim(ch_ctx *ctx, const ch_problem *prob, double *y, double tau0, double t0, double T,
               int max_steps, double tol, ch_run_stats *stats, ch_step_record *records);

/*
 * Adaptive (Fig. 2, tol > 0) or constant-step (tol <= 0) LIM on `count`
 * independent instances at once (ragged sizes, each with its own eps, step
 * sizes, final time and step limit; items as for ch_run_ee_batch): every
 * kernel launch covers all instances.  Each step's Chebyshev order p (eq. p)
 * is each instance's own; the stage launches run up to the largest, and an
 * instance skips those past its last stage.  Each instance's result equals
 * that of a separate ch_run_lim call (bit for bit) and does not depend on the
 * other members.  stats: NULL or `count` entries.  Returns the first failing
 * instance's status; the other instances complete.
 */
int ch_run_lim_batch(ch_ctx *ctx, int count, ch_batch_item *items, int dim, int eyre, double tol,
                     ch_run_stats *stats);

/* One LIM step (Fig. 1 with the controller of Fig. 2). */
int ch_step_lim(ch_ctx *ctx, const ch_problem *prob, double *y, double tau, double t, double T,
                double tol, ch_step_record *out);

/*
 * For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): ch_step_lim without
 * any allocation.  Same arguments, kernels and result as ch_step_lim; its
 * scratch (two state buffers and a stage buffer of up to
 * CH_NOALLOC_MAX_POINTS points, reduction partials, node order, stage
 * coefficients, control block, step record, instance table: 26.3 MB) is a
 * file-scope device array that every GPU the library runs on holds until the
 * process ends, located per device by ch_create.  A grid of more than
 * CH_NOALLOC_MAX_POINTS points returns CH_EINVAL (ch_last_error_message says
 * why); a device without that address returns CH_EDEVICE.  The call makes no
 * hipMalloc, hipFree or other allocating call; like ch_step_lim it reads the
 * Chebyshev order back to the host once and returns after its stream has
 * drained.  Every call on one GPU shares that GPU's scratch: calls that
 * overlap on one GPU (from several threads or contexts) race and must be
 * serialised by the caller.  The control block, the instance record and the
 * maps are rewritten by every call; nothing carries over between calls.
 */
int ch_step_lim_noalloc(ch_ctx *ctx, const ch_problem *prob, double *y, double tau, double t, double T,
                        double tol, ch_step_record *out);

enum ch_phi_mode {
    CH_PHI_SHRINK = 0,   /* one Fig. 3 cycle: the RT trace may shorten tau (nonlinear RT restart) */
    CH_PHI_RESTART = 1   /* linear RT restarts until the whole tau is covered */
};

/*
 * y_out = y + tau phi(-tau Ahat_n)(ghat^n - Ahat_n y) (eq. yt) with Ahat_n, ghat^n frozen
 * at y (eq. A_g / A_g_cs); y is not modified; y_out may not alias y.
 * out->tau is the step actually covered (< tau0 only in CH_PHI_SHRINK mode).
 * The Arnoldi process uses CH_ORTH_DCGS2.
 */
int ch_phiv(ch_ctx *ctx, const ch_problem *prob, const double *y, double *y_out, double tau0,
            int mode, double tol_phi, int m_max, ch_step_record *out);

/*
 * Serving: continuous batching of EE2 and LIM solve requests on one GPU.
 *
 * A server owns a private context and stream and a scheduler thread.  Each
 * request is copied to device memory at submit and queued.  Between batch
 * steps, the scheduler admits queued requests in arrival order while a control
 * block, pooled HBM for the request's footprint and workgroup-table room are
 * free.  The footprint is ((m_max + 1) w + 28) bytes per grid point, where
 * w = 8 (FP64) or 4 (FP32-mixed), whatever the method.  All admitted requests
 * advance together, one adaptive step per batch step (EE2: Fig. 4; LIM:
 * Fig. 2, always in FP64), each with its own grid, eps, tolerance, steps and
 * final time.  Finished requests leave the batch, freeing their slot and
 * memory for the queue.  A request's result does not depend on what else was
 * in the batch: it equals that of a separate ch_run_ee or ch_run_lim call.
 */
typedef struct ch_server ch_server;

enum ch_method { CH_METHOD_EE = 0, CH_METHOD_LIM = 1 };

typedef struct {
    int n;              /* points per direction (2-D periodic, h = 1/n), >= 5 */
    double eps;         /* interface parameter epsilon > 0 */
    const double *y0;   /* FP64 field, n*n values, device or host (y0_on_host); copied at submit */
    int steps;          /* accepted steps to take (<= 0: until T, which must then be finite) */
    double tau0;        /* first proposed step > 0 */
    int method;         /* ch_method */
    double T;           /* final time (INFINITY: the horizon is `steps`); the last step is clipped onto it */
    double tol;         /* > 0: this request's tolerance (eqs. EEdt / LIMdt, tol_phi); <= 0: the server's
                           (LIM with both <= 0: constant steps of tau0) */
    int y0_on_host;     /* 0: y0 is device memory; 1: host memory */
} ch_request;

enum ch_request_state { CH_REQ_QUEUED = 0, CH_REQ_RUNNING = 1, CH_REQ_DONE = 2, CH_REQ_FAILED = 3 };

/* Create a server on `device`: precision, Krylov dimension and the default
 * tolerances (opts; constant_step must be 0) are common to all EE2 requests;
 * hbm_budget is the pooled footprint in bytes; max_slots bounds the requests
 * in flight. */
int ch_server_create(int device, int prec, const ch_ee_opts *opts, size_t hbm_budget, int max_slots,
                     ch_server **out);
/* Stops admitting, finishes the requests in flight, fails the queued ones, frees everything. */
int ch_server_destroy(ch_server *srv);
/*
 * Queue a request; CH_ENOMEM if its footprint can never fit the budget.
 * Thread-safe.  y0 is copied on the server's own non-blocking stream before
 * the call returns, so the work that writes y0 must have completed when it is
 * called (the copy does not wait for other streams).  Request buffers are
 * recycled: steady serving makes no device allocation.  A request's latency
 * counts from the moment ch_submit is entered.
 */
int ch_submit(ch_server *srv, const ch_request *req, unsigned long long *ticket);
/*
 * State of a request.  When it is CH_REQ_DONE and y_out (DEVICE, n*n FP64) is
 * not NULL, the result is copied there (complete when the call returns) and
 * the ticket is released (later polls return CH_ENOENT).  stats and latency_s
 * (queue wait, service, total in seconds) may be NULL.  Thread-safe.
 */
int ch_poll(ch_server *srv, unsigned long long ticket, int *state, double *y_out, ch_run_stats *stats,
            double *latency_s);

enum ch_kernel {
    CH_KERNEL_MGS = 0,      /* one modified Gram-Schmidt pass (axpy + next dot) over the grid */
    CH_KERNEL_MATVEC = 1,   /* one fused Jacobian matvec Ahat v with its first dot */
    CH_KERNEL_PHI = 2,      /* one small-matrix phi evaluation of the last step's H (no trace) */
    /* the CH_ORTH_DCGS2 passes of the Arnoldi iteration j each launch names: */
    CH_KERNEL_DC_MATVEC = 3,   /* matvec Ahat u_j with the 2j + 2 dot products against the basis */
    CH_KERNEL_DC_UPDATE = 4,   /* q_j and u_{j+1} from one pass over the basis (without the phi
                                  test workgroup a run's update launch may carry) */
    CH_KERNEL_LIM_STAGE = 5,   /* one LIM Chebyshev stage */
    CH_KERNEL_DC_ITER = 6,     /* one whole DCGS2 iteration: matvec, dot totals, update */
    CH_KERNEL_LIM_STAGE2 = 7   /* two consecutive LIM stages in one launch (2-D only: the form
                                  ch_run_lim uses there for every stage after the first) */
};

/*
 * Measurement aid for the roofline figures: `count` back-to-back launches of
 * one kernel of the path, bracketed by HIP events on the context's stream, on
 * the workspace of an earlier run on this problem (ch_run_ee with Krylov
 * dimension >= m_max; ch_run_lim for CH_KERNEL_LIM_STAGE and CH_KERNEL_LIM_STAGE2).  iters[i] is the
 * Arnoldi iteration of launch i: CH_KERNEL_DC_MATVEC 0..m_max (w stored below
 * m_max), CH_KERNEL_DC_UPDATE and CH_KERNEL_DC_ITER 0..m_max-1, CH_KERNEL_MGS (pass 1 of the
 * iteration) 1..m_max-1, CH_KERNEL_MATVEC 0..m_max-1, CH_KERNEL_PHI (a
 * not-converged test of that dimension) 1..min(m_max-1, last step's j);
 * ignored (may be NULL) for the two LIM kernels; CH_KERNEL_LIM_STAGE2 on a 3-D
 * problem returns CH_EINVAL.  The DCGS2 and LIM kernels
 * are launched under a symbol of their own, so a profiler reports these
 * launches apart from the path's.  *total_us: elapsed time of the sequence;
 * *total_bytes: its algorithmic bytes (each operand vector read or written
 * once).  Overwrites basis columns and the control block with values of no
 * meaning; a later run re-initialises them.
 */
int ch_time_kernel(ch_ctx *ctx, const ch_problem *prob, int kernel, int m_max, const int *iters, int count,
                   double *total_us, double *total_bytes);

/*
 * Launch shape of one grid (dim, n, precision); the same for every instance of
 * that grid in single runs, batches and served requests on the context:
 *   vx    2-D: grid columns per lane of the row-strip kernels (1, 2, or 4 in
 *         FP32-mixed; a divisor of n); unused in 3-D;
 *   wblk  workgroups of the 2-D row-strip kernels or the 3-D marching matvec
 *         (1..2048; each loops over its share of strips, or of x-y blocks
 *         and runs of planes).  Built in: one per four strips, or 512 when
 *         that would exceed 2048; in 3-D one per work item, at most 2048;
 *   cblk  workgroups of the streaming passes (DCGS2 update, state update):
 *         1..512, each looping over chunks of 2048 points.
 * The shape changes the order in which the partial sums of dot products are
 * added, so results of two shapes agree to rounding, not bit for bit.  LIM runs
 * use the shape of (dim, n, CH_FP64).
 */
typedef struct {
    int vx;
    int wblk;
    int cblk;
} ch_shape;

/* The shape runs on this context use for (dim, n, prec): the one set or tuned
 * last, else the built-in choice.  CH_EINVAL for an invalid grid or precision. */
int ch_get_shape(ch_ctx *ctx, int dim, int n, int prec, ch_shape *out);

/* Sets the shape of (dim, n, prec) for later runs on this context; shape NULL
 * restores the built-in choice.  CH_EINVAL for an out-of-range shape. */
int ch_set_shape(ch_ctx *ctx, int dim, int n, int prec, const ch_shape *shape);

/*
 * Launch-shape tuner for one grid and precision (prob->dim, n, prec) at Krylov
 * dimension m_max (DCGS2): times the matvec with its dot products for every
 * valid vx and workgroup counts from the built-in choice down to a quarter of
 * it, plus the counts below it that make whole rounds of two to four
 * workgroups per CU, then the update pass for streaming workgroup counts
 * likewise, each over
 * Arnoldi iterations 1, m_max/2 and m_max - 1 (back-to-back launches under HIP
 * events, best of three), and keeps the fastest shape for later runs on this
 * context (as ch_set_shape).  *best: that shape; *best_us and *default_us: the
 * time of one matvec plus one update pass, averaged over those iterations, for
 * it and for the built-in choice.  Allocates the workspace of such a run and
 * overwrites its contents.
 */
int ch_tune_shape(ch_ctx *ctx, const ch_problem *prob, int m_max, ch_shape *best, double *best_us,
                  double *default_us);

/*
 * Launch-shape tuner for a batch (ch_run_ee_batch): the grids of items[0..count)
 * (n and eps are read; y, tau0, T and max_steps are not), all in precision
 * prec, timed together as ch_run_ee_batch launches them, one DCGS2 iteration
 * (matvec, dot totals, update pass) over all instances at Arnoldi iterations 1,
 * m_max/2 and m_max - 1 (best of three).  Starting from the built-in shapes, it
 * visits each distinct n, largest total size first, tries for it the candidate
 * shapes of ch_tune_shape with the others fixed, and keeps a change when the
 * whole batch's iteration gets at least 0.5% faster.  The chosen shapes are
 * kept for later runs on this context.  *best_us and *default_us: one batched
 * iteration with them and with the built-in shapes.  Allocates the workspace
 * of such a batch and overwrites its contents.
 */
int ch_tune_batch_shapes(ch_ctx *ctx, int count, const ch_batch_item *items, int dim, int eyre, int prec, int m_max,
                         double *best_us, double *default_us);


#ifdef __cplusplus
}
#endif
#endif /* CH_H */
