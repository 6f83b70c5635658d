/*
 * msfv.h -- C ABI of the MI355X (gfx950) adaptive multiscale finite volume
 * (MSFV) library.
 *
 * Method: Wu Fung & Ruthotto, "A Multiscale Method for Model Order Reduction
 * in PDE Parameter Estimation" (arXiv:1707.07598).
 *
 *   forward  F_k(m) = Rx^T S_k(m) A_k(m)^{-1} S_k(m)^T Q        (eq. fwdProbRed)
 *            A_k(m) = S_k(m)^T A(m) S_k(m)                       (eq. reducedPDE)
 *            S_k(m) = the parameter-dependent multiscale basis   (Sec. 3.2,
 *                     eq. multiscaleBasis_step3, rebuilt at every call)
 *   gradient J_k(m)^T v, the transposed adaptive sensitivity     (Sec. 4.1,
 *            eq. Jk; Sec. 4.3, eq. sensred; Sec. 4.5)
 *
 * Discretisation: -div(exp(m) grad u) = q on a uniform cell-centred grid with
 * unit spacing, harmonic-mean two-point fluxes, no-flux outer boundary, and
 * the potential fixed at coarse vertex 0 (Sec. 2.1-2.2).
 *
 * Conventions
 *   - All values are FP64, all indices int32.
 *   - cell id   = i + nx*(j + ny*k)            (x fastest; 2-D: nz = 1)
 *   - vertex id = I + Ncx*(J + Ncy*K), Nc = ceil(n/r) per axis, vertex I of an
 *     axis sits at cell I*r + floor(min(r, n - I*r)/2).
 *   - Sources and receivers are sparse columns given as CSR over columns:
 *     ptr[count+1], cell[ptr[count]], val[ptr[count]] (host arrays, copied).
 *   - D (data), v and d_obs are Nr x Ns, column j contiguous: D[j*Nr + i].
 *   - u (fields) is N x Ns, column j contiguous: u[j*N + cell].
 *   - S_k is CSR by fine cell, columns ascending; A_k is CSR by vertex.
 *
 * Ownership and streams
 *   - m, v, d_obs and every output pointer passed to msfv_forward,
 *     msfv_jtv and msfv_misfit_grad are DEVICE pointers owned by the caller.
 *     Calls are asynchronous on the problem's HIP stream; outputs are valid
 *     after msfv_sync() (or any synchronisation of that stream).
 *   - The library owns S_k, A_k, the coarse coefficients, all workspace and
 *     the plan; they stay resident on the device between calls.
 *   - Introspection calls (msfv_get_*) take HOST pointers and synchronise.
 *
 * Errors
 *   - Every call returns an msfv_status; nothing throws across the ABI.
 *     msfv_last_error() returns a thread-local message for the last failure.
 *   - Device-side conditions (non-finite m, a local or coarse iteration that
 *     reached its cap) are recorded on the device and reported by the next
 *     msfv_sync(): MSFV_ENONFINITE takes precedence over MSFV_ENOCONV.
 *     Outputs are still written in both cases.
 *   - msfv_jtv before any msfv_forward returns MSFV_ESTATE.
 */
#ifndef MSFV_H
#define MSFV_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct msfv_problem msfv_problem;

typedef enum {
  MSFV_OK = 0,
  MSFV_EINVAL = -1,     /* bad argument or unsupported geometry            */
  MSFV_ENOMEM = -2,     /* device or host allocation failed                */
  MSFV_ENOCONV = -3,    /* a local or coarse iteration reached its cap     */
  MSFV_ENONFINITE = -4, /* m contained NaN or Inf                          */
  MSFV_EDEVICE = -5,    /* a HIP runtime call failed                       */
  MSFV_ESTATE = -6      /* call out of order (e.g. jtv before forward)     */
} msfv_status;

/* Boundary data of the local problems (Sec. 3.2).
 *   MSFV_BC_REDUCED : edges, then faces, then dual-block interiors are all
 *                     solved with their reduced (tangential) operators, so
 *                     the block-boundary values depend on m.
 *   MSFV_BC_LAGRANGE: block-boundary values are products of 1-D linear
 *                     Lagrange factors ("Piecewise Lagrange Polynomials");
 *                     only dual-block interiors are solved.              */
enum { MSFV_BC_REDUCED = 0, MSFV_BC_LAGRANGE = 1 };

typedef struct {
  int dim;            /* 2 or 3; for dim 2, n[2] and r[2] are ignored        */
  int n[3];           /* fine cells per axis                                 */
  int r[3];           /* coarsening per axis, 3 <= r <= 16                   */
  int bc_mode;        /* MSFV_BC_REDUCED or MSFV_BC_LAGRANGE                 */
  double local_rtol;  /* local CG stop: ||r|| <= local_rtol*||b|| (0: 1e-13) */
  int local_maxit;    /* cap on local CG iterations (0: 1000)                */
  double coarse_rtol; /* coarse CG stop (0: 1e-13)                           */
  int coarse_maxit;   /* cap on coarse CG iterations (0: 20000)              */
  int coarse_precond;  /* MSFV_COARSE_TWOLEVEL or MSFV_COARSE_JACOBI (below) */
} msfv_config;

/* Preconditioner of the coarse CG (same stop test and iteration cap either
 * way; results agree to the coarse tolerance).
 *   MSFV_COARSE_TWOLEVEL: Jacobi plus an additive correction on boxes of
 *                         coarse vertices, M^-1 = D^-1 + Z (Z^T A Z)^-1 Z^T
 *                         (at most 64 boxes); falls back to Jacobi where its
 *                         tables do not fit in on-chip memory.
 *   MSFV_COARSE_JACOBI  : M^-1 = D^-1.
 *   MSFV_COARSE_MULTI   : M^-1 = D^-1 with the multi-launch solver that
 *                         grids of more than 8192 vertices always use (all
 *                         right-hand sides per launch; the call returns when
 *                         the solve has finished).                         */
enum { MSFV_COARSE_TWOLEVEL = 0, MSFV_COARSE_JACOBI = 1, MSFV_COARSE_MULTI = 2 };

typedef struct {
  long long ncell;     /* N                                                  */
  long long ncoarse;   /* Nc (columns of S_k)                                */
  long long nnz_p;     /* nonzeros of S_k                                    */
  long long nnz_k;     /* nonzeros of A_k                                    */
  int nsrc;            /* Ns                                                 */
  int nrec;            /* Nr                                                 */
  int nblock;          /* dual-block interiors solved per basis build        */
  int nface;           /* face entities (3-D)                                */
  int nedge;           /* edge entities                                      */
  long long workspace_bytes; /* device bytes held by the problem             */
  long long pairs_block; /* (own cell, corner) pairs of the dual-block solves */
  long long pairs_face;  /* the same for the faces (3-D) or 2-D blocks      */
} msfv_sizes;

/* The local-solve figures (iteration count, final residual) cover the
 * basis solves of the last forward and the adjoint solves of the J^T v
 * after it; the other counters run since the last forward, msfv_jvp or
 * msfv_jvp_fixed (each of these resets them; msfv_jtv and msfv_jtv_fixed add
 * to them).  Residuals are relative, ||r|| /
 * ||b|| of a solve's final iterate (local solves on the Jacobi-scaled local
 * system; coarse solves on the pinned Galerkin system); +inf marks a solve
 * that produced a non-finite residual.                                     */
typedef struct {
  int local_max_it;       /* largest local CG iteration count                */
  int local_noconv;       /* local solves that hit the cap                   */
  int coarse_max_it;      /* largest coarse CG iteration count               */
  int coarse_noconv;      /* coarse solves that hit the cap                  */
  int nonfinite;          /* 1 if m contained NaN/Inf                        */
  double local_max_res;   /* largest final relative residual, local solves  */
  double coarse_max_res;  /* the same for the coarse solves                  */
} msfv_stats;

/* Create a problem for one grid; builds the plan (entity tables, CSR
 * structure of S_k and A_k) and allocates its device state.  hip_stream is a
 * hipStream_t (NULL = default stream).  Unsupported geometry returns
 * MSFV_EINVAL: r outside [3, 16], n < 2 on an axis, more than 2^21 coarse
 * vertices or 2^31 cells.  Coarse grids of more than 8192 vertices are
 * solved by a multi-launch Jacobi-PCG whose forward and J^T v calls return
 * only when their coarse solves have finished (the host polls stop flags). */
msfv_status msfv_create(const msfv_config* cfg, void* hip_stream, msfv_problem** out);

/* Release all device and host state.  NULL is ignored. */
void msfv_destroy(msfv_problem* p);

/* Set the sources Q (Sec. 2.1, q_j) as sparse columns (host arrays). */
msfv_status msfv_set_sources(msfv_problem* p, int ns, const int* ptr, const int* cell,
                             const double* val);

/* Set the receivers Rx (Sec. 2.1, p_i) as sparse columns (host arrays). */
msfv_status msfv_set_receivers(msfv_problem* p, int nr, const int* ptr, const int* cell,
                               const double* val);

/* Forward problem (eq. fwdProbRed): rebuild S_k(m) and A_k(m), solve the
 * pinned coarse system for every source, write D = Rx^T S_k t (d_out, Nr*Ns)
 * and, if u_out != NULL, the fields u = S_k t (N*Ns).  m: device, N values. */
msfv_status msfv_forward(msfv_problem* p, const double* m, double* d_out, double* u_out);

/* Gradient g = J_k(m)^T v at the m of the last msfv_forward (Sec. 4.3,
 * transposed): v device Nr*Ns (same layout as D), g_out device N. */
msfv_status msfv_jtv(msfv_problem* p, const double* v, double* g_out);

/* msfv_forward(m, d_out, NULL) followed by msfv_jtv(v, g_out), for a v that
 * is known before the forward (it is not derived from this D): the adjoint
 * coarse problem A_k lambda_j = S_k^T Rx v_j (Sec. 4.3) needs only A_k, S_k
 * and v, so it is solved in the same coarse launch as the forward's A_k t_j
 * = S_k^T q_j (eq. fwdProbRed), 2 Ns columns at once.  Same arguments,
 * results (bit for bit) and errors as the two calls. */
msfv_status msfv_forward_jtv(msfv_problem* p, const double* m, const double* v, double* d_out,
                             double* g_out);

/* Forward-mode sensitivity J_k(m) dm at the m of the last msfv_forward
 * (Sec. 4.3 eq. sensred applied to dm, with the tangent of the adaptive basis
 * of Sec. 4.5): dD = Rx^T (dS_k t + S_k dt), A_k dt = dS_k^T q - dA_k t, where
 * dS_k is the basis tangent (the local problems differentiated along dm) and
 * dA_k the Galerkin operator's derivative.  dm: device N; dd_out: device
 * Nr*Ns (layout of D).  Entities of any size (faces and dual blocks wider
 * than one wavefront, coarsening above 8, run one workgroup an entity).
 * MSFV_ESTATE before a forward; MSFV_ENONFINITE (via msfv_sync) if dm holds
 * NaN or Inf. */
msfv_status msfv_jvp(msfv_problem* p, const double* dm, double* dd_out);

/* The same with the basis held fixed (eq. senssimple, the "fixed" basis of
 * Fig. 2): dD = -Rx^T S_k A_k^-1 S_k^T (dA/dm dm) u, and its transpose
 * g = -grad_m sum_j (S_k lambda_j)^T A(m) u_j with lambda = A_k^-1 S_k^T Rx v.
 * Same arguments and errors as msfv_jvp / msfv_jtv; both use device
 * workspace of 2 N Ns doubles (allocated on first use). */
msfv_status msfv_jvp_fixed(msfv_problem* p, const double* dm, double* dd_out);
msfv_status msfv_jtv_fixed(msfv_problem* p, const double* v, double* g_out);

/* Adaptive or frozen basis (Sec. 3.1, eq. optredadapt against the
 * fixed-basis surrogate of eq. optredfixed).
 *   MSFV_BASIS_ADAPTIVE (the default): every forward rebuilds S_k(m).
 *   MSFV_BASIS_FROZEN  : later forwards keep the S_k of the last forward
 *                        (the basis of the model m0 it ran at) and rebuild
 *                        only A_k(m) = S_k(m0)^T A(m) S_k(m0); msfv_jtv,
 *                        msfv_jvp and msfv_misfit_grad then return the exact
 *                        sensitivities of that surrogate, eq. senssimple with
 *                        the frozen basis (the same as msfv_jtv_fixed /
 *                        msfv_jvp_fixed).  Needs a forward first (MSFV_ESTATE
 *                        otherwise); allocates the fixed-basis workspace
 *                        (2 N Ns doubles) and synchronises the stream.
 * Switching back to MSFV_BASIS_ADAPTIVE makes the next forward rebuild S_k. */
enum { MSFV_BASIS_ADAPTIVE = 0, MSFV_BASIS_FROZEN = 1 };
msfv_status msfv_set_basis(msfv_problem* p, int mode);

/* Misfit phi = 1/2 ||D(m) - d_obs||_F^2 (Sec. 2.2) and its gradient
 * J_k^T (D - d_obs): forward + jtv.  phi_out: device, 1 value. */
msfv_status msfv_misfit_grad(msfv_problem* p, const double* m, const double* d_obs,
                             double* phi_out, double* g_out);

/* msfv_misfit_grad without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and errors as msfv_misfit_grad;
 * the data D and the residual D - d_obs live in a fixed library-owned device
 * array of 2^17 doubles (1 MiB per device, held until the process ends)
 * instead of the problem's buffers.
 *   - Nr * Ns above 65536 returns MSFV_EINVAL.
 *   - The problem's electrode tables and coarse vectors must already exist:
 *     after msfv_set_sources / msfv_set_receivers, run msfv_forward or
 *     msfv_misfit_grad once first; otherwise MSFV_ESTATE.
 *   - Stage profiling events are not recorded for this call.
 *   - Every call on one device shares that array: calls on one device whose
 *     executions overlap (different streams, or different problems on
 *     streams that are not ordered) race on it and must be serialised by
 *     the caller.  Every value read from the array is written earlier in the
 *     same call, so nothing carries over between calls. */
msfv_status msfv_misfit_grad_noalloc(msfv_problem* p, const double* m, const double* d_obs,
                                     double* phi_out, double* g_out);

/* Wait for the problem's stream; returns MSFV_ENONFINITE / MSFV_ENOCONV if
 * the last forward or jtv recorded that condition, else MSFV_OK. */
msfv_status msfv_sync(msfv_problem* p);

/* Introspection (host copies; synchronises).  Arrays sized by msfv_sizes:
 * row_ptr N+1, col nnz_p, val nnz_p (S_k); row_ptr Nc+1, col nnz_k,
 * val nnz_k (A_k before fixing vertex 0), t_out Nc*Ns (coarse
 * coefficients, column j contiguous).  Any pointer may be NULL. */
msfv_status msfv_get_sizes(msfv_problem* p, msfv_sizes* out);
msfv_status msfv_get_prolongation(msfv_problem* p, int* row_ptr, int* col, double* val);
msfv_status msfv_get_coarse(msfv_problem* p, int* row_ptr, int* col, double* val, double* t_out);
/* Iteration counts, cap hits and final relative residuals of the local
 * (Sec. 3.2, eq. multiscaleBasis_step3) and coarse (eq. reducedPDE) solves
 * (struct above); synchronises the problem's stream. */
msfv_status msfv_get_stats(msfv_problem* p, msfv_stats* out);

/* Stage profiling.  When enabled, every stage launched by msfv_forward,
 * msfv_jtv and msfv_misfit_grad is bracketed by HIP events on the problem's
 * stream; msfv_profile_read() synchronises, returns the summed event time
 * and launch count per stage since the previous read, plus work counters,
 * and resets them.  work[0..3]: local CG cell-iterations (sum over local
 * solves of iterations x own cells) of dual blocks forward / adjoint and of
 * faces (3-D) or 2-D blocks forward / adjoint; work[4..5]: coarse CG
 * row-iterations (iterations x coarse rows) forward / adjoint. */
enum {
  MSFV_STAGE_COPY_M = 0, MSFV_STAGE_CHECK, MSFV_STAGE_EDGE_FWD, MSFV_STAGE_FACE_FWD,
  MSFV_STAGE_BLOCK_FWD, MSFV_STAGE_KASSEMBLE, MSFV_STAGE_COARSE_RHS, MSFV_STAGE_COARSE_FWD,
  MSFV_STAGE_DATA, MSFV_STAGE_PROLONG, MSFV_STAGE_ADJ_RHS, MSFV_STAGE_COARSE_ADJ,
  MSFV_STAGE_SLOAD, MSFV_STAGE_BLOCK_ADJ, MSFV_STAGE_FACE_ADJ, MSFV_STAGE_EDGE_ADJ,
  MSFV_STAGE_GFINAL, MSFV_STAGE_RESIDUAL, MSFV_STAGE_COARSE_SETUP, MSFV_NSTAGE
};

typedef struct {
  double ms[MSFV_NSTAGE];
  int count[MSFV_NSTAGE];
  unsigned long long work[8];
} msfv_profile;

msfv_status msfv_profile_enable(msfv_problem* p, int enable);
msfv_status msfv_profile_read(msfv_problem* p, msfv_profile* out);
const char* msfv_stage_name(int stage);

/* ---- Many problems at once ------------------------------------------------
 * A batch runs forward (eq. fwdProbRed) followed by J_k^T v (Sec. 4.3) for
 * each of `count` problems of any shapes, sizes and source counts: the
 * independent instances of an inversion campaign, as in the paper's
 * parallel-over-workers setting (Sec. 5, Table 3), here concurrent on one
 * device.  Problems are issued largest first over a pool of HIP streams so
 * that small instances fill the compute units left idle by large ones; each
 * problem's per-call kernel sequence is captured once as a HIP graph per set
 * of buffer pointers and replayed.  The batch call is asynchronous: it is
 * ordered after prior work on hip_stream (the batch's stream) and later work
 * on that stream is ordered after it.  The problems stay owned by the caller
 * and must outlive the batch; while a batch call is in flight they must not
 * be used on their own.
 *
 * msfv_batch_create : problems[0..count) (not NULL, distinct); hip_stream
 *                     may be NULL (the null stream).  EINVAL on bad
 *                     arguments, EDEVICE if streams cannot be created.
 * msfv_batch_forward_jtv : m[i], v[i] device inputs of problem i (N_i and
 *                     Nr_i*Ns_i doubles), d_out[i] (Nr_i*Ns_i) and g_out[i]
 *                     (N_i) device outputs.  Sources and receivers must be
 *                     set on every problem (ESTATE otherwise).  Outputs are
 *                     valid after msfv_batch_sync.
 * msfv_batch_sync   : waits for the batch's work and reports the first
 *                     failing problem's status (ENOCONV, ENONFINITE).
 * msfv_batch_set_options / get_options : streams in [1, 16]; graphs 0/1;
 *                     shared in [0, 8].  With shared = P > 0 the local
 *                     solves (edges, faces, dual blocks, forward and
 *                     adjoint) run as shared launches: one launch per
 *                     stage and kernel class over (problem, entity) items, a
 *                     fixed grid of as many workgroups as fit the device
 *                     striding over them (dual blocks of different problems
 *                     fill the compute units together).  The problems are
 *                     dealt, largest first, over P pipelines; each pipeline
 *                     is issued by a host thread of its own, runs its shared
 *                     launches on one pool stream and the per-problem parts
 *                     (model copy, Galerkin assembly, coarse solves, data,
 *                     gradient gather) of its members on further pool
 *                     streams, so the local launches of one pipeline overlap
 *                     the coarse solves of another.  Problems with a frozen
 *                     basis use the per-problem path.  Graphs apply to the
 *                     per-problem path.  set_options waits for the batch's
 *                     work.
 * msfv_batch_autotune : times one call per candidate (shared launches in 1,
 *                     2, 4 or 8 pipelines, or the per-problem path with and
 *                     without graphs; streams 1, 2, 4, 8, 16 capped at
 *                     count) with the given buffers, keeps the fastest and
 *                     reports it. */
typedef struct msfv_batch msfv_batch;
msfv_status msfv_batch_create(int count, msfv_problem* const* problems, void* hip_stream,
                              msfv_batch** out);
void msfv_batch_destroy(msfv_batch* b);
msfv_status msfv_batch_forward_jtv(msfv_batch* b, const double* const* m, const double* const* v,
                                   double* const* d_out, double* const* g_out);
msfv_status msfv_batch_sync(msfv_batch* b);
msfv_status msfv_batch_set_options(msfv_batch* b, int streams, int graphs, int shared);
msfv_status msfv_batch_get_options(msfv_batch* b, int* streams, int* graphs, int* shared);
msfv_status msfv_batch_autotune(msfv_batch* b, const double* const* m, const double* const* v,
                                double* const* d_out, double* const* g_out, int* streams_out,
                                int* graphs_out, int* shared_out);

/* ---- Serving ----------------------------------------------------------------
 * A server runs forward (eq. fwdProbRed) + J_k^T v (Sec. 4.3) requests for
 * registered jobs -- the per-iteration evaluations of many concurrent
 * inversions (Sec. 2.2) -- as they arrive (continuous batching).  Each job
 * keeps its problem state (S_k, A_k, plan, workspace) resident on the device
 * and has a host worker thread of its own that prepares and issues its
 * requests on the job's stream, so one job's host work (a new source set's
 * electrode tables, the host-polled coarse solver of large grids) never
 * holds up another's.  Requests are admitted first come first served when
 *   - their job is idle (a job's requests share its problem state and run
 *     one at a time, in order),
 *   - fewer than max_inflight requests are running, and
 *   - the resident bytes of all jobs plus the admission bytes of the running
 *     requests and of this one stay within the memory budget;
 * no request is admitted past one that waits for memory.  Latency =
 * completion - submission (steady clock); each request also records device
 * times of its first and last kernel.
 *
 * Admission bytes.  A job's resident bytes are the device bytes its problem
 * holds once its source-count-dependent buffers are reserved for
 * max_sources sources (coarse vectors 3 Nc Ns, data buffers 2 Nr Ns, the
 * multi-launch coarse workspace).  A request's bytes are its device buffers:
 * m and g (N values each), v and d_out (Nr Ns values each), 16 (N + Nr Ns).
 *
 * msfv_server_create : max_inflight in [1, 64]; budget_bytes > 0 is the
 *                     memory budget, <= 0 the device's total memory.
 * msfv_server_add_job : registers a caller-owned problem (receivers set; give
 *                     every job its own stream for concurrency) for requests
 *                     of up to max_sources sources, reserving its buffers for
 *                     them.  ENOMEM if the resident bytes of the jobs would
 *                     exceed the budget (the job is not added).  The server
 *                     uses the problem exclusively until destroyed.
 * msfv_server_request_bytes : a job's resident bytes and the admission bytes
 *                     of a request of ns sources.
 * msfv_server_submit : copies the request's sources (host CSR columns, as
 *                     msfv_set_sources) and queues it; m (N), v (Nr*ns) are
 *                     device inputs and d_out (Nr*ns), g_out (N) device
 *                     outputs that must stay valid until the request is done.
 *                     The request is ordered after the work queued so far on
 *                     caller_stream (a hipStream_t; NULL = the null stream),
 *                     which may be producing m and v.  Returns its id in
 *                     *req.  EINVAL on bad arguments or ns outside
 *                     [1, max_sources]; ENOMEM if the request alone (with the
 *                     jobs' resident bytes) exceeds the budget: it could
 *                     never be admitted and is rejected.
 * msfv_server_wait   : blocks until request req is done; returns its status
 *                     and, for non-NULL pointers, its latency and the device
 *                     times (ms since the server's creation) at which its
 *                     job's stream reached its first kernel and finished its
 *                     last.  Several threads may wait for one request.
 * msfv_server_drain  : blocks until every submitted request is done, then
 *                     forgets completed requests that nobody waits for.
 * msfv_server_stats  : latency percentiles and throughput of the requests
 *                     completed since the last reset, rejections, the budget,
 *                     the jobs' resident bytes and the peak of resident plus
 *                     running-request bytes (reset clears them).
 * msfv_server_destroy: drains, stops the job workers, releases the server. */
typedef struct msfv_server msfv_server;
typedef struct {
  long long completed;   /* requests completed since the last reset        */
  long long failed;      /* of which ended with an error status            */
  double p50_ms, p90_ms, p99_ms, mean_ms, max_ms;  /* latency              */
  double span_s;         /* first submission to last completion            */
  double throughput;     /* completed / span_s (requests per second)       */
  long long rejected;    /* submissions refused for the memory budget      */
  double budget_bytes;   /* the memory budget                              */
  double resident_bytes; /* resident bytes of the registered jobs          */
  double peak_committed_bytes; /* peak of resident + running-request bytes */
} msfv_serve_stats;
msfv_status msfv_server_create(int max_inflight, double budget_bytes, msfv_server** out);
void msfv_server_destroy(msfv_server* s);
msfv_status msfv_server_add_job(msfv_server* s, msfv_problem* p, int max_sources, int* job);
msfv_status msfv_server_request_bytes(msfv_server* s, int job, int ns, long long* resident,
                                      long long* request);
msfv_status msfv_server_submit(msfv_server* s, int job, int ns, const int* ptr, const int* cell,
                               const double* val, const double* m, const double* v, double* d_out,
                               double* g_out, void* caller_stream, long long* req);
msfv_status msfv_server_wait(msfv_server* s, long long req, double* latency_ms, double* dev_start_ms,
                             double* dev_end_ms);
msfv_status msfv_server_drain(msfv_server* s);
msfv_status msfv_server_stats(msfv_server* s, msfv_serve_stats* out, int reset);

const char* msfv_status_string(msfv_status s);
const char* msfv_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MSFV_H */
