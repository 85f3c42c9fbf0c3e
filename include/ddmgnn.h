/*
 * ddmgnn.h - C ABI of the DDM-GNN preconditioned flexible-CG solver for
 * MI355X (gfx950).
 *
 * The operation is the paper's hybrid solver (arXiv 2402.08296): a Krylov
 * method (Algorithm 1; here flexible CG by default) whose preconditioner is the
 * DDM-GNN apply of Sec. III.A:
 *   1. coarse problem  r_c = R_0^T (R_0 A R_0^T)^{-1} R_0 r           (step 1)
 *   2. local problems  r~_i = DSS_theta(G_i), G_i = (Omega_{h,i}, R_i r/|R_i r|)
 *                      with the DSS_theta model of Sec. III.B         (step 2)
 *   3. gluing          z = r_c + sum_i R_i^T w_i |R_i r| r~_i          (step 3)
 * where w_i = 1 is the paper's glue and w_i = D_i (partition of unity) the
 * weighted variant.
 *
 * Conventions for every entry point:
 *   - Returns DDMGNN_OK (0) or a negative status; nothing aborts. The text of
 *     the last error of the calling thread is returned by ddmgnn_last_error().
 *   - Pointers documented as "host" are read during the call only; the library
 *     copies what it keeps. Pointers documented as "device" are HIP device
 *     memory owned by the caller, on the device current at ctx creation.
 *   - All device work is enqueued on the context's stream. Calls that return
 *     results (solve, apply, forward, spmv) synchronise that stream before
 *     returning.
 *   - Handles are owned by the library until the matching *_destroy call.
 *     One context per host thread. Destroy a context's problems, models and
 *     server before the context.
 */
#ifndef DDMGNN_H
#define DDMGNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    DDMGNN_OK = 0,
    DDMGNN_E_INVALID = -1,    /* malformed input or unsupported option */
    DDMGNN_E_NOMEM = -2,      /* device or host allocation failed */
    DDMGNN_E_HIP = -3,        /* HIP runtime error */
    DDMGNN_E_NOT_SPD = -4,    /* coarse matrix R_0 A R_0^T not positive definite */
    DDMGNN_E_BREAKDOWN = -5,  /* <p, A p> <= 0 in the Krylov recurrence */
    DDMGNN_E_MAXIT = -6,      /* not converged within max_it; u holds the last iterate */
    DDMGNN_E_NONFINITE = -7,  /* NaN/Inf in the residual; u holds the last finite iterate */
    DDMGNN_E_BUDGET = -8,     /* request exceeds the memory budget */
    DDMGNN_E_PENDING = -9     /* result not ready yet */
};

/* Krylov method (Algorithm 1 is PCG; FCG is its flexible variant; FGMRES is
 * restarted flexible GMRES with right preconditioning, cycles of `restart` steps). */
enum { DDMGNN_FCG = 0, DDMGNN_PCG = 1, DDMGNN_CG = 2, DDMGNN_FGMRES = 3 };
/* Arithmetic of the DSS_theta forward pass. Krylov vectors, dot products,
 * the residual update and the coarse level are always FP64. */
enum { DDMGNN_FP64 = 0, DDMGNN_FP32 = 1, DDMGNN_BF16 = 2 };
/* Weights of the gluing step 3: partition of unity D_i, or 1 (paper). */
enum { DDMGNN_PROLONG_POU = 0, DDMGNN_PROLONG_UNWEIGHTED = 1 };
/* Local solver of step 2: the DSS_theta model, or the exact solve of
 * R_i A R_i^T (the paper's DDM-LU comparator, eq. (7)). */
enum { DDMGNN_LOCAL_GNN = 0, DDMGNN_LOCAL_LU = 1 };

typedef struct ddmgnn_ctx ddmgnn_ctx;
typedef struct ddmgnn_model ddmgnn_model;
typedef struct ddmgnn_problem ddmgnn_problem;
typedef struct ddmgnn_server ddmgnn_server;

/* Text of the last error on this thread (empty when none). */
const char* ddmgnn_last_error(void);
const char* ddmgnn_version(void);

/* Context bound to the current HIP device and to `hip_stream` (a hipStream_t,
 * NULL = the null stream). The stream must outlive the context. */
int ddmgnn_ctx_create(void* hip_stream, ddmgnn_ctx** out);
int ddmgnn_ctx_destroy(ddmgnn_ctx* ctx);

/* DSS_theta hyper-parameters (Sec. IV.B: kbar = 30, d = 10, hidden width d,
 * alpha = 1e-3; Table II sweeps kbar and d). kbar >= 1 is a run-time value;
 * d is 5, 10 or 20 (E_INVALID otherwise). The BF16 matrix-core kernel runs
 * d = 10 only: a BF16 solve with another width runs the FP32 VALU kernel
 * (ddmgnn_stats.dss_kernel says which ran). */
typedef struct {
    int32_t kbar;
    int32_t d;
    double alpha;
} ddmgnn_model_desc;

/* Create a model from `theta` (host, float32, n_theta values). n_theta must be
 * kbar * (11 d^2 + 15 d + 1) (the parameter counts of Table II). Layout, block
 * k = 1..kbar in order, matrices row-major [out][in]:
 *   Phi_out {W1[d][2d+3], b1[d], W2[d][d], b2[d]}   inputs (h_j, h_l, d_jl, |d_jl|)
 *   Phi_in  {W1[d][2d+3], b1[d], W2[d][d], b2[d]}   inputs (h_j, h_l, d_lj, |d_lj|)
 *   Psi     {W1[d][3d+1], b1[d], W2[d][d], b2[d]}   inputs (h_j, c_j, phi_out_j, phi_in_j)
 *   Dec     {W1[d][d],    b1[d], W2[1][d], b2[1]}   input  h_j
 * (eqs. (14)-(18)). Copied at call time (to the host and to the device). Problems
 * keep a reference to the device copy, so the model may be destroyed before them. */
int ddmgnn_model_create(ddmgnn_ctx* ctx, const ddmgnn_model_desc* desc, const float* theta,
                        int64_t n_theta, ddmgnn_model** out);
int ddmgnn_model_destroy(ddmgnn_model* model);

/* Seeded Xavier-uniform weights in the layout above (Sec. IV.B initialisation),
 * host only: matrix entries in layout order take consecutive outputs x of one
 * splitmix64 stream from state `seed`; u = (x >> 11) 2^-53 and the entry is
 * a (2u - 1) in double with a = sqrt(6 / (fan_in + fan_out)), rounded to float.
 * Biases are 0. theta_out holds n_theta = kbar (11 d^2 + 15 d + 1) floats
 * (E_INVALID otherwise). */
int ddmgnn_model_init_xavier(const ddmgnn_model_desc* desc, uint64_t seed, float* theta_out, int64_t n_theta);

/* Where the arrays of a problem descriptor live. */
enum { DDMGNN_MEM_HOST = 0, DDMGNN_MEM_DEVICE = 1 };

/* One Poisson-Dirichlet problem A u = b (eqs. (1)-(2)) with its overlapping
 * decomposition (Sec. II.A). All pointers are host pointers, or all are device
 * pointers with mem_kind = DDMGNN_MEM_DEVICE (every entry point that takes a
 * descriptor then copies the arrays to the host once, synchronously, for
 * validation and setup).
 *   xy[2N]            node coordinates (x0, y0, x1, y1, ...)
 *   tri[3T]           triangles (node ids), used for the DSS graphs (Sec. III.B)
 *   dirichlet[N]      1 at Dirichlet nodes, else 0. Dirichlet rows of A must be
 *                     identity rows, decoupled from the free rows.
 *   a_rowptr[N+1], a_col[nnz], a_val[nnz]
 *                     A in CSR, symmetric, columns strictly ascending per row.
 *   b[N], u0[N]       right-hand side and initial guess.
 *   sub_ptr[K+1], sub_nodes[sub_ptr[K]]
 *                     sub-mesh i holds nodes sub_nodes[sub_ptr[i] .. sub_ptr[i+1]),
 *                     strictly ascending; the local index of a node is its rank.
 *                     Every node belongs to at least one sub-mesh.
 *   weights[sub_ptr[K]]
 *                     partition-of-unity weights D_i aligned with sub_nodes:
 *                     >= 0, summing to 1 over the sub-meshes of each free node
 *                     and 0 at Dirichlet nodes. They define the Nicolaides
 *                     coarse basis (column i of R_0^T is R_i^T D_i R_i 1).
 * Setup builds the local DSS graphs on the host (edges l -> j for mesh edges
 * inside the sub-mesh, none received by Dirichlet nodes), uploads them, and
 * forms R_0 A R_0^T and its inverse on the device (blocked Gauss-Jordan;
 * E_NOT_SPD when a pivot is not above 1e-12 of its diagonal entry). */
typedef struct {
    int64_t n_nodes;
    const double* xy;
    int64_t n_tri;
    const int32_t* tri;
    const uint8_t* dirichlet;
    const int32_t* a_rowptr;
    const int32_t* a_col;
    const double* a_val;
    const double* b;
    const double* u0;
    int32_t n_sub;
    const int64_t* sub_ptr;
    const int32_t* sub_nodes;
    const double* weights;
    int32_t mem_kind;    /* DDMGNN_MEM_HOST (0) or DDMGNN_MEM_DEVICE */
} ddmgnn_problem_desc;

/* Validate a descriptor on the host (no device needed). */
int ddmgnn_validate_problem(const ddmgnn_problem_desc* desc);

/* Largest sub-mesh accepted (nodes): 16384 (16-bit local ids; DDM-LU stages
 * R_i r in LDS). Sub-meshes of up to 2048 nodes keep their DSS state in
 * registers and LDS; larger ones run a form of the VALU DSS kernel that keeps
 * h, c and the neighbour projections in device memory (same arithmetic), in
 * every precision (BF16 requests run them in FP32). Training samples are
 * limited to 2048 nodes. */
int32_t ddmgnn_max_subdomain_nodes(void);

int ddmgnn_problem_create(ddmgnn_ctx* ctx, const ddmgnn_problem_desc* desc, const ddmgnn_model* model,
                          ddmgnn_problem** out);
int ddmgnn_problem_destroy(ddmgnn_problem* prob);

typedef struct {
    int32_t krylov;      /* DDMGNN_FCG / PCG / CG */
    int32_t m_max;       /* FCG truncation: directions kept for A-orthogonalisation (1) */
    double rtol;         /* stop when |r_i| <= rtol |r_0| (1e-6, Sec. IV.C) */
    int32_t max_it;
    int32_t precision;   /* DDMGNN_FP64 / FP32 / BF16 for the DSS forward */
    int32_t prolong;     /* DDMGNN_PROLONG_POU / UNWEIGHTED */
    int32_t coarse;      /* 1: add the coarse correction (step 1), 0: one-level */
    int32_t check_every; /* iterations between host checks of the converged flag */
    int32_t profile;     /* 1: time every stage with HIP events on the context stream */
    int32_t graph;       /* 1: replay chunks of check_every iterations as one captured HIP graph
                          * (ignored when profile = 1) */
    int32_t local_solver;/* DDMGNN_LOCAL_GNN, or DDMGNN_LOCAL_LU: exact local solves with the
                          * inverses of R_i A R_i^T (dense FP64, sum k_i^2 doubles of device
                          * memory), assembled and inverted on the device at the problem's
                          * first LU use (E_NOT_SPD when a pivot is not positive) */
    int32_t restart;     /* FGMRES: steps per cycle, 1..64 (30); the problem keeps
                          * (2 restart + 1) N doubles of device memory for it */
} ddmgnn_solve_opts;

typedef struct {
    int32_t iterations;
    int32_t converged;
    double rel_residual;       /* |r_it| / |r_0| of the recurrence */
    double true_rel_residual;  /* |b - A u| / |r_0| recomputed at exit */
    double solve_ms;           /* device time of the whole solve (HIP events) */
    /* Filled when opts.profile = 1 (HIP event pairs around each launch of the
     * iterations that did work): */
    int32_t dss_launches;      /* DSS forward launches timed */
    double dss_ms;             /* total time of the DSS forward kernel (steps 2 with restriction) */
    double coarse_ms;          /* coarse solve (step 1) */
    double prolong_ms;         /* gluing (step 3) with its fused dot products */
    double krylov_ms;          /* direction update, SpMV with dots, solution update */
    int32_t dss_kernel;        /* kernel that ran the local solves: 0 FP64 VALU DSS, 1 FP32 VALU DSS,
                                * 2 BF16 MFMA DSS for every sub-mesh, 3 exact local solves (DDM-LU),
                                * 4 BF16 MFMA DSS for some sub-meshes and the FP32 VALU DSS for those
                                * beyond its LDS or 2048-node budget (a BF16 request of a model with
                                * d = 20 runs 1 throughout; d = 5 runs on matrix cores) */
    int32_t status;            /* this problem's own status (DDMGNN_OK, E_MAXIT, E_BREAKDOWN, ...) */
    double latency_ms;         /* served requests: completion - submission (host clock);
                                * solves: equal to solve_ms */
    /* Served requests only (0 for solves), host clock: */
    double setup_ms;           /* host setup (validation, local graphs, the device-ready arrays) on a
                                * setup thread */
    double queue_ms;           /* waiting: for a setup thread, then for admission */
    double upload_ms;          /* admission: device buffers allocated and filled by the GPU thread */
} ddmgnn_stats;

/* Fill opts with defaults (FCG, m_max 1, rtol 1e-6, max_it 10000, FP32, POU, coarse on,
 * check_every 16, graph replay on, DSS local solver, FGMRES restart 30). */
void ddmgnn_default_opts(ddmgnn_solve_opts* opts);

/* Solve A u = b from the problem's u0. u_out: device, N doubles. On
 * E_MAXIT / E_NONFINITE / E_BREAKDOWN u_out holds the last finite iterate. */
int ddmgnn_solve(ddmgnn_ctx* ctx, ddmgnn_problem* prob, const ddmgnn_solve_opts* opts, double* u_out,
                 ddmgnn_stats* stats);

/* Solve n independent problems together (all created on ctx with the same
 * model): every kernel of an iteration is one launch over all of them, the
 * DSS forward over all their sub-meshes by decreasing size, and each problem
 * stops under its own converged flag (its workgroups return at once while
 * the others continue). u_out[i]: device, N_i doubles; stats (may be NULL):
 * n entries, each with the problem's own status. A problem's iterates do not
 * depend on the other members (per-problem reductions in a fixed order), so
 * they are bitwise those of ddmgnn_solve on it alone. Returns DDMGNN_OK when
 * every problem converged, else the status of the first that did not. */
int ddmgnn_solve_batch(ddmgnn_ctx* ctx, ddmgnn_problem* const* probs, int32_t n, const ddmgnn_solve_opts* opts,
                       double* const* u_out, ddmgnn_stats* stats);

/* ---- serving: a stream of independent requests with continuous batching ----
 * The server owns ctx (its stream and device) until ddmgnn_server_destroy:
 * the caller makes no other call on ctx meanwhile. Requests are copied at
 * submission; `setup_threads` host threads (0: 4) run their host setup
 * (validation, local graphs, every array the device needs); one GPU thread
 * admits set-up requests in submission order while their device memory
 * (ddmgnn_problem_device_bytes) fits `hbm_budget` bytes and at most
 * `max_active` are active, advances all active requests together by chunks
 * of opts.check_every iterations (as ddmgnn_solve_batch), creates newly
 * admitted problems on a stream of its own while a chunk runs, and retires
 * each request as it converges. Requests batch together only when their Krylov method,
 * m_max, precision, prolong and coarse options agree; one that differs from
 * the active set waits until that set has drained (rtol and max_it are per
 * request). A request larger than the budget fails with E_BUDGET. */
int ddmgnn_server_create(ddmgnn_ctx* ctx, const ddmgnn_model* model, int64_t hbm_budget, int32_t max_active,
                         int32_t setup_threads, ddmgnn_server** out);
/* Non-blocking. *ticket identifies the request (> 0). */
int ddmgnn_server_submit(ddmgnn_server* srv, const ddmgnn_problem_desc* desc, const ddmgnn_solve_opts* opts,
                         uint64_t* ticket);
/* DDMGNN_E_PENDING while the request runs; otherwise its status, with u_out
 * (host, N doubles, may be NULL) and stats filled (stats.latency_ms =
 * completion - submission). A finished request is collected once. */
int ddmgnn_server_poll(ddmgnn_server* srv, uint64_t ticket, double* u_out, ddmgnn_stats* stats);
/* Blocks until every submitted request has finished. */
int ddmgnn_server_drain(ddmgnn_server* srv);
/* Drains, stops the threads and frees uncollected results. */
int ddmgnn_server_destroy(ddmgnn_server* srv);

/* Host-only model of the serving loop (no device): the same admission rule as
 * the GPU thread, driven by simulated requests. Requests (in submission order)
 * go through `setup_threads` setup workers (0: 4) in order, taking setup_s each
 * from max(arrival, a free worker); set-up requests are admitted as by the
 * server (ticket order, hbm_budget, max_active, equal group keys batch, no
 * overtaking); every chunk_s seconds each active request completes one of its
 * `chunks` chunks and leaves after the last. out[i] gets the admission and
 * finish times (s) and the status (OK; E_BUDGET if larger than the budget;
 * E_INVALID if setup_ok is 0; such requests are rejected as soon as their
 * setup ends, even behind a waiting request, and finish at that time). */
typedef struct {
    double arrival;
    double setup_s;
    int64_t bytes;
    uint64_t group;
    int32_t chunks;
    int32_t setup_ok;
} ddmgnn_sim_request;
typedef struct {
    double admitted;
    double finished;
    int32_t status;
} ddmgnn_sim_result;
int ddmgnn_server_simulate(const ddmgnn_sim_request* reqs, int32_t n, int64_t hbm_budget, int32_t max_active,
                           int32_t setup_threads, double chunk_s, ddmgnn_sim_result* out);


/* One preconditioner apply z = M(r) (Sec. III.A steps 1-3). r, z: device, N
 * doubles, must not alias. */
int ddmgnn_precond_apply(ddmgnn_ctx* ctx, ddmgnn_problem* prob, const ddmgnn_solve_opts* opts,
                         const double* r, double* z);

/* Times the stages of one preconditioner apply z = M(r) as the solve runs them:
 * each stage (local solves, coarse solve, gluing), repeated `reps` times, is
 * captured as one HIP graph, launched once to warm up and once between events
 * recorded on the context's stream; outputs are milliseconds per stage (the
 * launch cost shared by the reps; NULL allowed). r, z: device, N doubles, must
 * not alias. */
int ddmgnn_time_apply_stages(ddmgnn_ctx* ctx, ddmgnn_problem* prob, const ddmgnn_solve_opts* opts,
                             const double* r, double* z, int32_t reps, double* local_ms, double* coarse_ms,
                             double* glue_ms);

/* Intermediates of the last ddmgnn_precond_apply on this problem, copied to
 * device buffers the caller owns (any pointer may be NULL):
 *   s[K]        |R_i r|
 *   y0[K]       R_0 r
 *   y[K]        (R_0 A R_0^T)^{-1} R_0 r
 *   local[sk]   |R_i r| r~_i per sub-mesh node, in sub_nodes order (sk = sub_ptr[K]). */
int ddmgnn_apply_intermediates(ddmgnn_ctx* ctx, ddmgnn_problem* prob, double* s, double* y0, double* y,
                               double* local);

/* DSS_theta forward pass (Sec. III.B) on every sub-mesh of the problem. c and
 * out: device, sub_ptr[K] doubles in sub_nodes order; c holds each sub-mesh's
 * input c_i, out receives r~_i = D^kbar(H^kbar). */
int ddmgnn_dss_forward(ddmgnn_ctx* ctx, ddmgnn_problem* prob, int32_t precision, const double* c,
                       double* out);
/* The same forward pass on sub-mesh `sub` alone: c and out are device arrays of
 * k_sub = sub_ptr[sub+1] - sub_ptr[sub] doubles (the sub-mesh's nodes in
 * sub_nodes order). Gives the bits of the matching slice of ddmgnn_dss_forward. */
int ddmgnn_dss_forward_sub(ddmgnn_ctx* ctx, ddmgnn_problem* prob, int32_t precision, int32_t sub,
                           const double* c, double* out);

/* ---- training of DSS_theta (Sec. III.B loss, Sec. IV.B set-up) ----
 * A sample is a local problem of the two-level preconditioner: sub-mesh i of
 * the problem, its local matrix A_i = R_i A R_i^T and a right-hand side c
 * (Sec. IV.A: local problems met during the iterations of a PCG solve).
 *
 * ddmgnn_train_rhs: the right-hand sides of every sub-mesh at the iterate u:
 * r = b - A u, c_i = R_i r / |R_i r| (0 where R_i r = 0). u: device, N
 * doubles; c_out: device, sub_ptr[K] floats in sub_nodes order. */
int ddmgnn_train_rhs(ddmgnn_ctx* ctx, ddmgnn_problem* prob, const double* u, float* c_out);
/* Loss and gradient over n samples, in FP32 on the device:
 *   loss = scale * sum_s sum_{k=1..kbar} sum_j ((A_i D^k(H^k))_j - c_j)^2,
 * the residual loss of Sec. II.B of every block's decoded state (Sec. III.B),
 * summed; scale = 1 / (total nodes) gives the mean over the batch as one graph.
 * model: kbar (1..64), d (10 only), alpha. theta: device, kbar(11d^2+15d+1)
 * floats in the layout of ddmgnn_model_create. subs, c_off: host, n entries:
 * sample s is sub-mesh subs[s] with right-hand side c + c_off[s] (device, k_i
 * floats). grad: device, same size as theta, receives d loss / d theta. The
 * gradient is deterministic (fixed-order sums; no atomics). *loss_out and
 * *gnorm_out (host, may be NULL) receive the loss (FP64 sum of the FP32
 * residuals) and |grad|_2. The first call builds the local matrices and edge
 * transposes on the device. Samples run in launches of 512 that share one
 * scratch region of about 4 (kbar + 33) d k_i bytes per sample of a launch, plus
 * 4 kbar(11d^2+15d+1) bytes per sample for the per-sample gradients. The
 * problem's training buffers serve one call at a time: calls on one problem from
 * several threads must be serialised. E_NONFINITE when the loss or the gradient
 * overflows. */
int ddmgnn_train_grad(ddmgnn_ctx* ctx, ddmgnn_problem* prob, const ddmgnn_model_desc* model, const float* theta,
                      const int32_t* subs, int32_t n, const float* c, const int64_t* c_off, double scale,
                      float* grad, double* loss_out, double* gnorm_out);
/* One Adam step (Sec. IV.B's optimiser, with bias correction) on device FP32
 * arrays of n entries: the gradient is first scaled to L2 norm `clip` when
 * gnorm (its norm, as returned by ddmgnn_train_grad) exceeds it (clip <= 0: no
 * clipping); then m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2 and
 * theta -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps). t >= 1 is the step. */
int ddmgnn_adam_step(ddmgnn_ctx* ctx, float* theta, const float* grad, float* m, float* v, int64_t n, double gnorm,
                     int32_t t, double lr, double beta1, double beta2, double eps, double clip);

/* y = A x with the problem's matrix (the q = A p step of Algorithm 1). x, y:
 * device, N doubles. */
int ddmgnn_spmv(ddmgnn_ctx* ctx, ddmgnn_problem* prob, const double* x, double* y);

/* Deterministic FP64 dot product of two device vectors of length n (the
 * reductions of Algorithm 1); result written to *out (host). */
int ddmgnn_dot(ddmgnn_ctx* ctx, int64_t n, const double* x, const double* y, double* out);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): ddmgnn_dot without any
 * allocation. It runs the same two kernels (so the result equals ddmgnn_dot's
 * bit for bit) with their per-workgroup partial sums in a static device array of
 * 1024 doubles (8 KiB per device, held until the process ends; its address is
 * looked up when the device's first context is created). x, y: device, n
 * doubles; out: DEVICE pointer to one double, written asynchronously on the
 * context's stream (no synchronisation, so the call can be captured). n = 0
 * writes 0. n above DDMGNN_NOALLOC_DOT_MAX_N: E_INVALID. Calls no hipMalloc,
 * hipFree or allocating routine. Every call on one device shares that array:
 * calls that overlap on one GPU (several streams or threads) race, and must be
 * serialised by the caller. */
#define DDMGNN_NOALLOC_DOT_MAX_N 2147483647LL
int ddmgnn_dot_noalloc(ddmgnn_ctx* ctx, int64_t n, const double* x, const double* y, double* out);

/* ---- host-only helpers (no device needed) ---- */

/* Overlapping sub-meshes: part i grown by `delta` layers of mesh adjacency
 * (Sec. II.A, overlap of Sec. IV.A). part[N] in [0, n_part). On success
 * *sub_ptr_out (n_part+1 int64) and *sub_nodes_out (int32, ascending per
 * sub-mesh) are allocated by the library; free them with ddmgnn_free. */
int ddmgnn_expand_overlap(int64_t n_nodes, int64_t n_tri, const int32_t* tri, const int32_t* part,
                          int32_t n_part, int32_t delta, int64_t** sub_ptr_out, int32_t** sub_nodes_out);

/* Partition-of-unity weights D_i = 1/multiplicity at free nodes, 0 at Dirichlet
 * nodes, aligned with sub_nodes (weights_out: caller-allocated, sub_ptr[K]). */
int ddmgnn_pou_weights(int64_t n_nodes, const uint8_t* dirichlet, int32_t n_sub, const int64_t* sub_ptr,
                       const int32_t* sub_nodes, double* weights_out);

void ddmgnn_free(void* p);

/* The overlapping decomposition on the device (Sec. II.A, overlap of Sec. IV.A):
 * the sub-meshes of ddmgnn_expand_overlap and the weights of ddmgnn_pou_weights,
 * equal to theirs, computed on the GPU of the context. tri (3 n_tri int32),
 * part (n_nodes int32 in [0, n_part)) and dirichlet (n_nodes uint8): device.
 * sub_ptr_out: host, n_part + 1 int64, always filled when the ids are valid.
 * sub_nodes_out (int32) and weights_out (double): device, room for cap
 * entries; when sub_ptr_out[n_part] > cap the call returns E_INVALID after
 * filling sub_ptr_out (cap = 0 asks for the size only). E_INVALID also for ids
 * out of range, a node in more than 16 sub-meshes or a sub-mesh above 16384
 * nodes. Synchronous on the context's stream; allocates device scratch. */
int ddmgnn_expand_overlap_device(ddmgnn_ctx* ctx, int64_t n_nodes, int64_t n_tri, const int32_t* tri,
                                 const int32_t* part, const uint8_t* dirichlet, int32_t n_part, int32_t delta,
                                 int64_t* sub_ptr_out, int32_t* sub_nodes_out, double* weights_out, int64_t cap);

/* Launch schedule of a problem: the choices of ddmgnn_autotune. small_lds never
 * changes a result; vec_blocks changes the order of the Krylov reductions (the
 * rounding, not the accuracy). */
typedef struct {
    int32_t small_lds;   /* BF16 MFMA DSS: sub-meshes of at most 1024 nodes whose LDS need is at
                          * most this many bytes run in 512-thread workgroups, two per compute
                          * unit; the others in 1024-thread workgroups, one per unit. 0: none;
                          * at most 80 KiB - 1 KiB */
    int32_t vec_blocks;  /* workgroups of the problem in the vector kernels (SpMV, gluing, Krylov
                          * updates): 0 = one per 256 rows up to 1024; else a multiple of 8 in
                          * [8, 1024], capped at the automatic count */
} ddmgnn_tuning;

/* Set / read a problem's schedule (E_INVALID for values out of range). Batches
 * built before a change are rebuilt on their next solve. */
int ddmgnn_problem_set_tuning(ddmgnn_problem* prob, const ddmgnn_tuning* t);
int ddmgnn_problem_get_tuning(const ddmgnn_problem* prob, ddmgnn_tuning* t);

/* Autotuner: times capped solves of `iterations` iterations with the options
 * `opts` (graph replay on) for each candidate schedule (small_lds in {0, 48, 64,
 * 79 KiB} when the MFMA kernel runs, then vec_blocks in {256, 512, 1024}
 * capped at the automatic count), keeps the fastest per iteration in the
 * problem and returns it with its time per iteration (ms). Leaves u and the
 * Krylov state of the problem undefined. */
int ddmgnn_autotune(ddmgnn_ctx* ctx, ddmgnn_problem* prob, const ddmgnn_solve_opts* opts, int32_t iterations,
                    ddmgnn_tuning* best, double* ms_per_iteration);

/* Sizes of a problem: N, nnz, K, sum k_i, number of directed DSS edges. */
int ddmgnn_problem_sizes(const ddmgnn_problem* prob, int64_t* n, int64_t* nnz, int32_t* k,
                         int64_t* sum_k, int64_t* n_edges);

/* Device memory a problem holds (the budget unit of the server), including the
 * local inverses of DDMGNN_LOCAL_LU once they are built. */
int ddmgnn_problem_device_bytes(const ddmgnn_problem* prob, int64_t* bytes);

/* Local DSS graph of sub-mesh `sub` as setup builds it from a descriptor
 * (Sec. III.B: edge l -> j for every mesh edge {j, l} inside the sub-mesh
 * whose receiver j is not a Dirichlet node). Outputs (host, caller-owned):
 * in-edge row pointers rowptr[k_sub+1] and sender local ids col[n_edges_sub],
 * receiver-major with senders ascending. Pass NULL rowptr/col to query
 * *n_edges_sub only. The descriptor is validated first. */
int ddmgnn_setup_local_graph(const ddmgnn_problem_desc* desc, int32_t sub, int32_t* rowptr, int32_t* col,
                             int64_t* n_edges_sub);

/* Inverse of the local matrix R_i A R_i^T of sub-mesh `sub` (the exact local
 * solver of DDM-LU, eq. (7)), formed on the host by Cholesky: dense, row-major
 * k_sub x k_sub, into a caller-owned host buffer (a host reference for the
 * device factorisation). E_NOT_SPD when the Cholesky factorisation fails. */
int ddmgnn_setup_local_inverse(const ddmgnn_problem_desc* desc, int32_t sub, double* inv);

/* Coarse operator A_0 = R_0 A R_0^T (eq. (7), Nicolaides basis from the
 * weights) and its inverse formed on the host (Cholesky), row-major K x K into
 * caller-owned host buffers (either may be NULL): a host reference for the
 * device setup. E_NOT_SPD when the Cholesky factorisation fails. */
int ddmgnn_setup_coarse(const ddmgnn_problem_desc* desc, double* a0, double* a0inv);

#ifdef __cplusplus
}
#endif
#endif /* DDMGNN_H */
