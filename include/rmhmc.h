/*
 * rmhmc.h -- C ABI of librmhmc.so: softabs Riemannian-manifold HMC for
 * latent Gaussian-process models on one AMD Instinct MI355X (gfx950).
 *
 * Method: Hayakawa & Asai, "Fast Riemannian-manifold Hamiltonian Monte
 * Carlo for hierarchical Gaussian-process models" (arXiv 2511.06407).
 * Each entry point names the passage of the paper that defines what it
 * computes.
 *
 * Conventions shared by every call
 *   - Parameter vector q = (f_1..f_N, eta_1..eta_P), D = N + P: latent GP
 *     values first, then log-hyperparameters in kernel-term order.
 *   - Matrices are column-major FP64 with a leading dimension >= rows.
 *   - Pointers marked [device] must be device memory on the current HIP
 *     device (e.g. torch.Tensor.data_ptr() of a CUDA tensor); [host] marks
 *     host memory.  The caller owns every array it passes; the library owns
 *     rmhmc_model and rmhmc_state and everything they hold.
 *   - Calls are asynchronous on the given stream unless they return a value
 *     through a [host] pointer or say otherwise; those synchronise the
 *     stream before returning.
 *   - Errors: every call returns an rmhmc_status; nothing throws across the
 *     ABI.  Argument errors are found on the host before any launch.  After
 *     a non-OK status, rmhmc_last_error() gives a message (thread-local) and
 *     the contents of output arrays are undefined.
 */
#ifndef RMHMC_H
#define RMHMC_H

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RMHMC_OK = 0,
  RMHMC_E_ARG = -1,        /* invalid argument (detected on the host)        */
  RMHMC_E_NOT_PD = -2,     /* kernel matrix K not positive definite          */
  RMHMC_E_EIG_NOCONV = -3, /* Jacobi sweeps exhausted before tolerance       */
  RMHMC_E_NONFINITE = -4,  /* NaN/Inf in an input or a computed quantity     */
  RMHMC_E_NOMEM = -5,      /* device allocation failed (create calls only)  */
  RMHMC_E_HIP = -6         /* a HIP runtime call failed                      */
} rmhmc_status;

typedef enum { RMHMC_FP64 = 0, RMHMC_MIXED = 1 } rmhmc_precision;

/* The soft-absolute map of the metric, G = sum g(lam) psi psi' (Sec. 2.2):
 *   RMHMC_SOFTABS_COTH  g = lam coth(alpha lam), the form the paper names
 *                       after earlier software (Sec. 2.5);
 *   RMHMC_SOFTABS_SQRT  g = sqrt(kappa^2 + lam^2), kappa = 1 / alpha, the form
 *                       the paper's own runs use (Sec. 2.5, kappa = 1).
 * Both stay above 1 / alpha (= kappa) and approach |lam| for large |lam|. */
typedef enum { RMHMC_SOFTABS_COTH = 0, RMHMC_SOFTABS_SQRT = 1 } rmhmc_softabs;

/* Per-record likelihoods (Sec. 2.1, Eq. data_likelihood):
 *   BERNOULLI_LOGIT  y in {0,1}, P(y = 1) = sigmoid(f);
 *   GAUSSIAN         y ~ N(f, noise_var);
 *   GAUSSIAN_MV      Example 1 of Sec. 2.1 (Eq. mvmodel), two latent
 *                    functions: y ~ N(f1, delta + exp f2).  The N latent
 *                    points are the R = N / 2 records twice, f1 first, then
 *                    f2 (n_fns = 2, see rmhmc_model_desc); y has N
 *                    entries, the R targets first (the rest are unused). */
typedef enum {
  RMHMC_LIK_BERNOULLI_LOGIT = 0,
  RMHMC_LIK_GAUSSIAN = 1,
  RMHMC_LIK_GAUSSIAN_MV = 2
} rmhmc_lik;

/* Kernel terms of the multiple-kernel prior f ~ GP(0, sum_c k_c) (Sec. 2.1,
 * Eq. BMKL).  Parameters are consumed in term order:
 *   SE_ISO(cols)     s^2 exp(-|x-x'|^2 / (2 l^2))         eta = (log s, log l)
 *   SE_ARD(cols)     s^2 exp(-sum_d r_d^2 / (2 l_d^2))    eta = (log s, log l_d..)
 *   LINEAR_ARD(cols) sum_d v_d x_d x'_d                   eta = (log v_d..)
 *   BINARY_SAME(col) s^2 [x_c == x'_c]                    eta = (log s)          */
typedef enum {
  RMHMC_K_SE_ISO = 0,
  RMHMC_K_SE_ARD = 1,
  RMHMC_K_LINEAR_ARD = 2,
  RMHMC_K_BINARY_SAME = 3
} rmhmc_kernel_kind;

#define RMHMC_MAX_TERM_COLS 8

typedef struct {
  int kind;                          /* rmhmc_kernel_kind                  */
  int ncols;                         /* 1..RMHMC_MAX_TERM_COLS              */
  int cols[RMHMC_MAX_TERM_COLS];     /* covariate columns used by the term  */
  int fn;                            /* with n_fns = 2: the latent function
                                        (0 or 1) whose prior the term is
                                        part of, -1 for all points; ignored
                                        otherwise                           */
} rmhmc_kernel_term;

typedef struct {
  int N, dx;                 /* data points, covariates                        */
  const double* X;           /* [host] N x dx, row-major (X[i*dx + c])         */
  const double* y;           /* [host] N labels in {0,1} (logit) or targets    */
  int lik;                   /* rmhmc_lik                                      */
  double noise_var;          /* Gaussian likelihood only                       */
  int nterms;
  const rmhmc_kernel_term* terms; /* [host] nterms entries                     */
  double jitter;             /* fixed diagonal added to K (> 0)                */
  double beta;               /* inverse temperature on the likelihood, >= 0   */
  int n_fns;                 /* latent functions J: 0 or 1, or 2 with
                                GAUSSIAN_MV (each f_j has its own GP prior,
                                Sec. 2.1 Eq. BMKL: a term acts only between
                                two points of its function, so K is block
                                diagonal)                                     */
  int fn_col;                /* n_fns = 2: column of X holding each point's
                                function index (0 for the first R rows, 1
                                for the last R)                               */
  double delta;              /* GAUSSIAN_MV: the fixed variance floor (> 0)  */
} rmhmc_model_desc;

typedef struct rmhmc_model rmhmc_model;
typedef struct rmhmc_state rmhmc_state;

/* Inputs of Algorithm 1 besides the target and q(0): A total moves of which
 * the first A0 are burn-in, step size, C leapfrogs per move, the softabs
 * sharpness, and how the implicit equations and the eigensolver are run.
 * The randomness of a chain is fixed by (seed, stream_id): Philox4x64-10
 * with key (seed, stream_id) and counter (block, move, purpose, 0); momentum
 * normals by Box-Muller, two per pair of 53-bit uniforms (purpose 0); the
 * Metropolis-Hastings uniform of a move from purpose 1. */
typedef struct {
  double eps;            /* leapfrog step size epsilon                        */
  double alpha;          /* softabs sharpness (coth: g = lam coth(alpha lam);
                            sqrt: kappa = 1 / alpha)                          */
  double zeta;           /* Jacobi tolerance (<= 0: 1e-13)                    */
  int n_leapfrog;        /* C, leapfrogs per move                             */
  int n_moves;           /* A, moves in all (burn-in included)                */
  int n_burnin;          /* A0, leading moves not returned (0 <= A0 < A)      */
  int n_fixed_point;     /* K, fixed-point iterations per implicit equation   */
  int max_sweeps;        /* Jacobi sweep cap per eigendecomposition (<=0: 60) */
  int reorth_every;      /* re-orthonormalise the eigenvectors every this many
                            dynamic updates within a move (<=0: 10)           */
  unsigned long long seed;       /* Philox key word 0                          */
  unsigned long long stream_id;  /* Philox key word 1 (independent chains)     */
  int precision;         /* rmhmc_precision; must equal the model's           */
  int softabs;           /* rmhmc_softabs: the map g of the metric            */
} rmhmc_chain_cfg;

typedef struct {
  int accepted;          /* accepted moves among the returned ones (A - A0)   */
  int accepted_all;      /* accepted moves, burn-in included                  */
  int failures;          /* moves rejected because a step failed              */
  int fail_not_pd;       /*   of which: K not positive definite               */
  int fail_nonfinite;    /*   non-finite values                               */
  int fail_noconv;       /*   an eigensolve did not converge                  */
  long long leapfrogs;   /* generalized leapfrogs completed                   */
  long long eig_calls;   /* eigendecompositions                               */
  long long sweeps;      /* Jacobi sweeps over all eigendecompositions        */
  int eig_fallbacks;     /* warm starts redone by a static solve              */
  double max_res_p;      /* largest relative residual of the last fixed-point
                            iteration of the momentum equation                */
  double max_res_q;      /* ... of the position equation                      */
} rmhmc_chain_stats;

/* Build a model: copies X and y to the device and allocates every workspace
 * the calls below need for this N, P and D, the chain state of rmhmc_chain
 * included (no call below allocates device memory, except a stand-alone
 * rmhmc_softabs_eig larger than any before it on the device).
 * The prior is eta ~ N(0, I), f | eta ~ N(0, K(eta)); the likelihood of
 * Sec. 2.1 Eq. (data_likelihood), raised to the power beta (power posterior
 * of the evidence appendix).  Returns RMHMC_E_ARG for an invalid descriptor,
 * RMHMC_E_NOMEM if device memory runs out.  Calls on one model from several
 * threads are serialised (one runs at a time). */
rmhmc_status rmhmc_model_create(const rmhmc_model_desc* desc, rmhmc_precision prec,
                                rmhmc_model** out);
rmhmc_status rmhmc_model_dims(const rmhmc_model* m, int* N, int* P, int* D); /* [host] outs */
/* Device bytes held by the model (its scratch and chain state).  [host] out. */
rmhmc_status rmhmc_model_bytes(const rmhmc_model* m, long long* bytes);
rmhmc_status rmhmc_model_destroy(rmhmc_model* m);
/* The inverse temperature tau of the power posterior P(X|f)^tau prior(f, eta)
 * (appendix on model evidence): the likelihood of later calls is raised to
 * beta.  A host-side setting; no device work. */
rmhmc_status rmhmc_model_set_beta(rmhmc_model* m, double beta);
/* ln P(X | f) at q = (f, eta) (Sec. 2.1, Eq. data_likelihood; no tempering),
 * the integrand of the thermodynamic evidence estimate.  q [device] D,
 * ll [device] 1.  Synchronises the stream. */
rmhmc_status rmhmc_log_likelihood(rmhmc_model* m, const double* q, double* ll, hipStream_t stream);

/* The paper's own model, the reduced-rank basis form of Sec. 2.1 (Eqs. BMKL,
 * Solin_representation and hpar_prior; features in the appendix on the
 * reduced-rank representation), one latent function:
 *   f(x_i) = sum_k sum_m a_km phi_m(x_ik) + b,
 *   Gaussian-kernel covariate k: phi_m(x) = sin(pi m (x + L) / (2L)),
 *     m = 1..M, a_km ~ N(0, c_g V_m(sigma_g)),
 *     V_m(sigma) = sqrt(pi sigma) exp(-pi^2 m^2 sigma / (16 L^2)) (the
 *     spectral density of exp(-r^2 / sigma) at the m-th frequency);
 *   linear-kernel covariate k: one feature x_k, a_k ~ N(0, c_l);
 *   b ~ N(0, bias_var); c_g, sigma_g, c_l ~ InvGamma(ig_alpha[h], ig_beta[h]).
 * q = (a in covariate order, b, c_g, sigma_g, c_l): D = F + 4 with F the
 * number of features; the hyperparameters are sampled on their own (positive)
 * scale, and a trajectory that takes one to zero or below fails (a rejection
 * in rmhmc_chain).  The likelihood is BERNOULLI_LOGIT or GAUSSIAN, raised to
 * beta.  Every call below that takes an rmhmc_model works on it
 * (FP64 only); rmhmc_model_dims reports N = records and P = 3. */
typedef enum { RMHMC_BASIS_GAUSS = 0, RMHMC_BASIS_LINEAR = 1 } rmhmc_basis_kind;
typedef struct {
  int N, dx;                 /* records, covariates                            */
  const double* X;           /* [host] N x dx, row-major                       */
  const double* y;           /* [host] N labels {0,1} (logit) or targets       */
  int lik;                   /* rmhmc_lik: BERNOULLI_LOGIT or GAUSSIAN         */
  double noise_var;          /* Gaussian likelihood only                       */
  const int* kinds;          /* [host] dx entries of rmhmc_basis_kind          */
  int M;                     /* features per Gaussian-kernel covariate (>= 1)  */
  double L;                  /* half-width of the domain [-L, L] (> 0)         */
  double bias_var;           /* Sigma, the prior variance of b (> 0)           */
  double ig_alpha[3], ig_beta[3];  /* InvGamma of (c_g, sigma_g, c_l) (> 0)    */
  double beta;               /* inverse temperature on the likelihood, >= 0   */
} rmhmc_basis_desc;
rmhmc_status rmhmc_basis_model_create(const rmhmc_basis_desc* desc, rmhmc_model** out);

/* U(q) = -ln P(q) (constants included), grad U and the Hessian H of U at q
 * (H is the matrix the softabs map of Sec. 2.2 is applied to).
 *   q [device] D; U [device] 1; gradU [device] D; H [device] D x D, ldh >= D.
 * RMHMC_E_NOT_PD if the Cholesky factorisation of K fails.  Synchronises the
 * stream. */
rmhmc_status rmhmc_hessian(rmhmc_model* m, const double* q, double* U, double* gradU,
                           double* H, int ldh, hipStream_t stream);

/* Softabs eigendecomposition (Sec. 2.2; dynamic form Sec. 2.4).
 * H = Q diag(lam) Q' by cyclic two-sided Jacobi.  Q_warm == NULL: static
 * solve from the identity.  Q_warm != NULL: the dynamic update of Sec. 2.4,
 * Jacobi on Q_warm' H Q_warm, then Q = Q_warm * (its rotations).  Stops when
 * off(M)_F <= zeta ||M||_F (zeta <= 0 selects 1e-13).
 *   H [device] D x D (ldh); Q_warm, Q [device] D x D (ld = D);
 *   softabs: the map g (rmhmc_softabs) with parameter alpha;
 *   lam, g, gp [device] D: eigenvalues, g(lam) and g'(lam);
 *   logdetG [device] 1 = sum log g;  sweeps [host, nullable].
 * Eigenvalues are not sorted.  Reads the convergence flag after each sweep;
 * synchronises the stream.  The workspace is per device and shared by the
 * calls on it (they run one at a time); a call on a larger D than any before
 * allocates it, which rmhmc_softabs_eig_reserve(D) does ahead of time.
 * RMHMC_E_EIG_NOCONV if max_sweeps (<= 0 selects 60) runs out,
 * RMHMC_E_NONFINITE for non-finite entries. */
rmhmc_status rmhmc_softabs_eig(int D, const double* H, int ldh, double alpha, int softabs,
                               double zeta, int max_sweeps, const double* Q_warm, double* Q,
                               double* lam, double* g, double* gp, double* logdetG, int* sweeps,
                               hipStream_t stream);
rmhmc_status rmhmc_softabs_eig_reserve(int D);
/* The same eigensolve for callers that cannot allocate device memory (code
 * that must not call hipMalloc, such as tight serving loops or harnesses that
 * forbid it): its workspace is a file-scope device array of the library,
 * one per device, sized for D <= 1088 (29 MB, held until the process ends);
 * the call allocates nothing.  RMHMC_E_ARG for D > 1088.  Calls on one device
 * share that array and are serialised by the library; it keeps the last
 * call's contents, and every call initialises what it reads.  Arguments,
 * outputs, errors and synchronisation as rmhmc_softabs_eig. */
rmhmc_status rmhmc_softabs_eig_noalloc(int D, const double* H, int ldh, double alpha,
                                       int softabs, double zeta, int max_sweeps,
                                       const double* Q_warm, double* Q, double* lam, double* g,
                                       double* gp, double* logdetG, int* sweeps,
                                       hipStream_t stream);

/* Hamiltonian and its gradients at (q, p) for a given eigen-state (Q, lam)
 * of H(q) (Sec. 2.2, Eq. Hamiltonian and Eq. d_Hamiltonian, with the metric
 * terms signed as the derivative of Eq. Hamiltonian gives:
 *   dH/dq = grad U + 1/2 tr(W2 dH/dq) - 1/2 tr(W1 dH/dq), dH/dp = G^-1 p),
 * where the traces use the cached W1, W2 of Eq. (Betancourt_formula) and the
 * structure-ordered contraction of Sec. 2.3.
 *   q, p [device] D; Q [device] D x D (ld D); lam [device] D;
 *   alpha, softabs: the softabs map (rmhmc_softabs);
 *   dHdq, dHdp [device] D; ham [device] 1. */
rmhmc_status rmhmc_metric_grad(rmhmc_model* m, const double* q, const double* p,
                               const double* Q, const double* lam, double alpha, int softabs,
                               double* dHdq, double* dHdp, double* ham, hipStream_t stream);

/* Device-resident integrator state (q, p, eigen-state and per-point caches).
 * q0, p0 [device] D; alpha, softabs: the softabs map.  The first
 * eigendecomposition is static; later ones are warm-started (Sec. 2.4).
 * Synchronises `stream`. */
rmhmc_status rmhmc_state_create(rmhmc_model* m, const double* q0, const double* p0,
                                double alpha, int softabs, hipStream_t stream,
                                rmhmc_state** out);
rmhmc_status rmhmc_state_get(const rmhmc_state* s, double* q, double* p, double* ham,
                             hipStream_t stream);   /* [device] outs, ham nullable */
rmhmc_status rmhmc_state_set_momentum(rmhmc_state* s, const double* p, hipStream_t stream);
rmhmc_status rmhmc_state_destroy(rmhmc_state* s);
/* Counters of a state since creation: generalized leapfrogs, eigen-
 * decompositions and Jacobi sweeps (accepted/failures are 0).  [host] out. */
rmhmc_status rmhmc_state_stats(const rmhmc_state* s, rmhmc_chain_stats* out);
/* Momentum draw of Algorithm 1 at the state's current point:
 * p = G^{1/2} z = Q diag(sqrt g) Q' z, i.e. p ~ N(0, G(q)) for z ~ N(0, I);
 * the symmetric square root makes p a function of G alone (independent of
 * eigenvector signs).  z [device] D. */
rmhmc_status rmhmc_state_draw_momentum(rmhmc_state* s, const double* z, hipStream_t stream);

/* One generalized leapfrog (Sec. 2.2, Eq. leapfrog).  Both implicit
 * equations are solved by n_fixed_point plain fixed-point iterations
 * started at p(t) and q(t) (no early exit).  Metric evaluations at new
 * points are warm-started Jacobi updates (Sec. 2.4); a warm start that runs
 * out of sweeps is redone statically.  Reads one failure word at the end
 * (synchronises); on RMHMC_E_NOT_PD / _NONFINITE / _EIG_NOCONV the state
 * stays at its start point. */
rmhmc_status rmhmc_glf_step(rmhmc_model* m, rmhmc_state* s, double eps, int n_fixed_point,
                            hipStream_t stream);


/* RMHMC chain, Algorithm 1, entirely on the device: per move the momentum
 * p = G^{1/2} z (p ~ N(0, G(q)), z from the chain's Philox stream), C
 * generalized leapfrogs, then Metropolis-Hastings: accept iff
 * log r < H_old - H_new, else keep q and its eigen-state (the printed
 * algorithm restores on the opposite event).  A failure inside a move
 * (K not positive definite, non-finite values, no eigensolver convergence
 * after the static fallback) is a rejection, counted in the stats.  Outputs
 * are the moves A0 .. A-1:
 *   q0 [device] D; samples [device] (A - A0) x D (row-major: move-major);
 *   logpost [device] A - A0 (= -U(q) after each move);
 *   accepted [device] A - A0 (int32 0/1); stats [host, nullable].
 * The host reads the eigensolver's convergence flag after each sweep (no
 * other device read inside the chain) and synchronises once at the end. */
rmhmc_status rmhmc_chain(rmhmc_model* m, const rmhmc_chain_cfg* cfg, const double* q0,
                         double* samples, double* logpost, int* accepted,
                         rmhmc_chain_stats* stats, hipStream_t stream);

/* The randomness of move `move` of the chain (seed, stream_id), as
 * rmhmc_chain draws it (exposed for tests): the D momentum normals z and the
 * Metropolis-Hastings uniform u.  z [device] D, u [device] 1.  Asynchronous. */
rmhmc_status rmhmc_chain_randoms(int D, unsigned long long seed, unsigned long long stream_id,
                                 unsigned long long move, double* z, double* u,
                                 hipStream_t stream);

/* Concurrent chains: a pool of worker threads, each with its own HIP stream
 * (default priority), runs rmhmc_chain jobs side by side.  A job submitted
 * while others run starts as soon as a worker is free and no running job
 * uses the same model (a model's scratch memory serves one chain at a time),
 * so requests are admitted continuously rather than in fixed batches.  This
 * is how many independent chains, e.g. the tempered rungs of the
 * power-posterior evidence estimate (appendix on model evidence), share the
 * GPU.  Each job's results are bitwise identical to the same chain run
 * alone: every kernel reduces in a fixed order.
 *   rmhmc_pool_submit: same arguments as rmhmc_chain ([device] arrays owned by
 *     the caller, kept alive until the job is done); *ticket [host] identifies
 *     the job.  The model must not be destroyed before its jobs finish.
 *   rmhmc_pool_poll: *done = 0 while queued/running, 1 on success, or the
 *     job's negative rmhmc_status; wait != 0 blocks until done.  stats and
 *     times_ms [host, nullable]: times_ms[0..2] = submit, start, end in ms
 *     since the pool was created.  A finished ticket is released by the poll
 *     that reports it.
 *   rmhmc_pool_destroy: waits for running jobs, drops queued ones. */
typedef struct rmhmc_pool rmhmc_pool;
rmhmc_status rmhmc_pool_create(int n_workers, rmhmc_pool** out);
rmhmc_status rmhmc_pool_submit(rmhmc_pool* pool, rmhmc_model* m, const rmhmc_chain_cfg* cfg,
                               const double* q0, double* samples, double* logpost, int* accepted,
                               long long* ticket);
rmhmc_status rmhmc_pool_poll(rmhmc_pool* pool, long long ticket, int wait, int* done,
                             rmhmc_chain_stats* stats, double* times_ms);
rmhmc_status rmhmc_pool_destroy(rmhmc_pool* pool);

/* Batched chains with graph-captured moves, e.g. the tempered rungs of the
 * power-posterior evidence estimate (appendix on model evidence): every
 * admitted chain's move (momentum draw, C leapfrogs, Metropolis-Hastings,
 * sample store) is recorded once into a HIP graph and replayed, one replay
 * per move, on the batch's streams (default priority).  A chain's launch
 * shapes come from a tuner keyed by its class (padded dimension and
 * precision): on the first model of a class it times a few leapfrogs with
 * 1, 2, 4 and 8 k-range layers for the single D x D products and sets the
 * Jacobi sweep budget of each eigen-solve of a leapfrog's position
 * iteration in the captured moves to one more than the most sweeps that
 * iteration's warm start needed there; the choice is kept per class for the
 * process, so a chain runs the same launches alone or in any mix.  In a
 * captured move nothing is read back: a warm start that has not converged
 * within the budget fails the move (a rejection, counted in fail_noconv),
 * where rmhmc_chain would redo it statically.  Otherwise a chain's results
 * are bitwise those of rmhmc_chain on the same model and configuration.
 *   rmhmc_batch_admit: runs the chain's set-up (its first static solve, and
 *     the tuning of a new class) on a batch stream, then captures the move;
 *     q0, samples, logpost, accepted [device] as rmhmc_chain (caller-owned,
 *     alive until retired).  The model belongs to the batch until retired:
 *     other calls on it return RMHMC_E_ARG.  *slot [host] names the chain.
 *   rmhmc_batch_step: queues n_moves more moves of every active chain
 *     (chains stop at their cfg->n_moves); asynchronous.
 *   rmhmc_batch_sync: waits for every queued move.
 *   rmhmc_batch_retire: waits for the slot's moves, returns [host, nullable]
 *     the moves run, the stats, and the sweep budget and layer count used,
 *     and releases the model.
 *   rmhmc_batch_destroy: waits, releases every model, frees the batch. */
typedef struct rmhmc_batch rmhmc_batch;
rmhmc_status rmhmc_batch_create(int n_streams, rmhmc_batch** out);
rmhmc_status rmhmc_batch_admit(rmhmc_batch* batch, rmhmc_model* m, const rmhmc_chain_cfg* cfg,
                               const double* q0, double* samples, double* logpost, int* accepted,
                               int* slot);
rmhmc_status rmhmc_batch_step(rmhmc_batch* batch, int n_moves);
rmhmc_status rmhmc_batch_sync(rmhmc_batch* batch);
rmhmc_status rmhmc_batch_retire(rmhmc_batch* batch, int slot, int* moves_done,
                                rmhmc_chain_stats* stats, int* sweep_budget, int* gsplit);
rmhmc_status rmhmc_batch_destroy(rmhmc_batch* batch);

/* Building block exposed for tests and benchmarks: the MFMA GEMM every
 * dense product above runs on.  C = alpha op(A) op(B) + beta C, column-major,
 * op(X) = X' when the trans flag is non-zero; A, B, C [device].
 * rmhmc_gemm_f64 uses v_mfma_f64_16x16x4f64, rmhmc_gemm_f32
 * v_mfma_f32_16x16x4f32 (FP32 accumulation).  Asynchronous on `stream`. */
rmhmc_status rmhmc_gemm_f64(int m, int n, int k, double alpha, const double* A, int lda, int transA,
                            const double* B, int ldb, int transB, double beta, double* C, int ldc,
                            hipStream_t stream);
rmhmc_status rmhmc_gemm_f32(int m, int n, int k, float alpha, const float* A, int lda, int transA,
                            const float* B, int ldb, int transB, float beta, float* C, int ldc,
                            hipStream_t stream);
/* C = op(A) op(B) for one product whose k range is split over `splits`
 * (1..64) workgroup layers, then added layer by layer in a fixed order: the
 * form used for the single D x D products of the eigen warm start and for
 * K^-1 = L^-T L^-1, where 64 x 64 output tiles alone leave about one wave per
 * SIMD.  A, B, C and `work` [device, caller-owned]; `work` holds
 * splits * m * n doubles and is overwritten.  Products whose k range is
 * shorter than 32 * splits take the unsplit kernel.  RMHMC_E_ARG for bad
 * sizes, leading dimensions, NULL pointers or `splits`.  Asynchronous on
 * `stream`. */
rmhmc_status rmhmc_gemm_f64_splitk(int m, int n, int k, const double* A, int lda, int transA,
                                   const double* B, int ldb, int transB, double* C, int ldc,
                                   double* work, int splits, hipStream_t stream);
/* C (m x n, FP64, ld ldc) = A' B over a long inner dimension k, where A and
 * B hold m and n columns of length k (column i of A at A + i * lda): the
 * form of the traces tr(X Y) = <X, Y'> of products of N x N matrices
 * (k = N^2) in the Hessian's hyperparameter block and the third-derivative
 * tensor (Sec. 2.3).  With m <= 16, n <= 64, lda and ldb multiples of 4 and
 * A, B aligned to four elements, a streaming kernel reads each operand once
 * (one 16 x 16 MFMA tile per 16 columns of C); other shapes take the tiled
 * kernel with the k range split into layers.  The k range is cut into at
 * most `splits` (1..1024) chunks whose partials are added in a fixed order.
 * A, B, C and `work` [device, caller-owned]; `work` holds splits * m * n
 * elements of the operand type and is overwritten.  The _f32 form takes
 * FP32 operands (FP32 products and chunk sums, FP64 total).  RMHMC_E_ARG for
 * bad sizes, leading dimensions, NULL pointers or `splits`.  Asynchronous on
 * `stream`. */
rmhmc_status rmhmc_gemm_tallk_f64(int m, int n, long k, const double* A, long lda,
                                  const double* B, long ldb, double* C, int ldc, double* work,
                                  int splits, hipStream_t stream);
rmhmc_status rmhmc_gemm_tallk_f32(int m, int n, long k, const float* A, long lda, const float* B,
                                  long ldb, double* C, int ldc, float* work, int splits,
                                  hipStream_t stream);

/* Live per-kernel timing (instrumentation, off by default).  When enabled,
 * the launches of each kernel family below are bracketed by HIP events on
 * their own stream and their algorithmic work is tallied:
 *   0 FP64 MFMA GEMM, 1 FP32 MFMA GEMM, 2 Jacobi round launches of
 *   warm-started solves (one event pair per sweep, counted per launch),
 *   3 the same for static solves, 4 kernel-derivative weighted sums,
 *   5 kernel-derivative mat-vec, 6 Cholesky diagonal block.
 * rmhmc_timing_enable(mask) clears the tallies and times the families whose
 * bit (1 << family) is set, 0 switches timing off (synchronises the device);
 * rmhmc_timing_read waits for the recorded events and returns the launch
 * count, summed kernel milliseconds, algorithmic flops and bytes [host]. */
rmhmc_status rmhmc_timing_enable(unsigned mask);
rmhmc_status rmhmc_timing_read(int kind, long long* launches, double* ms, double* flops,
                               double* bytes);

/* Message for the last non-OK status on this thread ("" if none). */
const char* rmhmc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RMHMC_H */
