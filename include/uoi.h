/*
 * uoi.h -- C ABI of the MI355X (gfx950) UoI_LASSO / UoI_VAR library (libuoi.so).
 *
 * Method: Union of Intersections LASSO and its vector-autoregressive variant,
 * arXiv 1808.06992 (Algorithm 1, Algorithm 2).  Model selection solves a LASSO
 * (Eq. (2)) for every bootstrap k = 1..B1 and every lambda_j, j = 1..q, with ADMM
 * (Eq. (ADMM), Sec. II-E); the supports are intersected over bootstraps
 * (Eq. (intersection)); model estimation refits every support by least squares
 * on B2 training/evaluation splits, keeps the best support per split and
 * averages the refits (Eq. (union)).
 *
 * Conventions shared by every entry point
 *  - Every array argument is a DEVICE pointer (hipMalloc'd or a torch CUDA
 *    tensor) on the HIP device that is current in the calling thread, unless the
 *    comment says HOST.  Matrices are row-major, float64, densely packed.
 *  - The caller owns every input and output buffer; the library never frees or
 *    keeps a pointer to them.  Scratch memory is allocated by the library itself
 *    (a grow-only pool per device, released by uoi_release_workspace).
 *  - Work is enqueued on opts->stream (a hipStream_t; NULL = the default
 *    stream).  The fit and solve entry points synchronise that stream before
 *    returning, so outputs are valid on return.
 *  - Return value: UOI_OK (0) or a negative code.  No C++ exception crosses the
 *    ABI.  On error, uoi_last_error() returns a message (thread-local).
 *    Argument validation (sizes, lambda ordering, NaN/Inf in the data) happens
 *    before any result is written.  UOI_ENOCONV means every output was written
 *    but at least one ADMM solve did not reach opts->kkt_tol within max_iter;
 *    the per-solve flags in uoi_diag say which (or, for the refits of the
 *    estimation step, uoi_diag.n_refit_unconverged counts them).
 *  - Objective scaling: for a sample of m rows the LASSO minimised is
 *        (1/(2m)) * sum_rows (y - x'b)^2 + lambda * ||b||_1,
 *    which has the same minimiser as Eq. (2) with penalty 2*m*lambda.  Lambdas
 *    are given in this scaling and must be strictly decreasing and >= 0.
 *  - KKT residual (the stopping rule and the reported accuracy): with
 *    G = X'X/m, c = X'y/m and g = c - G b,
 *        v_i = |g_i - lambda*sign(b_i)|   if b_i != 0,
 *        v_i = max(0, |g_i| - lambda)    if b_i == 0,
 *        kkt = ||v||_inf / ||c||_inf.
 *    It is always evaluated in float64 with the float64 Gram.
 *  - Not thread-safe: calls that overlap on one device must be serialised by
 *    the caller.
 */
#ifndef UOI_H
#define UOI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    UOI_OK = 0,
    UOI_EINVAL = -1,  /* invalid argument (nothing was written)                */
    UOI_ENOMEM = -2,  /* device allocation failed                              */
    UOI_EHIP = -3,    /* a HIP runtime call or kernel launch failed            */
    UOI_ENOCONV = -4  /* outputs written; some solves missed the KKT tolerance */
};

/* precision of the selection sweep */
enum {
    UOI_FP64 = 0,   /* float64 Gram, factor, ADMM and KKT                        */
    UOI_MIXED = 1   /* float64 Gram and factor, float32 ADMM state and operator
                       (solves parked on a KKT estimate), float64 KKT checks
                       decide convergence after float64 finishing iterations     */
};

/* ADMM warm start */
enum {
    UOI_COLD = 0,   /* z = u = 0                                                 */
    UOI_MLP = 1     /* (z, u) predicted by the loaded warm-start network          */
};

/* selection solver organisation */
enum {
    UOI_SOLVER_BATCHED = 0, /* per bootstrap, all lambdas (and VAR equations) of one
                               ADMM iteration form one matrix product              */
    UOI_SOLVER_PLAIN = 1    /* one solve per workgroup, matrix-vector products     */
};

/* opts.flags */
#define UOI_FLAG_TIMING 1u     /* fill uoi_diag.stage_ms with hipEvent stage times */
#define UOI_FLAG_INTERCEPT 2u  /* UoI_VAR: fit the intercept mu of Eq. (5) (see uoi_var_fit) */
#define UOI_FLAG_EAGER 4u      /* launch every ADMM iteration on its own; by default each
                                  chunk of iterations between two KKT checks is recorded
                                  once as a HIP graph (per distinct set of launch arguments,
                                  cached per device) and replayed with one launch          */
#define UOI_FLAG_PER_EQUATION 16u /* UoI_VAR: every equation chooses its own support index per
                                     split (argmin of its own loss) instead of one index per
                                     split from the loss summed over equations (Alg. 2 on
                                     Eq. (8) as written); jstar_out is then [B2*p] and
                                     uoi_diag.losses [B2*q*p] (per equation)                  */
#define UOI_FLAG_NO_TUNE 8u    /* do not time launch-shape candidates: use the choices
                                  already recorded (in this process, or read from the file
                                  named by the environment variable UOI_TUNE_FILE) or the
                                  defaults.  By default the library's autotuner times, on
                                  the first call of each problem shape, the candidates of
                                  the ADMM products' tile shape (columns, and rows per
                                  wave above 64 solves per Gram) and of the factor's
                                  matrices per pass on the live operands (the candidates
                                  give identical results) and keeps the fastest           */

/* Opaque warm-start network (see the uoi_mlp_* functions below). */
typedef struct uoi_mlp uoi_mlp;

typedef struct uoi_opts {
    int32_t B1;            /* selection bootstraps, >= 1                                   */
    int32_t B2;            /* estimation splits, >= 1                                      */
    int32_t q;             /* number of lambdas, >= 1                                      */
    const double *lambdas; /* HOST, q values, strictly decreasing, >= 0                    */
    uint64_t seed;         /* drives every random choice (bootstrap rows, splits, blocks)  */
    double rho;            /* ADMM penalty, > 0 (default 1); 0: scaled to the data, the    */
                           /* mean diagonal of the Grams, read back once per solve (not    */
                           /* for the allocation-free entry point)                          */
    double kkt_tol;        /* relative KKT tolerance, > 0 (default 1e-6)                   */
    int32_t max_iter;      /* ADMM iteration cap, >= 1 (default 20000)                     */
    int32_t check_every;   /* KKT check period in ADMM iterations, >= 1 (default 10)       */
    int32_t train_num;     /* estimation split: train = floor(m*train_num/train_den) rows  */
    int32_t train_den;     /*   (LASSO) or blocks (VAR); default 4/5                       */
    int32_t precision;     /* UOI_FP64 or UOI_MIXED                                        */
    int32_t warm_start;    /* UOI_COLD or UOI_MLP                                          */
    int32_t solver;        /* UOI_SOLVER_BATCHED or UOI_SOLVER_PLAIN                       */
    uint32_t flags;        /* UOI_FLAG_*                                                   */
    void *stream;          /* hipStream_t, NULL = default stream                           */
    uoi_mlp *mlp;          /* warm-start network, required when warm_start == UOI_MLP
                              (UoI_LASSO only; network input p+1, output p)               */
    double relax;          /* ADMM over-relaxation alpha in [1, 1.95] (default 1: the plain
                              scaled ADMM).  With alpha, the z- and u-updates use
                              alpha*x + (1-alpha)*z_old in place of x (Boyd et al. 2011,
                              Sec. 3.4.3); the fixed point, hence the solution, is the same. */
    int32_t cg_max_iter;   /* iteration cap of the conjugate-gradient refits of supports with
                              more than 256 members, >= 1 (default 4000).  A refit still above
                              its tolerance (relative residual 1e-13) at the cap is used as it
                              is, counted in uoi_diag.n_refit_unconverged, and the fit returns
                              UOI_ENOCONV.                                                      */
} uoi_opts;

/* Per-kernel totals gathered with UOI_FLAG_TIMING: device time from hipEvents
 * recorded on opts->stream around the launches, and the ALGORITHMIC bytes and
 * flops of those launches (bytes: every operand the kernel must read or write
 * once; flops: 2 per multiply-add of useful work).  Slots: */
enum {
    UOI_KSTAT_ADMM64 = 0, /* batched ADMM iteration, float64: per bootstrap with an active
                             solve p*p*8 bytes of M, per active solve 4*p*8 bytes of z,u
                             (read and write); 2*p*p flops per active solve                  */
    UOI_KSTAT_ADMM32 = 1, /* the same in float32 (4-byte M and state)                      */
    UOI_KSTAT_PLAIN = 2,  /* one-solve-per-workgroup kernel: per solve and iteration p*p*8
                             bytes of M and 2*p*p flops (plus the Gram at each check)       */
    UOI_KSTAT_GRAM = 3,   /* selection Gram: m*(p+pe)*8 bytes of gathered rows + p*(p+pe)*8
                             bytes of output per bootstrap; m*p*(p+1) + 2*m*p*pe flops     */
    UOI_KSTAT_N = 4
};
typedef struct uoi_kstat {
    double ms;        /* summed device time of the launches             */
    double bytes;     /* summed algorithmic bytes                       */
    double flops;     /* summed algorithmic flops                       */
    int64_t launches; /* number of launches                             */
} uoi_kstat;

/* Optional diagnostics.  Array members are DEVICE pointers owned by the caller
 * and may be NULL; scalar members are written by the library.  A selection
 * solve is indexed s = k*R + r, with R = q for LASSO and R = q*p for VAR
 * (r = j*p + e, e = equation). */
typedef struct uoi_diag {
    int32_t *iters;     /* [B1*R] ADMM iterations at convergence (-1 = not converged)   */
    double *kkt;        /* [B1*R] final float64 relative KKT residual                    */
    double *sel_beta;   /* [B1*R*p] selection estimates z, solve-major                   */
    double *losses;     /* [B2*q] estimation losses (VAR: summed over equations)         */
    int64_t n_solves;   /* B1*R                                                          */
    int64_t n_unconverged;
    int32_t max_iters;  /* largest iteration count among converged solves               */
    int64_t warm_used;  /* solves started from the network (the rest fell back to cold)  */
    float stage_ms[8];  /* with UOI_FLAG_TIMING: index/gram, factor, admm, verify,
                           support, estimation-gram, ols, loss+average                   */
    uoi_kstat kstat[UOI_KSTAT_N]; /* with UOI_FLAG_TIMING: per-kernel totals (see below) */
    int64_t n_refit_unconverged;  /* estimation refits (split x support [x equation]) that
                                     conjugate gradients left above its tolerance at
                                     opts.cg_max_iter (the fit then returns UOI_ENOCONV)     */
} uoi_diag;

/* Fill *o with the defaults listed above (B1 = B2 = q = 0, lambdas = NULL). */
void uoi_default_opts(uoi_opts *o);

/*
 * UoI_LASSO, Algorithm 1.
 *   n, p      rows and features (n >= 2, p >= 1)
 *   X         n*p row-major design; y: n responses
 *   beta_out  [p]   averaged estimate beta* (Eq. (union))
 *   supp_out  [q*W] intersected supports S_j (Eq. (intersection)), W = ceil(p/64)
 *             uint64 words, bit i of word i/64 set when feature i is in S_j
 *   jstar_out [B2]  support index chosen by each estimation split
 *   diag      nullable
 */
int uoi_lasso_fit(int32_t n, int32_t p, const double *X, const double *y, const uoi_opts *o,
                  double *beta_out, uint64_t *supp_out, int32_t *jstar_out, uoi_diag *diag);

/*
 * UoI_VAR, Algorithm 2, for a VAR(d) series (Eq. (5)): x_t = mu + sum_{l=1..d} A_l x_{t-l} + u_t.
 * The regression of Eq. (6)-(7) uses rows t = d..T-1 (response x_t, design
 * [x_{t-1}, ..., x_{t-d}]).  The vectorised LASSO of Eq. (8) is solved as p
 * per-equation LASSOs that share the design Gram and one lambda (the Kronecker
 * matrix of Eq. (8) is never formed).
 * Intercept (opts.flags & UOI_FLAG_INTERCEPT; Alg. 2 returns mu, which Eq. (5)
 * as printed omits): mu is unpenalised and always in the model.  Every sample
 * (bootstrap sample, training set) is centred by its own column means (repeated
 * rows counted with multiplicity); each refit's intercept is
 * ybar_T - xbar_T' b, its evaluation loss uses the residuals y - mu - x'b, and
 * mu-hat averages the chosen refits' intercepts like the coefficients.  Without
 * the flag mu = 0.  The lambdas are in the centred scaling when the flag is set.
 *   T, p, d    series length, dimension (p >= 1), order (d >= 1, d*p <= 65536), T >= d + 2
 *   series     T*p row-major, time ascending
 *   block_len  bootstrap block length in regression rows; 0 = smallest L with
 *              L^3 >= T-d
 *   A_out      [d*p*p] A_l[i][m] at ((l-1)*p + i)*p + m: coefficient of x_{t-l,m} in equation i
 *   mu_out     [p]   intercept estimate (zeros without UOI_FLAG_INTERCEPT)
 *   supp_out   [q*p*W] supports S_j per equation, W = ceil(d*p/64); bit (l-1)*p + m is the
 *              coefficient A_l[i][m] (Eq. (7)'s column order)
 *   jstar_out  [B2]  support index chosen per split (one for all equations), or with
 *              UOI_FLAG_PER_EQUATION [B2*p], jstar_out[k*p + i] for equation i
 * diag->losses is [B2*q] (summed over equations), or [B2*q*p] with UOI_FLAG_PER_EQUATION.
 * diag->sel_beta, when given, is [B1][q][p][d*p] with the coefficients of each
 * solve in the library's internal column order (lag d first, lag 1 last).
 */
int uoi_var_fit(int32_t T, int32_t p, int32_t d, const double *series, int32_t block_len,
                const uoi_opts *o, double *A_out, double *mu_out, uint64_t *supp_out,
                int32_t *jstar_out, uoi_diag *diag);

/*
 * Batch of LASSO solves by ADMM (the selection inner loop, Eq. (ADMM)) for nb
 * problems given by their normal-equation statistics, each at all q lambdas.
 *   G    [nb*p*p]  symmetric positive definite Grams
 *   c    [nb*p]    linear terms
 *   z0   [nb*q*p]  nullable warm start for z (u starts at 0 unless u0 given)
 *   u0   [nb*q*p]  nullable warm start for u
 *   z_out, u_out [nb*q*p] final iterates (u_out nullable), solve-major
 *   iters [nb*q], kkt [nb*q]  nullable per-solve diagnostics
 * opts: q, lambdas, rho, kkt_tol, max_iter, check_every, precision, solver, stream
 * are used; B1/B2/seed are ignored.
 */
int uoi_lasso_solve_batch(int32_t nb, int32_t p, const double *G, const double *c,
                          const uoi_opts *o, const double *z0, const double *u0,
                          double *z_out, double *u_out, int32_t *iters, double *kkt);

/*
 * uoi_lasso_solve_batch without any allocation, for callers that cannot
 * allocate (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc): same arguments, results and errors as
 * uoi_lasso_solve_batch, computed by the same kernels.  The scratch memory is a
 * static device array of UOI_NOALLOC_SCRATCH_BYTES (64 MiB) built into the
 * library, one per device, held until the process ends; the call allocates no
 * device or pinned host memory and creates no stream or event (the host reads
 * the convergence counts synchronously).  A problem whose scratch exceeds the
 * array (about 8*nb*p*p + 48*nb*q*p bytes in float64, more in UOI_MIXED) is
 * rejected with UOI_EINVAL before any device work.  opts.warm_start must be
 * UOI_COLD.  Every call on a device shares that device's array: calls that
 * overlap on one device race and must be serialised by the caller.
 */
#define UOI_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int uoi_lasso_solve_batch_noalloc(int32_t nb, int32_t p, const double *G, const double *c,
                                  const uoi_opts *o, const double *z0, const double *u0,
                                  double *z_out, double *u_out, int32_t *iters, double *kkt);

/*
 * LASSO solves sharing a Gram: for each of nb Grams G_b, pe linear terms
 * C_b[:, e] (C [nb*p*pe], c[b][i][e]), each at all q lambdas of opts; the
 * solves of one Gram run as one batched ADMM (the structure of the per-equation
 * VAR problems of Eq. (8)).  z_out [nb*q*pe*p] = z[b][j][e][i]; iters, kkt
 * [nb*q*pe] nullable.  opts as for uoi_lasso_solve_batch; cold start only.
 */
int uoi_lasso_solve_multi(int32_t nb, int32_t p, int32_t pe, const double *G, const double *C,
                          const uoi_opts *o, double *z_out, int32_t *iters, double *kkt);

/*
 * Gram of sampled rows (Alg. 1 bootstrap statistics): for b < nb,
 *   G_b = X_r'X_r / m,  C_b = X_r'Y_r / m  with r = rows[b*m .. b*m+m-1]
 * (rows counted with multiplicity), X row r at X + r*ldx (p values), Y row r at
 * Y + r*ldy (pe values).  G [nb*p*p], C [nb*p*pe] (nullable when pe == 0).
 */
int uoi_gram(int32_t nb, int32_t m, const int32_t *rows, int32_t p, const double *X,
             int32_t ldx, int32_t pe, const double *Y, int32_t ldy, double *G, double *C,
             void *stream);

/*
 * Index streams (device output; host-callable for tests).  Counter-based
 * SplitMix64 keys key(seed, tag, k, i) mapped to [0, m) by multiply-shift.
 *   uoi_bootstrap_rows:  rows[k*n + i] for k < nb: n draws with replacement
 *   uoi_split_rows:      train[k*ntr..], eval[k*(n-ntr)..], ascending, with
 *                        ntr = floor(n*num/den)
 *   uoi_var_boot_rows:   rows[k*N + i]: moving blocks of length L
 *   uoi_var_split_rows:  blocks split by key; train/eval rows ascending;
 *                        counts written to HOST ntr_out[nb], nev_out[nb];
 *                        train/eval rows at offsets k*N
 */
int uoi_bootstrap_rows(uint64_t seed, int32_t nb, int32_t n, int32_t *rows, void *stream);
int uoi_split_rows(uint64_t seed, int32_t nb, int32_t n, int32_t num, int32_t den,
                   int32_t *train, int32_t *eval, void *stream);
int uoi_var_boot_rows(uint64_t seed, int32_t nb, int32_t N, int32_t L, int32_t *rows,
                      void *stream);
int uoi_var_split_rows(uint64_t seed, int32_t nb, int32_t N, int32_t L, int32_t num,
                       int32_t den, int32_t *train, int32_t *eval, int32_t *ntr_out,
                       int32_t *nev_out, void *stream);

/* Batched inverse of G_b + rho*I (float64, blocked Gauss-Jordan sweep):
 * M [nb*p*p] may alias nothing else.  Used by the ADMM x-update. */
int uoi_spd_inverse(int32_t nb, int32_t p, const double *G, double rho, double *M, void *stream);

/*
 * Warm-start network (not part of the paper, whose ADMM starts cold): a 3-layer
 * ReLU MLP that maps one selection problem (bootstrap statistics c, penalty
 * lambda) to an ADMM starting point,
 *     input  x = [c / lambda_max, log(lambda / lambda_max)]   (n_in  = p + 1)
 *     output z / lambda_max                                  (n_out = p)
 * with lambda_max = ||c||_inf.  Layers y = x W' + b with W stored (out, in);
 * the flat parameter vector is [W1 (hidden x n_in), b1, W2 (hidden x hidden), b2,
 * W3 (n_out x hidden), b3], float32 master copy.  GEMM operands are bfloat16
 * (round to nearest even) with float32 accumulation on MFMA.  Loss = mean over
 * rows and outputs of (y - t)^2; optimiser Adam (beta 0.9 / 0.999, eps 1e-8).
 * With opts->warm_start == UOI_MLP the fit predicts z for every (bootstrap,
 * lambda), sets u = clip((c - G z) / rho, -lambda/rho, lambda/rho), and keeps
 * the cold start for a solve whose predicted z does not lower the LASSO
 * objective z'Gz/2 - c'z + lambda*|z|_1 below its value 0 at z = 0.
 * X, Y, T, theta, grad are DEVICE float32 arrays, row-major; loss is HOST.
 * A network is used by one stream at a time (it owns its activation buffers).
 */
int uoi_mlp_create(int32_t n_in, int32_t hidden, int32_t n_out, uoi_mlp **out); /* zero weights */
void uoi_mlp_destroy(uoi_mlp *m);
int64_t uoi_mlp_num_params(const uoi_mlp *m);
int uoi_mlp_set_params(uoi_mlp *m, const float *theta, void *stream); /* also resets Adam */
int uoi_mlp_get_params(const uoi_mlp *m, float *theta, void *stream);
int uoi_mlp_forward(uoi_mlp *m, int32_t n, const float *X, float *Y, void *stream);
int uoi_mlp_loss_grad(uoi_mlp *m, int32_t n, const float *X, const float *T, float *grad,
                      double *loss, void *stream);             /* grad nullable */
int uoi_mlp_train_step(uoi_mlp *m, int32_t n, const float *X, const float *T, float lr,
                       double *loss, void *stream);            /* one Adam step, enqueued on
                                                                  stream; loss nullable (when
                                                                  given, the call synchronises) */
/* Training pairs for the network from solved problems: nb Grams, pe linear
 * terms each, q lambdas:
 *   c [nb*p*pe] linear terms (c[b][i][e]), lambdas HOST [q],
 *   z [nb*q*pe*p] solutions (z[b][j][e][i])
 *   X [nb*q*pe*(p+1)] network inputs, T [nb*q*pe*p] targets z / lambda_max (float32),
 *   row (b*q + j)*pe + e.  (The network's training data; not part of the paper.) */
int uoi_ws_dataset(int32_t nb, int32_t p, int32_t q, int32_t pe, const double *c,
                   const double *lambdas, const double *z, float *X, float *T, void *stream);

/* Free the library's scratch pool on the current device. */
void uoi_release_workspace(void);

/* Forget the launch shapes the autotuner recorded in this process (see
 * UOI_FLAG_NO_TUNE); the file named by UOI_TUNE_FILE, if any, is read again at
 * the next use. */
void uoi_tune_reset(void);

/* Message for the last non-OK status returned in this thread ("" if none). */
const char *uoi_last_error(void);

/* Library version string. */
const char *uoi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* UOI_H */
