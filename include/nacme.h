/*
 * nacme.h - C ABI of the MI355X (gfx950) CCSD non-adiabatic derivative
 * coupling library (libnacme.so).
 *
 * The library evaluates, for the closed-shell CCSD model, the biorthonormal
 * derivative coupling F_ij = <psi_i^L | d psi_j^R>  between excited states i
 * and j (Kjonstad & Koch, Sec. II A, eq. nac) through the Lagrangian route of
 * Sec. II: ground-state amplitudes (Sec. II A), right and left EOM states
 * (Sec. II A), the multipliers gamma, zeta and kappa-bar (Sec. II B, eqs.
 * amplituderelax and orbitalrelax), effective densities (Sec. II C, eq.
 * NAC_NC_densities) and their contraction with Hamiltonian derivatives
 * (Sec. II C, eq. NAC_NC).
 *
 * Hamiltonian: H = sum_pq h_pq E_pq + 1/2 sum_pqrs g_pqrs e_pqrs over n = o + v
 * orthonormal spatial orbitals (o occupied first), with density-fitted
 * two-electron integrals g_pqrs = (pq|rs) = sum_P B[P][p][q] B[P][r][s] and
 * a canonical Hartree-Fock reference: the Fock matrix
 * f_pq = h_pq + sum_k (2 g_pqkk - g_pkkq) equals diag(eps).  The one-electron
 * integrals are implied by that condition and are never passed.
 *
 * Conventions
 *  - Every call returns a status: 0 OK, 1 CC_NOT_CONVERGED (outputs hold the
 *    last iterate), negative = error: -1 ARG, -2 STATE (call order), -3 HIP
 *    (device failure; sticky), -4 OOM, -5 NUMERIC (NaN/Inf), -6 COMPLEX_ROOT.
 *    cc_last_error() returns a readable message for the last failure.
 *  - Large arrays are DEVICE pointers owned by the caller, fp64, row-major;
 *    they are read during the call and copied where the library keeps them.
 *    Small results (energies, omega[], F[], iteration counts) are HOST
 *    pointers.  All device work is enqueued on the stream given to
 *    cc_create (NULL = default stream); the call synchronises that stream
 *    before it writes host outputs.  A context is not thread-safe.
 *  - Amplitude-shaped vectors (t, R_k, L_k, zeta, ...) are stored as
 *    [o*v singles x1[i][a]] followed by [o*o*v*v doubles x2[i][j][a][b]],
 *    with x2[i][j][a][b] == x2[j][i][b][a].  The doubles parameters are the
 *    unique pairs (ai) <= (bj), T2 = 1/2 sum t_aibj E_ai E_bj; the
 *    biorthonormal inner product is sum_mu x_mu y_mu over the unique
 *    parameters.  Left vectors are coefficients of the biorthonormal dual
 *    basis <mu~|.
 *  - Excited states are numbered 1..nroots in ascending excitation energy;
 *    0 is the ground state.  Right states are normalised to unit
 *    biorthonormal norm with their largest-magnitude parameter positive; left
 *    states satisfy L_k . R_l = delta_kl.
 *  - Call order: cc_create -> cc_ground -> eom_solve(RIGHT) and
 *    eom_solve(LEFT) (or BOTH) -> multipliers(pairs) -> densities(i,j) ->
 *    nacme(i,j).  Anything else returns -2.
 */
#ifndef NACME_H
#define NACME_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CC_OK 0
#define CC_NOT_CONVERGED 1
#define CC_ERR_ARG (-1)
#define CC_ERR_STATE (-2)
#define CC_ERR_HIP (-3)
#define CC_ERR_OOM (-4)
#define CC_ERR_NUMERIC (-5)
#define CC_ERR_COMPLEX_ROOT (-6)

#define CC_RIGHT 1
#define CC_LEFT 2
#define CC_BOTH 3

#define CC_FP64 0          /* every contraction in fp64                          */
#define CC_FP32_REFINE 1   /* large contractions with fp32 operands on the FP32
                              matrix cores inside the solvers; the current
                              solution gets fp64 operator images that correct
                              the subspace, and only fp64 residuals decide
                              convergence (iterative refinement)             */
#define CC_BF16X3_REFINE 2 /* as CC_FP32_REFINE, with the eigen- and linear
                              solvers' contractions run as bfloat16 pairs
                              (hi + lo, three bf16 matrix-core products, fp32
                              accumulation, ~1e-5 relative); ground state
                              with fp32 operands                            */

/* Export / guess selectors. */
#define CC_T 1        /* ground amplitudes (amplitude-shaped)                 */
#define CC_R 2        /* right EOM state idx (amplitude-shaped)               */
#define CC_L 3        /* left EOM state idx (amplitude-shaped)                */
#define CC_R0 4       /* reference weight R0 of right state idx (1 double)    */
#define CC_ZETA 5     /* zeta-bar of the pair (i, j) (amplitude-shaped)       */
#define CC_KAPPA 6    /* kappa-bar of the pair (i, j) ([o][v])                */
#define CC_D1 7       /* effective one-electron density of (i, j) ([n][n])   */
#define CC_ETA_T 8    /* right-hand side eta_t of the zeta equation of (i, j) */
#define CC_ETA_K 9    /* right-hand side eta_kappa of the kappa equation      */
#define CC_DTRANS 10  /* transition density <L_i|E_pq|R_j> ([n][n])           */

typedef struct cc_ctx cc_ctx;

typedef struct {
  int precision;       /* CC_FP64, CC_FP32_REFINE or CC_BF16X3_REFINE          */
  int relaxed;         /* 1: orbital-relaxed (kappa-bar solved), 0: fixed      */
                       /*    reference (kappa-bar = 0)                         */
  double tol_ground;   /* max |Omega_mu| of the ground state                   */
  double tol_eom;      /* biorthonormal norm of each EOM residual              */
  double tol_mult;     /* biorthonormal norm of the multiplier residuals      */
  int maxit;           /* iteration cap of every solver                        */
  int diis_dim;        /* DIIS history of the ground-state solver              */
  int davidson_block;  /* extra trial vectors beyond nroots                    */
  int davidson_max;    /* subspace size before a restart (Davidson; the      */
                       /* linear solvers use min(120, max(it, 4 k + 4)))     */
  double mixed_min_flops; /* CC_FP32_REFINE: contractions with fewer flops     */
                          /* stay fp64 (default 1e9)                           */
} cc_opts;

/* Defaults: FP64, relaxed, tolerances 1e-10 / 1e-9 / 1e-9, maxit 200,
 * diis_dim 8, davidson_block 2, davidson_max 120 (at most 128),
 * mixed_min_flops 1e9.                                                        */
void cc_default_opts(cc_opts* opts);

/* Creates a context.  eps[n]: canonical orbital energies (device); B[naux][n][n]
 * (device), symmetric in p, q.  Copies both; keeps the factor and builds from
 * it only the bare blocks (ac|bd), (kc|bd) and (kc|ld) (v^4, o v^3, o^2 v^2
 * doubles); every other integral block is formed from the factor where it is
 * used.  opts may be NULL (defaults).  stream: hipStream_t or NULL.
 * Errors: -1 bad sizes/pointers, -4 out of device memory, -3 HIP failure.   */
int cc_create(cc_ctx** ctx, int o, int v, int naux, const double* eps, const double* B,
              const cc_opts* opts, void* stream);

/* Solves the CCSD amplitude equations Omega(t) = 0 (Sec. II A) from t = 0 (or
 * from a guess set with cc_set_guess(CC_T)).  e_corr: correlation energy
 * <HF|exp(-T) H exp(T)|HF> - E_HF (host).  iters (host, may be NULL).       */
int cc_ground(cc_ctx* ctx, double* e_corr, int* iters);

/* Lowest nroots excitation energies of the CC Jacobian A = dOmega/dt
 * (Sec. II B) and the right (A R = omega R) and/or left (L A = omega L)
 * states; after both sides are known they are gauged and biorthonormalised
 * and R0_k = eta.R_k / omega_k is formed.  omega: host [nroots].
 * -6 if a requested root is complex.                                        */
int eom_solve(cc_ctx* ctx, int side, int nroots, double* omega, int* iters);

/* Multipliers of npairs ordered pairs (i, j), 0 <= i, j <= nroots, given as
 * pairs[2 p] = i, pairs[2 p + 1] = j (host array [npairs][2], no pair twice):
 *  - 1 <= i != j: coupling F_ij; gamma = L_i/(omega_j - omega_i), xi = 0
 *    (Sec. II B); zeta-bar from A^T zeta = -eta_t (eq. amplituderelax) and,
 *    when relaxed, kappa-bar from (A^HF)^T kappa = -eta_kappa (eq.
 *    orbitalrelax);
 *  - j = 0 < i: coupling F_i0 of the excited left state i with the CC ground
 *    state exp(T)|HF> (R0 = 1, R = 0): gamma = 0 and zeta = -L_i/omega_i in
 *    closed form (Sec. II C); only kappa-bar is solved;
 *  - i = 0 < j: coupling F_0j of the ground-state left state
 *    <HF| (1 + Lambda) exp(-T) (eq. nac with i = 0), Lambda from
 *    A^T Lambda = -eta (solved on first use, kept until the next cc_ground);
 *    gamma = Lambda/omega_j, and the reference row of the excited-state
 *    condition (multiplier 1/omega_j) adds d/dt (eta . R_j) / omega_j to
 *    eta_t and its f-derivative to the transition density;
 *  - i = j: gradient of the state energy E_j = E0 + omega_j (E0 for j = 0)
 *    from the same stationarity conditions, with dE0/dt + F(L_j) R_j in
 *    place of eta_t and no overlap term; then densities(j, j) and
 *    nacme(j, j, ...) give dE_j/dlambda^q (branching-plane vectors:
 *    g^q = dE_2^q - dE_1^q, h^q = (E_2 - E_1) F_12^q).
 * The zeta equations of all listed pairs are solved together: blocks of up
 * to 8 right-hand sides share one Galerkin subspace and go through every
 * left Jacobian transform as one batch.
 * Pair (0, 0) needs only cc_ground; every other pair needs both EOM sides.
 * iters: host [npairs][2] or NULL (zeta and kappa-bar iterations per pair).
 * Returns 1 if any solve missed its tolerance (results are the last
 * iterates); -1 for bad or repeated pairs, -2 before the states exist.     */
int multipliers(cc_ctx* ctx, int npairs, const int* pairs, int* iters);

/* Effective densities of the pair (i, j): D_eff (n x n) and the two-electron
 * density d_eff, such that F^q = sum D_eff dh^q + 1/2 sum d_eff dg^q
 * (Sec. II C, eq. NAC_NC_densities).  d_eff is never formed as an n^4
 * tensor: it is kept as occupied/virtual blocks against the density-fitted
 * factor (the adjoints of the places where the integrals enter) on the
 * device for nacme(); D1 (device [n][n], may be NULL) receives D_eff.       */
int densities(cc_ctx* ctx, int i, int j, double* D1);

/* Derivative coupling F_ij^q (or, for i = j, the energy gradient
 * dE_j/dlambda^q) for nq perturbation directions (Sec. II C):
 * dh[nq][n][n] one-electron derivatives, dB[nq][naux][n][n] derivative
 * factors with dg^q_pqrs = sum_P dB[q][P][p][q'] dB[q][P][r][s] (device).
 * F: host [nq].                                                              */
int nacme(cc_ctx* ctx, int i, int j, int nq, const double* dh, const double* dB, double* F);

/* ---- test / benchmark surface ------------------------------------------- */
/* Y = A X (side CC_RIGHT) or Y = X^T A (side CC_LEFT) at the current ground
 * amplitudes; X, Y amplitude-shaped device vectors.                          */
int cc_apply_jacobian(cc_ctx* ctx, int side, const double* X, double* Y);
/* Batched transforms (Sec. II B): Y[z] = A X[z] (CC_RIGHT) or X[z]^T A
 * (CC_LEFT) for k vectors stored [k][N] (N = o v + o^2 v^2, device), all k
 * pushed through each contraction together.  precision CC_FP64,
 * CC_FP32_REFINE or CC_BF16X3_REFINE for the low-precision contractions the
 * mixed-precision solvers use (results then carry that rounding).          */
int cc_apply_jacobian_block(cc_ctx* ctx, int side, int k, const double* X, double* Y,
                            int precision);
/* omega = Omega(t) for amplitudes t (device, amplitude-shaped).              */
int cc_residual(cc_ctx* ctx, const double* t, double* omega);
/* Copies a stored quantity (selectors above) to dst (device; CC_R0 host).
 * idx: state (CC_R, CC_L, CC_R0) or i (pair quantities); jdx: j.            */
int cc_export(cc_ctx* ctx, int what, int idx, int jdx, double* dst);
/* Sets a starting guess: CC_T (amplitudes for the next cc_ground), or CC_R /
 * CC_L with idx = 1..64 (starting vectors of the next right / left EOM
 * solve, e.g. the states of a neighbouring geometry; used once).  Every
 * answer is still judged by the solver's own residual tolerance.            */
int cc_set_guess(cc_ctx* ctx, int what, int idx, const double* src);
/* Counters since cc_create (host out[n], n <= 7): residual evaluations,
 * right transforms, left transforms, algorithmic GEMM flops issued,
 * peak and reserved bytes of the library's device work area, and the part
 * of the GEMM flops issued with fp32 operands.                             */
int cc_stats(const cc_ctx* ctx, double* out, int n);
const char* cc_last_error(const cc_ctx* ctx);
void cc_destroy(cc_ctx* ctx);

/* Engine surface.  C = alpha * einsum(spec)(A, B) + beta * C on device
 * arrays; spec "ab,bc->ac" (lowercase letters, <= 6 per operand, repeated
 * letters inside one operand select a diagonal).  dims* give the shapes.
 * precision: CC_FP64, CC_FP32_REFINE to run the contraction with fp32
 * operands (fp32 accumulation, fp64 result) whatever its size, or
 * CC_BF16X3_REFINE for bfloat16-pair operands (contracted range >= 32).     */
int nm_contract(const char* spec, double alpha, const double* A, const int64_t* dimsA,
                const double* B, const int64_t* dimsB, double beta, double* C,
                const int64_t* dimsC, int precision, void* stream);
/* Kernel surface: one launch of the matrix-core GEMM used by the engine,
 * C[M][N] = alpha op(A) op(B) + beta C (row-major, leading dimensions lda,
 * ldb, ldc; ta / tb select A stored [K][M] / B stored [N][K]).  precision
 * CC_FP64: A, B double; CC_FP32_REFINE: A, B float (fp32 accumulation);
 * CC_BF16X3_REFINE: bfloat16 pairs x = hi + lo (uint16 storage), A [M][lda]
 * and B given transposed (tb = 1) as [N][ldb], hi and lo interleaved in
 * 16-byte chunks: element k of a row has its hi at 2 (k - k % 8) + k % 8 and
 * its lo 8 further; K a multiple of 32, lda / ldb (uint16 units) >= 2 K and
 * multiples of 8, 16-byte aligned; each product formed as three bf16
 * products with fp32 accumulation.
 * Asynchronous on `stream`.                                                 */
int nm_gemm(int precision, int ta, int tb, int M, int N, int K, double alpha, const void* A,
            int64_t lda, const void* B, int64_t ldb, double beta, double* C, int64_t ldc,
            void* stream);
/* As nm_gemm, with the workgroup tile of the bfloat16-pair kernel chosen by
 * `tile` (precision CC_BF16X3_REFINE only): 0 = 128 x 128 outputs per
 * workgroup (two per CU), 1 = 256 x 256, 2 = 256 x 128, 3 = 128 x 256 (one
 * per CU), 4 = 256 x 128 and 5 = 128 x 256 with the global loads issued two
 * K steps ahead, 6 = 256 x 128 and 7 = 128 x 256 with the next K step's
 * fragments read from LDS during this step's products, -1 = the library's
 * model of the fastest shape (what nm_gemm and
 * the contraction engine use before the autotuner has timed a shape).
 * -1 (ARG) for a tile with another precision.                              */
int nm_gemm_tiled(int precision, int tile, int ta, int tb, int M, int N, int K, double alpha,
                  const void* A, int64_t lda, const void* B, int64_t ldb, double beta, double* C,
                  int64_t ldc, void* stream);
/* ---- learned initial guess --------------------------------------------- */
/* A three-layer perceptron y = W3^T s(W2^T s(W1^T x + b1) + b2) + b3 with
 * SiLU s(u) = u / (1 + exp(-u)) and row-major W[in][out], trained on the
 * amplitudes the method itself produces (learned guesses for the solvers).
 * fp32 master parameters updated by Adam (beta 0.9 / 0.999, eps 1e-8); every
 * product uses the bfloat16 rounding of the parameters with fp32
 * accumulation.  Loss: half the mean squared error over all outputs.
 * Parameters are flattened W1, b1, W2, b2, W3, b3.  Arrays X [n][n_in],
 * T and Y [n][n_out] are fp32 DEVICE pointers; parameter and gradient
 * copies are HOST arrays of mlp_num_params floats.  Work runs on the stream
 * given to mlp_create; calls return after it has finished.                  */
typedef struct nm_mlp nm_mlp;
/* N(0, 1/fan_in) weights from `seed`, zero biases.  -1 bad sizes, -4 OOM.  */
int mlp_create(nm_mlp** net, int n_in, int width, int n_out, uint64_t seed, void* stream);
int64_t mlp_num_params(const nm_mlp* net);
int mlp_dims(const nm_mlp* net, int* n_in, int* width, int* n_out);
/* Sets the master parameters (host src), their bfloat16 working copy, and
 * resets the optimiser state.                                              */
int mlp_set_params(nm_mlp* net, const float* src);
/* dst (host) <- master parameters, or their bfloat16 working copy.          */
int mlp_get_params(nm_mlp* net, float* dst, int working);
/* Y = net(X) for n rows.  Networks of width a multiple of 32 up to 256, up
 * to 32 inputs and up to 4 outputs run in one fused kernel on the bf16
 * matrix cores: inputs and hidden activations carried as bfloat16 pairs
 * (about 2^-16 relative), products with the bfloat16 working weights
 * accumulated in fp32, no intermediate rows in device memory.  Other shapes
 * run layer by layer as in training (fp32 activations, FP32 matrix cores).  */
int mlp_forward(nm_mlp* net, int64_t n, const float* X, float* Y);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): Y = net(X)
 * for n rows, as mlp_forward (bit for bit).  Shapes of the fused kernel
 * need no work area; the others keep every intermediate in a fixed 32 MiB
 * device work area of the library instead of buffers it allocates, rows
 * going through it in chunks.  No hipMalloc or hipFree is called.  The area is one
 * per GPU, shared by every call on that GPU: calls that overlap on one GPU
 * (other streams or host threads) race and must be serialised by the
 * caller.  -1 for a network whose rows do not fit 64 at a time.             */
int mlp_forward_noalloc(nm_mlp* net, int64_t n, const float* X, float* Y);
/* Loss of (X, T) over n rows (host *loss) and its gradient with respect to
 * the parameters (kept for mlp_adam_step; copied to host grad if non-NULL). */
int mlp_loss_grad(nm_mlp* net, int64_t n, const float* X, const float* T, double* loss,
                  float* grad);
/* One Adam update with step size lr from the last gradient.                 */
int mlp_adam_step(nm_mlp* net, float lr);
/* `steps` Adam updates on minibatches of `batch` rows drawn uniformly (with
 * replacement, from `seed`) out of the n rows of (X, T); *last_loss: loss
 * of the last minibatch before its update.                                  */
int mlp_train(nm_mlp* net, int64_t n, const float* X, const float* T, int64_t batch, int steps,
              float lr, uint64_t seed, double* last_loss);
const char* mlp_last_error(const nm_mlp* net);
void mlp_destroy(nm_mlp* net);

/* Doubles-amplitude guess from the network.  For every doubles index
 * (i, j, a, b), row-major, the 8 features are e_i, e_j, e_a, e_b,
 * D = e_a + e_b - e_i - e_j, (ia|jb), (ib|ja) and the MP2 amplitude
 * -(ia|jb)/D, each standardised as (f - mu[k]) / sd[k] (mu, sd host [8];
 * NULL = 0 and 1).  The network output z' gives the amplitude
 * t = -((ia|jb) + scale z') / D, so z' = 0 is the MP2 guess the amplitude
 * solver otherwise starts from (Sec. II A).
 * cc_t2_features: F (device fp32 [o^2 v^2][8]).
 * cc_t2_target:   Z (device fp32 [o^2 v^2]) = (-D t - (ia|jb)) / scale from
 *                 the converged ground amplitudes (after cc_ground).
 * cc_guess_t2:    sets the starting amplitudes of the next cc_ground to
 *                 t1 = 0 and the network's doubles (net: n_in 8, n_out 1). */
int cc_t2_features(cc_ctx* ctx, const float* mu, const float* sd, float* F);
int cc_t2_target(cc_ctx* ctx, float scale, float* Z);
int cc_guess_t2(cc_ctx* ctx, nm_mlp* net, const float* mu, const float* sd, float scale);

/* Host-only: eigen-decomposition of a real m x m row-major matrix used for
 * Davidson subspaces; wr, wi [m]; V [m][m] real parts of unit eigenvectors
 * (row k = vector k, phase chosen so its largest component is real).       */
int nm_eig_host(int m, const double* G, double* wr, double* wi, double* V);
/* Library version string. */
const char* nm_version(void);

#ifdef __cplusplus
}
#endif
#endif
