/*
 * rif.h -- C ABI of the RI-PNOF7 hot-path library (librif.so) for MI355X (gfx950).
 *
 * The library implements the per-iteration density-fitted tensor work of
 * PNOF7 with the resolution-of-the-identity (RI) approximation: the AO->MO
 * transforms of the three-index factors b^l_{mu nu} (Eqs. (12)-(13)), the MO
 * Coulomb and exchange matrices J_pq, K_pq (Eqs. (10)-(11), Table 2 step 4),
 * the per-MO AO Coulomb and exchange matrices J^q, K^q (Table 3 steps 3-4),
 * and the PNOF energy (Eq. (2)) with the orbital Lagrangian and gradient
 * needed by the orbital optimisation (Sec. II, "Orbital Optimization with RI").
 *
 * Conventions shared by every entry point
 *   - Arrays are row-major (C order).  Index names: l = auxiliary function
 *     (n_aux), mu/nu = AO (n_bf), p/q/r = orbital of the pairing scheme Omega
 *     (n_omega), a = any MO (n_mo).  Omega is the first n_omega columns of C.
 *   - Every array argument is a DEVICE pointer owned by the caller.  The
 *     library never frees caller memory; its own scratch lives in the context.
 *   - Calls are asynchronous on the context's stream; the caller synchronises
 *     (rif_sync or its own stream sync) before reading results on the host.
 *   - Errors are returned as status codes; nothing aborts and no exception
 *     crosses the ABI.  rif_last_error() returns the message of the last
 *     failing call on that context.  Shape and pointer checks happen on the
 *     host before any launch; checks that need device data (occupation
 *     numbers) run on the device and are reported by the next rif_sync().
 *   - One context per host thread.  b is assumed symmetric in (mu, nu) for
 *     every l (Eq. (9) produces such a factor); this is not checked.
 *   - Precision: RIF_FP64 computes everything in FP64.  The other modes run the
 *     GEMM-shaped contractions on lower-precision MFMA (FP32, or BF16/FP16
 *     pieces split from the FP64 operands) with FP32 accumulation recombined
 *     in FP64; J_pq/K_pq sums over l, the energy, the Lagrangian and its
 *     antisymmetrisation stay FP64.  In those modes b_half, b_mo, Jn and Kn
 *     are FP32 arrays (4 bytes per element) instead of FP64.
 */
#ifndef RIF_H
#define RIF_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rif_ctx rif_ctx;

/* Under C++ the enums below take int as their underlying type, so every int
 * a caller passes (from C, or through a foreign-function layer) is a valid
 * value of the type; the calls reject the values they do not know. */
#ifdef __cplusplus
#define RIF_ENUM enum : int
#else
#define RIF_ENUM enum
#endif

typedef RIF_ENUM {
  RIF_OK = 0,
  RIF_EINVAL = -1,  /* bad shape, NULL pointer, invalid occupations */
  RIF_ENOMEM = -2,  /* workspace allocation failed or exceeds the cap */
  RIF_EHIP = -3,    /* a HIP runtime call or kernel launch failed */
  RIF_ENOTSUP = -4  /* precision or feature not available */
} rif_status;

typedef RIF_ENUM {
  RIF_FP64 = 0,
  RIF_FP32 = 1,
  RIF_BF16X3 = 2,   /* two bf16 pieces, three products */
  RIF_BF16X6 = 3,   /* three bf16 pieces, six products */
  RIF_FP16X3 = 4    /* fp16 high piece + fp16 low piece scaled by 2^11, three
                       products (hi.hi + 2^-11 (hi.lo + lo.hi)); every operand of
                       the split GEMMs, intermediates included, must stay below
                       65504 in magnitude, else the outputs it reaches are not
                       finite. */
} rif_prec;

typedef RIF_ENUM { RIF_PNOF7 = 0, RIF_PNOF5 = 1 } rif_functional;

/* Create a context on HIP device `hip_device`.  `hip_stream` is a hipStream_t
 * to launch on (e.g. the caller's current stream); NULL makes the context
 * create and own a default-priority stream.  Returns RIF_EINVAL for a bad
 * device, RIF_EHIP if the runtime fails. */
rif_status rif_create(rif_ctx **out, int hip_device, void *hip_stream);
void rif_destroy(rif_ctx *ctx);
/* Message of the last failing call ("" if none).  Owned by the context. */
const char *rif_last_error(const rif_ctx *ctx);
/* Replace the stream later calls launch on (NULL = the context's own). */
rif_status rif_set_stream(rif_ctx *ctx, void *hip_stream);
/* Wait for the context's stream, then report any deferred device-side
 * validation error (RIF_EINVAL with a message) and clear it: occupations out
 * of range or not summing to 1 per pair, a bad pair map, or a build whose
 * energy or gradient came out non-finite (NaN/inf inputs, or in RIF_FP16X3 an
 * operand of a split product of magnitude 65504 or more, past fp16's range). */
rif_status rif_sync(rif_ctx *ctx);
/* Cap on the context's workspace in bytes (0 = no cap).  A call that would
 * need more returns RIF_ENOMEM. */
rif_status rif_set_workspace_limit(rif_ctx *ctx, unsigned long long bytes);

/* Half- and full-MO transforms: Eqs. (12)-(13); Table 2 steps 2-3 and
 * Table 3 steps 2-3 (Coulomb branch).
 *   b      [n_aux][n_bf][n_bf]  FP64, each slab symmetric          (in)
 *   C      [n_bf][n_mo]         FP64 MO coefficients              (in)
 *   b_half [n_omega][n_aux][n_bf]  b^l_{q nu} = sum_mu C_{mu q} b^l_{mu nu}   (out)
 *   b_mo   [n_aux][n_omega][n_omega] b^l_{pq} = sum_nu C_{nu q} b^l_{p nu}   (out)
 *   d      [n_aux][n_omega]     FP64 diagonal d[l][q] = b^l_{qq}   (out)
 * b_half and b_mo are FP64 for RIF_FP64, FP32 otherwise.
 * Requires 0 < n_omega <= n_mo <= n_bf, n_aux > 0. */
rif_status rif_transform(rif_ctx *ctx, int n_bf, int n_aux, int n_omega, int n_mo,
                         const double *b, const double *C, rif_prec prec,
                         void *b_half, void *b_mo, double *d);

/* MO Coulomb and exchange matrices: Eqs. (10)-(11); Table 2 step 4.
 *   b_mo [n_aux][n_omega][n_omega] (FP64 or FP32 as produced by rif_transform)
 *   d    [n_aux][n_omega] FP64
 *   J, K [n_omega][n_omega] FP64:  J_pq = sum_l d[l][p] d[l][q],  K_pq = sum_l (b^l_pq)^2
 * The sums over l are FP64 in every mode and deterministic (fixed order). */
rif_status rif_jk_mo(rif_ctx *ctx, int n_aux, int n_omega, const void *b_mo, const double *d,
                     rif_prec prec, double *J, double *K);

/* rif_jk_mo for callers that cannot allocate (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the same arguments, kernels
 * and results (bitwise), with the per-slice partials in a static device array
 * of 16 MiB per GPU instead of the context's workspace, which this call never
 * grows.  No hipMalloc, hipFree or other allocation happens in the call.  That
 * array holds 2 * s * n_omega^2 doubles, s = the slices of l (1 for
 * n_omega >= 64): RIF_ENOMEM beyond it (n_omega above 1024).  Every context
 * on one GPU shares that GPU's array, so two such calls that overlap on one
 * GPU (on different streams) race; calls on one stream are ordered.  Event
 * profiling (rif_profile_enable) is suspended during the call.  RIF_EHIP if
 * the array's device address could not be resolved at rif_create. */
rif_status rif_jk_mo_noalloc(rif_ctx *ctx, int n_aux, int n_omega, const void *b_mo, const double *d,
                             rif_prec prec, double *J, double *K);

/* Per-MO AO Coulomb and exchange matrices: Table 3 steps 3-4.
 *   b      [n_aux][n_bf][n_bf] FP64          (in)
 *   b_half [n_omega][n_aux][n_bf]            (in, as produced by rif_transform)
 *   d      [n_aux][n_omega] FP64             (in)
 *   Jn     [n_omega][n_bf][n_bf]  J^q_{mu nu} = sum_l b^l_qq b^l_{mu nu}      (out)
 *   Kn     [n_omega][n_bf][n_bf]  K^q_{mu nu} = sum_l b^l_{q mu} b^l_{q nu}   (out)
 * Jn and Kn are written in full and are exactly symmetric; FP64 for RIF_FP64,
 * FP32 otherwise. */
rif_status rif_jk_ao_per_mo(rif_ctx *ctx, int n_bf, int n_aux, int n_omega,
                            const double *b, const void *b_half, const double *d,
                            rif_prec prec, void *Jn, void *Kn);

/* PNOF energy (Eq. (2) with L = K) and orbital Lagrangian / gradient.
 *   pair_of [n_omega] int32 pair index of each orbital of Omega; orbital g
 *           (g < n_pairs) must be the strong orbital of pair g and each pair
 *           must hold exactly 1 + n_cwo orbitals.  NULL selects the default
 *           map: weak orbitals of pair g are n_pairs + n_cwo*(n_pairs-1-g) + k.
 *   H  [n_bf][n_bf] FP64 core Hamiltonian; C [n_bf][n_mo]; occ [n_omega] FP64 ONs
 *   J, K [n_omega][n_omega] FP64 (from rif_jk_mo); Jn, Kn from rif_jk_ao_per_mo
 *   energy  device FP64 scalar: 2 sum_p n_p H_pp + sum_pq (A_pq J_pq + B_pq K_pq)
 *   lambda  [n_mo][n_omega] FP64: lambda_aq = c_a^T F^(q) c_q with
 *           F^(q) = n_q H + sum_r (A_qr J^r + B_qr K^r)
 *   grad    [n_mo][n_mo] FP64: G = 4 (lambda - lambda^T), lambda zero-padded
 *           to n_mo columns; G_ab = dE/dtheta along C -> C exp(theta (E_ab - E_ba)).
 * A and B follow from the functional's Delta and Pi: within a pair A = 0 and
 * B = Pi (Pi_pp = n_p, +sqrt(n_p n_q) for two weak orbitals, -sqrt(n_p n_q)
 * with the strong one); between pairs A = 2 n_p n_q and
 * B = -n_p n_q - Phi_p Phi_q, Phi_p = sqrt(n_p (1 - n_p)) (PNOF7; PNOF5 has no
 * Phi term).  Host-side checks: n_omega = n_pairs (1 + n_cwo) <= n_mo <= n_bf.
 * Device-side checks (reported by rif_sync): 0 <= n_p <= 1, per-pair sums
 * within 1e-12 of 1, a valid pair map. */
rif_status pnof7_energy_grad(rif_ctx *ctx, int n_bf, int n_mo, int n_pairs, int n_cwo,
                             const int *pair_of, const double *H, const double *C,
                             const double *occ, const double *J, const double *K,
                             const void *Jn, const void *Kn, rif_prec prec,
                             double *energy, double *lambda, double *grad);

/* Same as pnof7_energy_grad with an explicit functional (RIF_PNOF7 or RIF_PNOF5). */
rif_status pnof_energy_grad(rif_ctx *ctx, rif_functional functional, int n_bf, int n_mo,
                            int n_pairs, int n_cwo, const int *pair_of, const double *H,
                            const double *C, const double *occ, const double *J,
                            const double *K, const void *Jn, const void *Kn, rif_prec prec,
                            double *energy, double *lambda, double *grad);

/* One molecule's inputs and outputs for rif_build / rif_batch_create.  Every
 * pointer is a device pointer owned by the caller, with the layouts and
 * element types of the four calls above (b_half, b_mo, Jn, Kn: double for
 * RIF_FP64, float otherwise); pair_of may be NULL (default map).
 * b_split: NULL, or b already split for the precision the build runs in
 * (rif_presplit_b with that precision); the half transform then reads it in
 * place of b.  Ignored for RIF_FP64. */
typedef struct rif_instance {
  int n_bf, n_aux, n_pairs, n_cwo, n_mo;
  const double *b, *C, *H, *occ;
  const int *pair_of;
  void *b_half, *b_mo;
  double *d, *J, *K;
  void *Jn, *Kn;
  double *energy, *lambda, *grad;
  const void *b_split;
} rif_instance;

/* The conventional four-centre path that the RI path replaces (Table 1,
 * Eqs. (3)-(5)), FP64 only, to compare the two on the same integrals.
 *
 * Step 0: rif_eri4_from_b forms (mu nu|sigma lambda) = sum_l b^l_{mu nu}
 * b^l_{sigma lambda} (the integrals the factors b of Eq. (9) fit, Eq. (6)) and
 * stores them with the first pair packed:
 *   eri [n_bf(n_bf+1)/2][n_bf][n_bf],  eri[(mu nu)][sigma][lambda] for mu <= nu,
 *   (mu nu) = mu*n_bf - mu*(mu-1)/2 + (nu - mu)  (row-major upper triangle).
 * rif_eri4_bytes gives its size (host function; 0 for bad sizes).  The call
 * also takes n_aux * n_bf(n_bf+1)/2 doubles of workspace (b packed).
 *
 * Steps 1-3: rif_jk_4c, with P^q = c_q c_q^T (Eq. (4)),
 *   Jn [n_omega][n_bf][n_bf]  J^q_{mu nu}    = sum P^q_{sigma lambda} (mu nu|sigma lambda)
 *   Kn [n_omega][n_bf][n_bf]  K^q_{mu sigma} = sum P^q_{nu lambda} (mu nu|sigma lambda)
 *   J, K [n_omega][n_omega]   J_pq = sum P^p_{mu nu} J^q_{mu nu}  (Eq. (3)),
 *                             K_pq = sum P^p_{mu sigma} K^q_{mu sigma}  (Eq. (5))
 * C [n_bf][n_mo]: Omega is its first n_omega columns.  Jn and Kn are written in
 * full and exactly symmetric.  Workspace: n_omega * n_bf^2 (n_bf+1)/2 doubles
 * (the integrals contracted with C over one index).  Device pointers owned by
 * the caller; asynchronous on the context's stream.  RIF_EINVAL unless
 * 0 < n_omega <= n_mo <= n_bf <= 2048, or for NULL pointers; RIF_ENOMEM if the
 * workspace cannot be had. */
unsigned long long rif_eri4_bytes(int n_bf);
rif_status rif_eri4_from_b(rif_ctx *ctx, int n_bf, int n_aux, const double *b, double *eri);
rif_status rif_jk_4c(rif_ctx *ctx, int n_bf, int n_omega, int n_mo, const double *eri, const double *C,
                     double *Jn, double *Kn, double *J, double *K);

/* b stored once for a reduced-precision mode (Sec. III: b is computed once
 * and kept in memory).  RIF_FP32: a float copy in b's layout.  RIF_BF16X3 /
 * RIF_BF16X6: P = 2 / 3 bf16 piece planes; RIF_FP16X3: P = 2 fp16 planes, hi
 * and lo * 2^11 (each the same split arithmetic as the kernels' staging), in
 * two regions of out (16-bit elements):
 *   - for the half transform: plane s at out + s * n_aux * n_bf * ld with ld =
 *     n_bf rounded up to a multiple of 32; element (l*n_bf + nu, mu) of a plane
 *     holds piece s of b[l][nu][mu] (b symmetric in mu, nu), zero from mu =
 *     n_bf up to ld;
 *   - for J^q (Table 3 step 4), after the first region (at out + P * n_aux *
 *     n_bf * ld): plane s at + s * n_bf^2 * lj with lj = n_aux rounded up to a
 *     multiple of 32; element (mu*n_bf + nu, l) holds piece s of b[l][mu][nu],
 *     zero from l = n_aux up to lj.
 * rif_presplit_b_bytes gives the size of out (host function, no GPU call; 0
 * for RIF_FP64 or bad sizes).  Asynchronous.  RIF_EINVAL for sizes or NULL
 * pointers, RIF_ENOTSUP for RIF_FP64. */
unsigned long long rif_presplit_b_bytes(int n_bf, int n_aux, rif_prec prec);
rif_status rif_presplit_b(rif_ctx *ctx, int n_bf, int n_aux, const double *b, rif_prec prec, void *out);

/* One build: rif_transform, rif_jk_mo, rif_jk_ao_per_mo and pnof_energy_grad
 * in sequence for one molecule (same checks and errors as those calls). */
rif_status rif_build(rif_ctx *ctx, const rif_instance *inst, rif_prec prec, rif_functional functional);

/* The energy, lambda and G of rif_build without forming the per-MO AO
 * matrices J^q, K^q (inst->Jn, inst->Kn are not used and may be NULL).  Since
 * b is symmetric, J^(r) c_q = sum_l d_lr b_half[q][l] and
 * K^(r) c_q = sum_l b_mo[l][r][q] b_half[r][l], so F^(q) c_q (Sec. II, the
 * orbital gradient) becomes one contraction over (r, l) of b_half with
 * coefficients B_qr b_mo[l][r][q], plus sum_l a_lq b_half[q][l] with
 * a_lq = sum_r A_qr d_lr on its r = q terms: 2 n_aux n_omega^2 n_bf flops in
 * place of the J^q/K^q build and the F^(q) c_q products.  b_half, b_mo, d,
 * J, K are written as by rif_build.  Same checks and errors as rif_build,
 * and RIF_EINVAL unless n_aux * n_omega < 2^31. */
rif_status rif_build_direct(rif_ctx *ctx, const rif_instance *inst, rif_prec prec, rif_functional functional);

/* Batched builds of many molecules of uneven size.  rif_batch_create checks
 * every instance (as rif_build would), orders them largest first, allocates
 * the batch's own workspace and uploads a work-list per step; it chooses
 * each step's tile variant for the batch as a whole (timing the candidates if
 * autotuning is on).  rif_batch_run enqueues one persistent grouped launch per
 * step covering all molecules; with use_graph != 0 the first run captures the
 * sequence in a hipGraph on the context's stream and every run replays it.
 * The instance pointers are baked into the plan: keep them valid and
 * unchanged while the batch lives.  Results for each molecule equal
 * rif_build's with the same tile variants.  `inst` is a HOST array of n_inst
 * structs (copied). */
typedef struct rif_batch rif_batch;
rif_status rif_batch_create(rif_ctx *ctx, int n_inst, const rif_instance *inst, rif_prec prec,
                            rif_functional functional, rif_batch **out);
rif_status rif_batch_run(rif_batch *batch, int use_graph);
void rif_batch_destroy(rif_batch *batch);

/* ---- Occupation-number (ON) optimisation and its learned warm start ----
 * The occupancy optimisation of Sec. II: minimise Eq. (2) over the ONs at
 * fixed H_pp, J, K through auxiliary variables gamma (unconstrained):
 *   n_g = (1 + cos^2 gamma_g)/2 for the strong orbital of pair g; the weak
 *   orbitals of g (ascending index) get (1 - n_g) w_k with hyperspherical
 *   weights w_1 = cos^2 b_1, w_k = prod_{j<k} sin^2 b_j cos^2 b_k,
 *   w_last = prod sin^2 b_j; variables [gamma_g, b_1..b_{ncwo-1}] at g*ncwo+j.
 * One problem per molecule; all pointers are device pointers.
 *   Hpp [n_omega], J, K [n_omega][n_omega] FP64 (from rif_hpp / rif_jk_mo)
 *   gamma [n_pairs*n_cwo] in: start, out: optimum; occ [n_omega] out
 *   energy, iters, status: out (status 0 converged to max|dE/dgamma| <= tol,
 *   1 max_it reached, 2 line search failed, 3 bad pair map)
 *   work: rif_on_work_size(...) doubles of scratch owned by the caller
 *   row0: first row of this problem in the per-pair feature/prediction arrays */
typedef struct rif_on_problem {
  int n_pairs, n_cwo, n_omega, functional, max_it, row0;
  double tol;
  const double *Hpp, *J, *K;
  const int *pair_of;
  double *gamma, *occ, *energy;
  int *iters, *status;
  double *work;
} rif_on_problem;

/* Scratch doubles one problem needs (host function, no GPU call). */
long rif_on_work_size(int n_omega, int n_pairs, int n_cwo);
/* H_pp = c_p^T H c_p for the n_omega orbitals of Omega (Eq. (1)). */
rif_status rif_hpp(rif_ctx *ctx, int n_bf, int n_mo, int n_omega, const double *H, const double *C,
                   double *Hpp);
/* L-BFGS (history 8; backtracking with the Armijo test, or the approximate
 * Wolfe conditions once energy changes are below rounding noise) in FP64, one
 * workgroup per problem, all problems in one launch.  probs is a HOST array
 * (copied). */
rif_status rif_on_optimize(rif_ctx *ctx, int n_prob, const rif_on_problem *probs);
/* Per-pair MLP features X [rows][39] (optionally standardised: (x - mu)/sigma
 * where sigma > 0), and, if T/M are non-NULL, targets T [rows][7] = the
 * pair's ONs from occ (strong, then weak slots) and masks M [rows][7].
 * Rows: problem i owns rows row0 .. row0 + n_pairs - 1. */
rif_status rif_on_features(rif_ctx *ctx, int n_prob, const rif_on_problem *probs, float *X, float *T,
                           float *M, const float *mu, const float *sigma);
/* Predicted pair ONs P [rows][7] -> starting gamma of every problem. */
rif_status rif_on_warmstart(rif_ctx *ctx, int n_prob, const rif_on_problem *probs, const float *P);

/* Warm-start MLP: 39 -> 128 -> 128 -> 128 -> 7, tanh hidden layers, masked
 * softmax output (FP32).  Parameters: one flat FP32 vector of
 * rif_mlp_n_params() values, layer l stored as W_aug = [W (in x out); b (out)]
 * row-major.  Buffers owned by the caller:
 *   X [rows][39], M [rows][7] masks, T [rows][7] targets,
 *   H [3][rows][128] hidden activations, Z [rows][7] logits, P [rows][7] ONs,
 *   dA [2][rows][128] scratch, grad [n_params], loss: device double (mean
 *   over rows of sum_k M (P - T)^2). */
long rif_mlp_n_params(void);
rif_status rif_mlp_forward(rif_ctx *ctx, int rows, const float *X, const float *M, const float *theta,
                           float *H, float *Z, float *P);
rif_status rif_mlp_backward(rif_ctx *ctx, int rows, const float *X, const float *M, const float *T,
                            const float *theta, const float *H, const float *Z, float *dA, float *grad,
                            double *loss);
/* Adam with bias correction; step counts from 1. */
rif_status rif_adam(rif_ctx *ctx, int n, float *theta, const float *grad, float *m, float *v, int step,
                    float lr, float beta1, float beta2, float eps);

/* b from the three-centre integrals and the metric (Sec. II, RI), done once
 * per molecule: the metric G_kl = (k|l) is factorised as G = P L D L^T P^T
 * (L unit lower triangular, D block diagonal with 1x1 and 2x2 blocks,
 * Bunch-Kaufman partial pivoting with alpha = (1 + sqrt 17)/8), the
 * eigenvalues of each D block below delta are raised to delta (D~), and
 *   P L D~^(1/2) b^T = T,  T[k][mu nu] = (mu nu|k),
 * is solved: b^T = D~^(-1/2) L^-1 P^T T.  Then sum_k b^k b^k = T^T G~^-1 T with
 * G~ = P L D~ L^T P^T (= G if nothing was raised).  Device pointers:
 *   T [n_aux][n_bf][n_bf] (symmetric in mu, nu: only nu >= mu is read),
 *   G [n_aux][n_aux] symmetric
 *   b [n_aux][n_bf][n_bf] out, exactly symmetric in mu, nu (the solve runs on
 *   the packed upper triangles; b's buffer also stages them)
 *   optional (NULL to skip): perm [n_aux] (P^T x)[i] = x[perm[i]]; L and D
 *   [n_aux][n_aux] dense; n_raised: number of raised eigenvalues
 * delta <= 0 takes 2^-26 * max_k sum_l |G_kl|.  The factorisation runs as
 * one cooperative launch where the metric's rows fit the LDS of at most 256
 * workgroups (n_aux up to about 1600; its waits are bounded by
 * rif_set_wait_limit, and a timed-out one leaves b all NaN), else as a pivot
 * and an update launch per column.  Uses 6 n_aux^2 + n_aux n_bf (n_bf + 1) / 2
 * doubles of the context arena, plus 5 n_aux^2 for the one-launch
 * factorisation's exchange slots.  Asynchronous.  RIF_EINVAL for sizes
 * (n_aux < 46341) or NULL T, G, b. */
rif_status rif_prepare_b(rif_ctx *ctx, int n_bf, int n_aux, const double *T, const double *G, double delta,
                         double *b, int *perm, double *L, double *D, int *n_raised);

/* ---- Orbital optimisation and the outer/inner loop ----
 * Sec. II, orbital optimisation with RI: at fixed ONs the natural orbitals are
 * found by repeated diagonalisation of a symmetric matrix F^lambda built from
 * the Lagrange multipliers, so orthonormality holds at every step; Fig. 1
 * alternates this (inner iterations) with the ON optimisation (outer).
 * F^lambda is not printed in the paper; the reading implemented here: off the
 * diagonal F_pq = lambda_{hi,lo} - lambda_{lo,hi} with hi = max(p,q),
 * lo = min(p,q) and lambda_ab = 0 for b outside Omega (F vanishes off the
 * diagonal exactly when the orbital gradient does); the diagonal is lambda_pp
 * at the first step of an inner loop and the previous step's eigenvalues
 * after that (aufbau order: eigenvectors by ascending eigenvalue, an
 * orbital's role -- strong, weak of a pair, or outside Omega -- by index).
 *
 * rif_orbital_step: one diagonalisation.  Device pointers:
 *   lambda  [n_mo][n_omega] FP64 (rif_build's lambda)
 *   eps_in  [n_mo] diagonal of F^lambda, or NULL for lambda_pp
 *   C       [n_bf][n_mo] in/out: replaced by C V, V the eigenvectors
 *   eps_out [n_mo] eigenvalues, ascending (may be eps_in)
 *   info    device int or NULL: 0; > 0 the tridiagonal eigensolver did not
 *           converge (rocSOLVER's failure count, or 1 from the library's own
 *           divide and conquer, which also reports a non-finite F that way);
 *           -1 a timed-out wait of the one-launch reduction
 *           (rif_set_wait_limit)
 * The eigen-decomposition runs on the context's stream with its workspace in
 * the context arena (solver chosen by rif_set_eigensolver); the rotation is an
 * FP64 MFMA GEMM.  info = -1 reports a timed-out wait inside the tridiagonal
 * reduction (the result is then invalid).  Asynchronous.  RIF_EINVAL: need
 * 0 < n_omega <= n_mo <= n_bf, non-NULL lambda, C and eps_out. */
rif_status rif_orbital_step(rif_ctx *ctx, int n_bf, int n_mo, int n_omega, const double *lambda,
                            const double *eps_in, double *C, double *eps_out, int *info);

/* Eigensolver of the orbital step (and of rif_pnof_optimize), per context:
 *   RIF_EIG_DC     Householder reduction to tridiagonal form T = Q^T F Q in ONE
 *                  cooperative launch (rows of F and of Q held in LDS across
 *                  `groups` workgroups, which exchange v and p of each column
 *                  through polled single-write slots), then the library's own
 *                  divide and conquer on T (Cuppen's tearing down to leaves of
 *                  at most 32 rows solved by implicit QR, rank-one merges with
 *                  the secular roots found by bisection and Gu and Eisenstat's
 *                  recomputed update vector, each merge's eigenvector product
 *                  an FP64 MFMA GEMM), and C <- (C Q) Z as two FP64 MFMA GEMMs.
 *                  Needs the rows of F and Q to fit 150 KB of LDS per
 *                  workgroup with at most 256 workgroups, one per CU (n_mo up
 *                  to about 1200); the orbital step returns RIF_ENOTSUP
 *                  otherwise.
 *   RIF_EIG_TRD    the same reduction, then rocSOLVER dstedc on T.
 *   RIF_EIG_SYEVD  rocSOLVER dsyevd (its own blocked reduction).
 *   RIF_EIG_AUTO   DC where it fits, else SYEVD (the default).
 * groups: workgroups of the reduction, 0 for the default (four rows each, one
 * per wave, at least 16 workgroups, more where the rows do not fit).  Results
 * of the solvers agree to rounding,
 * eigenvectors up to sign.  RIF_EINVAL for an unknown kind or groups outside
 * [0, 4096]. */
typedef RIF_ENUM { RIF_EIG_AUTO = 0, RIF_EIG_SYEVD = 1, RIF_EIG_TRD = 2, RIF_EIG_DC = 3 } rif_eigensolver;
rif_status rif_set_eigensolver(rif_ctx *ctx, int kind, int groups);

/* Bound on the waits inside the one-launch kernels (the tridiagonal reduction
 * of rif_orbital_step, the factorisation of rif_prepare_b): the number of
 * polls of one exchanged value before the kernel gives up (default 2^22,
 * seconds).  Workgroups exchange values through slots that each consumer
 * polls; a wait past the bound makes every workgroup return, and the call
 * reports it: rif_orbital_step sets info = -1 (rif_pnof_optimize then fails
 * with RIF_EHIP, status 2); rif_prepare_b leaves every element of b NaN.
 * Negative: every such wait gives up at once (to exercise those paths).
 * Per context; takes effect on the next call. */
rif_status rif_set_wait_limit(rif_ctx *ctx, long long polls);

/* Fig. 1 loop.  Each outer iteration: J, K (MO) and H_pp at the current
 * orbitals, then the ON optimisation (rif_on_optimize's L-BFGS, from the
 * current gamma); then inner iterations at the new ONs, each one build
 * (rif_build) followed, unless max|G| <= tol_grad, by one rif_orbital_step.
 * Converged when an outer iteration after the first ends with a converged
 * inner loop and an energy within tol_energy of the previous one.
 *   init_gamma 0: the first ON step starts from the ONs in occ (mapped to
 *   gamma through the warm-start map, in FP32); 1: from gamma as given. */
typedef struct rif_opt_params {
  int max_outer, max_inner, on_max_it, init_gamma;
  double tol_grad, tol_energy, on_tol;
} rif_opt_params;
/* status 0 converged, 1 iteration limit, 2 eigensolver failure (also an
 * RIF_EHIP return), 3 non-finite energy or gradient.  Times are HIP-event
 * milliseconds of the ON steps (J/K, H_pp, L-BFGS), the builds (with max|G|)
 * and the orbital steps. */
typedef struct rif_opt_result {
  int outer, inner_total, on_iters_total, on_status, status;
  double energy, max_grad, ms_on, ms_build, ms_orbital;
} rif_opt_result;
/* inst: buffers and inputs as for rif_build; inst->C and inst->occ are
 * ignored and C, occ used instead.  With inst->Jn or inst->Kn NULL the inner
 * builds are rif_build_direct's (no per-MO AO matrices), else rif_build's.
 * Device pointers: C [n_bf][n_mo] in/out,
 * occ [n_omega] in/out, gamma [n_pairs*n_cwo] in/out.  Host pointers: res,
 * and optionally hist_energy / hist_grad, which receive the energy and
 * max|G| of each inner iteration (first hist_len of them).  Blocks until the
 * loop ends (one stream synchronisation per inner iteration). */
rif_status rif_pnof_optimize(rif_ctx *ctx, const rif_instance *inst, rif_prec prec, rif_functional functional,
                             const rif_opt_params *par, double *C, double *occ, double *gamma,
                             rif_opt_result *res, double *hist_energy, double *hist_grad, int hist_len);

/* Tile-shape selection for the MFMA kernels.  Each GEMM-shaped kernel has up
 * to four tile variants (0: 128x128, 1: 64x64, 2: 128x64, 3: 64x128 outputs
 * per workgroup).  mode 0 picks one per shape with a wave-quantisation
 * model; mode 1 (autotune) times every variant on the first call with a new
 * shape -- synchronising the stream once -- and reuses the fastest for that
 * shape afterwards.  Results are identical to FP64 rounding across variants. */
rif_status rif_autotune(rif_ctx *ctx, int mode);
/* Force variant v (0..3, clamped to what each kernel has) for every kernel;
 * -1 returns to automatic selection. */
rif_status rif_set_tile_variant(rif_ctx *ctx, int v);
/* "kernel shape... -> variant | ms per variant" lines for every tuned shape. */
rif_status rif_tune_report(rif_ctx *ctx, char *buf, int len);
/* Tile choices from text in rif_tune_report's format (one line per tuned
 * shape; blank lines ignored), so that a process can start from choices
 * measured earlier: under autotuning (mode 1) a later call with a loaded
 * shape takes the loaded variant without timing (a variant the kernel does
 * not have is ignored and that shape is timed as usual).  A loaded line
 * replaces the context's entry for the same shape.  Host-only, no GPU work.
 * RIF_EINVAL for NULL text or a line that does not parse (nothing is loaded
 * then; the message names the line). */
rif_status rif_tune_load(rif_ctx *ctx, const char *text);

/* Per-kernel timing with HIP events on the context's stream.
 * rif_profile_enable(ctx, 1) starts recording an event pair around every
 * kernel launch; rif_profile_report synchronises, folds the pairs into
 * per-kernel totals and writes "name launches total_ms\n" lines into buf
 * (truncated to len bytes, NUL-terminated).  Enabling again clears totals. */
rif_status rif_profile_enable(rif_ctx *ctx, int on);
rif_status rif_profile_report(rif_ctx *ctx, char *buf, int len);
/* Restrict recording to launches whose report name equals name (a copy is
 * kept); NULL or "" records every launch again.  With one kernel selected the
 * recording adds two event records per launch of that kernel and nothing
 * elsewhere, so a timed loop can carry it.  Takes effect for launches issued
 * after the call; unknown names simply record nothing. */
rif_status rif_profile_only(rif_ctx *ctx, const char *name);

#ifdef __cplusplus
}
#endif
#endif /* RIF_H */
