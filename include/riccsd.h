/*
 * riccsd.h -- C ABI of the closed-shell RI-CCSD library for MI355X (gfx950).
 *
 * Conventions shared by every entry point
 *  - Array arguments are DEVICE pointers owned by the caller (for example the
 *    data pointer of a device tensor); the library never frees caller memory.
 *    Arrays are C-contiguous (row-major) and FP64 unless stated otherwise.
 *  - `stream` is a hipStream_t passed as void* (NULL: the legacy default stream).
 *    Calls enqueue work on it and return without synchronising, except where a
 *    host-side scalar result is documented (those synchronise `stream`).
 *  - Index conventions: MOs occupied first; B[Q][p][q] are the RI factors of
 *    the MO integrals, (pq|rs) = sum_Q B^Q_pq B^Q_rs (eq. RIM), and
 *    v^{pq}_{rs} = (pr|qs) (eq. eri).  t1[i][a] = t^a_i, t2[i][j][a][b] = t^{ab}_{ij}.
 *  - Every call returns a status (RI_OK on success).  On failure nothing is
 *    enqueued unless the status is RI_E_HIP; ri_last_error_msg() describes the
 *    failure of the calling thread's most recent call.  No exception crosses
 *    the ABI and the library never aborts the process.
 */
#ifndef RICCSD_H
#define RICCSD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define RI_OK 0
#define RI_E_ARG 1         /* null pointer, non-positive size, overflow, bad enum */
#define RI_E_ALIAS 2       /* an output overlaps an input */
#define RI_E_NOMEM 3       /* device workspace allocation failed or workspace too small */
#define RI_E_HIP 4         /* HIP runtime or launch error (see ri_last_hip_error) */
#define RI_E_NOCONV 5      /* iteration limit reached; amplitudes are valid */
#define RI_E_NUMERIC 6     /* NaN/Inf or divergence detected */
#define RI_E_UNSUPPORTED 7 /* precision or device not supported */

/* ladder arithmetic */
#define RI_PREC_FP64 0     /* FP64 MFMA throughout */
#define RI_PREC_FP32 1     /* operands rounded to FP32, FP32 MFMA, FP32 accumulation */
#define RI_PREC_BF16X3 2   /* bf16 hi+lo split, three products, FP32 accumulation */

const char* ri_status_str(int status);
/* Message describing the calling thread's most recent failure ("" if none). */
const char* ri_last_error_msg(void);
/* hipError_t value of the calling thread's most recent RI_E_HIP failure. */
int ri_last_hip_error(void);

/*
 * Particle-particle ladder (Sec. II.C, eq. pp-Ladder-0):
 *
 *     R[i][j][a][b] += sum_{c,d} (ac|bd) tau[i][j][c][d],
 *     (ac|bd)        = sum_Q B_vv[Q][a][c] B_vv[Q][b][d].
 *
 * B_vv : [naux][v][v]; the first virtual index is the external one (it matters
 *        when the factors are t1-dressed and therefore not symmetric).
 * tau  : [o][o][v][v], tau[i][j][c][d] = tau^{cd}_{ij} (eq. pp-Ladder-01).  The
 *        result is exact for the pair-symmetric part
 *        (tau[i][j][c][d] + tau[j][i][d][c]) / 2, which is tau itself for CCSD
 *        amplitudes (Sec. II.C); R therefore always satisfies
 *        R^{ab}_{ij} = R^{ba}_{ji} for the added part.
 * R    : [o][o][v][v], accumulated; must not overlap B_vv or tau (RI_E_ALIAS).
 * The v^4 integral tensor is never stored: it is rebuilt tile by tile from B_vv
 * and contracted with symmetric/antisymmetric packed tau (Scuseria's split,
 * Sec. II.C).  Workspace is allocated stream-ordered on `stream` and released
 * before the call returns control of it to the stream.  Deterministic: the same
 * inputs give bitwise the same R.
 * Debug check: with the environment variable RI_PPL_CHECK_TAU set (to anything but
 * "0") the ladder calls first measure tau with ri_tau_pair_asymmetry (synchronising
 * the stream) and return RI_E_ARG, leaving R untouched, unless
 * max |tau^{cd}_{ij} - tau^{dc}_{ji}| <= 1e-12 max |tau|.
 */
int ri_ppl(const double* B_vv, const double* tau, int o, int v, int naux, double* R,
           void* stream);

/* As ri_ppl with a choice of arithmetic (RI_PREC_*) and an optional caller
 * workspace: ws == NULL allocates internally; otherwise ws must be 256-byte
 * aligned and ws_bytes >= ri_ppl_workspace_bytes(o, v, naux, precision)
 * (RI_E_NOMEM if smaller).  The workspace contents are scratch.  The reduced
 * precisions round B_vv and the packed tau once to their operand type (FP32, or a
 * bf16 hi + lo pair), rebuild the integrals with FP32 accumulation, round them
 * again for the contraction and add the FP32 result into the FP64 R; the error of
 * an element is bounded by 2e-4 times the ladder of |B_vv| and |tau| (and is a few
 * 1e-6 of max |R| for bf16 hi + lo, less for FP32).  RI_PREC_BF16X3 needs
 * vp * Qp < 2^27 (vp = v rounded up to 16, Qp = naux rounded up to 32), RI_E_ARG
 * otherwise. */
int ri_ppl_ex(const double* B_vv, const double* tau, int o, int v, int naux, double* R,
              int precision, void* ws, size_t ws_bytes, void* stream);

/* Allocation-free ladder, for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * computation, arguments, error codes and error bound as ri_ppl_ex with ws == NULL,
 * but the workspace is a fixed device array inside the library,
 * RI_PPL_NOALLOC_MAX_BYTES (64 MiB) on every device that loads it, held until the
 * process ends; the call allocates and frees nothing (the per-kernel event profiler
 * stays off for it).  The slab of (ab) block pairs is the widest whose workspace fits
 * that array, so results can differ from ri_ppl_ex in rounding only (the summation
 * order of the contraction's k splits).  Sizes whose one-block-pair plan does not fit
 * return RI_E_NOMEM and change nothing; as a guide, the FP64 workspace is about
 * 8 vp^2 naux_p + 2 * 8 K (o^2/2 + 256) bytes with vp = v rounded up to 16,
 * naux_p = naux rounded up to 16 and K = 128 (vp/16)(vp/16 + 1), so o = 8, v = 96,
 * naux = 288 fits in FP64 and o = 8, v = 128, naux = 384 only in FP32 and bf16x3.
 * Every call on one device shares that device's array: calls that overlap on one
 * device (several streams or host threads) race, and the caller must serialise them.
 * `stream` must belong to the current device (RI_E_ARG otherwise). */
#define RI_PPL_NOALLOC_MAX_BYTES (64u << 20)
int ri_ppl_noalloc(const double* B_vv, const double* tau, int o, int v, int naux, double* R, int precision,
                   void* stream);

/* One shard of a ladder call split over several devices: the split of the virtual
 * index a across domains of Sec. II.D, at the granularity of the (ab) block-pair
 * slabs.  Shard k of n (0 <= k < n) builds and contracts the slabs k, k + n,
 * k + 2n, ... and accumulates only their (a, b) entries of R; every device holds
 * full replicas of B_vv and tau and packs all of tau.  The n shards together add
 * exactly (bitwise) what one ri_ppl_ex call adds, since every R entry comes from
 * one slab; a multi-device caller sums or gathers the shards' R.  The slab size
 * depends only on (o, v, naux, precision) and RI_PPL_W_BYTES / RI_PPL_SLAB_PAIRS,
 * which must agree across the shards.  ri_ppl_ex is shard 0 of 1.
 * RI_E_ARG for an invalid (shard, nshards). */
int ri_ppl_shard(const double* B_vv, const double* tau, int o, int v, int naux, double* R,
                 int precision, int shard, int nshards, void* ws, size_t ws_bytes, void* stream);

/* The same ladder in the paper's own arrangement (Sec. II.C, Fig. 2), FP64, kept as
 * an ablation of the tau+- form: for every virtual a the full (ac|bd) slice over
 * (b, c, d) is built from B_vv and contracted with tau over the packed occupied pairs
 * i <= j only; the i > j entries follow from R^{ab}_{ij} = R^{ba}_{ji}.  Arguments,
 * layouts, accumulation, the use of tau's pair-symmetric part and the error codes are
 * those of ri_ppl; the result agrees with ri_ppl to rounding.  Cost (ri_ppl_paper_flops):
 * 2 Naux v^4 + v^4 o(o+1) FLOP, about twice the build and four times the contraction of
 * ri_ppl.  Device workspace of 2 v^2 o(o+1)/2 + a v^3 doubles (a = the values of the
 * first virtual index per step, within RI_PPL_PAPER_V_BYTES, 4 GiB by default) is
 * taken stream-ordered for the call. */
int ri_ppl_paper(const double* B_vv, const double* tau, int o, int v, int naux, double* R, void* stream);
double ri_ppl_paper_flops(int o, int v, int naux);

/* The ladder of ri_ppl, FP64, for factors symmetric in their two virtual indices
 * (B_vv[Q][a][c] == B_vv[Q][c][a], the bare integrals of eq. RIM; not the t1-dressed
 * factors of the CCSD residual).  Then (ac|bd) has the eight-fold symmetry of real
 * two-electron integrals (Sec. II.C) and the integral matrix of the tau+- form is
 * symmetric under the exchange of the (ab) and (cd) pairs: each slab of (ab) block
 * pairs builds only the (cd) block pairs from its own first one on and uses every
 * built element twice, once for its own (ab) rows and once, through a second FP64
 * product, for the later (cd) rows.  With the default of at least 8 slab steps
 * (environment RI_PPL_SYM_SLABS) the build costs about 9/16 of ri_ppl's; the
 * contraction FLOP are unchanged.  Arguments, layouts, accumulation into R, the use of
 * tau's pair-symmetric part and the error codes are those of ri_ppl; the result agrees
 * with ri_ppl to rounding (the summation order differs).  The call first measures the
 * factors' asymmetry on `stream` (synchronising it) and returns RI_E_ARG, leaving R
 * untouched, unless max |B_ac - B_ca| <= 1e-12 max |B|.  Device workspace of about
 * ri_ppl_workspace_bytes(o, v, naux, RI_PREC_FP64) plus about v^2 o^2 / 2 doubles of
 * second-product accumulators is taken stream-ordered for the call. */
int ri_ppl_sym(const double* B_vv, const double* tau, int o, int v, int naux, double* R, void* stream);
/* The same with a choice of arithmetic (RI_PREC_*), on the slab schedule of the FP64 form.
 * The reduced precisions keep the error bound of ri_ppl_ex (2e-4 times the ladder of |B_vv|
 * and |tau|, element by element).  In RI_PREC_BF16X3 the integral tiles are stored with
 * the (cd) index innermost, so each slab's second product first transposes its block of
 * them (one read and one write of 8 bytes per element: the hi and lo words of V+ and V-)
 * and workspace for that transposed block is taken as well. */
int ri_ppl_sym_ex(const double* B_vv, const double* tau, int o, int v, int naux, double* R, int precision,
                  void* stream);
/* Algorithmic FLOP of one ri_ppl_sym call (build and both products over its slab
 * schedule, which depends on RI_PPL_W_BYTES, RI_PPL_SLAB_PAIRS and RI_PPL_SYM_SLABS);
 * 0 on invalid arguments. */
double ri_ppl_sym_flops(int o, int v, int naux);

/* Workspace bytes ri_ppl_ex needs for these sizes (0 on invalid arguments).  The
 * partial sums of the contraction's k splits are part of it, and their number follows
 * the current device (its compute units and the contraction kernel's occupancy): ask
 * with the device current that ri_ppl_ex will run on.  Without a device the count
 * assumes 256 compute units. */
size_t ri_ppl_workspace_bytes(int o, int v, int naux, int precision);

/* Algorithmic floating-point operation count of one ladder call as executed
 * (the a<=b half of the integral build plus the packed contraction; one fused
 * multiply-add counts two).  0 on invalid arguments. */
double ri_ppl_flops(int o, int v, int naux);

/* Per-kernel timing.  While enabled, the library brackets each of its kernel
 * launches with HIP events on the launch stream.  ri_prof_report synchronises
 * those events, writes a JSON array [{"name", "count", "ms", "flops", "bytes"}]
 * (summed per kernel name; flops/bytes are the algorithmic counts of the work
 * launched) into buf, and clears the records.  RI_E_ARG if buf is too small. */
int ri_prof_enable(int on);
int ri_prof_report(char* buf, size_t len);

/* Distance of tau [o][o][v][v] from pair symmetry (Sec. II.C):
 * result[0] = max |tau[i][j][c][d] - tau[j][i][d][c]|, result[1] = max |tau|
 * (host array of two doubles; NaN if tau holds one).  Synchronises stream. */
int ri_tau_pair_asymmetry(const double* tau, int o, int v, double* result, void* stream);

/* tau[i][j][a][b] = t2[i][j][a][b] + t1[i][a] t1[j][b]   (eq. pp-Ladder-01).
 * t1: [o][v], t2 and tau: [o][o][v][v]; tau may alias t2 (in place). */
int ri_build_tau(const double* t1, const double* t2, int o, int v, double* tau, void* stream);

/* ------------------------------------------------------------------------
 * Closed-shell RI-CCSD (Sec. II.A: eqs. ccsd-1..3 solved by Jacobi iterations
 * with DIIS; energy expression of Sec. II.A).  Canonical Hartree-Fock orbitals
 * are assumed: the Fock matrix is diag(eps), and the bare one-electron matrix is
 * derived from it as h = diag(eps) - sum_k [2 (pq|kk) - (pk|kq)].
 * ------------------------------------------------------------------------ */
typedef struct ri_system {
  int o, v, naux;
  const double* B;   /* [naux][n][n], n = o + v, RI factors symmetric in the MO pair */
  const double* eps; /* [n] orbital energies, occupied first */
} ri_system;

#define RI_GUESS_MP2 0  /* t1 = 0, t2 = (ia|jb) / D (iteration 0) */
#define RI_GUESS_USER 1 /* start from the t1, t2 passed in */
#define RI_GUESS_MLP 2  /* the MP2 guess corrected by the network opts->mlp (ri_mlp_guess);
                           falls back to RI_GUESS_MP2 if that fails or is non-finite */

typedef struct ri_mlp ri_mlp; /* learned starting guess, declared below */

typedef struct ri_ccsd_opts {
  int max_iter;        /* iteration limit (default 100) */
  double tol_residual; /* converged when max |Omega| <= tol_residual ... (default 1e-10) */
  double tol_energy;   /* ... and |E_k - E_{k-1}| <= tol_energy (default 1e-10) */
  int diis_size;       /* stored vectors, 2..16; < 2 disables DIIS (default 6) */
  int diis_start;      /* first iteration that extrapolates (default 2) */
  int ppl_precision;   /* RI_PREC_* of the ladder term (default RI_PREC_FP64) */
  int guess;           /* RI_GUESS_MP2, RI_GUESS_USER or RI_GUESS_MLP */
  int verbose;         /* one line per iteration on stderr */
  /* Reduced precision only (ladder or other_precision): once max |Omega| <=
   * polish_residual, every later residual uses the polish_precision ladder (and FP64
   * other contractions when that is FP64), and convergence is only declared on such
   * a residual (0 disables; default 0). */
  double polish_residual;
  /* Reduced precision only: evaluate max |Omega| of the returned amplitudes once more
   * in FP64 throughout into rep->residual_inf_fp64 (default 0). */
  int check_fp64;
  ri_mlp* mlp; /* network for RI_GUESS_MLP (default NULL) */
  int polish_precision; /* ladder after the polish switch: RI_PREC_FP64 (default) or RI_PREC_FP32 */
  /* Arithmetic of the large non-ladder contractions (the o^3 v^3 terms and the
   * integral builds from the dressed factors): RI_PREC_FP64 (default) or RI_PREC_FP32
   * (operands rounded to FP32, FP32 MFMA).  Setup, update, DIIS and energy stay FP64;
   * an FP64 polish also returns these contractions to FP64. */
  int other_precision;
} ri_ccsd_opts;

typedef struct ri_ccsd_report {
  double e_corr;       /* correlation energy of the returned amplitudes (Hartree) */
  double e_mp2;        /* MP2 energy of the guess (NaN unless RI_GUESS_MP2) */
  double residual_inf; /* max |Omega| at the last residual evaluation */
  int iterations;      /* residual evaluations minus one */
  int converged;
  double seconds_total; /* wall time of the call, guess included, check_fp64 excluded */
  double seconds_ppl;   /* GPU time of the ladder term */
  double residual_rms;  /* root mean square of Omega at the last residual evaluation */
  /* max |Omega| of the returned amplitudes evaluated in FP64 throughout: equals
   * residual_inf when a converged run's last residual was FP64 throughout (FP64 runs,
   * FP64-polished runs), else the check_fp64 evaluation, else NaN */
  double residual_inf_fp64;
  int polish_iteration; /* first iteration whose residual used the polish ladder after a
                           mixed start (-1: none) */
  double seconds_guess; /* wall time until the guess and its energy were ready */
  int guess_used;       /* RI_GUESS_* actually used: RI_GUESS_MLP falls back to RI_GUESS_MP2
                           when the network fails or gives non-finite amplitudes */
} ri_ccsd_report;

/* Fills the defaults listed above. */
void ri_ccsd_default_opts(ri_ccsd_opts* opts);

/* t1 = 0 ([o][v]); t2[i][j][a][b] = (ia|jb) / (e_i + e_j - e_a - e_b); optional MP2
 * energy on the host (synchronises stream when e_mp2 != NULL). */
int ri_mp2_guess(const ri_system* sys, double* t1, double* t2, double* e_mp2, void* stream);

/* E_corr = sum_ijab (2 (ia|jb) - (ib|ja)) (t2[i][j][a][b] + t1[i][a] t1[j][b]), reduced in
 * FP64 in a fixed order; written to the host (synchronises stream). */
int ri_ccsd_energy(const ri_system* sys, const double* t1, const double* t2, double* e_corr, void* stream);

/* CCSD residuals for the given amplitudes: omega1 [o][v], omega2 [o][o][v][v]
 * (projections of eqs. ccsd-2/-3 in the biorthogonal basis; at t = 0 omega2 is
 * (ia|jb) and omega1 is 0).  The ladder term uses ppl_precision, everything else
 * FP64.  Outputs must not overlap the amplitudes. */
int ri_ccsd_residual(const ri_system* sys, const double* t1, const double* t2, double* omega1, double* omega2,
                     int ppl_precision, void* stream);

/* Iterate t += Omega / D with DIIS from the chosen guess until converged or
 * opts->max_iter residual evaluations.  t1, t2 are overwritten with the final
 * amplitudes (t2 kept pair-symmetric).  Returns RI_E_NOCONV (amplitudes valid)
 * when the limit is reached, RI_E_NUMERIC on NaN/Inf or divergence.  `rep` may
 * be NULL.  opts == NULL uses the defaults.  Synchronises stream. */
int ri_ccsd_iterate(const ri_system* sys, double* t1, double* t2, const ri_ccsd_opts* opts,
                    ri_ccsd_report* rep, void* stream);

/* Perturbative triples energy of closed-shell CCSD(T) (Sec. II.A), FP64, from the
 * amplitudes t1 [o][v] and t2 [o][o][v][v] (device; t2 pair-symmetric) and the
 * RI factors of sys:
 *   E_(T) = sum_{ijk} sum_{abc} (4 W^{abc}_{ijk} + W^{bca}_{ijk} + W^{cab}_{ijk})
 *                               (V^{abc}_{ijk} - V^{cba}_{ijk}) / (3 D^{abc}_{ijk})
 * with W, V and D as defined there; written to *e_t (host).  The occupied triplets
 * i <= j <= k are visited once each (W and V of the other orderings are permutations
 * of theirs).  Cost ri_ccsd_triples_flops(o, v) = o(o+1)(o+2) 2 v^3 (v+o) FLOP;
 * device workspace of o v^2 (v+o) + o^2 v (v+o) + o^3 v + o^2 v^2 + 8 v^3 doubles
 * (plus small buffers) is taken stream-ordered.  Synchronises stream; RI_E_NUMERIC if the energy is not
 * finite. */
int ri_ccsd_triples(const ri_system* sys, const double* t1, const double* t2, double* e_t, void* stream);
/* The same with a choice of arithmetic for the term GEMMs: RI_PREC_FP64, or RI_PREC_FP32
 * (operands rounded to FP32, FP32 MFMA with FP32 accumulation over the summed index of
 * v + o, where the GEMM takes its 128 x 128 tile kernel; W, V and the energy sum stay
 * FP64).  The FP32 error of E_(T) was 1e-8 of its size at o = 24, v = 384.  RI_E_ARG
 * for other precision values. */
int ri_ccsd_triples_ex(const ri_system* sys, const double* t1, const double* t2, int precision, double* e_t,
                       void* stream);
double ri_ccsd_triples_flops(int o, int v);

/* ------------------------------------------------------------------------
 * Learned starting guess (not in the paper; an addition on top of the MP2 guess).
 * A fully connected network -- `layers` tanh hidden layers of `hidden` units and
 * one linear output -- maps 8 per-amplitude MP2 features to a relative correction
 * of the MP2 doubles amplitudes: t2 = t2_MP2 * (1 + y_scale * net((x - mean) / std)).
 * (A relative correction keeps the guess error proportional to each amplitude, so
 * the small amplitudes stay as accurate as MP2 makes them.)
 * Parameters form one FP32 vector W1 [d_in][h], b1 [h], ..., W_out [h][1], b_out [1].
 * Training runs on the GPU (loss: batch mean of (y - Y)^2, Adam with beta1 0.9,
 * beta2 0.999, eps 1e-8).  The handle owns its device memory; calls that take a
 * stream enqueue on it; a handle must not be used from two streams at once.
 * ------------------------------------------------------------------------ */
/* New network with zero parameters (NULL on failure, see ri_last_error_msg). */
ri_mlp* ri_mlp_create(int d_in, int hidden, int layers);
void ri_mlp_destroy(ri_mlp* net);
size_t ri_mlp_num_params(const ri_mlp* net);
/* Copy the flat parameter vector from / to host memory (set also resets Adam). */
int ri_mlp_set_params(ri_mlp* net, const float* params_host);
int ri_mlp_get_params(const ri_mlp* net, float* params_host);
/* Feature standardisation (mean, std: d_in host floats, std > 0) and output scale. */
int ri_mlp_set_scaling(ri_mlp* net, const float* mean, const float* std, float y_scale);
int ri_mlp_get_scaling(const ri_mlp* net, float* mean, float* std, float* y_scale);
/* y[n] = net(X) for device X [n][d_in] (already standardised), FP32. */
int ri_mlp_forward(ri_mlp* net, const float* X, long n, float* y, void* stream);
/* The same y without keeping the hidden activations: every 64 rows go through all
 * layers in one workgroup, in the operation order of ri_mlp_forward (equal results
 * bit for bit).  Needs d_in a multiple of 4 and hidden a multiple of 16, both at most
 * 256 (else RI_E_ARG); allocates nothing. */
int ri_mlp_infer(const ri_mlp* net, const float* X, long n, float* y, void* stream);
/* Loss and its gradient (device FP32 [num_params]; NULL uses internal storage) on a
 * batch of n <= 2^24 rows; the loss is written to *loss_host when not NULL
 * (synchronises stream).  Deterministic (fixed reduction order). */
int ri_mlp_gradient(ri_mlp* net, const float* X, const float* Y, long n, float* grad, float* loss_host,
                    void* stream);
/* One Adam step with learning rate lr on the batch; *loss_host gets the batch loss
 * before the step when not NULL (synchronises stream). */
int ri_mlp_train_step(ri_mlp* net, const float* X, const float* Y, long n, float lr, float* loss_host,
                      void* stream);
/* Seeded starting parameters, written on `stream`: weight number i of the flat vector
 * (layer fan-in f) is N(0, 1)/sqrt(f), the normal drawn by the Box-Muller transform
 * from SplitMix64 outputs 2i and 2i+1 of `seed`; biases are zero; Adam restarts. */
int ri_mlp_init(ri_mlp* net, unsigned long long seed, void* stream);
/* Options of ri_mlp_train (ri_mlp_default_train_opts fills the defaults shown). */
typedef struct ri_mlp_train_opts {
  int epochs;               /* passes over the training set (30) */
  long batch;               /* rows per Adam step (4096); an epoch takes max(1, n / batch)
                               steps of min(batch, n) rows, the rest of the rows wait
                               for a later shuffle */
  float lr;                 /* peak learning rate (5e-4) */
  float warmup;             /* fraction of all steps in the linear warm-up (0.05); after
                               it the rate decays to zero on a half cosine */
  unsigned long long seed;  /* shuffle seed (1) */
  int shuffle;              /* 1: rows in a new order each epoch (Fisher-Yates driven by
                               SplitMix64 of `seed`); 0: rows in the given order (1) */
} ri_mlp_train_opts;
void ri_mlp_default_train_opts(ri_mlp_train_opts* opts);
/* Fit the network to device X [n][d_in] (standardised) and Y [n] by Adam steps
 * (ri_mlp_train_step's update), the whole loop in the library: shuffle, batches,
 * learning-rate schedule (step t of T with W warm-up steps, W = max(1, floor(T warmup)):
 * lr min(1, (t+1)/W) (1 + cos(pi t / T)) / 2), and after each epoch the loss on the
 * validation set (X_val [n_val][d_in], Y_val [n_val]; n_val = 0 for none).
 * opts NULL takes the defaults.  train_loss / val_loss: host arrays of opts->epochs
 * floats (or NULL) for each epoch's mean batch loss and validation loss; when either
 * is given the call synchronises the stream and returns RI_E_NUMERIC if a loss is not
 * finite.  n <= 2^28, batch <= 2^24.  Device workspace of n (d_in + 2) + n_val floats
 * (about) is taken stream-ordered for the call; the host waits for each permutation copy
 * before it reuses the host buffer, not for the training steps. */
int ri_mlp_train(ri_mlp* net, const float* X, const float* Y, long n, const float* X_val, const float* Y_val,
                 long n_val, const ri_mlp_train_opts* opts, float* train_loss, float* val_loss, void* stream);
/* Raw (unstandardised) features of every amplitude, X [o][o][v][v][8] FP32, from the
 * MP2 t2 and the (ia|jb) integrals of sys: t2_ijab, t2_ijba, (ia|jb), (ib|ja),
 * e_i + e_j - e_a - e_b, (e_a - e_b)^2, (e_i - e_j)^2, sqrt((ia|ia)(jb|jb)). */
int ri_mlp_features(const ri_system* sys, const double* t2_mp2, float* X, void* stream);
/* Training data of the learned guess, built on the device.
 * ri_mlp_sample: n amplitude indices drawn with replacement, index k (0 <= k < total)
 * with probability t2_mp2[k]^2 / sum t2_mp2^2, by the inverse of the cumulative weight:
 * sample s takes u_s = ((x_s >> 11) + 1/2) 2^-53 of the total weight, x_s the
 * SplitMix64 output s of `seed` (as in ri_mlp_init), and picks the first index whose
 * running sum of weights (FP64, index order, in chunks of 4096) exceeds it.  idx: device
 * int64 [n].  Synchronises stream; RI_E_NUMERIC if the weights sum to zero or a non-finite
 * value.
 * ri_mlp_targets: Y[s] = clamp(t2_ccsd[idx[s]] / t2_mp2[idx[s]] - 1, -clip, clip), the
 * relative correction the network predicts (FP32 out, device arrays).
 * ri_mlp_fit_scaling: sets the network's feature standardisation to the column means and
 * standard deviations (FP64 sums in a fixed order, divided by n; a zero deviation becomes
 * 1) of X [n][d_in] and its output scale to the standard deviation of Y [n] (device
 * FP32 arrays); synchronises stream.
 * ri_mlp_standardize: Xn = (X - mean) / std and, when Y and Yn are given, Yn = Y / y_scale
 * with the network's scaling (d_in <= 8; in place allowed). */
int ri_mlp_sample(const double* t2_mp2, long total, long n, unsigned long long seed, long* idx, void* stream);
int ri_mlp_targets(const double* t2_ccsd, const double* t2_mp2, const long* idx, long n, float clip, float* Y,
                   void* stream);
int ri_mlp_fit_scaling(ri_mlp* net, const float* X, const float* Y, long n, void* stream);
int ri_mlp_standardize(const ri_mlp* net, const float* X, const float* Y, long n, float* Xn, float* Yn,
                       void* stream);
/* Learned guess: t1 = 0, t2 = t2_MP2 * (1 + y_scale * net) (FP64 outputs).  The network
 * runs on the amplitudes with i <= j and its value goes to both (i, j, a, b) and
 * (j, i, b, a); on i == j the two orders of (a, b) are averaged.  The network must have 8
 * inputs; with d_in and hidden as ri_mlp_infer needs it runs through that kernel. */
int ri_mlp_guess(ri_mlp* net, const ri_system* sys, double* t1, double* t2, void* stream);
/* Binary file with sizes, scaling and parameters. */
int ri_mlp_save(const ri_mlp* net, const char* path);
ri_mlp* ri_mlp_load(const char* path);

#ifdef __cplusplus
}
#endif

#endif /* RICCSD_H */
