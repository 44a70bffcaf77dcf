/*
 * afqmc.h - C ABI of the MI355X (gfx950) phaseless AFQMC walker update.
 *
 * Method: Shee, Arthur, Zhang, Reichman, Friesner, "Phaseless Auxiliary-Field
 * Quantum Monte Carlo on Graphical Processing Units" (arXiv 1804.03310),
 * Sec. II (imaginary-time projection, Eq. 1 Hamiltonian, Eq. 2
 * Hubbard-Stratonovich transform, Eq. 3 propagator, force bias, local energy,
 * phaseless constraint) and Sec. III (batched Sherman-Morrison-Woodbury
 * update for multi-determinant trials; energy through half-rotated
 * Cholesky vectors, the partial contraction inside Eq. Ys; sp/dp switching).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Matrices are row-major, float64, and all indices are 0-based.
 * - One system has M orbitals, N_up / N_dn electrons and n_chol Cholesky
 *   vectors with V_ijkl = sum_g L[g][i][k] L[g][j][l] (Eq. 1).
 * - A walker is a pair of Slater determinants stored side by side as an
 *   M x (N_up + N_dn) complex matrix in planar form: phi_re[w][m][c] and
 *   phi_im[w][m][c], columns 0..N_up-1 spin up, N_up.. spin down.
 * - Device pointers are HIP device memory on the device the Hamiltonian was
 *   created on; host pointers are ordinary host memory.  The library never
 *   frees caller memory.  Inputs passed to init_* are copied; the caller may
 *   free them when the call returns.
 * - Every call that takes a `stream` (a hipStream_t passed as void*, NULL =
 *   default stream) enqueues its work on it and returns without waiting,
 *   unless it writes a host pointer, in which case it synchronises that
 *   stream before returning.  Device outputs are valid once the stream has
 *   completed.
 * - Argument errors are detected before anything is enqueued and return
 *   AFQMC_ERR_ARG; afqmc_last_error() then gives a message (thread-local).
 *   Numerical trouble in a single walker is not an error: the walker dies
 *   (weight 0) and is reset to the reference determinant.
 * - No C++ exception crosses this interface.
 */
#ifndef AFQMC_H
#define AFQMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AFQMC_OK = 0,
  AFQMC_ERR_ARG = -1,         /* invalid argument (shape, pointer, value)      */
  AFQMC_ERR_OOM = -2,         /* device allocation failed                      */
  AFQMC_ERR_DEVICE = -3,      /* a HIP call failed                             */
  AFQMC_ERR_STATE = -4,       /* objects do not belong together                */
  AFQMC_ERR_SINGULAR = -5,    /* trial overlap with itself is singular         */
  AFQMC_ERR_NONFINITE = -6,   /* every walker is dead (sum of weights is 0)    */
  AFQMC_ERR_UNSUPPORTED = -7  /* size or precision outside the library's limits */
} afqmc_status;

/* Arithmetic of a contraction (Sec. III: single- vs double-precision).
 * AFQMC_BF16: bf16 operands with FP32 accumulation on the matrix cores
 * (contractions only; single-determinant trials).
 * AFQMC_BF16X3: every operand split in two bf16 terms, x = hi + lo with
 * hi = bf16(x) and lo = bf16(x - hi) (about 16 significant bits), and each
 * product taken as hi hi + hi lo + lo hi (the lo lo term, of relative size
 * 2^-18, dropped) on the bf16 matrix cores with FP32 accumulation: three
 * bf16 MFMAs per product, for the propagator build and the Ltil Theta
 * contraction (same limits as AFQMC_BF16). */
typedef enum { AFQMC_FP64 = 0, AFQMC_FP32 = 1, AFQMC_BF16 = 2, AFQMC_BF16X3 = 3 } afqmc_prec;

#define AFQMC_MAX_EXC 4      /* excitations per spin in one determinant      */
/* The Q exchange route (afqmc_trial_exchange_route) runs its contractions in
 * FP32 under chol_prec FP32 only while M * max(N_up, N_dn) is at most this;
 * above it, and under FP64, they are FP64 (the quadratic form sums M^2 N^2
 * terms of both signs per spin, and its FP32 error grows with their number). */
#define AFQMC_QROUTE_FP32_MAX_K 4096
#define AFQMC_MAX_NEL 64     /* electrons per spin                           */
#define AFQMC_MAX_M 256      /* orbitals                                     */

typedef struct afqmc_ham afqmc_ham;     /* library-owned, device resident */
typedef struct afqmc_trial afqmc_trial; /* library-owned, device resident */

/* A batch of walkers.  All buffers are caller-owned device memory.
 * phi_re/phi_im [n_walkers][M][N_up+N_dn]; weight, logovlp_*, eloc_*
 * [n_walkers].  logovlp is log <Psi_T|phi> (complex, imaginary part defined
 * modulo 2 pi), eloc the last local energy.  workspace is scratch the library
 * lays out itself (overlap inverses, Theta, force-bias traces, propagator
 * matrices, Taylor terms, comb snapshot); its size comes from
 * afqmc_walker_workspace_bytes and it must not be shared between batches
 * that run concurrently.  system_id enters the random-number counter. */
typedef struct {
  int32_t n_walkers;
  int32_t system_id;
  double *phi_re, *phi_im;
  double *weight;
  double *logovlp_re, *logovlp_im;
  double *eloc_re, *eloc_im;
  void *workspace;
  size_t workspace_bytes;
} afqmc_walkers;

/* Run options.  taylor_order: terms of the series for exp(A) (>= 1);
 * chol_prec may be AFQMC_BF16 or AFQMC_BF16X3, taylor_prec only AFQMC_FP64
 * or AFQMC_FP32.
 * ortho_every / pc_every: orthonormalise / comb after global step t when
 * (t+1) is a multiple (0 = never).  e_trial: E_T of the weight factor.
 * chol_prec: arithmetic of sum_g x_g L_g and of Ltil_g Theta;
 * taylor_prec: arithmetic of the Taylor products and of B1 phi.
 * Overlaps, inverses, determinants, MGS and all final sums are FP64.
 * weight_mode: AFQMC_WEIGHT_LOCAL_ENERGY (Sec. II; the default, 0) or
 * AFQMC_WEIGHT_HYBRID (Sec. IV.A: W <- W |I| exp(-dt (E_0 - e_trial))
 * max(0, cos dtheta), I = (<Psi_T|phi'>/<Psi_T|phi>) exp(sum_g
 * (x_g xbar_g - xbar_g^2 / 2)), E_0 = e_core - 1/2 sum_g lbar_g^2); in the
 * hybrid form E_L and E_mix are only evaluated after steps t with
 * (t+1) % meas_every == 0 (meas_every >= 1; ignored in the local-energy
 * form), the other entries of emix_dev are NaN and walkers' eloc keep the
 * last measured value. */
typedef enum { AFQMC_WEIGHT_LOCAL_ENERGY = 0, AFQMC_WEIGHT_HYBRID = 1 } afqmc_weight_mode;
typedef struct {
  int32_t taylor_order;
  int32_t ortho_every;
  int32_t pc_every;
  double e_trial;
  afqmc_prec chol_prec;
  afqmc_prec taylor_prec;
  int32_t weight_mode;
  int32_t meas_every;
} afqmc_options;

/* Hamiltonian of Eq. 1: one-body h [M][M] (symmetric), Cholesky vectors
 * L [n_chol][M][M] (each symmetric) with V_ijkl = sum_g L_g,ik L_g,jl, and a
 * constant e_core.  Host inputs, copied to `device`.  Symmetry is checked to
 * 1e-10 (relative to the largest entry); 1 <= M <= AFQMC_MAX_M, n_chol >= 0. */
afqmc_status afqmc_init_hamiltonian(afqmc_ham **out, int device, void *stream,
                                    int M, int n_chol, const double *h,
                                    const double *L, double e_core);

/* Trial wavefunction Psi_T = sum_i coeff[i] |D_i> (Sec. III).  C_up, C_dn
 * [M][M] host: orthonormal orbitals as columns; the reference determinant D_0
 * occupies columns 0..N_sigma-1.  exc [n_det][2][1 + 2*AFQMC_MAX_EXC] host
 * int32: for determinant i and spin s, exc[i][s][0] = E (number of
 * excitations), then E hole orbitals (< N_s), then at offset 1+AFQMC_MAX_EXC
 * E particle orbitals (>= N_s); hole e is replaced in place by particle e.
 * Row 0 must be the reference (E = 0 for both spins).  coeff [n_det] host.
 * For n_det = 1, coeff and exc may be NULL.  mf_subtract = 1 subtracts the
 * reference-determinant mean field lbar_g = <D_0|L_g|D_0> from the fields
 * (an exact rewrite of Eq. 2); 0 uses lbar = 0.  The multi-determinant path
 * supports E <= 2 per spin.  Returns AFQMC_ERR_SINGULAR if D_0^T D_0 is
 * singular. */
afqmc_status afqmc_init_trial(afqmc_trial **out, afqmc_ham *ham, int n_up, int n_dn,
                              const double *C_up, const double *C_dn, int n_det,
                              const double *coeff, const int32_t *exc, int mf_subtract);

/* Bytes of walker workspace for n_walkers walkers of this trial. */
afqmc_status afqmc_walker_workspace_bytes(const afqmc_trial *trial, int n_walkers,
                                          size_t *bytes);

/* Device bytes one system of these sizes occupies: Hamiltonian, trial
 * (including one cached B1 and the largest transient its set-up allocates),
 * the caller's walker buffers for n_walkers walkers and their workspace.
 * For admission decisions before anything is allocated. */
afqmc_status afqmc_footprint_bytes(int M, int n_chol, int n_up, int n_dn, int n_det,
                                   int n_walkers, size_t *bytes);

/* How the trial evaluates the exchange energy sum_g Tr(X_g X_g), X_g = Ltil_g
 * Theta (the contraction inside the paper's Eq. Ys): *route = 0 through the
 * half-rotated vectors Ltil_g per Cholesky index, or 1 through the
 * precomputed two-index tensor Q[(n a)][(m b)] = sum_g Ltil_g[a][m]
 * Ltil_g[b][n] per spin, as the quadratic form theta^T Q theta (chosen at
 * set-up for single-determinant trials with n_chol >= 2 M and M N_sigma <=
 * 16384; the BF16 contraction mode always takes route 0).  Route 1
 * contracts in FP32 under chol_prec FP32 only up to AFQMC_QROUTE_FP32_MAX_K,
 * else in FP64. */
afqmc_status afqmc_trial_exchange_route(const afqmc_trial *trial, int *route);

/* Select the exchange route of later measurements: 0 (Ltil) is always
 * available; 1 (Q) only where set-up built Q, else AFQMC_ERR_UNSUPPORTED and
 * the route is left as it was.  Not to be called while work that uses the
 * trial is in flight on any stream. */
afqmc_status afqmc_trial_set_exchange_route(afqmc_trial *trial, int route);

/* Sets every walker to the reference determinant D_0 with weight 1 and
 * fills logovlp / eloc with the reference values. */
afqmc_status afqmc_walkers_from_trial(afqmc_ham *ham, afqmc_trial *trial,
                                      afqmc_walkers *walkers, void *stream);

/* n_steps timesteps of length dt for every walker (Sec. II):
 *   fields x ~ N(0,1) (Philox4x64-10, key (seed, 0), counter
 *   (t, walker, gamma/4, system_id), Box-Muller), force bias
 *   xbar = -i sqrt(dt)(v - lbar) from the mixed estimate v_g = <L_g>,
 *   phi <- B1 exp(A) B1 phi with A = i sqrt(dt) sum_g (x_g - xbar_g) L_g and
 *   B1 = exp(-dt H1'/2), H1' = h - 1/2 sum L_g L_g + sum lbar_g L_g,
 *   new overlap, E_L = <Psi_T|H|phi>/<Psi_T|phi>, and the phaseless weight
 *   W <- W exp(-dt (Re E_L - e_trial)) max(0, cos dtheta) with
 *   dtheta = Im log(<Psi_T|phi'>/<Psi_T|phi>) including the mean-field
 *   phase.  Global step indices are step0 .. step0+n_steps-1.  The call
 *   first refreshes logovlp, eloc and v from phi.  emix_dev (device,
 *   [n_steps], nullable) receives sum W Re E_L / sum W after each step
 *   (before orthonormalisation / combing).  */
afqmc_status afqmc_propagate(afqmc_ham *ham, afqmc_trial *trial, afqmc_walkers *walkers,
                             int n_steps, double dt, uint64_t seed, uint64_t step0,
                             const afqmc_options *opt, double *emix_dev, void *stream);

/* Refreshes logovlp, eloc (and the stored force-bias traces) of every walker
 * from phi; weights unchanged.  If emix_host is non-NULL it receives
 * sum W Re E_L / sum W (synchronises the stream; AFQMC_ERR_NONFINITE if the
 * sum of weights is 0). */
afqmc_status afqmc_local_energy(afqmc_ham *ham, afqmc_trial *trial, afqmc_walkers *walkers,
                                double *emix_host, void *stream);

/* Modified Gram-Schmidt of each walker's spin blocks (positive real R
 * diagonal), then logovlp recomputed; weights and eloc unchanged
 * (Sec. IV.A: walkers orthonormalized periodically). */
afqmc_status afqmc_orthonormalize(afqmc_ham *ham, afqmc_trial *trial, afqmc_walkers *walkers,
                                  void *stream);

/* Population control by a systematic comb (Sec. IV.A, Sec. V): inclusive
 * prefix sums of the weights, left to right; one uniform xi (Philox key
 * (seed, 1), counter (pc_index, 0, 0, system_id), word 0); tooth j at
 * ((j + xi) W_tot) / K picks the first walker whose prefix sum exceeds it.
 * Walker state is copied from the parents and weights reset to 1.
 * norm_factor_host (nullable) receives W_tot / K (synchronises the stream).
 * If W_tot is not positive and finite (every walker dead) the population is
 * left unchanged and the norm factor is 0; with norm_factor_host the call
 * then returns AFQMC_ERR_NONFINITE.  Inside afqmc_propagate such a population
 * stays dead and its E_mix entries are not finite. */
afqmc_status afqmc_reconfigure(afqmc_trial *trial, afqmc_walkers *walkers, uint64_t seed,
                               uint64_t pc_index, double *norm_factor_host, void *stream);

/* ---------------------------------------------------------------------------
 * Groups: the walkers of several systems (uneven M, N, n_chol, walker counts)
 * propagated together, Sec. II's step for every walker of every member in
 * one launch of the walker-resident kernel: one workgroup per walker keeps
 * its orbitals, propagator, Taylor terms, overlap inverses and force bias in
 * LDS for a segment of steps; the operators are shared through L2.  Each
 * member's results are those of afqmc_propagate with the same arguments
 * (same readings of the method, same fields) computed in FP64 whatever the
 * options' precisions, and they are bitwise the same alone or in any group
 * and for every launch shape (every sum is taken in an order fixed by the
 * problem, not by the thread count).  A segment (steps, mixed energies,
 * combs, step counter) is captured once as a HIP graph and replayed; combs
 * fall at segment ends (segment length = gcd of the members' pc_every, else
 * a free length), ortho inside the kernel.
 * Limits: single-determinant trials, local-energy weights, M <= 64,
 * N_sigma <= M, and a walker's arrays plus the system's operators (L, Ltil,
 * B1, D_0, htil, lbar, staged in LDS once per segment) within one CU's LDS:
 * about 8 (n_chol (M^2 + M N) + 3 M^2 + 10 M N + 14 n_chol) bytes with
 * N = N_up + N_dn, so tiny systems (M = 10, N = 10, 40 vectors: 77 KB;
 * afqmc_resident_supported tells). 
 * The walker buffers of each member must keep their addresses while the
 * group exists.  At most 64 members, all on one device. */
typedef struct afqmc_group afqmc_group;
typedef struct {
  afqmc_ham *ham;
  afqmc_trial *trial;
  afqmc_walkers *walkers;
  double dt;
  uint64_t seed;
  afqmc_options opt;
} afqmc_group_member;

/* *ok = 1 if the trial's system fits the walker-resident kernel. */
afqmc_status afqmc_resident_supported(const afqmc_trial *trial, int *ok);

/* Builds a group (B1 per member, device tables, comb buffers).  Launch shape:
 * the tuning cache's entry for the group's shape signature (device, sorted
 * member shapes, segment rule), else 256 threads per walker block. */
afqmc_status afqmc_group_create(afqmc_group **out, int n_members,
                                const afqmc_group_member *members, void *stream);

/* n_steps steps of every member, global step indices step0 .. step0 +
 * n_steps - 1 (one field stream per member: its seed and system_id).  The
 * call first refreshes logovlp, eloc and the force-bias traces from phi.
 * emix_dev (nullable) holds n_members device pointers (each nullable) that
 * receive the member's E_mix after each step, as afqmc_propagate's emix_dev. */
afqmc_status afqmc_group_propagate(afqmc_group *group, int n_steps, uint64_t step0,
                                   double *const *emix_dev, void *stream);

/* Autotuner: times `steps` steps (at least two segments) of the group for each
 * launch shape (threads per walker block 64/128/256/512; segment length
 * 10/20/50 when no member combs), from the same saved walker state each time,
 * restores the state, keeps the fastest shape and writes it to the tuning
 * cache (if a cache path is set).  us_per_step (nullable) gets its time. */
afqmc_status afqmc_group_tune(afqmc_group *group, int steps, double *us_per_step, void *stream);
afqmc_status afqmc_group_config(const afqmc_group *group, int *threads, int *segment_steps,
                                int *tuned /* 0 default, 1 measured, 2 cached */);
afqmc_status afqmc_group_set_config(afqmc_group *group, int threads, int segment_steps);
/* Kernel timing of the resident kernel: while enabled, segments are launched
 * directly (not as graphs) with HIP events around each resident launch on
 * the call's stream; timing_read (synchronises) returns and clears the
 * launches, the steps they covered and their total time. */
afqmc_status afqmc_group_timing(afqmc_group *group, int enable);
afqmc_status afqmc_group_timing_read(afqmc_group *group, int64_t *launches, int64_t *steps,
                                     double *total_ms);
void afqmc_free_group(afqmc_group *group);

/* JSON file the autotuner reads and writes (NULL or "": none; default: the
 * environment variable AFQMC_TUNE_CACHE). */
afqmc_status afqmc_tune_cache_path(const char *path);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the comb of
 * afqmc_reconfigure, same arguments and results (bitwise), with its scratch
 * (prefix sums, parents, norm factor, gather snapshot) in a static device
 * array of AFQMC_NOALLOC_SCRATCH_BYTES per device instead of the walker
 * workspace; the workspace must still be passed (it holds the walkers'
 * force-bias traces).  Allocates nothing (no hipMalloc, hipFree or library
 * allocation).  AFQMC_ERR_ARG when the walker count does not fit the array
 * (n_walkers * 20 bytes + 768 bytes > AFQMC_NOALLOC_SCRATCH_BYTES); any
 * walker shape fits (the snapshot is taken column range by column range).
 * Every call on one device shares that device's array: calls that overlap on
 * one device race.  The array lives until the process ends. */
#define AFQMC_NOALLOC_SCRATCH_BYTES (32u << 20)
afqmc_status afqmc_reconfigure_noalloc(afqmc_trial *trial, afqmc_walkers *walkers, uint64_t seed,
                                       uint64_t pc_index, double *norm_factor_host, void *stream);

/* The auxiliary fields afqmc_propagate draws at global step t:
 * x_dev [n_walkers][n_chol] device float64. */
afqmc_status afqmc_fields(uint64_t seed, uint64_t t, int n_walkers, int n_chol,
                          int system_id, double *x_dev, void *stream);

/* Kernel timing.  For each class whose bit is set in class_mask (bit c for
 * class c, 0 turns timing off), every launch of the kernels of that class
 * made by this Hamiltonian's calls is bracketed by a pair of HIP events
 * recorded on the launch stream (events are created when timing is turned
 * on, not per launch).  Classes: 0 exchange (the per-vector L~ Theta
 * contraction with the force-bias traces, or the Q route's quadratic form),
 * 1 propagator build sum_g c_g L_g, 2 Taylor and B1 products, 3 overlap /
 * inverse / Theta, 4 MGS, 5 comb, 6 other per-walker kernels, 7 force-bias
 * GEMM (Q route and the hybrid form's steps without an E_L measurement).
 * afqmc_timing_read synchronises on the recorded events, returns the number
 * of timed launches and their summed duration in milliseconds for one class,
 * and clears that class. */
#define AFQMC_NUM_KERNEL_CLASSES 8
afqmc_status afqmc_timing_enable(afqmc_ham *ham, int class_mask);
afqmc_status afqmc_timing_read(afqmc_ham *ham, int kernel_class, int64_t *launches,
                               double *total_ms);

/* Statistics of energy series, on the host (host pointers, no device work,
 * no stream).  afqmc_reblock: blocking analysis of a correlated series x[n]
 * (finite values, n >= 2), used for the error bars of long population-
 * controlled runs (Sec. II remark; Flyvbjerg-Petersen blocking).  Level 0 is
 * the series, level k+1 averages neighbouring pairs of level k (an odd last
 * value is dropped), levels continue while they hold >= 2 values, at most
 * max_levels.  *mean = mean of the whole series; sem[k] (caller-allocated,
 * max_levels) = sqrt(s_k^2 / n_k) with the unbiased variance s_k^2 of level
 * k; *plateau = the first level k with sem[k+1] - sem[k] <= sem[k] /
 * sqrt(2 (n_k - 1)), or -1.  AFQMC_ERR_NONFINITE for a non-finite value.
 *
 * afqmc_cs_difference: correlated sampling (Sec. I, Sec. V: two systems
 * propagated with the same fields, i.e. the same seed and system id, in
 * independent repeats).  a, b: [repeats][steps] energy series (NaN where a
 * step has no measurement); per repeat the cumulative average of b - a from
 * step `first` on over the steps where both are finite; mean[t] and sem[t]
 * (caller-allocated [steps]) are its mean over the repeats and the standard
 * error of that mean (NaN before the first finite step, sem NaN for one
 * repeat). */
afqmc_status afqmc_reblock(const double *x, int n, int max_levels, double *mean, double *sem,
                           int *n_levels, int *plateau);
afqmc_status afqmc_cs_difference(const double *a, const double *b, int repeats, int steps,
                                 int first, double *mean, double *sem);

void afqmc_free_hamiltonian(afqmc_ham *ham);
void afqmc_free_trial(afqmc_trial *trial);

/* Message of the last failed call on this thread ("" if none). */
const char *afqmc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* AFQMC_H */
