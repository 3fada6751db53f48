/*
 * gbs_mpo.h -- C ABI of the MI355X (gfx950) lossy Gaussian boson sampling
 * matrix-product-operator simulator.
 *
 * Method: Liu, Oh, Liu, Jiang, Alexeev, "Simulating lossy Gaussian boson
 * sampling with matrix product operators" (arXiv 2301.12814).
 *
 * State.  The vectorised density operator |rho>> (Sec. II, vectorisation map)
 * of M optical modes is held in U(1)-symmetric Vidal form (App. D, charged
 * MPS): site matrices Gamma_j (mode j, no physical index), Schmidt values
 * lam_b and photon-number charges c_b = (n, n') on bonds b = 0..M, where
 * c_b counts the ket and bra photons in modes b..M-1 (App. D counts the
 * photons on the right of a bond).  Bond 0 is an auxiliary leg that carries
 * the total photon numbers (App. A).
 * Each mode has a per-mode Fock cutoff d (local index [0, d)^2, ket x bra).
 *
 * Conventions.
 *   * Modes are 0-based.  A gate "on left_site k" acts on modes (k, k+1).
 *   * Beam splitter T(theta, phi) = [[e^{i phi} cos t, -sin t],
 *                                    [e^{i phi} sin t,  cos t]],
 *     acting on creation operators as a^dag_j -> sum_i T[i][j] a^dag_i
 *     (App. B, creation-operator transform); rho -> U rho U^dag.
 *   * Truncation: singular values below 1e-14 of the largest are dropped;
 *     the i-th values of mirror charges (n, n') and (n', n) form one unit of
 *     size 2 (Hermiticity makes the spectra equal), self-mirror charges give
 *     units of size 1; units are kept by decreasing value (ties: charge, then
 *     rank) while the running size stays <= chi.  New bonds are ordered by
 *     charge, then by decreasing value.
 *
 * Ownership.  The caller owns every host buffer: inputs are read before the
 * call returns, outputs are written to caller memory.  A handle owns all its
 * device memory until mpo_free.  A handle is not thread-safe; distinct handles
 * may be used from distinct threads on distinct streams.
 *
 * Errors.  Every call returns MPO_OK or a negative code and sets a
 * thread-local message (mpo_last_error).  Argument errors leave the state
 * unchanged.  A numerical failure found on the device (non-converged SVD,
 * non-finite values, workspace overflow) is latched and returned by the next
 * synchronising call (mpo_entropy, mpo_photon_marginals, mpo_sync,
 * mpo_get_bond) or by the next layer.
 */
#ifndef GBS_MPO_H
#define GBS_MPO_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gbs_mpo gbs_mpo;

enum {
  MPO_OK = 0,
  MPO_EINVAL = -1,   /* invalid argument; state unchanged                    */
  MPO_ENOMEM = -2,   /* projected device memory exceeds the budget / alloc   */
  MPO_EDEVICE = -3,  /* HIP runtime error                                    */
  MPO_ENUMERIC = -4, /* latched device-side numerical failure                */
  MPO_EBUSY = -5
};

enum { MPO_FP64 = 0, MPO_MIXED = 1 };

/*
 * Initial lossy squeezed product state (Sec. II: uniform loss commutes with
 * the interferometer and is applied to the input; App. C: squeezed-vacuum
 * wavefunction; App. B: pure-loss Kraus operators).
 *   M        number of modes, M >= 2
 *   r        host array [M], squeezing per mode, r >= 0 (0 = vacuum input)
 *   eta      uniform transmission, 0 < eta <= 1
 *   d        per-mode Fock cutoff, 2 <= d <= 16
 *   chi      bond dimension, 1 <= chi <= 4096
 *   precision MPO_FP64, or MPO_MIXED: the block SVDs' Jacobi rotations run in
 *            FP32 on operands normalised to unit norm, everything else in FP64,
 *            kept singular values and vectors refined in FP64 (faster, less
 *            accurate: about 1e-7 relative on the kept vectors per gate)
 *   hip_stream  hipStream_t to run on (created with the HIP runtime this library links),
 *               or NULL for a stream owned by the handle
 *   out      receives the new handle
 * Each mode's state is built in a large internal Fock space, lossy, then
 * cropped to [0, d)^2 (no renormalisation).  The exact product Vidal form is
 * truncated to the top-chi charges of every bond by the rule above.
 */
int mpo_init_lossy_squeezed(int M, const double *r, double eta, int d, int chi,
                            int precision, void *hip_stream, gbs_mpo **out);

/*
 * Same, with the cutoff read as a cap on the TOTAL photon number (App. A: the
 * leftmost charge counts every photon, and the cutoff d bounds it): the
 * initial state is projected onto at most d - 1 photons in ket and in bra
 * over all modes (exact Vidal form of the projection, then the top chi per
 * bond).  Every bond charge then stays <= (d-1, d-1); the interferometer
 * conserves photon number, so no gate leaks trace and 1 - Tr rho measures
 * the bond truncation alone.  Arguments as above.
 */
int mpo_init_lossy_squeezed_total_cap(int M, const double *r, double eta, int d, int chi,
                                      int precision, void *hip_stream, gbs_mpo **out);

/*
 * One layer of disjoint nearest-neighbour beam splitters (App. D two-site
 * update with charge-blocked Theta(c), Eq. theta; per-sector SVD truncated to
 * chi; App. D.5 block SVD).  Gates must be disjoint: no two share a mode.
 *   left_site[g] in [0, M-2]; theta[g], phi[g] as in T(theta, phi).
 * Also updates the operator EE of each updated bond and the running maximum.
 * Host waits: the sector sizes are data dependent, so the call waits for the
 * device once after the planner's count pass (to size the workspaces) and,
 * while large sectors are still in their panel Jacobi rounds, once every 16
 * rounds (to compact the still-rotating sectors); everything else is enqueued
 * on the handle's stream.  Every workspace is sized before the first new
 * tensor is written, so an EINVAL / ENOMEM return leaves the state unchanged.
 */
int mpo_apply_bs_layer(gbs_mpo *h, int n_gates, const int *left_site,
                       const double *theta, const double *phi);

/* Output phase screen D: |n> -> e^{i n phase[j]} |n> on every mode j (any local
 * unitary of the vectorised map, Sec. II).  Leaves lam, charges, EE unchanged. */
int mpo_apply_phases(gbs_mpo *h, const double *phase);

/*
 * Operator entanglement entropy S_b = -sum p log2 p, p = lam^2 / sum lam^2
 * (Sec. II EE definition; App. B explicit normalisation, log base 2) on the
 * internal bonds b = 1..M-1.  S: host array [M-1]; S_max_so_far (nullable)
 * receives the maximum over bonds and over every layer applied so far.
 * Synchronises the handle's stream.
 */
int mpo_entropy(gbs_mpo *h, double *S, double *S_max_so_far);

/*
 * Photon-number marginals P[j*d + n] = Tr(rho Pi_{j,n}) / Tr rho and the trace
 * Tr rho (nullable), whose deficit 1 - Tr rho is the paper's error proxy
 * (Sec. III; App. A).  The trace contracts every site with the identity and
 * the auxiliary leg with the all-ones vector.  P: host array [M*d].
 * A truncated MPO need not be positive: at very small chi the trace can reach
 * zero or below, and P is then Tr(rho Pi) / Tr rho as computed (unnormalised
 * when Tr rho == 0).  MPO_ENUMERIC only for a non-finite trace.
 * Synchronises the handle's stream.
 */
int mpo_photon_marginals(gbs_mpo *h, double *P, double *trace);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as mpo_photon_marginals, computed by the same kernels, with every
 * intermediate (trace environments, partial sums, raw marginals, trace) in a
 * static device array of 16 MiB that the library holds on each GPU it runs on
 * until the process ends.  Calls no hipMalloc / hipFree and no allocating
 * library routine.  The state needs 2 (M+1) chi 16 + M d ceil(chi/4) 8 +
 * M d 8 + 8 bytes (each part rounded up to 256); a larger state returns
 * MPO_EINVAL.  All calls on one GPU share that array: calls that overlap on
 * one GPU (from several threads or streams) race.  Synchronises.
 */
int mpo_photon_marginals_noalloc(gbs_mpo *h, double *P, double *trace);

/*
 * Renyi-alpha operator entropies S_b = log2(sum p^alpha) / (1 - alpha) of the
 * same normalised spectra p = lam^2 / sum lam^2 as mpo_entropy (Sec. III.B and
 * App. B: Renyi entropies of the vectorised state), on bonds b = 1..M-1, in
 * bits.  alpha >= 0; alpha = 1 gives the EE, alpha = 0 log2 of the bond size.
 * S: host array [M-1].  Synchronises.
 */
int mpo_renyi(gbs_mpo *h, double alpha, double *S);

/*
 * Asymptotic estimate of the operator EE from a single input mode (App. C;
 * no device state needed).  A squeezed vacuum of squeezing r with loss
 * transmission mu, both the state and the Kraus operators on photon numbers
 * 0..n_max, is split by the basis transform of App. B (Eq. transform) with
 * cos(theta) on the up side and sin(theta) on the down side (App. C:
 * theta = pi/4 for the middle cut of a large Haar interferometer); the
 * entropy (alpha = 1) or Renyi-alpha entropy of the vectorised output
 * operator across the up/down cut, times n_inputs, is written to *S (bits).
 *   0 <= r <= 20, 0 < mu <= 1, 1 <= n_max <= 31, n_inputs >= 0, alpha >= 0
 *   spectrum (nullable) host [(n_max+1)^2]: the normalised eigenvalues of the
 *            reduced operator (unsorted)
 * Runs one workgroup on the current device (its own stream, synchronised;
 * temporary device buffers of 8 (n_max+1)^4 bytes).  MPO_ENUMERIC if its
 * Jacobi SVD does not converge.
 */
int gbs_asymptotic_ee(double r, double mu, int n_max, double theta, int n_inputs, double alpha,
                      double *S, double *spectrum);

/*
 * Experiment drivers (App. A), host orchestration of the calls above.
 *
 * EE-saturation stop rule: the initial state (arguments as
 * mpo_init_lossy_squeezed) is evolved through the Clements layers of U
 * (U_reim as in gbs_clements_decompose) one layer at a time; after each layer
 * the largest bond EE is read, and the run stops once it has not exceeded the
 * best value so far by more than 1e-12 bits for `patience` consecutive layers
 * (10 in App. A), or when the layers run out.  Outputs: layers applied, the
 * maximum EE (bits) and the layer count at which it was reached, and the
 * trace at the stop (nullable).
 */
int gbs_run_until_saturation(int M, const double *r, double eta, int d, int chi, int precision,
                             const double *U_reim, int patience, int *layers_used,
                             double *S_max, int *layer_of_max, double *trace);

/*
 * Fixed-accuracy bond-dimension search (App. A): the whole circuit of U is
 * run at chi0, chi is doubled (capped at chi_max) while 1 - Tr rho exceeds
 * `target`, then `refine` bisection runs between the last failing and the
 * first passing chi narrow the estimate.  *chi_found = the smallest passing
 * chi found (-1 if chi_max fails), *err_found = its 1 - Tr rho (or that of
 * chi_max).  The first max_trials runs are listed in trial_chi / trial_err
 * (host arrays, nullable when max_trials = 0), their count in *n_trials
 * (nullable).
 */
int gbs_chi_search(int M, const double *r, double eta, int d, int precision,
                   const double *U_reim, int chi0, int chi_max, double target, int refine,
                   int *chi_found, double *err_found, int max_trials, int *n_trials,
                   int *trial_chi, double *trial_err);

/* Waits for the handle's queued work; returns a latched device error if any. */
int mpo_sync(gbs_mpo *h);

/*
 * Inspection of bond b in 0..M (synchronises).  dim receives the bond size D;
 * lam [chi] and charges [2*chi] (n, n' pairs, nullable) receive the first D
 * entries, ordered by charge then decreasing value.
 */
int mpo_get_bond(gbs_mpo *h, int b, int *dim, double *lam, int *charges);

/*
 * Copy of site matrix Gamma_j (j in 0..M-1), D_j x D_{j+1}, row-major,
 * interleaved (re, im) doubles, into host buffer G [2 * chi * chi]
 * (leading dimension D_{j+1}).  Synchronises.
 */
int mpo_get_site(gbs_mpo *h, int j, double *G);

/*
 * Per-layer statistics of the last applied layer (synchronises):
 * stats[0] = number of sector blocks, stats[1] = sum over blocks of r*s,
 * stats[2] = sum of candidate singular values, stats[3] = largest block rows,
 * stats[4] = largest block cols, stats[5] = Jacobi sweeps of the slowest block.
 */
int mpo_layer_stats(gbs_mpo *h, long long *stats);

/*
 * Phase profiling (tracing).  mpo_set_profiling(h, 1) enables HIP events
 * around each phase of every subsequent layer and resets the accumulators
 * (0 disables).  Synchronises.
 */
int mpo_set_profiling(gbs_mpo *h, int enable);

/*
 * Accumulated profile since profiling was enabled (synchronises):
 *   phase_ms[8] (nullable): summed device time per phase, in milliseconds:
 *     0 Fock tables, 1 sector planning, 2 Theta contraction, 3 block SVD,
 *     4 truncation select, 5 zero + scatter, 6 entropy, 7 unused
 *   phase_launches[8] (nullable): layers timed per phase
 *   work[4] (nullable): [0] SVD work sum over blocks of 16 m n^2 + 36 n^3 real
 *     flops (complex m x n block, m >= n), [1] sector elements sum r*s,
 *     [2] candidate singular values, [3] layers.
 */
int mpo_get_profile(gbs_mpo *h, double *phase_ms, long long *phase_launches, double *work);

/*
 * Algorithmic work of the Theta contractions (App. D, Eq. theta) summed over
 * the layers applied since profiling was enabled, in real flops: 8 per
 * (a, alpha, b) term whose two local pairs c_a - c_alpha and c_alpha - c_b are
 * valid, plus 8 m_ket m_bra (m_ket + m_bra) per (a, b) for the Fock weights
 * applied factorised (m = valid splits of the two-mode photon number in ket /
 * bra).  No padding and no Hermitian-mirror saving are counted.
 * Synchronises.
 */
int mpo_get_contraction_work(gbs_mpo *h, double *flops);

/*
 * Sector histogram of the last applied layer (synchronises; still answers
 * after a latched numeric error, which it does not report).  For each block
 * Theta(q) of every gate, 8 ints: gate index in the layer, q = (n, n'), rows r,
 * cols s, computed here (1) or derived from its mirror (0), Jacobi sweeps,
 * singular vectors kept.  out: host [8 * max_blocks]; returns the total number
 * of blocks (may exceed max_blocks; only the first max_blocks are written).
 */
int mpo_layer_blocks(gbs_mpo *h, int max_blocks, int *out);

/* Process-wide routing of the block SVDs (App. D: every charge block is
 * SVD'd; these knobs only choose which kernels do it, the results agree to
 * rounding).  lds_limit_bytes > 0 lowers the LDS budget below the device's:
 * a block whose Jacobi operand exceeds it takes the multi-workgroup panel
 * rounds (in FP64 so does every block of at least 48 columns).  With
 * qr_enable != 0 a block exceeding it, or with at least 16
 * columns, is first reduced by a Householder QR with column pivoting;
 * qr_enable = 0 runs every Jacobi on the block itself.  lds_limit_bytes = 0
 * restores the device budget.  Affects layers planned after the call; not
 * thread-safe. */
int gbs_set_svd_route(int lds_limit_bytes, int qr_enable);

/* Free and total bytes of the current device's memory (hipMemGetInfo), for
 * callers that size admission budgets.  MPO_EDEVICE on a runtime error. */
int gbs_device_memory(long long *free_bytes, long long *total_bytes);

/* Releases every device allocation of the handle (NULL is a no-op). */
void mpo_free(gbs_mpo *h);

/*
 * ---------------------------------------------------------------------------
 * Batched and continuously batched simulations.
 *
 * An engine holds any number of simulations resident in HBM.  Every step
 * applies the next beam-splitter layer of every running simulation in one
 * batched launch sequence: the sector contractions, block SVDs, truncations
 * and scatters of all their gates run in the same kernels (App. D, the
 * two-site update of each gate is independent of every other gate of the
 * layer).  Simulations may be added at any step (continuous batching); a
 * simulation whose last layer was applied is retired: its operator EE maximum,
 * trace and photon marginals are stored and its device memory released.
 * A simulation's results do not depend on which other simulations share its
 * steps.  An engine is not thread-safe.
 * ---------------------------------------------------------------------------
 */
typedef struct gbs_engine gbs_engine;

/* Projected device bytes a simulation of this shape is admitted against
 * (its state plus its share of the per-layer sector workspace); -1 on bad
 * arguments. */
long long mpo_engine_projected_bytes(int M, int d, int chi);

/* New engine on hip_stream (NULL: own stream).  budget_bytes = admission
 * budget in bytes, 0 for 85% of the currently free HBM. */
int mpo_engine_create(void *hip_stream, int precision, long long budget_bytes, gbs_engine **out);

/* Admits one simulation: arguments as mpo_init_lossy_squeezed plus the
 * interferometer U (host [2*M*M], row-major, interleaved re/im), decomposed on
 * the host into Clements layers.  Returns MPO_ENOMEM (state unchanged) when
 * the projected bytes do not fit the remaining budget.  *id receives the
 * simulation id. */
int mpo_engine_add(gbs_engine *e, int M, const double *r, double eta, int d, int chi,
                   const double *U_reim, int *id);

/* One step: the next layer of every running simulation; finished ones are
 * retired.  *n_active (nullable) receives the number still running. */
int mpo_engine_step(gbs_engine *e, int *n_active);

/* Results of simulation id: *done = 1 once retired, then S_max (EE maximum over
 * bonds and layers, bits), trace (Tr rho) and P [M*d] (nullable each). */
int mpo_engine_result(gbs_engine *e, int id, int *done, double *S_max, double *trace,
                      double *P);

/* Forgets a retired simulation (MPO_EBUSY while it runs). */
int mpo_engine_release(gbs_engine *e, int id);

/* Failure injection for tests of failure isolation: lowers the Jacobi sweep
 * limit (normally 60) of every block SVD of one running simulation to
 * max_sweeps in [1, 60].  A block that has not converged within it latches
 * MPO_ENUMERIC on that simulation only (every kernel still exits normally);
 * the engine retires it with that error at the end of the step, and the other
 * simulations of the batch are unaffected.  Takes effect at the next step. */
int mpo_engine_set_sweep_limit(gbs_engine *e, int id, int max_sweeps);

/* Phase profiling of the engine's steps (same layout as mpo_get_profile). */
int mpo_engine_set_profiling(gbs_engine *e, int enable);
int mpo_engine_get_profile(gbs_engine *e, double *phase_ms, long long *phase_launches,
                           double *work);

/* Releases the engine and every simulation it holds. */
void mpo_engine_free(gbs_engine *e);

/* Thread-local message of the last failing call on this thread. */
const char *mpo_last_error(void);

/*
 * Host-only helper (no device work): Clements rectangular decomposition of an
 * interferometer into M(M-1)/2 beam splitters on neighbouring modes plus an
 * output phase screen (App. A M-layer array; Clements et al., Optica 2016),
 * grouped into as-soon-as-possible layers of disjoint gates.
 *   U_reim     host [2*M*M], U[i][j] row-major, interleaved (re, im); must be
 *              unitary to 1e-10
 *   layer_ptr  host [M+1]: gates of layer l are [layer_ptr[l], layer_ptr[l+1])
 *   left_site, theta, phi  host [M(M-1)/2], in application order
 *   phase      host [M], D = diag(e^{i phase})
 * Returns the number of layers (>= 0) or a negative error code.
 * U = D * T_L * ... * T_1 with theta in [0, pi/2], phi in (-pi, pi].
 */
int gbs_clements_decompose(int M, const double *U_reim, int *layer_ptr, int *left_site,
                           double *theta, double *phi, double *phase);

#ifdef __cplusplus
}
#endif
#endif /* GBS_MPO_H */
