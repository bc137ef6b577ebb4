/*
 * gocp.h -- C ABI of the MI355X (gfx950) GOCP ADAPT-VQE hot path.
 *
 * The library maps a molecular Hamiltonian to Pauli strings, builds the
 * excitation pool, partitions it into commuting families, and runs the
 * statevector work of adaptive VQE on the GPU: energies, the gradient screen
 * over the whole pool, and the fifth-order Taylor state update.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Qubit q is bit q of a basis index; |1> means occupied.  Spin-orbital /
 *   qubit 2p+s is spatial orbital p with spin s (0 alpha, 1 beta).
 * - A Pauli term is stored in folded form: bit masks (x, z) and a real
 *   coefficient c such that the term maps psi to
 *       (c P psi)[d] = c * (-1)^popcount(d & z) * psi[d ^ x].
 *   This equals c_std * P(x, z) with P(x, z) the tensor product of I, X, Z, Y
 *   (Y = iXZ) and c_std = c * i^popcount(x & z).
 * - Statevectors are caller-owned device buffers of 2^n interleaved complex
 *   numbers: GOCP_C128 = (double re, double im), GOCP_C64 = (float re,
 *   float im).  Work with GOCP_C64 keeps every accumulation, reduction,
 *   renormalisation and selection in FP64.
 * - Every call returns GOCP_OK (0) or a negative status; gocp_last_error()
 *   returns a thread-local message for the last failure.  No call throws.
 * - Host input arrays are copied during the call; output arrays are
 *   caller-allocated.  Handles (ham, pool) are immutable after creation,
 *   may be shared between threads, and are freed by their *_free call.
 * - Calls on a context are ordered on that context's HIP stream.  Calls that
 *   return host values synchronise that stream before returning.
 * - Host-only calls (Hamiltonian load, pool build, partition, queries) touch
 *   no GPU and work on hosts without one.
 */
#ifndef GOCP_H
#define GOCP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GOCP_OK        0
#define GOCP_EINVAL   -1   /* bad argument (null pointer, out-of-range value)   */
#define GOCP_ENOMEM   -2   /* host or device allocation failed                  */
#define GOCP_EDEVICE  -3   /* HIP runtime error, or no usable gfx950 device     */
#define GOCP_ESHAPE   -4   /* qubit counts of handles / buffers disagree        */
#define GOCP_ENOTSUP  -5   /* outside supported sizes (1..30 qubits)            */
#define GOCP_EBUSY    -6   /* serving: request not finished yet                 */
#define GOCP_ENUMERIC -7   /* a non-finite value was produced                   */
#define GOCP_ECANCELED -8  /* serving: request cancelled by server shutdown     */

#define GOCP_JW 0          /* Jordan-Wigner                                     */
#define GOCP_BK 1          /* Bravyi-Kitaev (Fenwick-tree encoding)             */

#define GOCP_C128 0        /* complex128 statevector                            */
#define GOCP_C64  1        /* complex64 statevector, FP64 accumulation          */

typedef struct gocp_ctx gocp_ctx;
typedef struct gocp_ham gocp_ham;
typedef struct gocp_pool gocp_pool;
typedef struct gocp_batch gocp_batch;
typedef struct gocp_server gocp_server;

/* Thread-local text of the last error (never NULL). */
const char *gocp_last_error(void);
/* Library version as an integer, major*10000 + minor*100 + patch. */
int gocp_version(void);

/* ======================================================================
 * Host-only calls
 * ==================================================================== */

/*
 * pauli_hamiltonian_load -- Eq. 2 to Eq. 3 (Sec. II.A).
 * Builds H = e_core + sum_PQ h_PQ a+_P a_Q + 1/2 sum_PQRS <PQ|RS> a+_P a+_Q a_S a_R
 * over 2*n_spatial spin-orbitals, with <PQ|RS> = (pr|qs) for matching spins,
 * and maps it with `mapping` (GOCP_JW or GOCP_BK) to a sum of folded Pauli
 * terms.  Terms whose coefficient magnitude is below 1e-12 are dropped.
 *   h1  : n_spatial*n_spatial FP64, row-major h[p][q], symmetric.
 *   eri : n_spatial^4 FP64, row-major (pq|rs) in chemist order.
 * Errors: EINVAL (null pointers, n_spatial < 1), ENOTSUP (2*n_spatial > 30).
 */
int pauli_hamiltonian_load(int n_spatial, const double *h1, const double *eri,
                           double e_core, int mapping, gocp_ham **out);

/*
 * Wrap an explicit folded Pauli sum (x[i], z[i], c[i]), i < n_terms, on
 * n_qubits qubits.  Like terms are combined; |c| < 1e-12 terms dropped.  The
 * sum must be a real symmetric matrix (every term with popcount(x&z) even).
 * Errors: EINVAL (odd-Y term, null pointers), ENOTSUP (n_qubits > 30).
 */
int pauli_hamiltonian_load_terms(int n_qubits, int64_t n_terms, const uint32_t *x,
                                 const uint32_t *z, const double *c, gocp_ham **out);

/* Sizes: qubits, Pauli terms, distinct X masks (classes).  Any output may be NULL. */
int gocp_ham_info(const gocp_ham *h, int32_t *n_qubits, int64_t *n_terms, int32_t *n_classes);

/*
 * Copy the terms, sorted by (x, z), into caller arrays of length >= capacity.
 * Errors: EINVAL if capacity < n_terms (query n_terms with gocp_ham_info).
 */
int gocp_ham_terms(const gocp_ham *h, int64_t capacity, uint32_t *x, uint32_t *z, double *c);
int gocp_ham_free(gocp_ham *h);

/*
 * pool_build -- the operator pool (Sec. II.B; sizes of Table II).
 * Spin-conserving occupied -> virtual singles tau = a+_a a_i and doubles
 * tau = a+_a a+_b a_j a_i (i<j occupied, a<b virtual, equal S_z), occupied
 * spin-orbitals 0..n_electrons-1; generator A = tau - tau^+ mapped with
 * `mapping`.  Order: singles by (i, a), then doubles by (i, j, a, b).
 * Every generator has one X mask and 2 (single) or 8 (double) strings.
 * Errors: EINVAL (n_electrons odd, <= 0 or >= n_qubits), ENOTSUP (> 30 qubits).
 */
int pool_build(int n_qubits, int n_electrons, int mapping, gocp_pool **out);

/*
 * pool_build_pauli -- the Pauli (qubit) pool of the same excitations: every
 * string of every pool_build generator (Sec. II.B, mapped as in Eq. 3) becomes
 * an operator of its own, B = sign(c) Z^z X^x with unit coefficient (anti-
 * Hermitian, B^2 = -1, so the line search and the Taylor chain of Sec. III.B
 * apply unchanged).  Order: generators in pool_build order, each one's strings
 * by ascending Z mask; M = S = 2 singles + 8 doubles.  gocp_pool_op reports
 * kind 3 (string of a single) or 4 (string of a double) with the parent's
 * indices.  Caller owns the handle (gocp_pool_free).  Errors as pool_build.
 */
int pool_build_pauli(int n_qubits, int n_electrons, int mapping, gocp_pool **out);

/* Sizes: qubits, operators M, total strings S.  Any output may be NULL. */
int gocp_pool_info(const gocp_pool *p, int32_t *n_qubits, int32_t *n_ops, int32_t *n_strings);

/* Operator k: kind (1 single, 2 double; 3, 4 one string of either, from
 * pool_build_pauli), spin-orbital indices (i, a, -1, -1) or (i, j, a, b), and
 * its X mask.  Errors: EINVAL if k is out of range. */
int gocp_pool_op(const gocp_pool *p, int32_t k, int32_t *kind, int32_t idx[4], uint32_t *xmask);

/* All strings: op_offsets[M+1] (CSR), z[S], c[S] folded coefficients; x per op
 * via gocp_pool_op.  Arrays caller-allocated with the sizes from gocp_pool_info. */
int gocp_pool_strings(const gocp_pool *p, int32_t *op_offsets, uint32_t *z, double *c);
int gocp_pool_free(gocp_pool *p);

/*
 * gocp_partition -- Greedy Operator Commutativity Partitioning (Sec. III.A,
 * Algorithm 1).  Edge (i, j) iff the operator commutator [A_i, A_j] != 0,
 * evaluated exactly in integer arithmetic.  Vertices are visited by
 * descending degree (ties: ascending pool index) and each joins the
 * lowest-indexed family (creation order) that holds none of its neighbours,
 * else opens a new family.  Bit-exact and deterministic.
 *   family_of : M int32 outputs (family index of each operator).
 *   n_families: output K.
 *   order     : optional M int32 outputs, the visit order (may be NULL).
 */
int gocp_partition(const gocp_pool *p, int32_t *family_of, int32_t *n_families, int32_t *order);

/* Number of conflict-graph edges and the degree of each operator (deg may be NULL). */
int gocp_conflict_degrees(const gocp_pool *p, int64_t *n_edges, int32_t *deg);

/*
 * Basis index of the Hartree-Fock reference: occupations of spin-orbitals
 * 0..n_electrons-1, encoded with `mapping` (BK: b = beta n over GF(2)).
 */
int gocp_hf_index(int n_qubits, int n_electrons, int mapping, uint64_t *index);

/*
 * Parity-aware decoding (Sec. IV.B: tree encodings spread the occupation
 * parity over several qubits): the spin-orbital occupations of basis index
 * `index` under `mapping`, bit j = occupation of spin-orbital j (JW: the index
 * itself; BK: beta^{-1} index over GF(2), each occupation the parity of a set
 * of qubits).  gocp_basis_occupation(n, m, gocp_hf_index(n, ne, m)) is the
 * HF occupation 2^ne - 1 under both mappings.  Errors: EINVAL (index >= 2^n).
 */
int gocp_basis_occupation(int n_qubits, int mapping, uint64_t index, uint64_t *occupation);

/* ======================================================================
 * Device calls
 * ==================================================================== */

/*
 * Create a context on HIP device `device`, ordering its work on `stream`
 * (a hipStream_t; NULL selects the default stream).  The context owns its
 * scratch device memory and uploads each ham/pool once per device, on first
 * use.  One context per host thread.
 * Errors: EDEVICE (no such device or not gfx950).
 */
int gocp_ctx_create(int device, void *stream, gocp_ctx **out);
int gocp_ctx_destroy(gocp_ctx *ctx);
/* Change the stream of later calls (e.g. to torch's current stream). */
int gocp_ctx_set_stream(gocp_ctx *ctx, void *stream);
/* Block until all work queued on the context's stream has finished. */
int gocp_ctx_synchronize(gocp_ctx *ctx);
/* Phase trace of the energy+screen launch, for measurement (a library built
 * with GOCP_PHASE_TRACE defined; ENOTSUP from any other build).  Such a build
 * records, in every ADAPT-iteration launch of that kernel, the device's
 * constant-rate clock (100 MHz) at *n_phases = 6 points of each of its first
 * 1024 workgroups: entry, end of the prologue, H stage written, end of the H
 * walk in the workgroup's last wave, sigma and energy partials done, end of
 * the screen in the last wave; later launches overwrite earlier ones.
 * Synchronises the context stream, then copies n_rows x 6 values (row =
 * workgroup) to the caller's host array `out`.  Errors: EINVAL (null out,
 * n_rows outside 1..1024), ENOTSUP. */
int gocp_phase_trace(gocp_ctx *ctx, uint64_t *out, int32_t n_rows, int32_t *n_phases);

/* Write the basis state |index> into psi_dev (2^n_qubits amplitudes). */
int gocp_state_basis(gocp_ctx *ctx, int n_qubits, uint64_t index, void *psi_dev, int dtype);

/*
 * The encoded Hartree-Fock reference: |gocp_hf_index(...)> into psi_dev.
 */
int gocp_state_hf(gocp_ctx *ctx, int n_qubits, int n_electrons, int mapping, void *psi_dev, int dtype);

/*
 * Weight of a state inside the pool's symmetry sector under an encoding
 * (Sec. IV.B): sum |psi_d|^2 over the basis states d whose decoded occupation
 * (gocp_basis_occupation) holds n_electrons electrons, as many spin-up (even
 * spin-orbitals) as spin-down (odd), divided by <psi|psi> (FP64 sums in a
 * fixed order).  The pool's operators conserve both numbers, so a state with
 * weight 0 (for example an occupation bitstring used as a BK index without
 * encoding it) stays outside the sector: every ADAPT iteration from it is
 * decoupled from the sector's ground state.  Synchronises.
 * Errors: EINVAL, ENUMERIC (zero norm).
 */
int gocp_sector_weight(gocp_ctx *ctx, int n_qubits, int n_electrons, int mapping, const void *psi_dev, int dtype,
                       double *weight);

/*
 * energy -- Eq. 1: E = Re<psi|H|psi> / <psi|psi>, FP64, written to *e_out
 * (host).  Synchronises.  Errors: ESHAPE, ENUMERIC (zero or non-finite norm).
 */
int energy(gocp_ctx *ctx, const gocp_ham *h, const void *psi_dev, int dtype, double *e_out);

/*
 * sigma = H psi into sigma_dev (2^n complex128, FP64 accumulation), and the
 * energy as in `energy` into *e_out if e_out is not NULL (then synchronises).
 */
int gocp_apply_hamiltonian(gocp_ctx *ctx, const gocp_ham *h, const void *psi_dev, int dtype,
                           void *sigma_dev, double *e_out);

/*
 * pool_gradients -- Eq. 4 for every pool operator, no pruning:
 *   g_j = <psi|[H, A_j]|psi> / <psi|psi> = 2 Re<H psi|A_j psi> / <psi|psi>.
 * g_out: M FP64 values, on the host (g_on_device = 0; synchronises) or on the
 * device (g_on_device = 1; stream-ordered, no synchronisation).
 * The screen runs one pass per commuting family of the pool's partition.
 * Errors: ESHAPE (qubit counts differ).
 */
int pool_gradients(gocp_ctx *ctx, const gocp_ham *h, const gocp_pool *p, const void *psi_dev,
                   int dtype, double *g_out, int g_on_device);

/*
 * pool_gradients_noalloc -- for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same gradients as pool_gradients with g_on_device = 1,
 * computed by the same kernels into g_dev (M FP64 values, caller-owned device
 * memory), with the call's workspace in a fixed 8 MiB device array that the
 * library holds on each device until the process ends.  The call allocates
 * nothing: no hipMalloc, hipFree or allocating library routine.
 *   - The Hamiltonian's and the pool's tables must already be on the device
 *     (any earlier device call taking them, e.g. energy or pool_gradients,
 *     uploads them); otherwise EINVAL.
 *   - Problems whose workspace exceeds the array (about 2^n (48 + M / 8)
 *     bytes for complex128 states: every pool at 14 qubits, the full
 *     singles+doubles pool at 16) are rejected with ENOTSUP; use pool_gradients.
 *   - Every call on one device shares that device's array: calls that overlap
 *     on one device (on different streams or host threads) race and must be
 *     serialised by the caller.  Nothing in the array needs to start at zero.
 * Asynchronous on the context stream (no status check of the result).
 * Errors: EINVAL, ESHAPE, ENOTSUP as above.
 */
int pool_gradients_noalloc(gocp_ctx *ctx, const gocp_ham *h, const gocp_pool *p, const void *psi_dev,
                           int dtype, double *g_dev);

/*
 * taylor5_apply -- Eq. 5-6: psi <- T5(theta/s)^s psi / ||.||, in place, with
 * T5(x) = sum_{n=0..5} x^n/n! A_k^n evaluated as the chain v_n = A_k v_{n-1},
 * s = max(1, ceil(|theta| * ||A_k||_1 / 0.5)) substeps, and one FP64
 * renormalisation at the end.  theta == 0 leaves psi unchanged and reports
 * s = 0.  *n_substeps_out (may be NULL) receives s.  Stream-ordered.
 * Errors: EINVAL (k out of range, non-finite theta).
 */
int taylor5_apply(gocp_ctx *ctx, const gocp_pool *p, int32_t k, double theta, void *psi_dev,
                  int dtype, int32_t *n_substeps_out);

/*
 * taylor5_apply_family -- GOCP multi-operator step:
 *   psi <- prod_i T5(theta_i / s_i A_{ops[i]})^{s_i} psi,  then psi <- psi / ||psi||
 * once (FP64), with T5 and s_i as in taylor5_apply.  The operators are
 * members of one GOCP family (Sec. III.A, Algorithm 1: they commute, so the
 * product is order-free), each with its own substepped O(5) chain (Eq. 5-6,
 * s_i = max(1, ceil(|theta_i| ||A||_1 / 0.5)); theta_i = 0 skips it), all
 * applied in one pass over the state.
 *   n           : 1..4 operators; ops[n] pool indices, distinct, one family,
 *                 X masks linearly independent over GF(2); thetas[n] finite.
 *   psi_dev     : device state of the pool's qubit count, dtype GOCP_C128 or
 *                 GOCP_C64 (FP64 arithmetic either way), updated in place.
 *   n_substeps_out: optional n outputs (s_i, 0 for a zero angle).
 * Asynchronous on the context stream.  Errors: EINVAL (counts, indices,
 * repeats, families, angles, null pointers), ENOTSUP (dependent X masks, or
 * n equal to the qubit count).
 */
int taylor5_apply_family(gocp_ctx *ctx, const gocp_pool *p, int32_t n, const int32_t *ops,
                         const double *thetas, void *psi_dev, int dtype, int32_t *n_substeps_out);

/* ---------------------------------------------------------------------
 * ADAPT loop (Sec. II.B with the Sec. III.B update), device-resident.
 * One iteration: gradient screen, selection (largest |g_j|; gradients within
 * a relative 1e-12 of the largest tie and the lowest index wins), stop if
 * ||g||_2 < grad_tol, exact line minimisation of the energy along the chosen
 * generator with earlier angles frozen, the taylor5 update, new energy.
 * ------------------------------------------------------------------- */
typedef struct {
    double grad_tol;        /* stop when ||g||_2 < grad_tol (0: never)               */
    int32_t max_iter;       /* operators appended at most                            */
    int32_t use_graph;      /* 1: replay captured hipGraphs of the iteration         */
    int32_t schedule;       /* amplitudes per lane of the tile kernels, R = 1, 2
                               or 4, plus 256 x 4 to run the compacted H v, H w
                               launch (complex64 states) with 4 workgroups per
                               tile slot instead of 8; 0 = autotune (R timed on
                               the instances, the fastest kept and remembered
                               per qubit-count mix; 4 parts when 8 would give
                               that launch more than four workgroups per compute
                               unit).  Results depend on the schedule (the order
                               of FP64 sums), bit for bit                          */
    int32_t reserved;
} gocp_adapt_params;

typedef struct {
    int32_t n_iter;         /* operators appended                                    */
    int32_t converged;      /* 1 if stopped by grad_tol                              */
    double *energies;       /* caller array, max_iter+1: E_0 (start) .. E_n_iter     */
    int32_t *ops;           /* caller array, max_iter: chosen pool indices           */
    double *thetas;         /* caller array, max_iter: angles                        */
    double *gnorms;         /* caller array, max_iter+1: ||g||_2 of each screen      */
    double *gmax;           /* caller array, max_iter+1: largest |g_j| (may be NULL) */
    int32_t *substeps;      /* caller array, max_iter: Taylor substeps (may be NULL) */
} gocp_adapt_result;

/*
 * adapt_solve -- ADAPT from the state in psi_dev (normally the HF state),
 * updating psi_dev in place.  Synchronises; fills *res.
 * Errors: ESHAPE, EINVAL (max_iter < 0, null arrays), ENUMERIC.
 */
int adapt_solve(gocp_ctx *ctx, const gocp_ham *h, const gocp_pool *p, void *psi_dev, int dtype,
                const gocp_adapt_params *params, gocp_adapt_result *res);

/* ---------------------------------------------------------------------
 * ADAPT with full re-optimisation (textbook ADAPT, Sec. II.B): after each
 * appended operator every angle of the ansatz is optimised again, instead of
 * freezing the earlier ones.  The ansatz state is the chain of layers of
 * Eq. 5, psi(theta) = L_k(theta_k) ... L_1(theta_1) psi_0, each layer the
 * substepped O(5) Taylor propagator of Eq. 6 of its generator,
 * L = T5(theta/s)^s with s = max(1, ceil(max(|theta|, pi) ||A||_1 / 0.5))
 * (constant for |theta| <= pi, so the energy is smooth in the angles).  The
 * energy (Eq. 1) and its exact gradient come from one forward pass over the
 * layers (intermediate states kept on the device), H psi, and one adjoint
 * backward pass; BFGS (host) optimises the angles from the previous ones and
 * 0 for the new angle: direction -Hinv g, backtracking from step 1 by halving
 * until E decreases by 1e-4 t g.p (up to 1e-14 (1 + |E|) of rounding), the
 * update skipped when s.y <= 1e-12 |s| |y|; it stops when max |dE/dtheta| <
 * bfgs_gtol, after bfgs_max_iter steps or when the line search fails.  The
 * screen (Eq. 4) and the selection (as in adapt_solve) run on the optimised
 * state; convergence when ||g||_2 < grad_tol.
 * ------------------------------------------------------------------- */
typedef struct {
    double grad_tol;        /* stop when ||g||_2 < grad_tol (0: never)               */
    int32_t max_iter;       /* operators appended at most                            */
    int32_t bfgs_max_iter;  /* BFGS steps per re-optimisation (<= 0: 200)            */
    double bfgs_gtol;       /* BFGS stops at max |dE/dtheta| < bfgs_gtol (<= 0: 1e-8) */
} gocp_reopt_params;

typedef struct {
    int32_t n_iter;         /* operators appended                                    */
    int32_t converged;      /* 1 if stopped by grad_tol                              */
    double *energies;       /* caller array, max_iter+1: E at the optimised angles   */
    int32_t *ops;           /* caller array, max_iter: chosen pool indices           */
    double *thetas;         /* caller array, max_iter: the final angles, one a layer */
    double *gnorms;         /* caller array, max_iter+1: ||g||_2 of each screen      */
    int32_t *bfgs_steps;    /* caller array, max_iter: BFGS steps (may be NULL)      */
    int32_t *bfgs_evals;    /* caller array, max_iter: energy+gradient evaluations
                               (may be NULL)                                         */
} gocp_reopt_result;

/*
 * adapt_reopt_solve -- from the state in psi_dev (normally the HF state);
 * psi_dev receives the final normalised state.  Allocates its workspace
 * ((max_iter + 1) states of the dtype, two complex128 vectors) for the call.
 * Synchronises; fills *res.  Errors: ESHAPE, EINVAL (null arrays, max_iter
 * < 0), ENUMERIC.
 */
int adapt_reopt_solve(gocp_ctx *ctx, const gocp_ham *h, const gocp_pool *p, void *psi_dev, int dtype,
                      const gocp_reopt_params *params, gocp_reopt_result *res);

/* ---------------------------------------------------------------------
 * Batched form: many independent ADAPT problems advanced in lock-step.
 * Every kernel of an iteration is launched once for the whole batch over a
 * table of (instance, tile) work items, so instances of different qubit
 * counts share each launch; with use_graph the iteration (and a chunk of
 * eight iterations) is captured once and replayed as hipGraphs.  Each
 * instance computes exactly what adapt_solve computes for it alone.
 * ------------------------------------------------------------------- */

/*
 * Create a batch of n instances: hams[i], pools[i] (equal qubit counts per i)
 * and caller-owned device states psi_dev[i] (starting states, updated in
 * place), all of one dtype.  The library allocates each instance's device
 * workspace.  Evaluates the starting energies (stream-ordered).
 * Errors: EINVAL, ESHAPE, ENOMEM.
 */
int gocp_batch_create(gocp_ctx *ctx, int32_t n, const gocp_ham *const *hams,
                      const gocp_pool *const *pools, void *const *psi_dev, int dtype,
                      const gocp_adapt_params *params, gocp_batch **out);
/* Enqueue n_iter iterations for every instance (asynchronous).  Instances that
 * converged or reached max_iter skip their work. */
int gocp_batch_step(gocp_batch *b, int32_t n_iter);
/*
 * Measurement form of gocp_batch_step: n_iter iterations launched directly
 * (no graph) on the context stream, with HIP events that take the dispatch
 * timestamps (start and end, hipExtLaunchKernel) of one kernel of the
 * iteration (kernel: 0 selection and line-search vectors, 1 H v / H w (the
 * first launch's start to the second one's end), 2 angle and Taylor update,
 * 3 energy and screen partials, 4 their group sums) in iterations 0, every,
 * 2 every, ...  Waits for the work;
 * returns the elapsed time of all n_iter iterations and the mean duration of
 * the sampled launches (ms).  The iterations are the same as
 * gocp_batch_step's.  Errors: EINVAL.
 */
int gocp_batch_step_timed(gocp_batch *b, int32_t n_iter, int32_t kernel, int32_t every,
                          double *total_ms, double *kernel_ms);
/* Run the remaining iterations, stopping early once every instance is done. */
int gocp_batch_run(gocp_batch *b);
/* Synchronise and count the instances still running. */
int gocp_batch_poll(gocp_batch *b, int32_t *n_active);
/* Synchronise, renormalise instance i's state and copy its record into *res
 * (arrays sized as for adapt_solve).  Errors: EINVAL (i out of range). */
int gocp_batch_result(gocp_batch *b, int32_t i, gocp_adapt_result *res);
/*
 * Measurement hook: launch one kernel of the iteration n_launch times back to
 * back over the whole batch and return its mean duration from HIP events
 * recorded on the context stream.  which: 0 = per-tile energy and gradient
 * screen partials with a fresh H psi, 1 = H v / H w products of the line
 * search, 2 = the partials with sigma carried through the last update (the
 * form most iterations of complex128 states run; complex64 states apply H
 * afresh every iteration, and 2 then times the same work as 0), 3 = the
 * reduction of the partials into energy, gradients and the selection.  The
 * launches write only scratch buffers (never sigma, the states or the
 * iteration record), so a run continues exactly as without them.
 */
int gocp_batch_time_kernel(gocp_batch *b, int32_t which, int32_t n_launch, double *avg_ms);
/* The schedule the batch runs with, in the encoding of
 * gocp_adapt_params.schedule (autotuned or given). */
int gocp_batch_schedule(gocp_batch *b, int32_t *amps_per_lane);
int gocp_batch_destroy(gocp_batch *b);

/* ---------------------------------------------------------------------
 * Serving form: continuous batching of ADAPT solves on one device.
 * Requests are queued from any thread.  The server allocates its device
 * memory once, at creation: an arena of the HBM budget, from which each
 * admitted request gets one block holding its workspace and its own copy of
 * its Hamiltonian's and pool's device tables (gocp_request_bytes), plus fixed
 * table and flag buffers; its worker thread never allocates or frees device
 * memory.  The worker admits requests in arrival order while a slot is free
 * and the request's block fits the arena, starts each from its Hartree-Fock
 * state, and advances all admitted requests together (iters_per_step
 * iterations per step, one launch per kernel for all of them).  Two steps stay
 * queued on the device: while one runs, the worker reads the previous step's
 * done flags (event polling), retires finished requests (converged or at
 * max_iter), admits waiting ones into free blocks and prepares the next
 * step's tables, so requests arriving while others run join the running set
 * and admission overlaps device work.  Each request computes exactly what
 * adapt_solve computes for it alone.
 * Test hook: with the environment variable GOCP_TEST_FAIL_ADMISSION=k at
 * gocp_server_create, the server's k-th admission fails as a device error
 * would (that request ends with GOCP_EDEVICE; the others are unaffected).
 * ------------------------------------------------------------------- */
typedef struct {
    int32_t status;         /* GOCP_OK, GOCP_ENOMEM (never fits the budget),
                               GOCP_ENUMERIC, GOCP_ECANCELED, GOCP_EDEVICE       */
    int32_t n_qubits;
    int64_t t_submit_ns;    /* steady-clock times of submission, admission and */
    int64_t t_admit_ns;     /* completion (nanoseconds, one clock per process) */
    int64_t t_done_ns;
} gocp_request_info;

/* An estimate, from the sizes alone, of the device bytes one request occupies
 * while admitted (workspace + term tables). */
int gocp_request_footprint(int n_qubits, int n_ops, int n_strings, int64_t n_terms, int n_classes,
                           int max_iter, int dtype, int64_t *bytes);
/* The exact bytes of the arena block a server gives the request (ham, pool,
 * max_iter, dtype): its workspace and its own copy of both handles' device
 * tables.  Lays the handles' tables out in pinned host memory if that was not
 * done yet (a host-side allocation; no device memory).  Errors: EINVAL, ESHAPE. */
int gocp_request_bytes(const gocp_ham *h, const gocp_pool *p, int32_t max_iter, int dtype, int64_t *bytes);
/* Start a server on ctx's device with its own stream and worker thread; the
 * tile kernels run with amps_per_lane (1, 2 or 4) amplitudes per lane, or with
 * 0 a schedule chosen whenever the active set changes: 1 while the set has
 * fewer than four 64-amplitude tiles per compute unit, else 4, and the
 * compacted H v, H w launch's parts by the rule of the
 * autotuned schedule (gocp_adapt_params.schedule).  A request's result is
 * bit-identical to adapt_solve with the same schedule (amps_per_lane, 8
 * parts); under the adaptive schedule it can change between steps, so results
 * agree with adapt_solve to rounding.
 * Errors: EINVAL (non-positive budget, slots or iters_per_step; bad schedule). */
int gocp_server_create(gocp_ctx *ctx, int64_t hbm_budget_bytes, int32_t max_slots, int dtype,
                       int32_t iters_per_step, int32_t amps_per_lane, gocp_server **out);
/* Queue one solve: ham and pool (equal qubit counts) must stay alive until
 * the request has been polled.  Stops at ||g||_2 < grad_tol or max_iter. */
int gocp_server_submit(gocp_server *s, const gocp_ham *h, const gocp_pool *p, int32_t max_iter,
                       double grad_tol, uint64_t *ticket);
/* GOCP_EBUSY while the request is queued or running; otherwise the request's
 * status, with its record in *res (arrays sized as for adapt_solve; may be
 * NULL) and its times in *info (may be NULL).  A finished ticket is released
 * by the poll that returns it.  GOCP_EDEVICE for an unfinished request once
 * the worker has failed (every unfinished request then ends with it). */
int gocp_server_poll(gocp_server *s, uint64_t ticket, gocp_adapt_result *res, gocp_request_info *info);
/* Running and queued requests, requests finished so far, bytes of the arena
 * in use (the blocks of admitted requests and of retired ones whose record is
 * still being copied), steps. */
int gocp_server_stats(gocp_server *s, int32_t *active, int32_t *queued, int64_t *completed,
                      int64_t *bytes_in_use, int64_t *steps);
/* Stop the worker; unfinished requests end with GOCP_ECANCELED. */
int gocp_server_destroy(gocp_server *s);

#ifdef __cplusplus
}
#endif
#endif /* GOCP_H */
