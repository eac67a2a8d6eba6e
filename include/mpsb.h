/*
 * mpsb: batched Monte Carlo simulation of noisy 1D brickwork circuits with matrix-product-
 * state trajectories and locally entanglement-optimal unravelings (arXiv 2508.05745),
 * native to AMD Instinct MI355X (gfx950).
 *
 * C ABI.  All functions return 0 (MPSB_OK) on success and a negative MPSB_E* code on
 * failure; a thread-local message is available from mps_last_error().  Arguments are
 * validated on the host before any device work is enqueued, so a failing call leaves its
 * outputs untouched.  Errors raised by the device (asynchronous) surface at the next call
 * on the same handle or at mps_batch_sync().
 *
 * Memory ownership: the library never allocates device memory.  The caller provides the
 * state and work buffers (sizes from mps_batch_plan) and every input/output buffer; they
 * must outlive the handle.  Pointers documented as "device" must be device-accessible
 * (hipMalloc / torch CUDA tensors); "host" pointers are ordinary host memory.  All device
 * work is enqueued on the stream given at creation (a hipStream_t passed as void*, NULL =
 * the default stream); calls return without waiting for it unless stated otherwise.
 *
 * Complex numbers are stored interleaved (re, im).  "c128" = two doubles, "c64" = two
 * floats.
 */
#ifndef MPSB_H
#define MPSB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status codes */
#define MPSB_OK 0
#define MPSB_EINVAL -1  /* bad shape or argument, non-unitary gate                     */
#define MPSB_ENOMEM -2  /* caller buffer too small / sizes beyond the supported maxima  */
#define MPSB_EHIP -3    /* a HIP runtime call failed                                   */
#define MPSB_ENOTSUP -4 /* combination not supported by this library                    */
#define MPSB_ENUM -5    /* non-finite value, or a forced branch with zero probability  */
#define MPSB_EKRAUS -6  /* Kraus set not trace preserving (sum K^dag K != I)            */

/* ------------------------------------------------------------------ enums */
#define MPSB_FP32_BULK 0 /* site tensors c64, contractions FP32 (FP32 accumulation);
                            eigen-solves, unravelling, probabilities, observables FP64 */
#define MPSB_FP64 1      /* everything complex128 / FP64                                */

/* Unravelling (choice of Kraus decomposition, eq. unitarity_kraus).  The mixed operators
 * are K'_j = sum_i U[j][i] K_i, j = 0..3 (always four outputs, some possibly zero). */
#define MPSB_ORTHOGONAL 0 /* the channel's own operators (U = identity, zero-padded)     */
#define MPSB_FIXED 1      /* a caller-given, state-independent 4 x r mixing U           */
#define MPSB_HAAR_OPT 2   /* the Haar Optimal unraveling (table of unravelings, Sec.
                             "Noisy random circuits"; appendix "Some common unravelings"):
                             the channel's operators rotated by H (two operators) or by
                             the printed 4 x 4 Hadamard matrix (four); 1, 2 or 4 operators */
#define MPSB_OPTIMAL 3    /* locally entanglement-optimal mixing (Thm. 2: Wootters'
                             decomposition of the effective two-qubit state)            */
#define MPSB_LEAST_UNITARY 4 /* the least unitary unraveling (appendix "Vectorized Kraus
                             operators and the least unitary unraveling"): the optimal
                             mixing for the maximally mixed reduced state, i.e. of the
                             channel's Choi state; state independent                    */

#define MPSB_MAX_CHI 256      /* largest supported bond dimension                       */
#define MPSB_MAX_QUBITS 4096
#define MPSB_MAX_CHANNELS 1048576   /* channel table entries (device table) */

typedef struct mpsb_batch* mpsb_handle;

/* Noisy brickwork circuit (the classical description D of the paper's truncated
 * trajectory sampling task: qubit order = chain order, initial state |0...0>, a string
 * of layers of two-qubit gates composed with single-qubit noise).  Host pointers; the
 * library copies what it needs into the caller's circuit buffer during
 * mps_batch_set_circuit.  W = the widest trajectory of the batch.
 *
 *   layer l (0-based) acts on the pairs (p, p+1), (p+2, p+3), ... with p = l % 2 (only the
 *          pairs inside a trajectory's own width);
 *   n_gates == 0: gates [depth][W/2][4][4] c128, one circuit shared by all trajectories:
 *          slot i of layer l is the pair (p+2i, p+2i+1), basis index 2*s + t with s the
 *          lower qubit of the pair;
 *   n_gates > 0: gates is a pool [n_gates][4][4] c128 and gate_id [n_traj][depth][W/2] the
 *          pool index of slot i of layer l of each trajectory, -1 = identity (used past a
 *          trajectory's own depth);
 *   kraus  [n_channels][4][2][2] c128, zero padded; n_kraus[c] in 1..4 operators used;
 *   events [depth][W] (events_per_traj == 0) or [n_traj][depth][W] (events_per_traj == 1)
 *          int32: channel applied to qubit q in layer l, -1 = none.  Noise on a gate's
 *          qubits follows that gate (lower qubit first); noise on an idle qubit is applied
 *          when the layer's sweep reaches it;
 *   fixed_u [n_channels][4][4] c128 (row j = output operator), used with MPSB_FIXED.
 * With MPSB_HAAR_OPT or MPSB_LEAST_UNITARY the library computes a fixed mixing per channel
 * when the circuit is set (the least unitary one by the unravelling kernel on the device)
 * and the batch runs as MPSB_FIXED with it (sample_kraus with MPSB_FIXED uses it too).
 */
typedef struct {
    int depth;
    const double* gates;
    int n_gates;
    const int32_t* gate_id;
    int n_channels;
    const double* kraus;
    const int32_t* n_kraus;
    const int32_t* events;
    int events_per_traj;
    int unravel_mode;
    const double* fixed_u; /* may be NULL unless unravel_mode == MPSB_FIXED (ignored with
                              MPSB_HAAR_OPT and MPSB_LEAST_UNITARY)                      */
} mpsb_circuit;

/* Sizes of the two caller buffers for n_traj trajectories of the truncated trajectory
 * sampling task (Sec. "Truncated Trajectory Sampling Task", Def. "Truncated Trajectory
 * Sampling": one pure-state MPS per trajectory, eq. def_MPS, bond dimension at most chi).
 * Trajectory t is a chain of width[t] qubits truncated to bond dimension chi[t]
 * (1..MPSB_MAX_CHI).  Bond k (between
 * qubits k and k+1) has the fixed capacity min(chi, 2^(k+1), 2^(n-k-1)).  Maximal runs of
 * consecutive trajectories with equal (width, chi) form the batch's uniform sub-batches
 * (group equal shapes together); a batch of one run is a uniform batch.  precision:
 * MPSB_FP32_BULK or MPSB_FP64.  Host arrays.  Returns MPSB_EINVAL for bad arguments. */
int mps_batch_plan(int n_traj, const int32_t* width, const int32_t* chi, int precision,
                   size_t* state_bytes, size_t* work_bytes);

/* Creates a batch in the initial state of the circuit description D (Sec. "Truncated
 * Trajectory Sampling Task": an initial MPS, here |0...0>, in the chain's qubit order) with
 * the orthogonality centre at qubit 0.  state_buf /
 * work_buf: device buffers of at least the planned sizes (256-byte aligned); seed keys the
 * counter-based branch sampler (SplitMix64 output number 1 + (traj<<32 | layer<<16 |
 * qubit)), traj = traj_offset + index in the batch: a run of T trajectories split into
 * batches with offsets 0, T1, T1 + T2, ... (memory waves, or shares of several devices)
 * draws exactly the branches of one batch of T (0 <= traj_offset, traj_offset + n_traj <=
 * 2^32, else MPSB_EINVAL).  The initial state is written on `stream`, which all
 * later calls use; a mixed batch also creates private streams (default priority) on which
 * its sub-batches run concurrently.  The handle owns host metadata, streams, events and
 * captured graphs only. */
int mps_batch_create(int n_traj, const int32_t* width, const int32_t* chi, int precision,
                     uint64_t seed, int64_t traj_offset, void* state_buf, size_t state_bytes,
                     void* work_buf, size_t work_bytes, void* stream, mpsb_handle* out);

/* For callers that cannot allocate device memory (code under graph capture, serving loops,
 * harnesses that forbid allocation): mps_batch_create for a uniform batch without a caller
 * work buffer.  The work memory is a static device area of MPSB_STATIC_WORK_BYTES per device
 * (held by the library's code object until the process ends); batches whose planned work
 * exceeds it fail with MPSB_ENOMEM, mixed batches with MPSB_ENOTSUP.  Nothing is allocated:
 * no device memory, no stream or event (graphs and the tile autotuner are off for such a
 * batch; mps_batch_set_graphs(h, 1) fails with MPSB_ENOTSUP).  One batch at a time may hold a
 * device's area: creating a second one on the same device while the first is alive fails with
 * MPSB_ENOTSUP (batches on the same area would overwrite each other's work); the area is
 * released by mps_batch_destroy.  The area keeps the previous batch's contents; the batch
 * clears what must start at zero when it is created.  Other arguments and results are those
 * of mps_batch_create. */
#define MPSB_STATIC_WORK_BYTES (64u << 20)
int mps_batch_create_static(int n_traj, const int32_t* width, const int32_t* chi, int precision,
                            uint64_t seed, int64_t traj_offset, void* state_buf,
                            size_t state_bytes, void* stream, mpsb_handle* out);

/* Bytes of the device circuit buffer mps_batch_set_circuit needs for circuit c on batch h. */
int mps_circuit_bytes(mpsb_handle h, const mpsb_circuit* c, size_t* bytes);

/* Validates the circuit and writes its device tables (gate pool, gate ids, channel table,
 * event ids, the device layer counter) into circuit_buf (device, 256-byte aligned, at least
 * mps_circuit_bytes; caller-owned, must stay allocated while layers are applied).  Checks:
 * every Kraus set ||sum_i K_i^dag K_i - I||_max <= 1e-12 (else MPSB_EKRAUS), every gate
 * ||G^dag G - I||_max <= 1e-12 (else MPSB_EINVAL), gate ids in -1..n_gates-1, event ids
 * name a channel or are -1, FIXED mixings unitary on the used columns.  Blocks until the
 * tables are on the device. */
int mps_batch_set_circuit(mpsb_handle h, const mpsb_circuit* c, void* circuit_buf,
                          size_t circuit_bytes);

/* Whole-layer graphs (default on): the first layer with a given launch signature (sweep
 * parity, operations, centre position) runs directly, the second is captured into a HIP
 * graph and every later one replays it with a single graph launch.  The addresses of the
 * record outputs of apply_layer are part of the signature (a caller that records into the
 * same buffers every layer gets graph replays that write them; the outputs are cleared by
 * direct calls before the graph launch).  Layers with replay inputs, or that run while
 * profiling, always run directly. */
int mps_batch_set_graphs(mpsb_handle h, int enable);

/* Autotuning of the theta kernel's tile shape (default on): the first time a shape occurs
 * outside a capture, each applicable variant is timed on the live operands and the faster
 * one is kept for the batch.  Disabling it (or re-enabling) clears the choices. */
int mps_batch_set_autotune(mpsb_handle h, int enable);

/* Applies brickwork layer `layer` (0 <= layer < depth) to every trajectory: for each pair
 * in sweep order (left to right for even layers, right to left for odd layers) the two-
 * site contraction with the gate, the noise events of the pair (unravel, draw, apply the
 * sampled Kraus operator; Alg. 1), truncation of the pair's bond to its capacity with
 * renormalisation, and the move of the orthogonality centre to the next pair; idle-qubit
 * noise when the sweep reaches the qubit.  Layers must be applied in order 0, 1, 2, ...
 * Optional device outputs (NULL to skip; W = the widest trajectory):
 *   discarded [n_traj][W/2] FP64: discarded weight sum_{i>D} lambda_i / sum_i lambda_i of
 *             each gate (slot i = pair p+2i; untouched slots are set to 0);
 *   branch    [n_traj][W] int32: sampled branch of the event on each qubit (-1 = no
 *             event);
 *   w_record  [n_traj][W][4][4] c128: the mixing U used by each event (K'_j =
 *             sum_i U[j][i] K_i), rows j, columns i (unused columns zero). */
int apply_layer(mpsb_handle h, int layer, double* discarded, int32_t* branch,
                double* w_record);

/* apply_layer following recorded decisions (Alg. 1 with its choices given): w_in [n_traj][W]
 * [4][4] c128 (the w_record layout) replaces the mixing the unravel mode would choose for each
 * event, branch_in [n_traj][W] int32 (the branch layout) replaces the draw; either may be NULL
 * (then chosen / drawn as in apply_layer); entries of qubits without an event are not read.
 * The branch weights are still computed from this batch's own state, so that a run in another
 * precision can follow a recorded run event by event (paired comparison); a replayed branch of
 * zero weight is reported as MPSB_ENUM by mps_batch_sync.  Device pointers; the outputs are
 * those of apply_layer.  Layers with replay inputs run without graphs. */
int apply_layer_replay(mpsb_handle h, int layer, const double* w_in, const int32_t* branch_in,
                       double* discarded, int32_t* branch, double* w_record);

/* Optional bond-entropy output of apply_layer / apply_layer_replay (Preliminaries,
 * "Entanglement measures": the von Neumann entanglement entropy of a bipartition, here the
 * cut at the pair's bond): entropy [n_traj][W/2] FP64 device array, or NULL to stop.  Every
 * gate-step of a layer writes, in slot i (pair p + 2i: the layout of `discarded`), the
 * entropy (base 2) of the pair's bond after the step, -sum_k s_k log2 s_k over the kept,
 * renormalised squared Schmidt coefficients s_k, i.e. the FP64 eigenvalues of the step's
 * Gram matrix (a step that discards nothing solves that Gram matrix for this output only);
 * slots without a gate in the layer are set to 0.  The array must stay allocated while it
 * is set; its address is part of the layer-graph signature.  mps_truncate, expect and
 * sample_kraus do not write it. */
int mps_batch_set_entropy(mpsb_handle h, double* entropy);

/* Channel-unravelling subprocedure (Alg. 1) for one noise event per trajectory on qubit
 * qubit[t] (host array [n_traj], the centre is moved there first) with channel
 * `channel`, mode `unravel_mode` (MPSB_FIXED uses the circuit's fixed_u).  forced: host
 * array [n_traj] of branch indices, -1 = draw with the sampler keyed by (traj,
 * rng_layer, qubit[t]); a forced branch of zero probability fails with MPSB_ENUM before
 * the state is changed.  Device outputs (NULL to skip): branch [n_traj] int32,
 * p [n_traj][4] FP64. */
int sample_kraus(mpsb_handle h, const int32_t* qubit, int channel, int unravel_mode,
                 int rng_layer, const int32_t* forced, int32_t* branch, double* p);

/* (sample_kraus and mps_truncate need a uniform batch: MPSB_ENOTSUP otherwise.) */

/* Approximation subprocedure on demand (Sec. "Class of Truncated Trajectory Sampling
 * Algorithms"): truncates every bond to min(chi, capacity) with a full left-to-right sweep
 * (discarding the smallest Schmidt values, renormalising), then moves the centre back to
 * qubit 0; discarded [n_traj] FP64 device (or NULL) receives the summed discarded weight
 * of the sweep.  1 <= chi <= the batch's chi.  (Named mps_truncate rather than truncate so
 * that it does not collide with the POSIX truncate(2) declaration.) */
int mps_truncate(mpsb_handle h, int chi, double* discarded);

/* Global layering (Sec. "Details of MPS-based trajectory sampling", the first of its two
 * layerings, Trunc^(n-1) o N^n o U^(n/2)): the layer's gates and noise events with no
 * truncation below the bond capacities, then every bond truncated to chi by mps_truncate's
 * left-to-right sweep (discarded [n_traj] FP64 or NULL: its summed discarded weight).  The
 * intermediate state is exact when the batch's chi is at least 2 chi (a gate can double the
 * bond it acts on); with a smaller capacity apply_layer's own truncation applies first.
 * Uniform batches only (MPSB_ENOTSUP otherwise); runs without graphs. */
int apply_layer_global(mpsb_handle h, int layer, int chi, double* discarded);

/* Output distribution sampling from the trajectories (Lemma "Output distribution sampling
 * from trajectory sampling": sampling each trajectory's Born distribution samples the
 * mixture): n_samples computational-basis bitstrings per trajectory, drawn site by site from
 * the conditional probabilities (the centre is moved to site 0, the rest being
 * right-orthonormal, so p(s_k = s | drawn prefix) is ||v A_k^s||^2 normalised, v the prefix's
 * normalised left vector; the products in the state's precision, the probabilities in FP64).
 * The draw of site k of sample i of trajectory t is the counter uniform of `seed` keyed by
 * (traj_offset + t, i, k), the layout of the branch keys; s_k = 0 if u < p_0 / (p_0 + p_1).
 * bits [n_traj][n_samples][n] uint8 device (0 or 1).  1 <= n_samples <= min(65535, 2 chi)
 * (MPSB_EINVAL otherwise); uniform batches only (MPSB_ENOTSUP). */
int mps_sample_bitstrings(mpsb_handle h, int n_samples, uint64_t seed, uint8_t* bits);

/* Host-only validation of a circuit for n_traj trajectories of widths width[] (host
 * array): the checks of mps_batch_set_circuit, without a handle or a device. */
int mps_circuit_validate(int n_traj, const int32_t* width, const mpsb_circuit* c);

/* Observable estimation from sampled trajectories (Sec. "Target classical simulation
 * tasks", Lemma "Expectation value estimation from trajectory sampling" and its corollary:
 * the estimator is the mean over trajectories of <psi_i|O|psi_i>).  Observables of every
 * trajectory: <Z_i> (i = 0..n-1) then <Z_i Z_{i+1}> (i = 0..n-2), in FP64, normalised by
 * <psi|psi>, from a measurement sweep: the orthogonality centre walks from site 0 to n-2 and
 * each pair's two-site reduced state is accumulated by the two-site contraction (so the call
 * leaves the centre at site n-2; the state itself is unchanged).  Device
 * outputs: mean [2n-1] and m2 [2n-1] (sum of squared deviations) over trajectories,
 * reduced in a fixed order (bitwise reproducible), or both NULL; per_traj [n_traj][2W-1]
 * (or NULL), rows NaN-padded past a trajectory's own 2n-1 entries.  For a mixed batch
 * (widths up to W) mean and m2 have 2W-1 entries in the widest trajectory's layout (<Z_i> at
 * i, <Z_i Z_(i+1)> at W + i), each over the trajectories that have that observable (width
 * > i, resp. > i + 1; NaN where none has it); the members' fixed-order reductions are merged
 * on the host in trajectory order (pairwise mean / M2 update), so the result is bitwise
 * reproducible too. */
int expect(mpsb_handle h, double* mean, double* m2, double* per_traj);

/* Optional per-kernel-class timing with HIP events recorded on the batch stream (for
 * roofline reports).  mps_profile(h, 1) resets and starts, (h, 0) stops (bit 1 of the
 * argument adds the schedule timing described below).  mps_profile_read
 * synchronises and returns, per class, the summed milliseconds and the number of timed
 * launches (host arrays of n entries); the return value is the number of classes.  Class
 * order: 0 theta contraction + gate + two-site RDM, 1 noise events (unravel + sample),
 * 2 Kraus-pair application, 3 truncation Gram matrix, 4 tridiagonalisation of matrices with
 * 128 < n <= 256, 5 tridiagonal eigenvalues + inverse iteration, 6 centre-hop factorisation
 * (all phases), 7 eigenvector back-transformation (n <= 256), 8 recomposition, 9 centre-hop
 * contractions, 10 idle-qubit events, 11 observables, 12 tridiagonalisation (n <= 128),
 * 13 tridiagonalisation (256 < n <= 512), 14 back-transformation (256 < n <= 512).  Classes
 * 4, 12 and 13 each time a single kernel instance (phases 4/12/13, 5, 7/14 are those of the
 * truncation eigensolver). */
int mps_profile(mpsb_handle h, int enable);
int mps_profile_read(mpsb_handle h, double* ms, long long* count, int n);

/* Schedule timing of a batch's members (the uniform sub-batches of a mixed batch, or the batch
 * itself), for the per-chi-class rates and the stream utilisation of mixed batches.  Enabled by
 * bit 1 of mps_profile's argument (2: schedule only, 3: with the kernel classes; 0..3, else
 * MPSB_EINVAL; like bit 0 it turns layer graphs off).  Each timed layer records an event pair
 * around the whole layer on the caller's stream and one around every member's share of it on
 * the private stream it was assigned (members with work in the layer are dealt round-robin to
 * up to four streams in trajectory order).  mps_schedule_read
 * synchronises and writes, for the first n members (host arrays of n entries, in trajectory
 * order): the index of the member's first trajectory, its trajectory count, the stream of its
 * last timed layer (-1 if none) and its summed milliseconds; elapsed_ms and layers (each may be
 * NULL) get the summed wall time of the timed layers and their number.  The return value is
 * the number of members; null arrays with n > 0 give MPSB_EINVAL. */
int mps_schedule_read(mpsb_handle h, int* first, int* count, int* stream, double* busy_ms, double* elapsed_ms,
                      long long* layers, int n);

/* Blocks until all work of the handle is done; reports asynchronous device errors. */
int mps_batch_sync(mpsb_handle h);
int mps_batch_destroy(mpsb_handle h);
const char* mps_last_error(void);

/* Certified error of the sampled trajectories (Sec. "Upper bounds on the simulation errors",
 * Thm. "Truncated Trajectory Sampling error"; Props. "Path error bound" and "systematic error
 * bound"; Sec. "Errors based on MPS truncations"; Sec. "Improvements of the error bounds due to
 * concentration").
 *
 * mps_error_accumulate: eps_tot[t] += weight * sum over the layer's truncation steps of the
 * step's trace-norm change, from discarded [n_traj][slots] FP64 (apply_layer's output, slots =
 * W/2; zero for steps that discard nothing): MPSB_STEP_EXACT = 2 sqrt(eps) (exact for one
 * truncated bond with renormalisation), MPSB_STEP_PAPER = 4 sqrt(2 eps) (the paper's bound).
 * weight = 1 gives Thm. 1's cumulated error; alpha^(L-l) or min(sqrt(8n)(1-p)^(L-l), 1) the
 * concentration variants (layers l = 1..L).  eps_tot [n_traj] is device memory that the
 * caller zeroes before the first layer.
 * mps_error_estimate: out[0] = eps_hat = mean over trajectories of eps_bound (eps_tot if
 * eps_tot <= eps_max - 2, else eps_max; 2 <= eps_max), out[1] = the Hoeffding buffer
 * sqrt(eps_max^2 log(1/delta) / (2 n_traj)), out[2] = out[0] + out[1]: with probability at
 * least 1 - delta the trace distance between the exact state and the sampled mixture is at
 * most out[2].  The sum runs in a fixed order.  Device pointers; asynchronous on `stream`. */
#define MPSB_STEP_EXACT 0
#define MPSB_STEP_PAPER 1
int mps_error_accumulate(int n_traj, int slots, const double* discarded, int step_kind,
                         double weight, double* eps_tot, void* stream);
int mps_error_estimate(int n_traj, const double* eps_tot, double eps_max, double delta,
                       double* out, void* stream);

/* Noisy circuits of Trotterised time-independent Lindbladians (Sec. "Time-independent
 * Lindbladian systems"; appendix "Exact decomposition of Trotterized Lindbladian
 * evolutions").  Host-only (host arrays, no device work), for building the gate and channel
 * tables of mps_batch_set_circuit:
 *   mps_trotter_gate: gate [4][4] c128 = exp(-i h dt) of a Hermitian pair term h [4][4] c128
 *     (MPSB_EINVAL if h is not Hermitian to 1e-12 of its largest entry, MPSB_ENUM for a
 *     non-finite input);
 *   mps_jump_channel: the Kraus operators of the single-site jump process exp(tau sum_j L_j),
 *     L_j = gamma_j (c_j (x) c_j^* - 1/2 c_j^dag c_j (x) I - 1/2 I (x) c_j^T c_j^*) for the n_jumps
 *     jump operators c [n_jumps][2][2] c128 with rates gamma [n_jumps] >= 0: the eigenvectors of
 *     its Choi matrix times the square roots of their eigenvalues, in descending eigenvalue
 *     order, eigenvalues below 1e-14 of the largest left out, each operator's largest-modulus
 *     entry real positive; kraus [4][2][2] c128 (unused operators zero), *n_kraus their number.
 *     A Trotter step of length dt applies the jump processes for tau = dt / 2 after each of its
 *     two brickwork layers. */
int mps_trotter_gate(const double* h, double dt, double* gate);
int mps_jump_channel(int n_jumps, const double* c, const double* gamma, double tau, double* kraus, int* n_kraus);

/* Batched locally entanglement-optimal unravelling (Sec. "Locally entanglement-optimal
 * unraveling"; appendix "Practical/closed-form version" of Wootters' decomposition): for
 * each of `batch` qubits with normalised reduced state rho_q [batch][2][2] c128 and the
 * channel kraus [n_k][r][2][2] c128 (channel of item b = kraus_id[b], or 0 if kraus_id is
 * NULL; r in 1..4), returns U [batch][4][r] c128 (K'_j = sum_i U[j][i] K_i; rows
 * orthonormal so the K'_j are a complete Kraus set), the branch weights p [batch][4]
 * (FP64) and the entanglement of formation eof [batch] reached by the decomposition.
 * All pointers are device pointers; 1 <= n_k <= MPSB_MAX_CHANNELS (MPSB_EINVAL otherwise).
 * kraus_id is read on the device only: an item whose id lies outside 0..n_k-1 reads no
 * channel and gets NaN in its U, p and eof. */
int unravel_opt(int batch, const double* rho_q, const double* kraus, int n_k,
                const int32_t* kraus_id, int r, double* U, double* p, double* eof,
                void* stream);

/* Largest batch of the unravelling-cost calls (unravel_cost*, their adjoints): larger batches
 * fail with MPSB_EINVAL. */
#define MPSB_MAX_COST_BATCH (1 << 26)

/* Expected entanglement of an unravelling, as a function of the mixing (differentiable
 * cost).  The mixing is the unitary freedom of a Kraus representation (Preliminaries,
 * eq. unitarity_kraus: K'_j = sum_i U_ji K_i describes the same channel); the cost is the
 * objective that the locally entanglement-optimal unravelling minimises (Sec. "Locally
 * entanglement-optimal unraveling", eq. target_optimal_unitary: the branch-weighted
 * entanglement between the noisy qubit and the rest), with the linear or Renyi-2 entropy in
 * place of the entanglement entropy so that it is smooth.  For `batch` two-site tensors theta [batch][chi_l][2][2][chi_r] (c64 when prec ==
 * MPSB_FP32_BULK, c128 when MPSB_FP64; noise on the first physical index) the reduced
 * state rho_q = sum_{a,t,b} theta[a,s,t,b] conj(theta[a,s',t,b]) is formed (FP64
 * accumulation) and written to rho_out [batch][2][2] c128, then
 *   kind 0: f = sum_j p_j (1 - Tr sigma_j^2)   (linear entropy)
 *   kind 1: f = sum_j p_j (-log2 Tr sigma_j^2) (Renyi-2)
 * with sigma_j = K'_j rho_q K'_j^dag / p_j, K'_j = sum_i U_ji K_i, U = exp(i sum_k
 * params[k] L_k) U_ref, the 16 generators L_k being E_kk (k<4), then for the pairs
 * (0,1),(0,2),(0,3),(1,2),(1,3),(2,3) the symmetric E_jk + E_kj and the antisymmetric
 * i(E_kj - E_jk).  kraus [4][2][2] c128 (zero padded), params [batch][16] FP64, u_ref
 * [batch][4][4] c128, f_out [batch] FP64.  Device pointers.  MPSB_EINVAL for batch < 0 or
 * above MPSB_MAX_COST_BATCH, chi_l or chi_r < 1, chi_l chi_r > 2^26, another precision or kind,
 * or a null pointer (batch > 0). */
int unravel_cost(int batch, const void* theta, int chi_l, int chi_r, int prec,
                 const double* kraus, const double* params, const double* u_ref, int kind,
                 double* f_out, double* rho_out, void* stream);

/* Adjoint of unravel_cost with respect to the 16 mixing parameters (theta is not
 * re-read): grad_out [batch][16] = grad_f[b] * d f_b / d params_b (grad_f NULL: 1), the
 * derivative of the same objective (Sec. "Locally entanglement-optimal unraveling") through
 * U = exp(i H) U_ref (eq. unitarity_kraus).  rho_q is the reduced state unravel_cost wrote.
 * Device pointers. */
int unravel_cost_grad(int batch, const double* rho_q, const double* kraus,
                      const double* params, const double* u_ref, int kind,
                      const double* grad_f, double* grad_out, void* stream);

/* The same objective taken across the two-site block's internal bond (a, s) : (t, b) instead
 * of between the noisy qubit and the rest: branch j of the block is theta_j = (K'_j on s)
 * theta with p_j = ||theta_j||^2 / ||theta||^2, and its bond purity is Tr Gamma_j^2 / p_j^2 with
 * Gamma_j = theta_j theta_j^dag over (a, s) (Sec. "Locally entanglement-optimal unraveling",
 * eq. target_optimal_unitary, applied to the bond that the truncation acts on; linear or
 * Renyi-2 entropy as in unravel_cost):
 *   kind 0: f = sum_j (p_j - Tr Gamma_j^2 / p_j),   kind 1: f = sum_j -p_j log2(Tr Gamma_j^2 / p_j^2)
 * (branches with p_j <= 1e-300 contribute 0).  The block Gram Gamma = theta theta^dag
 * (2 chi_l x 2 chi_l, FP64 accumulation on the matrix cores; O(chi_l^2 chi_r) work per state)
 * is reduced to rho_out [batch][2][2] c128 (the noisy qubit's reduced state) and the moment
 * matrix n_out [batch][4][4] c128, N[(w,x)][(y,z)] = sum_{a,a'} Gamma[(a,w),(a',x)]
 * conj(Gamma[(a,y),(a',z)]) / ||theta||^4, from which Tr Gamma_j^2 = sum E[s1][s2] E[s3][s4]
 * N[(s2,s3)][(s1,s4)] with E = K'_j^dag K'_j.  With chi_l = chi_r = 1 it equals unravel_cost.
 * Arguments, layouts and errors as in unravel_cost (theta [batch][chi_l][2][2][chi_r], noise on
 * the first physical index; a zero theta gives NaN).  Device pointers. */
int unravel_cost_bond(int batch, const void* theta, int chi_l, int chi_r, int prec,
                      const double* kraus, const double* params, const double* u_ref, int kind,
                      double* f_out, double* rho_out, double* n_out, void* stream);

/* Adjoint of unravel_cost_bond with respect to the 16 mixing parameters, from the rho_q and
 * N that it wrote (theta is not re-read): grad_out [batch][16] = grad_f[b] d f_b / d params_b
 * (grad_f NULL: 1), through U = exp(i H) U_ref (eq. unitarity_kraus); d Tr Gamma_j^2 / d U_ji
 * = 2 sum (K'_j^dag K_i)[s1][s2] E_j[s3][s4] N[(s2,s3)][(s1,s4)].  Device pointers. */
int unravel_cost_bond_grad(int batch, const double* rho_q, const double* n_mom,
                           const double* kraus, const double* params, const double* u_ref,
                           int kind, const double* grad_f, double* grad_out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* MPSB_H */
