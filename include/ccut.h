/*
 * ccut -- Clifford-based circuit cutting on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libccut.so.  The problem statement follows the paper
 * (SuperSim, arXiv 2303.10788): a circuit whose inputs start in |0> and
 * whose outputs are measured in Z (Sec. V-B), plus a list of wire cuts
 * (Secs. III-B, V-A), goes in; the uncut circuit's output marginal or
 * Z-string expectations, rebuilt from fragment variants by the tensor
 * contraction of Sec. V-C, come out.
 *
 * Conventions shared by every call:
 *  - every call returns a ccut_status; no C++ exception crosses the ABI;
 *    on failure ccut_last_error() describes the first error;
 *  - handles are owned by the library and freed by the matching *_destroy;
 *    objects created from a context (plans, batches, term models,
 *    networks) keep it alive: destroying the context first defers its
 *    release until the last of them is destroyed;
 *  - a context is not thread-safe: use one per host thread;
 *  - device work runs on the context's HIP stream; a call with host outputs
 *    returns after its results are in the caller's buffer, a call with
 *    device outputs (out_on_device != 0) returns once the copy into the
 *    caller's buffer is enqueued as the call's last work on that stream
 *    (read it in stream order, or after synchronizing the stream); host
 *    inputs are staged in pinned memory and may be reused when the call
 *    returns;
 *  - results are a pure function of (ops, cuts, request, seed, shots, mode):
 *    every random bit is Philox4x32-10 keyed by seed and counted by
 *    (variant id, shot, measurement index);
 *  - estimates are raw quasi-probabilities unless CCUT_FLAG_ML asks for
 *    the maximum-likelihood fragment correction: raw sampled marginals can
 *    be slightly negative.
 *
 * Readings of the method where the paper is silent:
 *  - quantum inputs are prepared in {|0>, |1>, |+>, |+i>}, quantum outputs
 *    measured in {X, Y, Z}; the I term of an output comes from its Z basis;
 *  - a fragment variant is numbered in mixed radix over the fragment's
 *    incident cut axes in cut-list order (upstream side before downstream
 *    side of the same cut), first axis least significant; bases radix 3
 *    (X, Y, Z), preparations radix 4 (0, 1, +, +i);
 *  - the variant id is (circuit << 40) | (fragment << 32) | variant;
 *  - a fragment measures only its measured set: requested circuit outputs
 *    plus quantum outputs, in ascending fragment-local order, local qubits
 *    being ordered by (wire, segment along the wire);
 *  - the Philox bit of measurement index a in shot s is bit (a & 31) of
 *    output word (s & 3) of philox(ctr = (a >> 5, s >> 2, lo32(vid),
 *    hi32(vid)), key = (lo32(seed), hi32(seed))); a random outcome equals
 *    its bit.
 */
#ifndef CCUT_ABI_H_
#define CCUT_ABI_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ccut_ctx ccut_ctx;   /* opaque, library-owned */
typedef struct ccut_plan ccut_plan; /* opaque, library-owned */

typedef enum {
  CCUT_OK = 0,
  CCUT_E_INVALID = -1,        /* malformed circuit, cut list or request */
  CCUT_E_OOM = -2,            /* a device or host allocation failed */
  CCUT_E_DEVICE = -3,         /* no device on this context, or a HIP error */
  CCUT_E_NC_TOO_WIDE = -4,    /* a non-Clifford fragment exceeds max_nc_qubits */
  CCUT_E_TOO_MANY_CUTS = -5,  /* k exceeds max_cuts */
  CCUT_E_CANCELLED = -6,      /* ccut_cancel() was called during the evaluation */
  CCUT_E_UNSUPPORTED = -7     /* a size beyond what the kernels implement */
} ccut_status;

/* Gates (Sec. II): Paulis, H = (Z+X)/sqrt2, S = Z^(1/2), S^dag, CX, CZ,
 * T = Z^(1/4) = diag(1, e^{i pi/4}), T^dag, RZ(theta) = diag(1, e^{i theta}).
 * H, S, SDG, X, Y, Z, CX, CZ are Clifford; T, TDG, RZ are not. */
typedef enum {
  CCUT_H = 0, CCUT_S = 1, CCUT_SDG = 2, CCUT_X = 3, CCUT_Y = 4, CCUT_Z = 5,
  CCUT_CX = 6, CCUT_CZ = 7, CCUT_T = 8, CCUT_TDG = 9, CCUT_RZ = 10
} ccut_gate_kind;

/* One gate.  q1 is the target of CX (q0 the control) and the second qubit
 * of CZ; it is ignored for one-qubit gates.  theta is used by RZ only. */
typedef struct {
  uint32_t kind;
  uint32_t q0;
  uint32_t q1;
  uint32_t reserved;
  double theta;
} ccut_op;

/* Cut wire `qubit` right after global op index `after_op`, which must act
 * on that wire (the cut locations of Sec. V-A). */
typedef struct {
  uint32_t qubit;
  uint32_t after_op;
} ccut_cut;

/* Automatic cut placement (the circuit cutter of Sec. V-A; no context or
 * device needed).  Chooses cut locations such that every fragment holding
 * a non-Clifford op (T, TDG, RZ) has at most max_width qubits, aiming at few
 * cuts (the recombination costs 4^k): a greedy search from one region per non-Clifford
 * op that merges regions, or stretches one to a wire's first or last op,
 * while the total cut count drops.  Never more than 2 cuts per non-Clifford
 * op (Sec. III-B's bound).  Writes min(k, cap) cuts, ascending by
 * (after_op, qubit), and k to *k (host).  CCUT_E_INVALID: malformed
 * circuit, max_width = 0; CCUT_E_TOO_MANY_CUTS: k > cap (*k still set). */
ccut_status ccut_find_cuts(uint32_t n_qubits, const ccut_op *ops, size_t n_ops, uint32_t max_width,
                           ccut_cut *cuts, size_t cap, size_t *k);

/* Optional device allocator (for example a framework's caching allocator).
 * alloc returns NULL on failure, which the library reports as CCUT_E_OOM. */
typedef void *(*ccut_alloc_fn)(size_t bytes, void *user);
typedef void (*ccut_free_fn)(void *ptr, void *user);

typedef struct {
  int device;             /* HIP device ordinal; -1 = host-only (plan and validate only) */
  void *hip_stream;       /* hipStream_t for all device work; NULL = null stream */
  ccut_alloc_fn alloc;    /* NULL: hipMalloc */
  ccut_free_fn free;      /* NULL: hipFree */
  void *user;             /* passed to alloc/free */
  uint32_t max_nc_qubits; /* 0 = default 12: the state vector of a non-Clifford fragment lives in LDS */
  uint32_t max_cuts;      /* 0 = default 12: exhaustive recombination sums 4^k terms */
} ccut_opts;

/* Precision of the recombination (Sec. V-C's contraction):
 *  CCUT_FP64: fp64 products and sums (fp64 matrix cores or fp64 VALU);
 *  CCUT_FP32_MFMA_FP64SUM: operands rounded to fp32, fp32 matrix-core
 *    products summed in fp32 over 8 cut terms, those partial sums added in
 *    fp64 (an output's error is about 2^-23 times the summed magnitude of its
 *    terms);
 *  CCUT_FP32X3_MFMA_FP64SUM: as above with every operand split into fp32
 *    hi + lo parts and three products (hi hi + hi lo + lo hi) per term: near
 *    fp64 products, still fp32 sums over 8 terms. */
enum { CCUT_FP64 = 0, CCUT_FP32_MFMA_FP64SUM = 1, CCUT_FP32X3_MFMA_FP64SUM = 2 };

/* How exact-mode Clifford fragments are evaluated (sampled mode always
 * evaluates every variant on the tableau):
 *  CCUT_METHOD_AUTO / CCUT_METHOD_HEISENBERG: the Pauli-basis tensor is read
 *    off directly in the Heisenberg picture (the Clifford-specific
 *    optimisation of Sec. IX): the requested Z's and the quantum outputs'
 *    X, Z are carried back through the fragment once, no variant is
 *    enumerated;
 *  CCUT_METHOD_VARIANTS: every variant is evaluated on the tableau, its
 *    exact dyadic outcome table formed, then rewritten in the Pauli basis. */
enum { CCUT_METHOD_AUTO = 0, CCUT_METHOD_VARIANTS = 1, CCUT_METHOD_HEISENBERG = 2 };

typedef struct {
  uint64_t seed;              /* Philox key */
  uint64_t shots_per_variant; /* 0 = exact ("strong simulation", Sec. V-C) Clifford tables; < 2^32 */
  int32_t precision;          /* CCUT_FP64, CCUT_FP32_MFMA_FP64SUM or CCUT_FP32X3_MFMA_FP64SUM */
  uint32_t circuit;           /* circuit index in variant ids (batch position) */
  uint32_t method;            /* CCUT_METHOD_*, exact mode only */
  uint32_t flags;             /* CCUT_FLAG_* (0: none) */
} ccut_eval_opts;

/* Clifford-specific cutting optimisations (Sec. IX):
 *  CCUT_FLAG_SPARSE (ccut_marginal only): the contraction sums only the cut
 *    terms P whose column T_f[.; P|f] is nonzero in every fragment (the
 *    others are exact zeros; for Clifford fragments most Pauli
 *    expectations vanish).  The support is found on the device and its size
 *    read back, so the call synchronizes and is never captured in a call
 *    graph.  With the plain fp64 sum the result equals the dense sum bit for
 *    bit; the matrix-core paths differ from it by rounding only.  (When the
 *    fragment with the most requested outputs has only quantum inputs and
 *    its tensor would come from variant tables, its tables stand in for the
 *    tensor with the input coefficients moved onto the upstream fragments'
 *    tensors; that fragment's columns are then indexed by preparations.)
 *  CCUT_FLAG_SKIP (ccut_marginal only): fewer downstream evaluations.  The
 *    support is fixed first from the Clifford fragments' exact Pauli
 *    tensors (known before any variant is sampled; non-Clifford fragments do
 *    not restrict it), every sampled Clifford variant that no supported cut
 *    term reads gets no sample model and draws no shots (a quantum input's
 *    |0> and |1> serve every Pauli, |+> only X, |+i> only Y; a quantum
 *    output's Z basis serves I and Z, X only X, Y only Y), the tensors stay
 *    in the Pauli basis and only the supported terms are summed.  Exact data: the dense result up to
 *    rounding.  Synchronizes (the support is read back); not with
 *    CCUT_FLAG_ML.  Non-Clifford variants are all evaluated (their state
 *    vectors share the gate program across preparations).
 *  CCUT_FLAG_SETTLE (ccut_zexpect in sampled mode only): each sampled
 *    Clifford variant's string expectation, which is -1, 0 or +1 on a
 *    stabilizer state, is settled from its shots: 0 if both parities
 *    occurred, else the common sign.
 * Maximum-likelihood fragment correction (Sec. V-C, distribution builder:
 * self-consistent fragment models before the contraction):
 *  CCUT_FLAG_ML (ccut_marginal, ccut_variant_tables, ccut_fragment_tensor):
 *    the variant tables of every fragment with quantum outputs are replaced
 *    by those of the physical model nearest the data.  Per preparation
 *    combination s of the quantum inputs, the model is the set of
 *    conditional states rho_x of the quantum outputs jointly with outcome x
 *    of the requested outputs; the data give rho_x by least-squares
 *    inversion (each Pauli coefficient the mean over the basis combinations
 *    that measure it); the correction projects the joint spectrum of the
 *    rho_x onto the probability simplex (every rho_x positive
 *    semidefinite, sum_x Tr rho_x = 1; the nearest such model in the
 *    Frobenius norm, the maximum-likelihood one under Gaussian noise) and
 *    writes back p(o, x | s, b) = Tr(Pi_{b,o} rho_x).  Exact data are left
 *    unchanged up to rounding.  At most 2 quantum outputs and 8 quantum
 *    inputs per corrected fragment (else CCUT_E_UNSUPPORTED); fragments
 *    whose tensors come from the Heisenberg picture (exact mode) have no
 *    tables and are exact already.
 * A flag outside its call's scope, or in a batch, is CCUT_E_UNSUPPORTED;
 * unknown bits are CCUT_E_INVALID. */
enum { CCUT_FLAG_SPARSE = 1, CCUT_FLAG_SETTLE = 2, CCUT_FLAG_ML = 4, CCUT_FLAG_SKIP = 8 };

/* ---------------------------------------------------------------- context */

/* Create a context.  opts may be NULL (device 0, null stream, hipMalloc,
 * defaults).  Selects the device; errors: CCUT_E_DEVICE (no such device),
 * CCUT_E_OOM. */
ccut_status ccut_ctx_create(const ccut_opts *opts, ccut_ctx **out);
void ccut_ctx_destroy(ccut_ctx *ctx);

/* Text of the last error on this context (valid until the next call on
 * it); "" if none.  ctx may be NULL for errors of ccut_ctx_create and
 * ccut_sample_terms_noalloc (per host thread). */
const char *ccut_last_error(const ccut_ctx *ctx);

/* Ask a running evaluation on this context to stop; it returns
 * CCUT_E_CANCELLED.  The flag is cleared when the next evaluation starts. */
void ccut_cancel(ccut_ctx *ctx);

/* ---------------------------------------------------------------- plans */

/* Validate the circuit and cut list, split cut wires into segments, form
 * fragments as connected components of segments joined by two-qubit gates
 * (Secs. III-B, V-A), tag each fragment Clifford or not (Sec. V-B) and
 * enumerate its variants.  ops/cuts are host arrays, copied.
 * Errors: CCUT_E_INVALID (qubit out of range, q0 == q1 on a two-qubit gate,
 * unknown kind, a cut whose after_op does not act on its qubit, duplicate
 * cut), CCUT_E_NC_TOO_WIDE, CCUT_E_TOO_MANY_CUTS, CCUT_E_OOM. */
ccut_status ccut_plan_create(ccut_ctx *ctx, uint32_t n_qubits, const ccut_op *ops, size_t n_ops,
                             const ccut_cut *cuts, size_t k, ccut_plan **out);
void ccut_plan_destroy(ccut_plan *plan);

/* Number of fragments, total fragment variants, and 4^k cut terms. */
ccut_status ccut_plan_info(const ccut_plan *plan, uint32_t *n_fragments, uint64_t *n_variants,
                           uint64_t *n_terms);

/* Fragment f: its width m, 1 if Clifford, number of incident cut axes, and
 * number of variants (4^inputs * 3^outputs). */
ccut_status ccut_fragment_info(const ccut_plan *plan, uint32_t f, uint32_t *m, int32_t *clifford,
                               uint32_t *n_axes, uint64_t *n_variants);

/* Fragment f's local qubits in order: wires[i], segments[i] (segment index
 * along the wire); arrays of length m. */
ccut_status ccut_fragment_segments(const ccut_plan *plan, uint32_t f, uint32_t *wires,
                                   uint32_t *segments);

/* Fragment f's cut axes in variant-digit order: cut index, side (0 = quantum
 * output, upstream of the cut; 1 = quantum input, downstream) and local
 * qubit; arrays of length n_axes. */
ccut_status ccut_fragment_axes(const ccut_plan *plan, uint32_t f, uint32_t *cut, uint32_t *side,
                               uint32_t *local);

/* ---------------------------------------------------------------- evaluation */

/* Reconstructed output marginal over qubits[0..nq) (Sec. V-C):
 *   R[b] = 2^-k sum_{P in {I,X,Y,Z}^k} prod_f T_f[b_f; P|f],
 * bit i of b = outcome of qubits[i].  out has 2^nq doubles, caller-owned,
 * on the device if out_on_device else on the host.  nq <= 24.
 * Errors: CCUT_E_INVALID (repeated or out-of-range qubit, nq > 24),
 * CCUT_E_DEVICE (host-only context), CCUT_E_UNSUPPORTED (an outcome
 * table over more than 24 measured qubits), CCUT_E_CANCELLED, CCUT_E_OOM. */
ccut_status ccut_marginal(ccut_plan *plan, const ccut_eval_opts *eo, const uint32_t *qubits,
                          uint32_t nq, double *out, int out_on_device);

/* <Z_z> for n_strings masks; masks is a host array [n_strings][ceil(n/64)]
 * of uint64 words (bit q of the mask = qubit q).  out has n_strings doubles.
 * Each fragment measures its circuit outputs that occur in any mask plus
 * its quantum outputs (at most 1024 for a Clifford fragment evaluated
 * from its variants: sampled, or exact with CCUT_METHOD_VARIANTS; beyond
 * 64 its sample models span several words per outcome vector).
 * In exact mode each Clifford variant gives -1, 0 or +1 (Sec. IX). */
ccut_status ccut_zexpect(ccut_plan *plan, const ccut_eval_opts *eo, const uint64_t *masks,
                         uint32_t n_strings, double *out, int out_on_device);

/* Call graphs (default on).  A ccut_marginal or ccut_zexpect call with a
 * device output that repeats an earlier call on the same plan exactly (same
 * options, request and output address) is captured as a HIP graph on its
 * second occurrence and replayed from then on: every kernel and copy runs
 * again, only the host-side planning and launch overhead is saved.  Up to 8
 * graphs per plan (least recently used out).  Calls with host outputs, with
 * kernel timing enabled, or issued while the context's stream is being
 * captured by the caller always run eagerly.  enable = 0 turns replay off
 * (captured graphs are kept until their plan is destroyed).  Errors:
 * CCUT_E_INVALID (NULL context). */
ccut_status ccut_call_graphs(ccut_ctx *ctx, int enable);

/* Parity hook: the sampled shot records of Clifford fragment `fragment`
 * for variants [v_begin, v_end) under the marginal request qubits[0..nq):
 * with RW = 1 for at most 64 measured qubits, else ceil(n_meas / 64),
 * out[((v - v_begin) * shots + s) * RW + w] holds outcome bits 64 w ..
 * 64 w + 63 of shot s (bit j = measurement j of the measured set, at most
 * 1024).  Needs shots > 0. */
ccut_status ccut_shot_records(ccut_plan *plan, const ccut_eval_opts *eo, const uint32_t *qubits,
                              uint32_t nq, uint32_t fragment, uint64_t v_begin, uint64_t v_end,
                              uint64_t *out, int out_on_device);

/* Parity hook: per-variant outcome distributions of fragment `fragment`
 * under the request: out[v][x], 2^|measured set| doubles per variant
 * (exact tables, state-vector marginals, or shot frequencies: count x
 * fl(1 / shots), the fp64 product with the rounded reciprocal). */
ccut_status ccut_variant_tables(ccut_plan *plan, const ccut_eval_opts *eo, const uint32_t *qubits,
                                uint32_t nq, uint32_t fragment, double *out, int out_on_device);

/* Parity hook: the fragment's Pauli-basis tensor T_f[p_f][b_f] (p_f =
 * sum_j P_j 4^j over its axes, I=0 X=1 Y=2 Z=3; b_f bit i = i-th requested
 * output of the fragment in measured order). */
ccut_status ccut_fragment_tensor(ccut_plan *plan, const ccut_eval_opts *eo, const uint32_t *qubits,
                                 uint32_t nq, uint32_t fragment, double *out, int out_on_device);

/* The op stream the kernels run for fragment f: number of one-qubit words
 * (fused runs: 2x2 unitaries on non-Clifford fragments, GF(2) maps on
 * Clifford ones) and of two-qubit gates. */
ccut_status ccut_fragment_ops(const ccut_plan *plan, uint32_t f, uint32_t *n_one, uint32_t *n_two);

/* Number of measured qubits and requested outputs of fragment `fragment`
 * under the marginal request (sizes of the two parity hooks above). */
ccut_status ccut_request_info(ccut_plan *plan, const uint32_t *qubits, uint32_t nq,
                              uint32_t fragment, uint32_t *n_measured, uint32_t *n_requested);

/* ---------------------------------------------------------------- batches */

/* Many circuits at once (each plan is one circuit; its variant ids use its
 * position i in the batch as the circuit index, eo->circuit is ignored).
 * The affine sample models of all Clifford fragment variants of all plans
 * come from one work-queue launch whose workgroup size and workgroups per
 * CU are picked by timing the candidates at creation.  The choice is kept
 * for the process, keyed by the device and the batch's model work (item
 * count and elimination cost, bucketed), and, when the environment variable
 * CCUT_TUNE_CACHE names a file, read from and appended to that file so
 * later processes skip the timing.  The remaining steps follow, and with
 * use_graph != 0 the whole evaluation is captured once as a HIP graph and
 * replayed by ccut_batch_run.
 * qubits[i] / nq[i] are each plan's marginal request (nq[i] <= 24).  The
 * batch owns its device memory; plans must outlive it.  Creating a batch
 * runs one full evaluation.  Errors: as ccut_marginal. */
typedef struct ccut_batch ccut_batch;
ccut_status ccut_batch_create(ccut_ctx *ctx, ccut_plan *const *plans, size_t n, const ccut_eval_opts *eo,
                              const uint32_t *const *qubits, const uint32_t *nq, int use_graph, ccut_batch **out);
/* Evaluate the batch again (graph replay when captured); outs[i] receives
 * plan i's 2^nq[i] marginal, on the device if outs_on_device.  Host
 * outputs: returns once they are written.  Device outputs: a replay's
 * contractions write them in place (an eager run, or a plan whose
 * contraction has a launch of its own, goes through one copy launch), and
 * the context's stream is ordered after the batch; the call returns without
 * waiting (work queued later on that stream sees the results).  Runs of one
 * batch are ordered among themselves; a run with other output addresses
 * than the previous one first waits for the previous one. */
ccut_status ccut_batch_run(ccut_batch *b, double *const *outs, int outs_on_device);
/* Work items of the affine-model launch, the chosen workgroup size and
 * grid, whether that choice came from the tuning cache (1) or from timing
 * at creation (0), whether a graph was captured, and the best tuned time of
 * the model launch in ms (the cached one on a cache hit).  Any pointer may
 * be NULL. */
ccut_status ccut_batch_info(const ccut_batch *b, uint64_t *n_items, uint32_t *block, uint32_t *grid,
                            int32_t *tune_cached, int32_t *graphed, double *models_ms);
void ccut_batch_destroy(ccut_batch *b);
/* One-shot convenience: create (no graph), run into host buffers, destroy. */
ccut_status ccut_run_batch(ccut_ctx *ctx, ccut_plan *const *plans, size_t n, const ccut_eval_opts *eo,
                           const uint32_t *const *qubits, const uint32_t *nq, double *const *outs);

/* ------------------------------------------------ learned term proposal */

/* Importance sampling of the recombination sum (Sec. V-C), whose 4^k cut
 * terms make exhaustive contraction the method's cost wall (Sec. III-B).
 * The paper has no learned part; readings of this extension:
 *  - the weight of term P is the vector w_P(b) = 2^-k prod_f T_f[b_f; P|f];
 *    its label is y(P) = ln(||w_P||_2 + 2^-60), and ||w_P||_2 is the
 *    product of the fragments' column norms;
 *  - features (width F = 6k rounded up to 64, bf16): per cut c, a one-hot
 *    of P_c, then phi(share_up(c, P_c)) and phi(share_down(c, P_c)), where
 *    share_side(c, p) is the fraction of the squared column-norm mass of the
 *    fragment on that side of c (up: c is its quantum output; down: its
 *    quantum input) held by columns with digit p on c, and
 *    phi(s) = max(ln s, -40) / 40;
 *  - proposal q = (1 - eps) softmax(logits) + eps / 4^k;
 *  - term j of a draw: u = (o1 2^32 + o0) mod C[4^k - 1] with
 *    (o0, o1) = philox(ctr = (j, 0, lo32(cid), hi32(cid)),
 *    key = (lo32(seed) ^ 0x7E570001, hi32(seed))), C the inclusive prefix sum
 *    of floor(q_P 2^40); the term is the smallest P with C[P] > u;
 *  - estimate R_hat[b] = (1/N) sum_j w_{P_j}(b) / q(P_j), summed in fp64.
 * Every device pointer below is caller-owned device memory. */
typedef struct ccut_learned ccut_learned; /* per-circuit term model */
typedef struct ccut_mlp ccut_mlp;         /* F -> H -> H -> H -> 1 ReLU network */

/* Evaluate every fragment tensor of the marginal request once (as
 * ccut_marginal would: shots, seed, method and circuit from eo) and keep
 * them with their column norms and per-cut share tables on the device. */
ccut_status ccut_learned_create(ccut_plan *plan, const ccut_eval_opts *eo, const uint32_t *qubits, uint32_t nq,
                                ccut_learned **out);
/* k cuts, 4^k terms, feature width F. */
ccut_status ccut_learned_info(const ccut_learned *L, uint32_t *k, uint64_t *n_terms, uint32_t *width);
/* Feature rows x[n][F] (bf16) of terms[0..n) (device u64), or of terms
 * first..first+n-1 when terms is NULL. */
ccut_status ccut_learned_features(ccut_learned *L, const uint64_t *terms, uint64_t first, uint64_t n,
                                  uint16_t *x);
/* kind 0: labels y(P) (fp32); kind 1: the product-of-shares log-weights
 * sum_c 40 (phi_up + phi_down) (the proposal without a network); kind 2:
 * y(P) / 40, the network's regression target. */
ccut_status ccut_learned_log_weights(ccut_learned *L, const uint64_t *terms, uint64_t first, uint64_t n, int kind,
                                     float *y);
/* The terms with nonzero weight in ascending order: the first min(count,
 * cap) go to terms[], the total count to *count (host). */
ccut_status ccut_learned_support(ccut_learned *L, uint64_t cap, uint64_t *terms, uint64_t *count);
/* Network logits over all 4^k terms (fp32 [4^k]): 40 times the network
 * output on each term's feature row. */
ccut_status ccut_learned_logits(ccut_learned *L, ccut_mlp *mlp, float *logits);
/* Draw n terms from q (fp64 [4^k]) with circuit id = eo->circuit of the
 * create call and contract them: out[2^nq] = R_hat (host or device).
 * terms_out (device, n entries) may be NULL. */
ccut_status ccut_learned_estimate(ccut_learned *L, const double *q, uint64_t n, uint64_t seed, double *out,
                                  int on_device, uint64_t *terms_out);
/* The exhaustive contraction of the kept tensors in eo->precision of the
 * create call (equals ccut_marginal with that precision). */
ccut_status ccut_learned_exhaustive(ccut_learned *L, double *out, int on_device);
void ccut_learned_destroy(ccut_learned *L);

/* The whole learned path of one marginal request (Sec. V-C importance
 * sampling with the network as proposal): fragment tensors as
 * ccut_learned_create (eo as there), logits of `mlp` over all 4^k terms, q
 * with eps = 0.05, n_terms (1 <= n_terms < 2^32) terms drawn with
 * seed = eo->seed and cid = eo->circuit, and the estimate into out[2^nq]
 * (host, or device when out_on_device).  When out_stderr_l1 (host) is not
 * NULL it receives sum_b se_b, se_b = sqrt(max(0, M2_b - R_hat[b]^2 / N))
 * with M2_b = (1/N^2) sum_j (w_{P_j}(b) / q(P_j))^2: the plug-in standard
 * error of each estimated entry, summed over b (one more term-list
 * contraction of squared operands, then a synchronization).  Temporary
 * state lives only for the call; mlp keeps its parameters. */
ccut_status ccut_learned_marginal(ccut_plan *plan, const ccut_eval_opts *eo, ccut_mlp *mlp, uint64_t n_terms,
                                  const uint32_t *qubits, uint32_t nq, double *out, int out_on_device,
                                  double *out_stderr_l1);

/* q[K] (fp64) from logits[K] (fp32), or uniform when logits is NULL. */
ccut_status ccut_proposal(ccut_ctx *ctx, const float *logits, uint64_t K, double eps, double *q);
/* n terms drawn from q[K] as above (device u64 out[n]). */
ccut_status ccut_sample_terms(ccut_ctx *ctx, const double *q, uint64_t K, uint64_t n, uint64_t seed, uint64_t cid,
                              uint64_t *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the draw
 * of ccut_sample_terms (same terms for the same q, n, seed, cid) without a
 * context and without any allocation.  The integer CDF and the scan
 * partials live in one fixed device array of the library, 8 MiB + 16 KiB on
 * each device it runs on, held until the process ends; so K <= 2^20 (the
 * 4^10 terms of ten cuts), larger K is CCUT_E_UNSUPPORTED.  Runs on the
 * current HIP device, enqueued on hip_stream (hipStream_t, NULL = null
 * stream); returns without waiting: out (device u64[n]) is valid in stream
 * order.  q (device fp64 [K]) and out are caller-owned.  Every call on one
 * device shares that array: calls that overlap on a device (other streams,
 * other host threads) race and must be ordered by the caller.  Errors
 * (text in ccut_last_error(NULL)): CCUT_E_INVALID (NULL q, NULL out with
 * n > 0, K = 0, n >= 2^32), CCUT_E_UNSUPPORTED (K > 2^20), CCUT_E_DEVICE (no
 * current device, symbol lookup or launch failure). */
ccut_status ccut_sample_terms_noalloc(void *hip_stream, const double *q, uint64_t K, uint64_t n, uint64_t seed,
                                      uint64_t cid, uint64_t *out);

/* Network with F inputs (F % 64 == 0) and width H (H % 64 == 0, H <= 256).
 * Parameters, flat fp32 in this order: W1[H][F], b1[H], W2[H][H], b2[H],
 * W3[H][H], b3[H], w4[H], b4 (count H F + 2 H^2 + 4 H + 1).  Products use
 * bf16 copies of the weights and activations with fp32 accumulation; the
 * master parameters and Adam state are fp32. */
ccut_status ccut_mlp_create(ccut_ctx *ctx, uint32_t F, uint32_t H, ccut_mlp **out);
/* Set (resets the Adam state) or read the parameters (host arrays). */
ccut_status ccut_mlp_set_params(ccut_mlp *M, const float *params, size_t count);
ccut_status ccut_mlp_get_params(ccut_mlp *M, float *params, size_t count);
/* y[n] (fp32, device) from x[n][F] (bf16, device). */
ccut_status ccut_mlp_forward(ccut_mlp *M, const uint16_t *x, uint64_t n, float *y);
/* Mean squared error against t[n] and its gradient (host, flat layout as
 * the parameters); n % 64 == 0. */
ccut_status ccut_mlp_gradients(ccut_mlp *M, const uint16_t *x, const float *t, uint64_t n, float *grads,
                               double *loss);
/* `steps` Adam steps (lr, b1 = 0.9, b2 = 0.999, eps = 1e-8), each on a
 * mini-batch of `batch` rows (batch % 64 == 0) of the data set x[n][F],
 * t[n]: row i of step s is data row philox(ctr = (i, s, 0x4D4C5000, 0),
 * key = seed) mod n, or row i when batch == n.  losses (host, `steps`
 * entries) may be NULL. */
ccut_status ccut_mlp_train(ccut_mlp *M, const uint16_t *x, const float *t, uint64_t n, uint32_t batch,
                           uint32_t steps, float lr, uint64_t seed, float *losses);
/* One Adam step (as ccut_mlp_train) on the whole batch x[n][F] (fp32,
 * device; rounded to bf16 to nearest-even before the products), t[n] (fp32,
 * device), rows in order; n % 64 == 0, n <= 2^24.  loss (host, may be
 * NULL) receives the batch's mean squared error before the step.  Equals
 * ccut_mlp_train(batch = n, steps = 1) on the bf16-rounded rows. */
ccut_status ccut_mlp_train_step(ccut_mlp *M, const float *x, const float *t, uint64_t n, float lr, float *loss);
void ccut_mlp_destroy(ccut_mlp *M);

/* ---------------------------------------------------------------- timing */

/* Kernel timing with HIP events recorded around every launch on the
 * context's stream.  While enabled, ccut_timing_read returns for kernel id
 * `kid` the number of launches and their summed duration in ms since the
 * last reset. */
enum {
  CCUT_K_AFFINE = 0, /* affine sample models (carry-back + per-variant elimination) */
  CCUT_K_SAMPLE = 1,
  CCUT_K_HIST_REDUCE = 2,
  CCUT_K_EXACT = 3,
  CCUT_K_SV = 4,
  CCUT_K_PARITY = 5,
  CCUT_K_TRANSFORM = 6,
  CCUT_K_RECOMBINE = 7,
  CCUT_K_ZRECOMBINE = 8,
  CCUT_K_HEISENBERG = 9,
  CCUT_K_MLP = 10,
  CCUT_K_TERMS = 11,
  CCUT_K_CARRY = 12, /* a batch's carry-back of the measured Paulis, all Clifford fragments */
  CCUT_K_COUNT = 13
};
ccut_status ccut_timing_enable(ccut_ctx *ctx, int enable);
ccut_status ccut_timing_reset(ccut_ctx *ctx);
ccut_status ccut_timing_read(ccut_ctx *ctx, uint32_t kid, uint64_t *launches, double *total_ms);
const char *ccut_kernel_name(uint32_t kid);

#ifdef __cplusplus
}
#endif
#endif /* CCUT_ABI_H_ */
