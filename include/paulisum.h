/* paulisum.h -- C ABI of the MI355X Pauli-sum product library.
 *
 * A Pauli sum H = sum_t i^{k_t} c_t P_t (Section III-A, eq. (2)) lives on one
 * GPU in bit-packed binary symplectic form (Section III-C, Table I).  The
 * library forms the outer product of two sums (Section IV-C, "Hamiltonian
 * Multiplication" in Section V), and combines duplicate strings by sorting
 * and one linear pass (Section III-H).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - n qubits, W = ceil(n/64) words, 1 <= n <= 1024.  Qubit q is bit (q % 64)
 *    of word (q / 64) in both the X words and the Z words; bits at or above
 *    n must be zero.  Letter per qubit (Table I): (x,z) = (0,0) I, (0,1) Z,
 *    (1,0) X, (1,1) Y.
 *  - Host-side string arrays are row-major [m][W] uint64.
 *  - A term's value is i^k * c * P with k in {0,1,2,3} (the 2-bit phase of
 *    Section III-C) and c complex.  Coefficients are interleaved (re, im):
 *    double pairs for PAULI_C128, float pairs for PAULI_C64.
 *  - "stream" is a hipStream_t (NULL = the default stream).  Every call is
 *    stream-ordered; a call returns once its work is enqueued, except where a
 *    call states that it synchronises.
 *  - Every call returns a pauli_status_t and never throws.  On error the
 *    out-parameters are left untouched and pauli_last_error() gives a
 *    message (per thread).
 *  - Every handle returned by a call is owned by the caller, who destroys it
 *    exactly once with paulisum_destroy.  Handles are bound to the device
 *    that was current when they were made.
 */
#ifndef PAULISUM_H
#define PAULISUM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PAULI_OK = 0,
  PAULI_ERR_INVALID = 1,  /* bad argument: null pointer, n out of range, padding bits, phase > 3 */
  PAULI_ERR_SHAPE = 2,    /* operands disagree (qubit count, coefficient type) */
  PAULI_ERR_OVERFLOW = 3, /* a size exceeds what the pair index or a count can hold */
  PAULI_ERR_OOM = 4,      /* device allocation failed or exceeded the memory budget */
  PAULI_ERR_CAPACITY = 5, /* a result did not fit its preallocated capacity */
  PAULI_ERR_DEVICE = 6    /* a HIP runtime call failed */
} pauli_status_t;

typedef enum { PAULI_C128 = 0, PAULI_C64 = 1 } pauli_dtype_t;

/* flags for paulisum_create / paulisum_export */
#define PAULI_PTR_DEVICE 1u /* the string/phase/coefficient pointers are device memory */

typedef struct paulisum* paulisum_t;

/* Merge options (Section III-H sort-and-combine, Section III-B truncation).
 *  mode        PAULI_MERGE_PLAIN: coefficient products and sums in the sum's
 *              own precision (FP64 for C128).
 *              PAULI_MERGE_COMPENSATED: products and sums in FP32 with
 *              compensated (TwoSum) accumulation; segments whose sum cancels
 *              (|sum| < remerge_tau * sum of |terms|) are recomputed in FP64
 *              from the original coefficients.
 *  drop_abs    terms whose merged modulus is strictly below drop_abs are
 *              removed; a negative value keeps every term (zeros included).
 *  remerge_tau cancellation threshold of the compensated mode (<= 0: 1e-3).
 *  key_bits    0 for the default; otherwise the sort uses only the top
 *              key_bits bits of the 64-bit string fingerprint (testing aid:
 *              forces fingerprint collisions, which are resolved exactly).
 *              A merge of more than 2^(key_bits + 12) records with a key
 *              narrower than 52 bits is refused (INVALID): the strings of a
 *              run of equal keys are put in order one run per thread.
 */
typedef enum { PAULI_MERGE_PLAIN = 0, PAULI_MERGE_COMPENSATED = 1 } pauli_merge_mode_t;
typedef struct {
  int32_t mode;
  double drop_abs;
  double remerge_tau;
  int32_t key_bits;
} pauli_merge_opts_t;

/* Launch shape of the batched form (a field of 0 takes its default; a
 * non-NULL tune turns the autotuner off).
 *  bucket_bits     every product's records are split into 2^bucket_bits
 *                  buckets by the top bits of their key, each bucket sorted
 *                  in LDS; 0..16 (0: from bucket_records).
 *  bucket_records  records per bucket the bucket bits aim at (the tile size
 *                  of the LDS bucket sort), 256..8192; default 3500.  A
 *                  bucket over 4096 records (the LDS capacity) is sorted in
 *                  global memory instead.
 *  class_bits      at most this many of a product's bucket bits come from
 *                  the class tiles of the record generation; the rest
 *                  (at most 8) form the radix digit of its partition pass
 *                  (the radix width); 0..8, default 8.
 *  expand_parts    work items per bucket of the expand kernel (the records
 *                  each wave takes at a time); 1, 2, 4 or 8, default 4. */
typedef struct {
  int32_t bucket_bits;
  int32_t bucket_records;
  int32_t class_bits;
  int32_t expand_parts;
} pauli_tune_t;

/* Text of a status code (static storage). */
const char* pauli_status_string(pauli_status_t s);
/* Detail of the last error on the calling thread ("" if none). */
const char* pauli_last_error(void);

/* paulisum_create: a device Pauli sum from packed words (Section III-D: a
 * coefficient vector alongside a binary matrix whose rows are the strings).
 *  n_qubits  1..1024
 *  n_terms   >= 0 (0 gives an empty sum)
 *  x_words, z_words  [n_terms][W] row-major
 *  phase     [n_terms] exponents 0..3, or NULL for all zero
 *  coef      [n_terms] interleaved (re, im) of dtype
 *  flags     PAULI_PTR_DEVICE if the four arrays are device memory; host
 *            arrays are copied before the call returns, device arrays are read
 *            on `stream` and must stay valid until that work completes
 *  Errors: INVALID for n out of range, n_terms < 0, a null array (with
 *  n_terms > 0), a set bit at or above n, a phase above 3.  Duplicate strings
 *  are allowed; their values add up under pauli_merge.  Synchronises the
 *  stream when the inputs are device arrays (to report validation errors).
 */
pauli_status_t paulisum_create(int32_t n_qubits, int64_t n_terms, const uint64_t* x_words,
                               const uint64_t* z_words, const uint8_t* phase, const void* coef,
                               pauli_dtype_t dtype, uint32_t flags, void* stream, paulisum_t* out);

/* Releases a sum (NULL is allowed).  Waits for the device to finish work
 * that may still read it. */
pauli_status_t paulisum_destroy(paulisum_t s);

/* Qubit count, term count and coefficient type of a sum (any pointer may be
 * NULL). */
pauli_status_t paulisum_info(paulisum_t s, int32_t* n_qubits, int64_t* n_terms,
                             pauli_dtype_t* dtype);

/* Copies a sum out in the create layout: x, z [m][W], phase [m], coef [m]
 * interleaved (re, im) of the sum's dtype, fingerprint [m] (the 64-bit key
 * that orders merged sums; see pauli_merge).  Any pointer may be NULL.
 * flags = PAULI_PTR_DEVICE for device destinations (stream-ordered), else
 * host destinations (the call synchronises the stream). */
pauli_status_t paulisum_export(paulisum_t s, uint64_t* x_words, uint64_t* z_words,
                               uint8_t* phase, void* coef, uint64_t* fingerprint,
                               uint32_t flags, void* stream);

/* pauli_outer_product: the unmerged outer product H1*H2 (Section IV-C,
 * "Thread-Level Parallelism"; Section V, "Hamiltonian Multiplication").
 * Output term p = j*|a| + i is a_i * b_j: strings X = X_a ^ X_b,
 * Z = Z_a ^ Z_b (Section III-E), phase exponent k_a + k_b + (phase of the
 * string product) mod 4 (Section III-A), coefficient c_a * c_b computed as
 * (re = ac - bd, im = ad + bc) without fused multiply-adds.  a == b is
 * allowed.  Errors: SHAPE if n or dtype differ; OVERFLOW if |a|*|b| >= 2^32.
 */
pauli_status_t pauli_outer_product(paulisum_t a, paulisum_t b, paulisum_t* out, void* stream);

/* pauli_merge: sort-and-combine (Section III-H).  The output holds one term
 * per distinct string of s, with phase 0 and coefficient
 * sum over equal strings of i^k * c, in ascending order of the 64-bit
 * fingerprint fp(P) = XOR over set bits of fixed random 64-bit columns
 * (ties between distinct strings with equal fingerprints are ordered by
 * their packed words).  Zero coefficients are kept unless opts->drop_abs
 * removes them.  opts may be NULL (plain, keep all).  Synchronises the
 * stream once to learn the output size. */
pauli_status_t pauli_merge(paulisum_t s, const pauli_merge_opts_t* opts, paulisum_t* out,
                           void* stream);

/* pauli_merge_into: pauli_merge for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The call allocates nothing: its temporaries live in a
 * fixed device scratch array of 128 MiB that the library holds on each
 * device it runs on until the process ends, and the result is written to
 * arrays the caller passes (device memory, stream-ordered):
 *   out_x, out_z   [W][out_ld] uint64: word w of term t at [w * out_ld + t]
 *   out_phase      [out_ld] uint8 (written 0)
 *   out_coef       [out_ld] interleaved (re, im): s's dtype in the plain
 *                  mode, C64 in the compensated mode
 *   out_fp         [out_ld] uint64 fingerprints
 *   out_m          host: the number of merged terms written
 * The result is merge(s) as pauli_merge defines it (same terms, same order,
 * same values).  Limits: |s| <= 2^20 terms; CAPACITY if |s| is larger, if
 * the merged terms exceed out_ld (out_ld >= |s| always suffices) or if the
 * scratch array is exhausted; then nothing is written to *out_m.  Every call
 * on one device shares that device's scratch array: calls that overlap on
 * one device (other threads, or other streams in flight) race and must be
 * serialised by the caller.  Synchronises the stream once.  Errors as
 * pauli_merge, plus INVALID for a NULL output array or out_ld < 1. */
pauli_status_t pauli_merge_into(paulisum_t s, const pauli_merge_opts_t* opts, uint64_t* out_x,
                                uint64_t* out_z, uint8_t* out_phase, void* out_coef,
                                uint64_t* out_fp, int64_t out_ld, int64_t* out_m, void* stream);

/* pauli_outer_product_merged: merge(outer_product(a, b)) without storing
 * the |a|*|b| unmerged products.  Same output definition as pauli_merge.
 * With |a|*|b| >= 2^32 (beyond one pipeline's 32-bit pair index) the plain
 * merge forms and merges the products of the smaller operand with ranges of
 * the larger one's terms (about 2^31 products each), then merges the merged
 * ranges once more; the drop applies to that final merge, and the sums add
 * the same products in another order.  The merged ranges must fit device
 * memory together (OOM otherwise) and hold fewer than 2^32 terms (OVERFLOW).
 * Errors as pauli_outer_product, except that OVERFLOW at |a|*|b| >= 2^32
 * applies to the compensated mode only. */
pauli_status_t pauli_outer_product_merged(paulisum_t a, paulisum_t b,
                                          const pauli_merge_opts_t* opts, paulisum_t* out,
                                          void* stream);

/* pauli_commutator: [a, b] = a*b - b*a, merged.  A pair of strings
 * commutes or anticommutes by the parity of its symplectic product
 * (Section III-F); a_i b_j - b_j a_i is 2 a_i b_j for an anticommuting pair
 * and zero for a commuting one (the commutator evaluation the conclusion
 * lists as planned work).  The output holds one term per string that at
 * least one anticommuting pair gives, with coefficient
 * sum over those pairs of 2 i^k c_a c_b, in the order and form of
 * pauli_merge (phase 0, zeros kept unless opts->drop_abs removes them).
 * Strings that only commuting pairs give are absent; [a, a] holds every
 * string of an anticommuting pair of a with coefficient exactly 0.
 * opts as pauli_merge (the compensated mode applies as in
 * pauli_outer_product_merged).  Errors as pauli_outer_product. */
pauli_status_t pauli_commutator(paulisum_t a, paulisum_t b, const pauli_merge_opts_t* opts,
                                paulisum_t* out, void* stream);

/* Gate kinds of pauli_apply_clifford (Section V-B lists H, S, CNOT, CZ;
 * S^dagger, the Pauli gates and SWAP are Cliffords of the same form). */
typedef enum {
  PAULI_GATE_H = 0,
  PAULI_GATE_S = 1,    /* diag(1, i) */
  PAULI_GATE_SDG = 2,  /* diag(1, -i) */
  PAULI_GATE_X = 3,
  PAULI_GATE_Y = 4,
  PAULI_GATE_Z = 5,
  PAULI_GATE_CX = 6,   /* control q0, target q1 */
  PAULI_GATE_CZ = 7,
  PAULI_GATE_SWAP = 8
} pauli_gate_kind_t;

typedef struct {
  int32_t kind; /* pauli_gate_kind_t */
  int32_t q0;   /* qubit (0-based) */
  int32_t q1;   /* second qubit of CX, CZ, SWAP; ignored otherwise */
} pauli_gate_t;

/* pauli_apply_clifford: conjugation of every term by a Clifford circuit
 * (Section III-B, Clifford paragraph: a Clifford maps each string to a single
 * string, so the number of terms does not change; Section V-B, "Gate
 * Application").  Term t of the output is C (i^k c P) C^dagger with
 * C = G_{n_gates-1} ... G_1 G_0 (gates[0] conjugates first): its string is
 * relabelled, its phase exponent gains 2 for every sign flip, its
 * coefficient is unchanged and its fingerprint is updated.  The output keeps
 * the input's term order (it is not re-sorted; pauli_merge restores the
 * canonical order).  gates is a host array; n_gates = 0 copies s.  Errors:
 * INVALID for an unknown kind, a qubit outside [0, n), or a two-qubit gate
 * on one qubit. */
pauli_status_t pauli_apply_clifford(paulisum_t s, int32_t n_gates, const pauli_gate_t* gates,
                                    paulisum_t* out, void* stream);

/* pauli_sort_lex: the terms of s in lexicographic order of their packed
 * words (Section III-H: the canonical sum is sorted on a key formed from the
 * bit-packed words of each string).  Terms are compared on the tuple
 * (X[W-1], ..., X[0], Z[W-1], ..., Z[0]) of their words, each compared as an
 * unsigned 64-bit integer (for n <= 32 the order of the integer x 2^32 + z).
 * pauli_merge orders its output by fingerprint instead; this call gives a
 * merged sum the string order.  Terms with equal strings keep
 * their input order; phases, coefficients and fingerprints travel with their
 * strings.  s is not changed; *out is a new sum of |s| terms that the caller
 * destroys.  Errors: INVALID for NULL arguments, CAPACITY beyond 2^32 terms,
 * OOM. */
pauli_status_t pauli_sort_lex(paulisum_t s, paulisum_t* out, void* stream);

/* pauli_outer_product_batched: nb independent products
 * out[t] = merge(a[t] * b[t]) (the outer product of Section IV-C and the
 * merge of Section III-H, each exactly as pauli_outer_product_merged gives
 * it: same terms, order and values) with one set of merge options.  The
 * pairs may differ in qubit count and term counts; a[t] and b[t] must agree
 * with each other.  Products with the same word count and coefficient type
 * run together: one launch per stage covers all of them (one generation
 * over the pair tiles of every product, one bucket sort whose bucket index
 * holds the product above the key bits, one expand), with no host
 * synchronisation between stages.  tune == NULL: each class of products
 * (word count, size, precision, mode) takes the launch shape measured
 * fastest for it, timed on the first batch of the class this process meets
 * (every candidate computes the same result) or read from the tune table
 * (pauli_tune_load, or the file named by the environment variable
 * PAULI_TUNE_FILE, which is also rewritten after each new measurement).
 * Results are views into one output block per class (released with the
 * last of them); with opts->drop_abs >= 0 one compaction per class moves
 * the kept terms of all its products into a block of exactly their size
 * (one more synchronisation).  Errors: those of pauli_outer_product_merged
 * for each pair; INVALID for a bad tune field or key_bits in 1..29.  On
 * error no output is returned.  Synchronises the stream once (twice with a
 * drop). */
pauli_status_t pauli_outer_product_batched(int32_t nb, const paulisum_t* a, const paulisum_t* b,
                                           const pauli_merge_opts_t* opts,
                                           const pauli_tune_t* tune, paulisum_t* out,
                                           void* stream);

/* Batch plans: the batched form captured once into a HIP graph and replayed.
 *  pauli_batch_plan_create  allocates the buffers of the batch (the inputs
 *      a[t], b[t] must stay alive and unchanged while the plan exists),
 *      tunes its launch shapes as pauli_outer_product_batched does, and
 *      captures the whole launch sequence into a graph.
 *  pauli_batch_plan_run     launches the graph, ordered after earlier work
 *      on `stream` and before later work on it; no host synchronisation.
 *  pauli_batch_plan_results waits for the last run and returns its nb
 *      products (as pauli_outer_product_batched does); the plan allocates
 *      new output blocks (and captures again) at its next run.  INVALID if
 *      the plan has not run since its last results.
 *  pauli_batch_plan_destroy releases the plan (NULL is allowed); results
 *      already returned stay valid. */
typedef struct pauli_batch_plan* pauli_batch_plan_t;
pauli_status_t pauli_batch_plan_create(int32_t nb, const paulisum_t* a, const paulisum_t* b,
                                       const pauli_merge_opts_t* opts, const pauli_tune_t* tune,
                                       void* stream, pauli_batch_plan_t* out);
pauli_status_t pauli_batch_plan_run(pauli_batch_plan_t plan, void* stream);
pauli_status_t pauli_batch_plan_results(pauli_batch_plan_t plan, paulisum_t* out, void* stream);
pauli_status_t pauli_batch_plan_destroy(pauli_batch_plan_t plan);

/* The autotuner's table of launch shapes per class, as text (one class per
 * line): pauli_tune_save writes it, pauli_tune_load merges a saved one into
 * the table.  INVALID if the file cannot be written or read, or a line is
 * malformed (then no line of the file is applied). */
pauli_status_t pauli_tune_save(const char* path);
pauli_status_t pauli_tune_load(const char* path);

/* pauli_propagate: a sequence of Pauli rotations applied to a sum (Section
 * III-B: eq. (5) and its truncation).  Step t uses the string
 * P_t = (p_x[t], p_z[t]) (packed as in paulisum_create, W words each, host
 * memory) and the angle theta[t] (host memory); R_t = cos(theta_t) I
 * - i sin(theta_t) P_t.
 *   PAULI_ROTATE_PRODUCT:   S <- merge(R_t * S), every term multiplied on
 *                           the left by the 2-term sum R_t (a fused outer
 *                           product on the first step; on a state already in
 *                           key order, the products I Q keep that order and
 *                           only the products P_t Q are sorted before the
 *                           merge).
 *   PAULI_ROTATE_CONJUGATE: terms commuting with P_t are kept; each
 *                           anticommuting term Q becomes
 *                           cos(theta_t) Q - i sin(theta_t) P_t Q; then merge.
 * Every step ends with the merge of opts (mode, drop_abs, ...), so a
 * drop_abs >= 0 truncates after each step.  steps == 0 returns merge(s).
 * In the compensated mode the state is carried between steps as
 * float-float pairs (about 48 significant bits; products by TwoProduct,
 * sums by TwoSum, cancelled segments re-merged in FP64 from the carried
 * state), starting from merge(s), and only the output is rounded to C64.
 * s is not modified; *out is a new sum (C64 once a compensated step ran).
 * Each step synchronises the stream once per size it has to learn.
 * Errors: INVALID for a NULL argument, steps < 0, an unknown mode or a
 * rotation string with bits at or above n. */
typedef enum { PAULI_ROTATE_PRODUCT = 0, PAULI_ROTATE_CONJUGATE = 1 } pauli_rotate_mode_t;
pauli_status_t pauli_propagate(paulisum_t s, int32_t steps, const uint64_t* p_x,
                               const uint64_t* p_z, const double* theta, int32_t rotate_mode,
                               const pauli_merge_opts_t* opts, paulisum_t* out, void* stream);

/* Propagation plans: the loop of pauli_propagate captured once into a HIP
 * graph (Section III-B eq. (5) and its truncation, step after step) with
 * every size kept on the device, so a run has no host synchronisation.
 * The input is first merged (so the state is in key order from the start;
 * the same sum as pauli_propagate up to the summation order of the first
 * step), then each step is merged into the next state.  Every state holds
 * at most max_terms terms; the plan allocates two such states (three in
 * the compensated mode, whose last step writes C64) and the temporaries of
 * one step (about 200 bytes per term of max_terms).
 *  pauli_propagate_plan_create  arguments as pauli_propagate plus
 *      max_terms (1..2^31-1); s must stay alive and unchanged while the plan
 *      exists; the rotation strings and angles are copied.
 *  pauli_propagate_plan_run     launches the graph, ordered after earlier
 *      work on `stream` and before later work on it.
 *  pauli_propagate_plan_result  waits for the last run and returns its
 *      state (the plan allocates a new state and captures again at its next
 *      run); CAPACITY if a state would have exceeded max_terms; INVALID if
 *      the plan has not run since its last result.
 *  pauli_propagate_plan_destroy releases the plan (NULL is allowed). */
typedef struct pauli_propagate_plan* pauli_propagate_plan_t;
pauli_status_t pauli_propagate_plan_create(paulisum_t s, int32_t steps, const uint64_t* p_x,
                                           const uint64_t* p_z, const double* theta,
                                           int32_t rotate_mode, const pauli_merge_opts_t* opts,
                                           int64_t max_terms, void* stream,
                                           pauli_propagate_plan_t* out);
pauli_status_t pauli_propagate_plan_run(pauli_propagate_plan_t plan, void* stream);
pauli_status_t pauli_propagate_plan_result(pauli_propagate_plan_t plan, paulisum_t* out);
pauli_status_t pauli_propagate_plan_destroy(pauli_propagate_plan_t plan);

/* Replaces the device allocator used for every buffer the library makes
 * (NULL, NULL restores the default: the library's own arena, which reserves
 * memory from the runtime in chunks of at least 256 MiB, hands out blocks by
 * best fit per device and stream, and keeps the chunks until the runtime
 * refuses a new one).  alloc returns NULL on failure.  Not thread-safe with
 * concurrent calls. */
typedef void* (*pauli_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*pauli_free_fn)(void* ptr, void* stream, void* ctx);
pauli_status_t pauli_set_allocator(pauli_alloc_fn alloc, pauli_free_fn free_fn, void* ctx);

/* Returns the device memory the library's arena holds but does not use, on
 * the current device, to the runtime (for callers that share the device with
 * another allocator).  Waits for the device.  No effect with an allocator
 * hook. */
pauli_status_t pauli_trim_memory(void);

/* Upper bound on device bytes the library may hold at once for temporaries
 * and results made by later calls (0 = no limit).  Exceeding it gives OOM. */
pauli_status_t pauli_set_memory_budget(uint64_t bytes);

/* Diagnostics: device time of each stage, measured with HIP events recorded
 * on the stream of the call that launched it, and the algorithmic bytes the
 * stage moves (its compulsory HBM reads and writes, a per-record or per-term
 * figure times the records or terms it processed).
 *   pauli_profile_enable(1) clears the totals and starts recording;
 *   pauli_profile_enable(0) stops.  pauli_profile_read waits for the events
 *   of finished calls and returns the totals of one stage (NULL pointers are
 *   skipped).  Recording adds two event records per kernel launch. */
typedef enum {
  PAULI_STAGE_OUTER_PRODUCT = 0, /* materialised product kernel */
  PAULI_STAGE_PREP = 1,          /* operand preparation */
  PAULI_STAGE_SORT = 2,          /* record generation and radix / partition passes */
  PAULI_STAGE_SEGMENT = 3,       /* bucket sorts, segment heads, segmented reduction */
  PAULI_STAGE_WRITE = 4,         /* output of the merged terms (fused: the expand kernel) */
  PAULI_STAGE_LONG = 5,          /* fused: long segments, drop compaction */
  PAULI_STAGE_CLIFFORD = 6,      /* Clifford gate application */
  PAULI_STAGE_LEX = 7,           /* lexicographic order (pauli_sort_lex) */
  PAULI_STAGE_FILTER = 8,        /* commutator: search for anticommuting pairs; its
                                    algorithmic figure counts 32-bit integer
                                    operations (8W + 2 per pair), not bytes */
  PAULI_STAGE_COUNT = 9
} pauli_stage_t;
pauli_status_t pauli_profile_enable(int32_t on);
pauli_status_t pauli_profile_read(int32_t stage, double* total_ms, int64_t* launches,
                                  double* bytes);

#ifdef __cplusplus
}
#endif

#endif /* PAULISUM_H */
