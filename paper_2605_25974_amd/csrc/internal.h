// Host-side internals: the device container, memory helpers, and the
// launchers each kernel file exports to the C-ABI layer (api.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>
#include <string>
#include <vector>

#include "paulisum.h"

namespace pauli {
constexpr int kMaxWordsHost = 16;  // n <= 1024
}

namespace pauli {
// One device block of SoA arrays X, Z [W][ld], phase, coefficients and
// fingerprints [ld], shared by several sums that are views into it (the
// outputs of a batched launch sequence); released with the last of them.
struct SharedBlock {
  SharedBlock(int W, int64_t ld, int32_t dtype, hipStream_t s);
  ~SharedBlock();
  SharedBlock(const SharedBlock&) = delete;
  SharedBlock& operator=(const SharedBlock&) = delete;
  int W = 0;
  int64_t ld = 0;
  int32_t dtype = 0;
  hipStream_t s = nullptr;
  void* block = nullptr;
  size_t bytes = 0;
  uint64_t* X = nullptr;
  uint64_t* Z = nullptr;
  uint8_t* ph = nullptr;
  void* coef = nullptr;
  uint64_t* fp = nullptr;
};
}  // namespace pauli

struct paulisum {
  int32_t n = 0, W = 0;
  int64_t m = 0;   // number of terms
  int64_t ld = 0;  // column length (capacity) of every SoA array
  int32_t dtype = PAULI_C128;  // pauli_dtype_t, or kDtypeFF inside a propagation loop
  int device = 0;
  void* block = nullptr;  // one allocation backing every array below
  size_t block_bytes = 0;
  uint64_t* X = nullptr;  // [W][ld]
  uint64_t* Z = nullptr;  // [W][ld]
  uint8_t* ph = nullptr;  // [ld]
  void* coef = nullptr;   // [ld] interleaved (re, im) of dtype
  uint64_t* fp = nullptr; // [ld]
  hipStream_t last_stream = nullptr;
  bool borrowed = false;  // arrays owned by the caller of pauli_merge_into
  std::shared_ptr<pauli::SharedBlock> shared;  // a view into a shared block
};

namespace pauli {

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);
struct Error {
  pauli_status_t status;
};
[[noreturn]] void fail(pauli_status_t s, const std::string& msg);
void hip_check(hipError_t e, const char* what);
#define PAULI_HIP(call) ::pauli::hip_check((call), #call)

// ------------------------------------------------------------------ memory
// alloc.cpp: the library's device arena (one per device and stream).
void* arena_alloc(int dev, hipStream_t s, size_t bytes);
void arena_free(void* p, hipStream_t s);
void arena_trim(int dev);  // returns the idle chunks of device dev

void* dalloc(size_t bytes, hipStream_t s);
void dfree(void* p, size_t bytes, hipStream_t s);

// True while a call that allocates nothing (pauli_merge_into) runs on the
// calling thread: dalloc then hands out consecutive pieces of the library's
// fixed device scratch array, dfree releases nothing, new_sum returns the
// caller's output arrays, and stage timing records no events.
bool workspace_active();

// While alive on the calling thread, temporaries (dalloc) come from the
// device region [base, base + bytes) as they do for pauli_merge_into, with
// no result container (CAPACITY when the region is exhausted).  rewind()
// hands the region out again from its start (the caller orders the reuse).
class ScratchScope {
 public:
  ScratchScope(void* base, size_t bytes);
  ~ScratchScope();
  ScratchScope(const ScratchScope&) = delete;
  ScratchScope& operator=(const ScratchScope&) = delete;
  void rewind();
  size_t used() const;

 private:
  void* ws_;
};

// RAII device buffer freed (stream-ordered) when it leaves scope.
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipStream_t s = nullptr;
  DBuf() = default;
  DBuf(size_t b, hipStream_t st) : p(b ? dalloc(b, st) : nullptr), bytes(b), s(st) {}
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), bytes(o.bytes), s(o.s) { o.p = nullptr; }
  DBuf& operator=(DBuf&& o) noexcept {
    reset();
    p = o.p; bytes = o.bytes; s = o.s; o.p = nullptr;
    return *this;
  }
  ~DBuf() { reset(); }
  void reset() {
    if (p) dfree(p, bytes, s);
    p = nullptr;
  }
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

inline int words_for(int n) { return (n + 63) / 64; }
// Internal coefficient type of a propagation state in the precision form:
// per term {re.hi, re.lo, im.hi, im.lo} as floats (float-float pairs).  It
// never leaves the library: the last step of a loop writes C64.
constexpr int32_t kDtypeFF = 2;
inline size_t coef_bytes(int32_t t) { return t == PAULI_C64 ? 8 : 16; }

// Allocates a container with capacity ld (>= m) on the current device.
paulisum* new_sum(int n, int64_t m, int64_t ld, int32_t dt, hipStream_t s);
void free_sum(paulisum* p);
// A sum of m terms on n qubits that are terms [first, first + m) of b.
paulisum* sum_view(const std::shared_ptr<SharedBlock>& b, int n, int64_t first, int64_t m);

// ---------------------------------------------------------------- profiling
// While a NoEvents guard lives on the calling thread, stages record no
// events (a launch sequence being captured into a graph).
struct NoEvents {
  NoEvents();
  ~NoEvents();
};
// Records HIP events around a stage on its stream while profiling is on.
struct StageScope {
  StageScope(int stage, hipStream_t s, double bytes);
  ~StageScope();
  void stop();  // records the end event now (else at destruction)
  int stage;
  hipStream_t s;
  double bytes;
  hipEvent_t a = nullptr;
  hipEvent_t b = nullptr;
};

// --------------------------------------------------------------- launchers
// k_basic.hip
void launch_rows_to_soa(const uint64_t* rows, int W, int64_t m, uint64_t* soa, int64_t ld,
                        hipStream_t s);
void launch_soa_to_rows(const uint64_t* soa, int W, int64_t m, int64_t ld, uint64_t* rows,
                        hipStream_t s);
void launch_validate(const uint64_t* xr, const uint64_t* zr, const uint8_t* ph, int n, int64_t m,
                     uint32_t* err, hipStream_t s);
void launch_fingerprint(const paulisum* t, hipStream_t s);
void launch_zero_bytes(void* p, int64_t n, hipStream_t s);
void launch_outer_product(const paulisum* a, const paulisum* b, paulisum* out, hipStream_t s);

// Per-term data of one operand of a pair product, gathered row-major so that
// a term's 2W words sit in one contiguous span (one 128-byte line at W = 8).
struct Side {
  const uint64_t* rows = nullptr;  // [m][2W]: X words then Z words
  const uint8_t* e = nullptr;      // [m] (phase + |X & Z|) mod 4
  const void* coef = nullptr;      // [m] the sum's coefficients
  const uint64_t* fp = nullptr;    // [m]
  int64_t m = 0;
};
void launch_prep_side(const paulisum* t, uint64_t* rows, uint8_t* e, hipStream_t s);

// k_sort.hip
size_t scan_workspace_bytes(int64_t n);
// out[i] = sum_{j<i} in[i]; *total (device) = sum of all; in may alias out.
// Device counts: with nd, the element count is *nd (device memory, read by
// the kernels) and n is only the host's upper bound of it (grid sizes and
// workspaces); likewise below.
void scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total,
                        void* work, hipStream_t s, const uint32_t* nd = nullptr);
size_t radix_workspace_bytes(int64_t n);
// Stable LSD radix sort of (key, val) by key bits [0, key_bits).  The sorted
// result ends up in (keys, vals) or (keys_alt, vals_alt): returns true if in
// the alternate pair.  An 8-bit digit with no bit set in vary is taken to be
// the same for every key and is not sorted on.
bool radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
                      int64_t n, int key_bits, void* work, hipStream_t s,
                      uint64_t vary = ~0ull, const uint32_t* nd = nullptr);
// Stable passes on the 8-bit digits at the given shifts, in order (a key's
// digit is (key >> shift) & 255).  Same result convention.
bool radix_sort_at(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
                   int64_t n, const int* shifts, int nshifts, void* work, hipStream_t s,
                   const uint32_t* nd = nullptr);

// k_fused.hip: (key, val) records of a key_bits-bit key put in key order by
// a partition on the top key bits and an LDS sort per bucket, for uniformly
// spread keys (fingerprints).  Equal keys end up ordered by val in buckets
// the LDS counting sort takes, in input order elsewhere (both deterministic;
// the same order when the vals ascend in input order).  Small inputs take
// radix_sort_pairs.  Same result convention as radix_sort_pairs.
bool sort_records_bucketed(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt,
                           uint32_t* vals_alt, int64_t n, int key_bits, hipStream_t s,
                           const uint32_t* nd = nullptr);

// k_merge.hip
// Internal merge mode: the precision form on float-float record values (a
// propagation state carried between steps); the public modes are 0 and 1.
constexpr int kModeFF = 2;
struct MergeArgs {
  int mode = PAULI_MERGE_PLAIN;
  int ff_out = 1;  // kModeFF: 1 writes a float-float sum, 0 a C64 sum
  double drop_abs = -1.0;
  double tau = 1e-3;
  int key_bits = 64;
  int bucket_bits = 0;  // fused pipeline: 0 = the size heuristic
  int comm = 0;         // the commutator [a, b] instead of the product
};
// Device-count form of a merge (a step of a captured propagation loop):
// the record count is *N on the device (the host passes its upper bound;
// null: the host count), the merged terms go to `into` (capacity into->ld)
// and their number to *U (device); a result larger than the capacity is
// cut and sets *flag.  No host synchronisation.
struct DevRun {
  const uint32_t* N = nullptr;
  paulisum* into = nullptr;
  uint32_t* U = nullptr;
  uint32_t* flag = nullptr;
};

// merge(a*b) (pair source) or merge(s) (term source, b == nullptr; with dv,
// written to a state as DevRun says).
paulisum* merge_generic(const paulisum* a, const paulisum* b, const MergeArgs& o, hipStream_t s,
                        const DevRun* dv = nullptr);

// merge(a) from records (key = fingerprint >> (64 - o.key_bits), index of a
// term of a), one per term, already in key order (equal keys adjacent).
// keys and vals are device arrays of a->m entries, used as scratch.
paulisum* merge_sorted_records(const paulisum* a, uint64_t* keys, uint32_t* vals,
                               const MergeArgs& o, hipStream_t s);

// The terms of s whose modulus is not below drop_abs (strict drop; none
// dropped when drop_abs < 0), in their order, as a new container.  With
// marked, terms whose phase byte is nonzero are removed too (the expand
// kernel marks the strings of a commutator that no anticommuting pair gave).
paulisum* drop_terms(const paulisum* s, double drop_abs, hipStream_t st, bool marked = false);
// The same drop over several sums held in one block, the ranges
// [r0[k], r0[k] + rm[k]) of in, in one keep count, one scan and one
// compaction: returns a block of exactly the kept terms, range k's at
// [first[k], first[k] + kept[k]), in range order.  Waits for the stream.
std::shared_ptr<SharedBlock> drop_ranges(const SharedBlock& in, const std::vector<int64_t>& r0,
                                         const std::vector<int64_t>& rm, double drop_abs,
                                         std::vector<int64_t>& first, std::vector<int64_t>& kept,
                                         hipStream_t s);

// k_merge.hip: the commutator [a, b] = sum over anticommuting pairs of
// 2 a_i b_j, the pairs found by a tiled parity test before any sorting and
// only they merged.  Returns nullptr (nothing allocated) when more than
// max_frac of the pairs anticommute.  Requires |a| |b| < 2^32.
paulisum* commutator_filtered(const paulisum* a, const paulisum* b, const MergeArgs& o,
                              double max_frac, hipStream_t s);

// k_basic.hip: the unmerged products 2 a_i b_j of the anticommuting pairs
// of a and b (the terms of [a, b] before merging), in pair order.
paulisum* commutator_products(const paulisum* a, const paulisum* b, hipStream_t s);

// k_clifford.hip: the sum with every term conjugated by the gates in order
// (validated by the caller).
paulisum* apply_clifford(const paulisum* s, const pauli_gate_t* gates, int32_t n_gates,
                         hipStream_t st);

// k_lex.hip: the terms of s in lexicographic order of their packed words
// (X[W-1], ..., X[0], Z[W-1], ..., Z[0]); equal strings keep their order.
paulisum* sort_lex(const paulisum* s, hipStream_t st);

// A rotation string P of a propagation step, passed to kernels by value.
struct RotString {
  uint64_t x[kMaxWordsHost];
  uint64_t z[kMaxWordsHost];
  uint64_t fp;
  int W;
  int y;  // |X & Z| of P
};

// Sort-and-combine of the conjugated sum of s under R = cos(theta) I
// - i sin(theta) P without storing it: record 2t is term t of s (times
// cos(theta) where it anticommutes with P, cnt[t] == 2), record 2t + 1 the
// new term -i sin(theta) P Q_t.  keys / vals: the N records in key order
// (equal keys adjacent), used as scratch.
paulisum* merge_rotated(const paulisum* s, const RotString& P, double theta,
                        const uint32_t* cnt, uint64_t* keys, uint32_t* vals, int64_t N,
                        const MergeArgs& o, hipStream_t st, const DevRun* dv = nullptr);

// k_rotate.hip: one rotation step (product or conjugation semantics),
// followed by the merge o.  px, pz: host words of the rotation string.
paulisum* rotate_step(const paulisum* s, const uint64_t* px, const uint64_t* pz, double theta,
                      int mode, const MergeArgs& o, bool sorted_input, hipStream_t st);

// k_batched.hip: the batched form.  A plan holds the buffers, tables and
// (with use_graph) the captured HIP graph of the launch sequence that forms
// merge(a[t] * b[t]) for every t; shape fixes the launch shape, else each
// class's shape is autotuned (or taken from the tune table).  run enqueues the sequence on st; results waits for it and
// returns each product's sum (views into the plan's output blocks, which
// the plan then no longer uses).
struct BatchPlan;
struct BatchShape {  // fixed launch shape (0 = the default of a field)
  int bucket_bits = 0, bucket_records = 0, class_bits = 0, expand_parts = 0;
};
BatchPlan* batch_plan_create(int nb, paulisum* const* a, paulisum* const* b, const MergeArgs& o,
                             const BatchShape* shape, bool use_graph, hipStream_t st);
void batch_plan_run(BatchPlan* plan, hipStream_t st);
void batch_plan_results(BatchPlan* plan, paulisum** out, hipStream_t st);
void batch_plan_destroy(BatchPlan* plan);
int batch_tune_save(const char* path);
int batch_tune_load(const char* path);

// k_rotate.hip: propagation plans (pauli_propagate_plan_*): the loop of
// pauli_propagate in device-count form, captured into one HIP graph.
struct PropPlan;
PropPlan* prop_plan_create(const paulisum* s, int steps, const uint64_t* px, const uint64_t* pz,
                           const double* theta, int mode, const MergeArgs& o, int64_t cap,
                           hipStream_t st);
void prop_plan_run(PropPlan* pl, hipStream_t st);
paulisum* prop_plan_result(PropPlan* pl);
void prop_plan_destroy(PropPlan* pl);

// k_fused.hip: merge(a*b) by the staged fused pipeline; nullptr when a
// fingerprint collision asks for merge_generic instead.
paulisum* fused_bucket(const paulisum* a, const paulisum* b, const MergeArgs& o, hipStream_t s);
// The bucket width the size heuristic picks for p products.
int fused_default_bucket_bits(int64_t p, int key_bits);

}  // namespace pauli
