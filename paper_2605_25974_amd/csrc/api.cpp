// The C ABI (include/paulisum.h): argument checks, device memory, and the
// order in which the kernels of each call run.  No exception leaves this
// file: every entry point catches and turns errors into status codes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

namespace pauli {

namespace {
thread_local std::string g_last_error;

pauli_alloc_fn g_alloc = nullptr;
pauli_free_fn g_free = nullptr;
void* g_alloc_ctx = nullptr;
std::atomic<uint64_t> g_in_use{0};
std::atomic<uint64_t> g_budget{0};

struct Fail {
  pauli_status_t status;
};

}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

[[noreturn]] void fail(pauli_status_t s, const std::string& msg) {
  set_error(msg);
  throw Fail{s};
}

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(e == hipErrorOutOfMemory ? PAULI_ERR_OOM : PAULI_ERR_DEVICE,
         std::string(what) + ": " + hipGetErrorString(e));
  }
}

// ------------------------------------------------- fixed scratch workspace
//
// pauli_merge_into runs the merge pipeline without allocating: its
// temporaries come from `scratch`, one fixed array per device that the
// library holds until the process ends, and its result goes to arrays the
// caller passes.  In host code the array's name is not a device address;
// its address on each device comes from hipGetSymbolAddress, made once per
// device with that device current.
constexpr size_t kScratchBytes = size_t(128) << 20;
constexpr int64_t kScratchMaxTerms = int64_t(1) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The scratch array's address on device dev (current on the calling thread).
void* scratch_address(int dev) {
  if (dev < 0 || dev >= kMaxDevices) fail(PAULI_ERR_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      fail(PAULI_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

struct Workspace {
  char* base = nullptr;
  size_t size = 0, used = 0;
  paulisum out;  // the caller's output arrays; out.ld is their capacity
  bool out_taken = false;
};
thread_local Workspace* g_ws = nullptr;

// Makes ws the calling thread's workspace for the lifetime of the guard.
struct WorkspaceGuard {
  explicit WorkspaceGuard(Workspace* ws) { g_ws = ws; }
  ~WorkspaceGuard() { g_ws = nullptr; }
};
}  // namespace

bool workspace_active() { return g_ws != nullptr; }

ScratchScope::ScratchScope(void* base, size_t bytes) : ws_(new Workspace) {
  if (g_ws) {
    delete static_cast<Workspace*>(ws_);
    fail(PAULI_ERR_DEVICE, "nested scratch regions");
  }
  Workspace* w = static_cast<Workspace*>(ws_);
  w->base = static_cast<char*>(base);
  w->size = bytes;
  w->out_taken = true;  // no result container: every merge writes to a given state
  g_ws = w;
}
ScratchScope::~ScratchScope() {
  g_ws = nullptr;
  delete static_cast<Workspace*>(ws_);
}
void ScratchScope::rewind() { static_cast<Workspace*>(ws_)->used = 0; }
size_t ScratchScope::used() const { return static_cast<Workspace*>(ws_)->used; }

void* dalloc(size_t bytes, hipStream_t s) {
  if (bytes == 0) return nullptr;
  bytes = (bytes + 255) & ~size_t(255);
  if (g_ws) {
    if (bytes > g_ws->size - g_ws->used)
      fail(PAULI_ERR_CAPACITY, "the fixed scratch array (" + std::to_string(g_ws->size) +
                                   " bytes) is too small for this call");
    void* p = g_ws->base + g_ws->used;
    g_ws->used += bytes;
    return p;
  }
  const uint64_t budget = g_budget.load();
  if (budget && g_in_use.load() + bytes > budget)
    fail(PAULI_ERR_OOM, "device memory budget exceeded (" + std::to_string(bytes) +
                            " bytes requested, " + std::to_string(g_in_use.load()) + " in use of " +
                            std::to_string(budget) + ")");
  void* p = nullptr;
  if (g_alloc) {
    p = g_alloc(bytes, s, g_alloc_ctx);
    if (!p) fail(PAULI_ERR_OOM, "allocator hook returned NULL for " + std::to_string(bytes));
  } else {
    int dev = 0;
    PAULI_HIP(hipGetDevice(&dev));
    p = arena_alloc(dev, s, bytes);
  }
  g_in_use += bytes;
  return p;
}

void dfree(void* p, size_t bytes, hipStream_t s) {
  if (!p) return;
  if (g_ws && static_cast<char*>(p) >= g_ws->base &&
      static_cast<char*>(p) < g_ws->base + g_ws->size)
    return;  // the workspace is released as a whole when its call ends
  bytes = (bytes + 255) & ~size_t(255);
  g_in_use -= bytes;
  if (g_alloc) {
    if (g_free) g_free(p, s, g_alloc_ctx);
    return;
  }
  arena_free(p, s);
}

paulisum* new_sum(int n, int64_t m, int64_t ld, int32_t dt, hipStream_t s) {
  const int W = words_for(n);
  if (g_ws) {
    // the result of a call that allocates nothing: the caller's arrays
    paulisum* p = &g_ws->out;
    if (g_ws->out_taken) fail(PAULI_ERR_DEVICE, "a result container inside a fixed scratch region");
    if (n != p->n || dt != p->dtype) fail(PAULI_ERR_DEVICE, "result shape differs from the output");
    if (m > p->ld)
      fail(PAULI_ERR_CAPACITY, "the result has " + std::to_string(m) +
                                   " terms; the output arrays hold " + std::to_string(p->ld));
    g_ws->out_taken = true;
    p->m = m;
    p->last_stream = s;
    return p;
  }
  const size_t L = static_cast<size_t>(ld);
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t bX = up(L * W * 8), bph = up(L), bc = up(L * coef_bytes(dt)), bfp = up(L * 8);
  const size_t total = 2 * bX + bph + bc + bfp;
  paulisum* p = new paulisum;
  p->n = n;
  p->W = W;
  p->m = m;
  p->ld = ld;
  p->dtype = dt;
  PAULI_HIP(hipGetDevice(&p->device));
  p->last_stream = s;
  try {
    p->block = total ? dalloc(total, s) : nullptr;
  } catch (...) {
    delete p;
    throw;
  }
  p->block_bytes = total;
  char* b = static_cast<char*>(p->block);
  p->X = reinterpret_cast<uint64_t*>(b);
  p->Z = reinterpret_cast<uint64_t*>(b + bX);
  p->ph = reinterpret_cast<uint8_t*>(b + 2 * bX);
  p->coef = b + 2 * bX + bph;
  p->fp = reinterpret_cast<uint64_t*>(b + 2 * bX + bph + bc);
  return p;
}

SharedBlock::SharedBlock(int W_, int64_t ld_, int32_t dtype_, hipStream_t s_)
    : W(W_), ld(ld_), dtype(dtype_), s(s_) {
  const size_t L = static_cast<size_t>(ld);
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t bX = up(L * W * 8), bph = up(L), bc = up(L * coef_bytes(dtype)), bfp = up(L * 8);
  bytes = 2 * bX + bph + bc + bfp;
  block = bytes ? dalloc(bytes, s) : nullptr;
  char* b = static_cast<char*>(block);
  X = reinterpret_cast<uint64_t*>(b);
  Z = reinterpret_cast<uint64_t*>(b + bX);
  ph = reinterpret_cast<uint8_t*>(b + 2 * bX);
  coef = b + 2 * bX + bph;
  fp = reinterpret_cast<uint64_t*>(b + 2 * bX + bph + bc);
}

SharedBlock::~SharedBlock() {
  try {
    if (block) dfree(block, bytes, s);
  } catch (...) {
  }
}

paulisum* sum_view(const std::shared_ptr<SharedBlock>& b, int n, int64_t first, int64_t m) {
  paulisum* p = new paulisum;
  p->n = n;
  p->W = words_for(n);
  p->m = m;
  p->ld = b->ld;
  p->dtype = b->dtype;
  PAULI_HIP(hipGetDevice(&p->device));
  p->last_stream = b->s;
  p->X = b->X + first;
  p->Z = b->Z + first;
  p->ph = b->ph + first;
  p->coef = static_cast<char*>(b->coef) + first * coef_bytes(b->dtype);
  p->fp = b->fp + first;
  p->shared = b;
  return p;
}

void free_sum(paulisum* p) {
  if (!p || p->borrowed) return;
  if (p->block) dfree(p->block, p->block_bytes, p->last_stream);
  delete p;
}

}  // namespace pauli

using namespace pauli;

namespace {

template <typename F>
pauli_status_t guarded(F&& f) {
  try {
    set_error("");
    f();
    return PAULI_OK;
  } catch (const Fail& e) {
    return e.status;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return PAULI_ERR_OOM;
  } catch (...) {
    set_error("unexpected internal error");
    return PAULI_ERR_DEVICE;
  }
}

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

void check_sum(paulisum_t s, const char* name) {
  if (!s) fail(PAULI_ERR_INVALID, std::string(name) + " is NULL");
}

void use_device(const paulisum* s) {
  int cur = -1;
  PAULI_HIP(hipGetDevice(&cur));
  if (cur != s->device) PAULI_HIP(hipSetDevice(s->device));
}

// Above this fraction of anticommuting pairs the commutator takes the fused
// product path (the filtered path merges its products through the general
// pipeline, whose cost grows with their number).
constexpr double kCommFilterFrac = 0.125;

// |a| |b| (term counts are below 2^32, so the product fits 64 bits).
uint64_t pair_count(const paulisum* a, const paulisum* b) {
  return static_cast<uint64_t>(a->m) * static_cast<uint64_t>(b->m);
}

// Operands of a binary call; with pair_limit, |a| |b| must fit the 32-bit
// pair index.
void check_pair(paulisum_t a, paulisum_t b, bool pair_limit = true) {
  check_sum(a, "a");
  check_sum(b, "b");
  if (a->n != b->n)
    fail(PAULI_ERR_SHAPE, "qubit counts differ: " + std::to_string(a->n) + " vs " +
                              std::to_string(b->n));
  if (a->dtype != b->dtype) fail(PAULI_ERR_SHAPE, "coefficient types differ");
  if (a->device != b->device) fail(PAULI_ERR_SHAPE, "operands live on different devices");
  if (pair_limit && pair_count(a, b) >= (uint64_t(1) << 32))
    fail(PAULI_ERR_OVERFLOW, "|a|*|b| = " + std::to_string(a->m) + "*" + std::to_string(b->m) +
                                 " exceeds the 32-bit pair index");
}

// Products per range of the chunked outer product (below the 32-bit pair
// index; 24 bytes of records each, double-buffered).
constexpr int64_t kChunkProducts = int64_t(1) << 31;

// The terms [j0, j0 + m) of b as a sum that borrows b's arrays.
paulisum slice_of(const paulisum* b, int64_t j0, int64_t m) {
  paulisum v;
  v.n = b->n;
  v.W = b->W;
  v.m = m;
  v.ld = b->ld;
  v.dtype = b->dtype;
  v.device = b->device;
  v.X = b->X + j0;
  v.Z = b->Z + j0;
  v.ph = b->ph + j0;
  v.coef = static_cast<char*>(b->coef) + j0 * coef_bytes(b->dtype);
  v.fp = b->fp + j0;
  v.last_stream = b->last_stream;
  v.borrowed = true;
  return v;
}

// The terms of several sums one after another in a new sum.
paulisum* concat_sums(const std::vector<paulisum*>& parts, int n, int32_t dt, hipStream_t s) {
  int64_t total = 0;
  for (const paulisum* p : parts) total += p->m;
  if (total >= (int64_t(1) << 32))
    fail(PAULI_ERR_OVERFLOW, "the merged ranges hold " + std::to_string(total) +
                                 " terms, beyond the 32-bit term index of a merge");
  paulisum* c = new_sum(n, total, total, dt, s);
  const size_t cb = coef_bytes(dt);
  int64_t off = 0;
  for (const paulisum* p : parts) {
    const size_t m = static_cast<size_t>(p->m);
    if (m == 0) continue;
    for (int w = 0; w < c->W; ++w) {
      PAULI_HIP(hipMemcpyAsync(c->X + w * c->ld + off, p->X + w * p->ld, m * 8,
                               hipMemcpyDeviceToDevice, s));
      PAULI_HIP(hipMemcpyAsync(c->Z + w * c->ld + off, p->Z + w * p->ld, m * 8,
                               hipMemcpyDeviceToDevice, s));
    }
    PAULI_HIP(hipMemcpyAsync(c->ph + off, p->ph, m, hipMemcpyDeviceToDevice, s));
    PAULI_HIP(hipMemcpyAsync(static_cast<char*>(c->coef) + off * cb, p->coef, m * cb,
                             hipMemcpyDeviceToDevice, s));
    PAULI_HIP(hipMemcpyAsync(c->fp + off, p->fp, m * 8, hipMemcpyDeviceToDevice, s));
    off += p->m;
  }
  return c;
}

// merge(a b) for |a| |b| at or beyond 2^32: the products of the smaller
// operand with ranges of the larger one's terms (at most
// max(kChunkProducts, smaller size) products per range, below the 32-bit
// pair index) are formed and merged by the fused pipeline, then the merged
// ranges are merged once more.  Every product is still summed into its
// string; only the order of the additions differs from a single call.  The
// drop applies to the final merge alone.  Plain mode only: the precision
// form re-merges cancelling sums from the operands' own coefficients, which
// the second merge no longer sees.
paulisum* product_merged_chunked(const paulisum* a, const paulisum* b, const MergeArgs& o,
                                 hipStream_t s) {
  if (o.mode != PAULI_MERGE_PLAIN)
    fail(PAULI_ERR_OVERFLOW, "|a|*|b| = " + std::to_string(a->m) + "*" + std::to_string(b->m) +
                                 " exceeds 2^32: only the plain merge takes more products");
  const bool cut_b = a->m <= b->m;  // ranges of the larger operand
  const paulisum* whole = cut_b ? a : b;
  const paulisum* cut = cut_b ? b : a;
  const int64_t step = std::max<int64_t>(1, kChunkProducts / whole->m);
  MergeArgs part = o;
  part.drop_abs = -1.0;  // a term of one range may combine with another range's
  std::vector<paulisum*> parts;
  paulisum* c = nullptr;
  try {
    for (int64_t k0 = 0; k0 < cut->m; k0 += step) {
      const paulisum v = slice_of(cut, k0, std::min(step, cut->m - k0));
      const paulisum* x = cut_b ? a : &v;
      const paulisum* y = cut_b ? &v : b;
      paulisum* r = fused_bucket(x, y, part, s);
      if (!r) r = merge_generic(x, y, part, s);
      parts.push_back(r);
    }
    c = concat_sums(parts, a->n, a->dtype, s);
    for (paulisum*& p : parts) {
      free_sum(p);
      p = nullptr;
    }
    paulisum* r = merge_generic(c, nullptr, o, s);
    free_sum(c);
    return r;
  } catch (...) {
    for (paulisum* p : parts) free_sum(p);
    free_sum(c);
    throw;
  }
}

MergeArgs merge_args(const pauli_merge_opts_t* o) {
  MergeArgs m;
  if (!o) return m;
  if (o->mode != PAULI_MERGE_PLAIN && o->mode != PAULI_MERGE_COMPENSATED)
    fail(PAULI_ERR_INVALID, "unknown merge mode " + std::to_string(o->mode));
  if (o->key_bits < 0 || o->key_bits > 64)
    fail(PAULI_ERR_INVALID, "key_bits must be in 0..64");
  m.mode = o->mode;
  m.drop_abs = o->drop_abs;
  m.tau = o->remerge_tau > 0 ? o->remerge_tau : 1e-3;
  m.key_bits = o->key_bits ? o->key_bits : 64;
  return m;
}

// Launch shape of a batched call from its tune argument (checked).
BatchShape batch_shape(const pauli_tune_t* t) {
  BatchShape b;
  if (t->bucket_bits < 0 || t->bucket_bits > 16)
    fail(PAULI_ERR_INVALID, "tune: bucket_bits must be in 0..16");
  if (t->bucket_records != 0 && (t->bucket_records < 256 || t->bucket_records > 8192))
    fail(PAULI_ERR_INVALID, "tune: bucket_records must be 0 or in 256..8192");
  if (t->class_bits < 0 || t->class_bits > 8)
    fail(PAULI_ERR_INVALID, "tune: class_bits must be in 0..8");
  if (t->expand_parts != 0 && t->expand_parts != 1 && t->expand_parts != 2 &&
      t->expand_parts != 4 && t->expand_parts != 8)
    fail(PAULI_ERR_INVALID, "tune: expand_parts must be 0, 1, 2, 4 or 8");
  b.bucket_bits = t->bucket_bits;
  b.bucket_records = t->bucket_records;
  b.class_bits = t->class_bits;
  b.expand_parts = t->expand_parts;
  return b;
}

void check_rotations(const paulisum* s, int32_t steps, const uint64_t* p_x, const uint64_t* p_z,
                     const double* theta, int32_t rotate_mode) {
  if (steps < 0) fail(PAULI_ERR_INVALID, "steps is negative");
  if (steps > 0 && (!p_x || !p_z || !theta))
    fail(PAULI_ERR_INVALID, "p_x, p_z and theta must not be NULL");
  if (rotate_mode != PAULI_ROTATE_PRODUCT && rotate_mode != PAULI_ROTATE_CONJUGATE)
    fail(PAULI_ERR_INVALID, "unknown rotate_mode " + std::to_string(rotate_mode));
  const int W = s->W;
  const int tail = s->n - 64 * (W - 1);
  const uint64_t pad = tail == 64 ? 0 : ~((uint64_t(1) << tail) - 1);
  for (int32_t t = 0; t < steps; ++t)
    if ((p_x[static_cast<size_t>(t) * W + W - 1] | p_z[static_cast<size_t>(t) * W + W - 1]) & pad)
      fail(PAULI_ERR_INVALID, "rotation string " + std::to_string(t) + " has a bit at or above n");
}

void check_batch(int32_t nb, const paulisum_t* a, const paulisum_t* b, const pauli_merge_opts_t* o) {
  if (nb < 0) fail(PAULI_ERR_INVALID, "nb is negative");
  if (nb > 0 && (!a || !b)) fail(PAULI_ERR_INVALID, "a and b must not be NULL");
  for (int32_t t = 0; t < nb; ++t) check_pair(a[t], b[t]);
  for (int32_t t = 1; t < nb; ++t)
    if (a[t]->device != a[0]->device) fail(PAULI_ERR_SHAPE, "products live on different devices");
  if (o && o->key_bits != 0 && o->key_bits < 30)
    fail(PAULI_ERR_INVALID, "the batched form needs key_bits 0 or at least 30");
}

}  // namespace

extern "C" {

const char* pauli_status_string(pauli_status_t s) {
  switch (s) {
    case PAULI_OK: return "ok";
    case PAULI_ERR_INVALID: return "invalid argument";
    case PAULI_ERR_SHAPE: return "operand shapes differ";
    case PAULI_ERR_OVERFLOW: return "size overflow";
    case PAULI_ERR_OOM: return "out of device memory";
    case PAULI_ERR_CAPACITY: return "result exceeds capacity";
    case PAULI_ERR_DEVICE: return "device error";
  }
  return "unknown status";
}

const char* pauli_last_error(void) { return g_last_error.c_str(); }

pauli_status_t paulisum_create(int32_t n_qubits, int64_t n_terms, const uint64_t* x_words,
                               const uint64_t* z_words, const uint8_t* phase, const void* coef,
                               pauli_dtype_t dtype, uint32_t flags, void* stream,
                               paulisum_t* out) {
  return guarded([&] {
    if (!out) fail(PAULI_ERR_INVALID, "out is NULL");
    if (n_qubits < 1 || n_qubits > 64 * kMaxWordsHost)
      fail(PAULI_ERR_INVALID, "n_qubits must be in 1..1024, got " + std::to_string(n_qubits));
    if (n_terms < 0) fail(PAULI_ERR_INVALID, "n_terms is negative");
    if (n_terms >= (int64_t(1) << 32)) fail(PAULI_ERR_OVERFLOW, "n_terms must be below 2^32");
    if (dtype != PAULI_C128 && dtype != PAULI_C64) fail(PAULI_ERR_INVALID, "unknown dtype");
    if (flags & ~PAULI_PTR_DEVICE) fail(PAULI_ERR_INVALID, "unknown flags");
    if (n_terms > 0 && (!x_words || !z_words || !coef))
      fail(PAULI_ERR_INVALID, "x_words, z_words and coef must not be NULL");
    const int W = words_for(n_qubits);
    const bool dev = flags & PAULI_PTR_DEVICE;
    const size_t m = static_cast<size_t>(n_terms);
    if (!dev && n_terms > 0) {  // validate host data before touching the device
      const int tail = n_qubits - 64 * (W - 1);
      const uint64_t pad = tail == 64 ? 0 : ~((uint64_t(1) << tail) - 1);
      for (size_t t = 0; t < m; ++t) {
        if ((x_words[t * W + W - 1] | z_words[t * W + W - 1]) & pad)
          fail(PAULI_ERR_INVALID, "term " + std::to_string(t) + " has a bit set at or above n");
        if (phase && phase[t] > 3)
          fail(PAULI_ERR_INVALID, "term " + std::to_string(t) + " has phase > 3");
      }
    }
    hipStream_t s = as_stream(stream);
    paulisum* p = new_sum(n_qubits, n_terms, n_terms, dtype, s);
    try {
      if (n_terms > 0) {
        const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        DBuf rx(m * W * 8, s), rz(m * W * 8, s);
        PAULI_HIP(hipMemcpyAsync(rx.p, x_words, m * W * 8, kind, s));
        PAULI_HIP(hipMemcpyAsync(rz.p, z_words, m * W * 8, kind, s));
        if (phase)
          PAULI_HIP(hipMemcpyAsync(p->ph, phase, m, kind, s));
        else
          launch_zero_bytes(p->ph, static_cast<int64_t>(m), s);
        PAULI_HIP(hipMemcpyAsync(p->coef, coef, m * coef_bytes(dtype), kind, s));
        if (dev) {
          DBuf err(4, s);
          launch_zero_bytes(err.p, 4, s);
          launch_validate(rx.as<uint64_t>(), rz.as<uint64_t>(), p->ph, n_qubits, n_terms,
                          err.as<uint32_t>(), s);
          uint32_t herr = 0;
          PAULI_HIP(hipMemcpyAsync(&herr, err.p, 4, hipMemcpyDeviceToHost, s));
          PAULI_HIP(hipStreamSynchronize(s));
          if (herr & 1u) fail(PAULI_ERR_INVALID, "a term has a bit set at or above n");
          if (herr & 2u) fail(PAULI_ERR_INVALID, "a term has phase > 3");
        }
        launch_rows_to_soa(rx.as<uint64_t>(), W, n_terms, p->X, p->ld, s);
        launch_rows_to_soa(rz.as<uint64_t>(), W, n_terms, p->Z, p->ld, s);
        launch_fingerprint(p, s);
        if (!dev) PAULI_HIP(hipStreamSynchronize(s));  // host arrays copied before return
      }
    } catch (...) {
      free_sum(p);
      throw;
    }
    *out = p;
  });
}

pauli_status_t paulisum_destroy(paulisum_t s) {
  return guarded([&] {
    if (!s) return;
    use_device(s);
    free_sum(s);
  });
}

pauli_status_t paulisum_info(paulisum_t s, int32_t* n_qubits, int64_t* n_terms,
                             pauli_dtype_t* dtype) {
  return guarded([&] {
    check_sum(s, "s");
    if (n_qubits) *n_qubits = s->n;
    if (n_terms) *n_terms = s->m;
    if (dtype) *dtype = static_cast<pauli_dtype_t>(s->dtype);
  });
}

pauli_status_t paulisum_export(paulisum_t s, uint64_t* x_words, uint64_t* z_words,
                               uint8_t* phase, void* coef, uint64_t* fingerprint, uint32_t flags,
                               void* stream) {
  return guarded([&] {
    check_sum(s, "s");
    if (flags & ~PAULI_PTR_DEVICE) fail(PAULI_ERR_INVALID, "unknown flags");
    use_device(s);
    hipStream_t st = as_stream(stream);
    s->last_stream = st;
    const size_t m = static_cast<size_t>(s->m);
    if (m == 0) return;
    const bool dev = flags & PAULI_PTR_DEVICE;
    const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const int W = s->W;
    if (x_words || z_words) {
      DBuf rows(m * W * 8, st);
      if (x_words) {
        launch_soa_to_rows(s->X, W, s->m, s->ld, rows.as<uint64_t>(), st);
        PAULI_HIP(hipMemcpyAsync(x_words, rows.p, m * W * 8, kind, st));
      }
      if (z_words) {
        if (x_words && !dev) PAULI_HIP(hipStreamSynchronize(st));
        launch_soa_to_rows(s->Z, W, s->m, s->ld, rows.as<uint64_t>(), st);
        PAULI_HIP(hipMemcpyAsync(z_words, rows.p, m * W * 8, kind, st));
      }
      if (!dev) PAULI_HIP(hipStreamSynchronize(st));
    }
    if (phase) PAULI_HIP(hipMemcpyAsync(phase, s->ph, m, kind, st));
    if (coef) PAULI_HIP(hipMemcpyAsync(coef, s->coef, m * coef_bytes(s->dtype), kind, st));
    if (fingerprint) PAULI_HIP(hipMemcpyAsync(fingerprint, s->fp, m * 8, kind, st));
    if (!dev) PAULI_HIP(hipStreamSynchronize(st));
  });
}

pauli_status_t pauli_outer_product(paulisum_t a, paulisum_t b, paulisum_t* out, void* stream) {
  return guarded([&] {
    if (!out) fail(PAULI_ERR_INVALID, "out is NULL");
    check_pair(a, b);
    use_device(a);
    hipStream_t s = as_stream(stream);
    const int64_t P = a->m * b->m;
    paulisum* o = new_sum(a->n, P, P, a->dtype, s);
    try {
      launch_outer_product(a, b, o, s);
    } catch (...) {
      free_sum(o);
      throw;
    }
    a->last_stream = b->last_stream = s;
    *out = o;
  });
}

pauli_status_t pauli_merge(paulisum_t sum, const pauli_merge_opts_t* opts, paulisum_t* out,
                           void* stream) {
  return guarded([&] {
    if (!out) fail(PAULI_ERR_INVALID, "out is NULL");
    check_sum(sum, "s");
    const MergeArgs m = merge_args(opts);
    use_device(sum);
    hipStream_t s = as_stream(stream);
    sum->last_stream = s;
    *out = merge_generic(sum, nullptr, m, s);
  });
}

pauli_status_t pauli_merge_into(paulisum_t sum, const pauli_merge_opts_t* opts,
                                uint64_t* out_x, uint64_t* out_z, uint8_t* out_phase,
                                void* out_coef, uint64_t* out_fp, int64_t out_ld, int64_t* out_m,
                                void* stream) {
  return guarded([&] {
    if (!out_m) fail(PAULI_ERR_INVALID, "out_m is NULL");
    check_sum(sum, "s");
    if (!out_x || !out_z || !out_phase || !out_coef || !out_fp)
      fail(PAULI_ERR_INVALID, "an output array is NULL");
    if (out_ld < 1) fail(PAULI_ERR_INVALID, "out_ld must be positive");
    if (sum->m > kScratchMaxTerms)
      fail(PAULI_ERR_CAPACITY, "pauli_merge_into takes at most " +
                                   std::to_string(kScratchMaxTerms) + " terms (got " +
                                   std::to_string(sum->m) + ")");
    const MergeArgs m = merge_args(opts);
    use_device(sum);
    hipStream_t s = as_stream(stream);
    sum->last_stream = s;
    int dev = 0;
    PAULI_HIP(hipGetDevice(&dev));
    Workspace ws;
    ws.base = static_cast<char*>(scratch_address(dev));
    ws.size = kScratchBytes;
    paulisum& o = ws.out;
    o.n = sum->n;
    o.W = sum->W;
    o.ld = out_ld;
    o.dtype = m.mode == PAULI_MERGE_COMPENSATED ? PAULI_C64 : sum->dtype;
    o.device = dev;
    o.X = out_x;
    o.Z = out_z;
    o.ph = out_phase;
    o.coef = out_coef;
    o.fp = out_fp;
    o.borrowed = true;
    WorkspaceGuard guard(&ws);
    paulisum* r = merge_generic(sum, nullptr, m, s);
    if (r != &ws.out) fail(PAULI_ERR_DEVICE, "the merge did not write the output arrays");
    *out_m = r->m;
  });
}

pauli_status_t pauli_outer_product_merged(paulisum_t a, paulisum_t b,
                                          const pauli_merge_opts_t* opts, paulisum_t* out,
                                          void* stream) {
  return guarded([&] {
    if (!out) fail(PAULI_ERR_INVALID, "out is NULL");
    check_pair(a, b, false);
    const MergeArgs m = merge_args(opts);
    use_device(a);
    hipStream_t s = as_stream(stream);
    a->last_stream = b->last_stream = s;
    if (pair_count(a, b) >= (uint64_t(1) << 32)) {
      // beyond the 32-bit pair index: ranges of one operand's terms
      *out = product_merged_chunked(a, b, m, s);
      return;
    }
    paulisum* r = nullptr;
    if (a->m > 0 && b->m > 0) r = fused_bucket(a, b, m, s);
    if (!r) r = merge_generic(a, b, m, s);
    *out = r;
  });
}

pauli_status_t pauli_commutator(paulisum_t a, paulisum_t b, const pauli_merge_opts_t* opts,
                                paulisum_t* out, void* stream) {
  return guarded([&] {
    if (!out) fail(PAULI_ERR_INVALID, "out is NULL");
    check_pair(a, b);
    MergeArgs m = merge_args(opts);
    use_device(a);
    hipStream_t s = as_stream(stream);
    a->last_stream = b->last_stream = s;
    paulisum* r = nullptr;
    if (a->m > 0 && b->m > 0) {
      // few anticommuting pairs (physical Hamiltonians): find them first and
      // merge only their products; many: the fused product with a kept flag
      r = commutator_filtered(a, b, m, kCommFilterFrac, s);
      if (r) {
        *out = r;
        return;
      }
      MergeArgs mc = m;
      mc.comm = 1;
      r = fused_bucket(a, b, mc, s);
      if (!r) {
        // a fingerprint collision: merge the materialised anticommuting products
        paulisum* prods = commutator_products(a, b, s);
        try {
          r = merge_generic(prods, nullptr, m, s);
        } catch (...) {
          free_sum(prods);
          throw;
        }
        free_sum(prods);
      }
    } else {
      r = merge_generic(a, b, m, s);  // empty
    }
    *out = r;
  });
}

pauli_status_t pauli_apply_clifford(paulisum_t s, int32_t n_gates, const pauli_gate_t* gates,
                                    paulisum_t* out, void* stream) {
  return guarded([&] {
    if (!s || !out) fail(PAULI_ERR_INVALID, "s and out must not be NULL");
    if (n_gates < 0) fail(PAULI_ERR_INVALID, "n_gates is negative");
    if (n_gates > 0 && !gates) fail(PAULI_ERR_INVALID, "gates is NULL");
    for (int32_t i = 0; i < n_gates; ++i) {
      const pauli_gate_t& g = gates[i];
      if (g.kind < PAULI_GATE_H || g.kind > PAULI_GATE_SWAP)
        fail(PAULI_ERR_INVALID, "gate " + std::to_string(i) + ": unknown kind");
      if (g.q0 < 0 || g.q0 >= s->n)
        fail(PAULI_ERR_INVALID, "gate " + std::to_string(i) + ": qubit outside [0, n)");
      if (g.kind >= PAULI_GATE_CX && (g.q1 < 0 || g.q1 >= s->n || g.q1 == g.q0))
        fail(PAULI_ERR_INVALID,
             "gate " + std::to_string(i) + ": second qubit outside [0, n) or equal to the first");
    }
    use_device(s);
    hipStream_t st = as_stream(stream);
    s->last_stream = st;
    *out = apply_clifford(s, gates, n_gates, st);
  });
}

pauli_status_t pauli_sort_lex(paulisum_t s, paulisum_t* out, void* stream) {
  return guarded([&] {
    if (!s || !out) fail(PAULI_ERR_INVALID, "s and out must not be NULL");
    use_device(s);
    hipStream_t st = as_stream(stream);
    s->last_stream = st;
    *out = sort_lex(s, st);
  });
}

pauli_status_t pauli_outer_product_batched(int32_t nb, const paulisum_t* a, const paulisum_t* b,
                                           const pauli_merge_opts_t* opts,
                                           const pauli_tune_t* tune, paulisum_t* out,
                                           void* stream) {
  return guarded([&] {
    check_batch(nb, a, b, opts);
    if (nb > 0 && !out) fail(PAULI_ERR_INVALID, "out must not be NULL");
    BatchShape shape;
    if (tune) shape = batch_shape(tune);
    const MergeArgs m = merge_args(opts);
    if (nb == 0) return;
    use_device(a[0]);
    hipStream_t s = as_stream(stream);
    for (int32_t t = 0; t < nb; ++t) a[t]->last_stream = b[t]->last_stream = s;
    std::unique_ptr<BatchPlan, void (*)(BatchPlan*)> plan(
        batch_plan_create(nb, a, b, m, tune ? &shape : nullptr, false, s), batch_plan_destroy);
    batch_plan_run(plan.get(), s);
    batch_plan_results(plan.get(), out, s);
  });
}

pauli_status_t pauli_batch_plan_create(int32_t nb, const paulisum_t* a, const paulisum_t* b,
                                       const pauli_merge_opts_t* opts, const pauli_tune_t* tune,
                                       void* stream, pauli_batch_plan_t* out) {
  return guarded([&] {
    if (!out) fail(PAULI_ERR_INVALID, "out is NULL");
    check_batch(nb, a, b, opts);
    BatchShape shape;
    if (tune) shape = batch_shape(tune);
    const MergeArgs m = merge_args(opts);
    if (nb > 0) use_device(a[0]);
    hipStream_t s = as_stream(stream);
    *out = reinterpret_cast<pauli_batch_plan_t>(
        batch_plan_create(nb, a, b, m, tune ? &shape : nullptr, true, s));
  });
}

pauli_status_t pauli_batch_plan_run(pauli_batch_plan_t plan, void* stream) {
  return guarded([&] {
    if (!plan) fail(PAULI_ERR_INVALID, "plan is NULL");
    batch_plan_run(reinterpret_cast<BatchPlan*>(plan), as_stream(stream));
  });
}

pauli_status_t pauli_batch_plan_results(pauli_batch_plan_t plan, paulisum_t* out, void* stream) {
  return guarded([&] {
    if (!plan) fail(PAULI_ERR_INVALID, "plan is NULL");
    if (!out) fail(PAULI_ERR_INVALID, "out is NULL");
    batch_plan_results(reinterpret_cast<BatchPlan*>(plan), out, as_stream(stream));
  });
}

pauli_status_t pauli_batch_plan_destroy(pauli_batch_plan_t plan) {
  return guarded([&] { batch_plan_destroy(reinterpret_cast<BatchPlan*>(plan)); });
}

pauli_status_t pauli_tune_save(const char* path) {
  return guarded([&] {
    if (!path) fail(PAULI_ERR_INVALID, "path is NULL");
    if (batch_tune_save(path) != 0) fail(PAULI_ERR_INVALID, std::string("cannot write ") + path);
  });
}

pauli_status_t pauli_tune_load(const char* path) {
  return guarded([&] {
    if (!path) fail(PAULI_ERR_INVALID, "path is NULL");
    if (batch_tune_load(path) != 0)
      fail(PAULI_ERR_INVALID, std::string("cannot read a tune table from ") + path);
  });
}

pauli_status_t pauli_propagate(paulisum_t s, int32_t steps, const uint64_t* p_x,
                               const uint64_t* p_z, const double* theta, int32_t rotate_mode,
                               const pauli_merge_opts_t* opts, paulisum_t* out, void* stream) {
  return guarded([&] {
    if (!out) fail(PAULI_ERR_INVALID, "out is NULL");
    check_sum(s, "s");
    check_rotations(s, steps, p_x, p_z, theta, rotate_mode);
    const MergeArgs m = merge_args(opts);
    const int W = s->W;
    use_device(s);
    hipStream_t st = as_stream(stream);
    s->last_stream = st;
    if (steps == 0) {
      *out = merge_generic(s, nullptr, m, st);
      return;
    }
    paulisum* cur = s;
    try {
      const bool ff = m.mode == PAULI_MERGE_COMPENSATED;
      MergeArgs ms = m;
      if (ff) {
        // the precision form carries the state as float-float pairs from
        // step to step; it starts as the merged input, in key order
        MergeArgs m0 = m;
        m0.mode = kModeFF;
        m0.ff_out = 1;
        m0.drop_abs = -1.0;
        cur = merge_generic(s, nullptr, m0, st);
        ms.mode = kModeFF;
      }
      for (int32_t t = 0; t < steps; ++t) {
        // after the first step (from the first, in the precision form) the
        // state is a merge's output, in key order
        ms.ff_out = t + 1 < steps ? 1 : 0;  // the last step writes C64
        paulisum* next = rotate_step(cur, p_x + static_cast<size_t>(t) * W,
                                     p_z + static_cast<size_t>(t) * W, theta[t], rotate_mode, ms,
                                     ff || t > 0, st);
        if (cur != s) free_sum(cur);
        cur = next;
      }
    } catch (...) {
      if (cur != s) free_sum(cur);
      throw;
    }
    *out = cur;
  });
}

pauli_status_t pauli_propagate_plan_create(paulisum_t s, int32_t steps, const uint64_t* p_x,
                                           const uint64_t* p_z, const double* theta,
                                           int32_t rotate_mode, const pauli_merge_opts_t* opts,
                                           int64_t max_terms, void* stream,
                                           pauli_propagate_plan_t* out) {
  return guarded([&] {
    if (!out) fail(PAULI_ERR_INVALID, "out is NULL");
    check_sum(s, "s");
    check_rotations(s, steps, p_x, p_z, theta, rotate_mode);
    if (max_terms < 1 || max_terms > 0x7FFFFFFFll)
      fail(PAULI_ERR_INVALID, "max_terms must be in 1..2^31-1");
    const MergeArgs m = merge_args(opts);
    use_device(s);
    hipStream_t st = as_stream(stream);
    s->last_stream = st;
    *out = reinterpret_cast<pauli_propagate_plan_t>(
        prop_plan_create(s, steps, p_x, p_z, theta, rotate_mode, m, max_terms, st));
  });
}

pauli_status_t pauli_propagate_plan_run(pauli_propagate_plan_t plan, void* stream) {
  return guarded([&] {
    if (!plan) fail(PAULI_ERR_INVALID, "plan is NULL");
    prop_plan_run(reinterpret_cast<PropPlan*>(plan), as_stream(stream));
  });
}

pauli_status_t pauli_propagate_plan_result(pauli_propagate_plan_t plan, paulisum_t* out) {
  return guarded([&] {
    if (!plan) fail(PAULI_ERR_INVALID, "plan is NULL");
    if (!out) fail(PAULI_ERR_INVALID, "out is NULL");
    *out = prop_plan_result(reinterpret_cast<PropPlan*>(plan));
  });
}

pauli_status_t pauli_propagate_plan_destroy(pauli_propagate_plan_t plan) {
  return guarded([&] { prop_plan_destroy(reinterpret_cast<PropPlan*>(plan)); });
}

pauli_status_t pauli_set_allocator(pauli_alloc_fn alloc, pauli_free_fn free_fn, void* ctx) {
  return guarded([&] {
    if ((alloc == nullptr) != (free_fn == nullptr))
      fail(PAULI_ERR_INVALID, "alloc and free must both be set or both be NULL");
    g_alloc = alloc;
    g_free = free_fn;
    g_alloc_ctx = ctx;
  });
}

pauli_status_t pauli_trim_memory(void) {
  return guarded([&] {
    int dev = 0;
    PAULI_HIP(hipGetDevice(&dev));
    arena_trim(dev);
  });
}

pauli_status_t pauli_set_memory_budget(uint64_t bytes) {
  return guarded([&] { g_budget = bytes; });
}

}  // extern "C"
