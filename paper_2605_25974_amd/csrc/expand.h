// Expand stage of the fused product-merge (the write stage): kernels that
// turn the sorted records of each bucket into merged terms.  Included by
// k_fused.hip only; kept apart so that the expand kernels' sources can be
// identified on their own.
#pragma once

#include <type_traits>

#include "common.h"
#include "internal.h"

namespace pauli {

namespace {

constexpr int kB = 256;
constexpr int kLong = 32;      // segments longer than this are reduced by a block
constexpr int kLongB = 1024;  // threads of that block (many records in flight)
constexpr int kBS = 32;    // terms per aligned store block of the expand kernel
constexpr int kParts = 4;  // work items per bucket of the expand kernel

enum : uint32_t { kErrCollision = 1u };

// What a record stands for.
//   kFormProduct: the product a_i b_j;
//   kFormSym:     a sum times itself, one record per unordered pair;
//   kFormComm:    the commutator [a, b] = ab - ba: a_i b_j - b_j a_i is
//                 2 a_i b_j for an anticommuting pair and nothing otherwise.
enum : int { kFormProduct = 0, kFormSym = 1, kFormComm = 2 };

// Per-term data of an operand as four 64-bit words: the coefficient's real
// and imaginary parts (one per word, in the sum's precision), the
// fingerprint, and a word holding e = (phase + |X & Z|) mod 4 in bits 0-1,
// the parity of |X & Z| in bit 2 and the term's class in bits 8 and up.
template <typename T>
struct alignas(32) Aux {
  uint64_t w[4];
};
template <typename T>
__host__ __device__ __forceinline__ uint64_t to_word(T v) {
  uint64_t u = 0;
  __builtin_memcpy(&u, &v, sizeof(T));
  return u;
}
template <typename T>
__device__ __forceinline__ T from_word(uint64_t u) {
  T v;
  __builtin_memcpy(&v, &u, sizeof(T));
  return v;
}

// Words per operand slot.  For G <= 4 the row (2G words) and the term's
// metadata (its Aux, 4 words) share one aligned slot of 64 or 128 bytes, so
// that a record's gathers from one operand touch one cache line (W <= 4 is
// 11-15% faster in the expand); wider rows fill a line on their own.
__host__ __device__ constexpr int slot_words(int G) {
  return G <= 2 ? 8 : (G <= 4 ? 16 : 2 * G);
}

template <int WT, typename T>
struct Operands {
  // [|a|][slot_words(G)]: word pairs (X_w, Z_w) padded to G pairs, then for
  // G <= 4 the term's Aux words (xa/xb are then not read)
  const uint64_t* ra;
  const uint64_t* rb;
  const Aux<T>* xa;
  const Aux<T>* xb;
  uint32_t ma;
  int ibits;  // pair id = (j << ibits) | i when ibits >= 0, else j*ma + i
  int nw;     // W
  int form;   // kFormProduct, kFormSym or kFormComm
};

__device__ __forceinline__ void split_id(uint32_t id, uint32_t ma, int ibits, uint32_t& i,
                                         uint32_t& j) {
  if (ibits >= 0) {
    j = id >> ibits;
    i = id & ((1u << ibits) - 1u);
  } else {
    j = id / ma;
    i = id - j * ma;
  }
}

// Records per lane group per chunk of the expand kernel: 2 for groups of one
// or two lanes (so that a wave's stage stays small), else 4.
template <int G>
struct Run {
  static constexpr int v = G <= 2 ? 2 : 4;
};

// DPP moves (cross-lane operands inside rows of 16 lanes, no LDS traffic).
template <int CTRL>
__device__ __forceinline__ uint32_t dpp32(uint32_t v) {
  return static_cast<uint32_t>(
      __builtin_amdgcn_update_dpp(0, static_cast<int>(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ uint64_t dpp64(uint64_t v) {
  const uint32_t lo = dpp32<CTRL>(static_cast<uint32_t>(v));
  const uint32_t hi = dpp32<CTRL>(static_cast<uint32_t>(v >> 32));
  return (static_cast<uint64_t>(hi) << 32) | lo;
}
constexpr int kDppSwap1 = 0xB1;       // quad_perm [1,0,3,2]
constexpr int kDppSwap2 = 0x4E;       // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;  // lane l <- lane 7 - l of each 8
constexpr int kDppRowMirror = 0x140;   // lane l <- lane 15 - l of each 16

// Sum of v over the G lanes of a group (groups of G <= 16 aligned lanes).
template <int G>
__device__ __forceinline__ int group_sum(int v) {
  if constexpr (G >= 2) v += static_cast<int>(dpp32<kDppSwap1>(static_cast<uint32_t>(v)));
  if constexpr (G >= 4) v += static_cast<int>(dpp32<kDppSwap2>(static_cast<uint32_t>(v)));
  if constexpr (G >= 8) v += static_cast<int>(dpp32<kDppHalfMirror>(static_cast<uint32_t>(v)));
  if constexpr (G >= 16) v += static_cast<int>(dpp32<kDppRowMirror>(static_cast<uint32_t>(v)));
  return v;
}

// G lanes hold one record: lane l holds word l of the product string's X and
// Z parts (rows are laid out as word pairs (X_w, Z_w)).  TV is the arithmetic
// type of the value.
template <int G, typename TV>
struct Rec {
  uint64_t w0, w1;  // X and Z word gl of the product string
  TV re, im;        // value i^k c_a c_b (the same in every lane of the group)
  uint64_t fp;
  bool keep;        // the record gives its string a term (false: a commuting pair of [a, b])
};

// Raw loads of one record: this lane's pieces (X_gl, Z_gl) of the two operand
// rows, and 16-byte pieces of the two metadata records (from the operands'
// slots when G <= 4, else from xa/xb).  Metadata piece k
// holds words 2(k & 1), 2(k & 1) + 1 of a's record (k < 2) or of b's
// (k >= 2).  In groups of four or more lanes every lane loads piece gl & 3;
// a pair loads pieces gl and gl + 2; a single lane loads all four.
template <int G>
struct Raw {
  static constexpr int NP = G >= 4 ? 1 : 4 / G;
  ulonglong2 a, b;
  ulonglong2 piece[NP];
  int ij;  // sign of i - j
};

template <int G, int WT, typename T>
__device__ __forceinline__ Raw<G> issue_rec(const Operands<WT, T>& op, uint32_t id, int gl) {
  uint32_t i, j;
  split_id(id, op.ma, op.ibits, i, j);
  Raw<G> r;
  r.ij = i < j ? -1 : (i > j ? 1 : 0);
  constexpr int SW = slot_words(G);
  const uint64_t* sa = op.ra + static_cast<size_t>(i) * SW;
  const uint64_t* sb = op.rb + static_cast<size_t>(j) * SW;
  r.a = reinterpret_cast<const ulonglong2*>(sa)[gl];
  r.b = reinterpret_cast<const ulonglong2*>(sb)[gl];
#pragma unroll
  for (int p = 0; p < Raw<G>::NP; ++p) {
    const int k = G >= 4 ? (gl & 3) : gl + p * G;
    const ulonglong2* src =
        G <= 4 ? reinterpret_cast<const ulonglong2*>((k < 2 ? sa : sb) + 2 * G)
               : reinterpret_cast<const ulonglong2*>(k < 2 ? op.xa[i].w : op.xb[j].w);
    r.piece[p] = src[k & 1];
  }
  return r;
}

// Word H of metadata piece K in every lane of the group (its low BITS bits).
template <int G, int K, int H, int BITS>
__device__ __forceinline__ uint64_t meta_word(const Raw<G>& raw) {
  if constexpr (G == 1) {
    return H ? raw.piece[K].y : raw.piece[K].x;
  } else {
    const ulonglong2 p = raw.piece[G == 2 ? (K >> 1) : 0];
    const uint64_t v = H ? p.y : p.x;
    // from lane K & 1 of each pair, or lane K of each quad
    constexpr int C = G == 2 ? ((K & 1) ? 0xF5 : 0xA0) : K * 0x55;
    if constexpr (BITS == 32) return dpp32<C>(static_cast<uint32_t>(v));
    else return dpp64<C>(v);
  }
}

// TS: type the operands' coefficients are stored in; TV: type the product
// is computed in (the stored coefficients are rounded to TV first).
template <int G, typename TS, typename TV>
__device__ __forceinline__ Rec<G, TV> finish_rec(const Raw<G>& raw, int gl, int form) {
  (void)gl;
  const ulonglong2 a = raw.a, b = raw.b;
  Rec<G, TV> r;
  r.w0 = a.x ^ b.x;
  r.w1 = a.y ^ b.y;
  // 2 |Z_a & X_b| - |X_3 & Z_3| over the words of the strings
  const int part = group_sum<G>(2 * popc64(a.y & b.x) - popc64(r.w0 & r.w1));
  constexpr int CB = static_cast<int>(sizeof(TS)) * 8;
  const uint64_t ar = meta_word<G, 0, 0, CB>(raw), ai = meta_word<G, 0, 1, CB>(raw);
  const uint64_t af = meta_word<G, 1, 0, 64>(raw), ae = meta_word<G, 1, 1, 32>(raw);
  const uint64_t br = meta_word<G, 2, 0, CB>(raw), bi = meta_word<G, 2, 1, CB>(raw);
  const uint64_t bf = meta_word<G, 3, 0, 64>(raw), be = meta_word<G, 3, 1, 32>(raw);
  const int k = static_cast<int>(ae + be) + part;  // bits 2 and up of e words add multiples of 4
  const cplx<TV> v =
      rot_ik(k, cmul(cplx<TV>{static_cast<TV>(from_word<TS>(ar)), static_cast<TV>(from_word<TS>(ai))},
                     cplx<TV>{static_cast<TV>(from_word<TS>(br)), static_cast<TV>(from_word<TS>(bi))}));
  r.re = v.re;
  r.im = v.im;
  r.keep = true;
  if (form != kFormProduct) {
    // The values of a_i b_j and b_j a_i are equal when the strings commute
    // and opposite when they anticommute (the phases differ by 2 exactly
    // then).  The parity of the anticommutation count is that of
    // |X3 & Z3| + |Xa & Za| + |Xb & Zb|, and part = 2(..) - |X3 & Z3|.
    const bool anti = ((part + static_cast<int>((ae >> 2) + (be >> 2))) & 1) != 0;
    TV f;
    if (form == kFormComm) {
      f = anti ? TV(2) : TV(0);
      r.keep = anti;
    } else {
      // the pair stands for (i, j) and (j, i)
      const bool same_class = (ae >> 8) == (be >> 8);
      f = anti ? TV(0) : TV(2);
      if (raw.ij == 0) f = TV(1);                        // i == j
      else if (same_class && raw.ij > 0) f = TV(0);      // (j, i) of a diagonal tile: counted at (i, j)
    }
    r.re = f * r.re;
    r.im = f * r.im;
  }
  r.fp = af ^ bf;
  return r;
}

template <int G, int WT, typename TS, typename TV>
__device__ __forceinline__ Rec<G, TV> load_rec(const Operands<WT, TS>& op, uint32_t id, int gl) {
  return finish_rec<G, TS, TV>(issue_rec<G, WT, TS>(op, id, gl), gl, op.form);
}

struct ExpandArgs {
  const uint32_t* boff;
  const uint32_t* vals;
  const uint32_t* segidx;
  const uint32_t* segoff;  // [bucket] first output index
  uint32_t nbk;
  uint32_t* err;
  uint32_t* work;  // work-item counter of k_expand, zero at launch
  uint64_t* OX;
  uint64_t* OZ;
  uint8_t* Oph;
  void* Oc;
  uint64_t* Ofp;
  int64_t ldo;  // a multiple of kBS
  double tau;   // cancellation threshold of the compensated form
  int marks;    // phase byte 1 marks a term no record kept (commutator), for a later compaction
  // A batched launch sequence (null: one product, the kernel's operands):
  // the product of each bucket, and per product its operands, its first
  // bucket, its first output term (a multiple of kBS; its terms are written
  // from there) and its collision flag.
  const uint16_t* bprod = nullptr;
  const void* optab = nullptr;  // Operands<WT, T>[product]
  const uint32_t* pbase = nullptr;
  const uint32_t* pout = nullptr;
  uint32_t* perr = nullptr;
  uint32_t parts = kParts;  // work items per bucket
};

// The operands and first output term of bucket b.
template <bool BATCH, int WT, typename T>
__device__ __forceinline__ void bucket_product(const ExpandArgs& E, const Operands<WT, T>& op0,
                                               uint32_t b, Operands<WT, T>& op, uint32_t& obase,
                                               uint32_t& prod) {
  if constexpr (BATCH) {
    prod = E.bprod[b];
    op = static_cast<const Operands<WT, T>*>(E.optab)[prod];
    obase = E.pout[prod] + (E.segoff[b] - E.segoff[E.pbase[prod]]);
  } else {
    prod = 0;
    op = op0;
    obase = E.segoff[b];
  }
}

// Merged terms of a wave, staged for aligned coalesced stores: a ring of CAP
// slots, output term o in slot o mod CAP.  The x and z rows are one word
// longer than CAP so that the words a lane group writes for one slot fall in
// different banks.
template <int WT, typename T, int CAP>
struct Stage {
  uint64_t x[WT][CAP + 1];
  uint64_t z[WT][CAP + 1];
  cplx<T> c[CAP];
  uint64_t fp[CAP];
  uint8_t valid[CAP];
};

// valid: 1 = a staged term, 2 = a staged term that no record kept.
template <int G, int WT, typename T, int CAP, typename TV>
__device__ __forceinline__ void stage_out(Stage<WT, T, CAP>& st, int nw, int gl, uint32_t slot,
                                          const Rec<G, TV>& r, T re, T im, bool kept) {
  if (gl < nw) {
    st.x[gl][slot] = r.w0;
    st.z[gl][slot] = r.w1;
  }
  if (gl == 0) {
    st.c[slot] = cplx<T>{re, im};
    st.fp[slot] = r.fp;
    st.valid[slot] = kept ? 1 : 2;
  }
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// FP64 sum of the records at bucket positions q0 .. q1-1, in order, from the
// operands' own coefficients (the re-merge of a cancelled segment).  The
// operands come by value: passed by reference, they had to live in scratch
// memory for the whole kernel (the precision form's write stage at n = 500
// took 6.68 instead of 5.72 ms).
template <int G, int WT, typename T>
__device__ __noinline__ cplx<double> remerge64(const uint32_t* __restrict__ vals,
                                               Operands<WT, T> op, uint32_t lo, uint32_t q0,
                                               uint32_t q1, int gl) {
  double re = 0.0, im = 0.0;
  for (uint32_t q = q0; q < q1; ++q) {
    const Rec<G, double> r = load_rec<G, WT, T, double>(op, vals[lo + q], gl);
    re = re + r.re;
    im = im + r.im;
  }
  return {re, im};
}

// Segment indices and ids of the KR records of a lane group's run, as
// loaded by the lane (distributed over the group's lanes when G allows).
template <int G>
struct Meta {
  static constexpr int KR = Run<G>::v;
  static constexpr bool kSplit = G >= KR + 2;
  uint32_t ms[kSplit ? 1 : KR + 2];
  uint32_t mi[kSplit ? 1 : KR];
};

// Every lane issues the same loads whatever the chunk's position (indices
// past the bucket are clamped to its last record).  The loaded words are kept
// as loaded; the past-the-end substitutions happen in unpack_meta, one chunk
// later, so the loads are not waited for when they are issued.  n >= 1.
template <int G>
__device__ __forceinline__ Meta<G> fetch_meta(const ExpandArgs& E, uint32_t lo, uint32_t n,
                                              uint32_t p0, int gl) {
  constexpr int KR = Run<G>::v;
  Meta<G> m;
  const uint32_t last = n - 1;
  auto at = [&](uint32_t q) { return lo + (q < n ? q : last); };
  if (Meta<G>::kSplit) {
    // lane gl: record p0 + gl (gl <= KR), or the record before the run
    const uint32_t q = gl <= KR ? p0 + gl : (p0 ? p0 - 1 : 0u);
    m.ms[0] = E.segidx[at(q)];
    m.mi[0] = E.vals[at(q)];
  } else {
#pragma unroll
    for (int t = 0; t <= KR; ++t) m.ms[t] = E.segidx[at(p0 + t)];
    m.ms[KR + 1] = E.segidx[at(p0 ? p0 - 1 : 0u)];
#pragma unroll
    for (int t = 0; t < KR; ++t) m.mi[t] = E.vals[at(p0 + t)];
  }
  return m;
}

// Segment indices sid[0..KR] of the run's records (0xFFFFFFFE past the
// bucket), their ids (0 past the bucket: a valid pair) and the segment index
// of the record before the run (0xFFFFFFFF at the bucket's start).
template <int G>
__device__ __forceinline__ void unpack_meta(const Meta<G>& m, int gl, uint32_t n, uint32_t p0,
                                            uint32_t* sid, uint32_t* ids, uint32_t& sprev) {
  constexpr int KR = Run<G>::v;
  if (Meta<G>::kSplit) {
    const int base = (threadIdx.x & 63) - gl;
#pragma unroll
    for (int t = 0; t <= KR; ++t) sid[t] = __shfl(m.ms[0], base + t, 64);
#pragma unroll
    for (int t = 0; t < KR; ++t) ids[t] = __shfl(m.mi[0], base + t, 64);
    sprev = __shfl(m.ms[0], base + KR + 1, 64);
  } else {
#pragma unroll
    for (int t = 0; t <= KR; ++t) sid[t] = m.ms[t];
#pragma unroll
    for (int t = 0; t < KR; ++t) ids[t] = m.mi[t];
    sprev = m.ms[KR + 1];
  }
#pragma unroll
  for (int t = 0; t <= KR; ++t)
    if (p0 + t >= n) sid[t] = 0xFFFFFFFEu;
#pragma unroll
  for (int t = 0; t < KR; ++t)
    if (p0 + t >= n) ids[t] = 0u;
  if (!(p0 && p0 < n)) sprev = 0xFFFFFFFFu;
}

// Stores the staged terms o in [o_lo, o_hi) of the aligned block
// [B, B + kBS) (every 8-byte array gets whole 128-byte lines when the block
// is complete): lanes 0-31 write the X words and lanes 32-63 the Z words of
// one word index per instruction; 16-byte coefficients are written as two
// halves, lanes 0-31 the real and lanes 32-63 the imaginary parts.  Clears
// the block's slots afterwards.
template <int WT, typename TV, int CAP>
__device__ __forceinline__ void store_block(const ExpandArgs& E, Stage<WT, TV, CAP>& st, int nw,
                                            uint32_t B, uint32_t o_lo, uint32_t o_hi, int lane) {
  const uint32_t t = static_cast<uint32_t>(lane & (kBS - 1));
  const bool upper = lane >= kBS;
  const uint32_t o = B + t;
  const uint32_t slot = o & (CAP - 1);
  const uint8_t vflag = st.valid[slot];
  // a term no record kept (commutator) is removed later: only its mark is stored
  const bool live = o >= o_lo && o < o_hi && vflag == 1;
  const bool mark = o >= o_lo && o < o_hi && vflag == 2;
#pragma unroll
  for (int w = 0; w < WT; ++w) {
    if (w < nw) {
      const uint64_t v = upper ? st.z[w][slot] : st.x[w][slot];
      uint64_t* dst = (upper ? E.OZ : E.OX) + static_cast<int64_t>(w) * E.ldo + o;
      if (live) __builtin_nontemporal_store(v, dst);
    }
  }
  const cplx<TV> c = st.c[slot];
  const uint64_t f = st.fp[slot];
  if constexpr (sizeof(TV) == 8) {
    uint64_t* dst = reinterpret_cast<uint64_t*>(static_cast<cplx<TV>*>(E.Oc) + o) + (upper ? 1 : 0);
    if (live) __builtin_nontemporal_store(to_word<TV>(upper ? c.im : c.re), dst);
    if (live && !upper) __builtin_nontemporal_store(f, E.Ofp + o);
  } else {
    // lanes 0-31 the coefficient (two floats), lanes 32-63 the fingerprint
    const uint64_t cw = (to_word<TV>(c.im) << 32) | (to_word<TV>(c.re) & 0xFFFFFFFFull);
    uint64_t* dst = upper ? E.Ofp + o : reinterpret_cast<uint64_t*>(static_cast<cplx<TV>*>(E.Oc) + o);
    if (live) __builtin_nontemporal_store(upper ? f : cw, dst);
  }
  if (mark && !upper) E.Oph[o] = 1;
  wave_sync();  // the slots are read before they are cleared
  if (!upper) st.valid[slot] = 0;
}

// Work items are quarters of buckets (kParts record ranges of equal length),
// taken from a counter by each wave.  A wave handles the segments whose first
// record lies in its range, chunk by chunk (RS records per chunk; group g of
// the wave takes KR consecutive records of a chunk and follows a segment past
// them when it continues, except segments longer than kLong, which
// k_expand_long sums).  The range's terms form one contiguous output range:
// they are staged in the wave's ring and stored in aligned blocks of kBS
// terms as the blocks fill, so that only the range's first and last blocks
// write partial lines.
//
// The ids two chunks ahead and the row/metadata gathers of the next chunk are
// issued before a chunk is processed.
template <int G, int WT, typename T, int MODE, bool BATCH = false>
__global__ void __launch_bounds__(kB, G >= 16 ? 2 : 3)
k_expand(ExpandArgs E, Operands<WT, T> op0) {
  using TV = typename std::conditional<MODE == kComp, float, T>::type;
  constexpr int KR = Run<G>::v;
  constexpr int NG = 64 / G;  // groups per wave
  constexpr uint32_t RS = NG * KR;
  constexpr int CAP = RS + kBS <= 64 ? 64 : (RS + kBS <= 128 ? 128 : 256);
  static_assert(RS + kBS <= CAP, "ring too small");
  constexpr int NW = kB / 64;
  __shared__ Stage<WT, TV, CAP> stage[NW];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  Stage<WT, TV, CAP>& st = stage[wave];
  const int g = lane / G, gl = lane % G;
  const uint32_t goff = static_cast<uint32_t>(g) * KR;
  const uint32_t parts = E.parts;
  const uint32_t items = E.nbk * parts;
  uint64_t coll = 0;
  for (;;) {
    uint32_t item = 0;
    if (lane == 0) item = atomicAdd(E.work, 1u);
    item = __builtin_amdgcn_readfirstlane(item);
    if (item >= items) break;
    const uint32_t b = item / parts, part = item % parts;
    const uint32_t lo = E.boff[b], n = E.boff[b + 1] - lo;
    const uint32_t q_beg = static_cast<uint32_t>(static_cast<uint64_t>(n) * part / parts);
    const uint32_t q_end = static_cast<uint32_t>(static_cast<uint64_t>(n) * (part + 1) / parts);
    if (q_beg >= q_end) continue;
    Operands<WT, T> op;
    uint32_t obase, prod;
    bucket_product<BATCH, WT, T>(E, op0, b, op, obase, prod);
    const int nw = op.nw;
    for (int k = lane; k < CAP; k += 64) st.valid[k] = 0;
    // pipeline prologue: ids of chunks 0 and 1, gathers of chunk 0
    const Meta<G> m_cur = fetch_meta<G>(E, lo, n, q_beg + goff, gl);
    Meta<G> m_next = fetch_meta<G>(E, lo, n, q_beg + RS + goff, gl);
    uint32_t sid[KR + 1], ids[KR], sprev;
    unpack_meta<G>(m_cur, gl, n, q_beg + goff, sid, ids, sprev);
    // ids past the bucket's end read as 0, a valid pair: the gathers are
    // issued unconditionally so that no stale registers stay live
    Raw<G> raw[KR];
#pragma unroll
    for (int t = 0; t < KR; ++t) raw[t] = issue_rec<G, WT, T>(op, ids[t], gl);
    // output terms [A, Ew) are staged and not yet stored; Bk = A rounded
    // down to a block
    uint32_t A, Bk, Ew;
    {
      const uint32_t s_at0 = __builtin_amdgcn_readfirstlane(__shfl(sid[0], 0, 64));
      const uint32_t s_before = __builtin_amdgcn_readfirstlane(__shfl(sprev, 0, 64));
      A = obase + (s_at0 == s_before ? s_at0 + 1 : s_at0);
      Bk = A & ~static_cast<uint32_t>(kBS - 1);
      Ew = A;
    }
    for (uint32_t R0 = q_beg; R0 < q_end; R0 += RS) {
      const uint32_t p0 = R0 + goff;
      const Meta<G> m_after = fetch_meta<G>(E, lo, n, R0 + 2 * RS + goff, gl);
      {
        // the chunk's last record (inside the range) and its segment
        const uint32_t rl = (R0 + RS < q_end ? R0 + RS : q_end) - 1 - R0;
        uint32_t s_mine = sid[0];
#pragma unroll
        for (int t = 1; t < KR; ++t)
          if (static_cast<int>(rl % KR) == t) s_mine = sid[t];
        const uint32_t s_last = __builtin_amdgcn_readfirstlane(
            __shfl(s_mine, static_cast<int>((rl / KR) * G), 64));
        if (obase + s_last + 1 > Ew) Ew = obase + s_last + 1;
      }
      Rec<G, TV> rec[KR];
#pragma unroll
      for (int t = 0; t < KR; ++t) rec[t] = finish_rec<G, T, TV>(raw[t], gl, op.form);
      wave_sync();  // slots cleared before any stage_out
      if (p0 < q_end) {
        Acc<MODE, TV> acc;
        acc.zero();
        uint64_t h0 = 0, h1 = 0, diff = 0;
        bool open = false, kept = false;
        int t_head = 0;
        Rec<G, TV> first;
        // stages segment [q0, q1) (bucket positions) once its sum is known
        auto emit = [&](uint32_t seg, uint32_t q0, uint32_t q1) {
          TV vr = acc.value_re(), vi = acc.value_im();
          if (MODE == kComp && acc.cancels(E.tau)) {
            const cplx<double> c = remerge64<G, WT, T>(E.vals, op, lo, q0, q1, gl);
            vr = static_cast<TV>(c.re);
            vi = static_cast<TV>(c.im);
          }
          stage_out<G, WT, TV, CAP, TV>(st, nw, gl, (obase + seg) & (CAP - 1), first, vr, vi, kept);
        };
        bool next_part = false;  // a segment head past the range: the rest is not ours
#pragma unroll
        for (int t = 0; t < KR; ++t) {
          if (next_part || p0 + t >= n) break;
          const bool head = sid[t] != (t ? sid[t - 1] : sprev);
          if (head) {
            if (p0 + t >= q_end) {
              next_part = true;
              break;
            }
            open = true;
            kept = rec[t].keep;
            t_head = t;
            acc.begin(rec[t].re, rec[t].im);
            first = rec[t];
            h0 = rec[t].w0;
            h1 = rec[t].w1;
          } else if (open) {
            acc.add(rec[t].re, rec[t].im);
            kept = kept || rec[t].keep;
            diff |= (rec[t].w0 ^ h0) | (rec[t].w1 ^ h1);
          }
          const bool ends = p0 + t + 1 >= n || sid[t + 1] != sid[t];
          if (open && ends) {
            emit(sid[t], p0 + t_head, p0 + t + 1);
            open = false;
          }
        }
        if (open) {
          // the run's last segment continues past the run: follow it,
          // unless it is longer than kLong (then k_expand_long sums it)
          const uint32_t s_cur = sid[KR - 1];
          uint32_t len = static_cast<uint32_t>(KR - t_head);
          uint32_t q = p0 + KR;
          bool is_long = false;
          while (q < n && E.segidx[lo + q] == s_cur) {
            if (++len > static_cast<uint32_t>(kLong)) {
              is_long = true;
              break;
            }
            const Rec<G, TV> r2 = load_rec<G, WT, T, TV>(op, E.vals[lo + q], gl);
            acc.add(r2.re, r2.im);
            kept = kept || r2.keep;
            diff |= (r2.w0 ^ h0) | (r2.w1 ^ h1);
            ++q;
          }
          if (!is_long) emit(s_cur, p0 + t_head, q);
        }
        coll |= diff;  // an equal key must be an equal string
      }
      // gathers of the next chunk
      unpack_meta<G>(m_next, gl, n, R0 + RS + goff, sid, ids, sprev);
#pragma unroll
      for (int t = 0; t < KR; ++t) raw[t] = issue_rec<G, WT, T>(op, ids[t], gl);
      m_next = m_after;
      wave_sync();  // staged terms visible to every lane
      // blocks completed by this chunk
      while (Bk + kBS <= Ew) {
        store_block<WT, TV, CAP>(E, st, nw, Bk, A, Bk + kBS, lane);
        Bk += kBS;
        A = Bk;
      }
    }
    // the range's last, partial block
    if (A < Ew) store_block<WT, TV, CAP>(E, st, nw, Bk, A, Ew, lane);
    if constexpr (BATCH) {  // each product's own flag
      if (__any(coll != 0) && lane == 0) atomicOr(E.perr + prod, kErrCollision);
      coll = 0;
    }
  }
  if (__any(coll != 0) && lane == 0) atomicOr(E.err, kErrCollision);
}

template <int G, typename TO, typename TV>
__device__ __forceinline__ void write_out(const ExpandArgs& E, int nw, int gl, int64_t o,
                                          const Rec<G, TV>& r, TO re, TO im, bool kept) {
  if (E.marks && !kept) {  // removed later: only the mark
    if (gl == 0) E.Oph[o] = 1;
    return;
  }
  if (gl < nw) {
    E.OX[static_cast<int64_t>(gl) * E.ldo + o] = r.w0;
    E.OZ[static_cast<int64_t>(gl) * E.ldo + o] = r.w1;
  }
  if (gl == 0) {
    E.Oph[o] = 0;
    static_cast<cplx<TO>*>(E.Oc)[o] = cplx<TO>{re, im};
    E.Ofp[o] = r.fp;
  }
}

// Segments longer than kLong: one block per segment; group g adds records
// g, g + NG, ... in order, then the NG partial sums are added in a fixed
// pairwise tree.
// In the compensated form a cancelled segment is summed again the same way
// in FP64.
template <int G, int WT, typename T, int MODE, bool BATCH = false>
__global__ void __launch_bounds__(kLongB)
k_expand_long(ExpandArgs E, Operands<WT, T> op0, const uint32_t* __restrict__ long_list,
              const uint32_t* __restrict__ nlong) {
  using TV = typename std::conditional<MODE == kComp, float, T>::type;
  constexpr int NG = kLongB / G;
  __shared__ Acc<MODE, TV> s_acc[NG];
  __shared__ double s_re[NG], s_im[NG];
  __shared__ uint32_t s_end;
  __shared__ int s_kept;
  const int g = threadIdx.x / G, gl = threadIdx.x % G;
  const uint32_t L = *nlong;
  for (uint32_t x = blockIdx.x; x < L; x += gridDim.x) {
    const uint32_t b = long_list[2 * x], q0 = long_list[2 * x + 1];
    const uint32_t lo = E.boff[b], n = E.boff[b + 1] - lo;
    const uint32_t s0 = E.segidx[lo + q0];
    Operands<WT, T> op;
    uint32_t obase, prod;
    bucket_product<BATCH, WT, T>(E, op0, b, op, obase, prod);
    if (threadIdx.x == 0) s_kept = 0;
    if (threadIdx.x == 0) {  // segment indices grow along the bucket: binary search
      uint32_t l = q0, h = n;    // first position past the segment is in (l, h]
      while (h - l > 1) {
        const uint32_t mid = l + (h - l) / 2;
        if (E.segidx[lo + mid] == s0) l = mid; else h = mid;
      }
      s_end = h;
    }
    __syncthreads();
    const uint32_t q1 = s_end;
    const Rec<G, TV> first = load_rec<G, WT, T, TV>(op, E.vals[lo + q0], gl);
    Acc<MODE, TV> acc;
    acc.zero();
    uint64_t diff = 0;
    bool kept = false;
    for (uint32_t q = q0 + g; q < q1; q += NG) {
      const Rec<G, TV> r = load_rec<G, WT, T, TV>(op, E.vals[lo + q], gl);
      acc.add(r.re, r.im);
      kept = kept || r.keep;
      diff |= (r.w0 ^ first.w0) | (r.w1 ^ first.w1);
    }
    if (gl == 0 && kept) atomicOr(&s_kept, 1);
#pragma unroll
    for (int off = 1; off < G; off <<= 1) diff |= __shfl_xor(diff, off, 64);
    if (gl == 0 && diff) atomicOr(BATCH ? E.perr + prod : E.err, kErrCollision);
    if (gl == 0) s_acc[g] = acc;
    __syncthreads();
    // the NG partial sums in a fixed pairwise tree
    for (int h = NG / 2; h > 0; h >>= 1) {
      if (gl == 0 && g < h) s_acc[g].add(s_acc[g + h]);
      __syncthreads();
    }
    // every thread reads the same total, so the branch below is uniform
    const Acc<MODE, TV> tot = s_acc[0];
    TV vr = tot.value_re(), vi = tot.value_im();
    if (MODE == kComp && tot.cancels(E.tau)) {
      double re = 0.0, im = 0.0;
      for (uint32_t q = q0 + g; q < q1; q += NG) {
        const Rec<G, double> r = load_rec<G, WT, T, double>(op, E.vals[lo + q], gl);
        re = re + r.re;
        im = im + r.im;
      }
      if (gl == 0) {
        s_re[g] = re;
        s_im[g] = im;
      }
      __syncthreads();
      for (int h = NG / 2; h > 0; h >>= 1) {
        if (gl == 0 && g < h) {
          s_re[g] = s_re[g] + s_re[g + h];
          s_im[g] = s_im[g] + s_im[g + h];
        }
        __syncthreads();
      }
      vr = static_cast<TV>(s_re[0]);
      vi = static_cast<TV>(s_im[0]);
    }
    if (threadIdx.x < G)
      write_out<G, TV, TV>(E, op.nw, gl, static_cast<int64_t>(obase) + s0, first, vr, vi,
                           s_kept != 0);
    __syncthreads();
  }
}

}  // namespace

}  // namespace pauli
