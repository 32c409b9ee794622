// Fused outer product + sort-and-combine: merge(H1*H2) without storing the
// N*M products (Section IV-C's product, Section III-H's sort and linear
// combine).
//
// Partition.  The sort key of a product is its fingerprint, and
// fp(a_i * b_j) = fp(a_i) ^ fp(b_j).  Its top d bits (the bucket) are
// therefore cls(a_i) ^ cls(b_j), with cls = the top d bits of an operand's
// key.  With one operand ("I") sorted by cls, the pairs of bucket b are, for
// every term o of the other operand ("O"), the I terms of class cls(o) ^ b:
// one contiguous range.  A block enumerates its bucket straight from the
// (cache-resident) operands; no product record is ever written to HBM.
//
// Per bucket, in LDS: the records (key, pair id) are radix-sorted on the 16
// key bits below the bucket bits (two 8-bit passes, wave-ballot ranks), runs
// whose 16 bits tie but whose keys differ are finished by insertion sort on
// the full key, equal keys form the segments, the segment values
// i^k c_a c_b are summed by a segmented scan (deterministic order), and the
// tails write the merged terms.  Output positions come from a decoupled
// look-back over buckets taken in ticket order, so the merged sum lands in
// ascending key order in one pass.  Equal keys are checked to be equal
// strings word by word; a genuine fingerprint collision (or a bucket with too
// many distinct strings) raises a flag and the caller redoes the call with
// the general sort-and-combine pipeline.
//
// A bucket larger than one chunk (kCapF records) is processed chunk by
// chunk: each chunk's segments become "running" entries carrying a partial
// sum, merged with the next chunk's records.
#include <cmath>
#include <memory>

#include "common.h"
#include "internal.h"
#include "sources.h"

namespace pauli {

namespace {

constexpr int kNT = 512;                  // threads per block
constexpr int kWaves = kNT / 64;          // 8
constexpr int kCapF = 2048;               // fresh records per chunk
constexpr int kCapR = 1024;               // running entries carried between chunks
constexpr int kCapE = kCapF + kCapR;      // entries per chunk
constexpr int kPerWave = kCapE / kWaves;  // most positions a wave can own
constexpr int kRounds = kPerWave / 64;    // most rounds of 64 positions per wave
constexpr int kOItems = 8;                // O terms per thread per enumeration tile
constexpr int kOTile = kNT * kOItems;

// Positions [0, N) are split into kWaves contiguous spans of whole rounds;
// wave w owns [w*span, (w+1)*span).
__device__ __forceinline__ uint32_t wave_span(uint32_t N) {
  return ((N + 64 * kWaves - 1) / (64 * kWaves)) * 64;
}
constexpr double kTargetBucket = 1536.0;  // mean records per bucket

enum : uint32_t { kErrCollision = 1u, kErrCapacity = 2u, kErrTimeout = 4u };

struct IRec {
  uint64_t key;
  uint32_t idx;
  uint32_t pad;
};

struct BucketArgs {
  const uint64_t* keyO;  // [mO] key of each O term
  const uint32_t* clsO;  // [mO] its top d key bits
  uint32_t mO;
  const IRec* recI;      // [mI] (key, term index) of the I terms, sorted by class
  const uint2* rangeI;   // [2^d] (first sorted position, count) per class
  const uint32_t* nzI;   // [2^d / 32] bit c set when class c of I is not empty
  int o_is_a;
  uint32_t ma;           // |a|, for the pair index p = j*|a| + i
  int sort_lo;           // lowest key bit of the in-bucket radix field
  int sort_passes;       // 8-bit passes over that field
  uint64_t field_mask;   // width mask of the field
  int drop;
  double drop2;
  uint32_t nbuckets;
  uint32_t* ticket;
  unsigned long long* status;
  uint32_t* err;
  unsigned long long* total;
  uint64_t* OX;
  uint64_t* OZ;
  uint8_t* Oph;
  void* Oc;
  uint64_t* Ofp;
  int64_t ldo;
  void* scratch;  // kCapR running entries per block
};

template <typename T>
struct Smem {
  uint64_t key[kCapE];
  uint32_t id[kCapE];
  uint16_t ord[kCapE];
  cplx<T> rv[kCapR];
  uint32_t cnt[kWaves][256];
  uint32_t scan[kWaves];
  uint32_t wcount[kWaves];
  uint32_t whead[kWaves];
  T wre[kWaves], wim[kWaves];
  T cin_re[kWaves], cin_im[kWaves];
  // deferred tail of each wave: the tail of the segment that was already
  // open when the wave's range began
  uint32_t dvalid[kWaves], did[kWaves], dseg[kWaves];
  uint64_t dkey[kWaves];
  T dre[kWaves], dim[kWaves];
  uint32_t keep[kCapE / 32];
  uint32_t kpre[kCapE / 32];
  uint32_t bcast[4];
  unsigned long long out_base;
};

template <typename T>
struct RunEntry {
  uint64_t key;
  uint32_t id;
  uint32_t pad;
  T re, im;
};

__device__ __forceinline__ uint32_t wave_incl_u32(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}

// Exclusive scan over the block; every thread must call it.
__device__ __forceinline__ uint32_t block_excl(uint32_t v, uint32_t* total, uint32_t* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t inc = wave_incl_u32(v);
  if (lane == 63) sh[wave] = inc;
  __syncthreads();
  uint32_t base = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    const uint32_t x = sh[w];
    if (w < wave) base += x;
    all += x;
  }
  __syncthreads();
  *total = all;
  return base + inc - v;
}

// Appends up to kCapF records of bucket b at entries [base, base + nf).
// (o_tile, skip) is where the previous chunk stopped; all threads keep the
// same copy of the state.  Each thread looks at kOItems consecutive O terms
// per tile; a class bitmap (small, cache-resident) rejects the terms whose
// partner class is empty before any range lookup, and all loads of a tile
// are issued before their results are used.
template <typename T>
__device__ uint32_t enumerate_chunk(const BucketArgs& A, uint32_t b, uint32_t base,
                                    uint32_t& o_tile, uint32_t& skip, bool& last, Smem<T>& S) {
  uint32_t nf = 0;
  last = false;
  for (;;) {
    const uint32_t o0 = o_tile * kOTile;
    if (o0 >= A.mO) {
      last = true;
      break;
    }
    const uint32_t ob = o0 + threadIdx.x * kOItems;
    uint32_t cls[kOItems];
    if (ob + kOItems <= A.mO) {
      const uint4* p = reinterpret_cast<const uint4*>(A.clsO + ob);
#pragma unroll
      for (int v = 0; v < kOItems / 4; ++v) {
        const uint4 x = p[v];
        cls[4 * v] = x.x;
        cls[4 * v + 1] = x.y;
        cls[4 * v + 2] = x.z;
        cls[4 * v + 3] = x.w;
      }
    } else {
#pragma unroll
      for (int u = 0; u < kOItems; ++u) cls[u] = ob + u < A.mO ? A.clsO[ob + u] : 0u;
    }
    uint32_t nzw[kOItems];
#pragma unroll
    for (int u = 0; u < kOItems; ++u) nzw[u] = A.nzI[(cls[u] ^ b) >> 5];
    uint32_t st[kOItems], cn[kOItems];
    uint32_t tsum = 0;
#pragma unroll
    for (int u = 0; u < kOItems; ++u) {
      const uint32_t c = cls[u] ^ b;
      const bool nz = ob + u < A.mO && ((nzw[u] >> (c & 31)) & 1u);
      uint2 r = make_uint2(0u, 0u);
      if (nz) r = A.rangeI[c];
      st[u] = r.x;
      cn[u] = r.y;
      tsum += cn[u];
    }
    uint32_t tile_total;
    uint32_t t0 = block_excl(tsum, &tile_total, S.scan);
    const uint32_t space = kCapF - nf;
    const uint32_t hi = skip + space;  // tile-local window [skip, hi)
    if (tsum) {
#pragma unroll
      for (int u = 0; u < kOItems; ++u) {
        if (cn[u]) {
          const uint32_t ks = skip > t0 ? skip - t0 : 0;
          uint32_t ke = hi > t0 ? hi - t0 : 0;
          if (ke > cn[u]) ke = cn[u];
          if (ks < ke) {
            const uint32_t o = ob + u;
            const uint64_t ko = A.keyO[o];
            for (uint32_t k = ks; k < ke; ++k) {
              const IRec rec = A.recI[st[u] + k];
              const uint32_t e = base + nf + (t0 + k - skip);
              S.key[e] = ko ^ rec.key;
              S.id[e] = A.o_is_a ? rec.idx * A.ma + o : o * A.ma + rec.idx;
            }
          }
        }
        t0 += cn[u];
      }
    }
    if (tile_total - skip <= space) {
      nf += tile_total - skip;
      ++o_tile;
      skip = 0;
      if (nf == kCapF) {
        last = o_tile * kOTile >= A.mO;
        break;
      }
    } else {
      nf += space;
      skip += space;
      break;
    }
  }
  __syncthreads();
  return nf;
}

// ord[0..N) = entries ordered stably by key bits [lo, lo + 8*passes).
// Wave w owns positions [w*span, (w+1)*span), visited in rounds of 64; the
// rank of an entry among equal digits is the count of equal digits at
// earlier positions, obtained from eight ballots per round and per-wave
// digit counters.
template <typename T>
__device__ void sort_entries(uint32_t N, int lo, int passes, Smem<T>& S) {
  for (uint32_t q = threadIdx.x; q < N; q += kNT) S.ord[q] = static_cast<uint16_t>(q);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t lt = (1ull << lane) - 1ull;
  const uint32_t span = wave_span(N);
  const int rounds = static_cast<int>(span / 64);
  for (int pass = 0; pass < passes; ++pass) {
    const int shift = lo + 8 * pass;
    for (int i = threadIdx.x; i < kWaves * 256; i += kNT) (&S.cnt[0][0])[i] = 0;
    __syncthreads();
    uint16_t ent[kRounds];
    uint16_t rk[kRounds];
    int dg[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      if (r >= rounds) break;
      const uint32_t q = wave * span + r * 64 + lane;
      const bool valid = q < N;
      ent[r] = valid ? S.ord[q] : 0;
      dg[r] = valid ? static_cast<int>((S.key[ent[r]] >> shift) & 255) : 0;
      uint64_t peers = __ballot(valid);
#pragma unroll
      for (int bit = 0; bit < 8; ++bit) {
        const bool on = valid && ((dg[r] >> bit) & 1);
        const uint64_t bm = __ballot(on);
        peers &= on ? bm : ~bm;
      }
      const uint32_t before = static_cast<uint32_t>(__popcll(peers & lt));
      uint32_t c0 = 0;
      if (valid) c0 = S.cnt[wave][dg[r]];
      rk[r] = static_cast<uint16_t>(c0 + before);
      if (valid && before == 0) S.cnt[wave][dg[r]] = c0 + static_cast<uint32_t>(__popcll(peers));
    }
    __syncthreads();
    uint32_t tot = 0;
    if (threadIdx.x < 256)
      for (int w = 0; w < kWaves; ++w) tot += S.cnt[w][threadIdx.x];
    uint32_t all;
    const uint32_t dstart = block_excl(threadIdx.x < 256 ? tot : 0u, &all, S.scan);
    if (threadIdx.x < 256) {
      uint32_t run = dstart;
      for (int w = 0; w < kWaves; ++w) {
        const uint32_t c = S.cnt[w][threadIdx.x];
        S.cnt[w][threadIdx.x] = run;
        run += c;
      }
    }
    __syncthreads();
    uint32_t np[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      if (r >= rounds) break;
      const uint32_t q = wave * span + r * 64 + lane;
      np[r] = q < N ? S.cnt[wave][dg[r]] + rk[r] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      if (r >= rounds) break;
      const uint32_t q = wave * span + r * 64 + lane;
      if (q < N) S.ord[np[r]] = ent[r];
    }
    __syncthreads();
  }
}

// Runs of positions whose radix field ties but whose full keys differ are put
// in (key, entry) order by the thread that owns the run's first position.
template <typename T>
__device__ void fix_runs(uint32_t N, int lo, uint64_t fmask, Smem<T>& S) {
  bool dirty = false;
  for (uint32_t q = threadIdx.x + 1; q < N; q += kNT) {
    const uint64_t k1 = S.key[S.ord[q - 1]], k2 = S.key[S.ord[q]];
    if (k1 != k2 && ((k1 >> lo) & fmask) == ((k2 >> lo) & fmask)) dirty = true;
  }
  if (!__syncthreads_or(dirty)) return;
  for (uint32_t q = threadIdx.x; q < N; q += kNT) {
    const uint64_t f = (S.key[S.ord[q]] >> lo) & fmask;
    if (q > 0 && ((S.key[S.ord[q - 1]] >> lo) & fmask) == f) continue;
    uint32_t e = q + 1;
    while (e < N && ((S.key[S.ord[e]] >> lo) & fmask) == f) ++e;
    for (uint32_t x = q + 1; x < e; ++x) {
      const uint16_t v = S.ord[x];
      const uint64_t kv = S.key[v];
      int y = static_cast<int>(x) - 1;
      while (y >= static_cast<int>(q)) {
        const uint16_t u = S.ord[y];
        const uint64_t ku = S.key[u];
        if (ku < kv || (ku == kv && u < v)) break;
        S.ord[y + 1] = u;
        --y;
      }
      S.ord[y + 1] = v;
    }
  }
  __syncthreads();
}

// Decoupled look-back over buckets: returns the number of merged terms in
// buckets before b and publishes b's inclusive count.  Only thread 0 calls.
__device__ unsigned long long lookback(const BucketArgs& A, uint32_t b, unsigned long long agg) {
  constexpr unsigned long long kAgg = 1ull << 62, kIncl = 2ull << 62, kMask = (1ull << 62) - 1;
  if (b == 0) {
    __hip_atomic_store(&A.status[0], kIncl | agg, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    return 0;
  }
  __hip_atomic_store(&A.status[b], kAgg | agg, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  unsigned long long excl = 0;
  int64_t j = static_cast<int64_t>(b) - 1;
  uint32_t spins = 0;
  while (j >= 0) {
    const unsigned long long v =
        __hip_atomic_load(&A.status[j], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long flag = v >> 62;
    if (flag == 0) {
      if (++spins > (1u << 26)) {  // a predecessor never published: give up
        atomicOr(A.err, kErrTimeout);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    excl += v & kMask;
    if (flag == 2) break;
    --j;
  }
  __hip_atomic_store(&A.status[b], kIncl | (excl + agg), __ATOMIC_RELEASE,
                     __HIP_MEMORY_SCOPE_AGENT);
  return excl;
}

template <int WT, typename T>
__device__ __forceinline__ void write_term(const BucketArgs& A, const PairSrc<WT, T>& src,
                                           int64_t o, const uint64_t* w, T re, T im,
                                           uint32_t id) {
#pragma unroll
  for (int q = 0; q < WT; ++q) {
    if (WT > 8 && q >= src.nw) break;
    A.OX[q * A.ldo + o] = w[q];
    A.OZ[q * A.ldo + o] = w[src.nw + q];
  }
  A.Oph[o] = 0;
  static_cast<cplx<T>*>(A.Oc)[o] = cplx<T>{re, im};
  A.Ofp[o] = src.fp(id);
}

// What a segment tail does with its finished sum.
enum : int {
  kEmitWrite = 0,      // write the merged term at out_base + segment index
  kEmitRun = 1,        // store (key, id, sum) as running entry `segment index`
  kEmitCount = 2,      // set the segment's keep bit (|sum|^2 >= t^2)
  kEmitWriteKept = 3,  // write the term if its keep bit is set, packed
};

template <int WT, typename T, int MODE>
__device__ __forceinline__ void emit(const BucketArgs& A, const PairSrc<WT, T>& src, Smem<T>& S,
                                     RunEntry<T>* run, unsigned long long out_base, uint32_t seg,
                                     const uint64_t* w, uint64_t key, uint32_t id, T re, T im) {
  if (MODE == kEmitWrite) {
    write_term<WT, T>(A, src, static_cast<int64_t>(out_base + seg), w, re, im, id);
  } else if (MODE == kEmitRun) {
    run[seg] = RunEntry<T>{key, id, 0u, re, im};
  } else if (MODE == kEmitCount) {
    const double dr = re, di = im;
    if (!(dr * dr + di * di < A.drop2)) atomicOr(&S.keep[seg >> 5], 1u << (seg & 31));
  } else {
    const uint32_t bits = S.keep[seg >> 5];
    if ((bits >> (seg & 31)) & 1u) {
      const uint32_t o = S.kpre[seg >> 5] + __popc(bits & ((1u << (seg & 31)) - 1u));
      write_term<WT, T>(A, src, static_cast<int64_t>(out_base + o), w, re, im, id);
    }
  }
}

// Segmented sums over positions [0, N) in position order: a wave scan inside
// each round of 64, a carried partial across the rounds of a wave, and the
// wave carries combined in wave order by one thread, so the additions happen
// in a fixed order.  Each segment's tail ends with the segment's sum and
// emits it (MODE).  The tail of the segment already open when a wave's span
// begins is finished after the wave carries are known.
template <int WT, typename T, int MODE>
__device__ void segment_pass(const BucketArgs& A, const PairSrc<WT, T>& src, uint32_t N,
                             uint32_t nR, uint32_t wbase, unsigned long long out_base, Smem<T>& S,
                             RunEntry<T>* run) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t lt = (1ull << lane) - 1ull;
  const uint32_t span = wave_span(N);
  const int rounds = static_cast<int>(span / 64);
  if (lane == 0) S.dvalid[wave] = 0;
  T cre = 0, cim = 0;
  bool copen = false;
  uint32_t hrun = wbase;
#pragma unroll 1
  for (int r = 0; r < rounds; ++r) {
    const uint32_t q = wave * span + r * 64 + lane;
    const bool valid = q < N;
    uint32_t e = 0, id = 0;
    uint64_t k = 0;
    bool head = false, tail = false;
    uint64_t w[2 * WT];
    T vre = 0, vim = 0;
    if (valid) {
      e = S.ord[q];
      k = S.key[e];
      id = S.id[e];
      head = q == 0 || S.key[S.ord[q - 1]] != k;
      tail = q + 1 >= N || S.key[S.ord[q + 1]] != k;
      const cplx<T> pv = src.term(id, w);
      if (e < nR) {
        vre = S.rv[e].re;
        vim = S.rv[e].im;
      } else {
        vre = pv.re;
        vim = pv.im;
      }
    }
    // equal keys must be equal strings
    const bool keq = valid && !head;
    if (__ballot(keq)) {
      // the predecessor's string: from lane - 1, or rebuilt for lane 0
      const uint32_t pid = (lane == 0 && keq) ? S.id[S.ord[q - 1]] : 0u;
      uint64_t diff = 0;
#pragma unroll
      for (int t = 0; t < 2 * WT; ++t) {
        if (WT > 8 && t >= 2 * src.nw) break;
        uint64_t pw = __shfl_up(w[t], 1, 64);
        if (lane == 0 && keq) pw = src.word(pid, t);
        diff |= pw ^ w[t];
      }
      if (keq && diff) atomicOr(A.err, kErrCollision);
    }
    // segmented inclusive scan within the round
    bool f = head;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const T ore = __shfl_up(vre, d, 64), oim = __shfl_up(vim, d, 64);
      const bool of = __shfl_up(static_cast<int>(f), d, 64) != 0;
      if (lane >= d) {
        if (!f) {
          vre = ore + vre;
          vim = oim + vim;
        }
        f = f || of;
      }
    }
    if (!f) {
      vre = cre + vre;
      vim = cim + vim;
    }
    const bool inwave = f || copen;
    const uint64_t hb = __ballot(head);
    const uint32_t seg = hrun + static_cast<uint32_t>(__popcll(hb & (lt | (1ull << lane)))) - 1;
    if (tail) {
      if (inwave) {
        emit<WT, T, MODE>(A, src, S, run, out_base, seg, w, k, id, vre, vim);
      } else {  // segment open since an earlier wave: finished below
        S.dvalid[wave] = 1;
        S.did[wave] = id;
        S.dseg[wave] = seg;
        S.dkey[wave] = k;
        S.dre[wave] = vre;
        S.dim[wave] = vim;
      }
    }
    cre = __shfl(vre, 63, 64);
    cim = __shfl(vim, 63, 64);
    copen = __shfl(static_cast<int>(inwave), 63, 64) != 0;
    hrun += static_cast<uint32_t>(__popcll(hb));
  }
  if (lane == 0) {
    S.whead[wave] = copen ? 1u : 0u;
    S.wre[wave] = cre;
    S.wim[wave] = cim;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    T c_re = 0, c_im = 0;
    for (int v = 0; v < kWaves; ++v) {
      S.cin_re[v] = c_re;
      S.cin_im[v] = c_im;
      if (S.whead[v]) {
        c_re = S.wre[v];
        c_im = S.wim[v];
      } else {
        c_re = c_re + S.wre[v];
        c_im = c_im + S.wim[v];
      }
    }
    for (int v = 0; v < kWaves; ++v)
      if (S.dvalid[v]) {
        S.dre[v] = S.cin_re[v] + S.dre[v];
        S.dim[v] = S.cin_im[v] + S.dim[v];
      }
  }
  __syncthreads();
  if (lane == 0 && S.dvalid[wave]) {
    uint64_t w[2 * WT];
    const uint32_t id = S.did[wave];
    if (MODE == kEmitWrite || MODE == kEmitWriteKept) src.string(id, w);
    emit<WT, T, MODE>(A, src, S, run, out_base, S.dseg[wave], w, S.dkey[wave], id, S.dre[wave],
                      S.dim[wave]);
  }
  __syncthreads();
}

// One block per resident slot; each takes buckets by ticket until none are
// left.  Taking tickets in order keeps the look-back free of deadlock: a
// bucket only waits for buckets whose tickets were taken by running blocks.
template <int WT, typename T>
__global__ void __launch_bounds__(kNT, 4)
k_bucket_merge(BucketArgs A, PairSrc<WT, T> src) {
  __shared__ Smem<T> S;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  RunEntry<T>* run = static_cast<RunEntry<T>*>(A.scratch) + static_cast<size_t>(blockIdx.x) * kCapR;
  for (;;) {
    if (threadIdx.x == 0) S.bcast[0] = atomicAdd(A.ticket, 1u);
    __syncthreads();
    const uint32_t b = S.bcast[0];
    __syncthreads();
    if (b >= A.nbuckets) return;

    uint32_t nR = 0, o_tile = 0, skip = 0;
    bool last = false;
    bool published = false;
    for (;;) {
      const uint32_t nf = enumerate_chunk(A, b, nR, o_tile, skip, last, S);
      const uint32_t N = nR + nf;
      sort_entries(N, A.sort_lo, A.sort_passes, S);
      fix_runs(N, A.sort_lo, A.field_mask, S);

      // segment heads: count per wave, then the block prefix
      const uint32_t span = wave_span(N);
      uint32_t hc = 0;
      for (uint32_t r = 0; r * 64 < span; ++r) {
        const uint32_t q = wave * span + r * 64 + lane;
        bool head = false;
        if (q < N) head = q == 0 || S.key[S.ord[q - 1]] != S.key[S.ord[q]];
        hc += static_cast<uint32_t>(__popcll(__ballot(head)));
      }
      if (lane == 0) S.wcount[wave] = hc;
      __syncthreads();
      uint32_t wbase = 0, nseg = 0;
      for (int v = 0; v < kWaves; ++v) {
        const uint32_t c = S.wcount[v];
        if (v < wave) wbase += c;
        nseg += c;
      }

      if (!last) {
        // the chunk's segments become the running entries of the next chunk
        if (nseg > static_cast<uint32_t>(kCapR)) {
          if (threadIdx.x == 0) atomicOr(A.err, kErrCapacity);
          break;
        }
        segment_pass<WT, T, kEmitRun>(A, src, N, nR, wbase, 0ull, S, run);
        for (uint32_t t = threadIdx.x; t < nseg; t += kNT) {
          const RunEntry<T> x = run[t];
          S.key[t] = x.key;
          S.id[t] = x.id;
          S.rv[t] = cplx<T>{x.re, x.im};
        }
        __syncthreads();
        nR = nseg;
        continue;
      }

      if (!A.drop) {
        // the merged count of this bucket is known: take the output range now
        // and let each tail write its term as soon as its sum is complete
        if (threadIdx.x == 0) {
          S.out_base = lookback(A, b, nseg);
          atomicAdd(A.total, static_cast<unsigned long long>(nseg));
        }
        published = true;
        __syncthreads();
        segment_pass<WT, T, kEmitWrite>(A, src, N, nR, wbase, S.out_base, S, run);
        break;
      }

      // drop threshold: a first pass marks the kept segments, then the
      // output range is taken and a second pass writes the kept terms
      for (uint32_t t = threadIdx.x; t < (N + 31) / 32; t += kNT) S.keep[t] = 0;
      __syncthreads();
      segment_pass<WT, T, kEmitCount>(A, src, N, nR, wbase, 0ull, S, run);
      if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (uint32_t t = 0; t < (nseg + 31) / 32; ++t) {
          S.kpre[t] = acc;
          acc += __popc(S.keep[t]);
        }
        S.out_base = lookback(A, b, acc);
        atomicAdd(A.total, static_cast<unsigned long long>(acc));
      }
      published = true;
      __syncthreads();
      segment_pass<WT, T, kEmitWriteKept>(A, src, N, nR, wbase, S.out_base, S, run);
      break;
    }
    if (!published && threadIdx.x == 0) lookback(A, b, 0);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- prep

__global__ void k_side_keys(const uint64_t* __restrict__ fp, uint32_t m, int kshift, int dshift,
                            int dbits, uint64_t* __restrict__ key, uint32_t* __restrict__ cls,
                            uint64_t* __restrict__ cls64, uint32_t* __restrict__ idx) {
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < m; t += gridDim.x * blockDim.x) {
    const uint64_t k = fp[t] >> kshift;
    const uint32_t c = dbits ? static_cast<uint32_t>(k >> dshift) : 0u;
    if (key) key[t] = k;
    if (cls) cls[t] = c;
    if (cls64) cls64[t] = c;
    if (idx) idx[t] = t;
  }
}

__global__ void k_class_hist(const uint64_t* __restrict__ cls_sorted, uint32_t m,
                             uint32_t* __restrict__ count) {
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < m; t += gridDim.x * blockDim.x)
    atomicAdd(&count[cls_sorted[t]], 1u);
}

__global__ void k_class_range(const uint32_t* __restrict__ count, const uint32_t* __restrict__ start,
                              uint32_t nc, uint2* __restrict__ range) {
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x)
    range[c] = make_uint2(start[c], count[c]);
}

__global__ void k_gather_records(const uint64_t* __restrict__ fp, const uint32_t* __restrict__ idx,
                                 uint32_t m, int kshift, IRec* __restrict__ rec) {
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < m; t += gridDim.x * blockDim.x) {
    const uint32_t i = idx[t];
    rec[t] = IRec{fp[i] >> kshift, i, 0u};
  }
}

__global__ void k_class_bitmap(const uint32_t* __restrict__ count, uint32_t nc,
                               uint32_t* __restrict__ bits) {
  const uint32_t nw = (nc + 31) / 32;
  for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < nw; w += gridDim.x * blockDim.x) {
    uint32_t v = 0;
    for (uint32_t t = 0; t < 32 && 32 * w + t < nc; ++t)
      if (count[32 * w + t]) v |= 1u << t;
    bits[w] = v;
  }
}

__global__ void k_bucket_init(uint32_t* ctr, int nctr, unsigned long long* status, uint32_t n) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < static_cast<uint32_t>(nctr)) ctr[g] = 0;
  for (uint32_t t = g; t < n; t += gridDim.x * blockDim.x) status[t] = 0;
}

__global__ void k_zero_u32_n(uint32_t* p, uint32_t n) {
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x)
    p[t] = 0;
}

inline unsigned grid_for(int64_t n, int per = 256) {
  int64_t g = (n + per - 1) / per;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return static_cast<unsigned>(g);
}

template <int WT, typename T>
paulisum* fused_t(const paulisum* a, const paulisum* b, const MergeArgs& o, hipStream_t s) {
  const int W = a->W;
  const int64_t P = a->m * b->m;
  const int kb = o.key_bits;
  const int kshift = 64 - kb;
  int d = 0;
  if (P > kCapF) d = static_cast<int>(std::ceil(std::log2(static_cast<double>(P) / kTargetBucket)));
  if (d < 0) d = 0;
  if (d > kb) d = kb;
  if (d > 22) d = 22;
  const uint32_t nb = 1u << d;
  const int rem = kb - d;
  int sort_lo, passes;
  uint64_t fmask;
  if (rem >= 16) {
    sort_lo = rem - 16;
    passes = 2;
    fmask = 0xFFFFull;
  } else {
    sort_lo = 0;
    passes = (rem + 7) / 8;
    fmask = rem ? ((1ull << rem) - 1) : 0;
  }

  const bool o_is_a = a->m <= b->m;
  const paulisum* O = o_is_a ? a : b;
  const paulisum* I = o_is_a ? b : a;
  const uint32_t mO = static_cast<uint32_t>(O->m), mI = static_cast<uint32_t>(I->m);

  DBuf ra(a->m * 2 * W * sizeof(uint64_t), s), ea(a->m, s);
  DBuf rb(b->m * 2 * W * sizeof(uint64_t), s), eb(b->m, s);
  DBuf keyO(mO * 8ull, s), clsO(mO * 4ull, s);
  DBuf clsI(mI * 8ull, s), clsI2(mI * 8ull, s), idxI(mI * 4ull, s), idxI2(mI * 4ull, s);
  DBuf recI(mI * sizeof(IRec), s), cnt(nb * 4ull, s), start(nb * 4ull + 4, s);
  DBuf range(nb * 8ull, s), nzI(((nb + 31) / 32) * 4ull, s);
  DBuf ctr(64, s), status(nb * 8ull, s);
  uint32_t* ctr32 = ctr.as<uint32_t>();
  unsigned long long* total = reinterpret_cast<unsigned long long*>(ctr32 + 2);
  uint32_t* idx_sorted = idxI.as<uint32_t>();
  {
    StageScope sc(PAULI_STAGE_PREP, s, (a->m + b->m) * (32.0 * W + 24.0));
    launch_prep_side(a, ra.as<uint64_t>(), ea.as<uint8_t>(), s);
    launch_prep_side(b, rb.as<uint64_t>(), eb.as<uint8_t>(), s);
    const int dshift = kb - d;
    hipLaunchKernelGGL(k_side_keys, dim3(grid_for(mO)), dim3(256), 0, s, O->fp, mO, kshift, dshift,
                       d, keyO.as<uint64_t>(), clsO.as<uint32_t>(), nullptr, nullptr);
    hipLaunchKernelGGL(k_side_keys, dim3(grid_for(mI)), dim3(256), 0, s, I->fp, mI, kshift, dshift,
                       d, nullptr, nullptr, clsI.as<uint64_t>(), idxI.as<uint32_t>());
    hipLaunchKernelGGL(k_bucket_init, dim3(grid_for(nb)), dim3(256), 0, s, ctr32, 16,
                       status.as<unsigned long long>(), nb);
    PAULI_HIP(hipGetLastError());
    uint64_t* cls_sorted = clsI.as<uint64_t>();
    if (d > 0) {
      DBuf rwork(radix_workspace_bytes(mI), s);
      if (radix_sort_pairs(clsI.as<uint64_t>(), idxI.as<uint32_t>(), clsI2.as<uint64_t>(),
                           idxI2.as<uint32_t>(), mI, d, rwork.p, s)) {
        cls_sorted = clsI2.as<uint64_t>();
        idx_sorted = idxI2.as<uint32_t>();
      }
    }
    hipLaunchKernelGGL(k_zero_u32_n, dim3(grid_for(nb)), dim3(256), 0, s, cnt.as<uint32_t>(), nb);
    hipLaunchKernelGGL(k_class_hist, dim3(grid_for(mI)), dim3(256), 0, s, cls_sorted, mI,
                       cnt.as<uint32_t>());
    DBuf swork(scan_workspace_bytes(nb), s);
    scan_exclusive_u32(cnt.as<uint32_t>(), start.as<uint32_t>(), nb, nullptr, swork.p, s);
    hipLaunchKernelGGL(k_class_range, dim3(grid_for(nb)), dim3(256), 0, s, cnt.as<uint32_t>(),
                       start.as<uint32_t>(), nb, range.as<uint2>());
    hipLaunchKernelGGL(k_class_bitmap, dim3(grid_for((nb + 31) / 32)), dim3(256), 0, s,
                       cnt.as<uint32_t>(), nb, nzI.as<uint32_t>());
    hipLaunchKernelGGL(k_gather_records, dim3(grid_for(mI)), dim3(256), 0, s, I->fp, idx_sorted,
                       mI, kshift, recI.as<IRec>());
    PAULI_HIP(hipGetLastError());
  }

  paulisum* out = new_sum(a->n, 0, P, a->dtype, s);
  BucketArgs A;
  A.keyO = keyO.as<uint64_t>();
  A.clsO = clsO.as<uint32_t>();
  A.mO = mO;
  A.recI = recI.as<IRec>();
  A.rangeI = range.as<uint2>();
  A.nzI = nzI.as<uint32_t>();
  A.o_is_a = o_is_a ? 1 : 0;
  A.ma = static_cast<uint32_t>(a->m);
  A.sort_lo = sort_lo;
  A.sort_passes = passes;
  A.field_mask = fmask;
  A.drop = o.drop_abs >= 0.0 ? 1 : 0;
  A.drop2 = o.drop_abs >= 0.0 ? o.drop_abs * o.drop_abs : -1.0;
  A.nbuckets = nb;
  A.ticket = ctr32;
  A.err = ctr32 + 1;
  A.total = total;
  A.status = status.as<unsigned long long>();
  A.OX = out->X;
  A.OZ = out->Z;
  A.Oph = out->ph;
  A.Oc = out->coef;
  A.Ofp = out->fp;
  A.ldo = out->ld;
  PairSrc<WT, T> src{ra.as<uint64_t>(), ea.as<uint8_t>(), static_cast<const cplx<T>*>(a->coef),
                     a->fp, rb.as<uint64_t>(), eb.as<uint8_t>(),
                     static_cast<const cplx<T>*>(b->coef), b->fp, static_cast<uint32_t>(a->m), W};
  // persistent grid: as many blocks as fit on the device at once
  int dev = 0, ncu = 0, per_cu = 0;
  PAULI_HIP(hipGetDevice(&dev));
  PAULI_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  PAULI_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_bucket_merge<WT, T>, kNT, 0));
  if (per_cu < 1) per_cu = 1;
  uint32_t grid = static_cast<uint32_t>(ncu) * static_cast<uint32_t>(per_cu);
  if (grid > nb) grid = nb;
  DBuf scratch(static_cast<size_t>(grid) * kCapR * sizeof(RunEntry<T>), s);
  A.scratch = scratch.p;
  StageScope sc(PAULI_STAGE_BUCKET, s, 0.0);
  hipLaunchKernelGGL((k_bucket_merge<WT, T>), dim3(grid), dim3(kNT), 0, s, A, src);
  PAULI_HIP(hipGetLastError());
  sc.stop();
  uint32_t host[4] = {0, 0, 0, 0};
  PAULI_HIP(hipMemcpyAsync(host, ctr32, sizeof(host), hipMemcpyDeviceToHost, s));
  PAULI_HIP(hipStreamSynchronize(s));
  const uint64_t U = static_cast<uint64_t>(host[2]) | (static_cast<uint64_t>(host[3]) << 32);
  if (host[1] != 0) {
    sc.bytes = 0;
    free_sum(out);
    return nullptr;  // collision / capacity / timeout: the caller falls back
  }
  // compulsory traffic: each merged term written once, each operand read once
  const double per = 16.0 * W + sizeof(cplx<T>) + 1 + 8;
  sc.bytes = per * static_cast<double>(U) + per * static_cast<double>(a->m + b->m);
  out->m = static_cast<int64_t>(U);
  return out;
}

template <typename T>
paulisum* fused_w(const paulisum* a, const paulisum* b, const MergeArgs& o, hipStream_t s) {
  switch (a->W) {
    case 1: return fused_t<1, T>(a, b, o, s);
    case 2: return fused_t<2, T>(a, b, o, s);
    case 3: return fused_t<3, T>(a, b, o, s);
    case 4: return fused_t<4, T>(a, b, o, s);
    case 5: return fused_t<5, T>(a, b, o, s);
    case 6: return fused_t<6, T>(a, b, o, s);
    case 7: return fused_t<7, T>(a, b, o, s);
    case 8: return fused_t<8, T>(a, b, o, s);
    default: return fused_t<kMaxWords, T>(a, b, o, s);
  }
}

}  // namespace

paulisum* fused_bucket(const paulisum* a, const paulisum* b, const MergeArgs& o, hipStream_t s) {
  if (a->dtype == PAULI_C128) return fused_w<double>(a, b, o, s);
  return fused_w<float>(a, b, o, s);
}

}  // namespace pauli
