// Kernels of the fused outer product + sort-and-combine: merge(H1*H2)
// without storing the
// |H1|*|H2| unmerged products (Section IV-C's product followed by
// Section III-H's sort and linear combine).
//
// The sort key of a product is its 64-bit fingerprint and
// fp(a_i * b_j) = fp(a_i) ^ fp(b_j) (the fingerprint is GF(2)-linear and
// the product XORs the symplectic bits, Section III-E).  The top d bits of
// the key name the product's bucket.  Stages:
//
//  1 prep      per operand: rows of word pairs (X_w, Z_w), coefficient +
//              fingerprint + phase metadata (in the row's slot when the row
//              leaves room in its cache line), key, and a stable sort of its
//              terms by class (top d1 key bits).
//  2 gen       the products of class hA of a and class hB of b all have top
//              bits hA ^ hB, so super-bucket s is the union of the class
//              tiles (hA, hA ^ s), whose sizes and offsets follow from the
//              class counts.  Records (key, pair id) are generated tile by
//              tile, counted by the next d2 key bits, and generated again
//              straight into their buckets (each record written once).  For
//              a sum times itself only the tiles hA <= hB are generated and
//              each record stands for an unordered pair.
//  3 sort      per bucket, in LDS: counting sort on the 13 key bits below
//              the bucket bits, then each bin in (key, pair id) order; writes
//              the sorted pair ids and each record's segment index (equal
//              keys = one segment).  A bucket with a bin of many equal keys
//              takes a stable LDS radix sort on 16 bits with ties finished on
//              the full key; a bucket too large for LDS is sorted on all
//              remaining key bits by one block in global memory.
//  4 scan      segment counts -> output offsets.
//  5 expand    per record: a group of G lanes loads the record's two operand
//              rows with one 16-byte load per lane (one cache line per row),
//              forms the product string and phase (cross-lane sums and
//              broadcasts by DPP), and the segment's value i^k c_a c_b is
//              summed in record order; each segment stages one merged term,
//              and staged terms are stored in aligned blocks.  Equal keys are
//              checked to be equal strings; a fingerprint collision raises a
//              flag and the caller redoes the call with the general pipeline.
//              Segments longer than kLong records are summed by a whole
//              block in a fixed tree.
//
// Included by k_fused.hip (one product per call) and k_batched.hip (many
// products per launch sequence); the expand kernels are in expand.h.
#pragma once

#include <cmath>
#include <type_traits>
#include <utility>

#include "common.h"
#include "expand.h"
#include "internal.h"

namespace pauli {

namespace {


// The generation kernels: blocks of kGenNT threads over partition tiles of
// kTile records (16 per thread).  Large tiles give long runs of equal digits
// in the scatter's output (64 records on average at 128 digits), whose writes
// cover whole lines.
constexpr int kGenNT = 512;
constexpr int kItems = 16;
constexpr int kTile = kGenNT * kItems;
static_assert(kTile <= 65536, "tile positions are 16-bit");
constexpr int kSortNT = 512;
constexpr int kSortWaves = kSortNT / 64;
constexpr int kSortBlocksPerCU = 2;  // two bucket sorts share a compute unit's LDS
constexpr int kCap = 4096;  // records of a bucket sorted in LDS
constexpr int kSortRounds = kCap / kSortWaves / 64;
constexpr int kMaxBits = 16;
constexpr double kTargetBucket = 3500.0;  // records per bucket; the LDS sort takes up to kCap

inline unsigned grid_for(int64_t n, int per = kB, int64_t cap = 65536) {
  int64_t g = (n + per - 1) / per;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return static_cast<unsigned>(g);
}

// Compute units of the current device.
inline uint32_t device_cus() {
  int dev = 0, n = 0;
  PAULI_HIP(hipGetDevice(&dev));
  PAULI_HIP(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev));
  return n > 0 ? static_cast<uint32_t>(n) : 1u;
}

__device__ __forceinline__ uint32_t wave_incl(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}

// Exclusive scan over a block of NW waves; every thread must call it.
template <int NW>
__device__ __forceinline__ uint32_t block_excl(uint32_t v, uint32_t* total, uint32_t* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t inc = wave_incl(v);
  if (lane == 63) sh[wave] = inc;
  __syncthreads();
  uint32_t base = 0, all = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const uint32_t x = sh[w];
    if (w < wave) base += x;
    all += x;
  }
  __syncthreads();
  if (total) *total = all;
  return base + inc - v;
}

// ------------------------------------------------------------------ prep

template <typename T>
__global__ void k_fprep(const uint64_t* __restrict__ X, const uint64_t* __restrict__ Z,
                        const uint8_t* __restrict__ ph, const cplx<T>* __restrict__ c,
                        const uint64_t* __restrict__ fp, int W, int Wp, int64_t ld, uint32_t m,
                        int kshift, int cshift, int d1, uint64_t* __restrict__ rows,
                        Aux<T>* __restrict__ aux, uint64_t* __restrict__ key,
                        uint64_t* __restrict__ cls, uint32_t* __restrict__ idx) {
  const int SW = slot_words(Wp);
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < m; t += gridDim.x * blockDim.x) {
    int y = 0;
    for (int w = 0; w < Wp; ++w) {
      const uint64_t x = w < W ? X[w * ld + t] : 0ull;
      const uint64_t z = w < W ? Z[w * ld + t] : 0ull;
      rows[static_cast<size_t>(t) * SW + 2 * w] = x;
      rows[static_cast<size_t>(t) * SW + 2 * w + 1] = z;
      y += popc64(x & z);
    }
    Aux<T> x;
    x.w[0] = to_word<T>(c[t].re);
    x.w[1] = to_word<T>(c[t].im);
    x.w[2] = fp[t];
    const uint64_t k = fp[t] >> kshift;
    const uint64_t c_id = d1 ? (k >> cshift) : 0ull;
    x.w[3] = static_cast<uint64_t>((ph[t] + y) & 3) | (static_cast<uint64_t>(y & 1) << 2) |
             (c_id << 8);
    aux[t] = x;
    if (Wp <= 4)
      for (int q = 0; q < 4; ++q) rows[static_cast<size_t>(t) * SW + 2 * Wp + q] = x.w[q];
    key[t] = k;
    cls[t] = c_id;
    idx[t] = t;
  }
}

// Terms per class from the class-sorted keys: a class occupies one run, so
// its first term adds -start and its last term adds end + 1 (two atomics per
// class, none per term).  g must be zero.
__global__ void k_class_count(const uint64_t* __restrict__ cls, uint32_t m,
                              uint32_t* __restrict__ g) {
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < m; t += gridDim.x * blockDim.x) {
    const uint64_t c = cls[t];
    if (t == 0 || cls[t - 1] != c) atomicAdd(&g[c], 0u - t);
    if (t + 1 == m || cls[t + 1] != c) atomicAdd(&g[c], t + 1);
  }
}

// The top 16 bits of a kb-bit key (left-aligned when kb < 16).  Every
// digit the generation passes histogram lies in them (bucket bits <= 16).
__host__ __device__ __forceinline__ uint16_t key_top16(uint64_t k, int kb) {
  return static_cast<uint16_t>(kb >= 16 ? k >> (kb - 16) : k << (16 - kb));
}

// (key, term index) of a term in class order, as one 16-byte piece.
__host__ __device__ __forceinline__ uint4 key_index(uint64_t k, uint32_t i) {
  return make_uint4(static_cast<uint32_t>(k), static_cast<uint32_t>(k >> 32), i, 0u);
}

__global__ void k_gather_keys(const uint64_t* __restrict__ key, const uint32_t* __restrict__ sidx,
                              uint32_t m, int kb, uint64_t* __restrict__ skey,
                              uint16_t* __restrict__ top, uint4* __restrict__ ki) {
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < m; t += gridDim.x * blockDim.x) {
    const uint32_t i = sidx[t];
    const uint64_t k = key[i];
    skey[t] = k;
    top[t] = key_top16(k, kb);
    ki[t] = key_index(k, i);
  }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t n, uint32_t v) {
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x)
    p[t] = v;
}

// Super-bucket s: T[s][hA] = offset of tile (hA, hA ^ s) inside s; S[s] = size.
// With sym (a sum times itself) tiles with hA > hA ^ s are empty.
__global__ void __launch_bounds__(kB)
k_tile_table(const uint32_t* __restrict__ gA, const uint32_t* __restrict__ gB, int d1, int sym,
             uint32_t* __restrict__ Tt, uint32_t* __restrict__ S) {
  __shared__ uint32_t sh[kB / 64];
  const uint32_t nc = 1u << d1, s = blockIdx.x, h = threadIdx.x;
  // a product of a sum with itself takes each unordered pair of classes once
  const bool skip = sym && h > (h ^ s);
  const uint32_t size = h < nc && !skip ? gA[h] * gB[h ^ s] : 0u;
  uint32_t tot;
  const uint32_t ex = block_excl<kB / 64>(size, &tot, sh);
  if (h < nc) Tt[s * nc + h] = ex;
  if (h == 0) S[s] = tot;
}

// Records of the class tiles, written in super-bucket order.
__global__ void __launch_bounds__(kB)
k_gen(const uint32_t* __restrict__ gA, const uint32_t* __restrict__ gsA,
      const uint32_t* __restrict__ sidxA, const uint64_t* __restrict__ skeyA,
      const uint32_t* __restrict__ gB, const uint32_t* __restrict__ gsB,
      const uint32_t* __restrict__ sidxB, const uint64_t* __restrict__ skeyB,
      const uint32_t* __restrict__ Tt, const uint32_t* __restrict__ soff, int d1, int sym,
      uint32_t ma, int ibits, uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  const uint32_t nc = 1u << d1, ntile = nc * nc;
  for (uint32_t tau = blockIdx.x; tau < ntile; tau += gridDim.x) {
    const uint32_t s = tau >> d1, hA = tau & (nc - 1), hB = hA ^ s;
    const uint32_t na = gA[hA], nb = gB[hB], n = sym && hA > hB ? 0u : na * nb;
    if (n == 0) continue;
    const uint32_t base = soff[s] + Tt[tau], a0 = gsA[hA], b0 = gsB[hB];
    for (uint32_t t = threadIdx.x; t < n; t += blockDim.x) {
      const uint32_t ia = t / nb, jb = t - ia * nb;
      const uint32_t i = sidxA[a0 + ia], j = sidxB[b0 + jb];
      keys[base + t] = skeyA[a0 + ia] ^ skeyB[b0 + jb];
      vals[base + t] = ibits >= 0 ? ((j << ibits) | i) : j * ma + i;
    }
  }
}

// ---------------------------------------------- partition of super-buckets

__global__ void k_tiles_per_sb(const uint32_t* __restrict__ S, uint32_t nc,
                               uint32_t* __restrict__ nt) {
  for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < nc; s += gridDim.x * blockDim.x)
    nt[s] = (S[s] + kTile - 1) / kTile;
}

// tile tau -> (super-bucket s, tile index inside s); false past the last tile.
__device__ __forceinline__ bool tile_of(uint32_t tau, const uint32_t* tb, uint32_t nc, uint32_t& s,
                                        uint32_t& tl) {
  if (tau >= tb[nc]) return false;
  uint32_t lo = 0, hi = nc;  // largest s with tb[s] <= tau
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (tb[mid] <= tau) lo = mid; else hi = mid;
  }
  s = lo;
  tl = tau - tb[s];
  return true;
}

// ------------------------------ generation fused with the partition pass
//
// Record q of super-bucket s (in k_gen's order) belongs to the class tile
// hA with Tt[s][hA] <= q < Tt[s][hA] + |A_hA| |B_{hA^s}|, the largest hA
// with Tt[s][hA] <= q.  k_gcount and k_gscatter enumerate the records of
// one partition tile that way, so the partition needs no stored copy of the
// generated records: k_gcount histograms their digits, k_gscatter ranks
// them and writes each record once, at its final place.

struct GenSides {
  const uint32_t* gA;
  const uint32_t* gsA;
  const uint4* kiA;  // key_index of each term of A in class order
  const uint32_t* gB;
  const uint32_t* gsB;
  const uint4* kiB;
  const uint32_t* Tt;
  uint32_t ma;
  int ibits;
  int d1;
  // key_top16 of the keys: the passes that need only a record's digit
  // gather 2 bytes per side instead of 8 (fewer lines per gather)
  const uint16_t* tA;
  const uint16_t* tB;
  int sh16;  // 16 - bucket bits: the digit is (tA ^ tB) >> sh16, masked
};

// The super-bucket's tile offsets and class sizes, staged in LDS, with
// mb[h] = floor((2^32 - 1) / nb[h]) for the division by nb[h], and the
// classes [h0, h1] that the block's partition tile spans.
struct GenRow {
  uint32_t t[256], na[256], a0[256], nb[256], b0[256], mb[256];
  uint32_t h0, h1;
};

// Every thread calls it; R is complete after the caller's next barrier.
__device__ __forceinline__ void load_gen_row(const GenSides& G, uint32_t s, uint32_t lo,
                                             uint32_t hi, GenRow& R) {
  const uint32_t nc = 1u << G.d1;
  for (uint32_t h = threadIdx.x; h < nc; h += blockDim.x) {
    R.t[h] = G.Tt[s * nc + h];
    R.na[h] = G.gA[h];
    R.a0[h] = G.gsA[h];
    const uint32_t nb = G.gB[h ^ s];
    R.nb[h] = nb;
    R.mb[h] = nb ? 0xFFFFFFFFu / nb : 0u;
    R.b0[h] = G.gsB[h ^ s];
  }
  __syncthreads();
  // record q lies in the largest class h with t[h] <= q
  const uint32_t last = hi > lo ? hi - 1 : lo;
  for (uint32_t h = threadIdx.x; h < nc; h += blockDim.x) {
    const uint32_t t0 = R.t[h], t1 = h + 1 < nc ? R.t[h + 1] : 0xFFFFFFFFu;
    if (t0 <= lo && lo < t1) R.h0 = h;
    if (t0 <= last && last < t1) R.h1 = h;
  }
}

// The operand positions a (in A's class order) and b of record q.
__device__ __forceinline__ void gen_pair(const GenRow& R, uint32_t q, uint32_t& a, uint32_t& b) {
  uint32_t lo = R.h0, hi = R.h1 + 1;  // largest h with t[h] <= q
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (R.t[mid] <= q) lo = mid; else hi = mid;
  }
  const uint32_t t = q - R.t[lo], nb = R.nb[lo];
  // t / nb: the estimate floor(t * mb / 2^32) is the quotient or one less
  uint32_t ia = __umulhi(t, R.mb[lo]);
  uint32_t jb = t - ia * nb;
  if (jb >= nb) {
    ++ia;
    jb -= nb;
  }
  a = R.a0[lo] + ia;
  b = R.b0[lo] + jb;
}

__device__ __forceinline__ void gen_record(const GenSides& G, const GenRow& R, uint32_t q,
                                           uint64_t& key, uint32_t& val) {
  uint32_t a, b;
  gen_pair(R, q, a, b);
  const uint4 ea = G.kiA[a], eb = G.kiB[b];  // one 16-byte gather per side
  const uint32_t i = ea.z, j = eb.z;
  key = (static_cast<uint64_t>(ea.y ^ eb.y) << 32) | (ea.x ^ eb.x);
  val = G.ibits >= 0 ? ((j << G.ibits) | i) : j * G.ma + i;
}

// The digit of record q alone.
__device__ __forceinline__ uint32_t gen_digit(const GenSides& G, const GenRow& R, uint32_t q,
                                              uint32_t mask) {
  uint32_t a, b;
  gen_pair(R, q, a, b);
  return (static_cast<uint32_t>(G.tA[a] ^ G.tB[b]) >> G.sh16) & mask;
}

// Products of a batched launch sequence: the super-buckets of all products
// are numbered consecutively (product p owns [sbbase[p], sbbase[p + 1])),
// and each product has its own generation tables and digit field.  Null
// tables: one product (the kernel arguments).
struct GenBatch {
  const uint16_t* sbprod;  // [super-bucket] product
  const uint32_t* sbbase;  // [product] first super-bucket
  const GenSides* gen;     // [product]
  const int* shift;        // [product] digit shift of the partition
  const uint32_t* mask;    // [product] digit mask
};

// The tables of the product that owns global super-bucket sg: G, the
// super-bucket's index inside its product (sl), shift and mask.
__device__ __forceinline__ void gen_product(const GenBatch& bt, uint32_t sg, GenSides& G,
                                            uint32_t& sl, int& shift, uint32_t& mask) {
  sl = sg;
  if (bt.sbprod == nullptr) return;
  const uint32_t p = bt.sbprod[sg];
  G = bt.gen[p];
  sl = sg - bt.sbbase[p];
  shift = bt.shift[p];
  mask = bt.mask[p];
}

// Digit histogram of one partition tile.  Count layout: super-bucket s owns
// C[tb[s]*256, tb[s+1]*256) as [digit][tile], so one exclusive scan of C
// gives every (s, digit, tile) its output offset.
__global__ void __launch_bounds__(kGenNT)
k_gcount(GenSides G, GenBatch bt, const uint32_t* __restrict__ S, const uint32_t* __restrict__ tb,
         uint32_t nc, int shift, uint32_t mask, uint32_t* __restrict__ C) {
  __shared__ uint32_t hist[256];
  __shared__ GenRow R;
  uint32_t s, tl, sl;
  if (!tile_of(blockIdx.x, tb, nc, s, tl)) return;
  gen_product(bt, s, G, sl, shift, mask);
  if (threadIdx.x < 256) hist[threadIdx.x] = 0;
  const uint32_t lo = tl * kTile;
  const uint32_t hi = S[s] - lo < kTile ? S[s] : lo + kTile;
  load_gen_row(G, sl, lo, hi, R);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const uint32_t q = lo + r * kGenNT + threadIdx.x;
    if (q < hi) atomicAdd(&hist[gen_digit(G, R, q, mask)], 1u);
  }
  __syncthreads();
  const uint32_t ns = tb[s + 1] - tb[s];
  if (threadIdx.x < 256) C[tb[s] * 256u + threadIdx.x * ns + tl] = hist[threadIdx.x];
}

// Stable scatter of one partition tile's generated records.  Wave w owns
// the tile positions [w*kItems*64, (w+1)*kItems*64) in rounds of 64, so
// ranking each wave's records by digit (ballots and a wave-private digit
// counter, no block barrier) and adding the counts of earlier waves keeps
// the tile's order within each digit.  Only each record's tile position is
// staged in LDS, in digit order; the record is generated again when its
// digit's run is written (coalesced), which keeps the kernel small enough
// for many resident blocks.
__global__ void __launch_bounds__(kGenNT)
k_gscatter(GenSides G, GenBatch bt, uint64_t* __restrict__ kout, uint32_t* __restrict__ vout,
           const uint32_t* __restrict__ S, const uint32_t* __restrict__ tb, uint32_t nc, int shift,
           uint32_t mask, const uint32_t* __restrict__ C) {
  constexpr int NW = kGenNT / 64;
  __shared__ uint16_t s_pos[kTile];
  __shared__ uint32_t s_start[256], s_goff[256];
  __shared__ uint32_t s_wc[NW][256];
  __shared__ uint32_t sh[NW];
  __shared__ GenRow R;
  uint32_t s, tl, sl;
  if (!tile_of(blockIdx.x, tb, nc, s, tl)) return;
  gen_product(bt, s, G, sl, shift, mask);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t lo = tl * kTile;
  const uint32_t hi = S[s] - lo < kTile ? S[s] : lo + kTile;
  const uint32_t ns = tb[s + 1] - tb[s];
  const bool dig = tid < 256;  // threads 0-255 own one digit each
  if (dig) {
#pragma unroll
    for (int w = 0; w < NW; ++w) s_wc[w][tid] = 0;
    s_goff[tid] = C[tb[s] * 256u + tid * ns + tl];
  }
  load_gen_row(G, sl, lo, hi, R);
  __syncthreads();
  const uint64_t lt = (1ull << lane) - 1ull;
  const int dbits = __popc(mask);  // digit bits (mask = 2^d2 - 1, d2 <= 8)
  // digit in bits 0-7 and rank among the wave's equal digits above, or ~0
  uint32_t dr[kItems];
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const uint32_t q = lo + (static_cast<uint32_t>(wave) * kItems + r) * 64 + lane;
    const int d = q < hi ? static_cast<int>(gen_digit(G, R, q, mask)) : -1;
    const bool valid = d >= 0;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      if (bit >= dbits) break;
      const bool on = valid && ((d >> bit) & 1);
      const uint64_t bm = __ballot(on);
      peers &= on ? bm : ~bm;
    }
    const uint32_t rank = static_cast<uint32_t>(__popcll(peers & lt));
    uint32_t base = 0;
    if (valid) base = s_wc[wave][d];
    dr[r] = valid ? static_cast<uint32_t>(d) | ((base + rank) << 8) : 0xFFFFFFFFu;
    if (valid && rank == 0) s_wc[wave][d] = base + static_cast<uint32_t>(__popcll(peers));
  }
  __syncthreads();
  // digit starts inside the tile, then each (wave, digit) start
  uint32_t tot = 0;
  if (dig) {
#pragma unroll
    for (int w = 0; w < NW; ++w) tot += s_wc[w][tid];
  }
  const uint32_t dstart = block_excl<NW>(tot, nullptr, sh);
  if (dig) {
    s_start[tid] = dstart;
    uint32_t run = dstart;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const uint32_t c = s_wc[w][tid];
      s_wc[w][tid] = run;
      run += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kItems; ++r)
    if (dr[r] != 0xFFFFFFFFu) {
      const uint32_t off = s_wc[wave][dr[r] & 255u] + (dr[r] >> 8);
      s_pos[off] = static_cast<uint16_t>((static_cast<uint32_t>(wave) * kItems + r) * 64 + lane);
    }
  __syncthreads();
  const uint32_t cnt = hi - lo;
  for (uint32_t e = tid; e < cnt; e += kGenNT) {
    uint64_t kk;
    uint32_t vv;
    gen_record(G, R, lo + s_pos[e], kk, vv);
    const uint32_t dd = static_cast<uint32_t>((kk >> shift) & mask);
    const uint32_t g = s_goff[dd] + (e - s_start[dd]);
    kout[g] = kk;
    vout[g] = vv;
  }
}

// Bucket bk = (s, digit): first record.
__global__ void k_bucket_offsets(const uint32_t* __restrict__ soff, const uint32_t* __restrict__ tb,
                                 const uint32_t* __restrict__ C, int d2, uint32_t nbk, uint32_t nc,
                                 uint32_t* __restrict__ boff) {
  const uint32_t mask = (1u << d2) - 1u;
  for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b <= nbk; b += gridDim.x * blockDim.x) {
    if (b == nbk) {
      boff[b] = soff[nc];  // all records
      continue;
    }
    const uint32_t s = b >> d2, dd = b & mask;
    const uint32_t ns = tb[s + 1] - tb[s];
    boff[b] = ns ? C[tb[s] * 256u + dd * ns] : soff[s];
  }
}

// ------------------------------------------------------------ bucket sort

// Counting sort of a bucket: 2^13 bins on the key bits just below the bucket
// bits, two 16-bit counters per word (a bucket holds at most kCap = 4096
// records, so neither counts nor starts carry into the other half).
constexpr int kBinBits = 13;
constexpr int kBins = 1 << kBinBits;
constexpr int kBinWords = kBins / 2;
// A bucket with a larger bin (many equal keys) takes the LDS radix sort.  A
// record's place in its bin costs one pass over the bin; a bin of more than
// kSmallBin records that holds a single key (one repeated string) is ranked
// on pair ids alone.  512 keeps the buckets of inputs with many repeated
// strings on the counting sort (segment stage of a 10,000 x 10,000 product
// at n = 64: 1.73 ms with 64, 1.46 with 256, 1.37 with 512 and the one-key
// ranking; the 2,000 x 2,000 product at n = 16: 0.25 -> 0.12 ms).
constexpr uint32_t kMaxBin = 512;
constexpr uint32_t kSmallBin = 16;  // larger bins are checked for holding one key only
constexpr int kWaitVm0 = 0x0F70;  // s_waitcnt vmcnt(0), expcnt and lgkmcnt not waited for

struct SortSmem {
  uint64_t key[kCap];
  uint32_t id[kCap];
  union {
    uint32_t cnt[kSortWaves][256];  // radix sort: per-wave digit counters
    uint32_t bins[kBinWords + 1];   // counting sort: counts, then starts; bin kBins starts at N
  };
  uint16_t perm[kCap];  // counting sort: position of the p-th record in key / id
  uint32_t mixed[kBins / 32];  // counting sort: large bins holding more than one key
  uint32_t cflag;  // counting sort: 1 a bin over kSmallBin records, 2 a bin over kMaxBin
  uint32_t scan[kSortWaves];
  uint32_t wcount[kSortWaves];
};

// Bit fields of the bucket sort: the counting sort takes bits
// [locnt, locnt + kBinBits) (locnt < 0: not used), the radix sort bits
// [lo16, lo16 + 8*passes) with ties on fmask finished on the full key.
struct SortField {
  int locnt;
  int lo16;
  int passes;
  uint64_t fmask;
  int rem;  // key bits below the bucket bits (the heavy sort's field)
};

// The fields for rem key bits below the bucket bits.
inline SortField sort_field_for(int rem) {
  SortField sf;
  sf.locnt = rem >= kBinBits ? rem - kBinBits : -1;
  if (rem >= 16) {
    sf.lo16 = rem - 16;
    sf.passes = 2;
    sf.fmask = 0xFFFFull;
  } else {
    sf.lo16 = 0;
    sf.passes = (rem + 7) / 8;
    sf.fmask = rem ? ((1ull << rem) - 1) : 0ull;
  }
  sf.rem = rem;
  return sf;
}

// Buckets of a batched launch sequence: the product of each bucket and each
// product's sort fields.  Null tables: one product (the kernel arguments).
struct SortBatch {
  const uint16_t* bprod;  // [bucket] product
  const SortField* sf;    // [product]
};
__device__ __forceinline__ SortField sort_field(const SortBatch& sb, uint32_t b,
                                                const SortField& f) {
  return sb.bprod ? sb.sf[sb.bprod[b]] : f;
}

__device__ __forceinline__ uint32_t sort_span(uint32_t N) {
  return ((N + 64 * kSortWaves - 1) / (64 * kSortWaves)) * 64;
}

// Stable LSD radix sort of the (key, id) pairs k[], v[] of a bucket on key
// bits [lo, lo + 8*passes).  Wave w holds positions [w*span, (w+1)*span) in
// rounds of 64 (item r of a lane: position w*span + r*64 + lane); the rank of
// an item among equal digits counts equal digits at earlier positions (eight
// ballots per round and per-wave digit counters).  Each pass scatters the
// pairs to their new positions in LDS and reads back the lane's positions;
// on return S.key / S.id hold the bucket in sorted order and k[], v[] the
// lane's items of it.
__device__ void lds_sort(uint32_t N, int lo, int passes, uint64_t (&k)[kSortRounds],
                         uint32_t (&v)[kSortRounds], SortSmem& S) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t lt = (1ull << lane) - 1ull;
  const uint32_t span = sort_span(N);
  const int rounds = static_cast<int>(span / 64);
  for (int pass = 0; pass < passes; ++pass) {
    const int shift = lo + 8 * pass;
    for (int i = threadIdx.x; i < kSortWaves * 256; i += kSortNT) (&S.cnt[0][0])[i] = 0;
    __syncthreads();
    uint16_t rk[kSortRounds];
    uint8_t dg[kSortRounds];
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
      if (r >= rounds) break;
      const uint32_t q = wave * span + r * 64 + lane;
      const bool valid = q < N;
      const int dgt = valid ? static_cast<int>((k[r] >> shift) & 255) : 0;
      dg[r] = static_cast<uint8_t>(dgt);
      uint64_t peers = __ballot(valid);
#pragma unroll
      for (int bit = 0; bit < 8; ++bit) {
        const bool on = valid && ((dgt >> bit) & 1);
        const uint64_t bm = __ballot(on);
        peers &= on ? bm : ~bm;
      }
      const uint32_t before = static_cast<uint32_t>(__popcll(peers & lt));
      uint32_t c0 = 0;
      if (valid) c0 = S.cnt[wave][dgt];
      rk[r] = static_cast<uint16_t>(c0 + before);
      if (valid && before == 0) S.cnt[wave][dgt] = c0 + static_cast<uint32_t>(__popcll(peers));
    }
    __syncthreads();
    uint32_t tot = 0;
    if (threadIdx.x < 256)
      for (int w = 0; w < kSortWaves; ++w) tot += S.cnt[w][threadIdx.x];
    const uint32_t dstart = block_excl<kSortWaves>(threadIdx.x < 256 ? tot : 0u, nullptr, S.scan);
    if (threadIdx.x < 256) {
      uint32_t run = dstart;
      for (int w = 0; w < kSortWaves; ++w) {
        const uint32_t c = S.cnt[w][threadIdx.x];
        S.cnt[w][threadIdx.x] = run;
        run += c;
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
      if (r >= rounds) break;
      const uint32_t q = wave * span + r * 64 + lane;
      if (q < N) {
        const uint32_t np = S.cnt[wave][dg[r]] + rk[r];
        S.key[np] = k[r];
        S.id[np] = v[r];
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
      if (r >= rounds) break;
      const uint32_t q = wave * span + r * 64 + lane;
      if (q < N) {
        k[r] = S.key[q];
        v[r] = S.id[q];
      }
    }
  }
}

// Runs of positions tied on the radix field but holding different full keys
// are put in key order (stable: equal keys keep their order) by the thread
// owning the run's first position.  Returns whether anything moved (then the
// lanes' register copies are stale).
__device__ bool lds_fix_runs(uint32_t N, int lo, uint64_t fmask, SortSmem& S) {
  bool dirty = false;
  for (uint32_t q = threadIdx.x + 1; q < N; q += kSortNT) {
    const uint64_t k1 = S.key[q - 1], k2 = S.key[q];
    if (k1 != k2 && ((k1 >> lo) & fmask) == ((k2 >> lo) & fmask)) dirty = true;
  }
  if (!__syncthreads_or(dirty)) return false;
  for (uint32_t q = threadIdx.x; q < N; q += kSortNT) {
    const uint64_t f = (S.key[q] >> lo) & fmask;
    if (q > 0 && ((S.key[q - 1] >> lo) & fmask) == f) continue;
    uint32_t e = q + 1;
    while (e < N && ((S.key[e] >> lo) & fmask) == f) ++e;
    for (uint32_t x = q + 1; x < e; ++x) {
      const uint64_t kv = S.key[x];
      const uint32_t iv = S.id[x];
      int y = static_cast<int>(x) - 1;
      while (y >= static_cast<int>(q) && S.key[y] > kv) {
        S.key[y + 1] = S.key[y];
        S.id[y + 1] = S.id[y];
        --y;
      }
      S.key[y + 1] = kv;
      S.id[y + 1] = iv;
    }
  }
  __syncthreads();
  return true;
}


__device__ __forceinline__ uint32_t bin_start(const SortSmem& S, uint32_t d) {
  return (S.bins[d >> 1] >> ((d & 1u) * 16u)) & 0xFFFFu;
}

// Counting sort of a bucket, first half: the (key, id) pairs k[], v[] are
// counted in 2^13 bins of the key bits at lo (a record's place in its bin
// comes from an LDS atomic) and scattered to S.key / S.id grouped by bin.
// Returns 0, with S.key / S.id untouched, when a bin holds more than
// kMaxBin records (many equal keys); else 2 when a bin holds more than
// kSmallBin records, 1 when none does.  k[], v[] are not read afterwards.
__device__ int count_scatter(uint32_t N, int lo, const uint64_t (&k)[kSortRounds],
                              const uint32_t (&v)[kSortRounds], SortSmem& S) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t span = sort_span(N);
  const int rounds = static_cast<int>(span / 64);
  for (int i = threadIdx.x; i <= kBinWords; i += kSortNT) S.bins[i] = 0;
  if (threadIdx.x == 0) S.cflag = 0;
  __syncthreads();
  // a lane past the end adds 0 to a counter of its own
  uint32_t dd[kSortRounds], old[kSortRounds];
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    dd[r] = 0;
    old[r] = 0;
    if (r >= rounds) break;
    const uint32_t q = wave * span + r * 64 + lane;
    const bool valid = q < N;
    const uint32_t d = valid ? static_cast<uint32_t>(k[r] >> lo) & (kBins - 1u) : 2u * lane;
    dd[r] = d;
    old[r] = atomicAdd(&S.bins[d >> 1], valid ? 1u << ((d & 1u) * 16u) : 0u);
  }
  __syncthreads();
  // bins [16t, 16t + 16) belong to thread t (words [8t, 8t + 8))
  static_assert(kBinWords == 8 * kSortNT, "eight words per thread");
  uint4* mine = reinterpret_cast<uint4*>(&S.bins[8 * threadIdx.x]);
  const uint4 w0 = mine[0], w1 = mine[1];
  uint32_t w[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
  uint32_t tot = 0, mx = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const uint32_t c0 = w[i] & 0xFFFFu, c1 = w[i] >> 16;
    tot += c0 + c1;
    mx = max(mx, max(c0, c1));
  }
  if (mx > kSmallBin) atomicOr(&S.cflag, mx > kMaxBin ? 3u : 1u);
  uint32_t run = block_excl<kSortWaves>(tot, nullptr, S.scan);  // (its barriers order the flag)
  const uint32_t fl = S.cflag;
  if (fl & 2u) {
    __syncthreads();  // every thread has read the flag before the next bucket clears it
    return 0;
  }
  const int large = (fl & 1u) ? 2 : 1;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const uint32_t c0 = w[i] & 0xFFFFu, c1 = w[i] >> 16;
    w[i] = run | ((run + c0) << 16);
    run += c0 + c1;
  }
  mine[0] = make_uint4(w[0], w[1], w[2], w[3]);
  mine[1] = make_uint4(w[4], w[5], w[6], w[7]);
  if (threadIdx.x == 0) S.bins[kBinWords] = N;
  __syncthreads();
  uint32_t np[kSortRounds];
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    np[r] = 0;
    if (r >= rounds) break;
    const uint32_t d = dd[r];
    np[r] = bin_start(S, d) + ((old[r] >> ((d & 1u) * 16u)) & 0xFFFFu);
  }
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    if (r >= rounds) break;
    const uint32_t q = wave * span + r * 64 + lane;
    if (q < N) {
      S.key[np[r]] = k[r];
      S.id[np[r]] = v[r];
    }
  }
  __syncthreads();
  return large;
}

// Counting sort, second half: every bin is put in (key, id) order.  The
// sorted position of a record is its bin's start plus the number of smaller
// records in the bin, and S.perm[p] = where the p-th record lies in S.key /
// S.id.  Equal keys end up ordered by pair id, so the result does not
// depend on the order of the atomics.
__device__ void count_order(uint32_t N, int lo, SortSmem& S, bool large) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t span = sort_span(N);
  const int rounds = static_cast<int>(span / 64);
  if (large) {
    // which large bins hold more than one key: records of one repeated
    // string fill a large bin with one key, ordered by pair id alone
    for (int i = threadIdx.x; i < kBins / 32; i += kSortNT) S.mixed[i] = 0;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
      if (r >= rounds) break;
      const uint32_t q = wave * span + r * 64 + lane;
      if (q < N) {
        const uint64_t kq = S.key[q];
        const uint32_t d = static_cast<uint32_t>(kq >> lo) & (kBins - 1u);
        const uint32_t s0 = bin_start(S, d), e0 = bin_start(S, d + 1);
        if (e0 - s0 > kSmallBin && kq != S.key[s0]) atomicOr(&S.mixed[d >> 5], 1u << (d & 31u));
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    if (r >= rounds) break;
    const uint32_t q = wave * span + r * 64 + lane;
    if (q < N) {
      const uint64_t kq = S.key[q];
      const uint32_t iq = S.id[q];
      const uint32_t d = static_cast<uint32_t>(kq >> lo) & (kBins - 1u);
      const uint32_t s0 = bin_start(S, d), e0 = bin_start(S, d + 1);
      uint32_t p = q;
      if (e0 - s0 > kSmallBin && ((S.mixed[d >> 5] >> (d & 31u)) & 1u) == 0) {
        uint32_t rank = 0;  // one key in the bin: the pair id decides
        for (uint32_t y = s0; y < e0; ++y) rank += S.id[y] < iq ? 1u : 0u;
        p = s0 + rank;
      } else if (e0 - s0 > 1) {
        uint32_t rank = 0;
        for (uint32_t y = s0; y < e0; ++y) {
          const uint64_t ky = S.key[y];
          const uint32_t iy = S.id[y];
          rank += (ky < kq || (ky == kq && iy < iq)) ? 1u : 0u;
        }
        p = s0 + rank;
      }
      S.perm[p] = static_cast<uint16_t>(q);
    }
  }
  __syncthreads();
}

// Radix path of a bucket (key fields narrower than the counting sort's):
// stable LSD sort on the radix field, ties finished on the full key.
__device__ void radix_bucket(uint32_t n, uint64_t (&k)[kSortRounds], uint32_t (&v)[kSortRounds],
                             const SortField& f, SortSmem& S) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t span = sort_span(n);
  const int rounds = static_cast<int>(span / 64);
  __syncthreads();  // the block's previous bucket is no longer read
  if (f.passes > 0) {
    lds_sort(n, f.lo16, f.passes, k, v, S);
  } else {
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
      if (r >= rounds) break;
      const uint32_t q = wave * span + r * 64 + lane;
      if (q < n) {
        S.key[q] = k[r];
        S.id[q] = v[r];
      }
    }
  }
  __syncthreads();
  lds_fix_runs(n, f.lo16, f.fmask, S);
}

struct SegOut {
  uint32_t* vals;    // sorted pair ids, written over the bucket's records
  uint32_t* segidx;  // [record] segment index inside the bucket
  uint32_t* nseg;    // [bucket] segment count
  uint32_t* long_list;  // (bucket, first record) of segments longer than kLong
  uint32_t* nlong;
  // sort only (no segments): the sorted keys are written over the bucket's
  // keys here, the ids over vals, and the other fields are not used
  uint64_t* keys_out = nullptr;
};

// Loads the (key, id) records of a bucket of n <= kCap records starting at
// lo into the lane's slots (position wave*span + r*64 + lane); a larger
// bucket loads nothing.
__device__ __forceinline__ void load_bucket(const uint64_t* __restrict__ keys,
                                            const uint32_t* vals, uint32_t lo, uint32_t n,
                                            uint64_t (&k)[kSortRounds],
                                            uint32_t (&v)[kSortRounds]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool fits = n <= static_cast<uint32_t>(kCap);
  const uint32_t span = sort_span(n);
  const int rounds = fits ? static_cast<int>(span / 64) : 0;
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    k[r] = 0;
    v[r] = 0;
    if (r >= rounds) continue;
    const uint32_t q = wave * span + r * 64 + lane;
    if (q < n) {
      k[r] = keys[lo + q];
      v[r] = vals[lo + q];
    }
  }
}

// Segments of a sorted bucket (the p-th record at S.key / S.id [at(p)],
// at = S.perm with PERM, else the identity): writes the sorted pair ids, the
// segment index of every record, the bucket's segment count and the long
// segments.
template <bool PERM>
__device__ void bucket_segments(uint32_t b, uint32_t lo, uint32_t n, SortSmem& S,
                                const SegOut& out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t span = sort_span(n);
  const int rounds = static_cast<int>(span / 64);
  if (out.keys_out) {
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
      if (r >= rounds) break;
      const uint32_t q = wave * span + r * 64 + lane;
      if (q < n) {
        const uint32_t at = PERM ? S.perm[q] : q;
        out.keys_out[lo + q] = S.key[at];
        out.vals[lo + q] = S.id[at];
      }
    }
    return;
  }
  // segment heads (a key differing from the one before), counted per wave
  uint64_t hb[kSortRounds];
  uint32_t hc = 0;
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    hb[r] = 0;
    if (r >= rounds) break;
    const uint32_t q = wave * span + r * 64 + lane;
    bool head = false;
    if (q < n) head = q == 0 || S.key[PERM ? S.perm[q - 1] : q - 1] != S.key[PERM ? S.perm[q] : q];
    hb[r] = __ballot(head);
    hc += static_cast<uint32_t>(__popcll(hb[r]));
  }
  if (lane == 0) S.wcount[wave] = hc;
  __syncthreads();
  uint32_t run = 0, total = 0;
  for (int w = 0; w < kSortWaves; ++w) {
    if (w < wave) run += S.wcount[w];
    total += S.wcount[w];
  }
  const uint64_t lt = (1ull << lane) - 1ull;
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    if (r >= rounds) break;
    const uint32_t q = wave * span + r * 64 + lane;
    if (q < n) {
      const uint32_t seg = run + static_cast<uint32_t>(__popcll(hb[r] & (lt | (1ull << lane)))) - 1;
      const uint32_t at = PERM ? S.perm[q] : q;
      out.vals[lo + q] = S.id[at];
      out.segidx[lo + q] = seg;
      if ((hb[r] >> lane) & 1) {
        // segments longer than kLong: queued for the block-wide reduction
        const uint64_t kq = S.key[at];
        const uint32_t lim = q + kLong + 1 < n ? q + kLong + 1 : n;
        uint32_t e = q + 1;
        while (e < lim && S.key[PERM ? S.perm[e] : e] == kq) ++e;
        if (e - q > static_cast<uint32_t>(kLong)) {
          const uint32_t slot = atomicAdd(out.nlong, 1u);
          out.long_list[2 * slot] = b;
          out.long_list[2 * slot + 1] = q;
        }
      }
    }
    run += static_cast<uint32_t>(__popcll(hb[r]));
  }
  if (threadIdx.x == 0) out.nseg[b] = total;
}

// Buckets that fit in LDS, counting sort.  Each block (kSortBlocksPerCU per
// compute unit) takes the buckets blockIdx.x, blockIdx.x + gridDim.x, ...; once a bucket
// is scattered into bins, the block loads the records of its next bucket,
// so that the loads overlap the rest of the work.  A bucket over kCap
// records is queued for k_heavy_sort, one with a bin of more than kMaxBin
// records (many equal keys) for k_bucket_radix.
__global__ void __launch_bounds__(kSortNT)
k_bucket_count(const uint64_t* keys, const uint32_t* __restrict__ boff,
               uint32_t nbk, SortField f0, SortBatch sb, SegOut out, uint32_t* __restrict__ heavy,
               uint32_t* __restrict__ nheavy, uint32_t* __restrict__ redo,
               uint32_t* __restrict__ nredo) {
  __shared__ SortSmem S;
  uint64_t k[kSortRounds];
  uint32_t v[kSortRounds];
  uint32_t b = blockIdx.x, lo = 0, n = 0;
  if (b < nbk) {
    lo = boff[b];
    n = boff[b + 1] - lo;
    load_bucket(keys, out.vals, lo, n, k, v);
  }
  for (; b < nbk; b += gridDim.x) {
    const SortField f = sort_field(sb, b, f0);
    const bool fits = n <= static_cast<uint32_t>(kCap);
    const int cs = fits ? count_scatter(n, f.locnt, k, v, S) : 0;
    const bool ok = cs != 0;
    // every load of this bucket has been used: the wait is free, and it
    // keeps the compiler from waiting for the next bucket's loads when it
    // reuses their registers
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    const uint32_t b2 = b + gridDim.x;
    uint32_t lo2 = 0, n2 = 0;
    if (b2 < nbk) {
      lo2 = boff[b2];
      n2 = boff[b2 + 1] - lo2;
    }
    load_bucket(keys, out.vals, lo2, n2, k, v);
    if (ok) {
      count_order(n, f.locnt, S, cs == 2);
      bucket_segments<true>(b, lo, n, S, out);
    } else if (threadIdx.x == 0) {
      if (fits) redo[atomicAdd(nredo, 1u)] = b;
      else heavy[atomicAdd(nheavy, 1u)] = b;
    }
    lo = lo2;
    n = n2;
  }
}

// Buckets that fit in LDS, radix sort: the buckets list[0, *nlist), or every
// bucket when list is null.  A bucket over kCap records is queued for
// k_heavy_sort.
__global__ void __launch_bounds__(kSortNT)
k_bucket_radix(const uint64_t* keys, const uint32_t* __restrict__ boff,
               uint32_t nbk, const uint32_t* __restrict__ list,
               const uint32_t* __restrict__ nlist, SortField f0, SortBatch sb, SegOut out,
               uint32_t* __restrict__ heavy, uint32_t* __restrict__ nheavy) {
  __shared__ SortSmem S;
  uint64_t k[kSortRounds];
  uint32_t v[kSortRounds];
  const uint32_t L = list ? *nlist : nbk;
  for (uint32_t x = blockIdx.x; x < L; x += gridDim.x) {
    const uint32_t b = list ? list[x] : x;
    const uint32_t lo = boff[b], n = boff[b + 1] - lo;
    if (n > static_cast<uint32_t>(kCap)) {
      if (threadIdx.x == 0) heavy[atomicAdd(nheavy, 1u)] = b;
      continue;
    }
    load_bucket(keys, out.vals, lo, n, k, v);
    radix_bucket(n, k, v, sort_field(sb, b, f0), S);
    bucket_segments<false>(b, lo, n, S, out);
  }
}

// Buckets larger than kCap: one block sorts the bucket's records on all key
// bits below the bucket bits (LSD, 8-bit digits, global memory, stable) and
// then marks the segments.
__global__ void __launch_bounds__(kSortNT)
k_heavy_sort(uint64_t* __restrict__ keys, uint64_t* __restrict__ tkeys,
             uint32_t* __restrict__ tvals, const uint32_t* __restrict__ boff, int rbits0,
             SortBatch sb, const uint32_t* __restrict__ heavy, const uint32_t* __restrict__ nheavy,
             SegOut out) {
  __shared__ uint32_t s_hist[256], s_start[256], s_run[256];
  __shared__ uint32_t s_wc[kSortWaves][256];
  __shared__ uint32_t sh[kSortWaves];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t lt = (1ull << lane) - 1ull;
  const uint32_t H = *nheavy;
  for (uint32_t hix = blockIdx.x; hix < H; hix += gridDim.x) {
    const uint32_t b = heavy[hix];
    const int rbits = sb.bprod ? sb.sf[sb.bprod[b]].rem : rbits0;
    const uint32_t lo = boff[b], n = boff[b + 1] - lo;
    uint64_t* ka = keys + lo;
    uint32_t* va = out.vals + lo;
    uint64_t* kb = tkeys + lo;
    uint32_t* vb = tvals + lo;
    const int passes = (rbits + 7) / 8;
    for (int pass = 0; pass < passes; ++pass) {
      const int shift = 8 * pass;
      if (tid < 256) {
        s_hist[tid] = 0;
        s_run[tid] = 0;
      }
      for (int i = tid; i < kSortWaves * 256; i += kSortNT) (&s_wc[0][0])[i] = 0;
      __syncthreads();
      for (uint32_t q = tid; q < n; q += kSortNT) atomicAdd(&s_hist[(ka[q] >> shift) & 255], 1u);
      __syncthreads();
      const uint32_t st = block_excl<kSortWaves>(tid < 256 ? s_hist[tid] : 0u, nullptr, sh);
      if (tid < 256) s_start[tid] = st;
      __syncthreads();
      for (uint32_t base = 0; base < n; base += kSortNT) {
        const uint32_t q = base + tid;
        const bool valid = q < n;
        uint64_t k = 0;
        uint32_t v = 0;
        int d = 0;
        if (valid) {
          k = ka[q];
          v = va[q];
          d = static_cast<int>((k >> shift) & 255);
        }
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
          const bool on = valid && ((d >> bit) & 1);
          const uint64_t bm = __ballot(on);
          peers &= on ? bm : ~bm;
        }
        const int rank = __popcll(peers & lt);
        if (valid && rank == 0) s_wc[wave][d] = static_cast<uint32_t>(__popcll(peers));
        __syncthreads();
        if (valid) {
          uint32_t off = s_start[d] + s_run[d];
          for (int w = 0; w < wave; ++w) off += s_wc[w][d];
          kb[off + rank] = k;
          vb[off + rank] = v;
        }
        __syncthreads();
        if (tid < 256) {
          uint32_t add = 0;
          for (int w = 0; w < kSortWaves; ++w) {
            add += s_wc[w][tid];
            s_wc[w][tid] = 0;
          }
          s_run[tid] += add;
        }
        __syncthreads();
      }
      uint64_t* tk = ka; ka = kb; kb = tk;
      uint32_t* tv = va; va = vb; vb = tv;
    }
    if (passes & 1) {  // the sorted records are in the scratch arrays: copy back
      for (uint32_t q = tid; q < n; q += kSortNT) {
        keys[lo + q] = ka[q];
        out.vals[lo + q] = va[q];
      }
      __syncthreads();
    }
    if (out.keys_out) continue;  // sort only
    const uint64_t* K = keys + lo;
    uint32_t run = 0;
    for (uint32_t base = 0; base < n; base += kSortNT) {
      const uint32_t q = base + tid;
      const bool head = q < n && (q == 0 || K[q - 1] != K[q]);
      const uint64_t hb = __ballot(head);
      if (lane == 0) sh[wave] = static_cast<uint32_t>(__popcll(hb));
      __syncthreads();
      uint32_t wb = run, tot = 0;
      for (int w = 0; w < kSortWaves; ++w) {
        if (w < wave) wb += sh[w];
        tot += sh[w];
      }
      if (q < n) {
        out.segidx[lo + q] = wb + static_cast<uint32_t>(__popcll(hb & (lt | (1ull << lane)))) - 1;
        if (head) {
          uint32_t e = q + 1;
          while (e < n && e <= q + kLong && K[e] == K[q]) ++e;
          if (e - q > static_cast<uint32_t>(kLong)) {
            const uint32_t slot = atomicAdd(out.nlong, 1u);
            out.long_list[2 * slot] = b;
            out.long_list[2 * slot + 1] = q;
          }
        }
      }
      run += tot;
      __syncthreads();
    }
    if (tid == 0) out.nseg[b] = run;
    __syncthreads();
  }
}
}  // namespace

}  // namespace pauli
