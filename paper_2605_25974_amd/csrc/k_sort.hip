// Device-wide exclusive scan and a stable LSD radix sort of (64-bit key,
// 32-bit value) records.  The sort is the "sort an index array by a
// fixed-width key" step of sort-and-combine (Section III-H), done as radix
// passes of 8-bit digits: per-tile digit counts, one scan of the counts,
// then a stable in-tile rank (wave ballots) and a coalesced scatter through
// LDS.
#include "common.h"
#include "internal.h"

namespace pauli {

namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanBlock * kScanItems;

constexpr int kRsBlock = 256;
constexpr int kRsItems = 16;
constexpr int kRsTile = kRsBlock * kRsItems;
constexpr int kRsWaves = kRsBlock / 64;

// Inclusive scan across one wave64.
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}

// Exclusive scan across a block of kScanBlock threads; *total gets the sum.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* total) {
  __shared__ T s_w[kScanBlock / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T inc = wave_inclusive_scan(v);
  if (lane == 63) s_w[wave] = inc;
  __syncthreads();
  T base = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kScanBlock / 64; ++w) {
    if (w < wave) base += s_w[w];
    all += s_w[w];
  }
  __syncthreads();
  if (total) *total = all;
  return base + inc - v;
}

__global__ void __launch_bounds__(kScanBlock)
k_scan_reduce(const uint32_t* __restrict__ in, int64_t n, const uint32_t* __restrict__ nd,
              uint32_t* __restrict__ partial) {
  if (nd && *nd < n) n = *nd;  // the count on the device, clamped to the host bound
  const int64_t base = blockIdx.x * (int64_t)kScanTile;
  uint32_t s = 0;
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    int64_t i = base + r * kScanBlock + threadIdx.x;
    if (i < n) s += in[i];
  }
  uint32_t tot;
  block_exclusive_scan<uint32_t>(s, &tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kScanBlock)
k_scan_partials(uint32_t* __restrict__ partial, int64_t nb, uint32_t* __restrict__ total) {
  uint32_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += kScanBlock) {
    int64_t b = b0 + threadIdx.x;
    uint32_t v = b < nb ? partial[b] : 0;
    uint32_t tot;
    uint32_t ex = block_exclusive_scan<uint32_t>(v, &tot);
    if (b < nb) partial[b] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

// A thread's kScanItems consecutive elements from `base`: as 16-byte loads
// when they all lie below n and the arrays are 16-byte aligned (a wave's
// loads then touch each line kScanItems / 4 times instead of kScanItems),
// else one by one.
__device__ __forceinline__ bool scan_vec(const uint32_t* in, const uint32_t* out, int64_t base,
                                         int64_t n) {
  return base + kScanItems <= n &&
         ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
}

__device__ __forceinline__ void scan_load(const uint32_t* in, int64_t base, int64_t n, bool vec,
                                          uint32_t (&v)[kScanItems]) {
  if (vec) {
    const uint4* p = reinterpret_cast<const uint4*>(in + base);
#pragma unroll
    for (int k = 0; k < kScanItems / 4; ++k) {
      const uint4 q = p[k];
      v[4 * k] = q.x;
      v[4 * k + 1] = q.y;
      v[4 * k + 2] = q.z;
      v[4 * k + 3] = q.w;
    }
  } else {
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) v[r] = base + r < n ? in[base + r] : 0u;
  }
}

// Writes the exclusive prefix run, run + v[0], ... of the thread's elements.
__device__ __forceinline__ void scan_store(uint32_t* out, int64_t base, int64_t n, bool vec,
                                           uint32_t run, const uint32_t (&v)[kScanItems]) {
  uint32_t o[kScanItems];
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    o[r] = run;
    run += v[r];
  }
  if (vec) {
    uint4* p = reinterpret_cast<uint4*>(out + base);
#pragma unroll
    for (int k = 0; k < kScanItems / 4; ++k)
      p[k] = make_uint4(o[4 * k], o[4 * k + 1], o[4 * k + 2], o[4 * k + 3]);
  } else {
#pragma unroll
    for (int r = 0; r < kScanItems; ++r)
      if (base + r < n) out[base + r] = o[r];
  }
}

__global__ void __launch_bounds__(kScanBlock)
k_scan_down(const uint32_t* in, uint32_t* out, int64_t n, const uint32_t* __restrict__ nd,
            const uint32_t* __restrict__ partial) {
  if (nd && *nd < n) n = *nd;
  const int64_t base = blockIdx.x * (int64_t)kScanTile + threadIdx.x * kScanItems;
  const bool vec = scan_vec(in, out, base, n);
  uint32_t v[kScanItems];
  scan_load(in, base, n, vec, v);
  uint32_t s = 0;
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) s += v[r];
  const uint32_t run = partial[blockIdx.x] + block_exclusive_scan<uint32_t>(s, nullptr);
  scan_store(out, base, n, vec, run, v);
}

// A scan of at most kScanTile elements in one launch (the three passes of
// the general scan in one block); in may equal out, and total may point
// just past out.
__global__ void __launch_bounds__(kScanBlock)
k_scan_one(const uint32_t* in, uint32_t* out, int64_t n, const uint32_t* __restrict__ nd,
           uint32_t* total) {
  if (nd && *nd < n) n = *nd;
  const int64_t base = threadIdx.x * static_cast<int64_t>(kScanItems);
  const bool vec = scan_vec(in, out, base, n);
  uint32_t v[kScanItems];
  scan_load(in, base, n, vec, v);
  uint32_t s = 0;
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) s += v[r];
  uint32_t tot;
  const uint32_t run = block_exclusive_scan<uint32_t>(s, &tot);
  scan_store(out, base, n, vec, run, v);
  if (threadIdx.x == 0 && total) *total = tot;
}

// ----------------------------------------------------------------- radix

__global__ void __launch_bounds__(kRsBlock)
k_rs_count(const uint64_t* __restrict__ keys, int64_t n, const uint32_t* __restrict__ nd, int shift,
           uint32_t* __restrict__ counts, int64_t ntiles) {
  __shared__ uint32_t hist[256];
  if (nd && *nd < n) n = *nd;  // tiles past the device count write zero counts
  hist[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = blockIdx.x * (int64_t)kRsTile;
#pragma unroll
  for (int r = 0; r < kRsItems; ++r) {
    int64_t i = base + r * kRsBlock + threadIdx.x;
    if (i < n) atomicAdd(&hist[(keys[i] >> shift) & 255], 1u);
  }
  __syncthreads();
  counts[threadIdx.x * ntiles + blockIdx.x] = hist[threadIdx.x];
}

// Stable scatter of one tile.  Each wave takes a contiguous quarter of the
// tile and visits it in rounds of 64 consecutive records; in a round the
// lanes holding the same digit are found with eight ballots, and the rank of
// a record among the equal digits of its wave is (the wave's count of that
// digit so far) + (earlier lanes of the round).  The wave counts are kept in
// LDS, read by all peers before the first peer adds the round's number (LDS
// operations of one wave take effect in program order).  One scan over the
// digits then gives each wave's offset per digit, the wave order being the
// input order, so the place of a record in the tile is its input order among
// equal digits.  Records are placed in LDS grouped by digit, then written
// out in LDS order so that each digit's run is stored contiguously.
__global__ void __launch_bounds__(kRsBlock)
k_rs_scatter(const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
             uint64_t* __restrict__ kout, uint32_t* __restrict__ vout, int64_t n,
             const uint32_t* __restrict__ nd, int shift, const uint32_t* __restrict__ offsets,
             int64_t ntiles) {
  if (nd && *nd < n) n = *nd;
  __shared__ uint64_t s_k[kRsTile];
  __shared__ uint32_t s_v[kRsTile];
  __shared__ uint32_t s_start[256], s_goff[256];
  __shared__ uint32_t s_wc[kRsWaves][256];  // wave counts, then wave offsets
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t base = blockIdx.x * (int64_t)kRsTile;
  const int64_t wbase = base + static_cast<int64_t>(wave) * (kRsItems * 64);
#pragma unroll
  for (int w = 0; w < kRsWaves; ++w) s_wc[w][tid] = 0;
  s_goff[tid] = offsets[tid * ntiles + blockIdx.x];
  __syncthreads();

  uint64_t k[kRsItems];
  uint32_t v[kRsItems];
  uint32_t rk[kRsItems];
#pragma unroll
  for (int r = 0; r < kRsItems; ++r) {
    const int64_t i = wbase + r * 64 + lane;
    k[r] = i < n ? kin[i] : 0ull;
    v[r] = i < n ? vin[i] : 0u;
  }
  const uint64_t lt = (1ull << lane) - 1ull;
#pragma unroll
  for (int r = 0; r < kRsItems; ++r) {
    const bool valid = wbase + r * 64 + lane < n;
    const int d = static_cast<int>((k[r] >> shift) & 255);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1;
      const uint64_t bm = __ballot(bit);
      peers &= bit ? bm : ~bm;
    }
    const uint32_t rank = static_cast<uint32_t>(__popcll(peers & lt));
    const uint32_t before = valid ? s_wc[wave][d] : 0u;
    if (valid && rank == 0) s_wc[wave][d] = before + static_cast<uint32_t>(__popcll(peers));
    rk[r] = before + rank;
  }
  __syncthreads();
  {  // thread tid is digit tid: the tile's start of the digit and each wave's offset
    uint32_t c[kRsWaves];
    uint32_t tot = 0;
#pragma unroll
    for (int w = 0; w < kRsWaves; ++w) {
      c[w] = s_wc[w][tid];
      tot += c[w];
    }
    uint32_t run = block_exclusive_scan<uint32_t>(tot, nullptr);
    s_start[tid] = run;
#pragma unroll
    for (int w = 0; w < kRsWaves; ++w) {
      s_wc[w][tid] = run;
      run += c[w];
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRsItems; ++r) {
    if (wbase + r * 64 + lane < n) {
      const int d = static_cast<int>((k[r] >> shift) & 255);
      const uint32_t off = s_wc[wave][d] + rk[r];
      s_k[off] = k[r];
      s_v[off] = v[r];
    }
  }
  __syncthreads();

  const int64_t cnt = (n - base) < kRsTile ? (n - base) : kRsTile;
  for (int e = tid; e < cnt; e += kRsBlock) {
    const uint64_t kk = s_k[e];
    const int dd = static_cast<int>((kk >> shift) & 255);
    const int64_t g = static_cast<int64_t>(s_goff[dd]) + (e - static_cast<int64_t>(s_start[dd]));
    kout[g] = kk;
    vout[g] = s_v[e];
  }
}

}  // namespace

size_t scan_workspace_bytes(int64_t n) {
  int64_t nb = (n + kScanTile - 1) / kScanTile;
  return static_cast<size_t>(nb + 1) * sizeof(uint32_t) + 256;
}

void scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total,
                        void* work, hipStream_t s, const uint32_t* nd) {
  if (n <= kScanTile) {  // one block: one launch instead of three
    hipLaunchKernelGGL(k_scan_one, dim3(1), dim3(kScanBlock), 0, s, in, out, n, nd, total);
    PAULI_HIP(hipGetLastError());
    return;
  }
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  uint32_t* partial = static_cast<uint32_t*>(work);
  if (n > 0)
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, n, nd,
                       partial);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanBlock), 0, s, partial, nb, total);
  if (n > 0)
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, out, n, nd,
                       partial);
  PAULI_HIP(hipGetLastError());
}

size_t radix_workspace_bytes(int64_t n) {
  int64_t ntiles = (n + kRsTile - 1) / kRsTile;
  if (ntiles < 1) ntiles = 1;
  size_t counts = static_cast<size_t>(256 * ntiles + 1) * sizeof(uint32_t);
  counts = (counts + 255) & ~size_t(255);
  return counts + scan_workspace_bytes(256 * ntiles);
}

bool radix_sort_at(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
                   int64_t n, const int* shifts, int nshifts, void* work, hipStream_t s,
                   const uint32_t* nd) {
  if (n <= 1) return false;
  int64_t ntiles = (n + kRsTile - 1) / kRsTile;
  uint32_t* counts = static_cast<uint32_t*>(work);
  size_t cbytes = (static_cast<size_t>(256 * ntiles + 1) * sizeof(uint32_t) + 255) & ~size_t(255);
  void* scan_work = static_cast<char*>(work) + cbytes;
  bool alt = false;
  for (int k = 0; k < nshifts; ++k) {
    const int shift = shifts[k];
    const uint64_t* kin = alt ? keys_alt : keys;
    const uint32_t* vin = alt ? vals_alt : vals;
    uint64_t* kout = alt ? keys : keys_alt;
    uint32_t* vout = alt ? vals : vals_alt;
    // one pass reads the keys for the counts, then reads and writes the
    // 12-byte records
    StageScope sc(PAULI_STAGE_SORT, s, 32.0 * n);
    hipLaunchKernelGGL(k_rs_count, dim3((unsigned)ntiles), dim3(kRsBlock), 0, s, kin, n, nd,
                       shift, counts, ntiles);
    PAULI_HIP(hipGetLastError());
    scan_exclusive_u32(counts, counts, 256 * ntiles, nullptr, scan_work, s);
    hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)ntiles), dim3(kRsBlock), 0, s, kin, vin,
                       kout, vout, n, nd, shift, counts, ntiles);
    PAULI_HIP(hipGetLastError());
    alt = !alt;
  }
  return alt;
}

bool radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
                      int64_t n, int key_bits, void* work, hipStream_t s, uint64_t vary,
                      const uint32_t* nd) {
  if (n <= 1 || key_bits <= 0) return false;
  int shifts[8];
  int ns = 0;
  for (int shift = 0; shift < key_bits; shift += 8)
    if (((vary >> shift) & 0xFFull) != 0) shifts[ns++] = shift;  // else the same digit in every key
  return radix_sort_at(keys, vals, keys_alt, vals_alt, n, shifts, ns, work, s, nd);
}

}  // namespace pauli
