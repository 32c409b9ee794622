// Sort-and-combine (Section III-H) on the device.
//
//   records   one (key, id) per term: key = the string's 64-bit fingerprint
//             (fp(a_i * b_j) = fp(a_i) ^ fp(b_j) for a pair), id = the term
//             index or the pair index p = j*|a| + i
//   sort      stable LSD radix sort on the key
//   heads     a record starts a segment when its key or its packed string
//             differs from its predecessor's (the strings are compared word
//             by word, so a fingerprint collision can never merge two
//             strings); runs of equal keys that hold several strings are
//             re-ordered by their packed words
//   reduce    per segment, the sum of i^k * c over its records in record
//             order (deterministic: sequential for short segments, a fixed
//             tree for long ones)
//   compact   drop |c| < drop_abs (strict), then write the surviving
//             segments' strings, coefficients and fingerprints
//
// The same pipeline serves a materialised sum (term source) and the fused
// outer product (pair source, no product is ever stored).
#include <algorithm>
#include <cmath>
#include <memory>
#include <optional>
#include <string>
#include <type_traits>

#include "common.h"
#include "internal.h"
#include "sources.h"

namespace pauli {

namespace {

constexpr int kBlock = 256;
constexpr int kLongSeg = 64;  // segments longer than this are reduced by a block

inline unsigned grid_for(int64_t n, int per_block = kBlock) {
  int64_t g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > (1 << 30)) g = 1 << 30;
  return static_cast<unsigned>(g);
}

// --------------------------------------------------------------- kernels

__global__ void k_pair_records(const uint64_t* __restrict__ fa, const uint64_t* __restrict__ fb,
                               uint32_t ma, int64_t P, int kshift, uint64_t* __restrict__ keys,
                               uint32_t* __restrict__ vals) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P;
       p += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t j = static_cast<uint32_t>(p) / ma;
    const uint32_t i = static_cast<uint32_t>(p) - j * ma;
    keys[p] = (fa[i] ^ fb[j]) >> kshift;
    vals[p] = static_cast<uint32_t>(p);
  }
}

__global__ void k_term_records(const uint64_t* __restrict__ f, int64_t m, int kshift,
                               uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m;
       t += (int64_t)gridDim.x * blockDim.x) {
    keys[t] = f[t] >> kshift;
    vals[t] = static_cast<uint32_t>(t);
  }
}

// head[r] in {0, 1}; v[r] = value of record r; *dirty |= 1 when a key run
// holds more than one string.  second_pass: only run if *dirty, and do not
// raise it again.
template <int WT, typename TV, typename Src>
__global__ void __launch_bounds__(kBlock)
k_heads(Src src, const uint64_t* __restrict__ keys, const uint32_t* __restrict__ vals, int64_t N,
        const uint32_t* __restrict__ nd, uint32_t* __restrict__ head, cplx<TV>* __restrict__ v,
        uint32_t* __restrict__ dirty, int second_pass) {
  if (second_pass && *dirty == 0) return;
  if (nd && *nd < N) N = *nd;  // the device count, clamped to the host bound
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < N;
       r += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t id = vals[r];
    v[r] = src.template value<TV>(id);
    uint32_t h = 1;
    if (r > 0 && keys[r] == keys[r - 1]) {  // the strings only where the keys are equal
      if (same_string<WT>(src, id, vals[r - 1]))
        h = 0;
      else if (!second_pass)
        atomicOr(dirty, 1u);
    }
    head[r] = h;
  }
}

// Re-orders every key run that holds several strings by (packed words, id),
// so that equal strings become adjacent.  One thread per run, insertion sort
// in place: runs with fingerprint ties are rare and short.
template <int WT, typename Src>
__global__ void k_fix_runs(Src src, const uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                           const uint32_t* __restrict__ head, int64_t N,
                           const uint32_t* __restrict__ nd, const uint32_t* __restrict__ dirty) {
  if (*dirty == 0) return;
  if (nd && *nd < N) N = *nd;
  uint64_t a[2 * WT], b[2 * WT];
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < N;
       r += (int64_t)gridDim.x * blockDim.x) {
    if (r > 0 && keys[r] == keys[r - 1]) continue;  // not a run start
    int64_t e = r + 1;
    bool mixed = false;
    while (e < N && keys[e] == keys[r]) {
      mixed |= head[e] != 0;
      ++e;
    }
    if (!mixed) continue;
    for (int64_t x = r + 1; x < e; ++x) {
      const uint32_t idx = vals[x];
      src.string(idx, a);
      int64_t y = x - 1;
      while (y >= r) {
        const uint32_t idy = vals[y];
        src.string(idy, b);
        const int c = words_cmp<WT>(b, a, src.nw);
        if (c < 0 || (c == 0 && idy < idx)) break;
        vals[y + 1] = idy;
        --y;
      }
      vals[y + 1] = idx;
    }
  }
}

__global__ void k_seg_starts(const uint32_t* __restrict__ head, const uint32_t* __restrict__ segid,
                             int64_t N, const uint32_t* __restrict__ nd,
                             const uint32_t* __restrict__ nseg, uint32_t* __restrict__ seg_start) {
  if (nd && *nd < N) N = *nd;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < N;
       r += (int64_t)gridDim.x * blockDim.x)
    if (head[r]) seg_start[segid[r]] = static_cast<uint32_t>(r);
  if (blockIdx.x == 0 && threadIdx.x == 0) seg_start[*nseg] = static_cast<uint32_t>(N);
}

__global__ void k_zero_u32(uint32_t* p, int n) {
  for (int t = threadIdx.x; t < n; t += blockDim.x) p[t] = 0;
}

__global__ void k_count_kept(const uint32_t* __restrict__ keep, const uint32_t* __restrict__ outidx,
                             const uint32_t* __restrict__ nseg, uint32_t* __restrict__ nkept) {
  const uint32_t U = *nseg;
  *nkept = U ? outidx[U - 1] + keep[U - 1] : 0u;
}

// drop < 0: every term is kept; otherwise the strict truncation |c| < drop
// of Section III-B, decided exactly.
template <typename T>
__device__ __forceinline__ bool keep_value(cplx<T> c, double drop) {
  if (drop < 0.0) return true;
  return !below_threshold(conv<double>(c.re), conv<double>(c.im), drop);
}

// FP64 value of record r (the re-merge of a cancelled segment).
template <int WT, typename Src>
__device__ __forceinline__ cplx<double> value64(const Src& src, uint32_t id) {
  return src.template value<double>(id);
}

// Short segments: one thread adds its records in order.  In the compensated
// form a cancelled segment is added again in FP64 from the source.
template <int WT, typename TV, int MODE, typename Src>
__global__ void k_seg_reduce(Src src, const uint32_t* __restrict__ vals,
                             const cplx<TV>* __restrict__ v, const uint32_t* __restrict__ seg_start,
                             const uint32_t* __restrict__ nseg, cplx<TV>* __restrict__ coef,
                             uint32_t* __restrict__ keep, uint32_t* __restrict__ long_list,
                             uint32_t* __restrict__ nlong, double drop, double tau) {
  const uint32_t U = *nseg;
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < U;
       u += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t s0 = seg_start[u], s1 = seg_start[u + 1];
    if (s1 - s0 > kLongSeg) {
      long_list[atomicAdd(nlong, 1u)] = static_cast<uint32_t>(u);
      continue;
    }
    Acc<MODE, TV> acc;
    acc.begin(v[s0].re, v[s0].im);
    for (uint32_t r = s0 + 1; r < s1; ++r) acc.add(v[r].re, v[r].im);
    cplx<TV> c{acc.value_re(), acc.value_im()};
    if (MODE == kComp && acc.cancels(tau)) {
      double re = 0.0, im = 0.0;
      for (uint32_t r = s0; r < s1; ++r) {
        const cplx<double> x = value64<WT>(src, vals[r]);
        re = re + x.re;
        im = im + x.im;
      }
      c = cplx<TV>{conv<TV>(re), conv<TV>(im)};
    }
    coef[u] = c;
    keep[u] = keep_value(c, drop) ? 1u : 0u;
  }
}

// Long segments: one block each; thread t adds records t, t+256, ... in
// order, then the 256 partial sums are added in thread order (the same in
// every thread, so the re-merge decision is uniform over the block).
template <int WT, typename TV, int MODE, typename Src>
__global__ void __launch_bounds__(kBlock)
k_seg_reduce_long(Src src, const uint32_t* __restrict__ vals, const cplx<TV>* __restrict__ v,
                  const uint32_t* __restrict__ seg_start, const uint32_t* __restrict__ long_list,
                  const uint32_t* __restrict__ nlong, cplx<TV>* __restrict__ coef,
                  uint32_t* __restrict__ keep, double drop, double tau) {
  __shared__ Acc<MODE, TV> s_acc[kBlock];
  __shared__ double s_re[kBlock], s_im[kBlock];
  const uint32_t L = *nlong;
  for (uint32_t b = blockIdx.x; b < L; b += gridDim.x) {
    const uint32_t u = long_list[b];
    const uint32_t s0 = seg_start[u], s1 = seg_start[u + 1];
    Acc<MODE, TV> acc;
    acc.zero();
    for (uint32_t r = s0 + threadIdx.x; r < s1; r += kBlock) acc.add(v[r].re, v[r].im);
    s_acc[threadIdx.x] = acc;
    __syncthreads();
    Acc<MODE, TV> tot;
    tot.zero();
    for (int h = 0; h < kBlock; ++h) tot.add(s_acc[h]);
    cplx<TV> c{tot.value_re(), tot.value_im()};
    if (MODE == kComp && tot.cancels(tau)) {
      double re = 0.0, im = 0.0;
      for (uint32_t r = s0 + threadIdx.x; r < s1; r += kBlock) {
        const cplx<double> x = value64<WT>(src, vals[r]);
        re = re + x.re;
        im = im + x.im;
      }
      s_re[threadIdx.x] = re;
      s_im[threadIdx.x] = im;
      __syncthreads();
      double tr = 0.0, ti = 0.0;
      for (int h = 0; h < kBlock; ++h) {
        tr = tr + s_re[h];
        ti = ti + s_im[h];
      }
      c = cplx<TV>{conv<TV>(tr), conv<TV>(ti)};
    }
    if (threadIdx.x == 0) {
      coef[u] = c;
      keep[u] = keep_value(c, drop) ? 1u : 0u;
    }
    __syncthreads();
  }
}

template <int WT, typename T, typename TO, typename Src>
__global__ void __launch_bounds__(kBlock)
k_write_output(Src src, const uint32_t* __restrict__ vals, const uint32_t* __restrict__ seg_start,
               const uint32_t* __restrict__ nseg, const uint32_t* __restrict__ keep,
               const uint32_t* __restrict__ outidx, const cplx<T>* __restrict__ coef,
               uint64_t* __restrict__ OX, uint64_t* __restrict__ OZ, uint8_t* __restrict__ Oph,
               cplx<TO>* __restrict__ Oc, uint64_t* __restrict__ Ofp, int64_t ldo) {
  const uint32_t U = *nseg;
  uint64_t w[2 * WT];
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < U;
       u += (int64_t)gridDim.x * blockDim.x) {
    if (!keep[u]) continue;
    const int64_t o = outidx[u];
    if (o >= ldo) continue;  // past a state's capacity (flagged by the caller)
    const uint32_t id = vals[seg_start[u]];
    src.string(id, w);
#pragma unroll
    for (int q = 0; q < WT; ++q) {
      if (WT > 8 && q >= src.nw) break;
      OX[q * ldo + o] = w[q];
      OZ[q * ldo + o] = w[src.nw + q];
    }
    Oph[o] = 0;
    Oc[o] = convc<TO>(coef[u]);
    Ofp[o] = src.fp(id);
  }
}

// -------------------------------------------------------------- pipeline

// presorted: the records are already in key order (equal keys adjacent).
// MODE kFF (record values in float-float) writes a float-float sum when
// o.ff_out is set, else a C64 sum rounded from it.
// A result count cut to a state's capacity; the flag records the cut.
__global__ void k_take_count(const uint32_t* __restrict__ U, uint32_t cap,
                             uint32_t* __restrict__ out, uint32_t* __restrict__ flag) {
  const uint32_t u = *U;
  *out = u < cap ? u : cap;
  if (u > cap) atomicOr(flag, 1u);
}

template <int WT, typename T, int MODE, typename Src>
paulisum* run_pipeline(const Src& src, int n, int64_t N, int32_t dt, uint64_t* keys,
                       uint32_t* vals, const MergeArgs& o, hipStream_t s, bool presorted = false,
                       const DevRun* dv = nullptr) {
  const uint32_t* nd = dv ? dv->N : nullptr;  // device count (N is then its bound)
  // a narrow key makes runs of about N / 2^key_bits records that one thread
  // each puts in string order (k_fix_runs): keep those runs short
  if (o.key_bits < 52 && N > (int64_t(1) << (o.key_bits + 12)))
    fail(PAULI_ERR_INVALID, "key_bits " + std::to_string(o.key_bits) + " is too narrow for " +
                                std::to_string(N) + " records (at most 2^(key_bits + 12))");
  using TV = typename std::conditional<MODE == kComp, float,
                                       typename std::conditional<MODE == kFF, ff, T>::type>::type;
  if (MODE == kComp) dt = PAULI_C64;
  if (MODE == kFF) dt = o.ff_out ? kDtypeFF : PAULI_C64;
  DBuf keys_alt, vals_alt;
  if (!presorted) {
    keys_alt = DBuf(N * sizeof(uint64_t), s);
    vals_alt = DBuf(N * sizeof(uint32_t), s);
    if (sort_records_bucketed(keys, vals, keys_alt.as<uint64_t>(), vals_alt.as<uint32_t>(), N,
                              o.key_bits, s, nd)) {
      keys = keys_alt.as<uint64_t>();
      vals = vals_alt.as<uint32_t>();
    }
  }

  // counters: [0] dirty, [1] segments, [2] kept, [3] long segments
  DBuf ctr_buf(64, s);
  uint32_t* ctr = ctr_buf.as<uint32_t>();
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, ctr, 16);
  DBuf head_buf(N * sizeof(uint32_t), s), segid_buf(N * sizeof(uint32_t), s);
  DBuf v_buf(N * sizeof(cplx<TV>), s);
  uint32_t* head = head_buf.as<uint32_t>();
  uint32_t* segid = segid_buf.as<uint32_t>();
  cplx<TV>* v = v_buf.as<cplx<TV>>();

  const unsigned g = grid_for(N);
  std::optional<StageScope> sc_seg;
  sc_seg.emplace(PAULI_STAGE_SEGMENT, s, N * (12.0 + 4.0 + sizeof(cplx<TV>)));
  hipLaunchKernelGGL((k_heads<WT, TV, Src>), dim3(g), dim3(kBlock), 0, s, src, keys, vals, N, nd,
                     head, v, ctr + 0, 0);
  // the next two return at once unless a key run holds several strings
  // (rare): a grid of a few blocks per compute unit, not one thread per record
  const unsigned gd = g < 2048u ? g : 2048u;
  hipLaunchKernelGGL((k_fix_runs<WT, Src>), dim3(gd), dim3(kBlock), 0, s, src, keys, vals, head, N,
                     nd, ctr + 0);
  hipLaunchKernelGGL((k_heads<WT, TV, Src>), dim3(gd), dim3(kBlock), 0, s, src, keys, vals, N, nd,
                     head, v, ctr + 0, 1);
  PAULI_HIP(hipGetLastError());

  DBuf swork(scan_workspace_bytes(N), s);
  scan_exclusive_u32(head, segid, N, ctr + 1, swork.p, s, nd);
  DBuf seg_buf((N + 1) * sizeof(uint32_t), s);
  uint32_t* seg_start = seg_buf.as<uint32_t>();
  hipLaunchKernelGGL(k_seg_starts, dim3(g), dim3(kBlock), 0, s, head, segid, N, nd, ctr + 1,
                     seg_start);
  head_buf.reset();

  DBuf coef_buf(N * sizeof(cplx<TV>), s);
  cplx<TV>* coef = coef_buf.as<cplx<TV>>();
  uint32_t* keep = segid;  // segid is dead after k_seg_starts
  DBuf long_buf(N * sizeof(uint32_t), s);
  uint32_t* long_list = long_buf.as<uint32_t>();
  const double drop = o.drop_abs < 0.0 ? -1.0 : o.drop_abs;  // threshold, not squared
  hipLaunchKernelGGL((k_seg_reduce<WT, TV, MODE, Src>), dim3(g), dim3(kBlock), 0, s, src, vals, v,
                     seg_start, ctr + 1, coef, keep, long_list, ctr + 3, drop, o.tau);
  hipLaunchKernelGGL((k_seg_reduce_long<WT, TV, MODE, Src>), dim3(1024), dim3(kBlock), 0, s, src,
                     vals, v, seg_start, long_list, ctr + 3, coef, keep, drop, o.tau);
  PAULI_HIP(hipGetLastError());
  sc_seg.reset();
  v_buf.reset();
  long_buf.reset();

  // keep[u] is defined for u < #segments only; entries past it do not
  // affect outidx[u] for u < #segments (an exclusive scan looks backwards).
  DBuf outidx_buf(N * sizeof(uint32_t), s);
  uint32_t* outidx = outidx_buf.as<uint32_t>();
  scan_exclusive_u32(keep, outidx, N, nullptr, swork.p, s, nd);
  hipLaunchKernelGGL(k_count_kept, dim3(1), dim3(1), 0, s, keep, outidx, ctr + 1, ctr + 2);
  if (dv) {
    // no host read: the terms go to the state's arrays, cut to its capacity
    paulisum* out = dv->into;
    hipLaunchKernelGGL(k_take_count, dim3(1), dim3(1), 0, s, ctr + 2,
                       static_cast<uint32_t>(out->ld), dv->U, dv->flag);
    StageScope sc_w(PAULI_STAGE_WRITE, s, 0.0);
    if (out->dtype == PAULI_C64 && MODE == kFF)
      hipLaunchKernelGGL((k_write_output<WT, TV, float, Src>), dim3(g), dim3(kBlock), 0, s, src,
                         vals, seg_start, ctr + 1, keep, outidx, coef, out->X, out->Z, out->ph,
                         static_cast<cplx<float>*>(out->coef), out->fp, out->ld);
    else
      hipLaunchKernelGGL((k_write_output<WT, TV, TV, Src>), dim3(g), dim3(kBlock), 0, s, src,
                         vals, seg_start, ctr + 1, keep, outidx, coef, out->X, out->Z, out->ph,
                         static_cast<cplx<TV>*>(out->coef), out->fp, out->ld);
    PAULI_HIP(hipGetLastError());
    return out;
  }

  uint32_t host_ctr[4];
  PAULI_HIP(hipMemcpyAsync(host_ctr, ctr, sizeof(host_ctr), hipMemcpyDeviceToHost, s));
  PAULI_HIP(hipStreamSynchronize(s));
  const uint32_t nseg = host_ctr[1];
  const int64_t U = host_ctr[2];

  paulisum* out = new_sum(n, U, U, dt, s);
  if (U > 0) {
    StageScope sc_w(PAULI_STAGE_WRITE, s, U * (16.0 * src.nw + coef_bytes(dt) + 1 + 8));
    if (MODE == kFF && !o.ff_out)
      hipLaunchKernelGGL((k_write_output<WT, TV, float, Src>), dim3(grid_for(nseg)), dim3(kBlock),
                         0, s, src, vals, seg_start, ctr + 1, keep, outidx, coef, out->X, out->Z,
                         out->ph, static_cast<cplx<float>*>(out->coef), out->fp, out->ld);
    else
      hipLaunchKernelGGL((k_write_output<WT, TV, TV, Src>), dim3(grid_for(nseg)), dim3(kBlock), 0,
                         s, src, vals, seg_start, ctr + 1, keep, outidx, coef, out->X, out->Z,
                         out->ph, static_cast<cplx<TV>*>(out->coef), out->fp, out->ld);
    PAULI_HIP(hipGetLastError());
  }
  return out;
}

template <int WT, typename T>
paulisum* merge_t(const paulisum* a, const paulisum* b, const MergeArgs& o, hipStream_t s,
                  const DevRun* dv) {
  const int kshift = 64 - o.key_bits;
  if (b == nullptr) {
    const int64_t N = a->m;
    DBuf keys(N * sizeof(uint64_t), s), vals(N * sizeof(uint32_t), s);
    StageScope sc(PAULI_STAGE_PREP, s, N * 20.0);
    hipLaunchKernelGGL(k_term_records, dim3(grid_for(N)), dim3(kBlock), 0, s, a->fp, N, kshift,
                       keys.as<uint64_t>(), vals.as<uint32_t>());
    PAULI_HIP(hipGetLastError());
    TermSrc<WT, T> src{a->X, a->Z, a->ph, static_cast<const cplx<T>*>(a->coef), a->fp, a->ld, a->W};
    if (o.mode == kModeFF)
      return run_pipeline<WT, T, kFF>(src, a->n, N, a->dtype, keys.as<uint64_t>(),
                                       vals.as<uint32_t>(), o, s, false, dv);
    return o.mode == PAULI_MERGE_COMPENSATED
               ? run_pipeline<WT, T, kComp>(src, a->n, N, a->dtype, keys.as<uint64_t>(),
                                            vals.as<uint32_t>(), o, s, false, dv)
               : run_pipeline<WT, T, kPlain>(src, a->n, N, a->dtype, keys.as<uint64_t>(),
                                             vals.as<uint32_t>(), o, s, false, dv);
  }
  const int64_t N = a->m * b->m;
  const int W = a->W;
  DBuf ra(a->m * 2 * W * sizeof(uint64_t), s), ea(a->m, s);
  DBuf rb(b->m * 2 * W * sizeof(uint64_t), s), eb(b->m, s);
  launch_prep_side(a, ra.as<uint64_t>(), ea.as<uint8_t>(), s);
  launch_prep_side(b, rb.as<uint64_t>(), eb.as<uint8_t>(), s);
  DBuf keys(N * sizeof(uint64_t), s), vals(N * sizeof(uint32_t), s);
  StageScope sc(PAULI_STAGE_PREP, s, N * 12.0);
  hipLaunchKernelGGL(k_pair_records, dim3(grid_for(N)), dim3(kBlock), 0, s, a->fp, b->fp,
                     static_cast<uint32_t>(a->m), N, kshift, keys.as<uint64_t>(),
                     vals.as<uint32_t>());
  PAULI_HIP(hipGetLastError());
  PairSrc<WT, T> src{ra.as<uint64_t>(), ea.as<uint8_t>(), static_cast<const cplx<T>*>(a->coef),
                     a->fp, rb.as<uint64_t>(), eb.as<uint8_t>(),
                     static_cast<const cplx<T>*>(b->coef), b->fp, static_cast<uint32_t>(a->m), W};
  return o.mode == PAULI_MERGE_COMPENSATED
             ? run_pipeline<WT, T, kComp>(src, a->n, N, a->dtype, keys.as<uint64_t>(),
                                          vals.as<uint32_t>(), o, s)
             : run_pipeline<WT, T, kPlain>(src, a->n, N, a->dtype, keys.as<uint64_t>(),
                                           vals.as<uint32_t>(), o, s);
}

// merge(a) of a float-float state (the precision form's carried state).
template <int WT>
paulisum* merge_ff_t(const paulisum* a, const MergeArgs& o, hipStream_t s) {
  const int64_t N = a->m;
  DBuf keys(N * sizeof(uint64_t), s), vals(N * sizeof(uint32_t), s);
  StageScope sc(PAULI_STAGE_PREP, s, N * 20.0);
  hipLaunchKernelGGL(k_term_records, dim3(grid_for(N)), dim3(kBlock), 0, s, a->fp, N,
                     64 - o.key_bits, keys.as<uint64_t>(), vals.as<uint32_t>());
  PAULI_HIP(hipGetLastError());
  TermSrc<WT, ff> src{a->X, a->Z, a->ph, static_cast<const cplx<ff>*>(a->coef), a->fp, a->ld, a->W};
  return run_pipeline<WT, ff, kFF>(src, a->n, N, a->dtype, keys.as<uint64_t>(),
                                   vals.as<uint32_t>(), o, s);
}

paulisum* merge_ff(const paulisum* a, const MergeArgs& o, hipStream_t s) {
  switch (a->W) {
    case 1: return merge_ff_t<1>(a, o, s);
    case 2: return merge_ff_t<2>(a, o, s);
    case 3: return merge_ff_t<3>(a, o, s);
    case 4: return merge_ff_t<4>(a, o, s);
    case 5: return merge_ff_t<5>(a, o, s);
    case 6: return merge_ff_t<6>(a, o, s);
    case 7: return merge_ff_t<7>(a, o, s);
    case 8: return merge_ff_t<8>(a, o, s);
    default: return merge_ff_t<kMaxWords>(a, o, s);
  }
}

// merge(a) from records (key, term index) of a that are already in key order.
template <int WT, typename T>
paulisum* merge_sorted_t(const paulisum* a, uint64_t* keys, uint32_t* vals, const MergeArgs& o,
                         hipStream_t s) {
  TermSrc<WT, T> src{a->X, a->Z, a->ph, static_cast<const cplx<T>*>(a->coef), a->fp, a->ld, a->W};
  return o.mode == PAULI_MERGE_COMPENSATED
             ? run_pipeline<WT, T, kComp>(src, a->n, a->m, a->dtype, keys, vals, o, s, true)
             : run_pipeline<WT, T, kPlain>(src, a->n, a->m, a->dtype, keys, vals, o, s, true);
}

template <typename T>
paulisum* merge_sorted_w(const paulisum* a, uint64_t* keys, uint32_t* vals, const MergeArgs& o,
                         hipStream_t s) {
  switch (a->W) {  // the term source reads exactly WT words when WT <= 8
    case 1: return merge_sorted_t<1, T>(a, keys, vals, o, s);
    case 2: return merge_sorted_t<2, T>(a, keys, vals, o, s);
    case 3: return merge_sorted_t<3, T>(a, keys, vals, o, s);
    case 4: return merge_sorted_t<4, T>(a, keys, vals, o, s);
    case 5: return merge_sorted_t<5, T>(a, keys, vals, o, s);
    case 6: return merge_sorted_t<6, T>(a, keys, vals, o, s);
    case 7: return merge_sorted_t<7, T>(a, keys, vals, o, s);
    case 8: return merge_sorted_t<8, T>(a, keys, vals, o, s);
    default: return merge_sorted_t<kMaxWords, T>(a, keys, vals, o, s);
  }
}

template <typename T>
paulisum* merge_w(const paulisum* a, const paulisum* b, const MergeArgs& o, hipStream_t s,
                  const DevRun* dv) {
  switch (a->W) {
    case 1: return merge_t<1, T>(a, b, o, s, dv);
    case 2: return merge_t<2, T>(a, b, o, s, dv);
    case 3: return merge_t<3, T>(a, b, o, s, dv);
    case 4: return merge_t<4, T>(a, b, o, s, dv);
    case 5: return merge_t<5, T>(a, b, o, s, dv);
    case 6: return merge_t<6, T>(a, b, o, s, dv);
    case 7: return merge_t<7, T>(a, b, o, s, dv);
    case 8: return merge_t<8, T>(a, b, o, s, dv);
    default: return merge_t<kMaxWords, T>(a, b, o, s, dv);
  }
}

// Stream compaction of the kept terms in two passes over tiles of kTileC
// terms: the first counts each tile's kept terms, an exclusive scan of the
// counts gives each tile its first output position, and the second pass
// finds the same flags again and copies the kept terms.  Wave w of a block
// owns the tile positions [w*64*kRoundsC, (w+1)*64*kRoundsC) in rounds of 64
// and ranks its kept terms by ballots.  Only the phase bytes (and, for a
// drop, the coefficients) are read twice.  Tile b is [b*kTileC, min(m,
// (b+1)*kTileC)) of one sum, or, given a tile table tb, [tb[2b], tb[2b+1])
// (at most kTileC terms) of a block holding several sums.
constexpr int kCompact = 256;
constexpr int kRoundsC = 16;
constexpr int kTileC = kCompact * kRoundsC;

template <typename T>
__device__ __forceinline__ bool keep_term(const cplx<T>* __restrict__ c,
                                          const uint8_t* __restrict__ ph, int64_t t, double drop,
                                          int marked) {
  return !(marked && ph[t] != 0) && (drop < 0.0 || keep_value(c[t], drop));
}

// Kept terms of the wave's part of tile blockIdx.x.
template <typename T>
__device__ __forceinline__ uint32_t wave_kept(const cplx<T>* __restrict__ c,
                                              const uint8_t* __restrict__ ph, int64_t end,
                                              double drop, int marked, int64_t w0, int lane) {
  uint32_t n = 0;
#pragma unroll 4
  for (int r = 0; r < kRoundsC; ++r) {
    const int64_t t = w0 + r * 64 + lane;
    n += static_cast<uint32_t>(__popcll(__ballot(t < end && keep_term(c, ph, t, drop, marked))));
  }
  return n;
}

// First and end position of this block's tile.
__device__ __forceinline__ void tile_range(const int64_t* __restrict__ tb, int64_t m,
                                           int64_t& base, int64_t& end) {
  if (tb) {
    base = tb[2 * blockIdx.x];
    end = tb[2 * blockIdx.x + 1];
  } else {
    base = blockIdx.x * static_cast<int64_t>(kTileC);
    end = m;
  }
}

template <typename T>
__global__ void __launch_bounds__(kCompact)
k_keep_count(const cplx<T>* __restrict__ c, const uint8_t* __restrict__ ph, int64_t m,
             const int64_t* __restrict__ tb, double drop, int marked,
             uint32_t* __restrict__ bcount) {
  __shared__ uint32_t sw[kCompact / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t base, end;
  tile_range(tb, m, base, end);
  const int64_t w0 = base + wave * (64 * kRoundsC);
  const uint32_t n = wave_kept(c, ph, end, drop, marked, w0, lane);
  if (lane == 0) sw[wave] = n;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
#pragma unroll
    for (int w = 0; w < kCompact / 64; ++w) tot += sw[w];
    bcount[blockIdx.x] = tot;
  }
}

template <typename T>
__global__ void __launch_bounds__(kCompact)
k_compact(const uint64_t* __restrict__ X, const uint64_t* __restrict__ Z,
          const uint8_t* __restrict__ ph, const cplx<T>* __restrict__ c,
          const uint64_t* __restrict__ fp, int W, int64_t m, const int64_t* __restrict__ tb,
          int64_t ld, double drop, int marked, const uint32_t* __restrict__ boff,
          uint64_t* __restrict__ OX, uint64_t* __restrict__ OZ, uint8_t* __restrict__ Oph,
          cplx<T>* __restrict__ Oc, uint64_t* __restrict__ Ofp, int64_t ldo) {
  __shared__ uint32_t sw[kCompact / 64];
  __shared__ uint16_t s_pos[kTileC];  // tile positions of the kept terms, in order
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t base, end;
  tile_range(tb, m, base, end);
  const int64_t w0 = base + wave * (64 * kRoundsC);
  const uint32_t n = wave_kept(c, ph, end, drop, marked, w0, lane);
  if (lane == 0) sw[wave] = n;
  __syncthreads();
  uint32_t o = 0, total = 0;
  for (int w = 0; w < kCompact / 64; ++w) {
    if (w < wave) o += sw[w];
    total += sw[w];
  }
  const uint64_t lt = (1ull << lane) - 1ull;
  for (int r = 0; r < kRoundsC; ++r) {
    const int64_t t = w0 + r * 64 + lane;
    const bool k = t < end && keep_term(c, ph, t, drop, marked);
    const uint64_t bal = __ballot(k);
    if (k) s_pos[o + __popcll(bal & lt)] = static_cast<uint16_t>(t - base);
    o += static_cast<uint32_t>(__popcll(bal));
  }
  __syncthreads();
  // every thread copies kept terms j, j + kCompact, ...: consecutive output
  // positions, and the loads of different terms in flight together
  const int64_t d0 = boff[blockIdx.x];
  for (uint32_t j = threadIdx.x; j < total; j += kCompact) {
    const int64_t t = base + s_pos[j], d = d0 + j;
    uint64_t xv[kMaxWords], zv[kMaxWords];
#pragma unroll
    for (int w = 0; w < kMaxWords; ++w)
      if (w < W) {
        xv[w] = X[w * ld + t];
        zv[w] = Z[w * ld + t];
      }
    const uint8_t p = ph[t];
    const cplx<T> v = c[t];
    const uint64_t f = fp[t];
#pragma unroll
    for (int w = 0; w < kMaxWords; ++w)
      if (w < W) {
        OX[w * ldo + d] = xv[w];
        OZ[w * ldo + d] = zv[w];
      }
    Oph[d] = p;
    Oc[d] = v;
    Ofp[d] = f;
  }
}

template <typename T>
paulisum* drop_t(const paulisum* a, double drop_abs, bool marked, hipStream_t s) {
  const int64_t m = a->m;
  const int64_t nb = (m + kTileC - 1) / kTileC;
  const double drop = drop_abs >= 0.0 ? drop_abs : -1.0;  // threshold, not squared
  DBuf cnt((nb + 1) * 4, s), off((nb + 1) * 4, s), tot(4, s);
  DBuf work(scan_workspace_bytes(nb), s);
  const auto c = static_cast<const cplx<T>*>(a->coef);
  hipLaunchKernelGGL(k_keep_count<T>, dim3(static_cast<unsigned>(nb)), dim3(kCompact), 0, s, c,
                     a->ph, m, nullptr, drop, marked ? 1 : 0, cnt.as<uint32_t>());
  scan_exclusive_u32(cnt.as<uint32_t>(), off.as<uint32_t>(), nb, tot.as<uint32_t>(), work.p, s);
  uint32_t kept = 0;
  PAULI_HIP(hipMemcpyAsync(&kept, tot.p, 4, hipMemcpyDeviceToHost, s));
  PAULI_HIP(hipStreamSynchronize(s));
  paulisum* out = new_sum(a->n, kept, kept, a->dtype, s);
  if (kept > 0)
    hipLaunchKernelGGL(k_compact<T>, dim3(static_cast<unsigned>(nb)), dim3(kCompact), 0, s, a->X,
                       a->Z, a->ph, c, a->fp, a->W, m, nullptr, a->ld, drop, marked ? 1 : 0,
                       off.as<uint32_t>(), out->X, out->Z, out->ph,
                       static_cast<cplx<T>*>(out->coef), out->fp, out->ld);
  PAULI_HIP(hipGetLastError());
  return out;
}

}  // namespace

paulisum* drop_terms(const paulisum* a, double drop_abs, hipStream_t s, bool marked) {
  if (a->m == 0) return new_sum(a->n, 0, 0, a->dtype, s);
  if (a->dtype == PAULI_C128) return drop_t<double>(a, drop_abs, marked, s);
  return drop_t<float>(a, drop_abs, marked, s);
}

namespace {

template <typename T>
std::shared_ptr<SharedBlock> drop_ranges_t(const SharedBlock& in, const std::vector<int64_t>& r0,
                                           const std::vector<int64_t>& rm, double drop_abs,
                                           std::vector<int64_t>& first,
                                           std::vector<int64_t>& kept, hipStream_t s) {
  const size_t nr = r0.size();
  std::vector<int64_t> tiles;   // (first, end) of every tile
  std::vector<size_t> tile0(nr + 1);  // first tile of every range
  for (size_t k = 0; k < nr; ++k) {
    tile0[k] = tiles.size() / 2;
    for (int64_t b = r0[k]; b < r0[k] + rm[k]; b += kTileC) {
      tiles.push_back(b);
      tiles.push_back(std::min<int64_t>(b + kTileC, r0[k] + rm[k]));
    }
  }
  const int64_t nt = static_cast<int64_t>(tiles.size() / 2);
  tile0[nr] = static_cast<size_t>(nt);
  first.assign(nr, 0);
  kept.assign(nr, 0);
  if (nt == 0) return std::make_shared<SharedBlock>(in.W, 0, in.dtype, s);
  const double drop = drop_abs >= 0.0 ? drop_abs : -1.0;  // threshold, not squared
  DBuf tb(static_cast<size_t>(nt) * 16, s), cnt((nt + 1) * 4, s), off((nt + 1) * 4, s),
      tot(4, s), work(scan_workspace_bytes(nt), s);
  PAULI_HIP(hipMemcpyAsync(tb.p, tiles.data(), tb.bytes, hipMemcpyHostToDevice, s));
  const auto c = static_cast<const cplx<T>*>(in.coef);
  hipLaunchKernelGGL(k_keep_count<T>, dim3(static_cast<unsigned>(nt)), dim3(kCompact), 0, s, c,
                     in.ph, int64_t{0}, tb.as<int64_t>(), drop, 0, cnt.as<uint32_t>());
  scan_exclusive_u32(cnt.as<uint32_t>(), off.as<uint32_t>(), nt, tot.as<uint32_t>(), work.p, s);
  std::vector<uint32_t> offs(static_cast<size_t>(nt) + 1);
  PAULI_HIP(hipMemcpyAsync(offs.data(), off.p, 4 * nt, hipMemcpyDeviceToHost, s));
  PAULI_HIP(hipMemcpyAsync(offs.data() + nt, tot.p, 4, hipMemcpyDeviceToHost, s));
  PAULI_HIP(hipStreamSynchronize(s));
  for (size_t k = 0; k < nr; ++k) {
    first[k] = offs[tile0[k]];
    kept[k] = static_cast<int64_t>(offs[tile0[k + 1]]) - first[k];
  }
  const int64_t total = offs[static_cast<size_t>(nt)];
  auto out = std::make_shared<SharedBlock>(in.W, total, in.dtype, s);
  if (total > 0)
    hipLaunchKernelGGL(k_compact<T>, dim3(static_cast<unsigned>(nt)), dim3(kCompact), 0, s, in.X,
                       in.Z, in.ph, c, in.fp, in.W, int64_t{0}, tb.as<int64_t>(), in.ld, drop, 0,
                       off.as<uint32_t>(), out->X, out->Z, out->ph,
                       static_cast<cplx<T>*>(out->coef), out->fp, out->ld);
  PAULI_HIP(hipGetLastError());
  return out;
}

}  // namespace

std::shared_ptr<SharedBlock> drop_ranges(const SharedBlock& in, const std::vector<int64_t>& r0,
                                         const std::vector<int64_t>& rm, double drop_abs,
                                         std::vector<int64_t>& first, std::vector<int64_t>& kept,
                                         hipStream_t s) {
  if (r0.size() != rm.size()) fail(PAULI_ERR_INVALID, "range lists of different lengths");
  for (size_t k = 0; k < r0.size(); ++k)
    if (r0[k] < 0 || rm[k] < 0 || r0[k] + rm[k] > in.ld)
      fail(PAULI_ERR_INVALID, "a range outside the block");
  if (in.dtype == PAULI_C128)
    return drop_ranges_t<double>(in, r0, rm, drop_abs, first, kept, s);
  if (in.dtype == PAULI_C64) return drop_ranges_t<float>(in, r0, rm, drop_abs, first, kept, s);
  fail(PAULI_ERR_INVALID, "a block of stored coefficients is complex128 or complex64");
}

namespace {

template <int WT, typename T>
paulisum* merge_rotated_t(const paulisum* a, const RotString& P, double theta,
                          const uint32_t* cnt, uint64_t* keys, uint32_t* vals, int64_t N,
                          const MergeArgs& o, hipStream_t s, const DevRun* dv) {
  RotSrc<WT, T> src{};
  src.X = a->X;
  src.Z = a->Z;
  src.ph = a->ph;
  src.c = static_cast<const cplx<T>*>(a->coef);
  src.f = a->fp;
  src.cnt = cnt;
  src.ld = a->ld;
  src.nw = a->W;
  src.py = P.y;
  src.pfp = P.fp;
  src.smask = 0;
  for (int q = 0; q < WT; ++q) {
    src.px[q] = q < a->W ? P.x[q] : 0ull;
    src.pz[q] = q < a->W ? P.z[q] : 0ull;
    if (src.px[q] | src.pz[q]) src.smask |= 1u << q;
  }
  src.co = RotScale::of(std::cos(theta));
  src.si = RotScale::of(std::sin(theta));
  // a float-float state (the precision form) merges in float-float; a
  // stored FP64 or FP32 state in its own precision
  if constexpr (std::is_same<T, ff>::value)
    return run_pipeline<WT, T, kFF>(src, a->n, N, a->dtype, keys, vals, o, s, true, dv);
  else
    return run_pipeline<WT, T, kPlain>(src, a->n, N, a->dtype, keys, vals, o, s, true, dv);
}

template <typename T>
paulisum* merge_rotated_w(const paulisum* a, const RotString& P, double theta,
                          const uint32_t* cnt, uint64_t* keys, uint32_t* vals, int64_t N,
                          const MergeArgs& o, hipStream_t s, const DevRun* dv) {
  switch (a->W) {  // the source reads exactly WT words when WT <= 8
    case 1: return merge_rotated_t<1, T>(a, P, theta, cnt, keys, vals, N, o, s, dv);
    case 2: return merge_rotated_t<2, T>(a, P, theta, cnt, keys, vals, N, o, s, dv);
    case 3: return merge_rotated_t<3, T>(a, P, theta, cnt, keys, vals, N, o, s, dv);
    case 4: return merge_rotated_t<4, T>(a, P, theta, cnt, keys, vals, N, o, s, dv);
    case 5: return merge_rotated_t<5, T>(a, P, theta, cnt, keys, vals, N, o, s, dv);
    case 6: return merge_rotated_t<6, T>(a, P, theta, cnt, keys, vals, N, o, s, dv);
    case 7: return merge_rotated_t<7, T>(a, P, theta, cnt, keys, vals, N, o, s, dv);
    case 8: return merge_rotated_t<8, T>(a, P, theta, cnt, keys, vals, N, o, s, dv);
    default: return merge_rotated_t<kMaxWords, T>(a, P, theta, cnt, keys, vals, N, o, s, dv);
  }
}

}  // namespace

namespace {

// Anticommuting pairs of a commutator, found before any sorting
// (Section III-F: two strings anticommute when their symplectic product is
// odd).  Tile (ti, tj) holds the left terms i = 64 ti + lane, whose words a
// lane keeps in registers, and the right terms j = 64 tj + r, r < 64, whose
// rows the block stages in LDS; wave w tests j = 64 tj + 16 w + c, c < 16.
// Each wave writes the pair ids p = j * ma + i it finds, in (j, i) order,
// into its own 1024 slots, and their number into wcount.
constexpr int kCommTile = 64;
constexpr int kCommSlots = kCommTile * kCommTile / 4;

template <int WT>
__global__ void __launch_bounds__(256)
k_comm_tiles(const uint64_t* __restrict__ ra, const uint64_t* __restrict__ rb, int nw,
             uint32_t ma, uint32_t mb, uint32_t nti, uint32_t* __restrict__ slots,
             uint32_t* __restrict__ wcount) {
  __shared__ uint64_t sb[kCommTile][2 * WT];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t ti = blockIdx.x % nti, tj = blockIdx.x / nti;
  const int rw = 2 * nw;
  for (int k = threadIdx.x; k < kCommTile * rw; k += blockDim.x) {
    const int r = k / rw, q = k - r * rw;
    const uint32_t j = tj * kCommTile + r;
    sb[r][q] = j < mb ? rb[static_cast<size_t>(j) * rw + q] : 0ull;
  }
  const uint32_t i = ti * kCommTile + lane;
  const bool vi = i < ma;
  uint64_t xa[WT], za[WT];
#pragma unroll
  for (int q = 0; q < WT; ++q) {
    const bool ld = vi && (WT <= 8 || q < nw);
    xa[q] = ld ? ra[static_cast<size_t>(i) * rw + q] : 0ull;
    za[q] = ld ? ra[static_cast<size_t>(i) * rw + nw + q] : 0ull;
  }
  __syncthreads();
  const uint64_t lt = (1ull << lane) - 1ull;
  uint32_t* out = slots + (static_cast<size_t>(blockIdx.x) * 4 + wave) * kCommSlots;
  uint32_t n = 0;
#pragma unroll 1
  for (int c = 0; c < kCommTile / 4; ++c) {
    const int r = wave * (kCommTile / 4) + c;
    const uint32_t j = tj * kCommTile + r;
    if (j >= mb) break;
    uint64_t acc = 0;
#pragma unroll
    for (int q = 0; q < WT; ++q)
      if (WT <= 8 || q < nw) acc ^= (xa[q] & sb[r][nw + q]) ^ (za[q] & sb[r][q]);
    const bool anti = vi && (popc64(acc) & 1);
    const uint64_t bal = __ballot(anti);
    if (anti) out[n + __popcll(bal & lt)] = j * ma + i;
    n += static_cast<uint32_t>(__popcll(bal));
  }
  if (lane == 0) wcount[blockIdx.x * 4 + wave] = n;
}

// Records (key, pair id) of the anticommuting pairs, in tile and wave order:
// one wave per slot group copies its ids to their compacted positions.
__global__ void __launch_bounds__(64)
k_comm_records(const uint32_t* __restrict__ slots, const uint32_t* __restrict__ wcount,
               const uint32_t* __restrict__ woff, const uint64_t* __restrict__ fa,
               const uint64_t* __restrict__ fb, uint32_t ma, int kshift,
               uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  const uint32_t g = blockIdx.x, n = wcount[g], o = woff[g];
  const uint32_t* src = slots + static_cast<size_t>(g) * kCommSlots;
  for (uint32_t k = threadIdx.x; k < n; k += 64) {
    const uint32_t p = src[k];
    const uint32_t j = p / ma, i = p - j * ma;
    keys[o + k] = (fa[i] ^ fb[j]) >> kshift;
    vals[o + k] = p;
  }
}

template <int WT, typename T>
paulisum* commutator_filtered_t(const paulisum* a, const paulisum* b, const MergeArgs& o,
                                double max_frac, hipStream_t s) {
  const int W = a->W;
  const uint32_t ma = static_cast<uint32_t>(a->m), mb = static_cast<uint32_t>(b->m);
  const uint32_t nti = (ma + kCommTile - 1) / kCommTile, ntj = (mb + kCommTile - 1) / kCommTile;
  const int64_t ntiles = static_cast<int64_t>(nti) * ntj, ngroups = ntiles * 4;
  DBuf ra(a->m * 2 * W * sizeof(uint64_t), s), ea(a->m, s);
  DBuf rb(b->m * 2 * W * sizeof(uint64_t), s), eb(b->m, s);
  DBuf slots(static_cast<size_t>(ngroups) * kCommSlots * 4, s);
  DBuf wcount(ngroups * 4 + 4, s), woff(ngroups * 4 + 4, s), tot(4, s);
  DBuf work(scan_workspace_bytes(ngroups), s);
  uint32_t K = 0;
  {
    StageScope sc(PAULI_STAGE_PREP, s, (a->m + b->m) * (16.0 * W) * 2);
    launch_prep_side(a, ra.as<uint64_t>(), ea.as<uint8_t>(), s);
    launch_prep_side(b, rb.as<uint64_t>(), eb.as<uint8_t>(), s);
  }
  {
    // per pair: an AND, an AND and two XORs on W word pairs (8W 32-bit
    // operations) and a 64-bit popcount (2)
    StageScope sc(PAULI_STAGE_FILTER, s, static_cast<double>(ma) * mb * (8.0 * W + 2.0));
    hipLaunchKernelGGL((k_comm_tiles<WT>), dim3(static_cast<unsigned>(ntiles)), dim3(256), 0, s,
                       ra.as<uint64_t>(), rb.as<uint64_t>(), W, ma, mb, nti,
                       slots.as<uint32_t>(), wcount.as<uint32_t>());
    PAULI_HIP(hipGetLastError());
  }
  {
    StageScope sc(PAULI_STAGE_PREP, s, ngroups * 8.0);
    scan_exclusive_u32(wcount.as<uint32_t>(), woff.as<uint32_t>(), ngroups, tot.as<uint32_t>(),
                       work.p, s);
    PAULI_HIP(hipMemcpyAsync(&K, tot.p, 4, hipMemcpyDeviceToHost, s));
    PAULI_HIP(hipStreamSynchronize(s));
  }
  if (static_cast<double>(K) > max_frac * static_cast<double>(a->m) * static_cast<double>(b->m))
    return nullptr;
  if (K == 0)
    return new_sum(a->n, 0, 0, o.mode == PAULI_MERGE_COMPENSATED ? PAULI_C64 : a->dtype, s);
  DBuf keys(K * 8ull, s), vals(K * 4ull, s);
  {
    StageScope sc(PAULI_STAGE_PREP, s, K * 16.0);
    hipLaunchKernelGGL(k_comm_records, dim3(static_cast<unsigned>(ngroups)), dim3(64), 0, s,
                       slots.as<uint32_t>(), wcount.as<uint32_t>(), woff.as<uint32_t>(), a->fp,
                       b->fp, ma, 64 - o.key_bits, keys.as<uint64_t>(), vals.as<uint32_t>());
    PAULI_HIP(hipGetLastError());
  }
  slots.reset();
  PairSrc<WT, T> src{ra.as<uint64_t>(), ea.as<uint8_t>(), static_cast<const cplx<T>*>(a->coef),
                     a->fp, rb.as<uint64_t>(), eb.as<uint8_t>(),
                     static_cast<const cplx<T>*>(b->coef), b->fp, ma, W, 1};
  return o.mode == PAULI_MERGE_COMPENSATED
             ? run_pipeline<WT, T, kComp>(src, a->n, K, a->dtype, keys.as<uint64_t>(),
                                          vals.as<uint32_t>(), o, s)
             : run_pipeline<WT, T, kPlain>(src, a->n, K, a->dtype, keys.as<uint64_t>(),
                                           vals.as<uint32_t>(), o, s);
}

template <typename T>
paulisum* commutator_filtered_w(const paulisum* a, const paulisum* b, const MergeArgs& o,
                                double max_frac, hipStream_t s) {
  switch (a->W) {  // the pair source reads exactly WT words when WT <= 8
    case 1: return commutator_filtered_t<1, T>(a, b, o, max_frac, s);
    case 2: return commutator_filtered_t<2, T>(a, b, o, max_frac, s);
    case 3: return commutator_filtered_t<3, T>(a, b, o, max_frac, s);
    case 4: return commutator_filtered_t<4, T>(a, b, o, max_frac, s);
    case 5: return commutator_filtered_t<5, T>(a, b, o, max_frac, s);
    case 6: return commutator_filtered_t<6, T>(a, b, o, max_frac, s);
    case 7: return commutator_filtered_t<7, T>(a, b, o, max_frac, s);
    case 8: return commutator_filtered_t<8, T>(a, b, o, max_frac, s);
    default: return commutator_filtered_t<kMaxWords, T>(a, b, o, max_frac, s);
  }
}

}  // namespace

paulisum* commutator_filtered(const paulisum* a, const paulisum* b, const MergeArgs& o,
                              double max_frac, hipStream_t s) {
  if (a->dtype == PAULI_C128) return commutator_filtered_w<double>(a, b, o, max_frac, s);
  return commutator_filtered_w<float>(a, b, o, max_frac, s);
}

paulisum* merge_rotated(const paulisum* s, const RotString& P, double theta,
                        const uint32_t* cnt, uint64_t* keys, uint32_t* vals, int64_t N,
                        const MergeArgs& o, hipStream_t st, const DevRun* dv) {
  if (s->dtype == kDtypeFF) {
    if (o.mode != kModeFF) fail(PAULI_ERR_INVALID, "a float-float state needs its own merge mode");
    if (N == 0 && !dv) return new_sum(s->n, 0, 0, o.ff_out ? kDtypeFF : PAULI_C64, st);
    return merge_rotated_w<ff>(s, P, theta, cnt, keys, vals, N, o, st, dv);
  }
  if (o.mode != PAULI_MERGE_PLAIN)
    fail(PAULI_ERR_INVALID, "a rotation step on a stored FP64/FP32 state merges in its precision");
  if (N == 0 && !dv) return new_sum(s->n, 0, 0, s->dtype, st);
  if (s->dtype == PAULI_C128)
    return merge_rotated_w<double>(s, P, theta, cnt, keys, vals, N, o, st, dv);
  return merge_rotated_w<float>(s, P, theta, cnt, keys, vals, N, o, st, dv);
}

paulisum* merge_sorted_records(const paulisum* a, uint64_t* keys, uint32_t* vals,
                               const MergeArgs& o, hipStream_t s) {
  if (a->m == 0) return new_sum(a->n, 0, 0, o.mode == PAULI_MERGE_COMPENSATED ? PAULI_C64 : a->dtype, s);
  if (a->dtype == PAULI_C128) return merge_sorted_w<double>(a, keys, vals, o, s);
  return merge_sorted_w<float>(a, keys, vals, o, s);
}

paulisum* merge_generic(const paulisum* a, const paulisum* b, const MergeArgs& o, hipStream_t s,
                        const DevRun* dv) {
  if (a->dtype == kDtypeFF) {
    if (b != nullptr || o.mode != kModeFF || dv)
      fail(PAULI_ERR_INVALID, "a float-float state is only merged on its own");
    return merge_ff(a, o, s);
  }
  if (o.mode == kModeFF && b != nullptr)
    fail(PAULI_ERR_INVALID, "the float-float merge takes one stored sum");
  if (dv && b != nullptr) fail(PAULI_ERR_INVALID, "a merge into a state takes one stored sum");
  if (a->dtype == PAULI_C128) return merge_w<double>(a, b, o, s, dv);
  return merge_w<float>(a, b, o, s, dv);
}

}  // namespace pauli
