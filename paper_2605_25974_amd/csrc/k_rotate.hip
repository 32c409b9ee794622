// Rotation steps of a Pauli-propagation loop (Section III-B, eq. (5)).
//
// R = cos(theta) I - i sin(theta) P.
//   product mode:     S <- merge(R * S), the fused outer product of the
//                     2-term sum R with S.
//   conjugation mode: a term Q that commutes with P is kept; an
//                     anticommuting Q becomes cos(theta) Q and
//                     -i sin(theta) P Q.  The 1 or 2 terms per input term are
//                     written by one streaming kernel, then merged.
// Both end with the merge options' truncation.
#include <algorithm>
#include <cmath>
#include <memory>
#include <string>
#include <type_traits>
#include <vector>

#include "common.h"
#include "internal.h"

namespace pauli {

namespace {

constexpr int kBlock = 256;

inline unsigned grid_for(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return static_cast<unsigned>(g);
}

// cnt[t] = 1 + (term t anticommutes with P): the parity of the symplectic
// product (Section III-F), sum over words of |X_t & Z_P| + |Z_t & X_P|.
__global__ void k_rot_count(const uint64_t* __restrict__ X, const uint64_t* __restrict__ Z,
                            int64_t ld, int64_t m, const uint32_t* __restrict__ md, RotString P,
                            uint32_t* __restrict__ cnt) {
  if (md && *md < m) m = *md;  // the device count, clamped to the host bound
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m;
       t += (int64_t)gridDim.x * blockDim.x) {
    int s = 0;
    for (int w = 0; w < P.W; ++w) {
      if ((P.x[w] | P.z[w]) == 0) continue;  // no letter of P in this word: nothing to read
      s += popc64((X[w * ld + t] & P.z[w]) ^ (Z[w * ld + t] & P.x[w]));
    }
    cnt[t] = 1u + static_cast<uint32_t>(s & 1);
  }
}

template <typename T>
__global__ void k_rot_write(const uint64_t* __restrict__ X, const uint64_t* __restrict__ Z,
                            const uint8_t* __restrict__ ph, const cplx<T>* __restrict__ c,
                            const uint64_t* __restrict__ fp, int64_t ld, int64_t m, RotString P,
                            T co, T si, const uint32_t* __restrict__ cnt,
                            const uint32_t* __restrict__ off, uint64_t* __restrict__ OX,
                            uint64_t* __restrict__ OZ, uint8_t* __restrict__ Oph,
                            cplx<T>* __restrict__ Oc, uint64_t* __restrict__ Ofp, int64_t ldo) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o = off[t];
    const bool anti = cnt[t] == 2;
    const cplx<T> v = c[t];
    int k = P.y;  // phase of P * Q (P on the left), Section III-A
    for (int w = 0; w < P.W; ++w) {
      const uint64_t xq = X[w * ld + t], zq = Z[w * ld + t];
      OX[w * ldo + o] = xq;
      OZ[w * ldo + o] = zq;
      if (anti) {
        const uint64_t x3 = P.x[w] ^ xq, z3 = P.z[w] ^ zq;
        k += popc64(xq & zq) + 2 * popc64(P.z[w] & xq) - popc64(x3 & z3);
        OX[w * ldo + o + 1] = x3;
        OZ[w * ldo + o + 1] = z3;
      }
    }
    Oph[o] = ph[t];
    Ofp[o] = fp[t];
    Oc[o] = anti ? cplx<T>{v.re * co, v.im * co} : v;
    if (anti) {
      // -i sin(theta) i^k P Q: the factor -i = i^3 joins the phase exponent
      Oph[o + 1] = static_cast<uint8_t>((ph[t] + k + 3) & 3);
      Oc[o + 1] = cplx<T>{v.re * si, v.im * si};
      Ofp[o + 1] = fp[t] ^ P.fp;
    }
  }
}

// Records of the conjugated sum when the input sum is in key order: the
// kept strings (every input term, in input order, so already sorted) and
// the new strings P Q of the anticommuting terms (compacted, to be sorted).
// Record ids address the conjugated sum without storing it: 2t is input
// term t, 2t + 1 its new term.
__global__ void k_rot_records(const uint64_t* __restrict__ fp, const uint32_t* __restrict__ cnt,
                              const uint32_t* __restrict__ off, int64_t m,
                              const uint32_t* __restrict__ md, uint64_t pfp, int kshift,
                              uint64_t* __restrict__ kk, uint32_t* __restrict__ kv,
                              uint64_t* __restrict__ nk, uint32_t* __restrict__ nv) {
  if (md && *md < m) m = *md;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m;
       t += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t f = fp[t];
    kk[t] = f >> kshift;
    kv[t] = static_cast<uint32_t>(2 * t);
    if (cnt[t] == 2) {
      const uint32_t j = off[t] - static_cast<uint32_t>(t);  // anticommuting terms before t
      nk[j] = (f ^ pfp) >> kshift;
      nv[j] = static_cast<uint32_t>(2 * t + 1);
    }
  }
}

// Merge of two key-ordered record lists a (first on equal keys) and b into
// o: output tile k is outputs [k kMergeOut, (k + 1) kMergeOut); where each
// tile starts in a and b is found first by a co-rank search (merge path),
// one thread per tile boundary (k_merge_splits); a block then stages its
// tile's two input ranges in LDS and merges them there, each thread finding
// its own kMergePer outputs' start the same way inside the block's ranges.
constexpr int kMergePer = 8;
constexpr int kMergeOut = kBlock * kMergePer;

__device__ __forceinline__ int64_t corank(const uint64_t* a, int64_t na, const uint64_t* b,
                                          int64_t nb, int64_t d) {
  // smallest i with a[i] > b[d - 1 - i]: the first d outputs take i from a
  int64_t lo = d - nb > 0 ? d - nb : 0, hi = d < na ? d : na;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (a[mid] <= b[d - 1 - mid]) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// split[k] = how many of the first min(k kMergeOut, |a| + |b|) outputs come
// from a, for k = 0 .. ntiles (every search at once, instead of two threads
// of each merging block waiting on theirs).
__global__ void k_merge_splits(const uint64_t* __restrict__ ak, int64_t na,
                               const uint64_t* __restrict__ bk, int64_t nb,
                               const uint32_t* __restrict__ nad, const uint32_t* __restrict__ nbd,
                               int64_t ntiles, int64_t* __restrict__ split) {
  if (nad && *nad < na) na = *nad;  // device counts, clamped to the host bounds
  if (nbd && *nbd < nb) nb = *nbd;
  const int64_t total = na + nb;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k <= ntiles;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t d = k * kMergeOut < total ? k * kMergeOut : total;
    split[k] = corank(ak, na, bk, nb, d);
  }
}

__global__ void __launch_bounds__(kBlock)
k_merge_path(const uint64_t* __restrict__ ak, const uint32_t* __restrict__ av, int64_t na,
             const uint64_t* __restrict__ bk, const uint32_t* __restrict__ bv, int64_t nb,
             const uint32_t* __restrict__ nad, const uint32_t* __restrict__ nbd,
             const int64_t* __restrict__ split, uint64_t* __restrict__ ok,
             uint32_t* __restrict__ ov) {
  if (nad && *nad < na) na = *nad;  // device counts, clamped to the host bounds
  if (nbd && *nbd < nb) nb = *nbd;
  __shared__ uint64_t sk[kMergeOut];
  __shared__ uint32_t sv[kMergeOut];
  __shared__ uint64_t so_k[kMergeOut];
  __shared__ uint32_t so_v[kMergeOut];
  const int64_t total = na + nb;
  for (int64_t tile = blockIdx.x; tile * kMergeOut < total; tile += gridDim.x) {
    const int64_t d0 = tile * kMergeOut;
    const int64_t d1 = d0 + kMergeOut < total ? d0 + kMergeOut : total;
    const int64_t i0 = split[tile], i1 = split[tile + 1];
    const int64_t j0 = d0 - i0, j1 = d1 - i1;
    const int la = static_cast<int>(i1 - i0), lb = static_cast<int>(j1 - j0);  // la + lb <= kMergeOut
    for (int e = threadIdx.x; e < la + lb; e += kBlock) {
      if (e < la) {
        sk[e] = ak[i0 + e];
        sv[e] = av[i0 + e];
      } else {
        sk[e] = bk[j0 + e - la];
        sv[e] = bv[j0 + e - la];
      }
    }
    __syncthreads();
    // this thread's outputs [e0, e1) of the block's la + lb
    const int e0 = static_cast<int>(threadIdx.x) * kMergePer;
    const int n = la + lb;
    if (e0 < n) {
      const int e1 = e0 + kMergePer < n ? e0 + kMergePer : n;
      const int i = static_cast<int>(corank(sk, la, sk + la, lb, e0));
      int x = i, y = e0 - i;
      for (int e = e0; e < e1; ++e) {
        const bool take_a = y >= lb || (x < la && sk[x] <= sk[la + y]);
        if (take_a) {
          so_k[e] = sk[x];
          so_v[e] = sv[x];
          ++x;
        } else {
          so_k[e] = sk[la + y];
          so_v[e] = sv[la + y];
          ++y;
        }
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n; e += kBlock) {
      ok[d0 + e] = so_k[e];
      ov[d0 + e] = so_v[e];
    }
    __syncthreads();
  }
}

RotString rot_string(int n, const uint64_t* px, const uint64_t* pz) {
  RotString P{};
  P.W = words_for(n);
  P.fp = 0;
  P.y = 0;
  for (int w = 0; w < P.W; ++w) {
    P.x[w] = px[w];
    P.z[w] = pz[w];
    P.y += __builtin_popcountll(px[w] & pz[w]);
    for (int b = 0; b < 64; ++b) {
      if ((px[w] >> b) & 1) P.fp ^= fp_column(2 * (64 * w + b));
      if ((pz[w] >> b) & 1) P.fp ^= fp_column(2 * (64 * w + b) + 1);
    }
  }
  return P;
}

// Every term gives two records: (cos theta) Q_t and (-i sin theta) P Q_t.
__global__ void k_rot_all(int64_t m, const uint32_t* __restrict__ md, uint32_t* __restrict__ cnt) {
  if (md && *md < m) m = *md;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m;
       t += (int64_t)gridDim.x * blockDim.x)
    cnt[t] = 2u;
}

template <typename T>
paulisum* conjugate_stored(const paulisum* s, const RotString& P, double theta,
                           const MergeArgs& o, uint32_t M2, const DBuf& cnt, const DBuf& off,
                           unsigned g, hipStream_t st);

// One rotation step on the records 2t (Q_t, times cos theta where cnt[t] is
// 2) and 2t + 1 (-i sin theta P Q_t, where cnt[t] is 2).  The conjugation
// P-rotation keeps the terms that commute with P as they are (cnt[t] = 1);
// the literal product (cos theta I - i sin theta P) Q_t gives both records
// for every term (all_new).
// sorted_input: s is in key order (a merge's output with the same key bits).
template <typename T>
paulisum* conjugate_t(const paulisum* s, const RotString& P, double theta, const MergeArgs& o,
                      bool sorted_input, bool all_new, hipStream_t st) {
  const int64_t m = s->m;
  DBuf cnt((m + 1) * 4, st), off((m + 1) * 4, st), tot(4, st), work(scan_workspace_bytes(m), st);
  const unsigned g = grid_for(m);
  uint32_t M2 = 0;
  {
    StageScope sc(PAULI_STAGE_PREP, st, m * (16.0 * s->W + 8));
    if (all_new)
      hipLaunchKernelGGL(k_rot_all, dim3(g), dim3(kBlock), 0, st, m, nullptr, cnt.as<uint32_t>());
    else
      hipLaunchKernelGGL(k_rot_count, dim3(g), dim3(kBlock), 0, st, s->X, s->Z, s->ld, m, nullptr,
                         P, cnt.as<uint32_t>());
    scan_exclusive_u32(cnt.as<uint32_t>(), off.as<uint32_t>(), m, tot.as<uint32_t>(), work.p, st);
    PAULI_HIP(hipMemcpyAsync(&M2, tot.p, 4, hipMemcpyDeviceToHost, st));
    PAULI_HIP(hipStreamSynchronize(st));
  }
  if (sorted_input && M2 <= 0x7FFFFFFFu && m <= 0x7FFFFFFFll) {
    // the kept strings are in key order already: sort only the new ones,
    // merge the two lists, and combine straight from the input terms (the
    // conjugated sum is never stored)
    const int64_t na = m, nb = static_cast<int64_t>(M2) - m;
    const int kshift = 64 - o.key_bits;
    DBuf keys(M2 * 8ull, st), vals(M2 * 4ull, st), kk(m * 8, st), kv(m * 4, st);
    DBuf nk(nb * 8 + 8, st), nv(nb * 4 + 4, st), nk2(nb * 8 + 8, st), nv2(nb * 4 + 4, st);
    {
      StageScope sc(PAULI_STAGE_SORT, st, m * 24.0 + nb * 12.0 * 2 + M2 * 36.0);
      hipLaunchKernelGGL(k_rot_records, dim3(g), dim3(kBlock), 0, st, s->fp, cnt.as<uint32_t>(),
                         off.as<uint32_t>(), m, nullptr, P.fp, kshift, kk.as<uint64_t>(),
                         kv.as<uint32_t>(), nk.as<uint64_t>(), nv.as<uint32_t>());
      PAULI_HIP(hipGetLastError());
      uint64_t* bk = nk.as<uint64_t>();
      uint32_t* bv = nv.as<uint32_t>();
      if (nb > 1 && sort_records_bucketed(bk, bv, nk2.as<uint64_t>(), nv2.as<uint32_t>(), nb,
                                          o.key_bits, st)) {
        bk = nk2.as<uint64_t>();
        bv = nv2.as<uint32_t>();
      }
      const int64_t ntiles = (static_cast<int64_t>(M2) + kMergeOut - 1) / kMergeOut;
      DBuf split((ntiles + 1) * 8ull, st);
      hipLaunchKernelGGL(k_merge_splits, dim3(grid_for(ntiles + 1)), dim3(kBlock), 0, st,
                         kk.as<uint64_t>(), na, bk, nb, nullptr, nullptr, ntiles,
                         split.as<int64_t>());
      const int64_t blocks = ntiles < 1 ? 1 : (ntiles > 65536 ? 65536 : ntiles);
      hipLaunchKernelGGL(k_merge_path, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, st,
                         kk.as<uint64_t>(), kv.as<uint32_t>(), na, bk, bv, nb, nullptr, nullptr,
                         split.as<int64_t>(), keys.as<uint64_t>(), vals.as<uint32_t>());
      PAULI_HIP(hipGetLastError());
    }
    return merge_rotated(s, P, theta, cnt.as<uint32_t>(), keys.as<uint64_t>(),
                         vals.as<uint32_t>(), M2, o, st);
  }
  // input in any order: store the conjugated sum and merge it
  if constexpr (std::is_same<T, ff>::value) {
    fail(PAULI_ERR_OVERFLOW, "a float-float state step needs the sorted path (< 2^31 records)");
  } else {
    return conjugate_stored<T>(s, P, theta, o, M2, cnt, off, g, st);
  }
}

template <typename T>
paulisum* conjugate_stored(const paulisum* s, const RotString& P, double theta,
                           const MergeArgs& o, uint32_t M2, const DBuf& cnt, const DBuf& off,
                           unsigned g, hipStream_t st) {
  const int64_t m = s->m;
  paulisum* mat = new_sum(s->n, M2, M2, s->dtype, st);
  paulisum* r = nullptr;
  try {
    {
      StageScope sc(PAULI_STAGE_PREP, st, m * (16.0 * s->W + 25) + M2 * (16.0 * s->W + 25));
      hipLaunchKernelGGL(k_rot_write<T>, dim3(g), dim3(kBlock), 0, st, s->X, s->Z, s->ph,
                         static_cast<const cplx<T>*>(s->coef), s->fp, s->ld, m, P,
                         static_cast<T>(std::cos(theta)), static_cast<T>(std::sin(theta)),
                         cnt.as<uint32_t>(), off.as<uint32_t>(), mat->X, mat->Z, mat->ph,
                         static_cast<cplx<T>*>(mat->coef), mat->fp, mat->ld);
      PAULI_HIP(hipGetLastError());
    }
    r = merge_generic(mat, nullptr, o, st);
  } catch (...) {
    free_sum(mat);
    throw;
  }
  free_sum(mat);
  return r;
}

// The 2-term sum cos(theta) I - i sin(theta) P in the dtype of s.
paulisum* rotation_sum(const paulisum* s, const RotString& P, double theta, hipStream_t st) {
  const int W = s->W;
  paulisum* R = new_sum(s->n, 2, 2, s->dtype, st);
  std::vector<uint64_t> words(4 * W, 0);  // X[w][2], then Z[w][2]
  for (int w = 0; w < W; ++w) {
    words[2 * w + 1] = P.x[w];
    words[2 * W + 2 * w + 1] = P.z[w];
  }
  const uint8_t ph[2] = {0, 0};
  const uint64_t fps[2] = {0, P.fp};
  const double co = std::cos(theta), si = std::sin(theta);
  double c128[4] = {co, 0.0, 0.0, -si};
  float c64[4] = {static_cast<float>(co), 0.0f, 0.0f, static_cast<float>(-si)};
  try {
    // R->ld == 2: word w of term t is X[w * 2 + t]
    PAULI_HIP(hipMemcpyAsync(R->X, words.data(), 2 * W * 8, hipMemcpyHostToDevice, st));
    PAULI_HIP(hipMemcpyAsync(R->Z, words.data() + 2 * W, 2 * W * 8, hipMemcpyHostToDevice, st));
    PAULI_HIP(hipMemcpyAsync(R->ph, ph, 2, hipMemcpyHostToDevice, st));
    PAULI_HIP(hipMemcpyAsync(R->fp, fps, 16, hipMemcpyHostToDevice, st));
    if (s->dtype == PAULI_C128)
      PAULI_HIP(hipMemcpyAsync(R->coef, c128, sizeof(c128), hipMemcpyHostToDevice, st));
    else
      PAULI_HIP(hipMemcpyAsync(R->coef, c64, sizeof(c64), hipMemcpyHostToDevice, st));
    PAULI_HIP(hipStreamSynchronize(st));  // the host staging arrays go out of scope
  } catch (...) {
    free_sum(R);
    throw;
  }
  return R;
}

__global__ void k_clear_u32(uint32_t* __restrict__ p, int n) {
  for (int t = threadIdx.x; t < n; t += blockDim.x) p[t] = 0;
}

// A state count above the bound its step was sized for raises the flag.
__global__ void k_check_bound(const uint32_t* __restrict__ m, int64_t bound,
                              uint32_t* __restrict__ flag) {
  if (static_cast<int64_t>(*m) > bound) atomicOr(flag, 1u);
}

// nb = M2 - m: the new records of a step (both counts on the device; m
// taken at most m_bound, as the step's kernels take it).  More than
// nb_bound new records are cut to nb_bound, M2 with them, and raise the
// capacity flag, so that no later kernel of the step reads past what the
// sort and the merge path wrote.
__global__ void k_new_count(uint32_t* __restrict__ M2, const uint32_t* __restrict__ m,
                            int64_t m_bound, int64_t nb_bound, uint32_t* __restrict__ nb,
                            uint32_t* __restrict__ flag) {
  const int64_t mm = static_cast<int64_t>(*m) < m_bound ? static_cast<int64_t>(*m) : m_bound;
  int64_t n = static_cast<int64_t>(*M2) - mm;  // M2 >= mm: every processed term gives a record
  if (n > nb_bound) {
    if (flag) atomicOr(flag, 1u);
    n = nb_bound;
    *M2 = static_cast<uint32_t>(mm + n);
  }
  *nb = static_cast<uint32_t>(n);
}

// One rotation step in device-count form: the sorted state s holds *md
// terms (at most mb), of which at most nbb give a new string; the merged
// successor goes to dv.into, its count to *dv.U.  The same kernels as the
// host-count steps, every size read on the device (no host
// synchronisation), grids and buffers sized for the bounds.  With nb_seen
// (a measuring run only) the step's count of new strings is read back.
template <typename T>
void conjugate_dev(const paulisum* s, const RotString& P, double theta, const MergeArgs& o,
                   bool all_new, int64_t mb, int64_t nbb, int64_t* nb_seen, const uint32_t* md,
                   const DevRun& dv0, hipStream_t st) {
  if (nbb > mb) nbb = mb;
  const int64_t M2b = mb + nbb;
  DBuf cnt((mb + 1) * 4, st), off((mb + 1) * 4, st), ctr(64, st);
  DBuf work(scan_workspace_bytes(mb), st);
  uint32_t* M2d = ctr.as<uint32_t>();
  uint32_t* nbd = M2d + 1;
  const unsigned g = grid_for(mb);
  if (all_new)
    hipLaunchKernelGGL(k_rot_all, dim3(g), dim3(kBlock), 0, st, mb, md, cnt.as<uint32_t>());
  else
    hipLaunchKernelGGL(k_rot_count, dim3(g), dim3(kBlock), 0, st, s->X, s->Z, s->ld, mb, md, P,
                       cnt.as<uint32_t>());
  scan_exclusive_u32(cnt.as<uint32_t>(), off.as<uint32_t>(), mb, M2d, work.p, st, md);
  hipLaunchKernelGGL(k_new_count, dim3(1), dim3(1), 0, st, M2d, md, mb, nbb, nbd, dv0.flag);
  if (nb_seen) {
    uint32_t h = 0;
    PAULI_HIP(hipMemcpyAsync(&h, nbd, 4, hipMemcpyDeviceToHost, st));
    PAULI_HIP(hipStreamSynchronize(st));
    *nb_seen = h;
  }
  const int kshift = 64 - o.key_bits;
  DBuf keys(M2b * 8ull + 8, st), vals(M2b * 4ull + 4, st), kk(mb * 8 + 8, st), kv(mb * 4 + 4, st);
  DBuf nk(mb * 8 + 8, st), nv(mb * 4 + 4, st), nk2(mb * 8 + 8, st), nv2(mb * 4 + 4, st);
  hipLaunchKernelGGL(k_rot_records, dim3(g), dim3(kBlock), 0, st, s->fp, cnt.as<uint32_t>(),
                     off.as<uint32_t>(), mb, md, P.fp, kshift, kk.as<uint64_t>(), kv.as<uint32_t>(),
                     nk.as<uint64_t>(), nv.as<uint32_t>());
  PAULI_HIP(hipGetLastError());
  uint64_t* bk = nk.as<uint64_t>();
  uint32_t* bv = nv.as<uint32_t>();
  if (nbb > 1 && sort_records_bucketed(bk, bv, nk2.as<uint64_t>(), nv2.as<uint32_t>(), nbb,
                                       o.key_bits, st, nbd)) {
    bk = nk2.as<uint64_t>();
    bv = nv2.as<uint32_t>();
  }
  const int64_t ntiles = (M2b + kMergeOut - 1) / kMergeOut;
  DBuf split((ntiles + 1) * 8ull, st);
  hipLaunchKernelGGL(k_merge_splits, dim3(grid_for(ntiles + 1)), dim3(kBlock), 0, st,
                     kk.as<uint64_t>(), mb, bk, nbb, md, nbd, ntiles, split.as<int64_t>());
  const int64_t blocks = ntiles < 1 ? 1 : (ntiles > 65536 ? 65536 : ntiles);
  hipLaunchKernelGGL(k_merge_path, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, st,
                     kk.as<uint64_t>(), kv.as<uint32_t>(), mb, bk, bv, nbb, md, nbd,
                     split.as<int64_t>(),
                     keys.as<uint64_t>(), vals.as<uint32_t>());
  PAULI_HIP(hipGetLastError());
  DevRun dv = dv0;
  dv.N = M2d;
  merge_rotated(s, P, theta, cnt.as<uint32_t>(), keys.as<uint64_t>(), vals.as<uint32_t>(), M2b, o,
                st, &dv);
}

}  // namespace

// ------------------------------------------------------- propagation plans
//
// The whole loop in device-count form, captured once into a HIP graph: the
// input is merged into state 0, and step t merges the rotated state t % 2
// into state (t + 1) % 2 (the precision form's last step into a C64 state),
// every state an array set of capacity max_terms with its term count on the
// device.  The host bound of step t's state is min(capacity, |s| 2^t) (a
// step at most doubles the terms); a state that would exceed the capacity
// is cut and raises a flag, which the results call turns into CAPACITY.
// The temporaries of a step come from one region, reused by every step.
struct PropPlan {
  const paulisum* in = nullptr;
  int steps = 0;
  std::vector<uint64_t> px, pz;
  std::vector<double> theta;
  int mode = PAULI_ROTATE_CONJUGATE;
  MergeArgs o;
  int64_t cap = 0;
  bool ff = false;
  std::shared_ptr<SharedBlock> blk[3];
  paulisum state[3];
  DBuf counts;  // [0..2] term counts of the states, [3] the capacity flag
  DBuf tmp;
  size_t tmp_bytes = 0;
  hipStream_t home = nullptr, priv = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraphExec_t exec = nullptr;
  int last = 0;  // the state holding the result
  bool ran = false;
  // host bounds of the state entering each step and of the result, and of
  // each step's new strings (from a measuring run of the same sequence;
  // empty: min(capacity, |s| 2^t), and the state's bound)
  std::vector<int64_t> bounds, new_bounds;
  ~PropPlan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (priv && ev_out) {
      (void)hipEventRecord(ev_out, priv);
      (void)hipStreamWaitEvent(home, ev_out, 0);
    }
    counts.reset();
    tmp.reset();
    for (auto& b : blk) b.reset();
    if (priv) {
      (void)hipStreamSynchronize(priv);
      (void)hipStreamDestroy(priv);
    }
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
  }
};

namespace {

void bind_state(PropPlan& pl, int k, int32_t dt) {
  pl.blk[k] = std::make_shared<SharedBlock>(pl.in->W, pl.cap, dt, pl.home);
  paulisum& c = pl.state[k];
  c.n = pl.in->n;
  c.W = pl.in->W;
  c.m = 0;
  c.ld = pl.cap;
  c.dtype = dt;
  c.device = pl.in->device;
  c.X = pl.blk[k]->X;
  c.Z = pl.blk[k]->Z;
  c.ph = pl.blk[k]->ph;
  c.coef = pl.blk[k]->coef;
  c.fp = pl.blk[k]->fp;
  c.last_stream = pl.home;
  c.borrowed = true;
}

int32_t state_dtype(const PropPlan& pl) { return pl.ff ? kDtypeFF : pl.in->dtype; }

// The state count c (device) read back on the host (measuring run only).
int64_t read_count(const uint32_t* c, hipStream_t st) {
  uint32_t h = 0;
  PAULI_HIP(hipMemcpyAsync(&h, c, 4, hipMemcpyDeviceToHost, st));
  PAULI_HIP(hipStreamSynchronize(st));
  return h;
}

// The loop's launch sequence on stream st (no host synchronisation).  With
// `measured`, the sequence runs eagerly and the count of every state is
// read back after it is formed (the plan's measuring run).
void launch_loop(PropPlan& pl, hipStream_t st, std::vector<int64_t>* measured = nullptr,
                 std::vector<int64_t>* measured_new = nullptr) {
  uint32_t* cnt = pl.counts.as<uint32_t>();
  hipLaunchKernelGGL(k_clear_u32, dim3(1), dim3(64), 0, st, cnt, 4);  // counts and flag
  ScratchScope scratch(pl.tmp.p, pl.tmp_bytes);
  // state 0: the merged input, in key order
  MergeArgs m0 = pl.o;
  m0.drop_abs = -1.0;
  if (pl.ff) {
    m0.mode = kModeFF;
    m0.ff_out = 1;
  }
  int cur = 0;
  if (pl.ff && pl.steps == 0) {
    m0.ff_out = 0;  // no step: the merged input is the result, in C64
    cur = 2;
  }
  DevRun dv{nullptr, &pl.state[cur], cnt + cur, cnt + 3};
  merge_generic(pl.in, nullptr, m0, st, &dv);
  if (measured) measured->push_back(read_count(cnt + cur, st));
  MergeArgs ms = pl.o;
  if (pl.ff) ms.mode = kModeFF;
  int64_t bound = pl.in->m;
  for (int t = 0; t < pl.steps; ++t) {
    scratch.rewind();  // the previous step's temporaries are dead (stream order)
    const int nxt = (pl.ff && t + 1 == pl.steps) ? 2 : 1 - cur;
    ms.ff_out = (pl.ff && t + 1 < pl.steps) ? 1 : 0;
    int64_t mb = bound < pl.cap ? bound : pl.cap;
    if (static_cast<size_t>(t) < pl.bounds.size()) mb = pl.bounds[t];
    const RotString P = rot_string(pl.in->n, pl.px.data() + static_cast<size_t>(t) * pl.in->W,
                                   pl.pz.data() + static_cast<size_t>(t) * pl.in->W);
    hipLaunchKernelGGL(k_check_bound, dim3(1), dim3(1), 0, st, cnt + cur, mb, cnt + 3);
    DevRun d{nullptr, &pl.state[nxt], cnt + nxt, cnt + 3};
    const bool all_new = pl.mode == PAULI_ROTATE_PRODUCT;
    int64_t nbb = mb;
    if (static_cast<size_t>(t) < pl.new_bounds.size() && pl.new_bounds[t] < mb)
      nbb = pl.new_bounds[t];
    int64_t seen = 0;
    int64_t* ps = measured_new ? &seen : nullptr;
    if (pl.ff)
      conjugate_dev<ff>(&pl.state[cur], P, pl.theta[t], ms, all_new, mb, nbb, ps, cnt + cur, d,
                        st);
    else if (pl.in->dtype == PAULI_C128)
      conjugate_dev<double>(&pl.state[cur], P, pl.theta[t], ms, all_new, mb, nbb, ps, cnt + cur,
                            d, st);
    else
      conjugate_dev<float>(&pl.state[cur], P, pl.theta[t], ms, all_new, mb, nbb, ps, cnt + cur, d,
                           st);
    if (measured) measured->push_back(read_count(cnt + nxt, st));
    if (measured_new) measured_new->push_back(seen);
    bound = 2 * mb;
    cur = nxt;
  }
  pl.last = cur;
}

void capture_loop(PropPlan& pl) {
  if (pl.exec) {
    PAULI_HIP(hipGraphExecDestroy(pl.exec));
    pl.exec = nullptr;
  }
  NoEvents ne;
  hipGraph_t graph = nullptr;
  PAULI_HIP(hipStreamBeginCapture(pl.priv, hipStreamCaptureModeThreadLocal));
  try {
    launch_loop(pl, pl.priv);
  } catch (...) {
    (void)hipStreamEndCapture(pl.priv, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    throw;
  }
  PAULI_HIP(hipStreamEndCapture(pl.priv, &graph));
  const hipError_t e = hipGraphInstantiate(&pl.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  PAULI_HIP(e);
}

}  // namespace

PropPlan* prop_plan_create(const paulisum* s, int steps, const uint64_t* px, const uint64_t* pz,
                           const double* theta, int mode, const MergeArgs& o, int64_t cap,
                           hipStream_t st) {
  auto pl = std::make_unique<PropPlan>();
  pl->in = s;
  pl->steps = steps;
  pl->px.assign(px, px + static_cast<size_t>(steps) * s->W);
  pl->pz.assign(pz, pz + static_cast<size_t>(steps) * s->W);
  pl->theta.assign(theta, theta + steps);
  pl->mode = mode;
  pl->o = o;
  pl->cap = cap;
  pl->ff = o.mode == PAULI_MERGE_COMPENSATED;
  pl->home = st;
  PAULI_HIP(hipStreamCreateWithFlags(&pl->priv, hipStreamNonBlocking));
  PAULI_HIP(hipEventCreateWithFlags(&pl->ev_in, hipEventDisableTiming));
  PAULI_HIP(hipEventCreateWithFlags(&pl->ev_out, hipEventDisableTiming));
  pl->counts = DBuf(64, st);
  bind_state(*pl, 0, state_dtype(*pl));
  bind_state(*pl, 1, state_dtype(*pl));
  if (pl->ff) bind_state(*pl, 2, PAULI_C64);
  // temporaries of the largest step (about 172 bytes per term of its bound,
  // with room for the alignment of each piece)
  const int64_t mmax = std::max<int64_t>(cap, s->m);
  pl->tmp_bytes = static_cast<size_t>(mmax) * 200 + (size_t(64) << 20);
  pl->tmp = DBuf(pl->tmp_bytes, st);
  PAULI_HIP(hipStreamSynchronize(st));  // the buffers exist before the capture
  // measuring run: the same sequence, eagerly, reading back every state's
  // size and every step's count of new strings; the graph's kernels are
  // then sized for those (with a margin; a count above a bound is cut on
  // the device and raises the flag)
  {
    NoEvents ne;
    std::vector<int64_t> sizes, news;
    launch_loop(*pl, st, &sizes, &news);
    pl->bounds.clear();
    for (size_t k = 0; k < sizes.size(); ++k) {
      const int64_t b = sizes[k] + sizes[k] / 64 + 4096;
      pl->bounds.push_back(b < cap ? b : cap);
    }
    pl->new_bounds.clear();
    for (size_t k = 0; k < news.size(); ++k) {
      const int64_t b = news[k] + news[k] / 64 + 4096;
      pl->new_bounds.push_back(b < cap ? b : cap);
    }
  }
  capture_loop(*pl);
  return pl.release();
}

void prop_plan_run(PropPlan* pl, hipStream_t st) {
  bool fresh = false;
  for (int k = 0; k < (pl->ff ? 3 : 2); ++k)
    if (!pl->blk[k]) {
      bind_state(*pl, k, k == 2 ? PAULI_C64 : state_dtype(*pl));
      fresh = true;
    }
  if (fresh || !pl->exec) capture_loop(*pl);
  PAULI_HIP(hipEventRecord(pl->ev_in, st));
  PAULI_HIP(hipStreamWaitEvent(pl->priv, pl->ev_in, 0));
  if (st != pl->home) {
    PAULI_HIP(hipEventRecord(pl->ev_in, pl->home));
    PAULI_HIP(hipStreamWaitEvent(pl->priv, pl->ev_in, 0));
  }
  PAULI_HIP(hipGraphLaunch(pl->exec, pl->priv));
  PAULI_HIP(hipEventRecord(pl->ev_out, pl->priv));
  PAULI_HIP(hipStreamWaitEvent(st, pl->ev_out, 0));
  pl->ran = true;
}

paulisum* prop_plan_result(PropPlan* pl) {
  if (!pl->ran) fail(PAULI_ERR_INVALID, "the plan has not run since its last result");
  pl->ran = false;
  PAULI_HIP(hipStreamSynchronize(pl->priv));
  uint32_t c[4] = {0, 0, 0, 0};
  PAULI_HIP(hipMemcpy(c, pl->counts.p, sizeof(c), hipMemcpyDeviceToHost));
  if (c[3] != 0)
    fail(PAULI_ERR_CAPACITY, "a propagation state exceeded the plan's capacity of " +
                                 std::to_string(pl->cap) + " terms");
  paulisum* r = sum_view(pl->blk[pl->last], pl->in->n, 0, c[pl->last]);
  pl->blk[pl->last].reset();  // the result owns that block now
  return r;
}

void prop_plan_destroy(PropPlan* pl) { delete pl; }

paulisum* rotate_step(const paulisum* s, const uint64_t* px, const uint64_t* pz, double theta,
                      int mode, const MergeArgs& o, bool sorted_input, hipStream_t st) {
  const RotString P = rot_string(s->n, px, pz);
  if (s->m == 0) return merge_generic(s, nullptr, o, st);  // an empty sum stays empty
  if (s->dtype == kDtypeFF) {
    // the precision form's float-float state, in key order
    if (!sorted_input) fail(PAULI_ERR_INVALID, "a float-float state must be in key order");
    return conjugate_t<ff>(s, P, theta, o, true, mode == PAULI_ROTATE_PRODUCT, st);
  }
  if (mode == PAULI_ROTATE_CONJUGATE) {
    return s->dtype == PAULI_C128 ? conjugate_t<double>(s, P, theta, o, sorted_input, false, st)
                                  : conjugate_t<float>(s, P, theta, o, sorted_input, false, st);
  }
  if (sorted_input) {
    // the product with cos(theta) I - i sin(theta) P: the products I Q_t are
    // the input strings, already in key order, so only the m strings P Q_t
    // are sorted and the two lists merged, as in a conjugation step
    return s->dtype == PAULI_C128 ? conjugate_t<double>(s, P, theta, o, true, true, st)
                                  : conjugate_t<float>(s, P, theta, o, true, true, st);
  }
  paulisum* R = rotation_sum(s, P, theta, st);
  paulisum* r = nullptr;
  try {
    r = fused_bucket(R, s, o, st);
    if (!r) r = merge_generic(R, s, o, st);
  } catch (...) {
    free_sum(R);
    throw;
  }
  free_sum(R);
  return r;
}

}  // namespace pauli
