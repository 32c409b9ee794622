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
#include <cmath>
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
                            int64_t ld, int64_t m, RotString P, uint32_t* __restrict__ cnt) {
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
                              const uint32_t* __restrict__ off, int64_t m, uint64_t pfp,
                              int kshift, uint64_t* __restrict__ kk, uint32_t* __restrict__ kv,
                              uint64_t* __restrict__ nk, uint32_t* __restrict__ nv) {
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
// o: each block takes kMergeOut consecutive outputs, finds where they start
// in a and b by a co-rank search (merge path), stages both input ranges in
// LDS and merges them there; each thread then finds its own kMergePer
// outputs' start the same way inside the block's ranges.
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

__global__ void __launch_bounds__(kBlock)
k_merge_path(const uint64_t* __restrict__ ak, const uint32_t* __restrict__ av, int64_t na,
             const uint64_t* __restrict__ bk, const uint32_t* __restrict__ bv, int64_t nb,
             uint64_t* __restrict__ ok, uint32_t* __restrict__ ov) {
  __shared__ uint64_t sk[kMergeOut];
  __shared__ uint32_t sv[kMergeOut];
  __shared__ uint64_t so_k[kMergeOut];
  __shared__ uint32_t so_v[kMergeOut];
  __shared__ int64_t s_split[2];
  const int64_t total = na + nb;
  for (int64_t d0 = static_cast<int64_t>(blockIdx.x) * kMergeOut; d0 < total;
       d0 += static_cast<int64_t>(gridDim.x) * kMergeOut) {
    const int64_t d1 = d0 + kMergeOut < total ? d0 + kMergeOut : total;
    if (threadIdx.x == 0) s_split[0] = corank(ak, na, bk, nb, d0);
    if (threadIdx.x == 1) s_split[1] = corank(ak, na, bk, nb, d1);
    __syncthreads();
    const int64_t i0 = s_split[0], i1 = s_split[1];
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
__global__ void k_rot_all(int64_t m, uint32_t* __restrict__ cnt) {
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
      hipLaunchKernelGGL(k_rot_all, dim3(g), dim3(kBlock), 0, st, m, cnt.as<uint32_t>());
    else
      hipLaunchKernelGGL(k_rot_count, dim3(g), dim3(kBlock), 0, st, s->X, s->Z, s->ld, m, P,
                         cnt.as<uint32_t>());
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
                         off.as<uint32_t>(), m, P.fp, kshift, kk.as<uint64_t>(),
                         kv.as<uint32_t>(), nk.as<uint64_t>(), nv.as<uint32_t>());
      PAULI_HIP(hipGetLastError());
      uint64_t* bk = nk.as<uint64_t>();
      uint32_t* bv = nv.as<uint32_t>();
      if (nb > 1 && sort_records_bucketed(bk, bv, nk2.as<uint64_t>(), nv2.as<uint32_t>(), nb,
                                          o.key_bits, st)) {
        bk = nk2.as<uint64_t>();
        bv = nv2.as<uint32_t>();
      }
      int64_t blocks = (static_cast<int64_t>(M2) + kMergeOut - 1) / kMergeOut;
      if (blocks > 65536) blocks = 65536;
      if (blocks < 1) blocks = 1;
      hipLaunchKernelGGL(k_merge_path, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, st,
                         kk.as<uint64_t>(), kv.as<uint32_t>(), na, bk, bv, nb,
                         keys.as<uint64_t>(), vals.as<uint32_t>());
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

}  // namespace

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
