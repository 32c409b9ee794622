// Record sources of the sort-and-combine kernels: how a record id maps to
// its packed string, its value i^k * c and its fingerprint.
#pragma once

#include <type_traits>

#include "common.h"

namespace pauli {


// A product a_i * b_j addressed by p = j*ma + i.
template <int WT, typename T>
struct PairSrc {
  const uint64_t* ra;
  const uint8_t* ea;
  const cplx<T>* ca;
  const uint64_t* fa;
  const uint64_t* rb;
  const uint8_t* eb;
  const cplx<T>* cb;
  const uint64_t* fb;
  uint32_t ma;
  int nw;
  int doubled = 0;  // 1: the value is 2 a_i b_j (a commutator's anticommuting pair)

  __device__ __forceinline__ void split(uint32_t id, uint32_t& i, uint32_t& j) const {
    j = id / ma;
    i = id - j * ma;
  }
  __device__ __forceinline__ void string(uint32_t id, uint64_t* w) const {
    uint32_t i, j;
    split(id, i, j);
    const uint64_t* A = ra + (size_t)i * 2 * nw;
    const uint64_t* B = rb + (size_t)j * 2 * nw;
#pragma unroll
    for (int q = 0; q < 2 * WT; ++q) {
      if (WT > 8 && q >= 2 * nw) break;
      w[q] = A[q] ^ B[q];
    }
  }
  // Product string (into w) and value i^k * c_a * c_b, computed in TV from
  // the coefficients rounded to TV.
  template <typename TV = T>
  __device__ __forceinline__ cplx<TV> term(uint32_t id, uint64_t* w) const {
    uint32_t i, j;
    split(id, i, j);
    const uint64_t* A = ra + (size_t)i * 2 * nw;
    const uint64_t* B = rb + (size_t)j * 2 * nw;
    int acc = ea[i] + eb[j];
#pragma unroll
    for (int q = 0; q < WT; ++q) {
      if (WT > 8 && q >= nw) break;
      const uint64_t xa = A[q], za = A[nw + q], xb = B[q], zb = B[nw + q];
      const uint64_t x = xa ^ xb, z = za ^ zb;
      acc += 2 * popc64(za & xb) - popc64(x & z);
      w[q] = x;
      w[nw + q] = z;
    }
    const cplx<T> a = ca[i], b = cb[j];
    const cplx<TV> v = rot_ik(acc, cmul(cplx<TV>{static_cast<TV>(a.re), static_cast<TV>(a.im)},
                                        cplx<TV>{static_cast<TV>(b.re), static_cast<TV>(b.im)}));
    return doubled ? cplx<TV>{v.re + v.re, v.im + v.im} : v;
  }
  // The value alone (the phase needs the words of both operands).
  template <typename TV = T>
  __device__ __forceinline__ cplx<TV> value(uint32_t id) const {
    uint64_t w[2 * WT];
    return term<TV>(id, w);
  }
  __device__ __forceinline__ uint64_t fp(uint32_t id) const {
    uint32_t i, j;
    split(id, i, j);
    return fa[i] ^ fb[j];
  }
  __device__ __forceinline__ uint64_t xword(uint32_t id, int q) const { return word(id, q); }
  __device__ __forceinline__ uint64_t zword(uint32_t id, int q) const { return word(id, nw + q); }
  // Word t of the product string (X words first, then Z words).
  __device__ __forceinline__ uint64_t word(uint32_t id, int t) const {
    uint32_t i, j;
    split(id, i, j);
    return ra[(size_t)i * 2 * nw + t] ^ rb[(size_t)j * 2 * nw + t];
  }
};

// Term t of a stored sum.
template <int WT, typename T>
struct TermSrc {
  const uint64_t* X;
  const uint64_t* Z;
  const uint8_t* ph;
  const cplx<T>* c;
  const uint64_t* f;
  int64_t ld;
  int nw;

  __device__ __forceinline__ void string(uint32_t id, uint64_t* w) const {
#pragma unroll
    for (int q = 0; q < WT; ++q) {
      if (WT > 8 && q >= nw) break;
      w[q] = X[q * ld + id];
      w[nw + q] = Z[q * ld + id];
    }
  }
  template <typename TV = T>
  __device__ __forceinline__ cplx<TV> term(uint32_t id, uint64_t* w) const {
    string(id, w);
    return rot_ik(ph[id], convc<TV>(c[id]));
  }
  template <typename TV = T>
  __device__ __forceinline__ cplx<TV> value(uint32_t id) const {
    return rot_ik(ph[id], convc<TV>(c[id]));
  }
  __device__ __forceinline__ uint64_t xword(uint32_t id, int q) const { return X[q * ld + id]; }
  __device__ __forceinline__ uint64_t zword(uint32_t id, int q) const { return Z[q * ld + id]; }
  __device__ __forceinline__ uint64_t fp(uint32_t id) const { return f[id]; }
};

// A real factor (cos theta or sin theta) in every precision a rotation
// step uses.
struct RotScale {
  double d;
  float f;
  ff x;  // the double as float-float
  static RotScale of(double v) {
    RotScale r;
    r.d = v;
    r.f = static_cast<float>(v);
    r.x.hi = r.f;
    r.x.lo = static_cast<float>(v - static_cast<double>(r.f));
    return r;
  }
};

// c * factor in the state's own precision: FP64, FP32 (a C64 state in the
// plain form) or float-float (the precision form's carried state).
__device__ __forceinline__ double scale_in(double c, const RotScale& k) { return c * k.d; }
__device__ __forceinline__ float scale_in(float c, const RotScale& k) { return c * k.f; }
__device__ __forceinline__ ff scale_in(ff c, const RotScale& k) { return ff_mul(c, k.x); }

// c * factor as a TV value.  In the state's precision when TV is it; an FP64
// value (the re-merge of a cancelled segment) is formed in FP64 from the
// state's value and the FP64 factor.
template <typename TV, typename T>
__device__ __forceinline__ cplx<TV> scaled(cplx<T> c, const RotScale& k) {
  if constexpr (std::is_same<TV, double>::value && !std::is_same<T, double>::value) {
    return {conv<double>(c.re) * k.d, conv<double>(c.im) * k.d};
  } else {
    return convc<TV>(cplx<T>{scale_in(c.re, k), scale_in(c.im, k)});
  }
}

// The conjugated sum of a rotation step (Section III-B, eq. (5)), not
// stored: record 2t is input term t, its coefficient times cos(theta) when
// Q_t anticommutes with P (cnt[t] == 2); record 2t + 1 is the new term
// -i sin(theta) P Q_t of an anticommuting Q_t, with the phase of the product
// P Q_t (Section III-A) and the fingerprint fp(P) ^ fp(Q_t).  The values are
// formed in the state's precision T and then converted, as a stored copy of
// them would be; FP64 values of a float-float state are formed in FP64.
template <int WT, typename T>
struct RotSrc {
  const uint64_t* X;
  const uint64_t* Z;
  const uint8_t* ph;
  const cplx<T>* c;
  const uint64_t* f;
  const uint32_t* cnt;
  int64_t ld;
  int nw;
  int py;
  uint64_t pfp;
  RotScale co, si;
  uint32_t smask;  // bit q: P has a letter in word q
  uint64_t px[WT], pz[WT];

  __device__ __forceinline__ void string(uint32_t id, uint64_t* w) const {
    const uint32_t t = id >> 1;
    const uint64_t nm = (id & 1u) ? ~0ull : 0ull;
#pragma unroll
    for (int q = 0; q < WT; ++q) {
      if (WT > 8 && q >= nw) break;
      w[q] = X[q * ld + t] ^ (px[q] & nm);
      w[nw + q] = Z[q * ld + t] ^ (pz[q] & nm);
    }
  }
  // The value alone: a word where P has no letter adds nothing to the phase
  // of P Q_t (its two popcounts cancel), so only P's words are read.
  template <typename TV = T>
  __device__ __forceinline__ cplx<TV> value(uint32_t id) const {
    const uint32_t t = id >> 1;
    const cplx<T> v = c[t];
    if ((id & 1u) == 0)
      return rot_ik(ph[t], cnt[t] == 2 ? scaled<TV>(v, co) : convc<TV>(v));
    int k = py;
#pragma unroll
    for (int q = 0; q < WT; ++q) {
      if (WT > 8 && q >= nw) break;
      if (((smask >> q) & 1u) == 0) continue;
      const uint64_t xq = X[q * ld + t], zq = Z[q * ld + t];
      const uint64_t x3 = px[q] ^ xq, z3 = pz[q] ^ zq;
      k += popc64(xq & zq) + 2 * popc64(pz[q] & xq) - popc64(x3 & z3);
    }
    return rot_ik((ph[t] + k + 3) & 3, scaled<TV>(v, si));
  }
  __device__ __forceinline__ uint64_t xword(uint32_t id, int q) const {
    return X[q * ld + (id >> 1)] ^ ((id & 1u) ? px[q] : 0ull);
  }
  __device__ __forceinline__ uint64_t zword(uint32_t id, int q) const {
    return Z[q * ld + (id >> 1)] ^ ((id & 1u) ? pz[q] : 0ull);
  }
  __device__ __forceinline__ uint64_t fp(uint32_t id) const {
    return f[id >> 1] ^ ((id & 1u) ? pfp : 0ull);
  }
};

template <int WT>
__device__ __forceinline__ bool words_equal(const uint64_t* a, const uint64_t* b, int nw) {
  uint64_t d = 0;
#pragma unroll
  for (int q = 0; q < 2 * WT; ++q) {
    if (WT > 8 && q >= 2 * nw) break;
    d |= a[q] ^ b[q];
  }
  return d == 0;
}

// Whether records a and b have the same string, one word pair at a time.
template <int WT, typename Src>
__device__ __forceinline__ bool same_string(const Src& src, uint32_t a, uint32_t b) {
  uint64_t d = 0;
#pragma unroll 2
  for (int q = 0; q < WT; ++q) {
    if (WT > 8 && q >= src.nw) break;
    d |= (src.xword(a, q) ^ src.xword(b, q)) | (src.zword(a, q) ^ src.zword(b, q));
  }
  return d == 0;
}

// Packed-word order used to break fingerprint ties: X words from the most
// significant word down, then Z words likewise.
template <int WT>
__device__ __forceinline__ int words_cmp(const uint64_t* a, const uint64_t* b, int nw) {
  for (int q = nw - 1; q >= 0; --q)
    if (a[q] != b[q]) return a[q] < b[q] ? -1 : 1;
  for (int q = nw - 1; q >= 0; --q)
    if (a[nw + q] != b[nw + q]) return a[nw + q] < b[nw + q] ? -1 : 1;
  return 0;
}


}  // namespace pauli
