// Device-side building blocks shared by the kernels of the Pauli-sum library.
//
// Representation (Section III-C, Table I): a string on n qubits is W =
// ceil(n/64) X words and W Z words; qubit q is bit q % 64 of word q / 64.
// On the device a sum is stored struct-of-arrays (Section III-G / IV-A):
// X[w][ld], Z[w][ld], phase[ld], coef[ld], fp[ld].
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pauli {

constexpr int kMaxWords = 16;  // n <= 1024

// ---------------------------------------------------------------- bit ops

__device__ __forceinline__ int popc64(uint64_t v) { return __popcll(v); }

// ------------------------------------------------------------ fingerprint
//
// fp(P) is a GF(2)-linear 64-bit function of the 2n symplectic bits: the XOR
// of one fixed pseudo-random column per set bit.  Linearity gives
// fp(P*Q) = fp(P) ^ fp(Q) (the product XORs the bits, Section III-E), so the
// key of a product is two loads and one XOR.  Column b (b = 2q for the X bit
// of qubit q, 2q + 1 for its Z bit) is the counter-based SplitMix64 output
// (Steele, Lea and Flood 2014) for counter b + 1 under a fixed seed.
constexpr uint64_t kFpSeed = 0x5041554C49420001ull;
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

__host__ __device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + counter * kGolden;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__host__ __device__ __forceinline__ uint64_t fp_column(int bit_index) {
  return splitmix64_at(kFpSeed, static_cast<uint64_t>(bit_index) + 1);
}

// ------------------------------------------------------------ complex math
//
// The library is compiled with floating-point contraction off, so these
// products round exactly like the operation-by-operation formula.

template <typename T>
struct cplx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

// i^k * v, exact.
template <typename T>
__device__ __forceinline__ cplx<T> rot_ik(int k, cplx<T> v) {
  switch (k & 3) {
    case 0: return v;
    case 1: return {-v.im, v.re};
    case 2: return {-v.re, -v.im};
    default: return {v.im, -v.re};
  }
}

// ------------------------------------------------- accumulation policies
//
// A segment's value is the sum of its records' values i^k * c_a * c_b, in
// record order.
//
// kPlain: products and sums in the operands' precision.
//
// kComp (the precision form): products in FP32 from the operands rounded to
// FP32, summed with Sum2 of Ogita, Rump and Oishi (2005): Knuth's TwoSum
// splits each addition into the rounded sum and its exact rounding error,
// and the errors are added up beside the sum.  The accumulator also keeps
// the mass A = sum of |record value|.  A segment whose result is below
// tau * A has cancelled; its records are then summed again in FP64 from the
// operands' own coefficients.
constexpr int kPlain = 0;
constexpr int kComp = 1;

__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

template <int MODE, typename TV>
struct Acc;

template <typename TV>
struct Acc<kPlain, TV> {
  TV re, im;
  __device__ __forceinline__ void zero() { re = im = TV(0); }
  __device__ __forceinline__ void begin(TV r, TV i) {
    re = r;
    im = i;
  }
  __device__ __forceinline__ void add(TV r, TV i) {
    re = re + r;
    im = im + i;
  }
  __device__ __forceinline__ void add(const Acc& o) { add(o.re, o.im); }
  __device__ __forceinline__ TV value_re() const { return re; }
  __device__ __forceinline__ TV value_im() const { return im; }
  __device__ __forceinline__ bool cancels(double) const { return false; }
};

template <>
struct Acc<kComp, float> {
  // mass = sum of |term|; after begin() it is formed only when a second term
  // comes (lazy), since a one-term segment cannot cancel for tau <= 1
  float sr, er, si, ei, mass;
  bool lazy;
  __device__ __forceinline__ void zero() {
    sr = er = si = ei = mass = 0.0f;
    lazy = false;
  }
  __device__ __forceinline__ void begin(float r, float i) {
    sr = r;
    si = i;
    er = ei = 0.0f;
    lazy = true;  // mass would be hypotf(r, i)
  }
  __device__ __forceinline__ float mass_now() const { return lazy ? hypotf(sr, si) : mass; }
  __device__ __forceinline__ void add(float r, float i) {
    if (lazy) {
      mass = hypotf(sr, si);  // sr, si still hold the first term
      lazy = false;
    }
    float s, e;
    two_sum(sr, r, s, e);
    sr = s;
    er = er + e;
    two_sum(si, i, s, e);
    si = s;
    ei = ei + e;
    mass = mass + hypotf(r, i);
  }
  // adds another partial sum (its rounding errors included)
  __device__ __forceinline__ void add(const Acc& o) {
    const float m0 = mass_now(), m1 = o.mass_now();
    float s, e;
    two_sum(sr, o.sr, s, e);
    sr = s;
    er = er + (o.er + e);
    two_sum(si, o.si, s, e);
    si = s;
    ei = ei + (o.ei + e);
    mass = m0 + m1;
    lazy = false;
  }
  __device__ __forceinline__ float value_re() const { return sr + er; }
  __device__ __forceinline__ float value_im() const { return si + ei; }
  __device__ __forceinline__ bool cancels(double tau) const {
    // one term: |v| < tau |v| only for tau > 1
    if (lazy && !(tau > 1.0)) return false;
    return static_cast<double>(hypotf(value_re(), value_im())) <
           tau * static_cast<double>(mass_now());
  }
};

// ------------------------------------------------------------- float-float
//
// The state of a propagation loop in the precision form is carried from one
// rotation step to the next as float-float pairs hi + lo (|lo| <= ulp(hi)/2,
// Dekker 1971): a coefficient keeps about 48 significant bits while every
// operation on it is an FP32 operation.  Rounding the state to FP32 after
// each step would add about 2^-24 of relative error per step (eq. (5) is
// applied 64 times in a row), which a float-float carry avoids.
//   TwoProduct: a*b = p + e exactly, e = fma(a, b, -p) (Ogita, Rump and
//               Oishi 2005).
//   FastTwoSum: for |a| >= |b|, a + b = s + e exactly, e = b - (s - a).
// kFF is the accumulation policy of a merge whose records carry
// float-float values (kept as FP32 sum and FP32 error term, as in kComp,
// with the low parts added to the error term).
constexpr int kFF = 2;

struct ff {
  float hi, lo;
};

__host__ __device__ __forceinline__ ff operator-(ff a) { return {-a.hi, -a.lo}; }

__device__ __forceinline__ ff fast_two_sum(float a, float b) {
  const float s = a + b;
  return {s, b - (s - a)};
}

// (a.hi + a.lo)(b.hi + b.lo) to float-float: the product of the high parts
// exactly, the two cross terms in FP32, the product of the low parts
// (below 2^-48 relative) left out.
__device__ __forceinline__ ff ff_mul(ff a, ff b) {
  const float p = a.hi * b.hi;
  const float e = fmaf(a.hi, b.hi, -p);
  const float c = a.hi * b.lo + a.lo * b.hi;
  return fast_two_sum(p, e + c);
}

// Conversions between the coefficient types (double, float, float-float).
template <typename TO>
struct conv_to;
template <>
struct conv_to<double> {
  __device__ __forceinline__ static double of(double x) { return x; }
  __device__ __forceinline__ static double of(float x) { return static_cast<double>(x); }
  __device__ __forceinline__ static double of(ff x) {
    return static_cast<double>(x.hi) + static_cast<double>(x.lo);
  }
};
template <>
struct conv_to<float> {
  __device__ __forceinline__ static float of(double x) { return static_cast<float>(x); }
  __device__ __forceinline__ static float of(float x) { return x; }
  __device__ __forceinline__ static float of(ff x) {
    return static_cast<float>(static_cast<double>(x.hi) + static_cast<double>(x.lo));
  }
};
template <>
struct conv_to<ff> {
  __device__ __forceinline__ static ff of(double x) {
    const float h = static_cast<float>(x);
    return {h, static_cast<float>(x - static_cast<double>(h))};
  }
  __device__ __forceinline__ static ff of(float x) { return {x, 0.0f}; }
  __device__ __forceinline__ static ff of(ff x) { return x; }
};
template <typename TO, typename TI>
__device__ __forceinline__ TO conv(TI x) {
  return conv_to<TO>::of(x);
}
template <typename TO, typename TI>
__device__ __forceinline__ cplx<TO> convc(cplx<TI> v) {
  return {conv<TO>(v.re), conv<TO>(v.im)};
}

template <>
struct Acc<kFF, ff> {
  float sr, er, si, ei, mass;
  bool lazy;  // as in Acc<kComp, float>: the mass is formed at the second term
  __device__ __forceinline__ void zero() {
    sr = er = si = ei = mass = 0.0f;
    lazy = false;
  }
  __device__ __forceinline__ void begin(ff r, ff i) {
    sr = r.hi;
    er = r.lo;
    si = i.hi;
    ei = i.lo;
    lazy = true;
  }
  __device__ __forceinline__ float mass_now() const { return lazy ? hypotf(sr, si) : mass; }
  __device__ __forceinline__ void add(ff r, ff i) {
    if (lazy) {
      mass = hypotf(sr, si);
      lazy = false;
    }
    float s, e;
    two_sum(sr, r.hi, s, e);
    sr = s;
    er = er + (e + r.lo);
    two_sum(si, i.hi, s, e);
    si = s;
    ei = ei + (e + i.lo);
    mass = mass + hypotf(r.hi, i.hi);
  }
  __device__ __forceinline__ void add(const Acc& o) {
    const float m0 = mass_now(), m1 = o.mass_now();
    float s, e;
    two_sum(sr, o.sr, s, e);
    sr = s;
    er = er + (o.er + e);
    two_sum(si, o.si, s, e);
    si = s;
    ei = ei + (o.ei + e);
    mass = m0 + m1;
    lazy = false;
  }
  __device__ __forceinline__ ff value_re() const { return fast_two_sum_any(sr, er); }
  __device__ __forceinline__ ff value_im() const { return fast_two_sum_any(si, ei); }
  __device__ __forceinline__ bool cancels(double tau) const {
    if (lazy && !(tau > 1.0)) return false;
    return static_cast<double>(hypotf(sr + er, si + ei)) < tau * static_cast<double>(mass_now());
  }

 private:
  // s + e renormalised; |e| may exceed |s| after cancellation, so TwoSum
  __device__ __forceinline__ static ff fast_two_sum_any(float s, float e) {
    float h, l;
    two_sum(s, e, h, l);
    return {h, l};
  }
};

// -------------------------------------------------------------- truncation
//
// Section III-B removes a merged term whose modulus is strictly below the
// threshold t.  below_threshold decides |re + i im| < t exactly, in integer
// arithmetic on the significands (no square is rounded, so neither underflow
// for tiny t nor rounding near |c| = t can flip the answer).  With
// a = max(|re|, |im|) and b = min(|re|, |im|):
//   a >= t            -> no;
//   2a < t            -> yes (a^2 + b^2 <= 2 a^2 < t^2 / 2);
//   otherwise t/2 <= a < t, so t and a are within one binade of each other:
//   with t = T 2^E, a = A 2^E (common exponent E, T and A integers below
//   2^54), |c| < t  <=>  b^2 < (T - A)(T + A) 2^(2E), and with b = B 2^F
//   that is  B^2 2^(2F - 2E) < (T - A)(T + A),  where B^2 < 2^106 and the
//   product is below 2^109: 128-bit integers hold both.  For
//   X < D 2^k (k >= 0, D integer) the test is floor(X / 2^k) < D.
__host__ __device__ __forceinline__ void dbl_split(double x, uint64_t& m, int& e) {
  uint64_t u;
  __builtin_memcpy(&u, &x, 8);
  const int be = static_cast<int>((u >> 52) & 0x7FF);
  m = u & ((uint64_t(1) << 52) - 1);
  if (be == 0) {
    e = -1074;  // subnormal or zero
  } else {
    m |= uint64_t(1) << 52;
    e = be - 1075;
  }
}

__host__ __device__ __forceinline__ bool below_threshold(double re, double im, double t) {
  if (!(t > 0.0)) return false;
  double a = re < 0.0 ? -re : re, b = im < 0.0 ? -im : im;
  if (b > a) {
    const double x = a;
    a = b;
    b = x;
  }
  if (!(a < t)) return false;           // also a NaN component: kept
  if (t > 1.7976931348623157e308) return true;  // t = inf, a finite
  if (a + a < t) return true;           // 2a is exact here (a < t / 2 <= max / 2)
  uint64_t mt, ma, mb;
  int et, ea, eb;
  dbl_split(t, mt, et);
  dbl_split(a, ma, ea);
  const int e0 = et < ea ? et : ea;      // |et - ea| <= 1
  const unsigned __int128 T = static_cast<unsigned __int128>(mt) << (et - e0);
  const unsigned __int128 A = static_cast<unsigned __int128>(ma) << (ea - e0);
  const unsigned __int128 D = (T - A) * (T + A);  // > 0 since a < t
  if (b == 0.0) return true;
  dbl_split(b, mb, eb);
  const unsigned __int128 B2 = static_cast<unsigned __int128>(mb) * mb;
  const int k = 2 * (e0 - eb);  // b^2 < D 2^(2 e0)  <=>  B^2 < D 2^k
  if (k >= 0) return k >= 128 ? true : (B2 >> k) < D;
  return (B2 << (-k)) < D;  // -k <= 4: b <= a
}

// ------------------------------------------------------------ phase rule
//
// Write each letter as L(x,z) = i^{xz} X^x Z^z (so L(1,1) = iXZ = Y, Table I
// and Section III-A).  Moving Z^{z1} past X^{x2} costs (-1)^{z1 x2}, hence
//   L(x1,z1) L(x2,z2) = i^{x1z1 + x2z2 + 2 z1x2 - x3z3} L(x3,z3),
// x3 = x1 ^ x2, z3 = z1 ^ z2.  Summed over qubits with popcounts (the
// bit-parallel phase of Section III-E) and with the input phases:
//   k = k1 + k2 + |X1&Z1| + |X2&Z2| + 2|Z1&X2| - |X3&Z3|  (mod 4).
// e = k + |X&Z| is precomputed per input term.

}  // namespace pauli
