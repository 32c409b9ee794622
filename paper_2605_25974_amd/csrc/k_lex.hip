// Lexicographic order of a Pauli sum (Section III-H: the sum is ordered by a
// key formed from the bit-packed words of each string).  The key of a term
// is the tuple of its packed words X[W-1], ..., X[0], Z[W-1], ..., Z[0],
// compared as unsigned 64-bit integers (for n <= 32 the order of the integer
// x 2^32 + z); equal strings keep their input order.  A merged sum comes out
// of sort-and-combine in fingerprint order; this gives it the string order.
//
// LSD over the words: the term positions are radix-sorted stably on Z[0],
// then Z[1], ..., then X[W-1], each word's values gathered in the order the
// previous words left.  One pass over the sum first finds, per word, the bits
// that differ between terms; a word that is the same for every term is
// skipped, and so is an 8-bit digit that is.  The rows are then gathered once
// in the final order.
#include "common.h"
#include "internal.h"

namespace pauli {

namespace {

constexpr int kLexBlock = 256;

__global__ void k_lex_iota(uint32_t* __restrict__ idx, int64_t m) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < m;
       r += (int64_t)gridDim.x * blockDim.x)
    idx[r] = static_cast<uint32_t>(r);
}

__global__ void k_lex_bits_init(unsigned long long* __restrict__ acc, int npos) {
  for (int p = threadIdx.x; p < npos; p += blockDim.x) {
    acc[2 * p] = 0ull;
    acc[2 * p + 1] = ~0ull;
  }
}

// acc[2p] = OR, acc[2p + 1] = AND of word position p over the terms
// (p < W: Z[p]; p >= W: X[p - W]); blockIdx.y is the position.
__global__ void __launch_bounds__(kLexBlock)
k_lex_bits(const uint64_t* __restrict__ X, const uint64_t* __restrict__ Z, int W, int64_t ld,
           int64_t m, unsigned long long* __restrict__ acc) {
  const int p = blockIdx.y;
  const uint64_t* w = p < W ? Z + p * ld : X + (p - W) * ld;
  uint64_t o = 0, a = ~0ull;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < m;
       r += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t v = w[r];
    o |= v;
    a &= v;
  }
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    o |= __shfl_xor(o, d, 64);
    a &= __shfl_xor(a, d, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicOr(&acc[2 * p], static_cast<unsigned long long>(o));
    atomicAnd(&acc[2 * p + 1], static_cast<unsigned long long>(a));
  }
}

__global__ void k_lex_gather(const uint64_t* __restrict__ w, const uint32_t* __restrict__ idx,
                             int64_t m, uint64_t* __restrict__ keys) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < m;
       r += (int64_t)gridDim.x * blockDim.x)
    keys[r] = w[idx[r]];
}

// The terms as rows of RW = 2W + 4 words: X[0..W), Z[0..W), the
// coefficient (two words, FP32 pairs packed in the first), the fingerprint
// and the phase byte, so that the final gather in sorted order reads whole
// lines instead of one 8-byte word per array.
template <typename T>
__global__ void __launch_bounds__(kLexBlock)
k_lex_rows(const uint64_t* __restrict__ X, const uint64_t* __restrict__ Z,
           const uint8_t* __restrict__ ph, const cplx<T>* __restrict__ c,
           const uint64_t* __restrict__ fp, int W, int64_t ld, int64_t m,
           uint64_t* __restrict__ R) {
  const int RW = 2 * W + 4;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m;
       t += (int64_t)gridDim.x * blockDim.x) {
    uint64_t* row = R + t * RW;
    for (int w = 0; w < W; ++w) {
      row[w] = X[w * ld + t];
      row[W + w] = Z[w * ld + t];
    }
    const cplx<T> v = c[t];
    uint64_t c0 = 0, c1 = 0;
    static_assert(sizeof(cplx<T>) <= 16, "coefficient fits two words");
    __builtin_memcpy(&c0, &v, sizeof(cplx<T>) < 8 ? sizeof(cplx<T>) : 8);
    if (sizeof(cplx<T>) > 8) __builtin_memcpy(&c1, reinterpret_cast<const char*>(&v) + 8, 8);
    row[2 * W] = c0;
    row[2 * W + 1] = c1;
    row[2 * W + 2] = fp[t];
    row[2 * W + 3] = ph[t];
  }
}

// Output term r is row idx[r].
template <typename T>
__global__ void __launch_bounds__(kLexBlock)
k_lex_permute(const uint64_t* __restrict__ R, int W, const uint32_t* __restrict__ idx,
              int64_t m, uint64_t* __restrict__ OX, uint64_t* __restrict__ OZ,
              uint8_t* __restrict__ Oph, cplx<T>* __restrict__ Oc, uint64_t* __restrict__ Ofp,
              int64_t ldo) {
  const int RW = 2 * W + 4;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < m;
       r += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t* row = R + static_cast<int64_t>(idx[r]) * RW;
    // the string words in 16-byte pieces (rows start on 16-byte boundaries)
    const ulonglong2* row2 = reinterpret_cast<const ulonglong2*>(row);
    for (int p = 0; p < W; ++p) {
      const ulonglong2 v = row2[p];
      const int w0 = 2 * p, w1 = 2 * p + 1;
      if (w0 < W) OX[w0 * ldo + r] = v.x;
      else OZ[(w0 - W) * ldo + r] = v.x;
      if (w1 < W) OX[w1 * ldo + r] = v.y;
      else OZ[(w1 - W) * ldo + r] = v.y;
    }
    const uint64_t c0 = row[2 * W], c1 = row[2 * W + 1];
    cplx<T> cv;
    __builtin_memcpy(&cv, &c0, sizeof(cplx<T>) < 8 ? sizeof(cplx<T>) : 8);
    if (sizeof(cplx<T>) > 8) __builtin_memcpy(reinterpret_cast<char*>(&cv) + 8, &c1, 8);
    Oc[r] = cv;
    Ofp[r] = row[2 * W + 2];
    Oph[r] = static_cast<uint8_t>(row[2 * W + 3]);
  }
}

unsigned lex_grid(int64_t m) {
  int64_t g = (m + kLexBlock - 1) / kLexBlock;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return static_cast<unsigned>(g);
}

template <typename T>
void lex_permute_t(const paulisum* s, const uint32_t* idx, paulisum* o, hipStream_t st) {
  const int RW = 2 * s->W + 4;
  DBuf rows(static_cast<size_t>(s->m) * RW * 8, st);
  hipLaunchKernelGGL((k_lex_rows<T>), dim3(lex_grid(s->m)), dim3(kLexBlock), 0, st, s->X, s->Z,
                     s->ph, static_cast<const cplx<T>*>(s->coef), s->fp, s->W, s->ld, s->m,
                     rows.as<uint64_t>());
  hipLaunchKernelGGL((k_lex_permute<T>), dim3(lex_grid(s->m)), dim3(kLexBlock), 0, st,
                     rows.as<uint64_t>(), s->W, idx, s->m, o->X, o->Z, o->ph,
                     static_cast<cplx<T>*>(o->coef), o->fp, o->ld);
  PAULI_HIP(hipGetLastError());
}

}  // namespace

paulisum* sort_lex(const paulisum* s, hipStream_t st) {
  const int64_t m = s->m;
  const int W = s->W;
  if (m > static_cast<int64_t>(0xFFFFFFFFll))
    fail(PAULI_ERR_CAPACITY, "lexicographic order: more than 2^32 terms");
  paulisum* o = new_sum(s->n, m, m, s->dtype, st);
  if (m == 0) return o;
  try {
    const double cb = s->dtype == PAULI_C128 ? 16.0 : 8.0;
    // algorithmic bytes: every term read once and written once
    StageScope sc(PAULI_STAGE_LEX, st, 2.0 * m * (16.0 * W + 1 + 8 + cb));
    const int npos = 2 * W;
    DBuf acc(static_cast<size_t>(npos) * 16, st);
    hipLaunchKernelGGL(k_lex_bits_init, dim3(1), dim3(64), 0, st,
                       acc.as<unsigned long long>(), npos);
    int64_t gx = (m + kLexBlock - 1) / kLexBlock;
    if (gx > 256) gx = 256;
    hipLaunchKernelGGL(k_lex_bits, dim3(static_cast<unsigned>(gx), static_cast<unsigned>(npos)),
                       dim3(kLexBlock), 0, st, s->X, s->Z, W, s->ld, m,
                       acc.as<unsigned long long>());
    PAULI_HIP(hipGetLastError());
    std::vector<uint64_t> bits(static_cast<size_t>(npos) * 2);
    PAULI_HIP(hipMemcpyAsync(bits.data(), acc.p, bits.size() * 8, hipMemcpyDeviceToHost, st));
    PAULI_HIP(hipStreamSynchronize(st));

    DBuf i0(m * 4ull, st), i1(m * 4ull, st), k0(m * 8ull, st), k1(m * 8ull, st);
    DBuf work(radix_workspace_bytes(m), st);
    uint32_t* cur = i0.as<uint32_t>();
    uint32_t* spare = i1.as<uint32_t>();
    uint64_t* keys = k0.as<uint64_t>();
    uint64_t* keys_alt = k1.as<uint64_t>();
    hipLaunchKernelGGL(k_lex_iota, dim3(lex_grid(m)), dim3(kLexBlock), 0, st, cur, m);
    for (int p = 0; p < npos; ++p) {  // least significant word first
      const uint64_t vary = bits[2 * p] ^ bits[2 * p + 1];
      if (vary == 0) continue;
      const uint64_t* w = p < W ? s->Z + p * s->ld : s->X + (p - W) * s->ld;
      hipLaunchKernelGGL(k_lex_gather, dim3(lex_grid(m)), dim3(kLexBlock), 0, st, w, cur, m,
                         keys);
      PAULI_HIP(hipGetLastError());
      if (radix_sort_pairs(keys, cur, keys_alt, spare, m, 64, work.p, st, vary)) {
        std::swap(cur, spare);
        std::swap(keys, keys_alt);
      }
    }
    if (s->dtype == PAULI_C128)
      lex_permute_t<double>(s, cur, o, st);
    else
      lex_permute_t<float>(s, cur, o, st);
  } catch (...) {
    free_sum(o);
    throw;
  }
  return o;
}

}  // namespace pauli
