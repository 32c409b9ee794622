// Lexicographic order of a Pauli sum (Section III-H: the sum is ordered by a
// key formed from the bit-packed words of each string).  The key of a term
// is the tuple of its packed words X[W-1], ..., X[0], Z[W-1], ..., Z[0],
// compared as unsigned 64-bit integers (for n <= 32 the order of the integer
// x 2^32 + z); equal strings keep their input order.  A merged sum comes out
// of sort-and-combine in fingerprint order; this gives it the string order.
//
// One pass over the sum first finds, per word, the bits that differ between
// terms; a word that is the same for every term is skipped, and so is an
// 8-bit digit that is.  Two ways to order the positions, both stable LSD
// radix sorts of 64-bit keys:
//  * strings with few bit transitions (sparse letters, Z ranges: the
//    Jordan-Wigner shape) sort on a few keys that code the places of their
//    transitions (k_lex_trans_keys), when those take fewer sorts than the
//    varying words;
//  * otherwise the positions are sorted on the most significant varying word
//    alone.  Terms whose value of that word is unique are then in their final
//    place; the others (runs of equal values) are listed and put in order by
//    a stable LSD over their varying words, least significant first and
//    ending with the top word again, which regroups the runs in the order
//    they had, and go back to the positions they came from.  For distinct
//    random strings of more than 64 bits the runs are the repeats of a
//    string, and the order costs the passes of one word.
// The rows are then gathered once in the final order, through LDS tiles that
// keep both the reads and the writes on whole lines.
#include "common.h"
#include "internal.h"

namespace pauli {

namespace {

constexpr int kLexBlock = 256;
constexpr int kLexMaxKeys = 16;  // transition keys at most

__global__ void k_fill_u32_lex(uint32_t* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

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

// Runs of equal keys: flag[r] = 1 if keys[r] equals a neighbour.
__global__ void k_lex_tied(const uint64_t* __restrict__ keys, int64_t m,
                           uint32_t* __restrict__ flag) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < m;
       r += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = keys[r];
    const bool t = (r > 0 && keys[r - 1] == k) || (r + 1 < m && keys[r + 1] == k);
    flag[r] = t ? 1u : 0u;
  }
}

// The flagged positions in order: off is the exclusive scan of the flags,
// total their sum.  pos[j] = position, sub[j] = the term at that position.
__global__ void k_lex_take(const uint32_t* __restrict__ off, const uint32_t* __restrict__ total,
                           const uint32_t* __restrict__ idx, int64_t m, uint32_t* __restrict__ pos,
                           uint32_t* __restrict__ sub) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < m;
       r += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t o = off[r];
    const uint32_t nx = r + 1 < m ? off[r + 1] : *total;
    if (nx != o) {
      pos[o] = static_cast<uint32_t>(r);
      sub[o] = idx[r];
    }
  }
}

__global__ void k_lex_put(const uint32_t* __restrict__ pos, const uint32_t* __restrict__ sub,
                          int64_t ms, uint32_t* __restrict__ idx) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < ms;
       j += (int64_t)gridDim.x * blockDim.x)
    idx[pos[j]] = sub[j];
}

// The varying word positions, most significant first (p < W: Z[p], else
// X[p - W]).
struct LexWords {
  int n;
  int pos[2 * kMaxWords];
};

__device__ __forceinline__ const uint64_t* lex_word(const uint64_t* X, const uint64_t* Z, int W,
                                                    int64_t ld, int p) {
  return p < W ? Z + p * ld : X + (p - W) * ld;
}

// Transition code of a string.  Read the varying words as one bit string,
// most significant bit first, with a 0 above the first bit; G is a bit's
// place (0 at the top, L = 64 x the number of words).  A string is fixed by
// the places of its transitions (bits that differ from the bit above), and
// two strings compare as the tuples c_1, c_2, ... with c_j = L - G_j for odd
// j (a 0 -> 1 transition: earlier means larger) and c_j = G_j for even j
// (1 -> 0: earlier means smaller), a missing transition taking 0 (odd j) or
// L (even j): at the first bit where two strings differ the same number of
// transitions lie above, and exactly one of the two has its next transition
// there.  Strings with few transitions (sparse letters, ranges of Z) thus
// sort on a few 64-bit keys of S codes of b bits each instead of on all their
// words.
__device__ __forceinline__ uint64_t lex_transitions(uint64_t w, uint64_t prev) {
  return w ^ ((w >> 1) | (prev << 63));
}

// The largest number of transitions over the terms.
__global__ void __launch_bounds__(kLexBlock)
k_lex_trans_max(const uint64_t* __restrict__ X, const uint64_t* __restrict__ Z, int W, int64_t ld,
                int64_t m, LexWords vw, unsigned* __restrict__ tmax) {
  unsigned mx = 0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m;
       t += (int64_t)gridDim.x * blockDim.x) {
    uint64_t prev = 0;
    unsigned c = 0;
    for (int i = 0; i < vw.n; ++i) {
      const uint64_t w = lex_word(X, Z, W, ld, vw.pos[i])[t];
      c += static_cast<unsigned>(__popcll(lex_transitions(w, prev)));
      prev = w & 1ull;
    }
    mx = c > mx ? c : mx;
  }
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const unsigned o = __shfl_xor(mx, d, 64);
    mx = o > mx ? o : mx;
  }
  if ((threadIdx.x & 63) == 0) atomicMax(tmax, mx);
}

// The K keys of every term (key k of term t at KS[k m + t]): the codes c_1,
// c_2, ... in order, S to a key, the first in the key's top bits.  The next
// word is loaded before the transitions of the current one are coded.
__global__ void __launch_bounds__(kLexBlock)
k_lex_trans_keys(const uint64_t* __restrict__ X, const uint64_t* __restrict__ Z, int W,
                 int64_t ld, int64_t m, LexWords vw, int b, int S, int K,
                 uint64_t* __restrict__ KS) {
  const uint32_t L = 64u * static_cast<uint32_t>(vw.n);
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m;
       t += (int64_t)gridDim.x * blockDim.x) {
    uint64_t prev = 0, key = 0;
    int j = 0, s = 0, k = 0;  // codes so far, codes in the current key, keys written
    uint64_t w = lex_word(X, Z, W, ld, vw.pos[0])[t];
    for (int i = 0; i < vw.n; ++i) {
      const uint64_t wn = i + 1 < vw.n ? lex_word(X, Z, W, ld, vw.pos[i + 1])[t] : 0ull;
      uint64_t tb = lex_transitions(w, prev);
      prev = w & 1ull;
      while (tb != 0ull) {
        const int bit = 63 - __clzll(static_cast<long long>(tb));
        tb &= ~(1ull << bit);
        const uint32_t G = 64u * static_cast<uint32_t>(i) + static_cast<uint32_t>(63 - bit);
        const uint32_t c = (j & 1) ? G : L - G;
        key |= static_cast<uint64_t>(c) << (b * (S - 1 - s));
        ++j;
        if (++s == S) {
          if (k < K) KS[k * m + t] = key;
          ++k;
          key = 0;
          s = 0;
        }
      }
      w = wn;
    }
    while (k < K) {  // missing transitions
      const uint32_t c = (j & 1) ? L : 0u;
      key |= static_cast<uint64_t>(c) << (b * (S - 1 - s));
      ++j;
      if (++s == S) {
        KS[k * m + t] = key;
        ++k;
        key = 0;
        s = 0;
      }
    }
  }
}

// The terms as rows of RW = 2W + 4 words: X[0..W), Z[0..W), the
// coefficient (two words; an FP32 pair fills the first), the fingerprint and
// the phase byte.  A tile of kLexTile terms is read column by column into LDS
// (rows padded to RW + 1 words) and written out as one contiguous block.
constexpr int kLexTile = 128;

template <typename T>
__global__ void __launch_bounds__(kLexBlock)
k_lex_rows(const uint64_t* __restrict__ X, const uint64_t* __restrict__ Z,
           const uint8_t* __restrict__ ph, const cplx<T>* __restrict__ c,
           const uint64_t* __restrict__ fp, int W, int64_t ld, int64_t m,
           uint64_t* __restrict__ R) {
  extern __shared__ uint64_t s_row[];
  constexpr int CW = sizeof(cplx<T>) / 8;  // coefficient words (1 or 2)
  const int RW = 2 * W + 4, RS = RW + 1;
  const uint64_t* C = reinterpret_cast<const uint64_t*>(c);
  const int64_t ntiles = (m + kLexTile - 1) / kLexTile;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t t0 = tile * kLexTile;
    const int nt = m - t0 < kLexTile ? static_cast<int>(m - t0) : kLexTile;
    for (int i = threadIdx.x; i < RW * kLexTile; i += kLexBlock) {
      const int col = i / kLexTile, r = i % kLexTile;
      if (r >= nt) continue;
      const int64_t t = t0 + r;
      uint64_t v;
      if (col < W) v = X[col * ld + t];
      else if (col < 2 * W) v = Z[(col - W) * ld + t];
      else if (col == 2 * W) v = C[t * CW];
      else if (col == 2 * W + 1) v = CW == 2 ? C[t * CW + 1] : 0ull;
      else if (col == 2 * W + 2) v = fp[t];
      else v = ph[t];
      s_row[r * RS + col] = v;
    }
    __syncthreads();
    // the tile's rows are the words [t0 RW, (t0 + nt) RW) of R, written in
    // 16-byte pieces (RW is even and R 16-byte aligned)
    ulonglong2* out = reinterpret_cast<ulonglong2*>(R + t0 * RW);
    const int npc = nt * RW / 2;
    for (int j = threadIdx.x; j < npc; j += kLexBlock) {
      const int q = 2 * j, r = q / RW, col = q % RW;
      out[j] = make_ulonglong2(s_row[r * RS + col], s_row[r * RS + col + 1]);
    }
    __syncthreads();
  }
}

// Output term r is row idx[r]: a tile's rows are read whole (consecutive
// lanes take consecutive 16-byte pieces of one row) into LDS, then written
// out column by column.
template <typename T>
__global__ void __launch_bounds__(kLexBlock)
k_lex_permute(const uint64_t* __restrict__ R, int W, const uint32_t* __restrict__ idx,
              int64_t m, uint64_t* __restrict__ OX, uint64_t* __restrict__ OZ,
              uint8_t* __restrict__ Oph, cplx<T>* __restrict__ Oc, uint64_t* __restrict__ Ofp,
              int64_t ldo) {
  extern __shared__ uint64_t s_row[];
  __shared__ uint32_t s_idx[kLexTile];
  constexpr int CW = sizeof(cplx<T>) / 8;
  const int RW = 2 * W + 4, RS = RW + 1, P = RW / 2;
  const ulonglong2* R2 = reinterpret_cast<const ulonglong2*>(R);
  uint64_t* OC = reinterpret_cast<uint64_t*>(Oc);
  const int64_t ntiles = (m + kLexTile - 1) / kLexTile;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t r0 = tile * kLexTile;
    const int nt = m - r0 < kLexTile ? static_cast<int>(m - r0) : kLexTile;
    for (int r = threadIdx.x; r < nt; r += kLexBlock) s_idx[r] = idx[r0 + r];
    __syncthreads();
    for (int i = threadIdx.x; i < nt * P; i += kLexBlock) {
      const int r = i / P, pc = i % P;
      const ulonglong2 v = R2[static_cast<int64_t>(s_idx[r]) * P + pc];
      s_row[r * RS + 2 * pc] = v.x;
      s_row[r * RS + 2 * pc + 1] = v.y;
    }
    __syncthreads();
    const int ncol = 2 * W + 2 + CW;  // string words, coefficient words, fp, phase
    for (int i = threadIdx.x; i < ncol * kLexTile; i += kLexBlock) {
      const int col = i / kLexTile, r = i % kLexTile;
      if (r >= nt) continue;
      const int64_t o = r0 + r;
      if (col < W) {
        OX[col * ldo + o] = s_row[r * RS + col];
      } else if (col < 2 * W) {
        OZ[(col - W) * ldo + o] = s_row[r * RS + col];
      } else if (col < 2 * W + CW) {
        OC[o * CW + (col - 2 * W)] = s_row[r * RS + col];
      } else if (col == 2 * W + CW) {
        Ofp[o] = s_row[r * RS + 2 * W + 2];
      } else {
        Oph[o] = static_cast<uint8_t>(s_row[r * RS + 2 * W + 3]);
      }
    }
    __syncthreads();
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
  const size_t lds = static_cast<size_t>(kLexTile) * (RW + 1) * 8;
  int64_t nt = (s->m + kLexTile - 1) / kLexTile;
  const unsigned g = static_cast<unsigned>(nt < 65536 ? nt : 65536);
  hipLaunchKernelGGL((k_lex_rows<T>), dim3(g), dim3(kLexBlock), lds, st, s->X, s->Z, s->ph,
                     static_cast<const cplx<T>*>(s->coef), s->fp, s->W, s->ld, s->m,
                     rows.as<uint64_t>());
  hipLaunchKernelGGL((k_lex_permute<T>), dim3(g), dim3(kLexBlock), lds, st, rows.as<uint64_t>(),
                     s->W, idx, s->m, o->X, o->Z, o->ph, static_cast<cplx<T>*>(o->coef), o->fp,
                     o->ld);
  PAULI_HIP(hipGetLastError());
}

// A key column of the stable LSD: col[t] for term t; digits with no bit in
// vary are skipped.
struct LexCol {
  const uint64_t* col;
  uint64_t vary;
};

// Stable LSD of the terms vals[0..n) on the columns, least significant
// first.  Returns the buffer holding the result.
uint32_t* lex_lsd(const std::vector<LexCol>& cols, uint32_t* vals, uint32_t* spare, int64_t n,
                  uint64_t* keys, uint64_t* keys_alt, void* work, hipStream_t st) {
  for (const LexCol& c : cols) {
    if (c.vary == 0) continue;
    hipLaunchKernelGGL(k_lex_gather, dim3(lex_grid(n)), dim3(kLexBlock), 0, st, c.col, vals, n,
                       keys);
    PAULI_HIP(hipGetLastError());
    if (radix_sort_pairs(keys, vals, keys_alt, spare, n, 64, work, st, c.vary)) {
      std::swap(vals, spare);
      std::swap(keys, keys_alt);
    }
  }
  return vals;
}

// Number of transition keys that hold every term's codes, or 0 when they
// would take as many sorts as the varying words (or more than kLexMaxKeys).
int lex_transition_keys(const paulisum* s, const LexWords& vw, int b, int S, hipStream_t st) {
  if (vw.n < 2) return 0;
  DBuf tm(256, st);
  hipLaunchKernelGGL(k_fill_u32_lex, dim3(1), dim3(64), 0, st, tm.as<uint32_t>(), 1);
  int64_t g = (s->m + kLexBlock - 1) / kLexBlock;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_lex_trans_max, dim3(static_cast<unsigned>(g)), dim3(kLexBlock), 0, st,
                     s->X, s->Z, s->W, s->ld, s->m, vw, tm.as<unsigned>());
  PAULI_HIP(hipGetLastError());
  uint32_t tmax = 0;
  PAULI_HIP(hipMemcpyAsync(&tmax, tm.p, 4, hipMemcpyDeviceToHost, st));
  PAULI_HIP(hipStreamSynchronize(st));
  const int K = static_cast<int>((tmax + S - 1) / S);
  return K >= 1 && K < vw.n && K <= kLexMaxKeys ? K : 0;
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
    LexWords vw{};  // the varying word positions, most significant first
    for (int p = npos - 1; p >= 0; --p)
      if (bits[2 * p] != bits[2 * p + 1]) vw.pos[vw.n++] = p;
    const int top = vw.n ? vw.pos[0] : -1;

    DBuf i0(m * 4ull, st), i1(m * 4ull, st), k0(m * 8ull, st), k1(m * 8ull, st);
    DBuf work(radix_workspace_bytes(m), st);
    uint32_t* cur = i0.as<uint32_t>();
    hipLaunchKernelGGL(k_lex_iota, dim3(lex_grid(m)), dim3(kLexBlock), 0, st, cur, m);
    const uint32_t L = 64u * static_cast<uint32_t>(vw.n);
    const int b = L ? 64 - __builtin_clzll(static_cast<unsigned long long>(L)) : 1;
    const int S = 64 / b;
    const int K = lex_transition_keys(s, vw, b, S, st);
    if (K > 0) {
      // few transitions: the K transition keys of all terms, least
      // significant first; the first sort takes its key column in place
      DBuf tk(static_cast<size_t>(K) * m * 8, st);
      hipLaunchKernelGGL(k_lex_trans_keys, dim3(lex_grid(m)), dim3(kLexBlock), 0, st, s->X, s->Z,
                         W, s->ld, m, vw, b, S, K, tk.as<uint64_t>());
      PAULI_HIP(hipGetLastError());
      const uint64_t used = S * b == 64 ? ~0ull : (1ull << (S * b)) - 1;
      uint64_t* last = tk.as<uint64_t>() + static_cast<int64_t>(K - 1) * m;
      if (radix_sort_pairs(last, cur, k0.as<uint64_t>(), i1.as<uint32_t>(), m, 64, work.p, st,
                           used))
        cur = i1.as<uint32_t>();
      std::vector<LexCol> cols;
      for (int k = K - 2; k >= 0; --k) cols.push_back({tk.as<uint64_t>() + k * m, used});
      cur = lex_lsd(cols, cur, cur == i0.as<uint32_t>() ? i1.as<uint32_t>() : i0.as<uint32_t>(),
                    m, k0.as<uint64_t>(), k1.as<uint64_t>(), work.p, st);
    } else if (top >= 0) {
      // the top varying word alone
      const uint64_t vary = bits[2 * top] ^ bits[2 * top + 1];
      const uint64_t* w = top < W ? s->Z + top * s->ld : s->X + (top - W) * s->ld;
      uint64_t* keys = k0.as<uint64_t>();
      uint64_t* keys_alt = k1.as<uint64_t>();
      hipLaunchKernelGGL(k_lex_gather, dim3(lex_grid(m)), dim3(kLexBlock), 0, st, w, cur, m,
                         keys);
      PAULI_HIP(hipGetLastError());
      if (radix_sort_pairs(keys, cur, keys_alt, i1.as<uint32_t>(), m, 64, work.p, st, vary)) {
        cur = i1.as<uint32_t>();
        keys = keys_alt;
      }
      if (vw.n > 1) {
        // the runs of equal top words, ordered on all their varying words
        DBuf off(m * 4ull, st), tot(256, st), sw(scan_workspace_bytes(m), st);
        hipLaunchKernelGGL(k_lex_tied, dim3(lex_grid(m)), dim3(kLexBlock), 0, st, keys, m,
                           off.as<uint32_t>());
        scan_exclusive_u32(off.as<uint32_t>(), off.as<uint32_t>(), m, tot.as<uint32_t>(), sw.p,
                           st);
        uint32_t ms = 0;
        PAULI_HIP(hipMemcpyAsync(&ms, tot.p, 4, hipMemcpyDeviceToHost, st));
        PAULI_HIP(hipStreamSynchronize(st));
        if (ms > 0) {
          DBuf pos(ms * 4ull, st), sa(ms * 4ull, st), sb(ms * 4ull, st);
          hipLaunchKernelGGL(k_lex_take, dim3(lex_grid(m)), dim3(kLexBlock), 0, st,
                             off.as<uint32_t>(), tot.as<uint32_t>(), cur, m, pos.as<uint32_t>(),
                             sa.as<uint32_t>());
          PAULI_HIP(hipGetLastError());
          std::vector<LexCol> cols;
          for (int p = 0; p <= top; ++p) {
            const uint64_t* wp = p < W ? s->Z + p * s->ld : s->X + (p - W) * s->ld;
            cols.push_back({wp, bits[2 * p] ^ bits[2 * p + 1]});
          }
          uint32_t* su = lex_lsd(cols, sa.as<uint32_t>(), sb.as<uint32_t>(), ms,
                                 k0.as<uint64_t>(), k1.as<uint64_t>(), work.p, st);
          hipLaunchKernelGGL(k_lex_put, dim3(lex_grid(ms)), dim3(kLexBlock), 0, st,
                             pos.as<uint32_t>(), su, static_cast<int64_t>(ms), cur);
          PAULI_HIP(hipGetLastError());
        }
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
