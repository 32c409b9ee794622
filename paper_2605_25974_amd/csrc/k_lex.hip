// Lexicographic order of a Pauli sum (Section III-H: the sum is ordered by a
// key formed from the bit-packed words of each string).  The key of a term
// is the tuple of its packed words X[W-1], ..., X[0], Z[W-1], ..., Z[0],
// compared as unsigned 64-bit integers (for n <= 32 the order of the integer
// x 2^32 + z); equal strings keep their input order.  A merged sum comes out
// of sort-and-combine in fingerprint order; this gives it the string order.
//
// One pass over the sum first finds, per word, the bits that differ between
// terms; a word that is the same for every term is skipped, and so is an
// 8-bit digit that is.  The term positions are then radix-sorted (stable) on
// the most significant varying word alone.  Terms whose value of that word is
// unique are in their final place.  The others (runs of equal values) are
// listed and put in order by a stable LSD over their varying words, least
// significant first and ending with the top word again, which regroups the
// runs in the order they had; they go back to the positions they came from.
// For distinct random strings of more than 64 bits the runs are the repeats
// of a string, and the whole order costs the passes of one word.  The rows
// are then gathered once in the final order, through LDS tiles that keep both
// the reads and the writes on whole lines.
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

// Stable LSD of the positions vals[0..n) on the varying words at positions
// [0, top] (least significant first).  Returns the buffer holding the result.
uint32_t* lex_lsd(const paulisum* s, const std::vector<uint64_t>& bits, int top, uint32_t* vals,
                  uint32_t* spare, int64_t n, uint64_t* keys, uint64_t* keys_alt, void* work,
                  hipStream_t st) {
  for (int p = 0; p <= top; ++p) {
    const uint64_t vary = bits[2 * p] ^ bits[2 * p + 1];
    if (vary == 0) continue;
    const uint64_t* w = p < s->W ? s->Z + p * s->ld : s->X + (p - s->W) * s->ld;
    hipLaunchKernelGGL(k_lex_gather, dim3(lex_grid(n)), dim3(kLexBlock), 0, st, w, vals, n, keys);
    PAULI_HIP(hipGetLastError());
    if (radix_sort_pairs(keys, vals, keys_alt, spare, n, 64, work, st, vary)) {
      std::swap(vals, spare);
      std::swap(keys, keys_alt);
    }
  }
  return vals;
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
    int top = -1;  // the most significant varying word position
    for (int p = npos - 1; p >= 0 && top < 0; --p)
      if (bits[2 * p] != bits[2 * p + 1]) top = p;

    DBuf i0(m * 4ull, st), i1(m * 4ull, st), k0(m * 8ull, st), k1(m * 8ull, st);
    DBuf work(radix_workspace_bytes(m), st);
    uint32_t* cur = i0.as<uint32_t>();
    hipLaunchKernelGGL(k_lex_iota, dim3(lex_grid(m)), dim3(kLexBlock), 0, st, cur, m);
    if (top >= 0) {
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
      bool lower = false;  // a varying word below the top one
      for (int p = 0; p < top; ++p) lower |= bits[2 * p] != bits[2 * p + 1];
      if (lower) {
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
          uint32_t* su = lex_lsd(s, bits, top, sa.as<uint32_t>(), sb.as<uint32_t>(), ms,
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
