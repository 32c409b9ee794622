// Layout conversion, validation, fingerprints and the materialised outer
// product (Section IV-C: output block j holds a_i * b_j for every i).
#include "common.h"
#include "internal.h"

namespace pauli {

namespace {

constexpr int kBlock = 256;

inline unsigned grid_for(int64_t n, int per_block = kBlock) {
  int64_t g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > (1 << 30)) g = 1 << 30;
  return static_cast<unsigned>(g);
}

__global__ void k_rows_to_soa(const uint64_t* __restrict__ rows, int W, int64_t m,
                              uint64_t* __restrict__ soa, int64_t ld) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m;
       t += (int64_t)gridDim.x * blockDim.x)
    for (int w = 0; w < W; ++w) soa[w * ld + t] = rows[t * W + w];
}

__global__ void k_soa_to_rows(const uint64_t* __restrict__ soa, int W, int64_t m, int64_t ld,
                              uint64_t* __restrict__ rows) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m;
       t += (int64_t)gridDim.x * blockDim.x)
    for (int w = 0; w < W; ++w) rows[t * W + w] = soa[w * ld + t];
}

// err bit 0: a set bit at or above n; bit 1: a phase above 3.
__global__ void k_validate(const uint64_t* __restrict__ xr, const uint64_t* __restrict__ zr,
                           const uint8_t* __restrict__ ph, int n, int64_t m,
                           uint32_t* __restrict__ err) {
  const int W = (n + 63) / 64;
  const int tail = n - 64 * (W - 1);
  const uint64_t pad = tail == 64 ? 0ull : ~((1ull << tail) - 1);
  uint32_t e = 0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m;
       t += (int64_t)gridDim.x * blockDim.x) {
    if ((xr[t * W + W - 1] | zr[t * W + W - 1]) & pad) e |= 1u;
    if (ph && ph[t] > 3) e |= 2u;
  }
  if (e) atomicOr(err, e);
}

// fp[t] = XOR of the columns of the set bits of term t.
__global__ void k_fingerprint(const uint64_t* __restrict__ X, const uint64_t* __restrict__ Z,
                              int W, int64_t m, int64_t ld, uint64_t* __restrict__ fp) {
  __shared__ uint64_t col[2 * 64 * kMaxWords];
  for (int b = threadIdx.x; b < 2 * 64 * W; b += blockDim.x) col[b] = fp_column(b);
  __syncthreads();
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m;
       t += (int64_t)gridDim.x * blockDim.x) {
    uint64_t f = 0;
    for (int w = 0; w < W; ++w) {
      uint64_t x = X[w * ld + t], z = Z[w * ld + t];
      while (x) {
        int b = __builtin_ctzll(x);
        f ^= col[2 * (64 * w + b)];
        x &= x - 1;
      }
      while (z) {
        int b = __builtin_ctzll(z);
        f ^= col[2 * (64 * w + b) + 1];
        z &= z - 1;
      }
    }
    fp[t] = f;
  }
}

__global__ void k_prep_side(const uint64_t* __restrict__ X, const uint64_t* __restrict__ Z,
                            const uint8_t* __restrict__ ph, int W, int64_t m, int64_t ld,
                            uint64_t* __restrict__ rows, uint8_t* __restrict__ e) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m;
       t += (int64_t)gridDim.x * blockDim.x) {
    int y = 0;
    for (int w = 0; w < W; ++w) {
      uint64_t x = X[w * ld + t], z = Z[w * ld + t];
      rows[t * 2 * W + w] = x;
      rows[t * 2 * W + W + w] = z;
      y += popc64(x & z);
    }
    e[t] = static_cast<uint8_t>((ph[t] + y) & 3);
  }
}

// One thread per product p = j*ma + i.  Reads of a's words are coalesced
// across the wave (consecutive i), b's words are the same address for the
// whole wave; every output column is written coalesced.
template <int WT, typename T>
__global__ void __launch_bounds__(kBlock)
k_outer_product(const uint64_t* __restrict__ AX, const uint64_t* __restrict__ AZ,
                const uint8_t* __restrict__ Aph, const cplx<T>* __restrict__ Ac,
                const uint64_t* __restrict__ Afp, int64_t ma, int64_t lda,
                const uint64_t* __restrict__ BX, const uint64_t* __restrict__ BZ,
                const uint8_t* __restrict__ Bph, const cplx<T>* __restrict__ Bc,
                const uint64_t* __restrict__ Bfp, int64_t ldb, int nw, int64_t P,
                uint64_t* __restrict__ OX, uint64_t* __restrict__ OZ, uint8_t* __restrict__ Oph,
                cplx<T>* __restrict__ Oc, uint64_t* __restrict__ Ofp, int64_t ldo) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = p / ma;
    const int64_t i = p - j * ma;
    int acc = Aph[i] + Bph[j];
#pragma unroll
    for (int w = 0; w < WT; ++w) {
      if (WT > 8 && w >= nw) break;
      const uint64_t xa = AX[w * lda + i], za = AZ[w * lda + i];
      const uint64_t xb = BX[w * ldb + j], zb = BZ[w * ldb + j];
      const uint64_t x = xa ^ xb, z = za ^ zb;
      acc += popc64(xa & za) + popc64(xb & zb) + 2 * popc64(za & xb) - popc64(x & z);
      OX[w * ldo + p] = x;
      OZ[w * ldo + p] = z;
    }
    Oph[p] = static_cast<uint8_t>(acc & 3);
    Oc[p] = cmul(Ac[i], Bc[j]);
    Ofp[p] = Afp[i] ^ Bfp[j];
  }
}

template <typename T>
void outer_product_t(const paulisum* a, const paulisum* b, paulisum* o, hipStream_t s) {
  const int64_t P = a->m * b->m;
  if (P == 0) return;
  const unsigned g = grid_for(P);
  // compulsory traffic: the P products written (2W words, phase, coefficient,
  // fingerprint); the operands are read once from HBM and then from cache
  const double per = 16.0 * a->W + sizeof(cplx<T>) + 1 + 8;
  StageScope sc(PAULI_STAGE_OUTER_PRODUCT, s, per * P);
  auto Ac = static_cast<const cplx<T>*>(a->coef);
  auto Bc = static_cast<const cplx<T>*>(b->coef);
  auto Oc = static_cast<cplx<T>*>(o->coef);
#define PAULI_OP_CASE(WW)                                                                    \
  case WW:                                                                                   \
    hipLaunchKernelGGL((k_outer_product<WW, T>), dim3(g), dim3(kBlock), 0, s, a->X, a->Z,     \
                       a->ph, Ac, a->fp, a->m, a->ld, b->X, b->Z, b->ph, Bc, b->fp, b->ld,    \
                       a->W, P, o->X, o->Z, o->ph, Oc, o->fp, o->ld);                         \
    break;
  switch (a->W) {
    PAULI_OP_CASE(1) PAULI_OP_CASE(2) PAULI_OP_CASE(3) PAULI_OP_CASE(4)
    PAULI_OP_CASE(5) PAULI_OP_CASE(6) PAULI_OP_CASE(7) PAULI_OP_CASE(8)
    default:
      hipLaunchKernelGGL((k_outer_product<kMaxWords, T>), dim3(g), dim3(kBlock), 0, s, a->X,
                         a->Z, a->ph, Ac, a->fp, a->m, a->ld, b->X, b->Z, b->ph, Bc, b->fp,
                         b->ld, a->W, P, o->X, o->Z, o->ph, Oc, o->fp, o->ld);
  }
#undef PAULI_OP_CASE
  PAULI_HIP(hipGetLastError());
}

// flag[p] = 1 if the pair p = j*|a| + i anticommutes: the parity of
// sum over words of |X_a & Z_b| + |Z_a & X_b| (Section III-F).
template <int WT>
__global__ void k_comm_flags(const uint64_t* __restrict__ AX, const uint64_t* __restrict__ AZ,
                             int64_t ma, int64_t lda, const uint64_t* __restrict__ BX,
                             const uint64_t* __restrict__ BZ, int64_t ldb, int nw, int64_t P,
                             uint32_t* __restrict__ flag) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = p / ma;
    const int64_t i = p - j * ma;
    int s = 0;
#pragma unroll
    for (int w = 0; w < WT; ++w) {
      if (WT > 8 && w >= nw) break;
      s += popc64((AX[w * lda + i] & BZ[w * ldb + j]) ^ (AZ[w * lda + i] & BX[w * ldb + j]));
    }
    flag[p] = static_cast<uint32_t>(s & 1);
  }
}

// The anticommuting products at their compacted positions off[p], each with
// coefficient 2 c_a c_b (a_i b_j - b_j a_i = 2 a_i b_j for such a pair).
template <int WT, typename T>
__global__ void k_comm_write(const uint64_t* __restrict__ AX, const uint64_t* __restrict__ AZ,
                             const uint8_t* __restrict__ Aph, const cplx<T>* __restrict__ Ac,
                             const uint64_t* __restrict__ Afp, int64_t ma, int64_t lda,
                             const uint64_t* __restrict__ BX, const uint64_t* __restrict__ BZ,
                             const uint8_t* __restrict__ Bph, const cplx<T>* __restrict__ Bc,
                             const uint64_t* __restrict__ Bfp, int64_t ldb, int nw, int64_t P,
                             const uint32_t* __restrict__ flag, const uint32_t* __restrict__ off,
                             uint64_t* __restrict__ OX, uint64_t* __restrict__ OZ,
                             uint8_t* __restrict__ Oph, cplx<T>* __restrict__ Oc,
                             uint64_t* __restrict__ Ofp, int64_t ldo) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P;
       p += (int64_t)gridDim.x * blockDim.x) {
    if (!flag[p]) continue;
    const int64_t j = p / ma;
    const int64_t i = p - j * ma;
    const int64_t o = off[p];
    int acc = Aph[i] + Bph[j];
#pragma unroll
    for (int w = 0; w < WT; ++w) {
      if (WT > 8 && w >= nw) break;
      const uint64_t xa = AX[w * lda + i], za = AZ[w * lda + i];
      const uint64_t xb = BX[w * ldb + j], zb = BZ[w * ldb + j];
      const uint64_t x = xa ^ xb, z = za ^ zb;
      acc += popc64(xa & za) + popc64(xb & zb) + 2 * popc64(za & xb) - popc64(x & z);
      OX[w * ldo + o] = x;
      OZ[w * ldo + o] = z;
    }
    Oph[o] = static_cast<uint8_t>(acc & 3);
    const cplx<T> v = cmul(Ac[i], Bc[j]);
    Oc[o] = cplx<T>{v.re + v.re, v.im + v.im};
    Ofp[o] = Afp[i] ^ Bfp[j];
  }
}

template <typename T>
paulisum* commutator_products_t(const paulisum* a, const paulisum* b, hipStream_t s) {
  const int64_t P = a->m * b->m;
  DBuf flag((P + 1) * 4, s), off((P + 1) * 4, s), tot(4, s), work(scan_workspace_bytes(P), s);
  const unsigned g = grid_for(P);
#define PAULI_CF_CASE(WW)                                                                     \
  case WW:                                                                                    \
    hipLaunchKernelGGL((k_comm_flags<WW>), dim3(g), dim3(kBlock), 0, s, a->X, a->Z, a->m,      \
                       a->ld, b->X, b->Z, b->ld, a->W, P, flag.as<uint32_t>());               \
    break;
  switch (a->W) {
    PAULI_CF_CASE(1) PAULI_CF_CASE(2) PAULI_CF_CASE(4) PAULI_CF_CASE(8)
    default:
      hipLaunchKernelGGL((k_comm_flags<kMaxWords>), dim3(g), dim3(kBlock), 0, s, a->X, a->Z,
                         a->m, a->ld, b->X, b->Z, b->ld, a->W, P, flag.as<uint32_t>());
  }
#undef PAULI_CF_CASE
  PAULI_HIP(hipGetLastError());
  scan_exclusive_u32(flag.as<uint32_t>(), off.as<uint32_t>(), P, tot.as<uint32_t>(), work.p, s);
  uint32_t M = 0;
  PAULI_HIP(hipMemcpyAsync(&M, tot.p, 4, hipMemcpyDeviceToHost, s));
  PAULI_HIP(hipStreamSynchronize(s));
  paulisum* o = new_sum(a->n, M, M, a->dtype, s);
  if (M == 0) return o;
  auto Ac = static_cast<const cplx<T>*>(a->coef);
  auto Bc = static_cast<const cplx<T>*>(b->coef);
  auto Oc = static_cast<cplx<T>*>(o->coef);
#define PAULI_CW_CASE(WW)                                                                     \
  case WW:                                                                                    \
    hipLaunchKernelGGL((k_comm_write<WW, T>), dim3(g), dim3(kBlock), 0, s, a->X, a->Z, a->ph,  \
                       Ac, a->fp, a->m, a->ld, b->X, b->Z, b->ph, Bc, b->fp, b->ld, a->W, P,   \
                       flag.as<uint32_t>(), off.as<uint32_t>(), o->X, o->Z, o->ph, Oc, o->fp, \
                       o->ld);                                                                \
    break;
  switch (a->W) {
    PAULI_CW_CASE(1) PAULI_CW_CASE(2) PAULI_CW_CASE(4) PAULI_CW_CASE(8)
    default:
      hipLaunchKernelGGL((k_comm_write<kMaxWords, T>), dim3(g), dim3(kBlock), 0, s, a->X, a->Z,
                         a->ph, Ac, a->fp, a->m, a->ld, b->X, b->Z, b->ph, Bc, b->fp, b->ld,
                         a->W, P, flag.as<uint32_t>(), off.as<uint32_t>(), o->X, o->Z, o->ph, Oc,
                         o->fp, o->ld);
  }
#undef PAULI_CW_CASE
  PAULI_HIP(hipGetLastError());
  return o;
}

}  // namespace

void launch_rows_to_soa(const uint64_t* rows, int W, int64_t m, uint64_t* soa, int64_t ld,
                        hipStream_t s) {
  if (m == 0) return;
  hipLaunchKernelGGL(k_rows_to_soa, dim3(grid_for(m)), dim3(kBlock), 0, s, rows, W, m, soa, ld);
  PAULI_HIP(hipGetLastError());
}

void launch_soa_to_rows(const uint64_t* soa, int W, int64_t m, int64_t ld, uint64_t* rows,
                        hipStream_t s) {
  if (m == 0) return;
  hipLaunchKernelGGL(k_soa_to_rows, dim3(grid_for(m)), dim3(kBlock), 0, s, soa, W, m, ld, rows);
  PAULI_HIP(hipGetLastError());
}

// Bytes [0, n) of p set to zero by a kernel (no memset node in a caller's
// captured graph).
__global__ void k_zero_bytes(uint8_t* __restrict__ p, int64_t n) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    p[t] = 0;
}

void launch_zero_bytes(void* p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_zero_bytes, dim3(static_cast<unsigned>(g)), dim3(kBlock), 0, s,
                     static_cast<uint8_t*>(p), n);
  PAULI_HIP(hipGetLastError());
}

void launch_validate(const uint64_t* xr, const uint64_t* zr, const uint8_t* ph, int n, int64_t m,
                     uint32_t* err, hipStream_t s) {
  if (m == 0) return;
  unsigned g = grid_for(m);
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_validate, dim3(g), dim3(kBlock), 0, s, xr, zr, ph, n, m, err);
  PAULI_HIP(hipGetLastError());
}

void launch_fingerprint(const paulisum* t, hipStream_t s) {
  if (t->m == 0) return;
  unsigned g = grid_for(t->m);
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_fingerprint, dim3(g), dim3(kBlock), 0, s, t->X, t->Z, t->W, t->m, t->ld,
                     t->fp);
  PAULI_HIP(hipGetLastError());
}

void launch_prep_side(const paulisum* t, uint64_t* rows, uint8_t* e, hipStream_t s) {
  if (t->m == 0) return;
  hipLaunchKernelGGL(k_prep_side, dim3(grid_for(t->m)), dim3(kBlock), 0, s, t->X, t->Z, t->ph,
                     t->W, t->m, t->ld, rows, e);
  PAULI_HIP(hipGetLastError());
}

paulisum* commutator_products(const paulisum* a, const paulisum* b, hipStream_t s) {
  if (a->dtype == PAULI_C128) return commutator_products_t<double>(a, b, s);
  return commutator_products_t<float>(a, b, s);
}

void launch_outer_product(const paulisum* a, const paulisum* b, paulisum* o, hipStream_t s) {
  if (a->dtype == PAULI_C128)
    outer_product_t<double>(a, b, o, s);
  else
    outer_product_t<float>(a, b, o, s);
}

}  // namespace pauli
