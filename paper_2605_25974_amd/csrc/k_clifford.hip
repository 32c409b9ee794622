// Clifford gates on a Pauli sum (Section III-B, Clifford paragraph: a
// Clifford conjugation maps every string to one string and keeps the number
// of terms; Section V-B: H, S, CNOT, CZ relabel strings in place; Section
// IV-B: on the struct-of-arrays layout the update is a branch-free loop over
// the words of independent terms).
//
// Term t becomes C (i^k P) C^dagger with C = G_{L-1} ... G_1 G_0: the gates
// conjugate the strings in list order.  Per gate only the bits of its
// qubits change, and the sign of the string may flip (phase k += 2); the
// fingerprint is updated by the columns of the bits that change.
#include "common.h"
#include "internal.h"

namespace pauli {

namespace {

constexpr int kBlock = 256;

// A gate as two lookup tables over the four letter bits it reads,
// idx = x0 | z0 << 1 | x1 << 2 | z1 << 3 (qubit q0's letter, then q1's;
// a one-qubit gate has q1 = q0 and leaves bits 2 and 3 as they are): the
// new bits are 4-bit entry idx of the 64-bit table (tlo holds entries 0-7,
// thi 8-15), and bit idx of ftab says whether the string's sign flips.
// Every gate is then the same branch-free update, done on 32-bit halves of
// the packed words: qubit q is bit q % 32 of half-word q / 32.
struct DevGate {
  int w0, b0, w1, b1;  // half-word and bit of q0 and of q1
  uint32_t tlo, thi, ftab, pad;
  uint32_t col[8];  // fingerprint columns of x_q0, z_q0, x_q1, z_q1 as (low, high) halves
};

// The half-words of the term a thread works on, in LDS: x[h][threadIdx.x].
// A gate's half-word index is the same for every thread, so the accesses of
// a wave are consecutive (no bank conflicts) and registers are never
// indexed dynamically.
template <int WT>
struct Words {
  uint32_t x[2 * WT][kBlock];
  uint32_t z[2 * WT][kBlock];
};

// One gate on a term: each half-word the gate touches is read once from LDS
// and written once; the fingerprint halves take the columns of the bits
// that change.  Returns 1 when the string's sign flips.
template <int WT>
__device__ __forceinline__ uint32_t apply_gate(Words<WT>& s, const DevGate& g, uint32_t& flo,
                                               uint32_t& fhi) {
  const int t = threadIdx.x;
  const int w0 = g.w0, b0 = g.b0, w1 = g.w1, b1 = g.b1;
  const uint32_t xa = s.x[w0][t], za = s.z[w0][t];
  uint32_t xb = xa, zb = za;
  if (w1 != w0) {
    xb = s.x[w1][t];
    zb = s.z[w1][t];
  }
  const uint32_t idx = ((xa >> b0) & 1u) | (((za >> b0) & 1u) << 1) | (((xb >> b1) & 1u) << 2) |
                       (((zb >> b1) & 1u) << 3);
  const uint32_t tw = idx < 8u ? g.tlo : g.thi;
  const uint32_t d = ((tw >> (4u * (idx & 7u))) & 15u) ^ idx;  // changed bits
  const uint32_t m0 = 0u - (d & 1u), m1 = 0u - ((d >> 1) & 1u);
  const uint32_t m2 = 0u - ((d >> 2) & 1u), m3 = 0u - (d >> 3);
  flo ^= (g.col[0] & m0) ^ (g.col[2] & m1) ^ (g.col[4] & m2) ^ (g.col[6] & m3);
  fhi ^= (g.col[1] & m0) ^ (g.col[3] & m1) ^ (g.col[5] & m2) ^ (g.col[7] & m3);
  const uint32_t dx0 = (d & 1u) << b0, dz0 = ((d >> 1) & 1u) << b0;
  const uint32_t dx1 = ((d >> 2) & 1u) << b1, dz1 = (d >> 3) << b1;
  if (w1 == w0) {
    s.x[w0][t] = xa ^ dx0 ^ dx1;
    s.z[w0][t] = za ^ dz0 ^ dz1;
  } else {
    s.x[w0][t] = xa ^ dx0;
    s.z[w0][t] = za ^ dz0;
    s.x[w1][t] = xb ^ dx1;
    s.z[w1][t] = zb ^ dz1;
  }
  return (g.ftab >> idx) & 1u;
}

template <int WT, typename T>
__global__ void __launch_bounds__(kBlock)
k_clifford(const uint64_t* __restrict__ X, const uint64_t* __restrict__ Z,
           const uint8_t* __restrict__ ph, const cplx<T>* __restrict__ c,
           const uint64_t* __restrict__ fp, int64_t m, int64_t ld, int nw,
           const DevGate* __restrict__ gates, int ngates,
           uint64_t* __restrict__ OX, uint64_t* __restrict__ OZ, uint8_t* __restrict__ Oph,
           cplx<T>* __restrict__ Oc, uint64_t* __restrict__ Ofp, int64_t ldo) {
  __shared__ Words<WT> s;
  const int tid = threadIdx.x;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + tid; t < m;
       t += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int w = 0; w < WT; ++w) {
      const uint64_t xv = w < nw ? X[w * ld + t] : 0ull;
      const uint64_t zv = w < nw ? Z[w * ld + t] : 0ull;
      s.x[2 * w][tid] = static_cast<uint32_t>(xv);
      s.x[2 * w + 1][tid] = static_cast<uint32_t>(xv >> 32);
      s.z[2 * w][tid] = static_cast<uint32_t>(zv);
      s.z[2 * w + 1][tid] = static_cast<uint32_t>(zv >> 32);
    }
    const uint64_t f0 = fp[t];
    uint32_t flo = static_cast<uint32_t>(f0), fhi = static_cast<uint32_t>(f0 >> 32);
    uint32_t flips = 0;
    // every thread reads the same gate: uniform (scalar) loads, the next
    // gate's issued before the current one is applied
    if (ngates > 0) {
      DevGate g = gates[0];
      for (int i = 0; i < ngates; ++i) {
        const DevGate nx = gates[i + 1 < ngates ? i + 1 : i];
        flips += apply_gate<WT>(s, g, flo, fhi);
        g = nx;
      }
    }
#pragma unroll
    for (int w = 0; w < WT; ++w)
      if (w < nw) {
        OX[w * ldo + t] = s.x[2 * w][tid] | (static_cast<uint64_t>(s.x[2 * w + 1][tid]) << 32);
        OZ[w * ldo + t] = s.z[2 * w][tid] | (static_cast<uint64_t>(s.z[2 * w + 1][tid]) << 32);
      }
    Oph[t] = static_cast<uint8_t>((ph[t] + 2 * flips) & 3);
    Oc[t] = c[t];
    Ofp[t] = flo | (static_cast<uint64_t>(fhi) << 32);
  }
}

template <typename T>
void clifford_t(const paulisum* s, const DevGate* dg, int ngates, paulisum* o, hipStream_t st) {
  const int64_t m = s->m;
  int64_t g = (m + kBlock - 1) / kBlock;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  const int W = s->W;
  StageScope sc(PAULI_STAGE_CLIFFORD, st, m * 2.0 * (16.0 * W + 1 + 8 + sizeof(cplx<T>)));
  auto Ic = static_cast<const cplx<T>*>(s->coef);
  auto Oc = static_cast<cplx<T>*>(o->coef);
#define PAULI_CL_CASE(WW)                                                                     \
  case WW:                                                                                    \
    hipLaunchKernelGGL((k_clifford<WW, T>), dim3(static_cast<unsigned>(g)), dim3(kBlock), 0,   \
                       st, s->X, s->Z, s->ph, Ic, s->fp, m, s->ld, W, dg, ngates, o->X, o->Z,  \
                       o->ph, Oc, o->fp, o->ld);                                              \
    break;
  switch (W <= 1 ? 1 : W <= 2 ? 2 : W <= 4 ? 4 : W <= 8 ? 8 : 16) {
    PAULI_CL_CASE(1) PAULI_CL_CASE(2) PAULI_CL_CASE(4) PAULI_CL_CASE(8) PAULI_CL_CASE(16)
  }
#undef PAULI_CL_CASE
  PAULI_HIP(hipGetLastError());
}

// The tables of a gate kind.  The rules are the images of X, Z (and
// Y = i X Z) under U . U^dag, letters by Table I ((x, z) = (1, 0) X,
// (0, 1) Z, (1, 1) Y):
//   H:   X <-> Z, Y -> -Y            S:   X -> Y, Y -> -X, Z -> Z
//   S^dag: X -> -Y, Y -> X           X, Y, Z: sign flips on anticommuting letters
//   CX(c,t): X_c -> X_c X_t, Z_t -> Z_c Z_t (X_t, Z_c unchanged)
//   CZ(a,b): X_a -> X_a Z_b, X_b -> Z_a X_b (Z unchanged)
//   SWAP: the two letters exchange places
void gate_tables(int kind, uint64_t* tab, uint32_t* ftab) {
  *tab = 0;
  *ftab = 0;
  for (uint32_t idx = 0; idx < 16; ++idx) {
    const uint32_t x0 = idx & 1u, z0 = (idx >> 1) & 1u, x1 = (idx >> 2) & 1u, z1 = (idx >> 3) & 1u;
    uint32_t nx0 = x0, nz0 = z0, nx1 = x1, nz1 = z1, flip = 0;
    switch (kind) {
      case PAULI_GATE_H:
        nx0 = z0; nz0 = x0; flip = x0 & z0;
        break;
      case PAULI_GATE_S:
        nz0 = z0 ^ x0; flip = x0 & z0;
        break;
      case PAULI_GATE_SDG:
        nz0 = z0 ^ x0; flip = x0 & (z0 ^ 1u);
        break;
      case PAULI_GATE_X:
        flip = z0;
        break;
      case PAULI_GATE_Y:
        flip = x0 ^ z0;
        break;
      case PAULI_GATE_Z:
        flip = x0;
        break;
      case PAULI_GATE_CX:
        nx1 = x1 ^ x0; nz0 = z0 ^ z1; flip = x0 & z1 & (x1 ^ z0 ^ 1u);
        break;
      case PAULI_GATE_CZ:
        nz0 = z0 ^ x1; nz1 = z1 ^ x0; flip = x0 & x1 & (z0 ^ z1);
        break;
      default:  // PAULI_GATE_SWAP
        nx0 = x1; nz0 = z1; nx1 = x0; nz1 = z0;
        break;
    }
    const uint64_t out = nx0 | (nz0 << 1) | (nx1 << 2) | (nz1 << 3);
    *tab |= out << (4 * idx);
    *ftab |= flip << idx;
  }
}

}  // namespace

paulisum* apply_clifford(const paulisum* s, const pauli_gate_t* gates, int32_t n_gates,
                         hipStream_t st) {
  std::vector<DevGate> dg(static_cast<size_t>(n_gates));
  for (int32_t i = 0; i < n_gates; ++i) {
    const pauli_gate_t& g = gates[i];
    DevGate& d = dg[static_cast<size_t>(i)];
    const int q0 = g.q0, q1 = g.kind >= PAULI_GATE_CX ? g.q1 : g.q0;
    d.w0 = q0 >> 5;
    d.b0 = q0 & 31;
    d.w1 = q1 >> 5;
    d.b1 = q1 & 31;
    uint64_t tab = 0;
    gate_tables(g.kind, &tab, &d.ftab);
    d.tlo = static_cast<uint32_t>(tab);
    d.thi = static_cast<uint32_t>(tab >> 32);
    d.pad = 0;
    const uint64_t cols[4] = {fp_column(2 * q0), fp_column(2 * q0 + 1), fp_column(2 * q1),
                              fp_column(2 * q1 + 1)};
    for (int k = 0; k < 4; ++k) {
      d.col[2 * k] = static_cast<uint32_t>(cols[k]);
      d.col[2 * k + 1] = static_cast<uint32_t>(cols[k] >> 32);
    }
  }
  paulisum* o = new_sum(s->n, s->m, s->m, s->dtype, st);
  if (s->m == 0) return o;
  try {
    DBuf gbuf(dg.size() * sizeof(DevGate) + 16, st);
    if (!dg.empty()) {
      PAULI_HIP(hipMemcpyAsync(gbuf.p, dg.data(), dg.size() * sizeof(DevGate),
                               hipMemcpyHostToDevice, st));
      PAULI_HIP(hipStreamSynchronize(st));  // the host gate list goes out of scope
    }
    if (s->dtype == PAULI_C128)
      clifford_t<double>(s, gbuf.as<DevGate>(), n_gates, o, st);
    else
      clifford_t<float>(s, gbuf.as<DevGate>(), n_gates, o, st);
  } catch (...) {
    free_sum(o);
    throw;
  }
  return o;
}

}  // namespace pauli
