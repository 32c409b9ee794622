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

struct DevGate {
  int kind, q0, q1, pad;
  uint64_t col[4];  // fingerprint columns of x_q0, z_q0, x_q1, z_q1
};

// The words of the term a thread works on, in LDS: x[w][threadIdx.x].
// A gate's word index is the same for every thread, so the accesses of a
// wave are consecutive (no bank conflicts) and registers are never indexed
// dynamically.
template <int WT>
struct Words {
  uint64_t x[WT][kBlock];
  uint64_t z[WT][kBlock];
};

// One gate's conjugation on the letters of its qubits (letters by Table I:
// (x, z) = (1, 0) X, (0, 1) Z, (1, 1) Y).  Returns 1 when the string's sign
// flips.  The rules are the images of X, Z (and Y = i X Z) under U . U^dag:
//   H:   X <-> Z, Y -> -Y            S:   X -> Y, Y -> -X, Z -> Z
//   S^dag: X -> -Y, Y -> X           X, Y, Z: sign flips on anticommuting letters
//   CX(c,t): X_c -> X_c X_t, Z_t -> Z_c Z_t (X_t, Z_c unchanged)
//   CZ(a,b): X_a -> X_a Z_b, X_b -> Z_a X_b (Z unchanged)
//   SWAP: the two letters exchange places
// Each word the gate touches is read once from LDS and written once.
template <int WT>
__device__ __forceinline__ uint32_t apply_gate(Words<WT>& s, const DevGate& g, uint64_t& fp) {
  const int t = threadIdx.x;
  const bool two = g.kind >= PAULI_GATE_CX;
  const int w0 = g.q0 >> 6, b0 = g.q0 & 63, w1 = g.q1 >> 6, b1 = g.q1 & 63;
  uint64_t xw0 = s.x[w0][t], zw0 = s.z[w0][t];
  uint64_t xw1 = xw0, zw1 = zw0;
  if (two && w1 != w0) {
    xw1 = s.x[w1][t];
    zw1 = s.z[w1][t];
  }
  const uint32_t x0 = static_cast<uint32_t>(xw0 >> b0) & 1u, z0 = static_cast<uint32_t>(zw0 >> b0) & 1u;
  const uint32_t x1 = static_cast<uint32_t>(xw1 >> b1) & 1u, z1 = static_cast<uint32_t>(zw1 >> b1) & 1u;
  uint32_t nx0 = x0, nz0 = z0, nx1 = x1, nz1 = z1, flip = 0;
  switch (g.kind) {
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
  // bit changes as XOR masks, then fingerprint columns of the changed bits
  const uint64_t dx0 = static_cast<uint64_t>(nx0 ^ x0) << b0, dz0 = static_cast<uint64_t>(nz0 ^ z0) << b0;
  const uint64_t dx1 = static_cast<uint64_t>(nx1 ^ x1) << b1, dz1 = static_cast<uint64_t>(nz1 ^ z1) << b1;
  if (dx0) fp ^= g.col[0];
  if (dz0) fp ^= g.col[1];
  if (two) {
    if (dx1) fp ^= g.col[2];
    if (dz1) fp ^= g.col[3];
  }
  if (two && w1 == w0) {
    s.x[w0][t] = xw0 ^ dx0 ^ dx1;
    s.z[w0][t] = zw0 ^ dz0 ^ dz1;
  } else {
    s.x[w0][t] = xw0 ^ dx0;
    s.z[w0][t] = zw0 ^ dz0;
    if (two) {
      s.x[w1][t] = xw1 ^ dx1;
      s.z[w1][t] = zw1 ^ dz1;
    }
  }
  return flip;
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
      s.x[w][tid] = w < nw ? X[w * ld + t] : 0ull;
      s.z[w][tid] = w < nw ? Z[w * ld + t] : 0ull;
    }
    uint64_t f = fp[t];
    uint32_t flips = 0;
    // every thread reads the same gate: uniform (scalar) loads
#pragma unroll 4
    for (int i = 0; i < ngates; ++i) flips += apply_gate<WT>(s, gates[i], f);
#pragma unroll
    for (int w = 0; w < WT; ++w)
      if (w < nw) {
        OX[w * ldo + t] = s.x[w][tid];
        OZ[w * ldo + t] = s.z[w][tid];
      }
    Oph[t] = static_cast<uint8_t>((ph[t] + 2 * flips) & 3);
    Oc[t] = c[t];
    Ofp[t] = f;
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

}  // namespace

paulisum* apply_clifford(const paulisum* s, const pauli_gate_t* gates, int32_t n_gates,
                         hipStream_t st) {
  std::vector<DevGate> dg(static_cast<size_t>(n_gates));
  for (int32_t i = 0; i < n_gates; ++i) {
    const pauli_gate_t& g = gates[i];
    DevGate& d = dg[static_cast<size_t>(i)];
    d.kind = g.kind;
    d.q0 = g.q0;
    d.q1 = g.kind >= PAULI_GATE_CX ? g.q1 : g.q0;
    d.pad = 0;
    d.col[0] = fp_column(2 * d.q0);
    d.col[1] = fp_column(2 * d.q0 + 1);
    d.col[2] = fp_column(2 * d.q1);
    d.col[3] = fp_column(2 * d.q1 + 1);
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
