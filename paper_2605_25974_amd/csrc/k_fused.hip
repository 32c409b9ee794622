// Fused outer product + sort-and-combine of one pair of sums: the host
// side of the staged pipeline whose kernels are in fused_kernels.h and
// expand.h.
#include <cmath>
#include <type_traits>
#include <utility>

#include "fused_kernels.h"

namespace pauli {

namespace {

// ------------------------------------------------------------------- host

template <typename T>
struct SidePrep {
  DBuf rows, aux, key, cls, cls2, idx, idx2, skey, top, ki, g, gs;
  uint32_t* sidx = nullptr;
};

template <typename T>
void prep_side(const paulisum* t, int Wp, int kb, int d1, SidePrep<T>& P, hipStream_t s) {
  const uint32_t m = static_cast<uint32_t>(t->m);
  const uint32_t nc = 1u << d1;
  P.rows = DBuf(static_cast<size_t>(m) * slot_words(Wp) * 8, s);
  P.aux = DBuf(static_cast<size_t>(m) * sizeof(Aux<T>), s);
  P.key = DBuf(m * 8ull, s);
  P.cls = DBuf(m * 8ull, s);
  P.cls2 = DBuf(m * 8ull, s);
  P.idx = DBuf(m * 4ull, s);
  P.idx2 = DBuf(m * 4ull, s);
  P.skey = DBuf(m * 8ull, s);
  P.top = DBuf(m * 2ull, s);
  P.ki = DBuf(m * 16ull, s);
  P.g = DBuf(nc * 4ull, s);
  P.gs = DBuf(nc * 4ull + 4, s);
  hipLaunchKernelGGL(k_fprep<T>, dim3(grid_for(m)), dim3(kB), 0, s, t->X, t->Z, t->ph,
                     static_cast<const cplx<T>*>(t->coef), t->fp, t->W, Wp, t->ld, m, 64 - kb,
                     kb - d1, d1, P.rows.template as<uint64_t>(), P.aux.template as<Aux<T>>(),
                     P.key.template as<uint64_t>(), P.cls.template as<uint64_t>(),
                     P.idx.template as<uint32_t>());
  PAULI_HIP(hipGetLastError());
  P.sidx = P.idx.template as<uint32_t>();
  uint64_t* scls = P.cls.template as<uint64_t>();
  if (d1 > 0) {
    DBuf w(radix_workspace_bytes(m), s);
    if (radix_sort_pairs(P.cls.template as<uint64_t>(), P.idx.template as<uint32_t>(),
                         P.cls2.template as<uint64_t>(), P.idx2.template as<uint32_t>(), m, d1,
                         w.p, s)) {
      P.sidx = P.idx2.template as<uint32_t>();
      scls = P.cls2.template as<uint64_t>();
    }
  }
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(nc)), dim3(kB), 0, s, P.g.template as<uint32_t>(),
                     nc, 0u);
  hipLaunchKernelGGL(k_class_count, dim3(grid_for(m)), dim3(kB), 0, s, scls, m,
                     P.g.template as<uint32_t>());
  DBuf w2(scan_workspace_bytes(nc), s);
  scan_exclusive_u32(P.g.template as<uint32_t>(), P.gs.template as<uint32_t>(), nc,
                     P.gs.template as<uint32_t>() + nc, w2.p, s);
  hipLaunchKernelGGL(k_gather_keys, dim3(grid_for(m)), dim3(kB), 0, s,
                     P.key.template as<uint64_t>(), P.sidx, m, kb, P.skey.template as<uint64_t>(),
                     P.top.template as<uint16_t>(), P.ki.template as<uint4>());
  PAULI_HIP(hipGetLastError());
}

template <int G, int WT, typename T, int MODE>
paulisum* fused_t(const paulisum* a, const paulisum* b, const MergeArgs& o, hipStream_t s) {
  using TV = typename std::conditional<MODE == kComp, float, T>::type;
  const int W = a->W;
  const int Wp = G;  // G == 1 iff W == 1; otherwise the next power of two >= W
  const uint32_t P = static_cast<uint32_t>(a->m * b->m);  // bound on the records
  // a sum times itself: one record per unordered pair (i, j), i <= j, in
  // about half of the class tiles; the values carry the factor 2, 1 or 0
  // (a commutator takes every ordered pair: [a, a] sums to zero pair by pair)
  const bool same = a == b && !o.comm;
  const int form = o.comm ? kFormComm : (same ? kFormSym : kFormProduct);
  const double Peff = same ? 0.5 * P : double(P);
  const int kb = o.key_bits;
  int d = o.bucket_bits > 0 ? o.bucket_bits : fused_default_bucket_bits(int64_t(Peff), kb);
  if (d > kMaxBits) d = kMaxBits;
  if (d > kb) d = kb;
  const int d1 = d < 8 ? d : 8;
  const int d2 = d - d1;
  const uint32_t nc = 1u << d1;
  const uint32_t nbk = 1u << d;
  const int rem = kb - d;  // key bits below the bucket bits
  const SortField sf = sort_field_for(rem);

  // pair id: (j << ibits) | i when that fits in 32 bits, else j*|a| + i
  int ibits = 0;
  while ((int64_t(1) << ibits) < a->m) ++ibits;
  if ((static_cast<uint64_t>(b->m) << ibits) > 0xFFFFFFFFull) ibits = -1;

  SidePrep<T> A, B;
  {
    StageScope sc(PAULI_STAGE_PREP, s, (a->m + (same ? 0 : b->m)) * (16.0 * W + 32.0 * 2));
    prep_side<T>(a, Wp, kb, d1, A, s);
    if (!same) prep_side<T>(b, Wp, kb, d1, B, s);
  }
  const SidePrep<T>& Bs = same ? A : B;

  DBuf keys(P * 8ull, s), vals(P * 4ull, s), keys2(P * 8ull, s), vals2(P * 4ull, s);
  DBuf Tt(static_cast<size_t>(nc) * nc * 4, s), S(nc * 4ull, s), soff(nc * 4ull + 4, s);
  DBuf boff((nbk + 1) * 4ull, s), ctr(64, s);
  // [0] heavy count [1] long count [2] err [3] total [4] expand work items [6] radix redo count
  uint32_t* ctr32 = ctr.as<uint32_t>();
  uint64_t* K = keys.as<uint64_t>();
  uint32_t* V = vals.as<uint32_t>();
  uint64_t* K2 = keys2.as<uint64_t>();
  uint32_t* V2 = vals2.as<uint32_t>();
  {
    StageScope sc(PAULI_STAGE_SORT, s, Peff * 12.0);  // each record written once
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, ctr32, 16u, 0u);
    hipLaunchKernelGGL(k_tile_table, dim3(nc), dim3(kB), 0, s, A.g.template as<uint32_t>(),
                       Bs.g.template as<uint32_t>(), d1, int(same), Tt.as<uint32_t>(),
                       S.as<uint32_t>());
    DBuf w(scan_workspace_bytes(nc), s);
    scan_exclusive_u32(S.as<uint32_t>(), soff.as<uint32_t>(), nc, soff.as<uint32_t>() + nc, w.p,
                       s);
    if (d2 == 0)  // the super-buckets are the buckets
      hipLaunchKernelGGL(k_gen, dim3(grid_for(static_cast<int64_t>(nc) * nc, 1, 16384)), dim3(kB),
                         0, s, A.g.template as<uint32_t>(), A.gs.template as<uint32_t>(), A.sidx,
                         A.skey.template as<uint64_t>(), Bs.g.template as<uint32_t>(),
                         Bs.gs.template as<uint32_t>(), Bs.sidx, Bs.skey.template as<uint64_t>(),
                         Tt.as<uint32_t>(), soff.as<uint32_t>(), d1, int(same),
                         static_cast<uint32_t>(a->m), ibits, K, V);
    PAULI_HIP(hipGetLastError());
    if (d2 > 0) {
      // the records are generated straight into their buckets
      DBuf nt(nc * 4ull, s), tb(nc * 4ull + 4, s);
      hipLaunchKernelGGL(k_tiles_per_sb, dim3(grid_for(nc)), dim3(kB), 0, s, S.as<uint32_t>(), nc,
                         nt.as<uint32_t>());
      scan_exclusive_u32(nt.as<uint32_t>(), tb.as<uint32_t>(), nc, tb.as<uint32_t>() + nc, w.p,
                         s);
      const uint32_t gb = P / kTile + nc + 1;  // bound on the number of tiles
      DBuf C(static_cast<size_t>(gb) * 256 * 4, s);
      const int shift = kb - d;
      const uint32_t mask = (1u << d2) - 1u;
      GenSides gs{A.g.template as<uint32_t>(), A.gs.template as<uint32_t>(),
                  A.ki.template as<uint4>(), Bs.g.template as<uint32_t>(),
                  Bs.gs.template as<uint32_t>(), Bs.ki.template as<uint4>(), Tt.as<uint32_t>(),
                  static_cast<uint32_t>(a->m), ibits, d1, A.top.template as<uint16_t>(),
                  Bs.top.template as<uint16_t>(), 16 - d};
      hipLaunchKernelGGL(k_gcount, dim3(gb), dim3(kGenNT), 0, s, gs, GenBatch{}, S.as<uint32_t>(),
                         tb.as<uint32_t>(), nc, shift, mask, C.as<uint32_t>());
      DBuf w3(scan_workspace_bytes(static_cast<int64_t>(gb) * 256), s);
      scan_exclusive_u32(C.as<uint32_t>(), C.as<uint32_t>(), static_cast<int64_t>(gb) * 256,
                         nullptr, w3.p, s);
      hipLaunchKernelGGL(k_gscatter, dim3(gb), dim3(kGenNT), 0, s, gs, GenBatch{}, K2, V2,
                         S.as<uint32_t>(),
                         tb.as<uint32_t>(), nc, shift, mask, C.as<uint32_t>());
      hipLaunchKernelGGL(k_bucket_offsets, dim3(grid_for(nbk + 1)), dim3(kB), 0, s,
                         soff.as<uint32_t>(), tb.as<uint32_t>(), C.as<uint32_t>(), d2, nbk, nc,
                         boff.as<uint32_t>());
      PAULI_HIP(hipGetLastError());
      std::swap(K, K2);
      std::swap(V, V2);
    } else {
      PAULI_HIP(hipMemcpyAsync(boff.p, soff.p, (nbk + 1) * 4ull, hipMemcpyDeviceToDevice, s));
    }
  }

  DBuf segidx(P * 4ull, s), nseg(nbk * 4ull + 4, s), segoff(nbk * 4ull + 4, s);
  DBuf heavy(nbk * 4ull, s), redo(nbk * 4ull, s);
  DBuf long_list(static_cast<size_t>(P / kLong + 2) * 8, s);
  SegOut so{V, segidx.as<uint32_t>(), nseg.as<uint32_t>(), long_list.as<uint32_t>(), ctr32 + 1};
  {
    StageScope sc(PAULI_STAGE_SEGMENT, s, Peff * 20.0);
    // two blocks per compute unit (the LDS of a block fills about half of one)
    const uint32_t cus = kSortBlocksPerCU * device_cus();
    const uint32_t gsort = nbk < cus ? nbk : cus;
    if (sf.locnt >= 0) {
      // the buckets the counting sort gives up on take the radix sort
      hipLaunchKernelGGL(k_bucket_count, dim3(gsort), dim3(kSortNT), 0, s, K, boff.as<uint32_t>(),
                         nbk, sf, SortBatch{}, so, heavy.as<uint32_t>(), ctr32, redo.as<uint32_t>(),
                         ctr32 + 6);
      // (usually none: a few blocks)
      hipLaunchKernelGGL(k_bucket_radix, dim3(gsort), dim3(kSortNT), 0, s, K,
                         boff.as<uint32_t>(), nbk, redo.as<uint32_t>(), ctr32 + 6, sf, SortBatch{}, so,
                         heavy.as<uint32_t>(), ctr32);
    } else {
      hipLaunchKernelGGL(k_bucket_radix, dim3(gsort), dim3(kSortNT), 0, s, K, boff.as<uint32_t>(),
                         nbk, nullptr, nullptr, sf, SortBatch{}, so, heavy.as<uint32_t>(), ctr32);
    }
    // as many blocks as the counting sort: a workload of many equal strings
    // can make most buckets heavy
    hipLaunchKernelGGL(k_heavy_sort, dim3(gsort), dim3(kSortNT), 0, s, K, K2, V2,
                       boff.as<uint32_t>(), rem, SortBatch{}, heavy.as<uint32_t>(), ctr32, so);
    PAULI_HIP(hipGetLastError());
    DBuf w(scan_workspace_bytes(nbk), s);
    scan_exclusive_u32(nseg.as<uint32_t>(), segoff.as<uint32_t>(), nbk,
                       segoff.as<uint32_t>() + nbk, w.p, s);
    PAULI_HIP(hipMemcpyAsync(ctr32 + 3, segoff.as<uint32_t>() + nbk, 4, hipMemcpyDeviceToDevice, s));
  }
  uint32_t host[4];
  PAULI_HIP(hipMemcpyAsync(host, ctr32, sizeof(host), hipMemcpyDeviceToHost, s));
  PAULI_HIP(hipStreamSynchronize(s));
  const uint32_t U = host[3];

  // the leading dimension is a multiple of the store block, so that blocks
  // of every output array start on a 256-byte boundary
  const int64_t ldo = (static_cast<int64_t>(U) + kBS - 1) / kBS * kBS;
  paulisum* out = new_sum(a->n, U, ldo, MODE == kComp ? PAULI_C64 : a->dtype, s);
  ExpandArgs E{boff.as<uint32_t>(), V, segidx.as<uint32_t>(), segoff.as<uint32_t>(), nbk,
               ctr32 + 2, ctr32 + 4, out->X, out->Z, out->ph, out->coef, out->fp, out->ld, o.tau,
               o.comm};
  Operands<WT, T> op{A.rows.template as<uint64_t>(), Bs.rows.template as<uint64_t>(),
                     A.aux.template as<Aux<T>>(), Bs.aux.template as<Aux<T>>(),
                     static_cast<uint32_t>(a->m), ibits, W, form};
  {
    // HBM bytes: ids and segment indices read per record, and per segment
    // the merged term written; a commutator writes only the phase byte of
    // the segments it removes later (their number is not known here, so its
    // count is the lower bound of one byte per segment)
    StageScope sc(PAULI_STAGE_WRITE, s,
                  (o.comm ? U * 1.0 : U * (16.0 * W + sizeof(cplx<TV>) + 1 + 8)) + Peff * 8.0);
    // merged terms carry phase 0 (the block of phase bytes is padded to 256)
    if (U > 0)
      hipLaunchKernelGGL(k_fill_u32, dim3(grid_for((U + 3) / 4)), dim3(kB), 0, s,
                         reinterpret_cast<uint32_t*>(out->ph), (U + 3) / 4, 0u);
    hipLaunchKernelGGL((k_expand<G, WT, T, MODE>), dim3(nbk < 1024u ? nbk : 1024u), dim3(kB), 0, s, E,
                       op);
    PAULI_HIP(hipGetLastError());
  }
  {
    StageScope sc(PAULI_STAGE_LONG, s, 0.0);
    const uint32_t nlong = host[1];  // the segment stage listed them all
    if (nlong > 0)
      hipLaunchKernelGGL((k_expand_long<G, WT, T, MODE>), dim3(nlong < 256u ? nlong : 256u),
                         dim3(kLongB), 0, s, E, op, long_list.as<uint32_t>(), ctr32 + 1);
    PAULI_HIP(hipGetLastError());
  }
  PAULI_HIP(hipMemcpyAsync(host, ctr32, sizeof(host), hipMemcpyDeviceToHost, s));
  PAULI_HIP(hipStreamSynchronize(s));
  if (host[2] != 0) {
    free_sum(out);
    return nullptr;  // a fingerprint collision: the caller uses the general path
  }
  return out;
}

template <typename T, int MODE>
paulisum* fused_w(const paulisum* a, const paulisum* b, const MergeArgs& o, hipStream_t s) {
  switch (a->W) {
    case 1: return fused_t<1, 1, T, MODE>(a, b, o, s);
    case 2: return fused_t<2, 2, T, MODE>(a, b, o, s);
    case 3: return fused_t<4, 3, T, MODE>(a, b, o, s);
    case 4: return fused_t<4, 4, T, MODE>(a, b, o, s);
    case 5: return fused_t<8, 5, T, MODE>(a, b, o, s);
    case 6: return fused_t<8, 6, T, MODE>(a, b, o, s);
    case 7: return fused_t<8, 7, T, MODE>(a, b, o, s);
    case 8: return fused_t<8, 8, T, MODE>(a, b, o, s);
    default: return fused_t<16, kMaxWords, T, MODE>(a, b, o, s);
  }
}

}  // namespace

int fused_default_bucket_bits(int64_t p, int key_bits) {
  int d = 0;
  if (p > kTargetBucket) d = static_cast<int>(std::ceil(std::log2(p / kTargetBucket)));
  if (d > kMaxBits) d = kMaxBits;
  if (d > key_bits) d = key_bits;
  return d;
}

namespace {

// boff[b] = first record whose key has top bits >= b (keys in bucket order),
// boff[nbk] = n.
__global__ void k_bucket_bounds(const uint64_t* __restrict__ keys, int64_t n,
                                const uint32_t* __restrict__ nd, int shift, uint32_t nbk,
                                uint32_t* __restrict__ boff) {
  if (nd && *nd < n) n = *nd;  // the device count, clamped to the host bound
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r <= n;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t cur = r < n ? static_cast<int64_t>(keys[r] >> shift) : nbk;
    const int64_t prev = r > 0 ? static_cast<int64_t>(keys[r - 1] >> shift) : -1;
    for (int64_t b = prev + 1; b <= cur; ++b) boff[b] = static_cast<uint32_t>(r);
  }
}

}  // namespace

bool sort_records_bucketed(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt,
                           uint32_t* vals_alt, int64_t n, int key_bits, hipStream_t s,
                           const uint32_t* nd) {
  // small sorts: the radix passes (the bucket pipeline's fixed costs dominate)
  if (n < (int64_t(1) << 16) || key_bits < 24 || n > 0xFFFFFFFFll) {
    DBuf w(radix_workspace_bytes(n), s);
    return radix_sort_pairs(keys, vals, keys_alt, vals_alt, n, key_bits, w.p, s, ~0ull, nd);
  }
  const int d = fused_default_bucket_bits(n, key_bits);
  if (d == 0) {
    DBuf w(radix_workspace_bytes(n), s);
    return radix_sort_pairs(keys, vals, keys_alt, vals_alt, n, key_bits, w.p, s, ~0ull, nd);
  }
  const uint32_t nbk = 1u << d;
  bool alt = false;
  {  // partition on the top d bits: stable passes on 8-bit digits
    int shifts[2];
    int ns = 0;
    shifts[ns++] = key_bits - d;
    if (d > 8) shifts[ns++] = key_bits - d + 8;
    DBuf w(radix_workspace_bytes(n), s);
    alt = radix_sort_at(keys, vals, keys_alt, vals_alt, n, shifts, ns, w.p, s, nd);
  }
  uint64_t* K = alt ? keys_alt : keys;
  uint32_t* V = alt ? vals_alt : vals;
  uint64_t* K2 = alt ? keys : keys_alt;
  uint32_t* V2 = alt ? vals : vals_alt;
  DBuf boff((nbk + 1) * 4ull, s), ctr(64, s), heavy(nbk * 4ull, s), redo(nbk * 4ull, s);
  uint32_t* ctr32 = ctr.as<uint32_t>();  // [0] heavy count [6] radix redo count
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, ctr32, 16u, 0u);
  hipLaunchKernelGGL(k_bucket_bounds, dim3(grid_for(n + 1)), dim3(kB), 0, s, K, n, nd,
                     key_bits - d, nbk, boff.as<uint32_t>());
  PAULI_HIP(hipGetLastError());
  const int rem = key_bits - d;
  const SortField sf = sort_field_for(rem);
  SegOut so{V, nullptr, nullptr, nullptr, nullptr, K};
  StageScope sc(PAULI_STAGE_SORT, s, n * 24.0);
  const uint32_t cus = kSortBlocksPerCU * device_cus();
  const uint32_t gsort = nbk < cus ? nbk : cus;
  if (sf.locnt >= 0) {
    hipLaunchKernelGGL(k_bucket_count, dim3(gsort), dim3(kSortNT), 0, s, K, boff.as<uint32_t>(),
                       nbk, sf, SortBatch{}, so, heavy.as<uint32_t>(), ctr32, redo.as<uint32_t>(),
                         ctr32 + 6);
    hipLaunchKernelGGL(k_bucket_radix, dim3(gsort), dim3(kSortNT), 0, s, K,
                       boff.as<uint32_t>(), nbk, redo.as<uint32_t>(), ctr32 + 6, sf, SortBatch{}, so,
                       heavy.as<uint32_t>(), ctr32);
  } else {
    hipLaunchKernelGGL(k_bucket_radix, dim3(gsort), dim3(kSortNT), 0, s, K, boff.as<uint32_t>(),
                       nbk, nullptr, nullptr, sf, SortBatch{}, so, heavy.as<uint32_t>(), ctr32);
  }
  hipLaunchKernelGGL(k_heavy_sort, dim3(gsort), dim3(kSortNT), 0, s, K, K2, V2,
                     boff.as<uint32_t>(), rem, SortBatch{}, heavy.as<uint32_t>(), ctr32, so);
  PAULI_HIP(hipGetLastError());
  return alt;
}

paulisum* fused_bucket(const paulisum* a, const paulisum* b, const MergeArgs& o, hipStream_t s) {
  paulisum* r;
  if (o.mode == PAULI_MERGE_COMPENSATED)
    r = a->dtype == PAULI_C128 ? fused_w<double, kComp>(a, b, o, s) : fused_w<float, kComp>(a, b, o, s);
  else
    r = a->dtype == PAULI_C128 ? fused_w<double, kPlain>(a, b, o, s)
                               : fused_w<float, kPlain>(a, b, o, s);
  if (r && (o.drop_abs >= 0.0 || o.comm)) {
    // the strict drop, and for a commutator the terms no record kept
    StageScope sc(PAULI_STAGE_LONG, s, r->m * (16.0 * r->W + coef_bytes(r->dtype) + 9) * 2);
    paulisum* kept = nullptr;
    try {
      kept = drop_terms(r, o.drop_abs, s, o.comm != 0);
    } catch (...) {
      free_sum(r);
      throw;
    }
    free_sum(r);
    r = kept;
  }
  return r;
}

}  // namespace pauli
