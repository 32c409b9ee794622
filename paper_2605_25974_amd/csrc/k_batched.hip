// Batched form of the fused outer product + sort-and-combine: many products
// out[p] = merge(a[p] * b[p]) of different term counts and qubit counts in
// one launch sequence (the outer product of Section IV-C and the merge of
// Section III-H, product by product).
//
// Products with the same word count W and coefficient type form a class;
// each class runs the stages of the fused pipeline once for all its
// products, every kernel covering every product:
//
//   prep    one launch over the concatenated terms of every operand; the
//           terms are sorted by (sum, class) in one radix sort (the sum
//           index above the class bits).
//   gen     the super-buckets of all products are numbered one after the
//           other (product p owns [sbbase[p], sbbase[p + 1])); one tile
//           table launch, and the partition tiles of every super-bucket of
//           every product form one work list for the generation kernels,
//           which write each record once, into its bucket.  The bucket
//           index is the product's first bucket plus the top d_p key bits
//           of the record: the batch index sits above the key bits of the
//           bucket sort's order.
//   sort    one LDS bucket sort over the buckets of all products (each
//           product has its own bucket bits, so each bucket looks up its
//           product's bit fields).
//   expand  one expand launch over the buckets of all products; each work
//           item looks up its product's operands and output offset.
//
// Outputs go to one block per class with room for |a_p| |b_p| terms per
// product (an upper bound of the merged count), so no size is read on the
// host between stages: the only host read is the per-product term count
// after the whole sequence.  The sequence can therefore be captured once
// into a HIP graph and replayed (a plan).  The results are views into the
// class block, which lives until the last of them is destroyed.
//
// An autotuner picks, per class (W, log2 of the class's records, precision,
// mode), the bucket size (records per LDS bucket sort), the class bits of
// the generation (the rest of the bucket bits are the partition's digit)
// and the expand work items per bucket, by timing each candidate once; the
// choices can be saved to and loaded from a text file.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "fused_kernels.h"

namespace pauli {

namespace {

// ----------------------------------------------------------- prep kernels

// One operand sum of a class, concatenated with the class's other sums of
// the same side.
struct SumDesc {
  const uint64_t* X;
  const uint64_t* Z;
  const uint8_t* ph;
  const void* coef;
  const uint64_t* fp;
  int64_t ld;
  int W;
  int kshift;  // 64 - key bits
  int cshift;  // key bits - d1
  int d1;      // class bits of the sum's product
};

// The sum u holding row r of a side: start[u] <= r < start[u + 1].
__device__ __forceinline__ uint32_t sum_of(const uint32_t* start, int nsums, uint32_t r) {
  uint32_t lo = 0, hi = static_cast<uint32_t>(nsums);
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (start[mid] <= r) lo = mid; else hi = mid;
  }
  return lo;
}

// Rows, metadata and keys of every term of a side (as k_fprep does for one
// sum), and the class sort key (sum index << 8 | class).
template <typename T>
__global__ void k_bprep(const SumDesc* __restrict__ sums, const uint32_t* __restrict__ start,
                        int nsums, uint32_t total, int Wp, uint64_t* __restrict__ rows,
                        Aux<T>* __restrict__ aux, uint64_t* __restrict__ key,
                        uint64_t* __restrict__ ckey, uint32_t* __restrict__ gidx) {
  for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < total;
       r += gridDim.x * blockDim.x) {
    const uint32_t u = sum_of(start, nsums, r);
    const SumDesc& D = sums[u];
    const uint32_t t = r - start[u];
    const int SW = slot_words(Wp);
    int y = 0;
    for (int w = 0; w < Wp; ++w) {
      const uint64_t x = w < D.W ? D.X[w * D.ld + t] : 0ull;
      const uint64_t z = w < D.W ? D.Z[w * D.ld + t] : 0ull;
      rows[static_cast<size_t>(r) * SW + 2 * w] = x;
      rows[static_cast<size_t>(r) * SW + 2 * w + 1] = z;
      y += popc64(x & z);
    }
    const cplx<T> c = static_cast<const cplx<T>*>(D.coef)[t];
    Aux<T> a;
    a.w[0] = to_word<T>(c.re);
    a.w[1] = to_word<T>(c.im);
    a.w[2] = D.fp[t];
    const uint64_t k = D.fp[t] >> D.kshift;
    const uint64_t cid = D.d1 ? (k >> D.cshift) : 0ull;
    a.w[3] = static_cast<uint64_t>((D.ph[t] + y) & 3) | (static_cast<uint64_t>(y & 1) << 2) |
             (cid << 8);
    aux[r] = a;
    if (Wp <= 4)
      for (int q = 0; q < 4; ++q) rows[static_cast<size_t>(r) * SW + 2 * Wp + q] = a.w[q];
    key[r] = k;
    ckey[r] = (static_cast<uint64_t>(u) << 8) | cid;
    gidx[r] = r;
  }
}

// After the class sort: the sorted keys, and each sorted term's index
// inside its own sum (the pair ids are local to a product).
__global__ void k_bgather(const uint64_t* __restrict__ key, const uint32_t* __restrict__ gidx,
                          const uint64_t* __restrict__ ckey, const uint32_t* __restrict__ start,
                          uint32_t total, int kb, uint16_t* __restrict__ top,
                          uint4* __restrict__ ki) {
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += gridDim.x * blockDim.x) {
    const uint32_t r = gidx[q];
    const uint64_t k = key[r];
    top[q] = key_top16(k, kb);
    ki[q] = key_index(k, r - start[ckey[q] >> 8]);
  }
}

// Super-bucket tables of every product (k_tile_table per product): block
// sg is super-bucket sg - sbbase[p] of product p = sbprod[sg].
__global__ void __launch_bounds__(kB)
k_btile_table(const GenSides* __restrict__ gen, const uint16_t* __restrict__ sbprod,
              const uint32_t* __restrict__ sbbase, const uint8_t* __restrict__ sym,
              uint32_t* __restrict__ Tt_all, const uint32_t* __restrict__ ttoff,
              uint32_t* __restrict__ S) {
  __shared__ uint32_t sh[kB / 64];
  const uint32_t sg = blockIdx.x, p = sbprod[sg];
  const GenSides& G = gen[p];
  const uint32_t nc = 1u << G.d1, s = sg - sbbase[p], h = threadIdx.x;
  const bool skip = sym[p] && h > (h ^ s);
  const uint32_t size = h < nc && !skip ? G.gA[h] * G.gB[h ^ s] : 0u;
  uint32_t tot;
  const uint32_t ex = block_excl<kB / 64>(size, &tot, sh);
  if (h < nc) Tt_all[ttoff[p] + s * nc + h] = ex;
  if (h == 0) S[sg] = tot;
}

// First record of every bucket of every product: bucket bl of product p
// is (super-bucket bl >> d2, digit bl & mask) of p.
__global__ void k_bbucket_offsets(const uint16_t* __restrict__ bprod,
                                  const uint32_t* __restrict__ bbase,
                                  const uint32_t* __restrict__ sbbase,
                                  const int* __restrict__ d2tab, const uint32_t* __restrict__ soff,
                                  const uint32_t* __restrict__ tb, const uint32_t* __restrict__ C,
                                  uint32_t nbk, uint32_t nsb, uint32_t* __restrict__ boff) {
  for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b <= nbk;
       b += gridDim.x * blockDim.x) {
    if (b == nbk) {
      boff[b] = soff[nsb];  // all records
      continue;
    }
    const uint32_t p = bprod[b], bl = b - bbase[p];
    const int d2 = d2tab[p];
    const uint32_t s = sbbase[p] + (bl >> d2), dd = bl & ((1u << d2) - 1u);
    const uint32_t ns = tb[s + 1] - tb[s];
    boff[b] = ns ? C[tb[s] * 256u + dd * ns] : soff[s];
  }
}

// Per product: merged terms and collision flag.
__global__ void k_binfo(const uint32_t* __restrict__ segoff, const uint32_t* __restrict__ bbase,
                        const uint32_t* __restrict__ perr, uint32_t np,
                        uint32_t* __restrict__ info) {
  for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < np; p += gridDim.x * blockDim.x) {
    info[2 * p] = segoff[bbase[p + 1]] - segoff[bbase[p]];
    info[2 * p + 1] = perr[p];
  }
}

// ------------------------------------------------------------- host side

struct ClassKey {
  int W, logp, dtype, mode;
  bool operator<(const ClassKey& o) const {
    if (W != o.W) return W < o.W;
    if (logp != o.logp) return logp < o.logp;
    if (dtype != o.dtype) return dtype < o.dtype;
    return mode < o.mode;
  }
};

// Launch-shape parameters of a class.
struct ClassParams {
  double target = kTargetBucket;  // records per bucket
  int d1cap = 8;           // class bits of the generation (at most)
  int parts = 4;           // expand work items per bucket
  int fixed_d = 0;         // > 0: every product's bucket bits
};

std::mutex g_tune_mu;
std::map<ClassKey, ClassParams> g_tune;
bool g_tune_env_loaded = false;

// Device memory carved into 256-byte aligned pieces of one buffer.
struct Carve {
  std::vector<size_t> off;
  size_t total = 0;
  size_t add(size_t bytes) {
    off.push_back(total);
    total += (bytes + 255) & ~size_t(255);
    return off.size() - 1;
  }
};

struct Product {
  int idx;  // position in the batch
  const paulisum* a;
  const paulisum* b;
  bool sym;
  uint32_t m1, m2;
  uint64_t P;    // |a| |b|
  double Peff;   // records: P, or about P / 2 for a sum times itself
  int d, d1, d2, ibits;
  uint32_t uA, uB;      // sum index on each side
  uint32_t sb0, nc;     // first super-bucket, super-buckets
  uint32_t bb0, nbk;    // first bucket, buckets
  uint32_t tt0;         // offset of the tile table
  uint64_t out0;        // first output term (multiple of kBS)
};

// One class: its products, device buffers and launch sequence.
struct ClassRun {
  int W = 0, G = 1;
  uint32_t cus = 1;  // compute units of the device
  int32_t dtype = PAULI_C128;
  int mode = PAULI_MERGE_PLAIN;
  int kb = 64;
  double tau = 1e-3;
  ClassParams par;
  std::vector<Product> prods;
  std::vector<const paulisum*> sumsA, sumsB;
  uint32_t totA = 0, totB = 0;  // terms per side
  uint32_t nsb = 0, nbk = 0, gb = 0;
  uint64_t rec = 0;  // bound on the records (sum of Peff rounded up)
  uint64_t cap = 0;  // output terms of the class block
  DBuf work;         // every table and temporary
  std::shared_ptr<SharedBlock> out;  // the output block
  // pieces of `work`
  struct Side {
    uint64_t* rows;
    void* aux;
    uint64_t *key, *ckey, *ckey2;
    uint16_t* top;  // key_top16 of the keys in class order
    uint4* ki;      // key_index: (key, term index within its sum) in class order
    uint32_t *gidx, *gidx2, *g, *gs;
    SumDesc* desc;
    uint32_t* start;
    void* rwork;
    void* swork;
  } A{}, B{};
  GenSides* gen = nullptr;
  uint16_t *sbprod = nullptr, *bprod = nullptr;
  uint32_t *sbbase = nullptr, *bbase = nullptr, *ttoff = nullptr, *Tt = nullptr;
  uint8_t* sym = nullptr;
  int *shift = nullptr, *d2tab = nullptr;
  uint32_t* mask = nullptr;
  uint32_t *S = nullptr, *soff = nullptr, *nt = nullptr, *tb = nullptr, *C = nullptr;
  void *w_sb = nullptr, *w_tb = nullptr, *w_c = nullptr, *w_seg = nullptr;
  uint64_t *K = nullptr, *K2 = nullptr;
  uint32_t *V = nullptr, *V2 = nullptr;
  uint32_t *boff = nullptr, *segidx = nullptr, *nseg = nullptr, *segoff = nullptr;
  uint32_t *heavy = nullptr, *redo = nullptr, *long_list = nullptr, *ctr = nullptr;
  SortField* sftab = nullptr;
  void* optab = nullptr;
  uint32_t *pout = nullptr, *perr = nullptr, *info = nullptr;
  // host copies of the tables (uploaded once)
  std::vector<uint8_t> host_tables;
  size_t tables_off = 0;  // where in `work` the uploaded tables start
  bool sideB = false;
};

int words_class(int W) { return W <= 8 ? W : kMaxWords; }
int group_of(int W) { return W == 1 ? 1 : (W == 2 ? 2 : (W <= 4 ? 4 : (W <= 8 ? 8 : 16))); }

// Fills the product plan of a class for the given parameters.
void plan_products(ClassRun& cr) {
  uint32_t sb = 0, bb = 0, tt = 0;
  uint64_t out = 0, rec = 0, gb = 1;
  for (auto& p : cr.prods) {
    p.P = static_cast<uint64_t>(p.m1) * p.m2;
    p.Peff = p.sym ? 0.5 * static_cast<double>(p.P) : static_cast<double>(p.P);
    int d = 0;
    if (cr.par.fixed_d > 0)
      d = cr.par.fixed_d;
    else if (p.Peff > cr.par.target)
      d = static_cast<int>(std::ceil(std::log2(p.Peff / cr.par.target)));
    if (d > kMaxBits) d = kMaxBits;
    if (d > cr.kb - 30) d = cr.kb - 30;  // keep 30 key bits below the bucket bits
    if (d < 0) d = 0;
    p.d = d;
    p.d1 = std::min(d, cr.par.d1cap);
    if (d - p.d1 > 8) p.d1 = d - 8;  // the partition digit has at most 8 bits
    p.d2 = d - p.d1;
    p.ibits = 0;
    while ((int64_t(1) << p.ibits) < static_cast<int64_t>(p.m1)) ++p.ibits;
    if ((static_cast<uint64_t>(p.m2) << p.ibits) > 0xFFFFFFFFull) p.ibits = -1;
    p.nc = 1u << p.d1;
    p.nbk = 1u << p.d;
    p.sb0 = sb;
    p.bb0 = bb;
    p.tt0 = tt;
    p.out0 = out;
    sb += p.nc;
    bb += p.nbk;
    tt += p.nc * p.nc;
    out += (p.P + kBS - 1) / kBS * kBS;
    // a sum times itself generates the class tiles hA <= hB, the diagonal
    // ones whole: at most P records
    rec += p.P;
    gb += (p.P + kTile - 1) / kTile + p.nc + 1;
  }
  cr.nsb = sb;
  cr.nbk = bb;
  cr.rec = rec;
  cr.cap = out;
  if (gb > 0x7FFFFFFFull || rec > 0xFFFFFFFFull || out > 0xFFFFFFFFull)
    fail(PAULI_ERR_OVERFLOW, "a batched class exceeds 2^32 records; split the batch");
  cr.gb = static_cast<uint32_t>(gb);
}

template <typename T>
void setup_class(ClassRun& cr, hipStream_t s);

// Allocates the class's buffers, uploads its tables and the output block.
template <typename T>
void setup_class(ClassRun& cr, hipStream_t s) {
  using TV = T;
  (void)sizeof(TV);
  plan_products(cr);
  const int G = cr.G;
  const uint32_t np = static_cast<uint32_t>(cr.prods.size());
  const uint32_t nsA = static_cast<uint32_t>(cr.sumsA.size()),
                 nsB = static_cast<uint32_t>(cr.sumsB.size());
  cr.sideB = nsB > 0;
  Carve cv;
  auto side_pieces = [&](uint32_t tot, uint32_t ns, std::vector<size_t>& id) {
    const size_t n = std::max<uint32_t>(tot, 1);
    id.push_back(cv.add(n * slot_words(G) * 8));   // rows
    id.push_back(cv.add(n * sizeof(Aux<T>)));      // aux
    for (int k = 0; k < 3; ++k) id.push_back(cv.add(n * 8));  // key ckey ckey2
    for (int k = 0; k < 2; ++k) id.push_back(cv.add(n * 4));  // gidx gidx2
    id.push_back(cv.add((ns * 256ull + 1) * 4));   // g
    id.push_back(cv.add((ns * 256ull + 1) * 4));   // gs
    id.push_back(cv.add(ns * sizeof(SumDesc)));    // desc
    id.push_back(cv.add((ns + 1) * 4ull));         // start
    id.push_back(cv.add(radix_workspace_bytes(n)));
    id.push_back(cv.add(scan_workspace_bytes(ns * 256ll)));
    id.push_back(cv.add(n * 2));                   // top
    id.push_back(cv.add(n * 16));                  // ki
  };
  std::vector<size_t> ia, ib;
  side_pieces(cr.totA, nsA, ia);
  if (cr.sideB) side_pieces(cr.totB, nsB, ib);
  uint32_t ttsize = 0;
  for (auto& p : cr.prods) ttsize += p.nc * p.nc;
  const size_t i_gen = cv.add(np * sizeof(GenSides)), i_sbprod = cv.add(cr.nsb * 2ull),
               i_bprod = cv.add(cr.nbk * 2ull), i_sbbase = cv.add((np + 1) * 4ull),
               i_bbase = cv.add((np + 1) * 4ull), i_ttoff = cv.add(np * 4ull),
               i_Tt = cv.add(std::max<uint32_t>(ttsize, 1) * 4ull), i_sym = cv.add(np),
               i_shift = cv.add(np * 4ull), i_d2 = cv.add(np * 4ull), i_mask = cv.add(np * 4ull),
               i_S = cv.add(cr.nsb * 4ull), i_soff = cv.add((cr.nsb + 1) * 4ull),
               i_nt = cv.add(cr.nsb * 4ull), i_tb = cv.add((cr.nsb + 1) * 4ull),
               i_C = cv.add(static_cast<size_t>(cr.gb) * 256 * 4),
               i_wsb = cv.add(scan_workspace_bytes(cr.nsb)),
               i_wc = cv.add(scan_workspace_bytes(static_cast<int64_t>(cr.gb) * 256)),
               i_wseg = cv.add(scan_workspace_bytes(cr.nbk));
  const size_t nrec = std::max<uint64_t>(cr.rec, 1);
  const size_t i_K = cv.add(nrec * 8), i_K2 = cv.add(nrec * 8), i_V = cv.add(nrec * 4),
               i_V2 = cv.add(nrec * 4), i_boff = cv.add((cr.nbk + 1) * 4ull),
               i_segidx = cv.add(nrec * 4), i_nseg = cv.add((cr.nbk + 1) * 4ull),
               i_segoff = cv.add((cr.nbk + 1) * 4ull), i_heavy = cv.add(cr.nbk * 4ull),
               i_redo = cv.add(cr.nbk * 4ull), i_long = cv.add((nrec / kLong + 2) * 8),
               i_ctr = cv.add(64), i_sf = cv.add(np * sizeof(SortField)),
               i_op = cv.add(np * sizeof(Operands<kMaxWords, T>)), i_pout = cv.add(np * 4ull),
               i_perr = cv.add(np * 4ull), i_info = cv.add(np * 8ull);
  cr.work = DBuf(cv.total, s);
  char* base = cr.work.as<char>();
  auto at = [&](size_t i) { return static_cast<void*>(base + cv.off[i]); };
  auto fill_side = [&](ClassRun::Side& sd, const std::vector<size_t>& id) {
    sd.rows = static_cast<uint64_t*>(at(id[0]));
    sd.aux = at(id[1]);
    sd.key = static_cast<uint64_t*>(at(id[2]));
    sd.ckey = static_cast<uint64_t*>(at(id[3]));
    sd.ckey2 = static_cast<uint64_t*>(at(id[4]));
    sd.gidx = static_cast<uint32_t*>(at(id[5]));
    sd.gidx2 = static_cast<uint32_t*>(at(id[6]));
    sd.g = static_cast<uint32_t*>(at(id[7]));
    sd.gs = static_cast<uint32_t*>(at(id[8]));
    sd.desc = static_cast<SumDesc*>(at(id[9]));
    sd.start = static_cast<uint32_t*>(at(id[10]));
    sd.rwork = at(id[11]);
    sd.swork = at(id[12]);
    sd.top = static_cast<uint16_t*>(at(id[13]));
    sd.ki = static_cast<uint4*>(at(id[14]));
  };
  fill_side(cr.A, ia);
  if (cr.sideB) fill_side(cr.B, ib);
  cr.gen = static_cast<GenSides*>(at(i_gen));
  cr.sbprod = static_cast<uint16_t*>(at(i_sbprod));
  cr.bprod = static_cast<uint16_t*>(at(i_bprod));
  cr.sbbase = static_cast<uint32_t*>(at(i_sbbase));
  cr.bbase = static_cast<uint32_t*>(at(i_bbase));
  cr.ttoff = static_cast<uint32_t*>(at(i_ttoff));
  cr.Tt = static_cast<uint32_t*>(at(i_Tt));
  cr.sym = static_cast<uint8_t*>(at(i_sym));
  cr.shift = static_cast<int*>(at(i_shift));
  cr.d2tab = static_cast<int*>(at(i_d2));
  cr.mask = static_cast<uint32_t*>(at(i_mask));
  cr.S = static_cast<uint32_t*>(at(i_S));
  cr.soff = static_cast<uint32_t*>(at(i_soff));
  cr.nt = static_cast<uint32_t*>(at(i_nt));
  cr.tb = static_cast<uint32_t*>(at(i_tb));
  cr.C = static_cast<uint32_t*>(at(i_C));
  cr.w_sb = at(i_wsb);
  cr.w_c = at(i_wc);
  cr.w_seg = at(i_wseg);
  cr.K = static_cast<uint64_t*>(at(i_K));
  cr.K2 = static_cast<uint64_t*>(at(i_K2));
  cr.V = static_cast<uint32_t*>(at(i_V));
  cr.V2 = static_cast<uint32_t*>(at(i_V2));
  cr.boff = static_cast<uint32_t*>(at(i_boff));
  cr.segidx = static_cast<uint32_t*>(at(i_segidx));
  cr.nseg = static_cast<uint32_t*>(at(i_nseg));
  cr.segoff = static_cast<uint32_t*>(at(i_segoff));
  cr.heavy = static_cast<uint32_t*>(at(i_heavy));
  cr.redo = static_cast<uint32_t*>(at(i_redo));
  cr.long_list = static_cast<uint32_t*>(at(i_long));
  cr.ctr = static_cast<uint32_t*>(at(i_ctr));
  cr.sftab = static_cast<SortField*>(at(i_sf));
  cr.optab = at(i_op);
  cr.pout = static_cast<uint32_t*>(at(i_pout));
  cr.perr = static_cast<uint32_t*>(at(i_perr));
  cr.info = static_cast<uint32_t*>(at(i_info));

  // the output block: X, Z [W][cap], phase, coefficients, fingerprints
  const int32_t odt = cr.mode == PAULI_MERGE_COMPENSATED ? PAULI_C64 : cr.dtype;
  cr.out = std::make_shared<SharedBlock>(cr.W, static_cast<int64_t>(cr.cap), odt, s);

  // ---- host tables, uploaded in one copy per table
  auto up = [&](void* dst, const void* src, size_t bytes) {
    if (bytes) PAULI_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
  };
  auto side_desc = [&](const std::vector<const paulisum*>& sums,
                       const std::vector<int>& d1s, ClassRun::Side& sd) {
    std::vector<SumDesc> desc(sums.size());
    std::vector<uint32_t> start(sums.size() + 1, 0);
    for (size_t u = 0; u < sums.size(); ++u) {
      const paulisum* x = sums[u];
      SumDesc& D = desc[u];
      D.X = x->X;
      D.Z = x->Z;
      D.ph = x->ph;
      D.coef = x->coef;
      D.fp = x->fp;
      D.ld = x->ld;
      D.W = x->W;
      D.kshift = 64 - cr.kb;
      D.d1 = d1s[u];
      D.cshift = cr.kb - d1s[u];
      start[u + 1] = start[u] + static_cast<uint32_t>(x->m);
    }
    up(sd.desc, desc.data(), desc.size() * sizeof(SumDesc));
    up(sd.start, start.data(), start.size() * 4);
  };
  std::vector<int> d1A(nsA, 0), d1B(nsB, 0);
  for (auto& p : cr.prods) {
    d1A[p.uA] = p.d1;
    if (!p.sym) d1B[p.uB] = p.d1;
  }
  side_desc(cr.sumsA, d1A, cr.A);
  if (cr.sideB) side_desc(cr.sumsB, d1B, cr.B);

  std::vector<GenSides> gen(np);
  std::vector<uint16_t> sbprod(cr.nsb), bprod(cr.nbk);
  std::vector<uint32_t> sbbase(np + 1), bbase(np + 1), ttoff(np), pout(np);
  std::vector<uint8_t> sym(np);
  std::vector<int> shift(np), d2t(np);
  std::vector<uint32_t> mask(np);
  std::vector<SortField> sf(np);
  std::vector<Operands<kMaxWords, T>> opsMax;
  std::vector<uint8_t> opbytes;
  for (uint32_t k = 0; k < np; ++k) {
    const Product& p = cr.prods[k];
    const ClassRun::Side& sa = cr.A;
    const ClassRun::Side& sbs = p.sym ? cr.A : cr.B;
    const uint32_t ub = p.sym ? p.uA : p.uB;
    GenSides& gs = gen[k];
    gs.gA = sa.g + p.uA * 256u;
    gs.gsA = sa.gs + p.uA * 256u;
    gs.kiA = sa.ki;
    gs.gB = sbs.g + ub * 256u;
    gs.gsB = sbs.gs + ub * 256u;
    gs.kiB = sbs.ki;
    gs.Tt = cr.Tt + p.tt0;
    gs.ma = p.m1;
    gs.ibits = p.ibits;
    gs.d1 = p.d1;
    gs.tA = sa.top;
    gs.tB = sbs.top;
    gs.sh16 = 16 - p.d;
    for (uint32_t x = 0; x < p.nc; ++x) sbprod[p.sb0 + x] = static_cast<uint16_t>(k);
    for (uint32_t x = 0; x < p.nbk; ++x) bprod[p.bb0 + x] = static_cast<uint16_t>(k);
    sbbase[k] = p.sb0;
    bbase[k] = p.bb0;
    ttoff[k] = p.tt0;
    pout[k] = static_cast<uint32_t>(p.out0);
    sym[k] = p.sym ? 1 : 0;
    shift[k] = cr.kb - p.d;
    d2t[k] = p.d2;
    mask[k] = (1u << p.d2) - 1u;
    sf[k] = sort_field_for(cr.kb - p.d);
  }
  sbbase[np] = cr.nsb;
  bbase[np] = cr.nbk;
  up(cr.gen, gen.data(), np * sizeof(GenSides));
  up(cr.sbprod, sbprod.data(), sbprod.size() * 2);
  up(cr.bprod, bprod.data(), bprod.size() * 2);
  up(cr.sbbase, sbbase.data(), sbbase.size() * 4);
  up(cr.bbase, bbase.data(), bbase.size() * 4);
  up(cr.ttoff, ttoff.data(), ttoff.size() * 4);
  up(cr.pout, pout.data(), pout.size() * 4);
  up(cr.sym, sym.data(), sym.size());
  up(cr.shift, shift.data(), shift.size() * 4);
  up(cr.d2tab, d2t.data(), d2t.size() * 4);
  up(cr.mask, mask.data(), mask.size() * 4);
  up(cr.sftab, sf.data(), sf.size() * sizeof(SortField));
  // the operands of every product, as the expand kernel of this class takes them
  auto put_ops = [&](auto tag) {
    using OpT = decltype(tag);
    std::vector<OpT> ops(np);
    for (uint32_t k = 0; k < np; ++k) {
      const Product& p = cr.prods[k];
      const ClassRun::Side& sbs = p.sym ? cr.A : cr.B;
      const uint32_t ub = p.sym ? p.uA : p.uB;
      // the rows of a product's sums start at the sums' first rows
      uint32_t rowA = 0, rowB = 0;
      for (uint32_t u = 0; u < p.uA; ++u) rowA += static_cast<uint32_t>(cr.sumsA[u]->m);
      const auto& sl = p.sym ? cr.sumsA : cr.sumsB;
      for (uint32_t u = 0; u < ub; ++u) rowB += static_cast<uint32_t>(sl[u]->m);
      OpT& o = ops[k];
      o.ra = cr.A.rows + static_cast<size_t>(rowA) * slot_words(G);
      o.rb = sbs.rows + static_cast<size_t>(rowB) * slot_words(G);
      o.xa = static_cast<const Aux<T>*>(cr.A.aux) + rowA;
      o.xb = static_cast<const Aux<T>*>(sbs.aux) + rowB;
      o.ma = p.m1;
      o.ibits = p.ibits;
      o.nw = cr.W;
      o.form = p.sym ? kFormSym : kFormProduct;
    }
    up(cr.optab, ops.data(), ops.size() * sizeof(OpT));
    PAULI_HIP(hipStreamSynchronize(s));  // the host tables go out of scope
  };
  switch (words_class(cr.W)) {
    case 1: put_ops(Operands<1, T>{}); break;
    case 2: put_ops(Operands<2, T>{}); break;
    case 3: put_ops(Operands<3, T>{}); break;
    case 4: put_ops(Operands<4, T>{}); break;
    case 5: put_ops(Operands<5, T>{}); break;
    case 6: put_ops(Operands<6, T>{}); break;
    case 7: put_ops(Operands<7, T>{}); break;
    case 8: put_ops(Operands<8, T>{}); break;
    default: put_ops(Operands<kMaxWords, T>{}); break;
  }
}

template <typename T>
void prep_side_b(ClassRun& cr, ClassRun::Side& sd, uint32_t tot, uint32_t ns, hipStream_t s) {
  if (tot == 0) return;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(ns * 256u + 1)), dim3(kB), 0, s, sd.g,
                     ns * 256u + 1, 0u);
  hipLaunchKernelGGL(k_bprep<T>, dim3(grid_for(tot)), dim3(kB), 0, s, sd.desc, sd.start,
                     static_cast<int>(ns), tot, cr.G, sd.rows, static_cast<Aux<T>*>(sd.aux),
                     sd.key, sd.ckey, sd.gidx);
  PAULI_HIP(hipGetLastError());
  int ubits = 0;
  while ((1u << ubits) < ns) ++ubits;
  uint64_t* ck = sd.ckey;
  uint32_t* gi = sd.gidx;
  if (radix_sort_pairs(sd.ckey, sd.gidx, sd.ckey2, sd.gidx2, tot, 8 + ubits, sd.rwork, s)) {
    ck = sd.ckey2;
    gi = sd.gidx2;
  }
  hipLaunchKernelGGL(k_bgather, dim3(grid_for(tot)), dim3(kB), 0, s, sd.key, gi, ck, sd.start,
                     tot, cr.kb, sd.top, sd.ki);
  hipLaunchKernelGGL(k_class_count, dim3(grid_for(tot)), dim3(kB), 0, s, ck, tot, sd.g);
  scan_exclusive_u32(sd.g, sd.gs, ns * 256ll, sd.gs + ns * 256u, sd.swork, s);
  PAULI_HIP(hipGetLastError());
}

// The whole launch sequence of a class (no host synchronisation).
template <int G, int WT, typename T, int MODE>
void launch_class(ClassRun& cr, hipStream_t s) {
  const uint32_t np = static_cast<uint32_t>(cr.prods.size());
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, cr.ctr, 16u, 0u);
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(np)), dim3(kB), 0, s, cr.perr, np, 0u);
  {
    StageScope sc(PAULI_STAGE_PREP, s, (cr.totA + cr.totB) * (16.0 * cr.W + 32.0 * 2));
    prep_side_b<T>(cr, cr.A, cr.totA, static_cast<uint32_t>(cr.sumsA.size()), s);
    if (cr.sideB) prep_side_b<T>(cr, cr.B, cr.totB, static_cast<uint32_t>(cr.sumsB.size()), s);
  }
  {
    StageScope sc(PAULI_STAGE_SORT, s, static_cast<double>(cr.rec) * 12.0);
    hipLaunchKernelGGL(k_btile_table, dim3(cr.nsb), dim3(kB), 0, s, cr.gen, cr.sbprod, cr.sbbase,
                       cr.sym, cr.Tt, cr.ttoff, cr.S);
    scan_exclusive_u32(cr.S, cr.soff, cr.nsb, cr.soff + cr.nsb, cr.w_sb, s);
    hipLaunchKernelGGL(k_tiles_per_sb, dim3(grid_for(cr.nsb)), dim3(kB), 0, s, cr.S, cr.nsb,
                       cr.nt);
    scan_exclusive_u32(cr.nt, cr.tb, cr.nsb, cr.tb + cr.nsb, cr.w_sb, s);
    const GenBatch bt{cr.sbprod, cr.sbbase, cr.gen, cr.shift, cr.mask};
    hipLaunchKernelGGL(k_gcount, dim3(cr.gb), dim3(kGenNT), 0, s, GenSides{}, bt, cr.S, cr.tb,
                       cr.nsb, 0, 0u, cr.C);
    scan_exclusive_u32(cr.C, cr.C, static_cast<int64_t>(cr.gb) * 256, nullptr, cr.w_c, s);
    hipLaunchKernelGGL(k_gscatter, dim3(cr.gb), dim3(kGenNT), 0, s, GenSides{}, bt, cr.K, cr.V, cr.S,
                       cr.tb, cr.nsb, 0, 0u, cr.C);
    hipLaunchKernelGGL(k_bbucket_offsets, dim3(grid_for(cr.nbk + 1)), dim3(kB), 0, s, cr.bprod,
                       cr.bbase, cr.sbbase, cr.d2tab, cr.soff, cr.tb, cr.C, cr.nbk, cr.nsb,
                       cr.boff);
    PAULI_HIP(hipGetLastError());
  }
  SegOut so{cr.V, cr.segidx, cr.nseg, cr.long_list, cr.ctr + 1};
  const SortBatch sb{cr.bprod, cr.sftab};
  const SortField f0 = sort_field_for(64);
  {
    StageScope sc(PAULI_STAGE_SEGMENT, s, static_cast<double>(cr.rec) * 20.0);
    const uint32_t gs_cap = kSortBlocksPerCU * cr.cus;
    const uint32_t gsort = cr.nbk < gs_cap ? cr.nbk : gs_cap;
    hipLaunchKernelGGL(k_bucket_count, dim3(gsort), dim3(kSortNT), 0, s, cr.K, cr.boff, cr.nbk,
                       f0, sb, so, cr.heavy, cr.ctr, cr.redo, cr.ctr + 6);
    hipLaunchKernelGGL(k_bucket_radix, dim3(gsort), dim3(kSortNT), 0, s, cr.K,
                       cr.boff, cr.nbk, cr.redo, cr.ctr + 6, f0, sb, so, cr.heavy, cr.ctr);
    hipLaunchKernelGGL(k_heavy_sort, dim3(gsort), dim3(kSortNT), 0, s, cr.K, cr.K2, cr.V2,
                       cr.boff, 64, sb, cr.heavy, cr.ctr, so);
    PAULI_HIP(hipGetLastError());
    scan_exclusive_u32(cr.nseg, cr.segoff, cr.nbk, cr.segoff + cr.nbk, cr.w_seg, s);
  }
  SharedBlock& ob = *cr.out;
  using TV = typename std::conditional<MODE == kComp, float, T>::type;
  ExpandArgs E{cr.boff, cr.V, cr.segidx, cr.segoff, cr.nbk, nullptr, cr.ctr + 4, ob.X, ob.Z,
               ob.ph, ob.coef, ob.fp, ob.ld, cr.tau, 0};
  E.bprod = cr.bprod;
  E.optab = cr.optab;
  E.pbase = cr.bbase;
  E.pout = cr.pout;
  E.perr = cr.perr;
  E.parts = static_cast<uint32_t>(cr.par.parts);
  {
    StageScope sc(PAULI_STAGE_WRITE, s,
                  static_cast<double>(cr.rec) * (16.0 * cr.W + sizeof(cplx<TV>) + 1 + 8 + 8));
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for((cr.cap + 3) / 4)), dim3(kB), 0, s,
                       reinterpret_cast<uint32_t*>(ob.ph), static_cast<uint32_t>((cr.cap + 3) / 4),
                       0u);
    hipLaunchKernelGGL((k_expand<G, WT, T, MODE, true>), dim3(cr.nbk < 1024u ? cr.nbk : 1024u),
                       dim3(kB), 0, s, E, Operands<WT, T>{});
    PAULI_HIP(hipGetLastError());
  }
  {
    StageScope sc(PAULI_STAGE_LONG, s, 0.0);
    hipLaunchKernelGGL((k_expand_long<G, WT, T, MODE, true>), dim3(256), dim3(kLongB), 0, s, E,
                       Operands<WT, T>{}, cr.long_list, cr.ctr + 1);
    hipLaunchKernelGGL(k_binfo, dim3(grid_for(np)), dim3(kB), 0, s, cr.segoff, cr.bbase, cr.perr,
                       np, cr.info);
    PAULI_HIP(hipGetLastError());
  }
}

template <typename T, int MODE>
void launch_class_w(ClassRun& cr, hipStream_t s) {
  switch (words_class(cr.W)) {
    case 1: return launch_class<1, 1, T, MODE>(cr, s);
    case 2: return launch_class<2, 2, T, MODE>(cr, s);
    case 3: return launch_class<4, 3, T, MODE>(cr, s);
    case 4: return launch_class<4, 4, T, MODE>(cr, s);
    case 5: return launch_class<8, 5, T, MODE>(cr, s);
    case 6: return launch_class<8, 6, T, MODE>(cr, s);
    case 7: return launch_class<8, 7, T, MODE>(cr, s);
    case 8: return launch_class<8, 8, T, MODE>(cr, s);
    default: return launch_class<16, kMaxWords, T, MODE>(cr, s);
  }
}

void setup(ClassRun& cr, hipStream_t s) {
  cr.cus = device_cus();
  if (cr.dtype == PAULI_C128) setup_class<double>(cr, s);
  else setup_class<float>(cr, s);
}

void launch(ClassRun& cr, hipStream_t s) {
  const bool comp = cr.mode == PAULI_MERGE_COMPENSATED;
  if (cr.dtype == PAULI_C128) {
    if (comp) launch_class_w<double, kComp>(cr, s);
    else launch_class_w<double, kPlain>(cr, s);
  } else {
    if (comp) launch_class_w<float, kComp>(cr, s);
    else launch_class_w<float, kPlain>(cr, s);
  }
}

// ------------------------------------------------------------- autotuner

int log2_bucket(uint64_t r) {
  int l = 0;
  while ((uint64_t(1) << (l + 1)) <= r) ++l;
  return l;
}

const std::vector<ClassParams>& candidates() {
  static const std::vector<ClassParams> c = {
      {3500.0, 8, 4}, {1750.0, 8, 4}, {3500.0, 6, 4}, {3500.0, 8, 2}, {3500.0, 8, 8}};
  return c;
}

std::string tune_file_from_env() {
  const char* f = std::getenv("PAULI_TUNE_FILE");
  return f ? std::string(f) : std::string();
}

bool save_tune_locked(const std::string& path) {
  std::ofstream out(path);
  if (!out) return false;
  out << "# W log2_records dtype mode target_records_per_bucket class_bits expand_parts\n";
  for (auto& kv : g_tune)
    out << kv.first.W << ' ' << kv.first.logp << ' ' << kv.first.dtype << ' ' << kv.first.mode
        << ' ' << kv.second.target << ' ' << kv.second.d1cap << ' ' << kv.second.parts << '\n';
  return static_cast<bool>(out);
}

bool load_tune_locked(const std::string& path) {
  std::ifstream in(path);
  if (!in) return false;
  // a malformed line rejects the whole file: nothing of it is applied
  std::vector<std::pair<ClassKey, ClassParams>> rows;
  std::string line;
  while (std::getline(in, line)) {
    if (line.empty() || line[0] == '#') continue;
    std::istringstream ls(line);
    ClassKey k{};
    ClassParams p;
    if (!(ls >> k.W >> k.logp >> k.dtype >> k.mode >> p.target >> p.d1cap >> p.parts)) return false;
    if (!(p.target >= 256.0 && p.target <= kCap) || p.d1cap < 0 || p.d1cap > 8 ||
        (p.parts != 1 && p.parts != 2 && p.parts != 4 && p.parts != 8))
      return false;
    rows.emplace_back(k, p);
  }
  if (in.bad()) return false;
  for (const auto& r : rows) g_tune[r.first] = r.second;
  return true;
}

}  // namespace

// ------------------------------------------------------------------ plans

struct BatchPlan {
  int nb = 0;
  std::vector<paulisum*> a, b;
  MergeArgs o;
  std::vector<std::unique_ptr<ClassRun>> classes;
  hipStream_t home = nullptr;  // stream of the plan's buffers (the create call's)
  hipStream_t priv = nullptr;  // graph launches (a graph cannot be captured on the null stream)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraphExec_t exec = nullptr;
  bool use_graph = false;
  bool ran = false;
  ~BatchPlan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (priv && ev_out) {
      // the buffers are released on home, after the plan's last run
      (void)hipEventRecord(ev_out, priv);
      (void)hipStreamWaitEvent(home, ev_out, 0);
    }
    classes.clear();
    if (priv) {
      (void)hipStreamSynchronize(priv);
      (void)hipStreamDestroy(priv);
    }
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
  }
};

namespace {

void capture(BatchPlan& pl) {
  if (pl.exec) {
    PAULI_HIP(hipGraphExecDestroy(pl.exec));
    pl.exec = nullptr;
  }
  NoEvents ne;
  hipGraph_t graph = nullptr;
  PAULI_HIP(hipStreamBeginCapture(pl.priv, hipStreamCaptureModeThreadLocal));
  try {
    for (auto& cr : pl.classes) launch(*cr, pl.priv);
  } catch (...) {
    (void)hipStreamEndCapture(pl.priv, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    throw;
  }
  PAULI_HIP(hipStreamEndCapture(pl.priv, &graph));
  const hipError_t e = hipGraphInstantiate(&pl.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  PAULI_HIP(e);
}

// Times one eager run of the class with the given parameters (ms).
float time_class(ClassRun& cr, const ClassParams& par, hipStream_t s) {
  cr.par = par;
  cr.work.reset();
  cr.out.reset();
  setup(cr, s);
  hipEvent_t e0, e1;
  PAULI_HIP(hipEventCreate(&e0));
  PAULI_HIP(hipEventCreate(&e1));
  float ms = 0.f;
  try {
    PAULI_HIP(hipEventRecord(e0, s));
    launch(cr, s);
    PAULI_HIP(hipEventRecord(e1, s));
    PAULI_HIP(hipEventSynchronize(e1));
    PAULI_HIP(hipEventElapsedTime(&ms, e0, e1));
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms;
}

}  // namespace

BatchPlan* batch_plan_create(int nb, paulisum* const* a, paulisum* const* b, const MergeArgs& o,
                             const BatchShape* shape, bool use_graph, hipStream_t st) {
  auto plan = std::make_unique<BatchPlan>();
  plan->nb = nb;
  plan->a.assign(a, a + nb);
  plan->b.assign(b, b + nb);
  plan->o = o;
  plan->use_graph = use_graph;
  plan->home = st;
  if (use_graph) {
    PAULI_HIP(hipStreamCreateWithFlags(&plan->priv, hipStreamNonBlocking));
    PAULI_HIP(hipEventCreateWithFlags(&plan->ev_in, hipEventDisableTiming));
    PAULI_HIP(hipEventCreateWithFlags(&plan->ev_out, hipEventDisableTiming));
  }
  hipStream_t s = st;
  // classes: (W, dtype) of the products with at least one term on each side
  std::map<std::pair<int, int>, ClassRun*> byk;
  for (int t = 0; t < nb; ++t) {
    const paulisum* x = a[t];
    const paulisum* y = b[t];
    if (x->m == 0 || y->m == 0) continue;
    const auto key = std::make_pair(x->W, static_cast<int>(x->dtype));
    ClassRun*& cr = byk[key];
    if (!cr) {
      plan->classes.push_back(std::make_unique<ClassRun>());
      cr = plan->classes.back().get();
      cr->W = x->W;
      cr->G = group_of(x->W);
      cr->dtype = x->dtype;
      cr->mode = o.mode;
      cr->kb = o.key_bits;
      cr->tau = o.tau;
    }
    Product p{};
    p.idx = t;
    p.a = x;
    p.b = y;
    p.sym = x == y;
    p.m1 = static_cast<uint32_t>(x->m);
    p.m2 = static_cast<uint32_t>(y->m);
    p.uA = static_cast<uint32_t>(cr->sumsA.size());
    cr->sumsA.push_back(x);
    cr->totA += p.m1;
    if (!p.sym) {
      p.uB = static_cast<uint32_t>(cr->sumsB.size());
      cr->sumsB.push_back(y);
      cr->totB += p.m2;
    }
    cr->prods.push_back(p);
  }
  for (auto& up : plan->classes) {
    ClassRun& cr = *up;
    if (cr.prods.size() > 65535) fail(PAULI_ERR_OVERFLOW, "more than 65535 products in a class");
    uint64_t recs = 0;
    for (auto& p : cr.prods)
      recs += p.sym ? static_cast<uint64_t>(p.m1) * p.m2 / 2 : static_cast<uint64_t>(p.m1) * p.m2;
    const ClassKey key{cr.W, log2_bucket(recs + 1), static_cast<int>(cr.dtype), cr.mode};
    if (shape) {
      cr.par = ClassParams{};
      if (shape->bucket_records > 0) cr.par.target = shape->bucket_records;
      if (shape->class_bits > 0) cr.par.d1cap = shape->class_bits;
      if (shape->expand_parts > 0) cr.par.parts = shape->expand_parts;
      cr.par.fixed_d = shape->bucket_bits;
      setup(cr, s);
      continue;
    }
    bool known = false;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      if (!g_tune_env_loaded) {
        g_tune_env_loaded = true;
        const std::string f = tune_file_from_env();
        if (!f.empty()) (void)load_tune_locked(f);
      }
      auto it = g_tune.find(key);
      if (it != g_tune.end()) {
        cr.par = it->second;
        known = true;
      }
    }
    if (known) {
      setup(cr, s);
      continue;
    }
    // time every candidate once (each computes the same result)
    float best = 0.f;
    ClassParams bestp = candidates()[0];
    for (size_t c = 0; c < candidates().size(); ++c) {
      const float ms = time_class(cr, candidates()[c], s);
      if (c == 0 || ms < best) {
        best = ms;
        bestp = candidates()[c];
      }
    }
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune[key] = bestp;
      const std::string f = tune_file_from_env();
      if (!f.empty()) (void)save_tune_locked(f);
    }
    cr.par = bestp;
    cr.work.reset();
    cr.out.reset();
    setup(cr, s);
  }
  if (use_graph) capture(*plan);
  return plan.release();
}

void batch_plan_run(BatchPlan* plan, hipStream_t st) {
  // outputs handed out by the last results call: fresh blocks (and a new graph)
  bool fresh = false;
  for (auto& cr : plan->classes)
    if (!cr->out) {
      const int32_t odt = cr->mode == PAULI_MERGE_COMPENSATED ? PAULI_C64 : cr->dtype;
      cr->out = std::make_shared<SharedBlock>(cr->W, static_cast<int64_t>(cr->cap), odt,
                                              plan->home);
      fresh = true;
    }
  if (plan->use_graph) {
    if (fresh || !plan->exec) capture(*plan);
    // the graph runs on the plan's stream, after the caller's earlier work
    // and before the caller's later work
    PAULI_HIP(hipEventRecord(plan->ev_in, st));
    PAULI_HIP(hipStreamWaitEvent(plan->priv, plan->ev_in, 0));
    if (st != plan->home) {
      PAULI_HIP(hipEventRecord(plan->ev_in, plan->home));
      PAULI_HIP(hipStreamWaitEvent(plan->priv, plan->ev_in, 0));
    }
    PAULI_HIP(hipGraphLaunch(plan->exec, plan->priv));
    PAULI_HIP(hipEventRecord(plan->ev_out, plan->priv));
    PAULI_HIP(hipStreamWaitEvent(st, plan->ev_out, 0));
  } else {
    if (st != plan->home) fail(PAULI_ERR_INVALID, "a plan without a graph runs on its own stream");
    for (auto& cr : plan->classes) launch(*cr, st);
  }
  plan->ran = true;
}

// Per product, a view of its terms in its class's output block (products
// with an empty side get an empty sum); a product whose records collided on
// a fingerprint is recomputed by the general pipeline (which applies the
// drop itself).  With a drop threshold, one compaction per class moves the
// kept terms of all its products into a block of exactly their size, and
// the views point there.  Waits for the run.
void batch_plan_results(BatchPlan* plan, paulisum** out, hipStream_t st) {
  if (!plan->ran) fail(PAULI_ERR_INVALID, "the plan has not run since its last results");
  if (plan->priv) PAULI_HIP(hipStreamSynchronize(plan->priv));
  PAULI_HIP(hipStreamSynchronize(plan->home));
  const bool drop = plan->o.drop_abs >= 0.0;
  std::vector<paulisum*> res(static_cast<size_t>(plan->nb), nullptr);
  try {
    for (auto& cr : plan->classes) {
      const uint32_t np = static_cast<uint32_t>(cr->prods.size());
      std::vector<uint32_t> info(2 * np);
      PAULI_HIP(hipMemcpy(info.data(), cr->info, 8ull * np, hipMemcpyDeviceToHost));
      std::vector<uint32_t> direct;  // products read from the class block
      std::vector<int64_t> r0, rm;
      for (uint32_t k = 0; k < np; ++k) {
        const Product& p = cr->prods[k];
        if (info[2 * k + 1] != 0) {
          res[p.idx] = merge_generic(p.a, p.b, plan->o, st);
          continue;
        }
        direct.push_back(k);
        r0.push_back(static_cast<int64_t>(p.out0));
        rm.push_back(info[2 * k]);
      }
      std::shared_ptr<SharedBlock> blk = cr->out;
      std::vector<int64_t> first = r0, kept = rm;
      if (drop && !direct.empty())
        blk = drop_ranges(*cr->out, r0, rm, plan->o.drop_abs, first, kept, plan->home);
      for (size_t j = 0; j < direct.size(); ++j) {
        const Product& p = cr->prods[direct[j]];
        res[p.idx] = sum_view(blk, p.a->n, first[j], kept[j]);
      }
      cr->out.reset();  // the views own the block now
    }
    // the compactions ran on the plan's stream: done before the caller's work
    if (drop) PAULI_HIP(hipStreamSynchronize(plan->home));
    for (int t = 0; t < plan->nb; ++t)
      if (!res[t]) {
        const int32_t odt =
            plan->o.mode == PAULI_MERGE_COMPENSATED ? PAULI_C64 : plan->a[t]->dtype;
        res[t] = new_sum(plan->a[t]->n, 0, 0, odt, st);
      }
  } catch (...) {
    for (paulisum* r : res) free_sum(r);
    throw;
  }
  plan->ran = false;
  for (int t = 0; t < plan->nb; ++t) out[t] = res[t];
}

void batch_plan_destroy(BatchPlan* plan) { delete plan; }

int batch_tune_save(const char* path) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return save_tune_locked(path) ? 0 : -1;
}

int batch_tune_load(const char* path) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return load_tune_locked(path) ? 0 : -1;
}

}  // namespace pauli
