// CPU oracle for Pauli-sum products and sort-and-combine.
//
// TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or
// calls this file; only the test suite, the smoke check and the CPU-baseline
// leg of the benchmark use it.  It shares no code, header, table or constant
// with the HIP library.
//
// It is written to be slow and plainly correct: every string is decoded into
// one letter per qubit, products are formed qubit by qubit from the
// single-qubit product table, and duplicate strings are combined in an
// ordered map.  Paper: "PauLIB: A High-Performance Library for Processing
// Pauli Strings" (arXiv 2605.25974).
//
//  * Letter encoding, Section III-C, Table I: (x,z) = (0,0) I, (0,1) Z,
//    (1,0) X, (1,1) Y.  Qubit q of a packed string is bit (q mod 64) of word
//    floor(q/64), for both the X words and the Z words.
//  * Single-qubit products, Section III-A: P*P = I, I*P = P*I = P,
//    XY = iZ, YZ = iX, ZX = iY and the reversed orders carry -i.
//  * String product, Section III-A eq. (1) and the worked example: multiply
//    letter by letter and add the phase exponents (mod 4).
//  * Pauli sum, Section III-A eq. (2): a term is i^k * c * (letters), c
//    complex.
//  * Sort-and-combine, Section III-H: one output term per distinct string,
//    carrying the sum of the input values.  Here an ordered map plays the role
//    of the sort.  Each product c1*c2 is split exactly into double pieces
//    (TwoProduct) and summed exactly in a floating-point expansion, so a
//    merged coefficient is the exact sum rounded once to the nearest double;
//    exact cancellation gives exactly zero.
//  * Truncation, Section III-B (non-Clifford paragraph): a merged term whose
//    modulus is strictly below a threshold is removed.
//  * Commutation, Section III-A: two strings anticommute when the number of
//    qubits holding two different non-identity letters is odd.
//  * Rotation step, Section III-B eq. (5): with R = cos(theta) I
//    - i sin(theta) P, "product" mode left-multiplies every term by R;
//    "conjugation" mode leaves a term Q that commutes with P unchanged and
//    maps an anticommuting Q to cos(theta) Q - i sin(theta) PQ.  Each step is
//    merged exactly, rounded, and truncated.
//
// Build: g++ -O2 -std=c++17 -ffp-contract=off -fPIC -shared oracle.cpp
// (contraction off so that the plain complex product matches a product
// computed without fused multiply-adds, operation for operation).
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <string>
#include <vector>

namespace {

enum : uint8_t { I_ = 0, X_ = 1, Y_ = 2, Z_ = 3 };

// Table I.
inline uint8_t letter_of(int xbit, int zbit) {
  if (!xbit && !zbit) return I_;
  if (!xbit && zbit) return Z_;
  if (xbit && !zbit) return X_;
  return Y_;
}
inline int xbit_of(uint8_t L) { return (L == X_ || L == Y_) ? 1 : 0; }
inline int zbit_of(uint8_t L) { return (L == Z_ || L == Y_) ? 1 : 0; }

// Single-qubit product a*b = i^k * letter, Section III-A.
struct Entry {
  uint8_t letter;
  uint8_t k;
};
const Entry TABLE[4][4] = {
    /* I* */ {{I_, 0}, {X_, 0}, {Y_, 0}, {Z_, 0}},
    /* X* */ {{X_, 0}, {I_, 0}, {Z_, 1}, {Y_, 3}},  // XY = iZ, XZ = -iY
    /* Y* */ {{Y_, 0}, {Z_, 3}, {I_, 0}, {X_, 1}},  // YX = -iZ, YZ = iX
    /* Z* */ {{Z_, 0}, {Y_, 1}, {X_, 3}, {I_, 0}},  // ZX = iY, ZY = -iX
};

// Test hook: lets a test plant a wrong table entry to show that the pins
// catch it.  Never set outside the oracle's own mutation tests.
Entry g_table[4][4];
bool g_table_init = false;
void table_init() {
  if (!g_table_init) {
    std::memcpy(g_table, TABLE, sizeof(TABLE));
    g_table_init = true;
  }
}

inline int words_for(int n) { return (n + 63) / 64; }

std::string decode(int n, const uint64_t* x, const uint64_t* z) {
  std::string s(static_cast<size_t>(n), '\0');
  for (int q = 0; q < n; ++q) {
    int xb = static_cast<int>((x[q / 64] >> (q % 64)) & 1u);
    int zb = static_cast<int>((z[q / 64] >> (q % 64)) & 1u);
    s[static_cast<size_t>(q)] = static_cast<char>(letter_of(xb, zb));
  }
  return s;
}

void encode(int n, const std::string& s, uint64_t* x, uint64_t* z) {
  const int W = words_for(n);
  for (int w = 0; w < W; ++w) x[w] = z[w] = 0;
  for (int q = 0; q < n; ++q) {
    uint8_t L = static_cast<uint8_t>(s[static_cast<size_t>(q)]);
    if (xbit_of(L)) x[q / 64] |= (uint64_t{1} << (q % 64));
    if (zbit_of(L)) z[q / 64] |= (uint64_t{1} << (q % 64));
  }
}

// Letter-by-letter product; returns the accumulated exponent of i (mod 4).
int multiply(const std::string& a, const std::string& b, std::string& out) {
  table_init();
  out.assign(a.size(), '\0');
  int k = 0;
  for (size_t q = 0; q < a.size(); ++q) {
    const Entry& e = g_table[static_cast<uint8_t>(a[q])][static_cast<uint8_t>(b[q])];
    out[q] = static_cast<char>(e.letter);
    k += e.k;
  }
  return k & 3;
}

// Multiply a complex number by i^k exactly (a swap and/or sign change).
inline void rot(int k, double re, double im, double& ore, double& oim) {
  switch (k & 3) {
    case 0: ore = re;  oim = im;  break;
    case 1: ore = -im; oim = re;  break;
    case 2: ore = -re; oim = -im; break;
    default: ore = im; oim = -re; break;
  }
}

// Exact accumulator: a nonoverlapping floating-point expansion (Shewchuk,
// "Adaptive Precision Floating-Point Arithmetic", 1997), grown one addend at
// a time with TwoSum (Knuth).  Its value is the exact sum of every addend.
struct Expansion {
  std::vector<double> p;  // partials, increasing magnitude, nonoverlapping
};
inline void exp_add(Expansion& e, double x) {
  if (x == 0.0) return;
  size_t i = 0;
  for (size_t t = 0; t < e.p.size(); ++t) {
    double y = e.p[t];
    if (std::fabs(x) < std::fabs(y)) std::swap(x, y);
    double hi = x + y;
    double lo = y - (hi - x);
    if (lo != 0.0) e.p[i++] = lo;
    x = hi;
  }
  e.p.resize(i);
  e.p.push_back(x);
}
// The exact value of the expansion rounded to the nearest double (ties to
// even), the final step of the exact-summation recipe built on Shewchuk's
// expansions (the method behind Python's math.fsum).
inline double exp_round(const Expansion& e) {
  const size_t n = e.p.size();
  if (n == 0) return 0.0;
  size_t i = n - 1;
  double hi = e.p[i], lo = 0.0;
  while (i > 0) {
    double x = hi, y = e.p[--i];
    hi = x + y;
    double yr = hi - x;
    lo = y - yr;
    if (lo != 0.0) break;
  }
  if (i > 0 && ((lo < 0.0 && e.p[i - 1] < 0.0) || (lo > 0.0 && e.p[i - 1] > 0.0))) {
    double y = lo * 2.0;
    double x = hi + y;
    double yr = x - hi;
    if (y == yr) hi = x;
  }
  return hi;
}
// Dekker's TwoProduct, with the error term from a fused multiply-add:
// a*b == p + e exactly.
inline void two_prod(double a, double b, double& p, double& e) {
  p = a * b;
  e = std::fma(a, b, -p);
}

struct Acc {
  Expansion re, im;
  double mass = 0.0;  // sum of |value| over the contributions
};

// Adds i^k * (c1 * c2) to acc, using the exact product (four two_prods).
void add_product(Acc& acc, int k, double a, double b, double c, double d) {
  double p[4], e[4];
  two_prod(a, c, p[0], e[0]);  // a*c
  two_prod(b, d, p[1], e[1]);  // b*d
  two_prod(a, d, p[2], e[2]);  // a*d
  two_prod(b, c, p[3], e[3]);  // b*c
  // re = ac - bd, im = ad + bc, each as four exact pieces.
  const double re_parts[4] = {p[0], e[0], -p[1], -e[1]};
  const double im_parts[4] = {p[2], e[2], p[3], e[3]};
  for (int t = 0; t < 4; ++t) {
    double r, i;
    rot(k, re_parts[t], 0.0, r, i);
    exp_add(acc.re, r);
    exp_add(acc.im, i);
    rot(k, 0.0, im_parts[t], r, i);
    exp_add(acc.re, r);
    exp_add(acc.im, i);
  }
  acc.mass += std::hypot(a, b) * std::hypot(c, d);
}

void add_value(Acc& acc, int k, double re, double im) {
  double r, i;
  rot(k, re, im, r, i);
  exp_add(acc.re, r);
  exp_add(acc.im, i);
  acc.mass += std::hypot(re, im);
}

// Truncation, Section III-B: is the modulus of re + i im strictly below t?
// Decided exactly: |c| < t  <=>  re^2 + im^2 < t^2.  Let a >= b be |re|, |im|.
// If a >= t the answer is no.  Otherwise multiply a, b and t by 2^-e with
// e = ilogb(t) (exact for every value that matters below), so that t lies in
// [1, 2).  If a < 2^-52, a^2 + b^2 < 2^-103 < t^2.  If b < 2^-52 the answer
// is yes too: t and a < t are doubles, so t^2 - a^2 = (t - a)(t + a) >=
// 2^-52 a > b a >= b^2.  In every remaining case the three squares are
// above 2^-104, TwoProduct splits each into two doubles exactly, and the
// exact sum of the six pieces is accumulated in an expansion; its largest
// component carries the sign.
bool below_threshold(double re, double im, double t) {
  if (!(t > 0.0)) return false;
  double a = std::fabs(re), b = std::fabs(im);
  if (b > a) std::swap(a, b);
  if (!(a < t)) return false;
  const int e = std::ilogb(t);
  a = std::ldexp(a, -e);
  b = std::ldexp(b, -e);
  t = std::ldexp(t, -e);
  const double small = std::ldexp(1.0, -52);
  if (a < small || b < small) return true;
  Expansion d;
  double p, q;
  two_prod(a, a, p, q);
  exp_add(d, p);
  exp_add(d, q);
  two_prod(b, b, p, q);
  exp_add(d, p);
  exp_add(d, q);
  two_prod(t, t, p, q);
  exp_add(d, -p);
  exp_add(d, -q);
  for (size_t k = d.p.size(); k > 0; --k)  // the largest nonzero component
    if (d.p[k - 1] != 0.0) return d.p[k - 1] < 0.0;
  return false;  // exactly |c| = t
}

struct Result {
  int n = 0;
  std::vector<std::string> keys;
  std::vector<double> coef;  // interleaved re, im
  std::vector<double> mass;
};

Result* finish(int n, const std::map<std::string, Acc>& m, double drop_abs) {
  Result* r = new Result;
  r->n = n;
  for (const auto& kv : m) {
    double re = exp_round(kv.second.re);
    double im = exp_round(kv.second.im);
    if (drop_abs >= 0.0 && below_threshold(re, im, drop_abs)) continue;
    r->keys.push_back(kv.first);
    r->coef.push_back(re);
    r->coef.push_back(im);
    r->mass.push_back(kv.second.mass);
  }
  return r;
}

struct Sum {
  int n;
  int64_t m;
  const uint64_t* x;
  const uint64_t* z;
  const uint8_t* ph;  // may be null (all zero)
  const double* c;    // interleaved re, im
  std::string letters(int64_t t) const {
    const int W = words_for(n);
    return decode(n, x + t * W, z + t * W);
  }
  int phase(int64_t t) const { return ph ? (ph[t] & 3) : 0; }
};

// Section III-A: anticommute iff an odd number of qubits hold two different
// non-identity letters.
int anticommutes(const std::string& a, const std::string& b) {
  int c = 0;
  for (size_t q = 0; q < a.size(); ++q)
    if (a[q] != I_ && b[q] != I_ && a[q] != b[q]) ++c;
  return c & 1;
}

}  // namespace

extern "C" {

int oracle_abi_version(void) { return 1; }

// Overwrites one entry of the single-qubit table (mutation tests only);
// oracle_table_reset restores the paper's table.
void oracle_table_set(int a, int b, int letter, int k) {
  table_init();
  g_table[a & 3][b & 3].letter = static_cast<uint8_t>(letter & 3);
  g_table[a & 3][b & 3].k = static_cast<uint8_t>(k & 3);
}
void oracle_table_reset(void) {
  std::memcpy(g_table, TABLE, sizeof(TABLE));
  g_table_init = true;
}

// Letters of m packed strings: out[t*n + q] in {0:I, 1:X, 2:Y, 3:Z}.
void oracle_decode(int n, int64_t m, const uint64_t* x, const uint64_t* z, uint8_t* out) {
  const int W = words_for(n);
  for (int64_t t = 0; t < m; ++t) {
    std::string s = decode(n, x + t * W, z + t * W);
    std::memcpy(out + t * n, s.data(), static_cast<size_t>(n));
  }
}

// One product (i^k1 P1)(i^k2 P2) = i^k3 P3; returns k3, writes P3's words.
int oracle_mul(int n, const uint64_t* x1, const uint64_t* z1, int k1, const uint64_t* x2,
               const uint64_t* z2, int k2, uint64_t* x3, uint64_t* z3) {
  std::string a = decode(n, x1, z1), b = decode(n, x2, z2), c;
  int k = multiply(a, b, c);
  encode(n, c, x3, z3);
  return (k1 + k2 + k) & 3;
}

// Unmerged outer product H1*H2 (Section IV-C): output p = j*m1 + i holds
// a_i * b_j with the phase exponent kept separate and the coefficient c1*c2
// computed as re = ac - bd, im = ad + bc in double precision.
int oracle_outer_product(int n, int64_t m1, const uint64_t* x1, const uint64_t* z1,
                         const uint8_t* ph1, const double* c1, int64_t m2, const uint64_t* x2,
                         const uint64_t* z2, const uint8_t* ph2, const double* c2, uint64_t* xo,
                         uint64_t* zo, uint8_t* pho, double* co) {
  const Sum A{n, m1, x1, z1, ph1, c1}, B{n, m2, x2, z2, ph2, c2};
  const int W = words_for(n);
  std::vector<std::string> la(static_cast<size_t>(m1));
  for (int64_t i = 0; i < m1; ++i) la[static_cast<size_t>(i)] = A.letters(i);
  std::string prod;
  for (int64_t j = 0; j < m2; ++j) {
    std::string lb = B.letters(j);
    const double c = c2[2 * j], d = c2[2 * j + 1];
    for (int64_t i = 0; i < m1; ++i) {
      const int64_t p = j * m1 + i;
      int k = multiply(la[static_cast<size_t>(i)], lb, prod);
      encode(n, prod, xo + p * W, zo + p * W);
      pho[p] = static_cast<uint8_t>((A.phase(i) + B.phase(j) + k) & 3);
      const double a = c1[2 * i], b = c1[2 * i + 1];
      co[2 * p] = a * c - b * d;
      co[2 * p + 1] = a * d + b * c;
    }
  }
  return 0;
}

// Sort-and-combine of one sum (Section III-H): the value of term t is
// i^{ph[t]} * c[t]; output phases are zero.
void* oracle_merge(int n, int64_t m, const uint64_t* x, const uint64_t* z, const uint8_t* ph,
                   const double* c, double drop_abs) {
  const Sum S{n, m, x, z, ph, c};
  std::map<std::string, Acc> acc;
  for (int64_t t = 0; t < m; ++t)
    add_value(acc[S.letters(t)], S.phase(t), c[2 * t], c[2 * t + 1]);
  return finish(n, acc, drop_abs);
}

// merge(H1*H2) over the pair block i in [i0,i1), j in [j0,j1) without
// materialising the products.
void* oracle_product_merge(int n, int64_t m1, const uint64_t* x1, const uint64_t* z1,
                           const uint8_t* ph1, const double* c1, int64_t m2, const uint64_t* x2,
                           const uint64_t* z2, const uint8_t* ph2, const double* c2,
                           double drop_abs, int64_t i0, int64_t i1, int64_t j0, int64_t j1) {
  const Sum A{n, m1, x1, z1, ph1, c1}, B{n, m2, x2, z2, ph2, c2};
  if (i1 > m1) i1 = m1;
  if (j1 > m2) j1 = m2;
  std::vector<std::string> la;
  for (int64_t i = i0; i < i1; ++i) la.push_back(A.letters(i));
  std::map<std::string, Acc> acc;
  std::string prod;
  for (int64_t j = j0; j < j1; ++j) {
    std::string lb = B.letters(j);
    for (int64_t i = i0; i < i1; ++i) {
      int k = multiply(la[static_cast<size_t>(i - i0)], lb, prod);
      k = (k + A.phase(i) + B.phase(j)) & 3;
      add_product(acc[prod], k, c1[2 * i], c1[2 * i + 1], c2[2 * j], c2[2 * j + 1]);
    }
  }
  return finish(n, acc, drop_abs);
}

// The commutator [H1, H2] = H1*H2 - H2*H1, merged.  For each pair both
// orders are multiplied letter by letter; when the two products differ (the
// strings anticommute, Section III-A, and the phases differ by 2), the pair
// contributes a_i b_j - b_j a_i to the product's string, summed exactly.
// Pairs whose two orders agree contribute nothing and create no term.
void* oracle_commutator(int n, int64_t m1, const uint64_t* x1, const uint64_t* z1,
                        const uint8_t* ph1, const double* c1, int64_t m2, const uint64_t* x2,
                        const uint64_t* z2, const uint8_t* ph2, const double* c2,
                        double drop_abs) {
  const Sum A{n, m1, x1, z1, ph1, c1}, B{n, m2, x2, z2, ph2, c2};
  std::vector<std::string> la;
  for (int64_t i = 0; i < m1; ++i) la.push_back(A.letters(i));
  std::map<std::string, Acc> acc;
  std::string ab, ba;
  for (int64_t j = 0; j < m2; ++j) {
    const std::string lb = B.letters(j);
    for (int64_t i = 0; i < m1; ++i) {
      const int kab = multiply(la[static_cast<size_t>(i)], lb, ab);
      const int kba = multiply(lb, la[static_cast<size_t>(i)], ba);
      if (ab != ba) return nullptr;  // both orders give one string; cannot fail
      if (((kab - kba) & 3) == 0) continue;  // the orders agree: no contribution
      const int k = A.phase(i) + B.phase(j);
      Acc& a = acc[ab];
      add_product(a, kab + k, c1[2 * i], c1[2 * i + 1], c2[2 * j], c2[2 * j + 1]);
      add_product(a, kba + k + 2, c1[2 * i], c1[2 * i + 1], c2[2 * j], c2[2 * j + 1]);  // minus b_j a_i
    }
  }
  return finish(n, acc, drop_abs);
}

// A sequence of rotation steps (Section III-B eq. (5)) applied to the merged
// input sum.  Step s uses the string (px, pz)[s] and angle theta[s]; mode 0
// multiplies every term on the left by cos(theta) I - i sin(theta) P, mode 1
// conjugates (commuting terms unchanged).  After each step equal strings are
// combined exactly, rounded to double and truncated at drop_abs.  The mass
// returned is that of the last step's contributions.
void* oracle_propagate(int n, int64_t m, const uint64_t* x, const uint64_t* z, const uint8_t* ph,
                       const double* c, int steps, const uint64_t* px, const uint64_t* pz,
                       const double* theta, int mode, double drop_abs) {
  const Sum S{n, m, x, z, ph, c};
  const int W = words_for(n);
  std::map<std::string, Acc> acc;
  for (int64_t t = 0; t < m; ++t)
    add_value(acc[S.letters(t)], S.phase(t), c[2 * t], c[2 * t + 1]);
  Result* cur = finish(n, acc, -1.0);
  std::string prod;
  for (int st = 0; st < steps; ++st) {
    const std::string P = decode(n, px + static_cast<size_t>(st) * W, pz + static_cast<size_t>(st) * W);
    const double co = std::cos(theta[st]), si = std::sin(theta[st]);
    std::map<std::string, Acc> next;
    for (size_t u = 0; u < cur->keys.size(); ++u) {
      const std::string& Q = cur->keys[u];
      const double re = cur->coef[2 * u], im = cur->coef[2 * u + 1];
      if (mode == 1 && !anticommutes(P, Q)) {
        add_value(next[Q], 0, re, im);
        continue;
      }
      add_product(next[Q], 0, re, im, co, 0.0);          // cos(theta) Q
      const int k = multiply(P, Q, prod);                 // P Q = i^k (letters)
      add_product(next[prod], k + 3, re, im, si, 0.0);    // -i sin(theta) P Q
    }
    delete cur;
    cur = finish(n, next, drop_abs);
  }
  return cur;
}

int64_t oracle_result_size(void* h) {
  return static_cast<int64_t>(static_cast<Result*>(h)->keys.size());
}

// Copies a result out: packed words [U][W], coefficients interleaved
// [U][2], contribution mass [U].  Any pointer may be null.
void oracle_result_copy(void* h, uint64_t* x, uint64_t* z, double* coef, double* mass) {
  const Result* r = static_cast<Result*>(h);
  const int W = words_for(r->n);
  for (size_t u = 0; u < r->keys.size(); ++u) {
    if (x && z) encode(r->n, r->keys[u], x + u * W, z + u * W);
    if (coef) {
      coef[2 * u] = r->coef[2 * u];
      coef[2 * u + 1] = r->coef[2 * u + 1];
    }
    if (mass) mass[u] = r->mass[u];
  }
}

void oracle_result_free(void* h) { delete static_cast<Result*>(h); }

// Coefficient of given strings s in merge(H1*H2), one query at a time: for
// each left term a_i the only right strings that can give s are those equal
// (as letters) to a_i * s, found by lookup; each match contributes
// i^k * c1 * c2 with k from the table.  Writes coefficient (interleaved),
// mass and the number of contributing pairs per query.
int oracle_product_coeff(int n, int64_t m1, const uint64_t* x1, const uint64_t* z1,
                         const uint8_t* ph1, const double* c1, int64_t m2, const uint64_t* x2,
                         const uint64_t* z2, const uint8_t* ph2, const double* c2, int64_t nq,
                         const uint64_t* xq, const uint64_t* zq, double* coef, double* mass,
                         int64_t* count) {
  const Sum A{n, m1, x1, z1, ph1, c1}, B{n, m2, x2, z2, ph2, c2};
  const int W = words_for(n);
  std::vector<std::string> la;
  for (int64_t i = 0; i < m1; ++i) la.push_back(A.letters(i));
  std::map<std::string, std::vector<int64_t>> index;
  for (int64_t j = 0; j < m2; ++j) index[B.letters(j)].push_back(j);
  std::string need, prod;
  for (int64_t q = 0; q < nq; ++q) {
    const std::string s = decode(n, xq + q * W, zq + q * W);
    Acc acc;
    int64_t cnt = 0;
    for (int64_t i = 0; i < m1; ++i) {
      multiply(la[static_cast<size_t>(i)], s, need);  // letters of a_i * s
      auto it = index.find(need);
      if (it == index.end()) continue;
      for (int64_t j : it->second) {
        int k = multiply(la[static_cast<size_t>(i)], need, prod);
        if (prod != s) return -1;  // cannot happen for a correct table
        k = (k + A.phase(i) + B.phase(j)) & 3;
        add_product(acc, k, c1[2 * i], c1[2 * i + 1], c2[2 * j], c2[2 * j + 1]);
        ++cnt;
      }
    }
    coef[2 * q] = exp_round(acc.re);
    coef[2 * q + 1] = exp_round(acc.im);
    if (mass) mass[q] = acc.mass;
    if (count) count[q] = cnt;
  }
  return 0;
}

}  // extern "C"
