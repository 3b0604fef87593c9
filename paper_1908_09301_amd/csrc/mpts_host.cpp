// C ABI of the library: contexts, exact parsing and rounding of the
// problem's numbers on the host, workspace layout, and the calls that run
// the device kernels (include/mpts.h documents every entry point).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <numeric>
#include <tuple>
#include <mutex>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mpts.h"
#include "mpts_common.h"
#include "mpts_kernels.h"
#include "mpts_mfma.h"

using namespace mpts;

// ---------------------------------------------------------------------------
// Host big integers (little-endian 32-bit words, no leading zero words).
namespace {

typedef std::vector<uint32_t> Big;

void trim(Big &a) {
  while (!a.empty() && a.back() == 0) a.pop_back();
}

long long bitlen(const Big &a) {
  if (a.empty()) return 0;
  uint32_t t = a.back();
  int b = 0;
  while (t) {
    ++b;
    t >>= 1;
  }
  return 32LL * (long long)(a.size() - 1) + b;
}

void mul_small_add(Big &a, uint32_t m, uint32_t add) {
  uint64_t c = add;
  for (auto &w : a) {
    uint64_t t = (uint64_t)w * m + c;
    w = (uint32_t)t;
    c = t >> 32;
  }
  if (c) a.push_back((uint32_t)c);
}

Big shl(const Big &a, long long s) {
  if (a.empty()) return a;
  long long ws = s / 32;
  int bs = (int)(s % 32);
  Big r((size_t)ws, 0u);
  uint32_t carry = 0;
  for (uint32_t w : a) {
    r.push_back((w << bs) | carry);
    carry = bs ? (w >> (32 - bs)) : 0;
  }
  if (carry) r.push_back(carry);
  trim(r);
  return r;
}

int cmp(const Big &a, const Big &b) {
  if (a.size() != b.size()) return a.size() < b.size() ? -1 : 1;
  for (size_t i = a.size(); i-- > 0;)
    if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
  return 0;
}

void sub_in(Big &a, const Big &b) {  // a -= b, a >= b
  int64_t br = 0;
  for (size_t i = 0; i < a.size(); ++i) {
    int64_t t = (int64_t)a[i] - (i < b.size() ? b[i] : 0) - br;
    br = t < 0;
    a[i] = (uint32_t)(t + (br ? (1LL << 32) : 0));
  }
  trim(a);
}

bool get_bit(const Big &a, long long i) {
  size_t w = (size_t)(i / 32);
  return w < a.size() && ((a[w] >> (i % 32)) & 1u);
}

// floor(n / d) and n mod d by binary long division (d > 0)
void divmod(const Big &n, const Big &d, Big &q, Big &r) {
  q.assign((n.size()), 0u);
  r.clear();
  for (long long i = bitlen(n) - 1; i >= 0; --i) {
    r = shl(r, 1);
    if (get_bit(n, i)) {
      if (r.empty()) r.push_back(1u);
      else r[0] |= 1u;
    }
    if (cmp(r, d) >= 0) {
      sub_in(r, d);
      q[(size_t)(i / 32)] |= 1u << (i % 32);
    }
  }
  trim(q);
}

struct Rational {
  int neg = 0;
  Big num, den;  // den > 0
};

Big pow10(long long e) {
  Big r{1u};
  for (long long i = 0; i < e; ++i) mul_small_add(r, 10u, 0u);
  return r;
}

Big mul(const Big &a, const Big &b) {
  if (a.empty() || b.empty()) return Big();
  Big r(a.size() + b.size(), 0u);
  for (size_t i = 0; i < a.size(); ++i) {
    uint64_t c = 0;
    for (size_t j = 0; j < b.size(); ++j) {
      uint64_t t = (uint64_t)a[i] * b[j] + r[i + j] + c;
      r[i + j] = (uint32_t)t;
      c = t >> 32;
    }
    r[i + b.size()] += (uint32_t)c;
  }
  trim(r);
  return r;
}

// decimal: [+-]digits[.digits][(e|E)[+-]digits]
bool parse_decimal(const std::string &s, Rational &out) {
  size_t i = 0;
  out = Rational();
  if (i < s.size() && (s[i] == '+' || s[i] == '-')) out.neg = s[i++] == '-';
  bool any = false;
  long long frac_digits = 0;
  Big m;
  while (i < s.size() && isdigit((unsigned char)s[i])) {
    mul_small_add(m, 10, (uint32_t)(s[i++] - '0'));
    any = true;
  }
  if (i < s.size() && s[i] == '.') {
    ++i;
    while (i < s.size() && isdigit((unsigned char)s[i])) {
      mul_small_add(m, 10, (uint32_t)(s[i++] - '0'));
      ++frac_digits;
      any = true;
    }
  }
  if (!any) return false;
  long long ex = 0;
  if (i < s.size() && (s[i] == 'e' || s[i] == 'E')) {
    ++i;
    int eneg = 0;
    if (i < s.size() && (s[i] == '+' || s[i] == '-')) eneg = s[i++] == '-';
    bool ed = false;
    while (i < s.size() && isdigit((unsigned char)s[i])) {
      ex = ex * 10 + (s[i++] - '0');
      ed = true;
      if (ex > 100000) return false;
    }
    if (!ed) return false;
    if (eneg) ex = -ex;
  }
  if (i != s.size()) return false;
  trim(m);
  long long e10 = ex - frac_digits;
  if (e10 >= 0) {
    out.num = mul(m, pow10(e10));
    out.den = Big{1u};
  } else {
    out.num = m;
    out.den = pow10(-e10);
  }
  return true;
}

bool parse_number(const char *text, Rational &out) {
  if (!text) return false;
  std::string s(text);
  s.erase(std::remove_if(s.begin(), s.end(), [](char c) { return isspace((unsigned char)c); }),
          s.end());
  size_t sl = s.find('/');
  if (sl == std::string::npos) return parse_decimal(s, out);
  Rational a, b;
  if (!parse_decimal(s.substr(0, sl), a) || !parse_decimal(s.substr(sl + 1), b)) return false;
  if (b.num.empty()) return false;
  out.neg = a.neg ^ b.neg;
  out.num = mul(a.num, b.den);
  out.den = mul(a.den, b.num);
  return true;
}

// Round (num/den) * 2^exp2 to p bits, ties to even, into [sign, E, M[L]].
void round_rational(const Rational &q, long long exp2, int L, std::vector<int32_t> &nv) {
  nv.assign((size_t)L + 2, 0);
  if (q.num.empty()) return;
  const long long p = 32LL * L;
  long long k = p - (bitlen(q.num) - bitlen(q.den));
  Big Q, R, D;
  for (;;) {
    Big n = q.num;
    D = q.den;
    if (k >= 0) n = shl(n, k);
    else D = shl(D, -k);
    divmod(n, D, Q, R);
    long long b = bitlen(Q);
    if (b > p) k -= 1;
    else if (b < p) k += 1;
    else break;
  }
  // round: compare 2R with D
  Big R2 = shl(R, 1);
  int c = cmp(R2, D);
  bool up = c > 0 || (c == 0 && !Q.empty() && (Q[0] & 1u));
  if (up) {
    mul_small_add(Q, 1, 1);  // Q += 1
    if (bitlen(Q) > p) {
      Q = Big((size_t)L, 0u);
      Q[L - 1] = 0x80000000u;
      k -= 1;
    }
  }
  Q.resize((size_t)L, 0u);
  nv[0] = q.neg ? -1 : 1;
  nv[1] = (int32_t)(exp2 - k);
  for (int j = 0; j < L; ++j) nv[2 + j] = (int32_t)Q[j];
}

void negate_nv(std::vector<int32_t> &nv) { nv[0] = -nv[0]; }

double nv_to_double(const int32_t *nv, int L) {
  int s = nv[0];
  if (s == 0) return 0.0;
  long long E = nv[1];
  const uint32_t *M = (const uint32_t *)(nv + 2);
  long long top = E + 32LL * L - 1;  // exponent of the leading bit
  int prec = 53;
  if (top < -1022) prec = (int)(53 - (-1022 - top));
  if (top > 1023) return s > 0 ? INFINITY : -INFINITY;
  if (prec <= 0) {
    // below half the smallest subnormal, or exactly around it
    if (prec < 0) return s > 0 ? 0.0 : -0.0;
    // prec == 0: value in [2^-1075, 2^-1074): rounds to 2^-1074 unless it is exactly the tie
    bool rest = false;
    for (int j = 0; j < L; ++j) rest |= (j == L - 1) ? (M[j] != 0x80000000u) : (M[j] != 0u);
    double v = rest ? std::ldexp(1.0, -1074) : 0.0;
    return s > 0 ? v : -v;
  }
  // take the top `prec` bits, round bit and sticky
  long long nbits = 32LL * L;
  long long drop = nbits - prec;  // bits below the kept mantissa
  auto bit = [&](long long i) -> uint64_t {
    return (i >= 0 && i < nbits) ? ((M[i / 32] >> (i % 32)) & 1u) : 0u;
  };
  uint64_t mant = 0;
  for (int j = prec - 1; j >= 0; --j) mant = (mant << 1) | bit(drop + j);
  bool rb = drop >= 1 ? bit(drop - 1) : false;
  bool st = false;
  for (long long i = 0; i < drop - 1; ++i)
    if (bit(i)) {
      st = true;
      break;
    }
  if (rb && (st || (mant & 1u))) {
    mant += 1;
    if (mant >> prec) {
      mant >>= 1;
      drop += 1;
    }
  }
  double v = std::ldexp((double)mant, (int)(E + drop));
  return s > 0 ? v : -v;
}

void add_in(Big &a, const Big &b) {  // a += b
  if (a.size() < b.size()) a.resize(b.size(), 0u);
  uint64_t c = 0;
  for (size_t i = 0; i < a.size(); ++i) {
    uint64_t t = (uint64_t)a[i] + (i < b.size() ? b[i] : 0u) + c;
    a[i] = (uint32_t)t;
    c = t >> 32;
  }
  if (c) a.push_back((uint32_t)c);
}

// x^2 + y^2 + z^2 of a normalised state [sign, E, M[L]] x 3, computed
// exactly and rounded once to the nearest double.
double exact_sqnorm(const int32_t *st, int L) {
  std::vector<Big> sq;
  std::vector<long long> ex;
  for (int c = 0; c < 3; ++c) {
    const int32_t *nv = st + (size_t)c * (L + 2);
    if (nv[0] == 0) continue;
    Big m((const uint32_t *)(nv + 2), (const uint32_t *)(nv + 2) + L);
    trim(m);
    sq.push_back(mul(m, m));
    ex.push_back(2LL * nv[1]);
  }
  if (sq.empty()) return 0.0;
  const long long emin = *std::min_element(ex.begin(), ex.end());
  Big S;
  for (size_t k = 0; k < sq.size(); ++k) add_in(S, shl(sq[k], ex[k] - emin));
  trim(S);
  // the exact sum as a normalised value of Lb limbs (no rounding), then RNE
  const long long bits = bitlen(S);
  const int Lb = (int)((bits + 31) / 32);
  const long long up = 32LL * Lb - bits;
  Big M = shl(S, up);
  M.resize((size_t)Lb, 0u);
  std::vector<int32_t> nv((size_t)Lb + 2);
  nv[0] = 1;
  const long long E = emin - up;
  if (E < INT32_MIN || E > INT32_MAX) return E > 0 ? INFINITY : 0.0;
  nv[1] = (int32_t)E;
  for (int j = 0; j < Lb; ++j) nv[2 + j] = (int32_t)M[j];
  return nv_to_double(nv.data(), Lb);
}

// The loss of a final state (MPTS_LOSS_*), rounded once to double.
double loss_of_state(const int32_t *st, int L, int loss) {
  if (loss == MPTS_LOSS_SQNORM) return exact_sqnorm(st, L);
  return nv_to_double(st + (size_t)(loss - 1) * (L + 2), L);
}

}  // namespace

// ---------------------------------------------------------------------------
struct mpts_ctx {
  int L, N, nd, RS, WB, CM;
  uint64_t gen = 0;          // creation number, never reused (keys the graph cache)
  int mfma = 0;              // 1: early Cauchy products on the int8 matrix cores
  // step size n/d with small n, d (tau_d > 0; else 0): d tau_p = n + r 2^E
  // exactly, tau_m1 2^28 + tau_m0 = r 2^(E - 28 tau_e), tau_e = floor(E / 28)
  int tau_n = 0, tau_d = 0, tau_m0 = 0, tau_m1 = 0, tau_e = 0;
  std::vector<int32_t> cn;  // NCONST x (L+2) normalised constants
  int wgs = 0;
  int cus = 0;
  int max_per_cu = 0;
  size_t lds = 0;
  int last_G = 0;            // workgroups of the last single-trajectory launch
  int max_per_cu_adj = -1;  // -1: not queried yet; 0: the adjoint kernel does not fit
  size_t lds_adj = 0;
  std::string err;
};

namespace {

int set_err(mpts_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  return code;
}

int hip_err(mpts_ctx *c, hipError_t e, const char *where) {
  return set_err(c, MPTS_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

int choose_cm(int nd) {
  int need = task_digits(nd);
  for (int cm : {4, 8, 16, 32})
    if (64 * cm >= need) return cm;
  return -1;
}

struct Layout {
  size_t prof, sync, cnorm, state, consts, rows, gframes, coefs, ckpt, adj, inst, wgmap, total;
};

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int kMaxWG = 4096;
constexpr size_t kLdsPerCU = 160 * 1024;  // LDS one gfx950 workgroup can hold
constexpr int kMfmaMinDigits = 140;       // rows from which the matrix cores take the early products

// Workspace of one trajectory.  The parts every call uses come first (the
// batch takes a region up to `inst` per trajectory); the coefficient output
// of mpts_coefficients (with_coefs) and the checkpoints and adjoint rows of
// the checkpointed calls (ckpt) follow.
Layout layout(const mpts_ctx *c, long long nsteps, bool ckpt, int nwg, bool with_coefs = true) {
  Layout l;
  size_t o = 0;
  l.prof = o;
  o = al(o + (2 * PH_NPHASE + (size_t)kMaxWG * PROF_RANK) * 8);
  l.sync = o;
  o = al(o + SY_WORDS * 4);
  l.cnorm = o;
  o = al(o + (size_t)NCONST * (c->L + 2) * 4);
  l.state = o;
  o = al(o + (size_t)3 * (c->L + 2) * 4);
  l.consts = o;
  o = al(o + (size_t)NCONST * c->RS * 4);
  l.rows = o;
  o = al(o + (size_t)3 * (c->N + 1) * c->RS * 4);
  l.gframes = o;
  o = al(o + (size_t)2 * NFR * c->WB * 8);
  l.inst = o;
  o = al(o + sizeof(Inst));
  l.wgmap = o;
  o = al(o + (size_t)kMaxWG * 4);
  l.coefs = o;
  if (with_coefs) o = al(o + (size_t)3 * (c->N + 1) * (c->L + 2) * 4);
  l.ckpt = o;
  if (ckpt) o = al(o + (size_t)(nsteps + 1) * 3 * (c->L + 2) * 4);
  l.adj = o;
  if (ckpt)
    o = al(o + ((size_t)6 * c->N * c->RS + (size_t)3 * (c->N + 1) * c->RS + (size_t)6 * (c->L + 2)) * 4);
  l.total = o;
  (void)nwg;
  return l;
}

int check_device(mpts_ctx *c) {
  if (c->cus > 0) return MPTS_OK;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_err(c, e, "hipGetDevice");
  hipDeviceProp_t pr;
  e = hipGetDeviceProperties(&pr, dev);
  if (e != hipSuccess) return hip_err(c, e, "hipGetDeviceProperties");
  if (strncmp(pr.gcnArchName, "gfx950", 6) != 0)
    return set_err(c, MPTS_EARCH, std::string("device is ") + pr.gcnArchName + ", need gfx950");
  c->cus = pr.multiProcessorCount;
  c->lds = lds_bytes(c->L, c->N, c->RS, c->WB, c->CM, false, c->mfma != 0);
  int occ = max_coresident(c->CM, c->lds, &c->max_per_cu, false);
  if (occ != 0 || c->max_per_cu < 1) {
    char msg[160];
    snprintf(msg, sizeof(msg), "kernel does not fit one compute unit (CM %d, LDS %zu bytes, query %d, blocks %d)",
             c->CM, c->lds, occ, c->max_per_cu);
    return set_err(c, MPTS_EUNSUPPORTED, msg);
  }
  return MPTS_OK;
}

int bf_to_nv(const mpts_ctx *c, const mpts_bf &b, int32_t *nv) {
  if (b.sign == 0) {
    for (int j = 0; j < c->L + 2; ++j) nv[j] = 0;
    return MPTS_OK;
  }
  if (!b.limbs || (b.sign != 1 && b.sign != -1)) return MPTS_EINVAL;
  if (!(b.limbs[c->L - 1] & 0x80000000u)) return MPTS_EINVAL;
  nv[0] = b.sign;
  nv[1] = b.exp;
  for (int j = 0; j < c->L; ++j) nv[2 + j] = (int32_t)b.limbs[j];
  return MPTS_OK;
}

int nv_to_bf(const mpts_ctx *c, const int32_t *nv, mpts_bf *b) {
  if (!b || !b->limbs) return MPTS_EINVAL;
  b->sign = nv[0];
  b->exp = nv[0] ? nv[1] : 0;
  for (int j = 0; j < c->L; ++j) b->limbs[j] = (uint32_t)nv[2 + j];
  return MPTS_OK;
}

// The rounded step size tau_p = M 2^E (nv: sign, E, M of L limbs) of a
// step size n/d with n < 2^27, d < 2^13 satisfies d tau_p = n + r 2^E with
// r = d M - n 2^-E, |r| <= d / 2 (M is n 2^-E / d rounded to an integer).
// Each Horner step round(tau_p h + c) of equation (2) is then
// round((n h + r 2^E h + d c) / d): three multiples of rows by small
// integers and one short division instead of a p x p-bit product.  Leaves
// tau_d = 0 (the full product) for other step sizes and under
// MPTS_TAU=product.
struct TauRat {
  int n = 0, d = 0, m0 = 0, m1 = 0, e = 0;  // d = 0: the full product
};

TauRat tau_rational(const Rational &q, const std::vector<int32_t> &nv, int L) {
  TauRat t;
  const char *env = getenv("MPTS_TAU");
  if (env && strcmp(env, "product") == 0) return t;
  if (nv[0] == 0 || q.num.size() > 2 || q.den.size() > 2) return t;
  auto u64 = [](const Big &a) {
    uint64_t v = 0;
    for (size_t i = a.size(); i-- > 0;) v = (v << 32) | a[i];
    return v;
  };
  uint64_t n = u64(q.num), d = u64(q.den);
  const uint64_t g = std::gcd(n, d);
  n /= g;
  d /= g;
  const long long E = nv[1];
  if (n == 0 || n >= (1u << 27) || d == 0 || d >= (1u << 13) || E > 0) return t;
  Big M(nv.begin() + 2, nv.begin() + 2 + L);
  trim(M);
  Big dM = M;
  mul_small_add(dM, (uint32_t)d, 0u);
  const Big nk = shl(Big{(uint32_t)n}, -E);
  Big r;
  int rs = 1;
  if (cmp(dM, nk) >= 0) {
    r = dM;
    sub_in(r, nk);
  } else {
    r = nk;
    sub_in(r, dM);
    rs = -1;
  }
  if (bitlen(r) > 31) return t;
  const long long eE = E >= 0 ? E / DBITS : -((-E + DBITS - 1) / DBITS);
  const int tE = (int)(E - eE * DBITS);
  const long long m = (long long)nv[0] * rs * (long long)(r.empty() ? 0u : r[0]) * (1LL << tE);
  t.n = nv[0] * (int)n;
  t.d = (int)d;
  t.m0 = (int)(m & (long long)DMASK);
  t.m1 = (int)(m >> DBITS);
  t.e = (int)eE;
  return t;
}

int make_ctx(const char *sigma, const char *R, const char *b, int L, int N, const char *tau,
             mpts_ctx **out) {
  if (!out) return MPTS_EINVAL;
  *out = nullptr;
  if (L < 1 || L > 1024 || N < 1 || N > 8192) return MPTS_EINVAL;
  Rational qs, qr, qb, qt;
  if (!parse_number(sigma, qs) || !parse_number(R, qr) || !parse_number(b, qb) ||
      !parse_number(tau, qt))
    return MPTS_EINVAL;
  mpts_ctx *c = new mpts_ctx();
  static std::atomic<uint64_t> next_gen{1};
  c->gen = next_gen.fetch_add(1);
  c->L = L;
  c->N = N;
  c->nd = digits_per_row(L);
  c->RS = row_stride(c->nd);
  c->WB = frame_width(c->nd);
  c->CM = choose_cm(c->nd);
  if (c->CM < 0) {
    delete c;
    return MPTS_EUNSUPPORTED;
  }
  // Early products on the matrix cores for rows of at least kMfmaMinDigits
  // digits (below that the VALU tiles are faster) that the accumulators
  // hold (at most 487 digits); MPTS_EARLY=valu or =mfma overrides the size
  // rule (both paths give the same bits)
  const char *early = getenv("MPTS_EARLY");
  bool use = c->nd >= kMfmaMinDigits;
  if (early && strcmp(early, "valu") == 0) use = false;
  if (early && strcmp(early, "mfma") == 0) use = true;
  c->mfma = use && mf_fits(c->nd) ? 1 : 0;
  // the staging buffers must leave the forward and adjoint kernels within
  // one compute unit's LDS, else the VALU tiles take the early products
  if (c->mfma && (lds_bytes(L, N, c->RS, c->WB, c->CM, false, true) > kLdsPerCU ||
                  lds_bytes(L, N, c->RS, c->WB, c->CM, true, true) > kLdsPerCU))
    c->mfma = 0;
  c->cn.assign((size_t)NCONST * (L + 2), 0);
  std::vector<int32_t> nv;
  auto put = [&](int idx, const std::vector<int32_t> &v) {
    std::copy(v.begin(), v.end(), c->cn.begin() + (size_t)idx * (L + 2));
  };
  round_rational(qs, 0, L, nv);
  put(C_SIGMA, nv);
  negate_nv(nv);
  put(C_NSIGMA, nv);
  round_rational(qr, 0, L, nv);
  put(C_R, nv);
  round_rational(qb, 0, L, nv);
  negate_nv(nv);
  put(C_NB, nv);
  round_rational(qt, 0, L, nv);
  put(C_TAU, nv);
  const TauRat tr = tau_rational(qt, nv, L);
  c->tau_n = tr.n;
  c->tau_d = tr.d;
  c->tau_m0 = tr.m0;
  c->tau_m1 = tr.m1;
  c->tau_e = tr.e;
  Rational one;
  one.num = Big{1u};
  one.den = Big{1u};
  round_rational(one, 0, L, nv);
  put(C_ONE, nv);
  *out = c;
  return MPTS_OK;
}

// Modelled milliseconds per step of one trajectory on G workgroups (the
// batch planner's estimate for sizes it has not timed): the serial latency
// per coefficient index plus the product work spread over the group.  The
// latencies are measured at K=100/N=40, where the work is negligible: 1.09
// ms per step on one workgroup, about 0.7 on groups of 8 to 256.
double model_ms(const mpts_ctx *c, int G) {
  const double lat = G == 1 ? 0.0136 : 0.0088;
  const double digit_macs = (double)c->N * (c->N + 5) * c->nd * (double)c->nd;
  const double wg_rate = 2.6e13 / 256.0 * 0.25;  // sustained digit-MAC/s of one workgroup
  return (c->N * 2 * lat) + digit_macs / (G * wg_rate) * 1e3;
}

int run_single(mpts_ctx *c, int mode, long long nsteps, const void *x0_dev, void *xout_dev,
               void *ckpt_dev, void *ws, size_t ws_bytes, hipStream_t s, bool x0_on_host,
               const int32_t *x0_host, void *adj_dev = nullptr, int loss = 0) {
  int dst = check_device(c);
  if (dst != MPTS_OK) return dst;
  const bool adj = mode == MODE_ADJOINT;
  if (adj && c->max_per_cu_adj < 0) {
    c->lds_adj = lds_bytes(c->L, c->N, c->RS, c->WB, c->CM, true, c->mfma != 0);
    int occ = max_coresident(c->CM, c->lds_adj, &c->max_per_cu_adj, true);
    if (occ != 0) c->max_per_cu_adj = 0;
  }
  if (adj && c->max_per_cu_adj < 1)
    return set_err(c, MPTS_EUNSUPPORTED, "adjoint kernel does not fit one compute unit");
  // automatic: every compute unit (measured fastest for one trajectory from
  // K=100/N=40 up, e.g. 0.69 ms per step there against 1.09 ms on one)
  int G = c->wgs > 0 ? c->wgs : c->cus;
  G = std::min(G, c->cus * (adj ? std::min(c->max_per_cu, c->max_per_cu_adj) : c->max_per_cu));
  G = std::max(std::min(G, kMaxWG), 1);
  Layout l = layout(c, nsteps, false, G, mode == MODE_COEFFS);
  if (ws_bytes < l.total) return set_err(c, MPTS_ENOSPC, "workspace too small");
  char *base = (char *)ws;
  hipError_t e;
  const bool phases = getenv("MPTS_PHASES") != nullptr;
  if (phases) {
    e = launch_clear(base + l.prof, (2 * PH_NPHASE + (size_t)G * PROF_RANK) * 8, s);
    if (e != hipSuccess) return hip_err(c, e, "clear");
  }
  e = launch_clear(base + l.sync, SY_WORDS * 4, s);
  if (e != hipSuccess) return hip_err(c, e, "clear");
  e = launch_clear(base + l.gframes, (size_t)2 * NFR * c->WB * 8, s);
  if (e != hipSuccess) return hip_err(c, e, "clear");
  e = hipMemcpyAsync(base + l.cnorm, c->cn.data(), c->cn.size() * 4, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_err(c, e, "copy constants");
  size_t sb = (size_t)3 * (c->L + 2) * 4;
  if (x0_on_host) e = hipMemcpyAsync(base + l.state, x0_host, sb, hipMemcpyHostToDevice, s);
  else e = hipMemcpyAsync(base + l.state, x0_dev, sb, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return hip_err(c, e, "copy state");
  Inst I;
  memset(&I, 0, sizeof(I));
  I.L = c->L;
  I.N = c->N;
  I.nd = c->nd;
  I.RS = c->RS;
  I.WB = c->WB;
  I.CM = c->CM;
  I.G = G;
  I.wg0 = 0;
  I.mode = mode;
  I.loss = loss;
  I.mfma = c->mfma;
  I.nsteps = nsteps;
  I.tau_n = c->tau_n;
  I.tau_d = c->tau_d;
  I.tau_m0 = c->tau_m0;
  I.tau_m1 = c->tau_m1;
  I.tau_e = c->tau_e;
  I.rows = (int32_t *)(base + l.rows);
  I.consts = (int32_t *)(base + l.consts);
  I.cnorm = (int32_t *)(base + l.cnorm);
  I.state = (int32_t *)(base + l.state);
  I.coefs = mode == MODE_COEFFS ? (int32_t *)(base + l.coefs) : nullptr;
  I.ckpt = (int32_t *)ckpt_dev;
  I.gframes = (long long *)(base + l.gframes);
  I.sync = (uint32_t *)(base + l.sync);
  I.adj = (int32_t *)adj_dev;
  I.prof = phases ? (unsigned long long *)(base + l.prof) : nullptr;
  c->last_G = G;
  e = hipMemcpyAsync(base + l.inst, &I, sizeof(I), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_err(c, e, "copy descriptor");
  e = launch_clear(base + l.wgmap, (size_t)G * 4, s);
  if (e != hipSuccess) return hip_err(c, e, "clear");
  if (mode == MODE_ADJOINT)
    e = launch_adj((const Inst *)(base + l.inst), (const int *)(base + l.wgmap), G, c->CM, c->lds_adj,
                   s);
  else
    e = launch_run((const Inst *)(base + l.inst), (const int *)(base + l.wgmap), G, c->CM, c->lds,
                   s, true);
  if (e != hipSuccess) return hip_err(c, e, "launch");
  if (xout_dev) {
    e = hipMemcpyAsync(xout_dev, base + l.state, sb, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_err(c, e, "copy state out");
  }
  return MPTS_OK;
}

int read_status(mpts_ctx *c, void *ws, hipStream_t s) {
  Layout l = layout(c, 0, false, 1);
  uint32_t w = 0;
  hipError_t e = hipMemcpyAsync(&w, (char *)ws + l.sync + SY_ERROR * 4, 4, hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return hip_err(c, e, "read status");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_err(c, e, "synchronize");
  if (getenv("MPTS_PHASES")) {
    unsigned long long ph[2 * PH_NPHASE];
    if (hipMemcpy(ph, (char *)ws + l.prof, sizeof(ph), hipMemcpyDeviceToHost) == hipSuccess) {
      int rate = 0;
      int dev = 0;
      (void)hipGetDevice(&dev);
      (void)hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, dev);
      double us = rate > 0 ? 1e3 / rate : 0.0;  // rate in kHz
      static const char *nm[16] = {"setup", "accum", "flush", "wait", "final", "release", "horner",
                                   "step0", "spare", "f.round1", "arrlag", "f.div", "f.row", "h.prod", "h.div", "h.round"};
      fprintf(stderr, "mpts phases (us):");
      for (int w2 = 0; w2 < 2; ++w2) {
        fprintf(stderr, w2 ? "\n  wg1:" : "\n  leader:");
        for (int j = 0; j < (w2 ? 8 : 16); ++j) fprintf(stderr, " %s=%.1f", nm[j], ph[w2 * PH_NPHASE + j] * us);
        if (w2)
          fprintf(stderr, " e.build=%.1f e.setup=%.1f e.stage=%.1f e.mma=%.1f e.flush=%.1f e.bar=%.1f",
                  ph[PH_NPHASE + PH_EBUILD] * us, ph[PH_NPHASE + PH_ESETUP] * us,
                  ph[PH_NPHASE + 9] * us, ph[PH_NPHASE + 11] * us, ph[PH_NPHASE + 12] * us,
                  ph[PH_NPHASE + 13] * us);
      }
      fprintf(stderr, "\n");
      const int G = c->last_G;
      std::vector<unsigned long long> pr((size_t)G * PROF_RANK);
      if (G > 0 && hipMemcpy(pr.data(), (char *)ws + l.prof + 2 * PH_NPHASE * 8, pr.size() * 8,
                             hipMemcpyDeviceToHost) == hipSuccess) {
        static const char *rn[5] = {"setup", "accum", "flush", "release", "final"};
        static const int rs[5] = {0, 1, 2, 3, 6};
        for (int q = 0; q < 5; ++q) {
          std::vector<std::pair<double, int>> v;
          for (int r = 0; r < G; ++r) v.push_back({pr[(size_t)r * PROF_RANK + rs[q]] * us, r});
          std::sort(v.begin(), v.end());
          fprintf(stderr, "  per-wg %s: min %.1f (wg %d) med %.1f max %.1f (wg %d) p90 %.1f\n", rn[q],
                  v[0].first, v[0].second, v[G / 2].first, v[G - 1].first, v[G - 1].second,
                  v[(G * 9) / 10].first);
          if (q == 4 && G > 8) {
            // the slowest followers' (xcc, se/cu) places
            fprintf(stderr, "  slowest final:");
            for (int k = G - 1; k >= G - 6 && k >= 1; --k) {
              const int r = v[k].second;
              const unsigned x = (unsigned)pr[(size_t)r * PROF_RANK + 4], hw = (unsigned)pr[(size_t)r * PROF_RANK + 5];
              fprintf(stderr, " wg%d %.1f (xcc %u hw 0x%x)", r, v[k].first, x, hw);
            }
            fprintf(stderr, "\n  fastest final:");
            for (int k = 1; k <= 5 && k < G; ++k) {
              const int r = v[k].second;
              const unsigned x = (unsigned)pr[(size_t)r * PROF_RANK + 4], hw = (unsigned)pr[(size_t)r * PROF_RANK + 5];
              fprintf(stderr, " wg%d %.1f (xcc %u hw 0x%x)", r, v[k].first, x, hw);
            }
            fprintf(stderr, "\n");
          }
        }
        std::map<unsigned, int> cu;
        int xcc_ok = 0;
        for (int r = 0; r < G; ++r) {
          unsigned x = (unsigned)pr[(size_t)r * PROF_RANK + 4], hw = (unsigned)pr[(size_t)r * PROF_RANK + 5];
          cu[(x << 16) | ((hw >> 8) & 0xff)]++;
          if ((int)x == r % 8) ++xcc_ok;
        }
        int shared = 0;
        for (auto &kv : cu) shared += kv.second > 1 ? kv.second : 0;
        fprintf(stderr, "  placement: %d of %d workgroups on xcc rank%%8; %d distinct (xcc, cu/se) slots, %d workgroups sharing one\n",
                xcc_ok, G, (int)cu.size(), shared);
      }
    }
  }
  if (w & 4u) return set_err(c, MPTS_EHIP, "device synchronisation timed out");
  if (w & 8u) return set_err(c, MPTS_EUNSUPPORTED, "per-term offset table overflow");
  if (w & 3u) {
    char msg[96];
    snprintf(msg, sizeof(msg), "%s (device status 0x%x)",
             (w & 1u) ? "exact sum outside the device window" : "exponent overflow in rounding", w);
    return set_err(c, MPTS_ERANGE, msg);
  }
  return MPTS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Batched ensembles: one launch, trajectory t on G[t] workgroups.
namespace {

struct BatchLayout {
  std::vector<size_t> region;      // byte offset of each trajectory's region
  std::vector<size_t> state_off;   // int32 offset of each packed state in `states`
  size_t insts = 0, wgmap = 0, states = 0, total = 0;
  size_t states_words = 0;
  size_t max_single = 0;           // largest single-trajectory layout (autotune probes)
  int CM = 4;
  size_t lds = 0;
};

int batch_layout(mpts_ctx *const *ctxs, int count, BatchLayout &bl) {
  bl = BatchLayout();
  size_t o = 0;
  bl.insts = o;
  o = al(o + (size_t)count * sizeof(Inst));
  bl.wgmap = o;
  o = al(o + (size_t)kMaxWG * 4);
  bl.states = o;
  for (int t = 0; t < count; ++t) {
    bl.state_off.push_back(bl.states_words);
    bl.states_words += (size_t)3 * (ctxs[t]->L + 2);
  }
  o = al(o + bl.states_words * 4);
  int maxnd = 0;
  for (int t = 0; t < count; ++t) {
    mpts_ctx *c = ctxs[t];
    bl.region.push_back(o);
    o = al(o + layout(c, 0, false, 1).inst);
    bl.max_single = std::max(bl.max_single, layout(c, 2, false, kMaxWG).total);
    maxnd = std::max(maxnd, c->nd);
  }
  bl.total = std::max(o, bl.max_single);
  bl.CM = choose_cm(maxnd);
  if (bl.CM < 0) return MPTS_EUNSUPPORTED;
  for (int t = 0; t < count; ++t) {
    mpts_ctx *c = ctxs[t];
    bl.lds = std::max(bl.lds, lds_bytes(c->L, c->N, c->RS, c->WB, bl.CM, false, c->mfma != 0));
  }
  return MPTS_OK;
}

// The graph and tuning caches are shared by every context of the process;
// g_cache_mu serialises their use (the kernels they launch are still
// ordered only by the caller's streams).
std::mutex g_cache_mu;

// Measured milliseconds per step of one trajectory class at each of the
// group sizes kTuneG (filled by the autotuner), keyed by the device
// architecture and the class's (L, N).  With MPTS_TUNE_CACHE set to a file
// path the table is read from that file once and every new entry appended
// to it ("arch L N ms..." per line), so later processes skip the probes.
constexpr int kTuneN = 6;
constexpr int kTuneG[kTuneN] = {1, 2, 4, 8, 16, 32};
struct TuneKey {
  std::string arch;
  int L, N;
  bool operator<(const TuneKey &o) const {
    if (arch != o.arch) return arch < o.arch;
    if (L != o.L) return L < o.L;
    return N < o.N;
  }
};
std::map<TuneKey, std::vector<double>> g_tune;
bool g_tune_loaded = false;

std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t pr;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&pr, dev) != hipSuccess)
    return "unknown";
  std::string a(pr.gcnArchName);
  size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

void tune_load() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char *path = getenv("MPTS_TUNE_CACHE");
  if (!path || !*path) return;
  FILE *f = fopen(path, "r");
  if (!f) return;
  char arch[64];
  int L, N;
  while (fscanf(f, "%63s %d %d", arch, &L, &N) == 3) {
    std::vector<double> ms(kTuneN, -1.0);
    bool ok = true;
    for (int k = 0; k < kTuneN && ok; ++k) ok = fscanf(f, "%lf", &ms[k]) == 1;
    if (!ok) break;
    g_tune[TuneKey{arch, L, N}] = ms;
  }
  fclose(f);
}

void tune_store(const TuneKey &k, const std::vector<double> &ms) {
  g_tune[k] = ms;
  const char *path = getenv("MPTS_TUNE_CACHE");
  if (!path || !*path) return;
  FILE *f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s %d %d", k.arch.c_str(), k.L, k.N);
  for (double v : ms) fprintf(f, " %.6f", v);
  fprintf(f, "\n");
  fclose(f);
}

double step_ms(const mpts_ctx *c, int G, const std::string &arch) {
  auto it = g_tune.find(TuneKey{arch, c->L, c->N});
  if (it != g_tune.end()) {
    // a group size the tuner did not time (it stopped once larger groups
    // got slower) is not a candidate
    for (int k = 0; k < kTuneN; ++k)
      if (kTuneG[k] == G) return it->second[k] > 0 ? it->second[k] : 1e30;
    return 1e30;
  }
  return model_ms(c, G);
}

// Time a few steps of one trajectory of context c at each group size of
// kTuneG (up to `gmax`), in the caller's workspace, and record them.
int autotune_class(mpts_ctx *c, void *ws, size_t ws_bytes, hipStream_t s, int gmax,
                   const std::string &arch) {
  if (g_tune.count(TuneKey{arch, c->L, c->N})) return MPTS_OK;
  std::vector<double> ms(kTuneN, -1.0);
  std::vector<int32_t> x((size_t)3 * (c->L + 2), 0);
  // a generic nonzero state: (1, 2, 3)
  for (int k = 0; k < 3; ++k) {
    Rational q;
    q.num = Big{(uint32_t)(k + 1)};
    q.den = Big{1u};
    std::vector<int32_t> nv;
    round_rational(q, 0, c->L, nv);
    std::copy(nv.begin(), nv.end(), x.begin() + (size_t)k * (c->L + 2));
  }
  const int saved = c->wgs;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return set_err(c, MPTS_EHIP, "event");
  int rc = MPTS_OK;
  for (int k = 0; k < kTuneN && rc == MPTS_OK; ++k) {
    if (kTuneG[k] > gmax) break;
    c->wgs = kTuneG[k];
    const long long steps = 2;
    rc = run_single(c, MODE_INTEGRATE, 1, nullptr, nullptr, nullptr, ws, ws_bytes, s, true, x.data());
    if (rc) break;
    (void)hipEventRecord(e0, s);
    rc = run_single(c, MODE_INTEGRATE, steps, nullptr, nullptr, nullptr, ws, ws_bytes, s, true,
                    x.data());
    (void)hipEventRecord(e1, s);
    if (rc) break;
    (void)hipEventSynchronize(e1);
    float t = 0.f;
    (void)hipEventElapsedTime(&t, e0, e1);
    ms[k] = t / steps;
    // a larger group that is already slower will not be chosen: stop probing
    if (k > 0 && ms[k] > ms[k - 1]) break;
  }
  c->wgs = saved;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  tune_store(TuneKey{arch, c->L, c->N}, ms);
  return MPTS_OK;
}

// Workgroups per trajectory: start with one each and repeatedly double the
// group of the trajectory with the longest predicted run while the launch
// still fits on the device at once.
// A batch schedule: slots of G workgroups, each running a list of
// trajectories one after another.
struct BatchPlan {
  std::vector<int> slot_G;                 // workgroups of each slot
  std::vector<std::vector<int>> slot_list; // trajectories of each slot, in order
  int total = 0;                           // workgroups of the launch
};

// Plans the batch: trajectories with the same (L, N, nsteps) form a class;
// for a makespan T each class takes, over the group sizes G of the tuning
// table, the fewest workgroups that finish it within T (m = floor(T / t(G))
// trajectories one after another per slot of G workgroups); the smallest T
// whose classes fit the resident workgroups is found by bisection.  Step
// times come from the tuner (MPTS_AUTOTUNE) or the model.
int plan_batch(mpts_ctx *const *ctxs, int count, const int64_t *nsteps, const BatchLayout &bl,
               bool autotune, void *ws, size_t ws_bytes, hipStream_t s, BatchPlan &plan) {
  mpts_ctx *c0 = ctxs[0];
  int per_cu = 0;
  if (max_coresident(bl.CM, bl.lds, &per_cu, false) != 0 || per_cu < 1)
    return set_err(c0, MPTS_EUNSUPPORTED, "kernel does not fit one compute unit");
  const int cap = std::min(c0->cus * per_cu, kMaxWG);
  std::lock_guard<std::mutex> lk(g_cache_mu);
  tune_load();
  const std::string arch = device_arch();
  const int gmax = std::max(1, std::min(kTuneG[kTuneN - 1], cap));
  if (autotune)
    for (int t = 0; t < count; ++t) {
      int st = autotune_class(ctxs[t], ws, ws_bytes, s, gmax, arch);
      if (st) return st;
    }
  // classes
  struct Cls {
    std::vector<int> members;
    double cost[kTuneN];  // ms of the whole run on kTuneG[k] workgroups (1e30: not a candidate)
    int G = 1, m = 1, slots = 0;
  };
  std::vector<Cls> cls;
  std::map<std::tuple<int, int, int64_t>, int> idx;
  for (int t = 0; t < count; ++t) {
    const auto key = std::make_tuple(ctxs[t]->L, ctxs[t]->N, (int64_t)nsteps[t]);
    auto it = idx.find(key);
    if (it == idx.end()) {
      Cls c;
      for (int k = 0; k < kTuneN; ++k)
        c.cost[k] = kTuneG[k] <= gmax ? std::max(1, (int)nsteps[t]) * step_ms(ctxs[t], kTuneG[k], arch)
                                      : 1e30;
      it = idx.emplace(key, (int)cls.size()).first;
      cls.push_back(c);
    }
    cls[it->second].members.push_back(t);
  }
  // workgroups class c needs to finish within T (and its choice), or -1
  auto need = [&](Cls &c, double T, bool keep) -> long long {
    long long best = -1;
    for (int k = 0; k < kTuneN; ++k) {
      if (c.cost[k] >= 1e29 || c.cost[k] > T) continue;
      const long long n = (long long)c.members.size();
      long long m = (long long)(T / c.cost[k]);
      if (m < 1) continue;
      if (m > n) m = n;
      const long long slots = (n + m - 1) / m, w = slots * kTuneG[k];
      if (best < 0 || w < best) {
        best = w;
        if (keep) {
          c.G = kTuneG[k];
          c.m = (int)m;
          c.slots = (int)slots;
        }
      }
    }
    return best;
  };
  auto feasible = [&](double T, bool keep) {
    long long used = 0;
    for (auto &c : cls) {
      const long long w = need(c, T, keep);
      if (w < 0) return false;
      used += w;
    }
    return used <= cap;
  };
  double hi = 0.0, lo = 0.0;
  for (auto &c : cls) {
    double best = 1e30;
    for (int k = 0; k < kTuneN; ++k) best = std::min(best, c.cost[k]);
    lo = std::max(lo, best);
    hi += best * (double)c.members.size();
  }
  plan = BatchPlan();
  if (!feasible(hi, false)) {
    // more classes than workgroups: one workgroup per slot, trajectories
    // dealt to the least loaded slot (largest first)
    const int nslot = std::min(cap, count);
    std::vector<double> load((size_t)nslot, 0.0);
    std::vector<int> order((size_t)count);
    for (int t = 0; t < count; ++t) order[t] = t;
    auto tcost = [&](int t) { return (double)std::max<int64_t>(1, nsteps[t]) * step_ms(ctxs[t], 1, arch); };
    std::sort(order.begin(), order.end(), [&](int x, int y) { return tcost(x) > tcost(y); });
    plan.slot_G.assign((size_t)nslot, 1);
    plan.slot_list.assign((size_t)nslot, {});
    for (int t : order) {
      const int sl = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      load[sl] += tcost(t);
      plan.slot_list[sl].push_back(t);
    }
    plan.total = nslot;
    return MPTS_OK;
  }
  lo = std::min(lo, hi);
  for (int it = 0; it < 60 && hi - lo > 1e-6 * hi; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (feasible(mid, false)) hi = mid;
    else lo = mid;
  }
  (void)feasible(hi, true);
  for (auto &c : cls) {
    const int base = (int)plan.slot_G.size();
    for (int k = 0; k < c.slots; ++k) {
      plan.slot_G.push_back(c.G);
      plan.slot_list.push_back({});
    }
    // round robin: the slots of a class differ by at most one trajectory
    for (size_t k = 0; k < c.members.size(); ++k)
      plan.slot_list[base + (int)(k % (size_t)c.slots)].push_back(c.members[k]);
    plan.total += c.slots * c.G;
  }
  return MPTS_OK;
}

// Workspace of a batch of gradients: descriptors, workgroup map, then one
// region per trajectory laid out like a single checkpointed run.
struct GradBatchLayout {
  std::vector<size_t> region;
  size_t insts = 0, wgmap = 0, total = 0;
  int CM = 4;
  size_t lds_fwd = 0, lds_adj = 0;
};

int grad_batch_layout(mpts_ctx *const *ctxs, int count, const int64_t *nsteps, GradBatchLayout &gl) {
  gl = GradBatchLayout();
  size_t o = 0;
  gl.insts = o;
  o = al(o + (size_t)count * sizeof(Inst));
  gl.wgmap = o;
  o = al(o + (size_t)kMaxWG * 4);
  int maxnd = 0;
  for (int t = 0; t < count; ++t) {
    gl.region.push_back(o);
    o = al(o + layout(ctxs[t], nsteps[t], true, 1).total);
    maxnd = std::max(maxnd, ctxs[t]->nd);
  }
  gl.total = o;
  gl.CM = choose_cm(maxnd);
  if (gl.CM < 0) return MPTS_EUNSUPPORTED;
  for (int t = 0; t < count; ++t) {
    mpts_ctx *c = ctxs[t];
    gl.lds_fwd = std::max(gl.lds_fwd, lds_bytes(c->L, c->N, c->RS, c->WB, gl.CM, false, c->mfma != 0));
    gl.lds_adj = std::max(gl.lds_adj, lds_bytes(c->L, c->N, c->RS, c->WB, gl.CM, true, c->mfma != 0));
  }
  return MPTS_OK;
}

// Cached instantiated graphs of batch launches.  A graph holds the kernel
// instance (CM), its dynamic LDS size, the workgroup count and the clear
// nodes of every trajectory's region, all of which follow from the
// trajectories' (L, N), nsteps and schedule: the key names each trajectory
// by its context's creation number (never reused, unlike an address) and
// its sizes, and mpts_destroy evicts every graph that names the context.
struct GraphKey {
  void *ws = nullptr;
  int device = 0;
  int CM = 0;
  size_t lds = 0;
  std::vector<uint64_t> gens;
  std::vector<int> LN;  // L, N per trajectory
  std::vector<int64_t> nsteps;
  std::vector<int> G;
  std::vector<int> sched;  // first workgroup and successor of each trajectory
  bool operator<(const GraphKey &o) const {
    if (ws != o.ws) return ws < o.ws;
    if (device != o.device) return device < o.device;
    if (CM != o.CM) return CM < o.CM;
    if (lds != o.lds) return lds < o.lds;
    if (gens != o.gens) return gens < o.gens;
    if (LN != o.LN) return LN < o.LN;
    if (nsteps != o.nsteps) return nsteps < o.nsteps;
    if (G != o.G) return G < o.G;
    return sched < o.sched;
  }
};
std::map<GraphKey, hipGraphExec_t> g_graphs;

hipGraphExec_t graph_lookup(const GraphKey &k) {
  auto it = g_graphs.find(k);
  return it == g_graphs.end() ? nullptr : it->second;
}

void graph_store(const GraphKey &k, hipGraphExec_t e) {
  if (g_graphs.size() > 64) {
    for (auto &kv : g_graphs) (void)hipGraphExecDestroy(kv.second);
    g_graphs.clear();
  }
  g_graphs[k] = e;
}

void graph_evict(uint64_t gen) {
  for (auto it = g_graphs.begin(); it != g_graphs.end();) {
    if (std::find(it->first.gens.begin(), it->first.gens.end(), gen) != it->first.gens.end()) {
      (void)hipGraphExecDestroy(it->second);
      it = g_graphs.erase(it);
    } else {
      ++it;
    }
  }
}

}  // namespace

namespace mpts {

int noalloc_scratch(void **ptr);  // mpts_noalloc.hip

int integrate_fits(mpts_ctx *c, int64_t nsteps, size_t limit) {
  const size_t need = layout(c, nsteps, false, kMaxWG, false).total;
  if (need <= limit) return MPTS_OK;
  char msg[160];
  snprintf(msg, sizeof(msg),
           "needs %zu bytes of workspace; the library's scratch array holds %zu (L=%d, N=%d)", need,
           limit, c->L, c->N);
  return set_err(c, MPTS_ENOSPC, msg);
}

}  // namespace mpts

// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Polynomial vector fields of degree at most two (k_poly).

struct mpts_poly {
  int V = 0, L = 0, N = 0, nd = 0, RS = 0, WB = 0, CM = 0, Q = 0, nconst = 0, maxn = 0;
  size_t lds = 0;
  PolyInst proto;           // every field but the pointers
  std::vector<int32_t> cn;  // nconst x (L+2) normalised constants
  std::string err;
};

namespace {

int poly_err(mpts_poly *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  return code;
}

bool rational_is_unit(const Rational &q) {
  Big n = q.num, d = q.den;
  trim(n);
  trim(d);
  return n.size() == 1 && n[0] == 1u && d.size() == 1 && d[0] == 1u;
}

int make_poly(int32_t nvar, const mpts_poly_term *terms, int32_t nterms, int32_t L, int32_t N,
              const char *tau, mpts_poly **out) {
  if (!out) return MPTS_EINVAL;
  *out = nullptr;
  if (nvar < 1 || nterms < 0 || (nterms > 0 && !terms) || L < 1 || L > 1024 || N < 1 ||
      N > 8192 || !tau)
    return MPTS_EINVAL;
  if (nvar > PMAXV) return MPTS_EUNSUPPORTED;
  Rational qt;
  if (!parse_number(tau, qt)) return MPTS_EINVAL;
  mpts_poly *c = new mpts_poly();
  memset(&c->proto, 0, sizeof(c->proto));
  PolyInst &P = c->proto;
  c->V = nvar;
  c->L = L;
  c->N = N;
  c->nd = digits_per_row(L);
  c->RS = row_stride(c->nd);
  c->WB = frame_width(c->nd);
  c->CM = choose_cm(c->nd);
  // the Horner addend prefetch holds rows of at most 1024 words
  if (c->CM < 0 || c->RS > 1024) {
    delete c;
    return MPTS_EUNSUPPORTED;
  }
  std::vector<std::vector<int32_t>> consts;
  std::vector<int32_t> nv;
  for (int v = 0; v < nvar; ++v) P.cc[v] = -1;
  // product pairs first (their operand codes follow the variables)
  std::vector<std::pair<int, int>> pairs;
  for (int t = 0; t < nterms; ++t) {
    const mpts_poly_term &m = terms[t];
    if (m.eq < 0 || m.eq >= nvar || m.u < -1 || m.u >= nvar || m.w < -1 || m.w >= nvar ||
        (m.u < 0 && m.w >= 0) || !m.coef) {
      delete c;
      return MPTS_EINVAL;
    }
    if (m.w >= 0) {
      const std::pair<int, int> q(std::min(m.u, m.w), std::max(m.u, m.w));
      if (std::find(pairs.begin(), pairs.end(), q) == pairs.end()) pairs.push_back(q);
    }
  }
  if ((int)pairs.size() > PMAXQ) {
    delete c;
    return MPTS_EUNSUPPORTED;
  }
  c->Q = (int)pairs.size();
  for (int q = 0; q < c->Q; ++q) {
    P.pu[q] = pairs[q].first;
    P.pw[q] = pairs[q].second;
  }
  for (int t = 0; t < nterms; ++t) {
    const mpts_poly_term &m = terms[t];
    Rational q;
    if (!parse_number(m.coef, q)) {
      delete c;
      return MPTS_EINVAL;
    }
    if (q.num.empty()) continue;  // a zero coefficient adds nothing
    round_rational(q, 0, L, nv);
    const int v = m.eq;
    if (m.u < 0) {
      if (P.cc[v] >= 0) {  // one constant term per equation
        delete c;
        return MPTS_EUNSUPPORTED;
      }
      P.cc[v] = (int)consts.size();
      consts.push_back(nv);
      continue;
    }
    int opnd = m.u;
    if (m.w >= 0) {
      const std::pair<int, int> pq(std::min(m.u, m.w), std::max(m.u, m.w));
      opnd = nvar + (int)(std::find(pairs.begin(), pairs.end(), pq) - pairs.begin());
    }
    // coefficient +-1: a row addend (the constant term of index 0 keeps one slot)
    if (rational_is_unit(q) && P.na[v] < PMAXA - 1) {
      P.asg[v][P.na[v]] = q.neg ? -1 : 1;
      P.ao[v][P.na[v]] = opnd;
      ++P.na[v];
      continue;
    }
    if (P.np[v] >= PMAXP) {
      delete c;
      return MPTS_EUNSUPPORTED;
    }
    P.cp[v][P.np[v]] = (int)consts.size();
    P.op[v][P.np[v]] = opnd;
    ++P.np[v];
    consts.push_back(nv);
  }
  round_rational(qt, 0, L, nv);
  const TauRat tr = tau_rational(qt, nv, L);
  P.ctau = (int)consts.size();
  consts.push_back(nv);
  c->nconst = (int)consts.size();
  c->cn.assign((size_t)c->nconst * (L + 2), 0);
  for (int k = 0; k < c->nconst; ++k)
    std::copy(consts[k].begin(), consts[k].end(), c->cn.begin() + (size_t)k * (L + 2));
  c->maxn = std::max(c->Q * ((N + 16) & ~15), nvar * PMAXP * 16);
  c->lds = poly_lds_bytes(nvar, c->Q, c->RS, c->WB, c->CM, c->maxn);
  if (c->lds > kLdsPerCU) {
    delete c;
    return MPTS_EUNSUPPORTED;
  }
  P.L = L;
  P.N = N;
  P.nd = c->nd;
  P.RS = c->RS;
  P.WB = c->WB;
  P.CM = c->CM;
  P.V = nvar;
  P.Q = c->Q;
  P.tau_n = tr.n;
  P.tau_d = tr.d;
  P.tau_m0 = tr.m0;
  P.tau_m1 = tr.m1;
  P.tau_e = tr.e;
  P.nconst = c->nconst;
  P.maxn = c->maxn;
  *out = c;
  return MPTS_OK;
}

int poly_bf_to_nv(int L, const mpts_bf &b, int32_t *nv) {
  if (b.sign == 0) {
    for (int j = 0; j < L + 2; ++j) nv[j] = 0;
    return MPTS_OK;
  }
  if (!b.limbs || (b.sign != 1 && b.sign != -1) || !(b.limbs[L - 1] & 0x80000000u))
    return MPTS_EINVAL;
  nv[0] = b.sign;
  nv[1] = b.exp;
  for (int j = 0; j < L; ++j) nv[2 + j] = (int32_t)b.limbs[j];
  return MPTS_OK;
}

int poly_nv_to_bf(int L, const int32_t *nv, mpts_bf *b) {
  if (!b->limbs) return MPTS_EINVAL;
  b->sign = nv[0];
  b->exp = nv[0] ? nv[1] : 0;
  for (int j = 0; j < L; ++j) b->limbs[j] = (uint32_t)nv[2 + j];
  return MPTS_OK;
}

// Device bytes of one trajectory's region (rows, sums, constants, state,
// coefficients, error word), 256-byte aligned parts.
struct PolyLayout {
  size_t rows, sums, consts, cnorm, state, coefs, err, total;
};

PolyLayout poly_layout(const mpts_poly *c, bool coefs) {
  PolyLayout l;
  size_t o = 0;
  auto put = [&](size_t bytes) {
    size_t at = o;
    o = al(o + bytes);
    return at;
  };
  l.rows = put((size_t)c->V * (c->N + 1) * c->RS * 4);
  l.sums = put((size_t)std::max(c->Q, 1) * c->RS * 4);
  l.consts = put((size_t)c->nconst * c->RS * 4);
  l.cnorm = put((size_t)c->nconst * (c->L + 2) * 4);
  l.state = put((size_t)c->V * (c->L + 2) * 4);
  l.coefs = put(coefs ? (size_t)c->V * (c->N + 1) * (c->L + 2) * 4 : 0);
  l.err = put(4);
  l.total = o;
  return l;
}

int poly_run(mpts_poly *c, int32_t count, const mpts_bf *x0, int64_t nsteps, mpts_bf *x_out,
             mpts_bf *coefs, void *stream) {
  if (!c || count < 1 || !x0 || !x_out || nsteps < 0 || (coefs && count != 1))
    return poly_err(c, MPTS_EINVAL, "bad argument");
  hipStream_t s = (hipStream_t)stream;
  const int V = c->V, L = c->L;
  const PolyLayout l = poly_layout(c, coefs != nullptr);
  const size_t region = l.total;
  const size_t ibytes = al((size_t)count * sizeof(PolyInst));
  const size_t total = ibytes + (size_t)count * region;
  // host image: descriptors, and each region's constants and state
  std::vector<PolyInst> insts((size_t)count, c->proto);
  std::vector<int32_t> st((size_t)V * (L + 2));
  char *base = nullptr;
  hipError_t e = hipMalloc((void **)&base, total);
  if (e != hipSuccess) return poly_err(c, MPTS_EHIP, std::string("allocate: ") + hipGetErrorString(e));
  auto fail = [&](int code, const std::string &msg) {
    (void)hipStreamSynchronize(s);
    (void)hipFree(base);
    return poly_err(c, code, msg);
  };
  e = launch_clear(base, total, s);
  if (e != hipSuccess) return fail(MPTS_EHIP, "clear");
  for (int t = 0; t < count; ++t) {
    char *rb = base + ibytes + (size_t)t * region;
    PolyInst &P = insts[t];
    P.nsteps = nsteps;
    P.rows = (int32_t *)(rb + l.rows);
    P.sums = (int32_t *)(rb + l.sums);
    P.consts = (int32_t *)(rb + l.consts);
    P.cnorm = (int32_t *)(rb + l.cnorm);
    P.state = (int32_t *)(rb + l.state);
    P.coefs = coefs ? (int32_t *)(rb + l.coefs) : nullptr;
    P.err = (uint32_t *)(rb + l.err);
    for (int v = 0; v < V; ++v)
      if (poly_bf_to_nv(L, x0[(size_t)t * V + v], st.data() + (size_t)v * (L + 2)) != MPTS_OK)
        return fail(MPTS_EINVAL, "bad initial state");
    e = hipMemcpyAsync(rb + l.cnorm, c->cn.data(), c->cn.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(rb + l.state, st.data(), st.size() * 4, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return fail(MPTS_EHIP, "copy inputs");
    // the copies read st: finish them before it is refilled
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(MPTS_EHIP, "synchronize");
  }
  e = hipMemcpyAsync(base, insts.data(), insts.size() * sizeof(PolyInst), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return fail(MPTS_EHIP, "copy descriptors");
  e = launch_poly((const PolyInst *)base, count, c->CM, c->lds, s);
  if (e != hipSuccess) return fail(MPTS_EHIP, std::string("launch: ") + hipGetErrorString(e));
  std::vector<uint32_t> errs((size_t)count);
  std::vector<int32_t> outs((size_t)count * V * (L + 2));
  for (int t = 0; t < count; ++t) {
    char *rb = base + ibytes + (size_t)t * region;
    e = hipMemcpyAsync(&errs[t], rb + l.err, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(outs.data() + (size_t)t * V * (L + 2), rb + l.state,
                         (size_t)V * (L + 2) * 4, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return fail(MPTS_EHIP, "copy results");
  }
  std::vector<int32_t> cf;
  if (coefs) {
    cf.resize((size_t)V * (c->N + 1) * (L + 2));
    e = hipMemcpyAsync(cf.data(), base + ibytes + l.coefs, cf.size() * 4, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return fail(MPTS_EHIP, "copy coefficients");
  }
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(MPTS_EHIP, std::string("synchronize: ") + hipGetErrorString(e));
  (void)hipFree(base);
  for (int t = 0; t < count; ++t) {
    const uint32_t w = errs[t];
    if (w & 8u) return poly_err(c, MPTS_EUNSUPPORTED, "per-term offset table overflow");
    if (w & 3u) return poly_err(c, MPTS_ERANGE, "exact sum outside the device window");
  }
  for (size_t j = 0; j < (size_t)count * V; ++j)
    if (poly_nv_to_bf(L, outs.data() + j * (L + 2), &x_out[j]) != MPTS_OK)
      return poly_err(c, MPTS_EINVAL, "output without limb storage");
  if (coefs)
    for (size_t j = 0; j < (size_t)V * (c->N + 1); ++j)
      if (poly_nv_to_bf(L, cf.data() + j * (L + 2), &coefs[j]) != MPTS_OK)
        return poly_err(c, MPTS_EINVAL, "output without limb storage");
  return MPTS_OK;
}

}  // namespace

extern "C" {

int mpts_create(const char *sigma, const char *R, const char *b, int32_t K_digits, int32_t N,
                const char *tau, mpts_ctx **out) {
  if (K_digits < 1 || K_digits > 9864) return MPTS_EINVAL;
  // L = 2 ceil(ceil(K log2 10) / 64); ceil(K log2 10) is the bit length of 10^K
  Big t = pow10(K_digits);
  long long bits = bitlen(t);
  int L = (int)(2 * ((bits + 63) / 64));
  return make_ctx(sigma, R, b, L, N, tau, out);
}

int mpts_create_limbs(const char *sigma, const char *R, const char *b, int32_t L, int32_t N,
                      const char *tau, mpts_ctx **out) {
  return make_ctx(sigma, R, b, L, N, tau, out);
}

void mpts_destroy(mpts_ctx *ctx) {
  if (!ctx) return;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    graph_evict(ctx->gen);
  }
  delete ctx;
}

int mpts_release_caches(void) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  for (auto &kv : g_graphs) (void)hipGraphExecDestroy(kv.second);
  g_graphs.clear();
  return MPTS_OK;
}

int mpts_limbs(const mpts_ctx *c, int32_t *L, int32_t *p_bits, int32_t *N) {
  if (!c) return MPTS_EINVAL;
  if (L) *L = c->L;
  if (p_bits) *p_bits = 32 * c->L;
  if (N) *N = c->N;
  return MPTS_OK;
}

int mpts_param(const mpts_ctx *c, int32_t which, mpts_bf *out) {
  if (!c || !out || which < 0 || which > 3) return MPTS_EINVAL;
  static const int idx[4] = {C_SIGMA, C_R, C_NB, C_TAU};
  std::vector<int32_t> nv(c->cn.begin() + (size_t)idx[which] * (c->L + 2),
                          c->cn.begin() + (size_t)(idx[which] + 1) * (c->L + 2));
  if (which == 2) nv[0] = -nv[0];
  return nv_to_bf(c, nv.data(), out);
}

int mpts_bf_from_str(const mpts_ctx *c, const char *s, mpts_bf *out) {
  if (!c || !out) return MPTS_EINVAL;
  Rational q;
  if (!parse_number(s, q)) return MPTS_EINVAL;
  std::vector<int32_t> nv;
  round_rational(q, 0, c->L, nv);
  return nv_to_bf(c, nv.data(), out);
}

int mpts_bf_from_double(const mpts_ctx *c, double v, mpts_bf *out) {
  if (!c || !out || !std::isfinite(v)) return MPTS_EINVAL;
  Rational q;
  if (v != 0.0) {
    int ex;
    double m = std::frexp(std::fabs(v), &ex);  // v = m 2^ex, m in [0.5, 1)
    uint64_t mi = (uint64_t)std::ldexp(m, 53);
    q.neg = v < 0;
    q.num = Big{(uint32_t)mi, (uint32_t)(mi >> 32)};
    trim(q.num);
    q.den = Big{1u};
    std::vector<int32_t> nv;
    round_rational(q, ex - 53, c->L, nv);
    return nv_to_bf(c, nv.data(), out);
  }
  std::vector<int32_t> nv((size_t)c->L + 2, 0);
  return nv_to_bf(c, nv.data(), out);
}

int mpts_bf_to_double(const mpts_ctx *c, const mpts_bf *v, double *out) {
  if (!c || !v || !out) return MPTS_EINVAL;
  std::vector<int32_t> nv((size_t)c->L + 2);
  int st = bf_to_nv(c, *v, nv.data());
  if (st) return st;
  *out = nv_to_double(nv.data(), c->L);
  return MPTS_OK;
}

int mpts_set_schedule(mpts_ctx *c, int32_t workgroups) {
  if (!c || workgroups < 0) return MPTS_EINVAL;
  c->wgs = workgroups;
  return MPTS_OK;
}

int mpts_workspace_bytes(const mpts_ctx *c, int64_t nsteps, uint32_t flags, size_t *bytes) {
  if (!c || !bytes || nsteps < 0) return MPTS_EINVAL;
  *bytes = layout(c, nsteps, (flags & MPTS_CHECKPOINTS) != 0, kMaxWG).total;
  return MPTS_OK;
}

int mpts_state_bytes(const mpts_ctx *c, size_t *bytes) {
  if (!c || !bytes) return MPTS_EINVAL;
  *bytes = (size_t)3 * (c->L + 2) * 4;
  return MPTS_OK;
}

int mpts_pack_state(const mpts_ctx *c, const mpts_bf x[3], void *packed) {
  if (!c || !x || !packed) return MPTS_EINVAL;
  int32_t *p = (int32_t *)packed;
  for (int k = 0; k < 3; ++k) {
    int st = bf_to_nv(c, x[k], p + (size_t)k * (c->L + 2));
    if (st) return st;
  }
  return MPTS_OK;
}

int mpts_unpack_state(const mpts_ctx *c, const void *packed, mpts_bf x[3]) {
  if (!c || !x || !packed) return MPTS_EINVAL;
  const int32_t *p = (const int32_t *)packed;
  for (int k = 0; k < 3; ++k) {
    int st = nv_to_bf(c, p + (size_t)k * (c->L + 2), &x[k]);
    if (st) return st;
  }
  return MPTS_OK;
}

int mpts_integrate_dev(mpts_ctx *c, const void *x0_dev, int64_t nsteps, void *xout_dev,
                       void *ckpt_dev, void *ws, size_t ws_bytes, void *stream) {
  if (!c || !x0_dev || !xout_dev || !ws || nsteps < 0) return MPTS_EINVAL;
  return run_single(c, MODE_INTEGRATE, nsteps, x0_dev, xout_dev, ckpt_dev, ws, ws_bytes,
                    (hipStream_t)stream, false, nullptr);
}

int mpts_check(mpts_ctx *c, void *ws, void *stream) {
  if (!c) return MPTS_EINVAL;
  if (!ws) {
    // the calls without a workspace record their status in the library's
    // scratch array of the current device
    int st = mpts::noalloc_scratch(&ws);
    if (st != MPTS_OK) return set_err(c, st, "no scratch array on this device");
  }
  return read_status(c, ws, (hipStream_t)stream);
}

int mpts_integrate(mpts_ctx *c, const mpts_bf x0[3], int64_t nsteps, mpts_bf x_out[3],
                   mpts_bf *checkpoints, void *ws, size_t ws_bytes, void *stream,
                   uint32_t flags) {
  if (!c || !x0 || !x_out || !ws || nsteps < 0) return MPTS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  std::vector<int32_t> packed((size_t)3 * (c->L + 2));
  int st = mpts_pack_state(c, x0, packed.data());
  if (st) return set_err(c, st, "bad initial state");
  if (checkpoints && !(flags & MPTS_CHECKPOINTS))
    return set_err(c, MPTS_EINVAL, "checkpoints need MPTS_CHECKPOINTS");
  Layout l = layout(c, nsteps, (flags & MPTS_CHECKPOINTS) != 0, 1);
  if (ws_bytes < l.total) return set_err(c, MPTS_ENOSPC, "workspace too small");
  void *ck = (flags & MPTS_CHECKPOINTS) ? (char *)ws + l.ckpt : nullptr;
  size_t ckb = (size_t)(nsteps + 1) * 3 * (c->L + 2) * 4;
  hipError_t e;
  st = run_single(c, MODE_INTEGRATE, nsteps, nullptr, nullptr, ck, ws, ws_bytes, s, true,
                  packed.data());
  if (st) return st;
  e = hipMemcpyAsync(packed.data(), (char *)ws + l.state, packed.size() * 4, hipMemcpyDeviceToHost,
                     s);
  if (e != hipSuccess) return hip_err(c, e, "copy result");
  std::vector<int32_t> ckh;
  if (checkpoints) {
    ckh.resize(ckb / 4);
    e = hipMemcpyAsync(ckh.data(), ck, ckb, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_err(c, e, "copy checkpoints");
  }
  st = read_status(c, ws, s);
  if (st) return st;
  st = mpts_unpack_state(c, packed.data(), x_out);
  if (st) return st;
  if (checkpoints)
    for (long long n = 0; n <= nsteps; ++n) {
      st = mpts_unpack_state(c, ckh.data() + (size_t)n * 3 * (c->L + 2), checkpoints + 3 * n);
      if (st) return st;
    }
  return MPTS_OK;
}

int mpts_coefficients(mpts_ctx *c, const mpts_bf x0[3], mpts_bf *alpha, mpts_bf *beta,
                      mpts_bf *gamma, void *ws, size_t ws_bytes, void *stream) {
  if (!c || !x0 || !alpha || !beta || !gamma || !ws) return MPTS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  std::vector<int32_t> packed((size_t)3 * (c->L + 2));
  int st = mpts_pack_state(c, x0, packed.data());
  if (st) return set_err(c, st, "bad initial state");
  st = run_single(c, MODE_COEFFS, 1, nullptr, nullptr, nullptr, ws, ws_bytes, s, true,
                  packed.data());
  if (st) return st;
  Layout l = layout(c, 1, false, 1);
  std::vector<int32_t> co((size_t)3 * (c->N + 1) * (c->L + 2));
  hipError_t e =
      hipMemcpyAsync(co.data(), (char *)ws + l.coefs, co.size() * 4, hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return hip_err(c, e, "copy coefficients");
  st = read_status(c, ws, s);
  if (st) return st;
  mpts_bf *outs[3] = {alpha, beta, gamma};
  for (int a = 0; a < 3; ++a)
    for (int i = 0; i <= c->N; ++i) {
      st = nv_to_bf(c, co.data() + ((size_t)a * (c->N + 1) + i) * (c->L + 2), &outs[a][i]);
      if (st) return st;
    }
  return MPTS_OK;
}

int mpts_batch_workspace_bytes(mpts_ctx *const *ctxs, int32_t count, const int64_t *nsteps,
                               uint32_t flags, size_t *bytes) {
  if (!ctxs || count < 1 || !nsteps || !bytes) return MPTS_EINVAL;
  (void)flags;
  BatchLayout bl;
  int st = batch_layout(ctxs, count, bl);
  if (st) return st;
  *bytes = bl.total;
  return MPTS_OK;
}

int mpts_integrate_batch(mpts_ctx *const *ctxs, int32_t count, const mpts_bf *x0,
                         const int64_t *nsteps, mpts_bf *x_out, void *ws, size_t ws_bytes,
                         void *stream, uint32_t flags) {
  if (!ctxs || count < 1 || !x0 || !nsteps || !x_out || !ws) return MPTS_EINVAL;
  for (int t = 0; t < count; ++t)
    if (!ctxs[t] || nsteps[t] < 0) return MPTS_EINVAL;
  mpts_ctx *c0 = ctxs[0];
  hipStream_t s = (hipStream_t)stream;
  int st = check_device(c0);
  if (st) return st;
  for (int t = 1; t < count; ++t) {
    st = check_device(ctxs[t]);
    if (st) return st;
  }
  BatchLayout bl;
  st = batch_layout(ctxs, count, bl);
  if (st) return set_err(c0, st, "batch layout");
  if (ws_bytes < bl.total) return set_err(c0, MPTS_ENOSPC, "workspace too small");
  char *base = (char *)ws;
  // schedule: workgroups per trajectory
  BatchPlan plan;
  st = plan_batch(ctxs, count, nsteps, bl, (flags & MPTS_AUTOTUNE) != 0, ws, ws_bytes, s, plan);
  if (st) return st;
  const int total = plan.total;
  // per trajectory: its slot's workgroups, first workgroup and successor
  std::vector<int> G((size_t)count, 1), wg0((size_t)count, 0), nxt((size_t)count, 0);
  std::vector<int> wgmap((size_t)total, -1);
  {
    int w = 0;
    for (size_t sl = 0; sl < plan.slot_G.size(); ++sl) {
      const auto &lst = plan.slot_list[sl];
      for (size_t k = 0; k < lst.size(); ++k) {
        G[lst[k]] = plan.slot_G[sl];
        wg0[lst[k]] = w;
        nxt[lst[k]] = k + 1 < lst.size() ? lst[k + 1] + 1 : 0;
      }
      for (int j = 0; j < plan.slot_G[sl]; ++j) wgmap[w + j] = lst.empty() ? -1 : lst[0];
      w += plan.slot_G[sl];
    }
  }
  if (getenv("MPTS_PLAN")) {
    // the schedule: workgroups per trajectory, by (L, N)
    std::map<std::pair<int, int>, std::map<int, int>> by;
    for (int t = 0; t < count; ++t) by[{ctxs[t]->L, ctxs[t]->N}][G[t]]++;
    int per_cu = 0;
    (void)max_coresident(bl.CM, bl.lds, &per_cu, false);
    fprintf(stderr, "mpts plan: %d trajectories, %zu slots, %d workgroups, CM %d, LDS %zu, %d per CU\n",
            count, plan.slot_G.size(), total, bl.CM, bl.lds, per_cu);
    for (auto &kv : by) {
      fprintf(stderr, "  L=%d N=%d:", kv.first.first, kv.first.second);
      for (auto &g : kv.second) fprintf(stderr, " G%d x%d", g.first, g.second);
      fprintf(stderr, "\n");
    }
  }
  // descriptors, workgroup map, packed states
  std::vector<Inst> insts((size_t)count);
  std::vector<int32_t> states(bl.states_words, 0);
  for (int t = 0; t < count; ++t) {
    mpts_ctx *c = ctxs[t];
    st = mpts_pack_state(c, x0 + 3 * t, states.data() + bl.state_off[t]);
    if (st) return set_err(c0, st, "bad initial state");
    char *rb = base + bl.region[t];
    Layout l = layout(c, 0, false, 1);
    Inst &I = insts[t];
    memset(&I, 0, sizeof(I));
    I.L = c->L;
    I.N = c->N;
    I.nd = c->nd;
    I.RS = c->RS;
    I.WB = c->WB;
    I.CM = bl.CM;
    I.G = G[t];
    I.wg0 = wg0[t];
    I.next = nxt[t];
    I.mode = MODE_INTEGRATE;
    I.mfma = c->mfma;
    I.nsteps = nsteps[t];
    I.tau_n = c->tau_n;
    I.tau_d = c->tau_d;
    I.tau_m0 = c->tau_m0;
    I.tau_m1 = c->tau_m1;
    I.tau_e = c->tau_e;
    I.rows = (int32_t *)(rb + l.rows);
    I.consts = (int32_t *)(rb + l.consts);
    I.cnorm = (int32_t *)(rb + l.cnorm);
    I.state = (int32_t *)(base + bl.states) + bl.state_off[t];
    I.gframes = (long long *)(rb + l.gframes);
    I.sync = (uint32_t *)(rb + l.sync);
    hipError_t e = hipMemcpyAsync(rb + l.cnorm, c->cn.data(), c->cn.size() * 4,
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_err(c0, e, "copy constants");
  }
  hipError_t e = hipMemcpyAsync(base + bl.states, states.data(), states.size() * 4,
                                hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_err(c0, e, "copy states");
  e = hipMemcpyAsync(base + bl.insts, insts.data(), insts.size() * sizeof(Inst),
                     hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_err(c0, e, "copy descriptors");
  e = hipMemcpyAsync(base + bl.wgmap, wgmap.data(), wgmap.size() * 4, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_err(c0, e, "copy map");
  // device work: clear the synchronisation words and frames, run
  auto device_work = [&](bool cooperative) -> hipError_t {
    for (int t = 0; t < count; ++t) {
      mpts_ctx *c = ctxs[t];
      Layout l = layout(c, 0, false, 1);
      char *rb = base + bl.region[t];
      hipError_t e2 = launch_clear(rb + l.sync, SY_WORDS * 4, s);
      if (e2 != hipSuccess) return e2;
      if (G[t] > 1) {
        e2 = launch_clear(rb + l.gframes, (size_t)2 * NFR * c->WB * 8, s);
        if (e2 != hipSuccess) return e2;
      }
    }
    return launch_run((const Inst *)(base + bl.insts), (const int *)(base + bl.wgmap), total,
                      bl.CM, bl.lds, s, cooperative);
  };
  if (flags & MPTS_GRAPH) {
    GraphKey key;
    key.ws = ws;
    (void)hipGetDevice(&key.device);
    key.CM = bl.CM;
    key.lds = bl.lds;
    for (int t = 0; t < count; ++t) {
      key.gens.push_back(ctxs[t]->gen);
      key.LN.push_back(ctxs[t]->L);
      key.LN.push_back(ctxs[t]->N);
    }
    key.nsteps.assign(nsteps, nsteps + count);
    key.G = G;
    for (int t = 0; t < count; ++t) {
      key.sched.push_back(wg0[t]);
      key.sched.push_back(nxt[t]);
    }
    std::lock_guard<std::mutex> lk(g_cache_mu);
    hipGraphExec_t exec = graph_lookup(key);
    if (!exec) {
      // capture on a private stream (the caller's may be the legacy default
      // stream, which cannot be captured); the graph is launched on the
      // caller's stream below
      e = set_kernel_lds(bl.CM, bl.lds, false);
      if (e != hipSuccess) return hip_err(c0, e, "kernel attributes");
      hipStream_t cap;
      e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
      if (e != hipSuccess) return hip_err(c0, e, "capture stream");
      hipStream_t user = s;
      s = cap;
      hipGraph_t graph = nullptr;
      e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
      hipError_t we = hipSuccess;
      if (e == hipSuccess) {
        we = device_work(false);
        e = hipStreamEndCapture(cap, &graph);
      }
      s = user;
      (void)hipStreamDestroy(cap);
      if (we != hipSuccess) return hip_err(c0, we, "captured launch");
      if (e != hipSuccess) return hip_err(c0, e, "capture");
      e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) return hip_err(c0, e, "instantiate graph");
      graph_store(key, exec);
    }
    e = hipGraphLaunch(exec, s);
    if (e != hipSuccess) return hip_err(c0, e, "graph launch");
  } else {
    e = device_work(true);
    if (e != hipSuccess) return hip_err(c0, e, "launch");
  }
  e = hipMemcpyAsync(states.data(), base + bl.states, states.size() * 4, hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return hip_err(c0, e, "copy states out");
  std::vector<uint32_t> errs((size_t)count, 0u);
  for (int t = 0; t < count; ++t) {
    Layout l = layout(ctxs[t], 0, false, 1);
    e = hipMemcpyAsync(&errs[t], base + bl.region[t] + l.sync + SY_ERROR * 4, 4,
                       hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_err(c0, e, "read status");
  }
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_err(c0, e, "synchronize");
  for (int t = 0; t < count; ++t) {
    if (errs[t] & 4u) return set_err(c0, MPTS_EHIP, "device synchronisation timed out");
    if (errs[t] & 3u) return set_err(c0, MPTS_ERANGE, "exact sum outside the device window");
  }
  for (int t = 0; t < count; ++t) {
    st = mpts_unpack_state(ctxs[t], states.data() + bl.state_off[t], x_out + 3 * t);
    if (st) return st;
  }
  return MPTS_OK;
}

int mpts_grad(mpts_ctx *c, const mpts_bf x0[3], int64_t nsteps, int32_t loss,
              double grad_out[6], double *loss_out, mpts_bf *grad_bf, mpts_bf x_out[3],
              void *ws, size_t ws_bytes, void *stream) {
  if (!c || !x0 || !grad_out || !ws || nsteps < 0) return MPTS_EINVAL;
  if (loss < MPTS_LOSS_SQNORM || loss > MPTS_LOSS_Z) return set_err(c, MPTS_EINVAL, "unknown loss");
  hipStream_t s = (hipStream_t)stream;
  std::vector<int32_t> packed((size_t)3 * (c->L + 2));
  int st = mpts_pack_state(c, x0, packed.data());
  if (st) return set_err(c, st, "bad initial state");
  Layout l = layout(c, nsteps, true, 1);
  if (ws_bytes < l.total) return set_err(c, MPTS_ENOSPC, "workspace too small");
  char *base = (char *)ws;
  // forward run keeping every step's state
  st = run_single(c, MODE_INTEGRATE, nsteps, nullptr, nullptr, base + l.ckpt, ws, ws_bytes, s, true,
                  packed.data());
  if (st) return st;
  st = read_status(c, ws, s);
  if (st) return st;
  // reverse sweep (the state buffer is not read in this mode)
  st = run_single(c, MODE_ADJOINT, nsteps, nullptr, nullptr, base + l.ckpt, ws, ws_bytes, s, true,
                  packed.data(), base + l.adj, loss);
  if (st) return st;
  const size_t nvw = (size_t)c->L + 2;
  std::vector<int32_t> bars(6 * nvw), fin(3 * nvw);
  const size_t bar_off =
      l.adj + ((size_t)6 * c->N * c->RS + (size_t)3 * (c->N + 1) * c->RS) * 4;
  hipError_t e = hipMemcpyAsync(bars.data(), base + bar_off, bars.size() * 4, hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return hip_err(c, e, "copy gradient");
  e = hipMemcpyAsync(fin.data(), base + l.ckpt + (size_t)nsteps * 3 * nvw * 4, fin.size() * 4,
                     hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return hip_err(c, e, "copy final state");
  st = read_status(c, ws, s);
  if (st) return st;
  for (int j = 0; j < 6; ++j) {
    grad_out[j] = nv_to_double(bars.data() + j * nvw, c->L);
    if (grad_bf) {
      st = nv_to_bf(c, bars.data() + j * nvw, &grad_bf[j]);
      if (st) return st;
    }
  }
  if (loss_out) *loss_out = loss_of_state(fin.data(), c->L, loss);
  if (x_out) return mpts_unpack_state(c, fin.data(), x_out);
  return MPTS_OK;
}

int mpts_grad_batch_workspace_bytes(mpts_ctx *const *ctxs, int32_t count, const int64_t *nsteps,
                                    size_t *bytes) {
  if (!ctxs || count < 1 || !nsteps || !bytes) return MPTS_EINVAL;
  GradBatchLayout gl;
  int st = grad_batch_layout(ctxs, count, nsteps, gl);
  if (st) return st;
  *bytes = gl.total;
  return MPTS_OK;
}

int mpts_grad_batch(mpts_ctx *const *ctxs, int32_t count, const mpts_bf *x0, const int64_t *nsteps,
                    int32_t loss, double *grad_out, double *loss_out, mpts_bf *x_out, void *ws,
                    size_t ws_bytes, void *stream) {
  if (!ctxs || count < 1 || !x0 || !nsteps || !grad_out || !ws) return MPTS_EINVAL;
  for (int t = 0; t < count; ++t)
    if (!ctxs[t] || nsteps[t] < 0) return MPTS_EINVAL;
  mpts_ctx *c0 = ctxs[0];
  if (loss < MPTS_LOSS_SQNORM || loss > MPTS_LOSS_Z) return set_err(c0, MPTS_EINVAL, "unknown loss");
  hipStream_t s = (hipStream_t)stream;
  for (int t = 0; t < count; ++t) {
    int st = check_device(ctxs[t]);
    if (st) return st;
  }
  GradBatchLayout gl;
  int st = grad_batch_layout(ctxs, count, nsteps, gl);
  if (st) return set_err(c0, st, "batch layout");
  if (ws_bytes < gl.total) return set_err(c0, MPTS_ENOSPC, "workspace too small");
  // residency of both kernels at the batch's chunk size and LDS sizes
  int pf = 0, pa = 0;
  if (max_coresident(gl.CM, gl.lds_fwd, &pf, false) != 0 || pf < 1)
    return set_err(c0, MPTS_EUNSUPPORTED, "kernel does not fit one compute unit");
  if (max_coresident(gl.CM, gl.lds_adj, &pa, true) != 0 || pa < 1)
    return set_err(c0, MPTS_EUNSUPPORTED, "adjoint kernel does not fit one compute unit");
  const int cap = std::min(c0->cus * std::min(pf, pa), kMaxWG);
  if (count > cap) return set_err(c0, MPTS_EUNSUPPORTED, "more trajectories than resident workgroups");
  // workgroups per trajectory: each trajectory's own single-run choice,
  // within an equal share of the resident workgroups
  int share = 1;
  while (share * 2 * count <= cap) share *= 2;
  std::vector<int> G((size_t)count);
  int total = 0;
  for (int t = 0; t < count; ++t) {
    G[t] = std::max(1, std::min(ctxs[t]->wgs > 0 ? ctxs[t]->wgs : share, share));
    total += G[t];
  }
  char *base = (char *)ws;
  std::vector<Inst> insts((size_t)count);
  std::vector<int> wgmap((size_t)total);
  int wg = 0;
  hipError_t e;
  // packed initial states (alive until the stream is synchronised below)
  std::vector<std::vector<int32_t>> packs((size_t)count);
  for (int t = 0; t < count; ++t) {
    mpts_ctx *c = ctxs[t];
    char *rb = base + gl.region[t];
    Layout l = layout(c, nsteps[t], true, 1);
    std::vector<int32_t> &packed = packs[t];
    packed.resize((size_t)3 * (c->L + 2));
    st = mpts_pack_state(c, x0 + 3 * t, packed.data());
    if (st) return set_err(c0, st, "bad initial state");
    Inst &I = insts[t];
    memset(&I, 0, sizeof(I));
    I.L = c->L;
    I.N = c->N;
    I.nd = c->nd;
    I.RS = c->RS;
    I.WB = c->WB;
    I.CM = gl.CM;
    I.G = G[t];
    I.wg0 = wg;
    I.mode = MODE_INTEGRATE;
    I.loss = loss;
    I.mfma = c->mfma;
    I.nsteps = nsteps[t];
    I.tau_n = c->tau_n;
    I.tau_d = c->tau_d;
    I.tau_m0 = c->tau_m0;
    I.tau_m1 = c->tau_m1;
    I.tau_e = c->tau_e;
    I.rows = (int32_t *)(rb + l.rows);
    I.consts = (int32_t *)(rb + l.consts);
    I.cnorm = (int32_t *)(rb + l.cnorm);
    I.state = (int32_t *)(rb + l.state);
    I.ckpt = (int32_t *)(rb + l.ckpt);
    I.gframes = (long long *)(rb + l.gframes);
    I.sync = (uint32_t *)(rb + l.sync);
    I.adj = (int32_t *)(rb + l.adj);
    for (int j = 0; j < G[t]; ++j) wgmap[wg + j] = t;
    wg += G[t];
    e = hipMemcpyAsync(rb + l.cnorm, c->cn.data(), c->cn.size() * 4, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_err(c0, e, "copy constants");
    e = hipMemcpyAsync(rb + l.state, packed.data(), packed.size() * 4, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_err(c0, e, "copy state");
  }
  e = hipMemcpyAsync(base + gl.wgmap, wgmap.data(), wgmap.size() * 4, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_err(c0, e, "copy map");
  auto clear_regions = [&]() -> hipError_t {
    for (int t = 0; t < count; ++t) {
      Layout l = layout(ctxs[t], nsteps[t], true, 1);
      char *rb = base + gl.region[t];
      hipError_t e2 = launch_clear(rb + l.sync, SY_WORDS * 4, s);
      if (e2 != hipSuccess) return e2;
      e2 = launch_clear(rb + l.gframes, (size_t)2 * NFR * ctxs[t]->WB * 8, s);
      if (e2 != hipSuccess) return e2;
    }
    return hipSuccess;
  };
  // 1. forward runs with per-step checkpoints
  e = hipMemcpyAsync(base + gl.insts, insts.data(), insts.size() * sizeof(Inst),
                     hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = clear_regions();
  if (e == hipSuccess)
    e = launch_run((const Inst *)(base + gl.insts), (const int *)(base + gl.wgmap), total, gl.CM,
                   gl.lds_fwd, s, true);
  if (e != hipSuccess) return hip_err(c0, e, "forward launch");
  e = hipStreamSynchronize(s);  // the descriptors are rewritten below
  if (e != hipSuccess) return hip_err(c0, e, "synchronize");
  // 2. reverse sweeps
  for (auto &I : insts) I.mode = MODE_ADJOINT;
  e = hipMemcpyAsync(base + gl.insts, insts.data(), insts.size() * sizeof(Inst),
                     hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = clear_regions();
  if (e == hipSuccess)
    e = launch_adj((const Inst *)(base + gl.insts), (const int *)(base + gl.wgmap), total, gl.CM,
                   gl.lds_adj, s);
  if (e != hipSuccess) return hip_err(c0, e, "adjoint launch");
  // 3. results: six adjoints, the final state and the status of each
  std::vector<std::vector<int32_t>> bars((size_t)count), fins((size_t)count);
  std::vector<uint32_t> errs((size_t)count, 0u);
  for (int t = 0; t < count; ++t) {
    mpts_ctx *c = ctxs[t];
    Layout l = layout(c, nsteps[t], true, 1);
    char *rb = base + gl.region[t];
    const size_t nvw = (size_t)c->L + 2;
    bars[t].resize(6 * nvw);
    fins[t].resize(3 * nvw);
    const size_t bar_off =
        l.adj + ((size_t)6 * c->N * c->RS + (size_t)3 * (c->N + 1) * c->RS) * 4;
    e = hipMemcpyAsync(bars[t].data(), rb + bar_off, bars[t].size() * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(fins[t].data(), rb + l.ckpt + (size_t)nsteps[t] * 3 * nvw * 4,
                         fins[t].size() * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(&errs[t], rb + l.sync + SY_ERROR * 4, 4, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_err(c0, e, "copy results");
  }
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_err(c0, e, "synchronize");
  for (int t = 0; t < count; ++t) {
    if (errs[t] & 4u) return set_err(c0, MPTS_EHIP, "device synchronisation timed out");
    if (errs[t] & 8u) return set_err(c0, MPTS_EUNSUPPORTED, "per-term offset table overflow");
    if (errs[t] & 3u) return set_err(c0, MPTS_ERANGE, "exact sum outside the device window");
  }
  for (int t = 0; t < count; ++t) {
    mpts_ctx *c = ctxs[t];
    const size_t nvw = (size_t)c->L + 2;
    for (int j = 0; j < 6; ++j) grad_out[6 * t + j] = nv_to_double(bars[t].data() + j * nvw, c->L);
    if (loss_out) loss_out[t] = loss_of_state(fins[t].data(), c->L, loss);
    if (x_out) {
      st = mpts_unpack_state(c, fins[t].data(), x_out + 3 * t);
      if (st) return st;
    }
  }
  return MPTS_OK;
}

const char *mpts_strerror(int status) {
  switch (status) {
    case MPTS_OK: return "ok";
    case MPTS_EINVAL: return "invalid argument";
    case MPTS_ENOSPC: return "workspace too small";
    case MPTS_EHIP: return "HIP runtime error";
    case MPTS_ERANGE: return "exact sum outside the device window or exponent overflow";
    case MPTS_EARCH: return "device is not gfx950";
    case MPTS_EUNSUPPORTED: return "unsupported size or call";
    default: return "unknown status";
  }
}

const char *mpts_last_error(const mpts_ctx *c) { return c ? c->err.c_str() : ""; }

int mpts_poly_create(int32_t nvar, const mpts_poly_term *terms, int32_t nterms, int32_t L,
                     int32_t N, const char *tau, mpts_poly **out) {
  return make_poly(nvar, terms, nterms, L, N, tau, out);
}

void mpts_poly_destroy(mpts_poly *ctx) { delete ctx; }

int mpts_poly_bf_from_str(const mpts_poly *c, const char *s, mpts_bf *out) {
  if (!c || !out || !s) return MPTS_EINVAL;
  Rational q;
  if (!parse_number(s, q)) return MPTS_EINVAL;
  std::vector<int32_t> nv;
  round_rational(q, 0, c->L, nv);
  return poly_nv_to_bf(c->L, nv.data(), out);
}

int mpts_poly_integrate(mpts_poly *ctx, int32_t count, const mpts_bf *x0, int64_t nsteps,
                        mpts_bf *x_out, void *stream) {
  return poly_run(ctx, count, x0, nsteps, x_out, nullptr, stream);
}

int mpts_poly_coefficients(mpts_poly *ctx, const mpts_bf *x0, mpts_bf *coefs, void *stream) {
  if (!ctx || !coefs) return MPTS_EINVAL;
  std::vector<uint32_t> store((size_t)ctx->V * ctx->L);
  std::vector<mpts_bf> out((size_t)ctx->V);
  for (int v = 0; v < ctx->V; ++v) out[v].limbs = store.data() + (size_t)v * ctx->L;
  return poly_run(ctx, 1, x0, 1, out.data(), coefs, stream);
}

const char *mpts_poly_last_error(const mpts_poly *c) { return c ? c->err.c_str() : ""; }

}  // extern "C"
