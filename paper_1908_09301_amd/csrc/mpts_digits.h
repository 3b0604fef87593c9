// Single-wavefront exact arithmetic on digit vectors held in registers, for
// the serial path of each coefficient index and of each Horner step.
//
// A magnitude D is a vector of radix-2^28 digits, lane l holding digits
// [l C, l C + C) in registers; its value is D * 2^(28 base).  C is a
// compile-time constant of each instantiation (a power of two); callers pick
// the smallest one that holds the operands (with_chunks), so that every
// loop below is straight-line code without per-digit predicates.  Results
// are produced directly as rows (the form every product reads: header e, s
// and nd signed digits, zero padding), so no conversion to 32-bit limbs sits
// on the serial path.  A p-bit value M 2^E (M of exactly p = 32 L bits) has
// the row e = floor(E / 28), digits of M 2^(E - 28 e).
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>
#include "mpts_common.h"
#include "mpts_wave.h"

namespace mpts {

template <int C>
using chunk_t = std::integral_constant<int, C>;

// Calls f(chunk_t<Ct>) with Ct the smallest of 2, 4, 8, 12, 16, 24, 32 that
// is >= c and at most CMAX (c <= CMAX is the caller's contract).
template <int CMAX, typename F>
__device__ __forceinline__ void with_chunks(int c, F &&f) {
  if (c <= 2) {
    f(chunk_t<2>());
    return;
  }
  if constexpr (CMAX >= 4) {
    if (c <= 4) {
      f(chunk_t<4>());
      return;
    }
  }
  if constexpr (CMAX >= 8) {
    if (c <= 8) {
      f(chunk_t<8>());
      return;
    }
  }
  if constexpr (CMAX >= 16) {
    if (c <= 12) {
      f(chunk_t<12>());
      return;
    }
    if (c <= 16) {
      f(chunk_t<16>());
      return;
    }
  }
  if constexpr (CMAX >= 32) {
    if (c <= 24) {
      f(chunk_t<24>());
      return;
    }
    f(chunk_t<32>());
  }
}

// + x (0 <= x < 2^62) at the bottom of the lane's chunk; returns the carry out.
template <int C>
__device__ __forceinline__ long long dchunk_add(int (&d)[C], long long x) {
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const long long t = (long long)d[j] + x;
    d[j] = (int)(t & DMASK);
    x = t >> DBITS;
  }
  return x;
}

// - x (0 <= x < 2^62) at the bottom of the lane's chunk; returns the borrow out.
template <int C>
__device__ __forceinline__ long long dchunk_sub(int (&d)[C], long long x) {
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const long long t = (long long)d[j] - x;
    d[j] = (int)(t & DMASK);
    x = -(t >> DBITS);
  }
  return x;
}

template <int C>
__device__ __forceinline__ bool dchunk_all(const int (&d)[C], int val) {
  bool all = true;
#pragma unroll
  for (int j = 0; j < C; ++j) all &= d[j] == val;
  return all;
}

// +1 into every lane whose lower neighbours generate a carry (g) through
// lanes that propagate it; returns the carry out of lane 63.
template <int C>
__device__ __forceinline__ bool dwave_carry(int (&d)[C], bool g) {
  bool top;
  const bool cin = lookahead(g, dchunk_all<C>(d, (int)DMASK), &top);
  if (cin) {
    int x = 1;
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int t = d[j] + x;
      d[j] = t & (int)DMASK;
      x = t >> DBITS;
    }
  }
  return top;
}

template <int C>
__device__ __forceinline__ bool dwave_borrow(int (&d)[C], bool b) {
  bool top;
  const bool bin = lookahead(b, dchunk_all<C>(d, 0), &top);
  if (bin) {
    int x = 1;
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int t = d[j] - x;
      d[j] = t & (int)DMASK;
      x = (t >> DBITS) & 1;
    }
  }
  return top;
}

// Signed column sums v (|v| < 2^62, lane l: columns [l C, l C + C)) ->
// sign and magnitude digits d.  Returns -1, 0 or +1; *ovf is set when the
// magnitude needs more than 64 C digits.
template <int C>
__device__ __forceinline__ int resolve_c(const long long (&v)[C], int (&d)[C], bool *ovf) {
  const int lane = lane_id();
  long long carry = 0;
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const long long t = v[j] + carry;
    d[j] = (int)(t & DMASK);
    carry = t >> DBITS;
  }
  const long long top = __shfl(carry, 63, 64);
  const long long cin = shfl_up1(carry);
  const long long g = dchunk_add<C>(d, cin > 0 ? cin : 0);
  const bool t1 = dwave_carry<C>(d, g != 0);
  const long long b = dchunk_sub<C>(d, cin < 0 ? -cin : 0);
  const bool t2 = dwave_borrow<C>(d, b != 0);
  const long long T = top + (t1 ? 1 : 0) - (t2 ? 1 : 0);
  int sign = 1;
  if (T == -1) {
#pragma unroll
    for (int j = 0; j < C; ++j) d[j] = (int)DMASK - d[j];
    bool g1 = false;
    if (lane == 0) g1 = dchunk_add<C>(d, 1) != 0;
    (void)dwave_carry<C>(d, g1);
    sign = -1;
  } else if (T != 0) {
    *ovf = true;
  }
  if (__ballot(!dchunk_all<C>(d, 0)) == 0ull) sign = 0;
  return sign;
}

// Leading bit index of the magnitude (-1 when zero); uniform.
template <int C>
__device__ __forceinline__ int top_bit_c(const int (&d)[C]) {
  int hi = -1, dsel = 0;
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const bool nz = d[j] != 0;
    hi = nz ? j : hi;
    dsel = nz ? d[j] : dsel;
  }
  const unsigned long long mask = __ballot(hi >= 0);
  if (mask == 0ull) return -1;
  const int tl = 63 - __clzll(mask);
  const int hj = __builtin_amdgcn_readlane(hi, tl);
  const uint32_t dt = (uint32_t)__builtin_amdgcn_readlane(dsel, tl);
  return (tl * C + hj) * DBITS + (31 - __clz(dt));
}

// Digit k of D (uniform k, 0 <= k < 64 C), read on every lane.
template <int C>
__device__ __forceinline__ int digit_at(const int (&d)[C], int k) {
  const int kl = k / C, kj = k - kl * C;
  int v = 0;
#pragma unroll
  for (int j = 0; j < C; ++j) v = j == kj ? d[j] : v;
  return __builtin_amdgcn_readlane(v, kl);
}

// Whether bits [a, b) of D (0 <= a < b, uniform) are all zeros or all ones
// (uniform).
template <int C>
__device__ __forceinline__ bool bits_uniform(const int (&d)[C], int a, int b) {
  const int k0 = lane_id() * C;
  bool any0 = false, any1 = false;
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const int lo = (k0 + j) * DBITS;  // bit index of the digit's bit 0
    const int s = min(max(a - lo, 0), DBITS), e = min(max(b - lo, 0), DBITS);
    const uint32_t mask = e > s ? ((1u << (e - s)) - 1u) << s : 0u;
    const uint32_t x = (uint32_t)d[j];
    any1 |= (x & mask) != 0u;
    any0 |= (~x & mask) != 0u;
  }
  return __ballot(any0) == 0ull || __ballot(any1) == 0ull;
}

// Round sign * D * 2^(28 base) to p = 32 L bits (nearest, ties to even;
// sticky_in: a nonzero value below D) and write it as a row into the LDS
// row `row` (RS words).  D must have a zero top digit (room for the carry of
// rounding up).  Returns false on exponent overflow.
//
// The round bit and the last kept bit sit in two digits whose indices are
// uniform, so they are read once (readlane) instead of tested in every
// digit; the kept part is at least 32 bits long, so rounding up changes the
// top bit only through a carry out of the cut digit (rare, general path).
template <int C>
__device__ __forceinline__ bool round_to_row(int (&d)[C], int sign, long long base, bool sticky_in,
                                             int L, int nd, int RS, int32_t *row_) {
  const int lane = lane_id();
  l_i32 *row = (l_i32 *)row_;
  for (int w = lane; w < RS; w += 64) row[w] = 0;
  int B = sign != 0 ? top_bit_c<C>(d) : -1;
  if (B < 0) {
    __builtin_amdgcn_wave_barrier();
    return true;
  }
  const int p = 32 * L;
  const int shc = B + 1 - p;  // first kept bit of D
  const int k0 = lane * C;
  if (shc > 0) {
    const int rb = shc - 1;
    const int kr = rb / DBITS, rr = rb - kr * DBITS;
    const int kc = shc / DBITS, rc = shc - kc * DBITS;
    const int xr = digit_at<C>(d, kr), xc = digit_at<C>(d, kc);
    // sticky: the bits of digit kr below the round bit and every digit below kr
    int below = 0;
#pragma unroll
    for (int j = 0; j < C; ++j) below |= k0 + j < kr ? d[j] : 0;
    const bool sticky = sticky_in || (xr & ((1 << rr) - 1)) != 0 || __ballot(below != 0) != 0ull;
    const bool up = ((xr >> rr) & 1) && (sticky || ((xc >> rc) & 1));
    int xcut = xc & ~((1 << rc) - 1);
    if (up) xcut += 1 << rc;
    const bool carry = (xcut >> DBITS) != 0;  // uniform
    // digits below kc cleared, digit kc replaced
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int k = k0 + j;
      d[j] = k < kc ? 0 : (k == kc ? (xcut & (int)DMASK) : d[j]);
    }
    if (carry) {
      // + 1 at digit kc + 1, carried through the digits and across lanes
      int x = 0;
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const int t = d[j] + x + (k0 + j == kc + 1 ? 1 : 0);
        d[j] = t & (int)DMASK;
        x = t >> DBITS;
      }
      (void)dwave_carry<C>(d, x != 0);
      B = top_bit_c<C>(d);  // B + 1 when the carry reached the top
    }
  }
  const int Erel = B + 1 - p;  // exponent of the mantissa's last bit, relative to D
  const int erel = Erel >= 0 ? Erel / DBITS : -((-Erel + DBITS - 1) / DBITS);
  // row digit (k - erel) = sign * D[k]; every nonzero digit of D lies in the
  // row, so positions outside it (clamped into the zero padding) get zeros
  l_i32 *rd = row + HDR + RPAD;
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const int r = k0 + j - erel;
    const int rcl = min(max(r, -1), nd);
    const int val = sign < 0 ? -d[j] : d[j];
    rd[rcl] = r == rcl ? val : 0;
  }
  if (lane == 0) {
    row[0] = (int32_t)(base + erel);
    row[1] = sign;
  }
  __builtin_amdgcn_wave_barrier();
  const long long E = base * DBITS + Erel;
  return E > -(1LL << 30) && E < (1LL << 30);
}

// (r 2^28 + x) / d and its remainder for 0 <= r < d < 2^13, 0 <= x < 2^28,
// in doubles (all exact).
__device__ __forceinline__ double dstep(double r, double x, double dd, double inv, double *q) {
  const double n = fma(r, 268435456.0, x);  // < 2^41
  double qq = floor(n * inv);
  double m = fma(-qq, dd, n);
  const bool lo = m < 0.0, hi = m >= dd;
  qq = lo ? qq - 1.0 : (hi ? qq + 1.0 : qq);
  m = lo ? m + dd : (hi ? m - dd : m);
  *q = qq;
  return m;
}

// (a b + c) mod d for 0 <= a, b, c < d < 2^13, in doubles.  a b + c < 2^27,
// so the quotient estimate is short by at most one.
__device__ __forceinline__ double dmuladd(double a, double b, double c, double dd, double inv) {
  const double n = fma(a, b, c);
  const double q = floor(n * inv);
  const double m = fma(-q, dd, n);
  return m >= dd ? m - dd : m;
}

// Divide the magnitude D (lane l: digits [l C, l C + C)) by dv in place,
// 1 <= dv < 2^13; returns whether the remainder is nonzero (uniform).  Each
// lane's chunk is cut into blocks of S digits whose remainders are formed
// side by side and folded; a scan over the lanes (from the top lane down,
// x -> x 2^(28 C s) + r mod dv, with the uniform power 2^(28 C s) mod dv)
// gives each lane its incoming remainder; each block's incoming remainder
// then follows from it directly, and the blocks' quotient digits are again
// formed side by side.
template <int C>
__device__ __forceinline__ bool div_small_c(int (&x)[C], int dv) {
  constexpr int S = C >= 4 ? 4 : C;  // digits per block (C is 2, 4, 8, 12, 16, 24 or 32)
  constexpr int NB = C / S;
  const int lane = lane_id();
  const double dd = (double)dv, inv = 1.0 / dd;
  double xd[C];
#pragma unroll
  for (int j = 0; j < C; ++j) xd[j] = (double)x[j];
  // powers of 2^28 mod d: PS = 2^(28 S), PK[k] = PS^k, P = PS^NB
  double qd;
  const double b28 = dstep(dv > 1 ? 1.0 : 0.0, 0.0, dd, inv, &qd);
  double PS = b28;
#pragma unroll
  for (int t = 1; t < S; t <<= 1) PS = dmuladd(PS, PS, 0.0, dd, inv);
  double PK[NB + 1];
  PK[0] = dv > 1 ? 1.0 : 0.0;
  PK[1] = PS;
#pragma unroll
  for (int k = 2; k <= NB; ++k) PK[k] = dmuladd(PK[k / 2], PK[k - k / 2], 0.0, dd, inv);
  // block remainders, side by side
  double rb[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    double r = 0.0;
#pragma unroll
    for (int j = S - 1; j >= 0; --j) r = dstep(r, xd[b * S + j], dd, inv, &qd);
    rb[b] = r;
  }
  // fold from the top block: above[b] = the blocks above b, modulo d
  double above[NB];
  double r = 0.0;
#pragma unroll
  for (int b = NB - 1; b >= 0; --b) {
    above[b] = r;
    r = dmuladd(r, PS, rb[b], dd, inv);
  }
  // suffix scan over the lanes: lane l ends with lanes [l, 63], modulo d
  double Ps = PK[NB];
#pragma unroll
  for (int s = 1; s < 64; s <<= 1) {
    const double r2 = (double)__shfl_down((int)r, s, 64);
    if (lane + s < 64) r = dmuladd(Ps, r2, r, dd, inv);
    Ps = dmuladd(Ps, Ps, 0.0, dd, inv);
  }
  const int rup = __shfl_down((int)r, 1, 64);
  const double rin = lane == 63 ? 0.0 : (double)rup;
  // quotient digits, block by block side by side
  double rlow = 0.0;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    double rr = dmuladd(rin, PK[NB - 1 - b], above[b], dd, inv);
#pragma unroll
    for (int j = S - 1; j >= 0; --j) {
      rr = dstep(rr, xd[b * S + j], dd, inv, &qd);
      x[b * S + j] = (int)qd;
    }
    if (b == 0) rlow = rr;
  }
  return __builtin_amdgcn_readlane((int)rlow, 0) != 0;
}

// The quotient part of div_to_row: the dividend is D[lowcut..t] (in LDS
// scratch sc) shifted up by m zero digits, C2 digits per lane.
template <int C2>
__device__ __forceinline__ bool div_window(const l_i32 *sc, int t, int lowcut, int m, bool low_nz,
                                           int sign, long long base, int dv, int L, int nd, int RS,
                                           int32_t *row) {
  const int lane = lane_id();
  int x[C2];
#pragma unroll
  for (int j = 0; j < C2; ++j) {
    const int k = lane * C2 + j - m + lowcut;
    x[j] = (k >= lowcut && k <= t) ? sc[k] : 0;
  }
  const bool sticky = div_small_c<C2>(x, dv) || low_nz;
  return round_to_row<C2>(x, sign, base + lowcut - m, sticky, L, nd, RS, row);
}

// Round (sign * D * 2^(28 base)) / dv to p bits into the LDS row `row`,
// 1 <= dv < 2^13.  Only the top nd + 3 digits of D enter the long division
// (the quotient then has at least p + 2 bits; lower digits and the final
// remainder only decide the sticky bit); a short D is extended with zero
// digits at the bottom until the quotient has p + 2 bits.  The division
// runs in parallel: each lane's chunk remainder, a scan of the chunk maps
// x -> (x 2^(28 C2) + r_l) mod d from the top lane down, then each lane's
// quotient digits.  scratch: 64 CMAX digits of LDS.
template <int C, int CMAX>
__device__ __forceinline__ bool div_to_row(const int (&d)[C], int sign, long long base, int dv,
                                           int L, int nd, int RS, int32_t *scratch, int32_t *row) {
  const int lane = lane_id();
  l_i32 *sc = (l_i32 *)scratch;
  const int B = sign != 0 ? top_bit_c<C>(d) : -1;
  if (B < 0) {
    int z[2] = {0, 0};
    return round_to_row<2>(z, 0, 0, false, L, nd, RS, row);
  }
  const int t = B / DBITS;  // top digit
  const int keep = nd + 3;
  const int lowcut = t + 1 - keep > 0 ? t + 1 - keep : 0;
  bool lz = false;
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const int k = lane * C + j;
    lz |= k < lowcut && d[j] != 0;
    sc[k] = d[j];
  }
  const bool low_nz = __ballot(lz) != 0ull;
  const int bits = B + 1 - lowcut * DBITS;  // bits of the window
  const int need = 32 * L + 16;
  const int m = bits < need ? (need - bits + DBITS - 1) / DBITS : 0;
  const int n2 = t + 1 - lowcut + m;  // dividend digits
  const int c2 = (n2 + 1 + 63) >> 6;  // one spare digit on top for rounding up
  __builtin_amdgcn_wave_barrier();
  bool ok = true;
  with_chunks<CMAX>(c2, [&](auto ct) {
    constexpr int C2 = decltype(ct)::value;
    ok = div_window<C2>(sc, t, lowcut, m, low_nz, sign, base, dv, L, nd, RS, row);
  });
  return ok;
}

}  // namespace mpts
