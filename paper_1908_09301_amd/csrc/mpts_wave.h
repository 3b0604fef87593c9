// Single-wavefront (64 lanes) exact big-integer primitives on radix-2^28
// digit vectors, used on the serial path of each coefficient: resolving
// signed column sums into a sign and magnitude, rounding to p bits
// (round-to-nearest, ties-to-even), and exact division by a small integer
// followed by one rounding.
//
// A vector of n digits is split into 64 consecutive chunks of C = n/64 digits
// (lane l owns digits [l*C, l*C + C)), kept in registers (C <= CM, a compile
// time bound).  Carries between chunks are resolved with wave ballots: a
// chunk "generates" a carry or "propagates" one (all digits at the maximum),
// and the carry into every lane is read off one 64-bit addition of the two
// ballot masks, as in a carry-lookahead adder.
#pragma once
#include <hip/hip_runtime.h>
#include "mpts_common.h"

namespace mpts {

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ long long shfl_up1(long long v) {
  long long u = __shfl_up(v, 1, 64);
  return lane_id() == 0 ? 0 : u;
}

// Carry into each lane from per-lane generate / propagate bits; the carry out
// of lane 63 is returned in *out.
__device__ __forceinline__ bool lookahead(bool g, bool p, bool *out) {
  unsigned long long G = __ballot(g);
  unsigned long long P = __ballot(p && !g);
  unsigned long long a = G | P;
  unsigned long long s = a + G;
  unsigned long long cin = s ^ a ^ G;
  *out = s < a;
  return (cin >> lane_id()) & 1ull;
}

template <int CM>
__device__ __forceinline__ long long chunk_add(long long (&v)[CM], int C, long long x) {
  // v += x at the chunk bottom (x >= 0); returns the carry out of the chunk
#pragma unroll
  for (int j = 0; j < CM; ++j) {
    if (j < C) {
      long long t = v[j] + x;
      v[j] = t & DMASK;
      x = t >> DBITS;
    }
  }
  return x;
}

template <int CM>
__device__ __forceinline__ long long chunk_sub(long long (&v)[CM], int C, long long x) {
  // v -= x at the chunk bottom (x >= 0); returns the borrow out of the chunk
#pragma unroll
  for (int j = 0; j < CM; ++j) {
    if (j < C) {
      long long t = v[j] - x;
      v[j] = t & DMASK;
      x = -(t >> DBITS);
    }
  }
  return x;
}

template <int CM>
__device__ __forceinline__ bool chunk_all(const long long (&v)[CM], int C, long long val) {
  bool all = true;
#pragma unroll
  for (int j = 0; j < CM; ++j) {
    if (j < C) {
      all &= (v[j] == val);
    }
  }
  return all;
}

// Add the lane's carry-out bit g into the next lane, propagating across lanes.
template <int CM>
__device__ __forceinline__ bool wave_carry(long long (&v)[CM], int C, bool g) {
  bool top;
  bool cin = lookahead(g, chunk_all<CM>(v, C, DMASK), &top);
  if (cin) chunk_add<CM>(v, C, 1);
  return top;
}

template <int CM>
__device__ __forceinline__ bool wave_borrow(long long (&v)[CM], int C, bool b) {
  bool top;
  bool bin = lookahead(b, chunk_all<CM>(v, C, 0), &top);
  if (bin) chunk_sub<CM>(v, C, 1);
  return top;
}

// Resolve signed 64-bit column sums held in registers, lane l owning
// columns [l*C, l*C + C) (value sum v 2^(28 c), |v| < 2^62, C >= 2), into a
// sign and a magnitude of 64*C digits in [0, 2^28) written to dig[0..64*C).
// Returns -1, 0 or +1; *ovf is set when the magnitude does not fit.
template <int CM>
__device__ __forceinline__ int wave_resolve_regs(long long (&v)[CM], int C, int32_t *dig_, bool *ovf) {
  const int lane = lane_id();
  l_i32 *dig = (l_i32 *)dig_;
  const int lo = lane * C;
  // local carry propagation: digits in [0, 2^28) and a signed chunk carry
  long long carry = 0;
#pragma unroll
  for (int j = 0; j < CM; ++j) {
    if (j < C) {
      long long t = v[j] + carry;
      v[j] = t & DMASK;
      carry = t >> DBITS;
    }
  }
  long long top = __shfl(carry, 63, 64);
  long long cin = shfl_up1(carry);
  // add the positive part of the incoming carry, then subtract the negative part
  long long g = chunk_add<CM>(v, C, cin > 0 ? cin : 0);
  bool t1 = wave_carry<CM>(v, C, g != 0);
  long long b = chunk_sub<CM>(v, C, cin < 0 ? -cin : 0);
  bool t2 = wave_borrow<CM>(v, C, b != 0);
  long long T = top + (t1 ? 1 : 0) - (t2 ? 1 : 0);
  int sign;
  if (T == 0) {
    sign = 1;
  } else if (T == -1) {
    // negative: magnitude = 2^(28*64C) - v
#pragma unroll
    for (int j = 0; j < CM; ++j) {
      if (j < C) {
        v[j] = DMASK - v[j];
      }
    }
    long long c0 = (lane == 0) ? chunk_add<CM>(v, C, 1) : 0;
    (void)wave_carry<CM>(v, C, c0 != 0);
    sign = -1;
  } else {
    *ovf = true;
    sign = 1;
  }
  bool nz = !chunk_all<CM>(v, C, 0);
  if (__ballot(nz) == 0ull) sign = 0;
#pragma unroll
  for (int j = 0; j < CM; ++j) {
    if (j < C) {
      dig[lo + j] = (int32_t)v[j];
    }
  }
  __builtin_amdgcn_wave_barrier();
  return sign;
}

// floor(b / 28) and b mod 28 for any int b.
__device__ __forceinline__ int fdiv28(int b, int *r) {
  const int k = b >= 0 ? b / DBITS : -((-b + DBITS - 1) / DBITS);
  *r = b - k * DBITS;
  return k;
}

// 32 bits of a digit vector starting at bit position b (bits outside
// [0, 28 n) read as zero).
__device__ __forceinline__ uint32_t dig_bits32(const l_i32 *dig, int n, int b) {
  int r;
  const int k = fdiv28(b, &r);  // r in 0..27
  // the 32-bit window spans at most three digits
  unsigned long long d0 = (k >= 0 && k < n) ? (uint32_t)dig[k] : 0u;
  unsigned long long d1 = (k + 1 >= 0 && k + 1 < n) ? (uint32_t)dig[k + 1] : 0u;
  unsigned long long d2 = (k + 2 >= 0 && k + 2 < n) ? (uint32_t)dig[k + 2] : 0u;
  unsigned long long w = (d0 >> r) | (d1 << (DBITS - r)) | (d2 << (2 * DBITS - r));
  return (uint32_t)w;
}

// Highest nonzero digit index of dig[0..64C) (-1 if all zero); every lane
// gets the result.
__device__ __forceinline__ int wave_top_digit(const l_i32 *dig, int C) {
  const int lane = lane_id();
  int hi = -1;
  for (int j = 0; j < C; ++j)
    if (dig[lane * C + j] != 0) hi = lane * C + j;
  unsigned long long m = __ballot(hi >= 0);
  if (m == 0ull) return -1;
  int src = 63 - __clzll(m);
  return __shfl(hi, src, 64);
}

// Round sign * (dig * 2^(28*dexp)) to p = 32 L bits (RNE) into the
// normalised form out = [sign, E, M[0..L)].  sticky_in marks a nonzero value
// below the digit vector (a division remainder).  Returns false on exponent
// overflow.
__device__ bool wave_round(const int32_t *dig_, int C, int sign, long long dexp, bool sticky_in,
                           int L, int32_t *out_) {
  const int lane = lane_id();
  const int n = 64 * C;
  const l_i32 *dig = (const l_i32 *)dig_;
  l_i32 *out = (l_i32 *)out_;
  int t = wave_top_digit(dig, C);
  if (t < 0 || sign == 0) {
    for (int j = lane; j < L + 2; j += 64) out[j] = 0;
    __builtin_amdgcn_wave_barrier();
    return true;
  }
  uint32_t dt = (uint32_t)dig[t];
  const int B = t * DBITS + (31 - __clz(dt));  // leading bit index
  const int p = 32 * L;
  int sh = B + 1 - p;  // bits dropped below the mantissa (may be <= 0)
  bool rbit = false, sticky = sticky_in;
  if (sh > 0) {
    const int rb = sh - 1;  // round bit position
    const int kr = rb / DBITS;
    const int rr = rb - kr * DBITS;
    // sticky: any bit below rb
    bool s = false;
    for (int j = 0; j < C; ++j) {
      const int k = lane * C + j;
      if (k < kr) s |= (dig[k] != 0);
      if (k == kr) {
        uint32_t d = (uint32_t)dig[k];
        rbit = (d >> rr) & 1u;
        s |= (rr > 0) && ((d & ((1u << rr) - 1u)) != 0);
      }
    }
    sticky |= (__ballot(s) != 0ull);
    rbit = (__ballot(rbit) != 0ull);
  }
  // mantissa limbs: limb j = bits [sh + 32 j, +32)
  const int CL = (L + 63) >> 6;
  uint32_t mv[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    mv[j] = 0u;
    if (j >= CL) continue;
    int li = lane * CL + j;
    if (li < L) mv[j] = dig_bits32(dig, n, sh + 32 * li);
  }
  bool lsb = (__shfl((int)(mv[0] & 1u), 0, 64) & 1) != 0;
  bool up = rbit && (sticky || lsb);
  if (up) {
    // +1 at limb 0 with carry across lanes (propagate: all limbs 0xffffffff)
    bool g = false, allones = true;
    uint32_t cin = (lane == 0) ? 1u : 0u;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      int li = lane * CL + j;
      if (j < CL && li < L) {
        allones &= (mv[j] == 0xffffffffu);
        unsigned long long s2 = (unsigned long long)mv[j] + cin;
        mv[j] = (uint32_t)s2;
        cin = (uint32_t)(s2 >> 32);
      }
    }
    g = cin != 0;
    bool topc;
    bool in = lookahead(g, allones && lane != 0, &topc);
    if (in) {
      uint32_t c2 = 1u;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        int li = lane * CL + j;
        if (j < CL && li < L) {
          unsigned long long s2 = (unsigned long long)mv[j] + c2;
          mv[j] = (uint32_t)s2;
          c2 = (uint32_t)(s2 >> 32);
        }
      }
    }
    // the mantissa reached 2^p exactly when every limb wrapped to zero
    bool z = true;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      int li = lane * CL + j;
      if (j < CL && li < L) z &= (mv[j] == 0u);
    }
    if (__ballot(!z) == 0ull) {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        int li = lane * CL + j;
        if (j < CL && li < L) mv[j] = (li == L - 1) ? 0x80000000u : 0u;
      }
      sh += 1;
    }
  }
  long long E = dexp * DBITS + (long long)sh;
  bool ok = (E > -(1LL << 30) && E < (1LL << 30));
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    int li = lane * CL + j;
    if (j < CL && li < L) out[2 + li] = (int32_t)mv[j];
  }
  if (lane == 0) {
    out[0] = sign;
    out[1] = (int32_t)E;
  }
  __builtin_amdgcn_wave_barrier();
  return ok;
}

__device__ __forceinline__ long long divmod_small(long long val, int d, double inv, long long *rem) {
  // floor(val / d) for 0 <= val < 2^41, d < 2^13
  long long q = (long long)((double)val * inv);
  long long r = val - q * d;
  if (r < 0) { q -= 1; r += d; }
  if (r >= d) { q += 1; r -= d; }
  if (r >= d) { q += 1; r -= d; }
  *rem = r;
  return q;
}

// Round (sign * mag * 2^(28 dexp)) / d to p bits.  mag = dig[0..64C) is a
// magnitude digit vector.  Only its top nd+3 digits (nd = digits of a p-bit
// row) enter the division: the quotient then carries at least p + 2 bits,
// and the digits below can only make the value larger by less than one unit
// of the quotient's last digit, so they count as sticky bits, as does the
// final remainder.  Short magnitudes are extended with zero digits at the
// bottom until the quotient has p + 2 bits.  q is scratch of 64*CM digits.
template <int CM>
__device__ __forceinline__ bool wave_div_round(const int32_t *dig_, int C, int sign, long long dexp, int d, int L,
                               int nd, int32_t *q_, int32_t *out) {
  const int lane = lane_id();
  const l_i32 *dig = (const l_i32 *)dig_;
  l_i32 *q = (l_i32 *)q_;
  int t = wave_top_digit(dig, C);
  if (t < 0 || sign == 0) return wave_round(dig_, C, 0, 0, false, L, out);
  uint32_t dt = (uint32_t)dig[t];
  const int keep = nd + 3;
  int lowcut = t + 1 - keep;
  if (lowcut < 0) lowcut = 0;
  // digits below lowcut only matter through "nonzero"
  bool lz = false;
  for (int j = 0; j < C; ++j) {
    int k = lane * C + j;
    if (k < lowcut) lz |= (dig[k] != 0);
  }
  const bool low_nz = __ballot(lz) != 0ull;
  const int bits = (t - lowcut) * DBITS + (32 - __clz(dt));  // window bit length
  const int need = 32 * L + 16;
  int m = 0;
  if (bits < need) m = (int)((need - bits + DBITS - 1) / DBITS);
  int n2 = t + 1 - lowcut + m;  // dividend digits: dig[lowcut..t] shifted up by m
  int C2 = (n2 + 63) >> 6;
  if (C2 < 1) C2 = 1;
  const double inv = 1.0 / (double)d;
  // chunk remainder from the top
  long long r = 0;
  for (int j = C2 - 1; j >= 0; --j) {
    int k = lane * C2 + j - m + lowcut;
    long long x = (k >= lowcut && k <= t) ? (long long)(uint32_t)dig[k] : 0;
    divmod_small((r << DBITS) | x, d, inv, &r);
  }
  // P = 2^(28 C2) mod d
  long long P = 1;
  for (int j = 0; j < C2; ++j) divmod_small(P << DBITS, d, inv, &P);
  // suffix scan of x -> (x P + r_l) mod d, composed from the top lane down
  long long A = P, Bv = r;
  for (int s = 1; s < 64; s <<= 1) {
    long long A2 = __shfl_down(A, s, 64);
    long long B2 = __shfl_down(Bv, s, 64);
    if (lane + s < 64) {
      long long nb, na;
      divmod_small(A * B2 + Bv, d, inv, &nb);
      divmod_small(A * A2, d, inv, &na);
      A = na;
      Bv = nb;
    }
  }
  long long rin = __shfl_down(Bv, 1, 64);
  if (lane == 63) rin = 0;
  // quotient digits
  r = rin;
  for (int j = C2 - 1; j >= 0; --j) {
    int k = lane * C2 + j - m + lowcut;
    long long x = (k >= lowcut && k <= t) ? (long long)(uint32_t)dig[k] : 0;
    long long qq = divmod_small((r << DBITS) | x, d, inv, &r);
    q[lane * C2 + j] = (int32_t)qq;
  }
  bool sticky = (__shfl((int)(r != 0), 0, 64) != 0) || low_nz;
  __builtin_amdgcn_wave_barrier();
  return wave_round(q_, C2, sign, dexp + lowcut - m, sticky, L, out);
}

}  // namespace mpts
