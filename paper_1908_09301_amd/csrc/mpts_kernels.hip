// Persistent forward kernel: Taylor coefficients by the Leibniz recursion
// (equation (3)) and the Horner evaluation of the series (equation (2)) for
// one or many Lorenz trajectories, each trajectory on a group of G
// workgroups.
//
// Per coefficient index i every workgroup of a group accumulates its share
// of five exact product frames into LDS:
//   F0 = sum_k a_{i-k} g_k     (the Cauchy sum s1_i of equation (3))
//   F1 = sum_k a_{i-k} b_k     (s2_i)
//   F2 = sigma b_i - sigma a_i (numerator of a_{i+1})
//   F3 = R a_i                 (with -b_i - s1_i: numerator of b_{i+1})
//   F4 = -b g_i                (with + s2_i: numerator of g_{i+1})
// and adds them into global column sums (G > 1) with L2-bypassing atomics.
// The group's first workgroup then rounds s1_i and s2_i, forms the three
// exact numerators, divides by i+1 with one rounding each, and publishes
// a_{i+1}, b_{i+1}, g_{i+1} as rows; one flag per index orders the group.
#include <hip/hip_runtime.h>
#include "mpts_common.h"
#include "mpts_wave.h"
#include "mpts_digits.h"
#include "mpts_rows.h"
#include "mpts_mfma.h"
#include "mpts_kernels.h"

namespace mpts {

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct Addend {
  const int32_t *p;  // row (is_row; global memory) or normalised value [sign, E, M]
  int is_row;
  int sgn;
  int lds;           // a normalised value in LDS (else in global memory)
};

// Exact sum of one product frame (columns from global memory or LDS) and up
// to three addends, resolved into sign and magnitude digits dig[0..64C).
// Each lane gathers its own chunk of columns straight into registers.
// Single wavefront.
template <int CM>
__device__ __forceinline__ int combine_resolve(const long long *frame, bool frame_global, const FrameD *fd,
                               int nd, int L, const Addend *adds, int nadd, int32_t *dig,
                               int *C, long long *dexp, uint32_t *err) {
  const int lane = lane_id();
  long long lo = (1LL << 40), hi = -(1LL << 40);
  int fcols = 0;
  if (fd && fd->nz) {
    fcols = frame_cols(*fd, nd);
    lo = fd->base;
    hi = (long long)fd->base + fcols;
  }
  long long ae[3], ash[3];
  int as[3];
  for (int a = 0; a < nadd; ++a) {
    long long e;
    int s;
    ash[a] = 0;
    const int32_t *ap = adds[a].p;
    int h0, h1;
    if (adds[a].lds) {
      h0 = ((const l_i32 *)ap)[0];
      h1 = ((const l_i32 *)ap)[1];
    } else {
      h0 = ((const g_i32 *)ap)[0];
      h1 = ((const g_i32 *)ap)[1];
    }
    if (adds[a].is_row) {
      e = h0;
      s = h1;
    } else {
      s = h0;
      e = floordiv28(h1, &ash[a]);
    }
    ae[a] = e;
    as[a] = s;
    if (s != 0) {
      lo = min(lo, e);
      hi = max(hi, e + nd);
    }
  }
  if (lo > hi || hi - lo + 2 > 64LL * CM) {
    if (lo <= hi && lane == 0) atomicOr(err, 1u);
    *C = 2;
    *dexp = 0;
    for (int j = lane; j < 128; j += 64) dig[j] = 0;
    __builtin_amdgcn_wave_barrier();
    return 0;
  }
  const int W = (int)(hi - lo + 2);
  int Cc = (W + 63) >> 6;
  if (Cc < 2) Cc = 2;
  *C = Cc;
  const int c0 = lane * Cc;
  long long v[CM];
#pragma unroll
  for (int j = 0; j < CM; ++j) v[j] = 0;
  if (fcols) {
    const int o = (int)(fd->base - lo);
    if (frame_global) {
      // branch-free: offsets outside the lane's chunk or the frame read 0
      const __amdgpu_buffer_rsrc_t rs = dev_rsrc(frame, fcols * 8);
#pragma unroll
      for (int j = 0; j < CM; ++j) {
        int fc = c0 + j - o;
        int off = (j < Cc && fc >= 0) ? fc * 8 : 0x7ffffff0;
        v[j] = ld_dev64(rs, off);
      }
    } else {
      const l_i64 *lfr = (const l_i64 *)frame;
#pragma unroll
      for (int j = 0; j < CM; ++j) {
        if (j < Cc) {
          int fc = c0 + j - o;
          if (fc >= 0 && fc < fcols) v[j] = lfr[fc];
        }
      }
    }
  }
  for (int a = 0; a < nadd; ++a) {
    if (as[a] == 0) continue;
    const int o = (int)(ae[a] - lo);
    const long long sg = adds[a].sgn;
    if (adds[a].is_row) {
      // digits of the row (global): gathered branch-free through a buffer
      // resource, whose range check reads 0 outside the row's digits
      const __amdgpu_buffer_rsrc_t rs = dev_rsrc(adds[a].p + HDR + RPAD, nd * 4);
#pragma unroll
      for (int j = 0; j < CM; ++j) {
        const int k = c0 + j - o;
        const int off = (j < Cc && k >= 0) ? k * 4 : 0x7ffffff0;
        v[j] += sg * (long long)(int32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
      }
    } else {
      const long long sgs = sg * as[a];
      const int sh = (int)ash[a];
      if (adds[a].lds) {
        const l_i32 *M = (const l_i32 *)(adds[a].p + 2);
#pragma unroll
        for (int j = 0; j < CM; ++j) {
          if (j < Cc) {
            int k = c0 + j - o;
            if (k >= 0 && k < nd) v[j] += sgs * (long long)mant_bits28_l(M, L, DBITS * k - sh);
          }
        }
      } else {
        const g_i32 *M = (const g_i32 *)(adds[a].p + 2);
#pragma unroll
        for (int j = 0; j < CM; ++j) {
          if (j < Cc) {
            int k = c0 + j - o;
            if (k >= 0 && k < nd) v[j] += sgs * (long long)mant_bits28_g(M, L, DBITS * k - sh);
          }
        }
      }
    }
  }
  bool ovf = false;
  int sgn = wave_resolve_regs<CM>(v, Cc, dig, &ovf);
  if (ovf && lane == 0) atomicOr(err, 1u);
  *dexp = lo;
  return sgn;
}

// A row addend of a gather: row (global memory, or LDS when lds), times sgn.
struct RowAdd {
  const int32_t *row;
  int sgn;
  int lds;
};

// Digit window [lo, lo + W) of the exact sum of a product frame and up to
// three row addends (W includes two digits of headroom for carries).  Sets
// *C = ceil(W / 64) (at least 2) and the addends' exponents and signs.
// Returns false, flagging the error word, when the window needs more than
// the task's 64 CM digits; a sum with no nonzero operand has C = 2, lo = 0.
template <int CM>
__device__ __forceinline__ bool sum_window(const FrameD *fd, int nd, const RowAdd *adds, int nadd,
                                           long long *lo_out, int *C, int *ae, int *as,
                                           uint32_t *err) {
  long long lo = (1LL << 40), hi = -(1LL << 40);
  if (fd && fd->nz) {
    lo = fd->base;
    hi = (long long)fd->base + frame_cols(*fd, nd);
  }
  for (int a = 0; a < nadd; ++a) {
    if (adds[a].lds) {
      ae[a] = ((const l_i32 *)adds[a].row)[0];
      as[a] = ((const l_i32 *)adds[a].row)[1];
    } else {
      ae[a] = ((const g_i32 *)adds[a].row)[0];
      as[a] = ((const g_i32 *)adds[a].row)[1];
    }
    if (as[a] != 0) {
      lo = min(lo, (long long)ae[a]);
      hi = max(hi, (long long)ae[a] + nd);
    }
  }
  *C = 2;
  *lo_out = 0;
  if (lo > hi) return true;
  if (hi - lo + 2 > 64LL * CM) {
    if (lane_id() == 0) atomicOr(err, 1u | 32u);
    return false;
  }
  const int W = (int)(hi - lo + 2);
  *C = W > 128 ? (W + 63) >> 6 : 2;
  *lo_out = lo;
  return true;
}

// The sum of sum_window, gathered into registers (lane l: columns
// [l C, l C + C) over 2^(28 lo)) and resolved into sign and magnitude
// digits.  Single wavefront.
template <int C>
__device__ __forceinline__ int gather_c(const long long *frame, bool frame_global, const FrameD *fd,
                                        int nd, const RowAdd *adds, int nadd, const int *ae,
                                        const int *as, long long lo, int (&d)[C], uint32_t *err) {
  const int lane = lane_id();
  const int c0 = lane * C;
  long long v[C];
#pragma unroll
  for (int j = 0; j < C; ++j) v[j] = 0;
  if (fd && fd->nz) {
    const int fcols = frame_cols(*fd, nd);
    const int o = (int)(fd->base - lo);
    if (frame_global) {
      // branch-free: offsets outside the frame read 0
      const __amdgpu_buffer_rsrc_t rs = dev_rsrc(frame, fcols * 8);
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const int fc = c0 + j - o;
        v[j] = ld_dev64(rs, fc >= 0 ? fc * 8 : 0x7ffffff0);
      }
    } else {
      const l_i64 *lfr = (const l_i64 *)frame;
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const int fc = c0 + j - o;
        if (fc >= 0 && fc < fcols) v[j] = lfr[fc];
      }
    }
  }
  for (int a = 0; a < nadd; ++a) {
    if (as[a] == 0) continue;
    const int o = (int)(ae[a] - lo);
    const long long sg = adds[a].sgn;
    if (adds[a].lds) {
      const l_i32 *dg = (const l_i32 *)adds[a].row + HDR + RPAD;
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const int k = c0 + j - o;
        if (k >= 0 && k < nd) v[j] += sg * (long long)dg[k];
      }
    } else {
      const __amdgpu_buffer_rsrc_t rs = dev_rsrc(adds[a].row + HDR + RPAD, nd * 4);
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const int k = c0 + j - o;
        v[j] += sg * (long long)(int32_t)__builtin_amdgcn_raw_buffer_load_b32(
                         rs, k >= 0 ? k * 4 : 0x7ffffff0, 0, 0);
      }
    }
  }
  bool ovf = false;
  const int sgn = resolve_c<C>(v, d, &ovf);
  if (ovf && lane == 0) atomicOr(err, 1u | 64u);
  return sgn;
}

// Round the exact sum of a frame and row addends to p bits into the LDS row
// `out` (div == 0), or divide it by div and round (div >= 1; scratch: 64 CM
// LDS digits).  Single wavefront.  Returns false on an error (flagged).
template <int CM>
__device__ __forceinline__ bool sum_to_row(const long long *frame, bool frame_global,
                                           const FrameD *fd, int nd, const RowAdd *adds, int nadd,
                                           int div, int L, int RS, int32_t *scratch, int32_t *out,
                                           uint32_t *err) {
  long long lo;
  int C, ae[3], as[3];
  const bool okw = sum_window<CM>(fd, nd, adds, nadd, &lo, &C, ae, as, err);
  bool ok = okw;
  with_chunks<CM>(C, [&](auto ct) {
    constexpr int Ct = decltype(ct)::value;
    int d[Ct];
    int sgn = 0;
    if (okw) {
      sgn = gather_c<Ct>(frame, frame_global, fd, nd, adds, nadd, ae, as, lo, d, err);
    } else {
#pragma unroll
      for (int j = 0; j < Ct; ++j) d[j] = 0;
    }
    if (div == 0) ok &= round_to_row<Ct>(d, sgn, lo, false, L, nd, RS, out);
    else ok &= div_to_row<Ct, CM>(d, sgn, lo, div, L, nd, RS, scratch, out);
  });
  return ok;
}

// A rational step size: d tau = n + m 2^(28 e) exactly, m = m1 2^28 + m0
// (0 <= m0 < 2^28, |n| < 2^27, 1 <= d < 2^13).
struct TauQ {
  int n, m0, m1, e, dv;
};

// Columns [lo, lo + 64 Ct) of the numerator n h + m 2^(28 e) h + d c of a
// rational Horner step into registers (lane l: columns lo + l Ct + j).
// Rows carry RPAD >= Ct + 1 zero digits on each side (and a zero row has
// zero digits): a chunk that overlaps a row's digits is read whole, one
// that does not is pointed at the zeros, so no read is predicated.
template <int Ct>
__device__ __forceinline__ void tau_gather(const TauQ &q, const l_i32 *h, int eh, const l_i32 *c,
                                           int ec, long long lo, int nd, long long (&v)[Ct]) {
  const int lane = lane_id();
  const l_i32 *hd = h + HDR + RPAD;
  int kh = (int)(lo - eh) + lane * Ct;
  int km = kh - q.e;
  kh = min(max(kh, -Ct), nd);
  km = min(max(km, -Ct), nd + 1);
#pragma unroll
  for (int j = 0; j < Ct; ++j)
    v[j] = (long long)q.n * hd[kh + j] + (long long)q.m0 * hd[km + j] +
           (long long)q.m1 * hd[km + j - 1];
  if (c) {
    const l_i32 *cd = c + HDR + RPAD;
    int kc = (int)(lo - ec) + lane * Ct;
    kc = min(max(kc, -Ct), nd);
#pragma unroll
    for (int j = 0; j < Ct; ++j) v[j] += (long long)q.dv * cd[kc + j];
  }
}

// One step h <- round(tau h + c) of equation (2) for a rational step size
// (c: an LDS row, or null for h <- round(tau h)), in place on the LDS row
// h.  The exact value tau h + c is (n h + m 2^(28 e) h + d c) / d.
//
// First try: the numerator's columns from G = 3 digits below its lowest
// operand (about half the columns: the m term lies about p bits below n h).
// Its columns below that window add, in units of the window's lowest
// column, less than 2^30 in magnitude (each column sum is below 2^57), so
// the quotient q of the truncated numerator is within 2^31 of the exact
// one.  When q's bits from 2^31 up to the one below its round bit are
// neither all zeros nor all ones, the exact quotient has the same kept bits
// and round bit and a nonzero remainder, so q rounded with sticky set is
// the correctly rounded result.  Otherwise (or on cancellation) the whole
// numerator is gathered: resolved, divided by d in registers and rounded
// once, or through div_to_row when it is too short for p + 2 quotient bits.
// Single wavefront; scratch: 64 CM LDS digits.
template <int CM, typename Mark>
__device__ __forceinline__ bool tau_step_rational(const TauQ &q, int L, int nd, int RS, int32_t *h_,
                                                  const int32_t *c_, int32_t *scratch,
                                                  uint32_t *err, Mark &&mark) {
  const int lane = lane_id();
  const l_i32 *h = (const l_i32 *)h_;
  const l_i32 *c = (const l_i32 *)c_;
  const int eh = h[0], sh = h[1];
  const int ec = c ? c[0] : 0, sc = c ? c[1] : 0;
  const bool mterm = q.m0 != 0 || q.m1 != 0;
  // window: the m term lies about p bits below n h; without it, one zero
  // digit below the lowest operand keeps p + 2 quotient bits
  long long lo = 1LL << 40, hi = -(1LL << 40), lop = 1LL << 40;
  if (sh != 0) {
    lo = mterm ? (long long)eh + q.e : (long long)eh - 1;
    lop = eh;
    hi = (long long)eh + nd + 1;  // n h: |n| < 2^27 adds one digit
    if (mterm) hi = max(hi, (long long)eh + q.e + nd + 1);
  }
  if (sc != 0) {
    lo = min(lo, (long long)ec - 1);
    lop = min(lop, (long long)ec);
    hi = max(hi, (long long)ec + nd + 1);
  }
  bool ok = true;
  // the truncated window
  bool done = false;
  constexpr int G = 3;
  if (lo <= hi && hi - (lop - G) + 2 <= 64LL * CM) {
    const long long lot = lop - G;
    const int Wt = (int)(hi - lot + 2);
    with_chunks<CM>(Wt > 128 ? (Wt + 63) >> 6 : 2, [&](auto ct) {
      constexpr int Ct = decltype(ct)::value;
      long long v[Ct];
      tau_gather<Ct>(q, h, eh, c, ec, lot, nd, v);
      int d[Ct];
      bool ovf = false;
      const int sgn = resolve_c<Ct>(v, d, &ovf);
      mark(13);
      if (sgn == 0 || ovf) return;
      (void)div_small_c<Ct>(d, q.dv);
      const int B = top_bit_c<Ct>(d);
      const int rb = B + 1 - 32 * L - 1;  // the round bit
      if (rb < 40 || bits_uniform<Ct>(d, 31, rb)) return;
      ok &= round_to_row<Ct>(d, sgn, lot, true, L, nd, RS, h_);
      done = true;
      mark(14);
    });
  }
  if (done) return ok;
  int C = 2;
  if (lo > hi) {
    lo = 0;
  } else if (hi - lo + 2 > 64LL * CM) {
    if (lane == 0) atomicOr(err, 1u | 32u);
    ok = false;
    lo = 0;
  } else {
    const int W = (int)(hi - lo + 2);
    C = W > 128 ? (W + 63) >> 6 : 2;
  }
  const bool any = ok && (sh != 0 || sc != 0);
  with_chunks<CM>(C, [&](auto ct) {
    constexpr int Ct = decltype(ct)::value;
    long long v[Ct];
#pragma unroll
    for (int j = 0; j < Ct; ++j) v[j] = 0;
    if (any) tau_gather<Ct>(q, h, eh, c, ec, lo, nd, v);
    int d[Ct];
    bool ovf = false;
    const int sgn = resolve_c<Ct>(v, d, &ovf);
    if (ovf && lane == 0) atomicOr(err, 1u | 64u);
    const int B = sgn != 0 ? top_bit_c<Ct>(d) : -1;
    if (B >= 32 * L + 15) {
      const bool sticky = div_small_c<Ct>(d, q.dv);
      ok &= round_to_row<Ct>(d, sgn, lo, sticky, L, nd, RS, h_);
    } else {
      ok &= div_to_row<Ct, CM>(d, sgn, lo, q.dv, L, nd, RS, scratch, h_);
    }
    mark(14);
  });
  return ok;
}

// Normalised value [sign, E, M] of an LDS row (exact: a row holds p bits).
// scratch: 64 CM digits of LDS; out: L + 2 words of LDS.  Single wavefront.
template <int CM>
__device__ void row_to_norm(const int32_t *row_, int L, int nd, int32_t *scratch_, int32_t *out) {
  const int lane = lane_id();
  const l_i32 *row = (const l_i32 *)row_;
  l_i32 *sc = (l_i32 *)scratch_;
  const int C = (nd + 1 + 63) >> 6;
  for (int j = 0; j < C; ++j) {
    const int k = lane * C + j;
    const int d = k < nd ? row[HDR + RPAD + k] : 0;
    sc[k] = d < 0 ? -d : d;
  }
  const int sign = row[1];
  const long long e = row[0];
  __builtin_amdgcn_wave_barrier();
  (void)wave_round(scratch_, C, sign, e, false, L, out);
}

// Copy an LDS row (RS words) to global memory (relaxed: L2-bypassing
// stores, for rows that other workgroups read).  Single wavefront.
__device__ __forceinline__ void publish_row(const int32_t *src_, int32_t *dst, int RS, bool relaxed) {
  const int lane = lane_id();
  const l_i32 *src = (const l_i32 *)src_;
  for (int w = lane; w < RS; w += 64) {
    if (relaxed) st_relaxed(dst + w, src[w]);
    else ((g_i32 *)dst)[w] = src[w];
  }
}

struct Carve {
  long long *lf;       // NFR * WB frame columns
  long long *tcols;    // 3 task buffers of 64*CM 64-bit words: digits, then quotient digits
  int32_t *tnorm;      // 3 tasks x 2 normalised values, NV each (aliases trow)
  int32_t *trow;       // 3 tasks x 2 LDS rows (RS each): a rounded sum, the result
  int32_t *hrow;       // 4 LDS rows (3 Horner accumulators, tau)
  FrameSrc *fs;        // NFR frames of an index, then the 2 early Cauchy frames of the next
  FrameD *fd;          // the same
  int *red;            // 64
  int *geo;            // geometry of the late frames (LG_WORDS)
  unsigned long long *tmark;  // phase timer: time of the last mark
  int *span;           // 2 NFR column ranges of this workgroup, then 4 of the early frames
  int *hc;             // exponent caches: [3][N+1] coefficient rows, NCONST constants, then
                       // the constants' nonzero digit ranges (2 NCONST)
  int8_t *offs;        // adjoint: per-term offset tables of parts without caches
  int maxn;            // bytes of offs
  int NV;
  uint8_t *stage;      // followers' MFMA staging buffers (alias tcols .. hrow, extended
                       // when they need more)
};

// Bytes of the task columns, task rows and Horner rows (contiguous in the
// carve), raised to what the MFMA staging buffers need; the adjoint's
// per-term offset tables alias the task columns (they live from frame setup
// to the end of the products, the task columns only during finalisation).
__host__ __device__ inline size_t task_region_bytes(int L, int N, int nd, int RS, int CM,
                                                   bool adjoint, bool mfma) {
  const int NV = (L + 2 + 3) & ~3;
  size_t b = (size_t)3 * 64 * CM * 8 + (size_t)6 * (NV > RS ? NV : RS) * 4 + (size_t)4 * RS * 4;
  if (mfma && mf_fits(nd)) {
    const size_t st = (size_t)mf_stage_bytes(nd);
    if (st > b) b = st;
  }
  if (adjoint && (size_t)adj_table_bytes(N) > b) b = (size_t)adj_table_bytes(N);
  return b;
}

__device__ Carve carve(unsigned char *smem, const Inst &I) {
  Carve c;
  const int NV = (I.L + 2 + 3) & ~3;
  c.NV = NV;
  unsigned char *p = smem;
  c.lf = (long long *)p;
  p += (size_t)NFR * I.WB * 8;
  unsigned char *task0 = p;
  c.tcols = (long long *)p;
  c.stage = (uint8_t *)p;
  p += (size_t)3 * 64 * I.CM * 8;
  c.tnorm = (int32_t *)p;
  c.trow = (int32_t *)p;
  p += (size_t)6 * (NV > I.RS ? NV : I.RS) * 4;
  c.hrow = (int32_t *)p;
  p = task0 + task_region_bytes(I.L, I.N, I.nd, I.RS, I.CM, I.mode == MODE_ADJOINT,
                                (I.mfma & 1) != 0);
  c.fs = (FrameSrc *)p;
  p += sizeof(FrameSrc) * (NFR + 2);
  c.fd = (FrameD *)p;
  p += sizeof(FrameD) * (NFR + 2);
  c.red = (int *)p;
  p += 64 * 4;
  c.geo = (int *)p;
  p += 32 * 4;
  c.tmark = (unsigned long long *)p;
  p += 8;
  c.span = (int *)p;
  p += 4 * NFR * 4;
  c.hc = (int *)p;
  p += ((size_t)3 * (I.N + 1) + 3 * NCONST) * 4;
  c.maxn = I.mode == MODE_ADJOINT ? adj_table_bytes(I.N) : 0;
  c.offs = c.maxn ? (int8_t *)task0 : nullptr;
  return c;
}

// Phase timers (thread 0 of the group's first two workgroups, when
// Inst::prof is set): the ticks since the previous mark go to slot ph.
// Every workgroup also adds its setup, product, flush and release ticks to
// its own slots (PROF_RANK words per rank after the first 2 PH_NPHASE).
__device__ __forceinline__ void prof_mark(const Inst &I, const Carve &cv, int ph) {
  if (I.prof == nullptr || threadIdx.x != 0) return;
  const int rank = blockIdx.x - I.wg0;
  const unsigned long long t = wall_clock64();
  const unsigned long long dt = t - *cv.tmark;
  if (rank <= 1) atomicAdd(I.prof + rank * PH_NPHASE + ph, dt);
  const int slot = ph == PH_SETUP    ? 0
                   : ph == PH_ACCUM ? 1
                   : ph == PH_FLUSH ? 2
                   : ph == PH_CLEAR ? 3
                   : ph == PH_FINAL ? 6
                                    : -1;
  if (slot >= 0) atomicAdd(I.prof + 2 * PH_NPHASE + rank * PROF_RANK + slot, dt);
  *cv.tmark = t;
}

#if MPTS_CM == 4
size_t lds_bytes(int L, int N, int RS, int WB, int CM, bool adjoint, bool mfma) {
  const int nd = digits_per_row(L);
  size_t b = (size_t)NFR * WB * 8 + task_region_bytes(L, N, nd, RS, CM, adjoint, mfma) +
             sizeof(FrameSrc) * (NFR + 2) + sizeof(FrameD) * (NFR + 2) + 96 * 4 +
             8 + 4 * NFR * 4 + ((size_t)3 * (N + 1) + 3 * NCONST) * 4;
  return (b + 255) & ~(size_t)255;
}
#endif

__device__ __forceinline__ int32_t *row_ptr(const Inst &I, int arr, int idx) {
  return I.rows + ((long long)arr * (I.N + 1) + idx) * I.RS;
}

// Adjoint rows: u, v, w and their negations (N rows each), the powers of
// tau times the incoming adjoints (3 x (N+1) rows), and six normalised
// values: the adjoints of the state and of sigma, R, b.
enum { A_U = 0, A_V, A_W, A_NU, A_NV, A_NW };
__device__ __forceinline__ int32_t *adj_row(const Inst &I, int arr, int idx) {
  return I.adj + ((long long)arr * I.N + idx) * I.RS;
}
__device__ __forceinline__ int32_t *q_row(const Inst &I, int c, int idx) {
  return I.adj + (long long)6 * I.N * I.RS + ((long long)c * (I.N + 1) + idx) * I.RS;
}
__device__ __forceinline__ int32_t *bar_ptr(const Inst &I, int j) {
  return I.adj + (long long)6 * I.N * I.RS + (long long)3 * (I.N + 1) * I.RS + (long long)j * (I.L + 2);
}

__device__ __forceinline__ void copy_norm(const int32_t *src, int32_t *dst, int L, bool relaxed,
                                          int tid, int nthr) {
  for (int j = tid; j < L + 2; j += nthr) {
    if (relaxed) st_relaxed(dst + j, src[j]);
    else dst[j] = src[j];
  }
}

// Wave 0 of the leader: spin until the NSPLIT arrival counters (one per
// 128-byte line) sum to at least target; gives up like spin_until.
// A spin gives up when its own poll budget runs out or, checked now and
// then, when another workgroup has already given up (error bit 4): then
// every wait of the launch ends quickly and the host reports the timeout.
__device__ __forceinline__ bool spin_abandoned(long long polls, const uint32_t *err) {
  if (polls > (1LL << 25)) return true;
  if ((polls & 1023) != 0) return false;
  return (__builtin_amdgcn_raw_buffer_load_b32(dev_rsrc(err, 4), 0, 0, 16) & 4u) != 0;
}

__device__ void spin_until_sum(uint32_t *ctr, uint32_t target, uint32_t *err) {
  const int lane = threadIdx.x & 63;
  const __amdgpu_buffer_rsrc_t rs = dev_rsrc(ctr, NSPLIT * 128);
  const int off = lane < NSPLIT ? lane * 128 : 0x7ffffff0;
  long long polls = 0;
  while (true) {
    uint32_t v = __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 16);
#pragma unroll
    for (int o = 1; o < NSPLIT; o <<= 1) v += __shfl_xor(v, o, 64);
    if (__shfl(v, 0, 64) >= target) break;
    __builtin_amdgcn_s_sleep(2);
    if (spin_abandoned(++polls, err)) {
      if (lane == 0) atomicOr(err, 4u);
      break;
    }
  }
}

// Spin until *flag >= target (thread 0 only); gives up after ~2 s, marking
// the error word so that the host reports it instead of hanging.
__device__ void spin_until(uint32_t *flag, uint32_t target, uint32_t *err, bool slow = false) {
  long long polls = 0;
  // device-coherent (sc1) plain loads: they see the other workgroups'
  // atomics without turning every poll into a write at the coherence point.
  // A slow spin (a wait of milliseconds) polls every few microseconds, so
  // that hundreds of waiting workgroups do not crowd the memory path of the
  // ones at work.
  const __amdgpu_buffer_rsrc_t rs = dev_rsrc(flag, 4);
  while ((uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, 0, 0, 16) < target) {
    if (slow)
      __builtin_amdgcn_s_sleep(127);
    else
      __builtin_amdgcn_s_sleep(2);
    if (spin_abandoned(++polls, err)) {
      atomicOr(err, 4u);
      break;
    }
  }
}

// One finalisation task (one wavefront): which = 0 -> beta_{i+1},
// 1 -> gamma_{i+1}, 2 -> alpha_{i+1}.  Works on rows: the beta task keeps
// b_i as its previous result row.
template <int CM>
__device__ void finalize_task(const Inst &I, const Carve &cv, int which, int i,
                              const long long *frames, bool frames_global, uint32_t *err) {
  const int lane = lane_id();
  const bool timed = I.prof != nullptr && which == 0 && lane == 0 && blockIdx.x == I.wg0;
  unsigned long long tq = timed ? wall_clock64() : 0;
  auto sub = [&](int slot) {
    if (timed) {
      unsigned long long t = wall_clock64();
      atomicAdd(I.prof + slot, t - tq);
      tq = t;
    }
  };
  const int L = I.L, nd = I.nd, WB = I.WB, RS = I.RS;
  int32_t *scratch = (int32_t *)(cv.tcols + (size_t)which * 64 * I.CM);
  int32_t *srow = cv.trow + (size_t)(2 * which) * RS;  // rounded Cauchy sum
  int32_t *orow = srow + RS;                            // result (beta: b_i before)
  int arr_out;
  bool ok = true;
  if (which == 0 || which == 1) {
    // s1 (which 0) or s2 (which 1): one rounding of the exact Cauchy sum
    ok &= sum_to_row<CM>(frames + (size_t)which * WB, frames_global, &cv.fd[which], nd, nullptr, 0,
                         0, L, RS, scratch, srow, err);
    sub(9);
    RowAdd ad[2];
    int nad, f;
    if (which == 0) {
      // R a_i - b_i - s1_i
      ad[0] = RowAdd{orow, -1, 1};
      ad[1] = RowAdd{srow, -1, 1};
      nad = 2;
      f = 3;
      arr_out = 1;
    } else {
      // s2_i - b g_i
      ad[0] = RowAdd{srow, 1, 1};
      nad = 1;
      f = 4;
      arr_out = 2;
    }
    ok &= sum_to_row<CM>(frames + (size_t)f * WB, frames_global, &cv.fd[f], nd, ad, nad, i + 1, L,
                         RS, scratch, orow, err);
  } else {
    // sigma (b_i - a_i)
    ok &= sum_to_row<CM>(frames + (size_t)2 * WB, frames_global, &cv.fd[2], nd, nullptr, 0, i + 1,
                         L, RS, scratch, orow, err);
    arr_out = 0;
  }
  sub(11);
  if (!ok && lane == 0) atomicOr(err, 2u);
  publish_row(orow, row_ptr(I, arr_out, i + 1), RS, I.G > 1);
  sub(12);
  if (I.coefs) {
    int32_t *nv = scratch + 64 * I.CM;
    row_to_norm<CM>(orow, L, nd, scratch, nv);
    copy_norm(nv, I.coefs + ((long long)arr_out * (I.N + 1) + i + 1) * (L + 2), L, false, lane,
              64);
  }
}

// ---------------------------------------------------------------------------
// Group protocol: one coefficient (or adjoint) index at a time.
struct GroupSync {
  uint32_t gen;
  unsigned long long nbulk;    // rounds of group frames so far (their parity picks the buffer)
  unsigned long long arrived;  // arrivals the leader has waited for so far
};

// Leader: after writing rows that the group will read, publish them.
// Followers: wait for that publication.
__device__ void group_publish(const Inst &I, bool leader, GroupSync &gs, uint32_t *err) {
  const int tid = threadIdx.x;
  if (leader) {
    wait_vmem();
    __syncthreads();
    ++gs.gen;
    if (I.G > 1 && tid < NSPLIT) st_relaxed(I.sync + SY_FLAG + 32 * tid, gs.gen);
  } else {
    ++gs.gen;
    const int rank = blockIdx.x - I.wg0;
    if (tid == 0) spin_until(I.sync + SY_FLAG + 32 * (rank % NSPLIT), gs.gen, err);
    __syncthreads();
  }
}

// Every workgroup of the group: frame descriptors, this workgroup's share
// of the products into LDS, and (G > 1) the L2-bypassing atomic adds of
// its columns into the group's global frames.  The leader then waits for
// every workgroup's adds.  Returns the frames the leader finalises from.
__device__ __forceinline__ const long long *group_bulk(const Inst &I, const Carve &cv, int nf, int rank,
                                       GroupSync &gs, uint32_t *err) {
  const int tid = threadIdx.x;
  const int G = I.G, WB = I.WB;
  frame_setup(cv.fs, cv.fd, nf, I.nd, I.RS, cv.red, cv.offs, cv.maxn, err);
  prof_mark(I, cv, PH_SETUP);
  frames_accumulate(cv.fs, cv.fd, nf, I.nd, I.RS, WB, cv.lf, rank, G, cv.span);
  __syncthreads();
  prof_mark(I, cv, PH_ACCUM);
  ++gs.nbulk;
  gs.arrived += (unsigned long long)G;
  long long *gf = I.gframes + (size_t)(gs.nbulk & 1) * NFR * WB;
  if (G == 1) return cv.lf;
  for (int f = 0; f < nf; ++f) {
    int c0 = cv.span[2 * f], c1 = cv.span[2 * f + 1];
    for (int c = c0 + tid; c < c1; c += WGS) {
      long long v = cv.lf[(size_t)f * WB + c];
      if (v != 0) {
        __hip_atomic_fetch_add((unsigned long long *)(gf + (size_t)f * WB + c),
                               (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        cv.lf[(size_t)f * WB + c] = 0;
      }
    }
  }
  wait_vmem();
  __syncthreads();
  prof_mark(I, cv, PH_FLUSH);
  if (tid == 0)
    __hip_atomic_fetch_add(I.sync + SY_ARRIVE + 32 * (rank % NSPLIT), 1u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
  if (rank == 0) {
    if (tid < 64) spin_until_sum(I.sync + SY_ARRIVE, (uint32_t)gs.arrived, err);
    __syncthreads();
    prof_mark(I, cv, PH_WAIT);
  }
  return gf;
}

// Leader: clear the frames it finalised from, then publish its new rows.
// Followers: wait for the publication.
// Exponent cache entries: coefficient row (arr, idx) and constant row c.
__device__ __forceinline__ int *hc_row(const Inst &I, const Carve &cv, int arr) {
  return cv.hc + (size_t)arr * (I.N + 1);
}
__device__ __forceinline__ int *hc_const(const Inst &I, const Carve &cv, int c) {
  return cv.hc + (size_t)3 * (I.N + 1) + c;
}
__device__ __forceinline__ int *hc_span(const Inst &I, const Carve &cv, int c) {
  return cv.hc + (size_t)3 * (I.N + 1) + NCONST + 2 * c;
}

// Leader: clear the frames it finalised from.  The clears are issued after
// the publication and not waited for here: the frames (of this index parity)
// are next written at index + 2, after the leader's next publication, whose
// wait covers these stores.
__device__ void clear_frames(const Inst &I, const Carve &cv, int nf, const long long *frames) {
  const int tid = threadIdx.x;
  for (int f = 0; f < nf; ++f) {
    int nc = cv.fd[f].nz ? frame_cols(cv.fd[f], I.nd) : 0;
    long long *fr = const_cast<long long *>(frames) + (size_t)f * I.WB;
    for (int c = tid; c < nc; c += WGS) {
      if (I.G > 1) st_relaxed(fr + c, 0LL);
      else fr[c] = 0;
    }
  }
}

// Leader: publish its new rows, then clear the frames.  Followers: wait for
// the publication.
__device__ void group_release(const Inst &I, const Carve &cv, int nf, bool leader,
                              const long long *frames, GroupSync &gs, uint32_t *err) {
  group_publish(I, leader, gs, err);
  if (leader) clear_frames(I, cv, nf, frames);
}

// Thread 0 of a follower: wait for the coefficient-row flag of generation
// gen on its line (six 64-bit words, gen in the high half, a header word in
// the low half: written whole, so a word that carries gen carries its value)
// and return the six header words.
__device__ void spin_hdr(const uint32_t *line, uint32_t gen, int *vals, uint32_t *err) {
  const __amdgpu_buffer_rsrc_t rs = dev_rsrc(line, 48);
  long long polls = 0;
  while (true) {
    unsigned long long w[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) w[j] = (unsigned long long)ld_dev64(rs, 8 * j);
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 6; ++j) ok &= (uint32_t)(w[j] >> 32) == gen;
    if (ok) {
#pragma unroll
      for (int j = 0; j < 6; ++j) vals[j] = (int)(uint32_t)w[j];
      return;
    }
    __builtin_amdgcn_s_sleep(2);
    if (spin_abandoned(++polls, err)) {
      atomicOr(err, 4u);
      for (int j = 0; j < 6; ++j) vals[j] = 0;
      return;
    }
  }
}

// Coefficient index i done: the leader publishes rows i+1 (three LDS result
// rows of its finalisation tasks) with their headers in the coefficient-row
// flag, then clears the frames; every workgroup caches the exponents of
// rows i+1.
__device__ void release_rows(const Inst &I, const Carve &cv, bool leader,
                             const long long *frames, GroupSync &gs, int i, uint32_t *err) {
  const int tid = threadIdx.x;
  const int RS = I.RS;
  // result rows of the tasks: beta (task 0) -> array 1, gamma (1) -> 2, alpha (2) -> 0
  if (leader) {
    wait_vmem();
    __syncthreads();
    ++gs.gen;
    if (I.G > 1 && tid < 6 * NSPLIT) {
      const int line = tid / 6, j = tid - 6 * line;
      const int arr = j >> 1;
      const int task = arr == 0 ? 2 : arr - 1;
      const int v = ((const l_i32 *)(cv.trow + (size_t)(2 * task + 1) * RS))[j & 1];
      __hip_atomic_store((unsigned long long *)(I.sync + SY_HFLAG + 32 * line) + j,
                         ((unsigned long long)gs.gen << 32) | (uint32_t)v, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }

    if (tid < 3) {
      const int task = tid == 0 ? 2 : tid - 1;
      const l_i32 *row = (const l_i32 *)(cv.trow + (size_t)(2 * task + 1) * RS);
      hc_row(I, cv, tid)[i + 1] = row[1] != 0 ? row[0] : HZ;
    }
    if (frames) clear_frames(I, cv, NFR, frames);
    __syncthreads();
  } else {
    ++gs.gen;
    if (tid == 0) {
      const int rank = blockIdx.x - I.wg0;
      int v[6];
      spin_hdr(I.sync + SY_HFLAG + 32 * (rank % NSPLIT), gs.gen, v, err);
      for (int a = 0; a < 3; ++a) hc_row(I, cv, a)[i + 1] = v[2 * a + 1] != 0 ? v[2 * a] : HZ;
    }
    __syncthreads();
  }
}

// Digit range [lo, hi] of the row of each constant that holds all its
// nonzero digits (from the normalised constants; threads 0..NCONST-1).
__device__ void const_spans(const Inst &I, const Carve &cv) {
  const int c = threadIdx.x;
  if (c >= NCONST) return;
  const g_i32 *nv = (const g_i32 *)(I.cnorm + (size_t)c * (I.L + 2));
  int *sp = hc_span(I, cv, c);
  if (nv[0] == 0) {
    sp[0] = 0;
    sp[1] = I.nd - 1;
    return;
  }
  int lb = 0;
  for (int j = 0; j < I.L; ++j) {
    const uint32_t m = (uint32_t)nv[2 + j];
    if (m != 0u) {
      lb = 32 * j + __builtin_ctz(m);
      break;
    }
  }
  long long shl;
  (void)floordiv28(nv[1], &shl);  // row digit k = bits [28 k - sh, +28) of M
  const int sh = (int)shl;
  sp[0] = (lb + sh) / DBITS;
  sp[1] = (32 * I.L - 1 + sh) / DBITS;
}

// Rows 0 of the three coefficient arrays from a normalised state, published
// to the group; then, once per step, drop cached copies of rows that are
// about to be rewritten, and cache the exponents of rows 0 and the constants.
__device__ void start_step(const Inst &I, const Carve &cv, bool leader, const int32_t *state,
                           GroupSync &gs, uint32_t *err, bool rows_ready = false) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  if (!rows_ready) {
    if (leader && wave < 3)
      write_row(state + (size_t)wave * (I.L + 2), I.L, I.nd, I.RS, row_ptr(I, wave, 0), I.G > 1,
                lane, 64);
    group_publish(I, leader, gs, err);
  }
  if (I.G > 1) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    __syncthreads();
  }
  if (tid < 3) hc_row(I, cv, tid)[0] = row_exp(row_ptr(I, tid, 0));
  else if (tid < 3 + NCONST) *hc_const(I, cv, tid - 3) = row_exp(I.consts + (size_t)(tid - 3) * I.RS);
  __syncthreads();
}

// Exponent sum of the first nonzero term U[idx - k] V[k], k = k0..k1, from
// the exponent caches (HZ if every term is zero).
__device__ __forceinline__ int first_esum(const int *hU, const int *hV, int idx, int k0, int k1) {
  const l_i32 *u = (const l_i32 *)hU, *v = (const l_i32 *)hV;
  for (int k = k0; k <= k1; ++k) {
    const int a = u[idx - k], b = v[k];
    if (a != HZ && b != HZ) return a + b;
  }
  return HZ;
}

// Base of the Cauchy frame sum_k U[i-k] V[k] of index i: SMAX digits below
// the exponent sum of its first nonzero term, the terms k = 1..i-1 (which do
// not involve the newest rows) taken first.  The terms of an exact sum
// spread over at most SMAX digits, so every offset lies in [0, 2 SMAX].
__device__ __forceinline__ int cauchy_base(const int *hU, const int *hV, int i) {
  int e = i >= 2 ? first_esum(hU, hV, i, 1, i - 1) : HZ;
  if (e == HZ) e = first_esum(hU, hV, i, 0, 0);
  if (e == HZ && i > 0) e = first_esum(hU, hV, i, i, i);
  return e == HZ ? HZ : e - SMAX;
}

// ---------------------------------------------------------------------------
// The late frames of index i: the products with the newest rows i.
//   frame 0: a_i g_0 + a_0 g_i (the terms k = 0 and k = i of sum_k a_{i-k} g_k)
//   frame 1: a_i b_0 + a_0 b_i
//   frame 2: sigma b_i + (-sigma) a_i
//   frame 3: R a_i
//   frame 4: (-b) g_i
// (index 0: frames 0 and 1 hold the single term a_0 g_0, a_0 b_0).  The U
// operand gives the tile rows, the V operand the tile columns, read shifted
// by the term's offset from the frame base, so that a tile's 16 output
// columns do not depend on the offset.

// Largest term offset of late frame f: the Cauchy frames take their base
// SMAX below their first old term, the two terms of frame 2 spread over at
// most SMAX digits, and the single products have none.
enum { LG_N = 0, LG_MT0 = NFR, LG_MTF = 2 * NFR, LG_NT = 3 * NFR, LG_PRE = 4 * NFR,
       LG_WORDS = 5 * NFR + 1 };
static_assert(LG_WORDS <= 32, "late geometry fits its LDS words");

__device__ __forceinline__ int late_smax(int f) { return f < 2 ? 2 * SMAX : f == 2 ? SMAX : 0; }

// Geometry of the late frames in cv.geo, fixed for the launch (thread 0,
// after the constants' digit spans): terms per frame, tile rows [mt0, mt0 +
// MTf) holding the U operands' nonzero digits (the constants are often
// short), tile columns [0, NT) covering the largest offset, and the prefix
// sums of the (tile, term) items, which the followers deal among themselves.
__device__ void late_geometry(const Inst &I, const Carve &cv) {
  if (threadIdx.x != 0) return;
  const int nd = I.nd, MT = (nd + TQ - 1) / TQ;
  l_i32 *g = (l_i32 *)cv.geo;
  int pre = 0;
  for (int f = 0; f < NFR; ++f) {
    int lo = 0, hi = nd - 1;
    if (f == 2) {
      lo = min(hc_span(I, cv, C_SIGMA)[0], hc_span(I, cv, C_NSIGMA)[0]);
      hi = max(hc_span(I, cv, C_SIGMA)[1], hc_span(I, cv, C_NSIGMA)[1]);
    } else if (f >= 3) {
      const int c = f == 3 ? C_R : C_NB;
      lo = hc_span(I, cv, c)[0];
      hi = hc_span(I, cv, c)[1];
    }
    const int m0 = max(lo, 0) / TQ, m1 = min(hi, nd - 1) / TQ;
    const bool ok = m1 >= m0 && m0 < MT;
    g[LG_N + f] = f < 3 ? 2 : 1;
    g[LG_MT0 + f] = ok ? m0 : 0;
    g[LG_MTF + f] = ok ? min(m1, MT - 1) - m0 + 1 : MT;
    g[LG_NT + f] = (nd + late_smax(f) + TQ - 1) / TQ;
    g[LG_PRE + f] = pre;
    pre += g[LG_MTF + f] * g[LG_NT + f] * g[LG_N + f];
  }
  g[LG_PRE + NFR] = pre;
}

// Operands and exponents of term k of late frame f at index i.
__device__ __forceinline__ void late_term(const Inst &I, const Carve &cv, int f, int k, int i,
                                          const int32_t **U, const int32_t **V, int *eu,
                                          int *ev) {
  const l_i32 *ha = (const l_i32 *)hc_row(I, cv, 0), *hb = (const l_i32 *)hc_row(I, cv, 1),
              *hg = (const l_i32 *)hc_row(I, cv, 2);
  auto cst = [&](int c) { return (const int32_t *)(I.consts + (size_t)c * I.RS); };
  auto hcst = [&](int c) { return ((const l_i32 *)hc_const(I, cv, c))[0]; };
  if (f < 2) {
    const int arr = f == 0 ? 2 : 1;
    const l_i32 *hv = f == 0 ? hg : hb;
    const int iu = k == 0 ? i : 0, iv = k == 0 ? 0 : i;
    *U = row_ptr(I, 0, iu);
    *V = row_ptr(I, arr, iv);
    *eu = ha[iu];
    *ev = hv[iv];
  } else if (f == 2) {
    const int c = k == 0 ? C_SIGMA : C_NSIGMA;
    *U = cst(c);
    *V = row_ptr(I, k == 0 ? 1 : 0, i);
    *eu = hcst(c);
    *ev = k == 0 ? hb[i] : ha[i];
  } else {
    const int c = f == 3 ? C_R : C_NB;
    *U = cst(c);
    *V = row_ptr(I, f == 3 ? 0 : 2, i);
    *eu = hcst(c);
    *ev = f == 3 ? ha[i] : hg[i];
  }
}

__device__ __forceinline__ int esum2(int eu, int ev) { return (eu == HZ || ev == HZ) ? HZ : eu + ev; }

__device__ __forceinline__ int late_nterms(int f, int i) { return f < 2 ? (i == 0 ? 1 : 2) : f == 2 ? 2 : 1; }

// Exponent base of late frame f at index i: the Cauchy frames' given base,
// else the smallest exponent sum of the frame's nonzero terms (HZ: none).
__device__ int late_base(const Inst &I, const Carve &cv, int f, int i) {
  if (f < 2) return cauchy_base(hc_row(I, cv, 0), hc_row(I, cv, f == 0 ? 2 : 1), i);
  int b = 0x7fffffff;
  for (int k = 0; k < late_nterms(f, i); ++k) {
    const int32_t *U, *V;
    int eu, ev;
    late_term(I, cv, f, k, i, &U, &V, &eu, &ev);
    const int e = esum2(eu, ev);
    if (e != HZ) b = min(b, e);
  }
  return b == 0x7fffffff ? HZ : b;
}

// Leader: descriptor of frame f of index i as finalised (early and late
// terms together).  The Cauchy frames span every offset in [0, 2 SMAX] from
// their given base; the others are set up from their terms.
__device__ FrameD late_desc(const Inst &I, const Carve &cv, int f, int i, uint32_t *err) {
  int a = 0x7fffffff, b = -0x7fffffff;
  const int n = late_nterms(f, i);
  for (int k = 0; k < n; ++k) {
    const int32_t *U, *V;
    int eu, ev;
    late_term(I, cv, f, k, i, &U, &V, &eu, &ev);
    const int e = esum2(eu, ev);
    if (e != HZ) {
      a = min(a, e);
      b = max(b, e);
    }
  }
  const int fb = f < 2 ? late_base(I, cv, f, i) : HZ;
  FrameD d = make_desc(n, fb, 0, 0x7fffffff, a, b, I.nd, err);
  if (f < 2 && fb != HZ) {
    d.nz = 1;
    d.base = fb;
    d.nt0 = 0;
    d.S = 2 * SMAX;
    d.NT = (I.nd + 2 * SMAX + TQ - 1) / TQ;
  }
  return d;
}

// Follower: this workgroup's share of the late products of index i (a
// contiguous range of the items, one per thread in the usual case) into its
// LDS frames, then the columns it holds (with the early products of frames
// 0 and 1 of this index, accumulated there before) added into the group's
// frames in global memory, then its arrival.
__device__ __forceinline__ void late_step(const Inst &I, const Carve &cv, int rank, int i,
                                          GroupSync &gs) {
  const int tid = threadIdx.x, WB = I.WB;
  const l_i32 *g = (const l_i32 *)cv.geo;
  l_i32 *span = (l_i32 *)cv.span;
  const unsigned total = (unsigned)g[LG_PRE + NFR];
  const unsigned W = (unsigned)(I.G - 1), r = (unsigned)(rank - 1);
  const unsigned lo = (unsigned)(((unsigned long long)total * r) / W);
  const unsigned hi = (unsigned)(((unsigned long long)total * (r + 1)) / W);
  if (tid < NFR) {
    // columns of this workgroup's tiles of frame f (whole anti-diagonals)
    const int f = tid;
    const unsigned p0 = (unsigned)g[LG_PRE + f], p1 = (unsigned)g[LG_PRE + f + 1];
    const unsigned a = max(lo, p0), b = min(hi, p1);
    int c0 = 0, c1 = 0;
    if (a < b) {
      const int n = g[LG_N + f], MTf = g[LG_MTF + f], NT = g[LG_NT + f], mt0 = g[LG_MT0 + f];
      int mt, nt;
      tile_coords((int)((a - p0) / n), MTf, NT, &mt, &nt);
      const int d0 = mt + nt;
      tile_coords((int)((b - 1 - p0) / n), MTf, NT, &mt, &nt);
      const int d1 = mt + nt;
      c0 = (min(d0, d1) + mt0) * TQ;
      c1 = (max(d0, d1) + mt0) * TQ + 2 * TQ;
    }
    if (f < 2) {
      // frames 0 and 1 also hold the early products (then forget their range)
      l_i32 *es = span + 2 * NFR + 2 * f;
      if (es[0] < es[1]) {
        if (c0 < c1) {
          c0 = min(c0, (int)es[0]);
          c1 = max(c1, (int)es[1]);
        } else {
          c0 = es[0];
          c1 = es[1];
        }
      }
      es[0] = 0;
      es[1] = 0;
    }
    span[2 * f] = c0;
    span[2 * f + 1] = c1;
  }
  for (unsigned q = lo + tid; q < hi; q += WGS) {
    int f = 0;
    while (f < NFR - 1 && q >= (unsigned)g[LG_PRE + f + 1]) ++f;
    const unsigned rel = q - (unsigned)g[LG_PRE + f];
    const bool two = g[LG_N + f] == 2;
    const int t = (int)(two ? rel >> 1 : rel), k = (int)(two ? rel & 1u : 0u);
    if (k >= late_nterms(f, i)) continue;
    int mt, nt;
    tile_coords(t, g[LG_MTF + f], g[LG_NT + f], &mt, &nt);
    mt += g[LG_MT0 + f];
    const int32_t *U, *V;
    int eu, ev;
    late_term(I, cv, f, k, i, &U, &V, &eu, &ev);
    const int base = late_base(I, cv, f, i);
    const int e = esum2(eu, ev);
    const int off = (e == HZ || base == HZ) ? 0 : min(max(e - base, 0), late_smax(f));
    int32_t uu[TQ], vv[TQ];
    tile_load_g(uu, vv, (const g_i32 *)U, (const g_i32 *)V, mt, nt, off);
    long long acc[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[j] = 0;
    tile_fma(acc, uu, vv);
    acc_flush(acc, cv.lf + (size_t)f * WB + (mt + nt) * TQ);
  }
  __syncthreads();
  prof_mark(I, cv, PH_ACCUM);
  ++gs.nbulk;
  gs.arrived += (unsigned long long)(I.G - 1);
  long long *gf = I.gframes + (size_t)(gs.nbulk & 1) * NFR * WB;
  for (int f = 0; f < NFR; ++f) {
    const int c0 = span[2 * f], c1 = span[2 * f + 1];
    for (int c = c0 + tid; c < c1; c += WGS) {
      l_i64 *lc = (l_i64 *)cv.lf + (size_t)f * WB + c;
      const long long v = *lc;
      if (v != 0) {
        __hip_atomic_fetch_add((unsigned long long *)(gf + (size_t)f * WB + c),
                               (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        *lc = 0;
      }
    }
  }
  wait_vmem();
  __syncthreads();
  if (tid == 0)
    __hip_atomic_fetch_add(I.sync + SY_ARRIVE + 32 * (rank % NSPLIT), 1u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
  if (I.prof && tid == 0)  // the latest arrival time of the index (phase timers)
    __hip_atomic_fetch_max(I.prof + PROF_ARRT, wall_clock64(), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
  prof_mark(I, cv, PH_FLUSH);
}

// Follower: the early part of the two Cauchy frames of index j (terms
// k = 1..j-1, no row j) on the int8 matrix cores, added into the LDS frames
// 0 and 1 from their fixed bases (cv.fd[NFR], cv.fd[NFR + 1]).  The terms
// are dealt to the followers in contiguous ranges; a workgroup stages one
// term at a time (the next term's digits are loaded while the current one
// is multiplied) and its wavefronts split the U blocks.  Terms k0..k1-1.
template <int NQA, int JQA, int NQB, int JQB>
__device__ void mfma_terms(const Inst &I, const Carve &cv, int rank, int j, int k0, int k1,
                           const MfGeo &g, const MfPrefetch *first, long long *gf, uint32_t gen,
                           uint32_t *err) {
  const int tid = threadIdx.x, nd = I.nd;
  const l_i32 *ha = (const l_i32 *)hc_row(I, cv, 0), *hb = (const l_i32 *)hc_row(I, cv, 1),
              *hg = (const l_i32 *)hc_row(I, cv, 2);
  const int b0 = ((const l_i32 *)&cv.fd[NFR].base)[0], b1 = ((const l_i32 *)&cv.fd[NFR + 1].base)[0];
  auto offset = [&](int eu, int ev, int base) {
    if (eu == HZ || ev == HZ) return 0;
    return min(max(eu + ev - base, 0), 2 * SMAX);
  };
  mf_v16i acc[2][MF_NTMAX];
#pragma unroll
  for (int f = 0; f < 2; ++f)
#pragma unroll
    for (int q = 0; q < MF_NTMAX; ++q)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[f][q][e] = 0;
  // phase timers (one thread of the group's first follower): staging (with
  // the wait for its global loads), barrier, products, flush
  unsigned long long *tp = (I.prof && rank == 1 && tid == 0) ? I.prof + PH_NPHASE : nullptr;
  unsigned long long tq = tp ? wall_clock64() : 0;
  auto mark = [&](int slot) {
    if (tp) {
      const unsigned long long now = wall_clock64();
      tp[slot] += now - tq;
      tq = now;
    }
  };
  int32_t *P = (int32_t *)(cv.stage + 2 * (size_t)g.BUF);
  // the piece sums go straight into the group frames of index j (frame
  // generation gen), once the leader has published their clear; the first
  // barrier below orders this wait before every add
  if (tid == 0) spin_until(I.sync + SY_CLEAR, gen, err);
  MfPrefetch pf;
  if (first) pf = *first;
  else mf_load(pf, row_ptr(I, 0, j - k0), row_ptr(I, 2, k0), row_ptr(I, 1, k0), nd);
  int cnt = 0;
  for (int k = k0; k < k1; ++k) {
    uint8_t *buf = cv.stage + (size_t)((k - k0) & 1) * g.BUF;
    const int eu = ha[j - k];
    mf_store(pf, buf, g, nd, offset(eu, hg[k], b0), offset(eu, hb[k], b1));
    mark(9);
    __syncthreads();
    mark(13);
    if (k + 1 < k1) mf_load(pf, row_ptr(I, 0, j - k - 1), row_ptr(I, 2, k + 1), row_ptr(I, 1, k + 1), nd);
    mf_term<NQA, JQA, NQB, JQB>(acc, buf, g);
    mark(11);
    if (++cnt == g.FT) {
      mf_flush<2>(acc, P, g);
      __syncthreads();
      mf_columns_global(P, gf, I.WB, g);
      cnt = 0;
      mark(12);
    }
  }
  if (cnt > 0) {
    mf_flush<2>(acc, P, g);
    __syncthreads();
    mf_columns_global(P, gf, I.WB, g);
  }
  mark(12);
}

// Sets the early column spans of frames 0 and 1, then runs the terms with
// the operand counts of this row size (every size mf_fits admits is one of
// the cases below).
__device__ __forceinline__ void mfma_early(const Inst &I, const Carve &cv, int rank, int j, uint32_t *err,
                                           const MfPrefetch *first, long long *gf, uint32_t gen) {
  const int tid = threadIdx.x;
  const MfGeo g = mf_geo(I.nd);
  const int n = j - 1;
  const unsigned W = (unsigned)(I.G - 1), r = (unsigned)(rank - 1);
  const int k0 = 1 + (int)(((unsigned long long)n * r) / W);
  const int k1 = 1 + (int)(((unsigned long long)n * (r + 1)) / W);
  // the products go straight to the group frames: no early columns in LDS
  if (tid < 2) {
    l_i32 *es = (l_i32 *)cv.span + 2 * NFR + 2 * tid;
    es[0] = 0;
    es[1] = 0;
  }
  if (k1 <= k0) return;
  const int key = ((g.NQA * 8 + g.JQA) * 8 + g.NQB) * 8 + g.JQB;
  switch (key) {
#define MF_CASE(a, b, c, d)                                        \
  case ((a * 8 + b) * 8 + c) * 8 + d:                              \
    mfma_terms<a, b, c, d>(I, cv, rank, j, k0, k1, g, first, gf, gen, err); \
    break;
    MF_CASE(1, 0, 1, 0)
    MF_CASE(1, 0, 2, 0)
    MF_CASE(2, 0, 2, 0)
    MF_CASE(2, 0, 3, 0)
    MF_CASE(2, 2, 3, 2)
    MF_CASE(2, 2, 3, 3)
    MF_CASE(3, 3, 3, 3)
    MF_CASE(3, 3, 4, 3)
#undef MF_CASE
    default:
      if (tid == 0) atomicOr(err, 8u);  // a size mf_fits should have refused
  }
}

// The Taylor coefficients 1..N of one step (equation (3)), rows 0 given.
//
// One workgroup: every frame of index i in LDS, then the three
// finalisation tasks.
//
// Two or more: the leader (workgroup 0) only finalises.  The Cauchy sums
// are computed one index ahead: while the leader finalises index i, every
// follower accumulates its share of the terms of the Cauchy sums of index
// i+1 that involve no row i+1 (k = 1..i) into its LDS frames.  Once rows
// i+1 are published, the followers deal the late products among themselves
// (late_step), add their columns into the group's frames and arrive; the
// leader waits for them, finalises index i+1 from the group's frames and
// publishes rows i+2.  The early and late parts of a Cauchy frame share the
// base of cauchy_base, which needs no row i+1.  The leader clears each
// index's group frames while it waits for the next index's arrivals.
template <int CM>
__device__ void forward_coefficients(const Inst &I, const Carve &cv, int rank, GroupSync &gs,
                                     const int32_t *state, uint32_t *err) {
  const int tid = threadIdx.x, wave = tid >> 6;
  const bool leader = rank == 0;
  const int RS = I.RS, nd = I.nd, WB = I.WB;
  (void)state;
  // the beta task keeps b_i in LDS (its result row): start with the row b_0
  if (leader && wave == 0) {
    const g_i32 *b0 = (const g_i32 *)row_ptr(I, 1, 0);
    l_i32 *dst = (l_i32 *)(cv.trow + RS);
    for (int w = threadIdx.x & 63; w < RS; w += 64) dst[w] = b0[w];
  }
  const int *ha = hc_row(I, cv, 0), *hb = hc_row(I, cv, 1), *hg = hc_row(I, cv, 2);
  // the followers' staging buffers alias LDS that other phases use: their
  // zero padding is restored once per step
  if (I.G > 1 && !leader && (I.mfma & 1)) {
    mf_clear(cv.stage, mf_geo(nd));
    __syncthreads();
  }
  if (I.G == 1) {
    auto cst = [&](int c) { return I.consts + (size_t)c * RS; };
    for (int i = 0; i < I.N; ++i) {
      if (tid == 0) {
        FrameSrc fs[NFR];  // built in registers, stored to LDS below
        fs[0] = mk_frame1(mk_part(PK_CAUCHY, i + 1, i, row_ptr(I, 0, 0), row_ptr(I, 2, 0), ha, hg));
        fs[1] = mk_frame1(mk_part(PK_CAUCHY, i + 1, i, row_ptr(I, 0, 0), row_ptr(I, 1, 0), ha, hb));
        fs[0].fbase = cauchy_base(ha, hg, i);
        fs[1].fbase = cauchy_base(ha, hb, i);
        fs[2] = mk_frame2(mk_part(PK_ONE, 1, 0, cst(C_SIGMA), row_ptr(I, 1, i),
                                  hc_const(I, cv, C_SIGMA), hb + i),
                          mk_part(PK_ONE, 1, 0, cst(C_NSIGMA), row_ptr(I, 0, i),
                                  hc_const(I, cv, C_NSIGMA), ha + i));
        fs[3] = mk_frame1(mk_part(PK_ONE, 1, 0, cst(C_R), row_ptr(I, 0, i),
                                  hc_const(I, cv, C_R), ha + i));
        // sigma and R are often short: only their nonzero digit rows take tiles
        fs[2].mlo = min(hc_span(I, cv, C_SIGMA)[0], hc_span(I, cv, C_NSIGMA)[0]);
        fs[2].mhi = max(hc_span(I, cv, C_SIGMA)[1], hc_span(I, cv, C_NSIGMA)[1]);
        fs[3].mlo = hc_span(I, cv, C_R)[0];
        fs[3].mhi = hc_span(I, cv, C_R)[1];
        fs[4] = mk_frame1(mk_part(PK_ONE, 1, 0, cst(C_NB), row_ptr(I, 2, i),
                                  hc_const(I, cv, C_NB), hg + i));
#pragma unroll
        for (int f = 0; f < NFR; ++f) lds_put(cv.fs + f, fs[f]);
      }
      __syncthreads();
      const long long *frames = group_bulk(I, cv, NFR, rank, gs, err);
      if (tid < 2) {
        // frames 0 and 1 as finalised: from their base, wide enough for
        // every offset in [0, 2 SMAX]
        const int eb = cauchy_base(ha, tid == 0 ? hg : hb, i);
        if (eb != HZ) {
          FrameD d = lds_get(cv.fd + tid);
          d.nz = 1;
          d.base = eb;
          d.nt0 = 0;
          d.S = 2 * SMAX;
          d.NT = (nd + 2 * SMAX + TQ - 1) / TQ;
          lds_put(cv.fd + tid, d);
        }
      }
      __syncthreads();
      if (wave < 3) finalize_task<CM>(I, cv, wave, i, frames, false, err);
      __syncthreads();
      prof_mark(I, cv, PH_FINAL);
      release_rows(I, cv, true, frames, gs, i, err);
      prof_mark(I, cv, PH_CLEAR);
    }
    return;
  }
  if (leader) {
    l_i32 *ccols = (l_i32 *)cv.span;  // column counts of the frames still to clear
    const long long *pend = nullptr;  // the previous index's group frames
    for (int i = 0; i < I.N; ++i) {
      if (tid < NFR) lds_put(cv.fd + tid, late_desc(I, cv, tid, i, err));
      if (pend && wave == 1) {
        // the previous index's group frames, next used by index i+1 (frame
        // generation gs.nbulk + 2), whose early products the followers add
        // in as soon as this clear is published
        for (int f = 0; f < NFR; ++f) {
          long long *fr = const_cast<long long *>(pend) + (size_t)f * WB;
          const int nc = ccols[f];
          for (int c = tid - 64; c < nc; c += 64) st_relaxed(fr + c, 0LL);
        }
        wait_vmem();
        if (tid == 64)
          __hip_atomic_store(I.sync + SY_CLEAR, (uint32_t)(gs.nbulk + 2), __ATOMIC_RELEASE,
                             __HIP_MEMORY_SCOPE_AGENT);
      }
      prof_mark(I, cv, PH_SETUP);
      ++gs.nbulk;
      gs.arrived += (unsigned long long)(I.G - 1);
      if (tid < 64) spin_until_sum(I.sync + SY_ARRIVE, (uint32_t)gs.arrived, err);
      __syncthreads();
      if (I.prof && tid == 0) {
        // from the last arrival to the end of this wait
        const unsigned long long t = wall_clock64();
        const unsigned long long a = __hip_atomic_load(I.prof + PROF_ARRT, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
        if (a != 0 && t > a) atomicAdd(I.prof + PH_ARRLAG, t - a);
        __hip_atomic_store(I.prof + PROF_ARRT, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      prof_mark(I, cv, PH_WAIT);
      const long long *frames = I.gframes + (size_t)(gs.nbulk & 1) * NFR * WB;
      if (wave < 3) finalize_task<CM>(I, cv, wave, i, frames, true, err);
      __syncthreads();
      prof_mark(I, cv, PH_FINAL);
      if (tid < NFR) ccols[tid] = cv.fd[tid].nz ? frame_cols(cv.fd[tid], nd) : 0;
      pend = frames;
      release_rows(I, cv, true, nullptr, gs, i, err);
      prof_mark(I, cv, PH_CLEAR);
    }
    // the last index's frames: the wait before the group's next publication
    // covers these stores
    if (pend) {
      for (int f = 0; f < NFR; ++f) {
        long long *fr = const_cast<long long *>(pend) + (size_t)f * WB;
        const int nc = ccols[f];
        for (int c = tid; c < nc; c += WGS) st_relaxed(fr + c, 0LL);
      }
    }
    __syncthreads();
    return;
  }
  for (int i = 0; i < I.N; ++i) {
    // the digits of this follower's first early term of index i+1 (rows
    // <= i, already published) load while the late products of i run
    MfPrefetch pre;
    bool have_pre = false;
    if ((I.mfma & 1) && i + 1 < I.N && i + 1 >= 2) {
      const int n = i;
      const unsigned W = (unsigned)(I.G - 1), r = (unsigned)(rank - 1);
      const int k0 = 1 + (int)(((unsigned long long)n * r) / W);
      const int k1 = 1 + (int)(((unsigned long long)n * (r + 1)) / W);
      if (k1 > k0) {
        mf_load(pre, row_ptr(I, 0, i + 1 - k0), row_ptr(I, 2, k0), row_ptr(I, 1, k0), nd);
        have_pre = true;
      }
    }
    late_step(I, cv, rank, i, gs);
    if (i + 1 < I.N && i + 1 >= 2) {
      // early part of index j = i+1: Cauchy terms k = 1..j-1 (rows <= i).
      // Fixed descriptors: base SMAX below the first nonzero term, columns
      // for every offset in [0, 2 SMAX] (as the leader finalises them).
      const int j = i + 1;
      if (tid < 2) {
        const int *hv = tid == 0 ? hg : hb;
        const int e = first_esum(ha, hv, j, 1, j - 1);
        FrameSrc fs = mk_frame1(mk_part(PK_CAUCHY, j - 1, j - 1, row_ptr(I, 0, 0),
                                        row_ptr(I, tid == 0 ? 2 : 1, 1), ha, hv + 1));
        fs.fbase = e == HZ ? HZ : e - SMAX;
        lds_put(cv.fs + NFR + tid, fs);
        FrameD d;
        d.n = j - 1;
        d.nz = e != HZ ? 1 : 0;
        d.base = e == HZ ? 0 : e - SMAX;
        d.S = 2 * SMAX;
        d.nt0 = 0;
        d.NT = (nd + 2 * SMAX + TQ - 1) / TQ;
        d.mt0 = 0;
        d.MTf = (nd + TQ - 1) / TQ;
        lds_put(cv.fd + NFR + tid, d);
      }
      __syncthreads();
      prof_mark(I, cv, PH_EBUILD);
      {
        // every term must lie in its frame's window (else the sum is not
        // exact: reported through the error word, no barrier needed); on
        // the matrix cores each follower checks the terms it multiplies
        // (contiguous ranges that cover 1..j-1), else every term is checked
        const int b0 = cv.fd[NFR].base, b1 = cv.fd[NFR + 1].base;
        const l_i32 *la = (const l_i32 *)ha, *lg = (const l_i32 *)hg, *lb = (const l_i32 *)hb;
        int ka = 1, kn = j - 1;
        if (I.mfma & 1) {
          const unsigned W = (unsigned)(I.G - 1), r = (unsigned)(rank - 1);
          ka = 1 + (int)(((unsigned long long)(j - 1) * r) / W);
          kn = 1 + (int)(((unsigned long long)(j - 1) * (r + 1)) / W) - ka;
        }
        for (int t = tid; t < 2 * kn; t += WGS) {
          const int f = t >= kn ? 1 : 0;
          const int k = t - f * kn + ka;
          const int e = esum2(la[j - k], f == 0 ? lg[k] : lb[k]);
          const int base = f == 0 ? b0 : b1;
          if (e != HZ && (e < base || e > base + 2 * SMAX)) atomicOr(err, 1u | 16u);
        }
      }
      prof_mark(I, cv, PH_ESETUP);
      unsigned long long *tp = I.prof && rank == 1 ? I.prof + PH_NPHASE + 9 : nullptr;
      unsigned long long *tmx = (unsigned long long *)(cv.red + 32);
      if (I.mfma & 1)
        mfma_early(I, cv, rank, j, err, have_pre ? &pre : nullptr,
                   I.gframes + (size_t)((gs.nbulk + 1) & 1) * NFR * I.WB, (uint32_t)(gs.nbulk + 1));
      else
        frames_accumulate(cv.fs + NFR, cv.fd + NFR, 2, nd, RS, I.WB, cv.lf, rank, I.G,
                          cv.span + 2 * NFR, true, tp, tmx);
      __syncthreads();
      if (tp && tid == 0) {
        atomicAdd(tp + 2, *tmx);  // slowest thread's products
        *tmx = 0;
      }
      // the early columns go into the group frames of index j now (frame
      // generation gs.nbulk + 1, cleared by the leader once index j-2 was
      // finalised), so that only the late ones wait for rows j
      {
        const unsigned long long B = gs.nbulk + 1;
        if (tid == 0) spin_until(I.sync + SY_CLEAR, (uint32_t)B, err);
        __syncthreads();
        long long *gf = I.gframes + (size_t)(B & 1) * NFR * I.WB;
        l_i32 *es = (l_i32 *)cv.span + 2 * NFR;
        for (int f = 0; f < 2; ++f) {
          const int c0 = es[2 * f], c1 = es[2 * f + 1];
          for (int c = c0 + tid; c < c1; c += WGS) {
            l_i64 *lc = (l_i64 *)cv.lf + (size_t)f * I.WB + c;
            const long long v = *lc;
            if (v != 0) {
              __hip_atomic_fetch_add((unsigned long long *)(gf + (size_t)f * I.WB + c),
                                     (unsigned long long)v, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
              *lc = 0;
            }
          }
        }
        __syncthreads();
        if (tid < 4) es[tid] = 0;
      }
      prof_mark(I, cv, PH_FINAL);
    }
    release_rows(I, cv, false, nullptr, gs, i, err);
    prof_mark(I, cv, PH_CLEAR);
  }
}

// The Horner chains (mode 0) or the adjoint's powers of tau (mode 1) for a
// rational step size: chain c0 + w on wavefront w < nc, the coefficient
// rows c_i staged into LDS by wavefront 3, every operand read once into
// registers.
template <int CM>
__device__ __noinline__ void tau_chains_rational(const Inst &I, const Carve &cv, int count,
                                                 int mode, uint32_t *err, int c0, int nc) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int L = I.L, nd = I.nd, RS = I.RS, N = I.N;
  const TauQ q{I.tau_n, I.tau_m0, I.tau_m1, I.tau_e, I.tau_d};
  const bool rel = I.G > 1;
  const int32_t *rows = I.rows;
  int32_t *qrows = mode == 1 ? q_row(I, 0, 0) : nullptr;
  unsigned long long *prof = (I.prof != nullptr && tid == 0 && blockIdx.x == I.wg0) ? I.prof : nullptr;
  int32_t *const abuf = cv.trow;
  int32_t *const h = cv.hrow + (size_t)(c0 + (wave < nc ? wave : 0)) * RS;
  int32_t *const scratch = (int32_t *)(cv.tcols + (size_t)wave * 64 * I.CM);
  unsigned long long tq = prof ? wall_clock64() : 0;
  auto sub = [&](int slot) {
    if (prof) {
      const unsigned long long t = wall_clock64();
      atomicAdd(prof + slot, t - tq);
      tq = t;
    }
  };
  // coefficient rows c_i (i = N-1-it) into LDS buffer it & 1
  auto stage = [&](int it_, int t0, int tstep) {
    int32_t *dst = abuf + (size_t)(it_ & 1) * nc * RS;
    for (int f = 0; f < nc; ++f) {
      const g_i32 *src = (const g_i32 *)(rows + ((long long)(c0 + f) * (N + 1) + (N - 1 - it_)) * RS);
      for (int w = t0; w < RS; w += tstep) ((l_i32 *)dst)[(size_t)f * RS + w] = src[w];
    }
  };
  if (mode == 0 && count > 0) {
    stage(0, tid, WGS);
    __syncthreads();
  }
  for (int it = 0; it < count; ++it) {
    if (mode == 0 && wave == 3 && it + 1 < count) stage(it + 1, lane, 64);
    if (wave < nc) {
      const int32_t *ad = mode == 0 ? abuf + (size_t)((it & 1) * nc + wave) * RS : nullptr;
      if (!tau_step_rational<CM>(q, L, nd, RS, h, ad, scratch, err, sub) && lane == 0)
        atomicOr(err, 2u);
      if (mode == 1)
        publish_row(h, qrows + ((long long)(c0 + wave) * (N + 1) + it + 1) * RS, RS, rel);
    }
    __syncthreads();
    sub(15);
  }
}

// Three single-workgroup chains at once on the leader: h_c <- round(tau h_c
// + addend_c(i)) for `count` iterations.  h_c starts as the row start_c (an
// LDS row in cv.hrow[c] must already hold it).  Used for the Horner sums of
// equation (2) (addend: coefficient rows) and for the adjoint's powers of tau
// (no addend; each result row is also stored to out rows).
template <int CM>
__device__ __noinline__ void tau_chains(const Inst &I, const Carve &cv, int count, int mode,
                                        uint32_t *err,
                           int c0 = 0, int nc = 3) {
  if (I.tau_d > 0) {
    tau_chains_rational<CM>(I, cv, count, mode, err, c0, nc);
    return;
  }
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int L = I.L, nd = I.nd, RS = I.RS, WB = I.WB, N = I.N;
  const int32_t *tau_lds = cv.hrow + (size_t)3 * RS;
  const bool timed = I.prof != nullptr && tid == 0 && blockIdx.x == I.wg0;
  unsigned long long tq = timed ? wall_clock64() : 0;
  auto sub = [&](int slot) {
    if (timed) {
      unsigned long long t = wall_clock64();
      atomicAdd(I.prof + slot, t - tq);
      tq = t;
    }
  };
  // Horner addends c_i (i = N-1-it) staged in LDS, two buffers of nc rows
  // in the task-row area (free while the chains run): wavefront 3, idle
  // here, loads iteration it+1's rows while iteration it runs
  int32_t *abuf = cv.trow;
  auto stage = [&](int it_, int t0, int tstep) {
    int32_t *dst = abuf + (size_t)(it_ & 1) * nc * RS;
    for (int f = 0; f < nc; ++f) {
      const g_i32 *src = (const g_i32 *)row_ptr(I, c0 + f, N - 1 - it_);
      for (int w = t0; w < RS; w += tstep) ((l_i32 *)dst)[(size_t)f * RS + w] = src[w];
    }
  };
  if (mode == 0 && count > 0) {
    stage(0, tid, WGS);
    __syncthreads();
  }
  for (int it = 0; it < count; ++it) {
    // the previous iteration's rows are complete (its closing barrier)
    lds_products(tau_lds, cv.hrow + (size_t)c0 * RS, RS, nc, nd, WB, cv.lf);
    __syncthreads();
    sub(13);
    if (mode == 0 && wave == 3 && it + 1 < count) stage(it + 1, lane, 64);
    if (wave < nc) {
      const int c = c0 + wave;  // chain of this wavefront; frame `wave`
      const FrameD fdw = single_desc(tau_lds, cv.hrow + (size_t)c * RS, nd);
      RowAdd ad;
      int nad = 0;
      if (mode == 0) {  // Horner: i = N-1-it
        ad = RowAdd{abuf + (size_t)((it & 1) * nc + wave) * RS, 1, 1};
        nad = 1;
      }
      int32_t *h = cv.hrow + (size_t)c * RS;
      int32_t *scratch = (int32_t *)(cv.tcols + (size_t)wave * 64 * I.CM);
      bool ok = sum_to_row<CM>(cv.lf + (size_t)wave * WB, false, &fdw, nd, &ad, nad, 0, L, RS,
                               scratch, h, err);
      if (!ok && lane == 0) atomicOr(err, 2u);
      if (mode == 1) publish_row(h, q_row(I, c, it + 1), RS, I.G > 1);
      int ncol = fdw.nz ? frame_cols(fdw, nd) : 0;
      for (int q = lane; q < ncol; q += 64) ((l_i64 *)cv.lf)[(size_t)wave * WB + q] = 0;
    }
    __syncthreads();
    sub(15);
  }
}

template <int CM>
__device__ __forceinline__ void run_instance(const Inst &I) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int rank = blockIdx.x - I.wg0, G = I.G;
  const bool leader = rank == 0;
  const int L = I.L, N = I.N, nd = I.nd, RS = I.RS, WB = I.WB;
  uint32_t *err = I.sync + SY_ERROR;
  Carve cv = carve(smem, I);
  for (int j = tid; j < NFR * WB; j += WGS) cv.lf[j] = 0;
  GroupSync gs{0u, 0ull};
  red_reset(cv.red);
  const_spans(I, cv);
  if (tid == 0) {
    *cv.tmark = wall_clock64();
    if (I.prof) {
      // where this workgroup runs: XCC and hardware id registers
      unsigned long long *pr = I.prof + 2 * PH_NPHASE + rank * PROF_RANK;
      pr[4] = (unsigned)__builtin_amdgcn_s_getreg((3 << 11) | 20);
      pr[5] = (unsigned)__builtin_amdgcn_s_getreg((31 << 11) | 4);
    }
  }
  if (leader) {
    for (int c = wave; c < NCONST; c += 4)
      write_row(I.cnorm + (size_t)c * (L + 2), L, nd, RS, I.consts + (size_t)c * RS, G > 1, lane,
                64);
  }
  __syncthreads();
  late_geometry(I, cv);
  if (tid < 4 * NFR) cv.span[tid] = 0;
  if (tid == 0) *(unsigned long long *)(cv.red + 32) = 0;
  __syncthreads();

  for (long long step = 0; step < I.nsteps; ++step) {
    if (leader && wave < 3) {
      const int32_t *sv = I.state + (size_t)wave * (L + 2);
      if (step == 0 && I.ckpt) copy_norm(sv, I.ckpt + (size_t)wave * (L + 2), L, false, lane, 64);
      if (I.coefs) copy_norm(sv, I.coefs + (size_t)wave * (N + 1) * (L + 2), L, false, lane, 64);
    }
    // with three or more workgroups the Horner chains of the previous step
    // have already written rows 0
    start_step(I, cv, leader, I.state, gs, err, G >= 3 && step > 0);
    prof_mark(I, cv, PH_STEP0);
    forward_coefficients<CM>(I, cv, rank, gs, I.state, err);
    if (I.mode == MODE_COEFFS) break;
    // Horner (equation (2)): h = c_N; h <- round(h tau + c_i), i = N-1..0
    if (G >= 3) {
      // chain c on workgroup c; it writes row 0 of the next step and the state
      if (rank < 3) {
        const int c = rank;
        int32_t *h = cv.hrow + (size_t)c * RS;
        for (int j = tid; j < RS; j += WGS) {
          h[j] = row_ptr(I, c, N)[j];
          cv.hrow[(size_t)3 * RS + j] = (I.consts + (size_t)C_TAU * RS)[j];
        }
        __syncthreads();
        tau_chains<CM>(I, cv, N, 0, err, c, 1);
        if (wave == 0) {
          publish_row(h, row_ptr(I, c, 0), RS, true);
          int32_t *scratch = (int32_t *)cv.tcols;
          int32_t *hn = scratch + 64 * I.CM;
          row_to_norm<CM>(h, L, nd, scratch, hn);
          copy_norm(hn, I.state + (size_t)c * (L + 2), L, true, lane, 64);
          if (I.ckpt)
            copy_norm(hn, I.ckpt + ((size_t)(step + 1) * 3 + c) * (L + 2), L, true, lane, 64);
        }
        wait_vmem();
        __syncthreads();
        if (tid == 0)
          __hip_atomic_fetch_add(I.sync + SY_HDONE, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (tid == 0) spin_until(I.sync + SY_HDONE, (uint32_t)(3 * (step + 1)), err, rank >= 3);
      __syncthreads();
      prof_mark(I, cv, PH_HORNER);
    } else if (leader) {
      for (int j = tid; j < 4 * RS; j += WGS) {
        int c = j / RS, w = j - c * RS;
        cv.hrow[j] = c < 3 ? row_ptr(I, c, N)[w] : (I.consts + (size_t)C_TAU * RS)[w];
      }
      __syncthreads();
      tau_chains<CM>(I, cv, N, 0, err);
      if (wave < 3) {
        int32_t *scratch = (int32_t *)(cv.tcols + (size_t)wave * 64 * I.CM);
        int32_t *h = scratch + 64 * I.CM;
        row_to_norm<CM>(cv.hrow + (size_t)wave * RS, L, nd, scratch, h);
        copy_norm(h, I.state + (size_t)wave * (L + 2), L, false, lane, 64);
        if (I.ckpt)
          copy_norm(h, I.ckpt + ((size_t)(step + 1) * 3 + wave) * (L + 2), L, false, lane, 64);
      }
      __syncthreads();
      prof_mark(I, cv, PH_HORNER);
    }
  }
}

// Every workgroup runs the instance wg_inst[blockIdx.x], then the ones
// chained after it on the same workgroups (a batch may run several
// trajectories one after another on one group).
template <int CM>
__global__ void __launch_bounds__(WGS) k_run(const Inst *__restrict__ insts,
                                             const int *__restrict__ wg_inst) {
  for (int q = wg_inst[blockIdx.x]; q >= 0;) {
    const Inst I = insts[q];
    run_instance<CM>(I);
    q = I.next - 1;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Polynomial vector fields of degree at most two.  Every product term of a
// right-hand side contributes a Cauchy-product sum of the kind equation (3)
// holds for the Lorenz system (Section 2, the paragraph on automatic
// differentiation): with x_{v,0} the state, for i = 0..N-1
//   S_q       = round(sum_{k=0}^{i} x_{u_q,i-k} x_{w_q,k})            (each pair q)
//   x_{v,i+1} = round(([i=0] c_v + sum A_vu x_{u,i} + sum B_vq S_q) / (i+1))
// then the Horner sums of equation (2).  One workgroup integrates one
// trajectory (a launch runs a batch), with the frames of an index in LDS:
// the Cauchy frames of all pairs in one pass of the product tiles, each
// rounded by one wavefront, then the numerator frames (constants times
// rows) in a second pass, each divided and rounded by one wavefront.

// LDS carve of one workgroup of k_poly.
struct PolyCarve {
  long long *lf;     // NFR * WB frame columns
  FrameSrc *fs;      // NFR
  FrameD *fd;        // NFR
  int *red;          // 2 NFR (frame_setup's reduction)
  int *span;         // 2 NFR
  int8_t *offs;      // maxn bytes: per-term offset tables
  long long *scr;    // 4 wavefronts x 64 CM words of task scratch
  int32_t *cur;      // V rows: x_{v,i} (the Horner accumulators after the index loop)
  int32_t *srow;     // Q rows: S_q
  int32_t *orow;     // V rows: x_{v,i+1}
  int32_t *crow;     // V rows: the constant term c_v (zero row: none)
  int32_t *hb;       // 2 V rows: Horner addends; then the tau row
};

__host__ __device__ inline size_t poly_carve(int V, int Q, int RS, int WB, int CM, int maxn,
                                             unsigned char *base, PolyCarve *cv) {
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += (bytes + 15) & ~(size_t)15;
    return base ? base + at : nullptr;
  };
  PolyCarve c;
  c.lf = (long long *)take((size_t)NFR * WB * 8);
  c.fs = (FrameSrc *)take(sizeof(FrameSrc) * NFR);
  c.fd = (FrameD *)take(sizeof(FrameD) * NFR);
  c.red = (int *)take(2 * NFR * 4);
  c.span = (int *)take(2 * NFR * 4);
  c.offs = (int8_t *)take((size_t)maxn);
  c.scr = (long long *)take((size_t)4 * 64 * CM * 8);
  c.cur = (int32_t *)take((size_t)V * RS * 4);
  c.srow = (int32_t *)take((size_t)(Q > 0 ? Q : 1) * RS * 4);
  c.orow = (int32_t *)take((size_t)V * RS * 4);
  c.crow = (int32_t *)take((size_t)V * RS * 4);
  c.hb = (int32_t *)take((size_t)(2 * V + 1) * RS * 4);
  if (cv) *cv = c;
  return o;
}

__device__ __forceinline__ int32_t *poly_row(const PolyInst &P, int v, int i) {
  return P.rows + ((long long)v * (P.N + 1) + i) * P.RS;
}

// Operand o of index i in global memory (rows, or the published sums).
__device__ __forceinline__ const int32_t *poly_opnd(const PolyInst &P, int o, int i) {
  return o < P.V ? poly_row(P, o, i) : P.sums + (long long)(o - P.V) * P.RS;
}

// Copy a row (RS words) between LDS and global memory by `nthr` threads.
__device__ __forceinline__ void poly_copy(const int32_t *src, int32_t *dst, int RS, int t, int nthr) {
  for (int w = t; w < RS; w += nthr) dst[w] = src[w];
}

// Round the frame lf[f] (descriptor fd[f], row addends ad) into the LDS row
// out (div: divide by it first; 0: none) and clear the frame's columns.
// Single wavefront.
template <int CM>
__device__ __forceinline__ void poly_task(const PolyInst &P, const PolyCarve &cv, int f,
                                          const RowAdd *ad, int nad, int div, int32_t *out) {
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  int32_t *scratch = (int32_t *)(cv.scr + (size_t)wave * 64 * CM);
  const FrameD d = lds_get(cv.fd + f);
  if (!sum_to_row<CM>(cv.lf + (size_t)f * P.WB, false, &d, P.nd, ad, nad, div, P.L, P.RS, scratch,
                      out, P.err) &&
      lane == 0)
    atomicOr(P.err, 2u);
  const int ncol = d.nz ? frame_cols(d, P.nd) : 0;
  for (int c = lane; c < ncol; c += 64) ((l_i64 *)cv.lf)[(size_t)f * P.WB + c] = 0;
}

template <int CM>
__global__ void __launch_bounds__(WGS) k_poly(const PolyInst *__restrict__ insts) {
  extern __shared__ __align__(16) unsigned char smem[];
  const PolyInst P = insts[blockIdx.x];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int L = P.L, N = P.N, nd = P.nd, RS = P.RS, WB = P.WB, V = P.V, Q = P.Q;
  PolyCarve cv;
  (void)poly_carve(V, Q, RS, WB, CM, P.maxn, smem, &cv);
  for (int j = tid; j < NFR * WB; j += WGS) cv.lf[j] = 0;
  red_reset(cv.red);
  // constants as rows (global), the constant terms and the state as LDS rows
  for (int c = 0; c < P.nconst; ++c)
    write_row(P.cnorm + (size_t)c * (L + 2), L, nd, RS, P.consts + (size_t)c * RS, false, tid, WGS);
  for (int v = 0; v < V; ++v) {
    if (P.cc[v] >= 0)
      write_row(P.cnorm + (size_t)P.cc[v] * (L + 2), L, nd, RS, cv.crow + (size_t)v * RS, false,
                tid, WGS);
    else
      for (int w = tid; w < RS; w += WGS) cv.crow[(size_t)v * RS + w] = 0;
    write_row(P.state + (size_t)v * (L + 2), L, nd, RS, cv.cur + (size_t)v * RS, false, tid, WGS);
  }
  __syncthreads();
  const TauQ tq{P.tau_n, P.tau_m0, P.tau_m1, P.tau_e, P.tau_d};
  auto nomark = [](int) {};
  for (long long step = 0; step < P.nsteps; ++step) {
    // the state rows x_{v,0}
    for (int w = tid; w < V * RS; w += WGS) {
      const int v = w / RS, k = w - v * RS;
      poly_row(P, v, 0)[k] = cv.cur[w];
    }
    if (P.coefs && step == 0 && wave < V) {
      int32_t *scratch = (int32_t *)(cv.scr + (size_t)wave * 64 * CM);
      int32_t *nv = scratch + 64 * CM;
      row_to_norm<CM>(cv.cur + (size_t)wave * RS, L, nd, scratch, nv);
      copy_norm(nv, P.coefs + (size_t)wave * (N + 1) * (L + 2), L, false, lane, 64);
    }
    wait_vmem();
    __syncthreads();
    for (int i = 0; i < N; ++i) {
      // Cauchy sums of the pairs
      if (Q > 0) {
        if (tid == 0)
          for (int q = 0; q < Q; ++q)
            lds_put(cv.fs + q, mk_frame1(mk_part(PK_CAUCHY, i + 1, i, poly_row(P, P.pu[q], 0),
                                                 poly_row(P, P.pw[q], 0))));
        __syncthreads();
        frame_setup(cv.fs, cv.fd, Q, nd, RS, cv.red, cv.offs, P.maxn, P.err);
        frames_accumulate(cv.fs, cv.fd, Q, nd, RS, WB, cv.lf, 0, 1, cv.span);
        __syncthreads();
        for (int q = wave; q < Q; q += 4) {
          poly_task<CM>(P, cv, q, nullptr, 0, 0, cv.srow + (size_t)q * RS);
          poly_copy(cv.srow + (size_t)q * RS, P.sums + (size_t)q * RS, RS, lane, 64);
        }
        wait_vmem();
        __syncthreads();
      }
      // numerators: constants times operands in one frame per equation
      if (tid == 0)
        for (int v = 0; v < V; ++v) {
          FrameSrc f;
          FramePart pt[PMAXP];
          for (int j = 0; j < PMAXP; ++j)
            pt[j] = j < P.np[v] ? mk_part(PK_ONE, 1, 0, P.consts + (size_t)P.cp[v][j] * RS,
                                          poly_opnd(P, P.op[v][j], i))
                                : mk_part(PK_ONE, 0, 0, P.consts, P.consts);
          f = mk_frame4(pt[0], pt[1], pt[2], pt[3]);
          f.nparts = P.np[v];
          f.n = P.np[v];
          lds_put(cv.fs + v, f);
        }
      __syncthreads();
      frame_setup(cv.fs, cv.fd, V, nd, RS, cv.red, cv.offs, P.maxn, P.err);
      frames_accumulate(cv.fs, cv.fd, V, nd, RS, WB, cv.lf, 0, 1, cv.span);
      __syncthreads();
      for (int v = wave; v < V; v += 4) {
        RowAdd ad[PMAXA];
        int nad = 0;
        for (int k = 0; k < P.na[v]; ++k) {
          const int o = P.ao[v][k];
          ad[nad++] = RowAdd{o < V ? cv.cur + (size_t)o * RS : cv.srow + (size_t)(o - V) * RS,
                             P.asg[v][k], 1};
        }
        if (i == 0 && P.cc[v] >= 0 && nad < PMAXA) ad[nad++] = RowAdd{cv.crow + (size_t)v * RS, 1, 1};
        poly_task<CM>(P, cv, v, ad, nad, i + 1, cv.orow + (size_t)v * RS);
      }
      __syncthreads();
      // the new rows x_{v,i+1}: global memory and the current rows
      for (int w = tid; w < V * RS; w += WGS) {
        const int v = w / RS, k = w - v * RS;
        const int32_t x = cv.orow[w];
        poly_row(P, v, i + 1)[k] = x;
        cv.cur[w] = x;
      }
      if (P.coefs && step == 0 && wave < V) {
        int32_t *scratch = (int32_t *)(cv.scr + (size_t)wave * 64 * CM);
        int32_t *nv = scratch + 64 * CM;
        row_to_norm<CM>(cv.orow + (size_t)wave * RS, L, nd, scratch, nv);
        copy_norm(nv, P.coefs + ((size_t)wave * (N + 1) + i + 1) * (L + 2), L, false, lane, 64);
      }
      wait_vmem();
      __syncthreads();
    }
    // Horner (equation (2)): h_v = x_{v,N}; h_v <- round(tau h_v + x_{v,i}), i = N-1..0
    if (P.tau_d > 0) {
      // one chain per wavefront, the next addend row loaded while a step runs
      if (wave < V) {
        int32_t *h = cv.cur + (size_t)wave * RS;
        int32_t *hb = cv.hb + (size_t)wave * 2 * RS;
        int32_t *scratch = (int32_t *)(cv.scr + (size_t)wave * 64 * CM);
        constexpr int PRE = 16;  // RS <= 64 PRE words per row
        int32_t pre[PRE];
        auto load = [&](int idx) {
          const int32_t *src = poly_row(P, wave, idx);
#pragma unroll
          for (int j = 0; j < PRE; ++j) {
            const int w = lane + 64 * j;
            pre[j] = w < RS ? src[w] : 0;
          }
        };
        auto store = [&](int32_t *dst) {
#pragma unroll
          for (int j = 0; j < PRE; ++j) {
            const int w = lane + 64 * j;
            if (w < RS) dst[w] = pre[j];
          }
        };
        if (N > 0) {
          load(N - 1);
          store(hb);
        }
        for (int it = 0; it < N; ++it) {
          int32_t *cur_add = hb + (size_t)(it & 1) * RS;
          if (it + 1 < N) load(N - 2 - it);
          __builtin_amdgcn_wave_barrier();
          if (!tau_step_rational<CM>(tq, L, nd, RS, h, cur_add, scratch, P.err, nomark) && lane == 0)
            atomicOr(P.err, 2u);
          if (it + 1 < N) store(hb + (size_t)((it + 1) & 1) * RS);
          __builtin_amdgcn_wave_barrier();
        }
      }
      __syncthreads();
    } else {
      int32_t *tau_lds = cv.hb + (size_t)2 * V * RS;
      for (int w = tid; w < RS; w += WGS) tau_lds[w] = P.consts[(size_t)P.ctau * RS + w];
      __syncthreads();
      for (int it = 0; it < N; ++it) {
        for (int w = tid; w < V * RS; w += WGS) {
          const int v = w / RS, k = w - v * RS;
          cv.hb[w] = poly_row(P, v, N - 1 - it)[k];
        }
        lds_products(tau_lds, cv.cur, RS, V, nd, WB, cv.lf);
        __syncthreads();
        if (wave < V) {
          int32_t *h = cv.cur + (size_t)wave * RS;
          const FrameD fdw = single_desc(tau_lds, h, nd);
          const RowAdd ad{cv.hb + (size_t)wave * RS, 1, 1};
          int32_t *scratch = (int32_t *)(cv.scr + (size_t)wave * 64 * CM);
          if (!sum_to_row<CM>(cv.lf + (size_t)wave * WB, false, &fdw, nd, &ad, 1, 0, L, RS, scratch,
                              h, P.err) &&
              lane == 0)
            atomicOr(P.err, 2u);
          const int ncol = fdw.nz ? frame_cols(fdw, nd) : 0;
          for (int c = lane; c < ncol; c += 64) ((l_i64 *)cv.lf)[(size_t)wave * WB + c] = 0;
        }
        __syncthreads();
      }
    }
  }
  // the final state, normalised
  if (wave < V) {
    int32_t *scratch = (int32_t *)(cv.scr + (size_t)wave * 64 * CM);
    int32_t *nv = scratch + 64 * CM;
    row_to_norm<CM>(cv.cur + (size_t)wave * RS, L, nd, scratch, nv);
    copy_norm(nv, P.state + (size_t)wave * (L + 2), L, false, lane, 64);
  }
}

#if MPTS_CM == 4
size_t poly_lds_bytes(int V, int Q, int RS, int WB, int CM, int maxn) {
  return poly_carve(V, Q, RS, WB, CM, maxn, nullptr, nullptr);
}
#endif

// ---------------------------------------------------------------------------
// Adjoint: reverse sweep over the steps of a checkpointed forward run.
//
// For step n (from the last to the first), with incoming adjoints X, Y, Z of
// the step's end state, the coefficients a, b, g are recomputed from the
// checkpoint (the same code as the forward run, hence the same bits), the
// powers q^c_i = round(q^c_{i-1} tau) of each adjoint are formed (the
// derivative of the Horner sum of equation (2) with respect to c_i is
// tau^i), and the recursion of equation (3) is differentiated backwards:
// for m = N..0
//   abar_m = round(qx_m + sum_{j=m}^{N-1} (-v_j g_{j-m} + w_j b_{j-m}) - sigma u_m + R v_m)
//   bbar_m = round(qy_m + sum_{j=m}^{N-1} w_j a_{j-m} + sigma u_m - v_m)
//   gbar_m = round(qz_m - sum_{j=m}^{N-1} v_j a_{j-m} - b w_m)
//   u_{m-1} = round(abar_m / m), v_{m-1} = round(bbar_m / m), w_{m-1} = round(gbar_m / m)
// (terms with u_m, v_m, w_m only for m < N).  The gathers are correlation
// frames over the stored rows u, v, w and their negations nu, nv, nw.  The
// parameter derivatives of the step are the dot products
//   dsigma = sum u_i b_i + sum nu_i a_i, dR = sum v_i a_i, db = sum nw_i g_i,
// each added into its running adjoint with one rounding.
template <int CM>
__global__ void __launch_bounds__(WGS) k_adj(const Inst *__restrict__ insts,
                                             const int *__restrict__ wg_inst) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const Inst I = insts[wg_inst[blockIdx.x]];
  const int rank = blockIdx.x - I.wg0, G = I.G;
  const bool leader = rank == 0;
  const int L = I.L, N = I.N, nd = I.nd, RS = I.RS, WB = I.WB;
  uint32_t *err = I.sync + SY_ERROR;
  Carve cv = carve(smem, I);
  for (int j = tid; j < NFR * WB; j += WGS) cv.lf[j] = 0;
  GroupSync gs{0u, 0ull};
  const bool rel = G > 1;
  red_reset(cv.red);
  const_spans(I, cv);
  if (tid == 0) *cv.tmark = wall_clock64();
  if (leader) {
    for (int c = wave; c < NCONST; c += 4)
      write_row(I.cnorm + (size_t)c * (L + 2), L, nd, RS, I.consts + (size_t)c * RS, rel, lane, 64);
    // seed: the adjoint of ||x(T)||^2 is 2 x(T), that of one component of
    // x(T) the unit vector (both exact); parameter adjoints 0
    if (wave < 3) {
      int32_t *b = bar_ptr(I, wave);
      if (I.loss == 0) {
        const int32_t *xT = I.ckpt + ((size_t)I.nsteps * 3 + wave) * (L + 2);
        for (int j = lane; j < L + 2; j += 64) b[j] = (j == 1 && xT[0] != 0) ? xT[1] + 1 : xT[j];
      } else {
        const int32_t *one = I.cnorm + (size_t)C_ONE * (L + 2);
        const bool unit = wave == I.loss - 1;
        for (int j = lane; j < L + 2; j += 64) b[j] = unit ? one[j] : 0;
      }
      int32_t *pb = bar_ptr(I, 3 + wave);
      for (int j = lane; j < L + 2; j += 64) pb[j] = 0;
    }
  }
  __syncthreads();
  late_geometry(I, cv);
  if (tid < 4 * NFR) cv.span[tid] = 0;
  __syncthreads();
  const int32_t *cs = I.consts;
  for (long long n = I.nsteps - 1; n >= 0; --n) {
    // 1. the step's coefficients from its checkpoint
    start_step(I, cv, leader, I.ckpt + (size_t)n * 3 * (L + 2), gs, err);
    forward_coefficients<CM>(I, cv, rank, gs, I.ckpt + (size_t)n * 3 * (L + 2), err);
    // 2. q^c_0 = incoming adjoint, q^c_i = round(q^c_{i-1} tau)
    if (leader) {
      if (wave < 3) {
        write_row(bar_ptr(I, wave), L, nd, RS, q_row(I, wave, 0), rel, lane, 64);
        write_row(bar_ptr(I, wave), L, nd, RS, cv.hrow + (size_t)wave * RS, false, lane, 64);
      } else {
        for (int j = lane; j < RS; j += 64) cv.hrow[(size_t)3 * RS + j] = cs[(size_t)C_TAU * RS + j];
      }
      __syncthreads();
      tau_chains<CM>(I, cv, N, 1, err);
    }
    group_publish(I, leader, gs, err);
    // 3. reverse sweep over the coefficient index
    for (int m = N; m >= 0; --m) {
      if (tid == 0) {
        const int k = N - m;          // terms of each gather
        const int one = m < N ? 1 : 0;
        const int mi = m < N ? m : 0;
        FrameSrc *fs = cv.fs;
        const int *ha = hc_row(I, cv, 0), *hb = hc_row(I, cv, 1), *hg = hc_row(I, cv, 2);
        fs[0] = mk_frame4(
            mk_part(PK_CORR, k, m, adj_row(I, A_NV, 0), row_ptr(I, 2, 0), nullptr, hg),
            mk_part(PK_CORR, k, m, adj_row(I, A_W, 0), row_ptr(I, 1, 0), nullptr, hb),
            mk_part(PK_ONE, one, 0, cs + (size_t)C_NSIGMA * RS, adj_row(I, A_U, mi),
                    hc_const(I, cv, C_NSIGMA), nullptr),
            mk_part(PK_ONE, one, 0, cs + (size_t)C_R * RS, adj_row(I, A_V, mi),
                    hc_const(I, cv, C_R), nullptr));
        fs[1] = mk_frame2(
            mk_part(PK_CORR, k, m, adj_row(I, A_W, 0), row_ptr(I, 0, 0), nullptr, ha),
            mk_part(PK_ONE, one, 0, cs + (size_t)C_SIGMA * RS, adj_row(I, A_U, mi),
                    hc_const(I, cv, C_SIGMA), nullptr));
        fs[2] = mk_frame2(
            mk_part(PK_CORR, k, m, adj_row(I, A_NV, 0), row_ptr(I, 0, 0), nullptr, ha),
            mk_part(PK_ONE, one, 0, cs + (size_t)C_NB * RS, adj_row(I, A_W, mi),
                    hc_const(I, cv, C_NB), nullptr));
      }
      __syncthreads();
      const long long *frames = group_bulk(I, cv, 3, rank, gs, err);
      if (leader && wave < 3) {
        int32_t *dig = (int32_t *)(cv.tcols + (size_t)wave * 64 * I.CM);
        int32_t *q = dig + 64 * I.CM;
        int32_t *res = cv.tnorm + (size_t)wave * 2 * cv.NV;
        int32_t *out = res + cv.NV;
        Addend ad[2];
        int nad = 1;
        ad[0] = Addend{q_row(I, wave, m), 1, 1, 0};
        if (wave == 1 && m < N) {
          ad[1] = Addend{adj_row(I, A_NV, m), 1, 1, 0};
          nad = 2;
        }
        int C;
        long long dexp;
        int sgn = combine_resolve<CM>(frames + (size_t)wave * WB, rel, &cv.fd[wave], nd, L, ad, nad,
                                      dig, &C, &dexp, err);
        bool ok = wave_round(dig, C, sgn, dexp, false, L, res);
        if (m > 0) {
          Addend a1 = Addend{res, 0, 1, 1};
          sgn = combine_resolve<CM>(nullptr, false, nullptr, nd, L, &a1, 1, dig, &C, &dexp, err);
          ok &= wave_div_round<CM>(dig, C, sgn, dexp, m, L, nd, q, out);
          // wave 0 -> u, 1 -> v, 2 -> w, with their negations
          write_row(out, L, nd, RS, adj_row(I, A_U + wave, m - 1), rel, lane, 64);
          write_row(out, L, nd, RS, adj_row(I, A_NU + wave, m - 1), rel, lane, 64, true);
        } else {
          copy_norm(res, bar_ptr(I, wave), L, false, lane, 64);
        }
        if (!ok && lane == 0) atomicOr(err, 2u);
      }
      group_release(I, cv, 3, leader, frames, gs, err);
    }
    // 4. parameter derivatives of this step, one rounded add each
    if (tid == 0) {
      FrameSrc *fs = cv.fs;
      const int *ha = hc_row(I, cv, 0), *hb = hc_row(I, cv, 1), *hg = hc_row(I, cv, 2);
      fs[0] = mk_frame2(mk_part(PK_DOT, N, 0, adj_row(I, A_U, 0), row_ptr(I, 1, 0), nullptr, hb),
                        mk_part(PK_DOT, N, 0, adj_row(I, A_NU, 0), row_ptr(I, 0, 0), nullptr, ha));
      fs[1] = mk_frame1(mk_part(PK_DOT, N, 0, adj_row(I, A_V, 0), row_ptr(I, 0, 0), nullptr, ha));
      fs[2] = mk_frame1(mk_part(PK_DOT, N, 0, adj_row(I, A_NW, 0), row_ptr(I, 2, 0), nullptr, hg));
    }
    __syncthreads();
    const long long *frames = group_bulk(I, cv, 3, rank, gs, err);
    if (leader && wave < 3) {
      int32_t *dig = (int32_t *)(cv.tcols + (size_t)wave * 64 * I.CM);
      int32_t *res = cv.tnorm + (size_t)wave * 2 * cv.NV;
      Addend ad = Addend{bar_ptr(I, 3 + wave), 0, 1, 0};
      int C;
      long long dexp;
      int sgn = combine_resolve<CM>(frames + (size_t)wave * WB, rel, &cv.fd[wave], nd, L, &ad, 1,
                                    dig, &C, &dexp, err);
      bool ok = wave_round(dig, C, sgn, dexp, false, L, res);
      if (!ok && lane == 0) atomicOr(err, 2u);
      copy_norm(res, bar_ptr(I, 3 + wave), L, false, lane, 64);
    }
    group_release(I, cv, 3, leader, frames, gs, err);
  }
}

// ---------------------------------------------------------------------------
// Launchers.  This file is compiled once per finalisation chunk size
// (MPTS_CM = 4, 8, 16 or 32, the largest digit chunk a lane holds), so the
// kernel instances build in parallel; mpts_dispatch.cpp picks the instance.
#ifndef MPTS_CM
#error "compile with -DMPTS_CM=4, 8, 16 or 32"
#endif
#define MPTS_CAT2(a, b) a##b
#define MPTS_CAT(a, b) MPTS_CAT2(a, b)

namespace MPTS_CAT(cm, MPTS_CM) {

hipError_t launch_run(const Inst *d_insts, const int *d_wg_inst, int nwg, size_t lds, hipStream_t s,
                      bool cooperative) {
  auto kern = k_run<MPTS_CM>;
  hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  if (cooperative) {
    void *args[] = {(void *)&d_insts, (void *)&d_wg_inst};
    return hipLaunchCooperativeKernel((const void *)kern, dim3(nwg), dim3(WGS), args,
                                      (unsigned)lds, s);
  }
  hipLaunchKernelGGL(kern, dim3(nwg), dim3(WGS), lds, s, d_insts, d_wg_inst);
  return hipGetLastError();
}

hipError_t launch_adj(const Inst *d_insts, const int *d_wg_inst, int nwg, size_t lds, hipStream_t s) {
  auto kern = k_adj<MPTS_CM>;
  hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  void *args[] = {(void *)&d_insts, (void *)&d_wg_inst};
  return hipLaunchCooperativeKernel((const void *)kern, dim3(nwg), dim3(WGS), args, (unsigned)lds,
                                    s);
}

hipError_t launch_poly(const PolyInst *d_insts, int count, size_t lds, hipStream_t s) {
  auto kern = k_poly<MPTS_CM>;
  hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(count), dim3(WGS), lds, s, d_insts);
  return hipGetLastError();
}

hipError_t set_lds(size_t lds, bool adjoint) {
  const void *k = adjoint ? (const void *)k_adj<MPTS_CM> : (const void *)k_run<MPTS_CM>;
  return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t occupancy(int *nb, size_t lds, bool adjoint) {
  if (adjoint) return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, k_adj<MPTS_CM>, WGS, lds);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, k_run<MPTS_CM>, WGS, lds);
}

}  // namespace cmN

#if MPTS_CM == 4
__global__ void k_clear(uint32_t *p, size_t nwords) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < nwords; i += stride) p[i] = 0u;
}

hipError_t launch_clear(void *p, size_t bytes, hipStream_t s) {
  size_t words = bytes / 4;
  int blocks = (int)((words + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_clear, dim3(blocks), dim3(256), 0, s, (uint32_t *)p, words);
  return hipGetLastError();
}
#endif

}  // namespace mpts
