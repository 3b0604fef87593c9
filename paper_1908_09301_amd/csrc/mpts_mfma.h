// Exact Cauchy-product sums on the int8 matrix cores (MFMA).
//
// A Cauchy sum sum_k U_k V_k (U_k = a_{i-k}, V_k = g_k or b_k, equation (3))
// is a sum of digit convolutions.  Here every row is re-split into 7-bit
// pieces: a 28-bit row digit D = s |D| (all digits of a row carry the row's
// sign s) is s (p0 + p1 2^7 + p2 2^14 + p3 2^21) with p_q in [0, 127], so the
// signed pieces s p_q fit int8 and a product of two pieces fits 15 bits.
// A row of nd digits is NP = 4 nd pieces; the row exponent (28-bit units) is
// 4x as many piece units, so the term offsets stay whole pieces.
//
// The convolution of pieces is cast as a matrix product by cutting the
// output position pi = 32 R + t into an output block R and a row t, and the
// U piece index x = 32 m + t - s into a U block m and an inner index s:
//   O[t][R] = sum_k sum_m sum_{s<32} W_k[t][(m,s)] X_k[(m,s)][R],
//   W_k[t][(m,s)] = U_k[32 m + t - s]                 (Toeplitz in t - s),
//   X_k[(m,s)][R] = V_k[32 (R - m) + s - 4 off_k]     (V shifted by its offset),
// which is v_mfma_i32_32x32x32_i8 with M = 32 (t), N = 32 (R of one output
// tile), K = 32 (s) per U block m and term.  Every output position
// then holds an exact int32 sum of piece products (no Toeplitz redundancy
// on the output side); the i32 accumulators are flushed into the frame's
// 64-bit columns (28-bit weights) before they can overflow.
//
// One workgroup takes a contiguous range of terms of the two Cauchy frames
// of an index (they share U_k = a_{i-k}); for each term it stages the three
// rows as pieces in LDS, and its four wavefronts split the (m, output tile)
// pairs, each holding the accumulators of both frames for its pairs.
#pragma once
#include <hip/hip_runtime.h>
#include "mpts_common.h"
#include "mpts_rows.h"

namespace mpts {

typedef __attribute__((address_space(3))) uint8_t l_u8;
typedef __attribute__((address_space(3))) uint32_t l_u32;
typedef int mf_v16i __attribute__((ext_vector_type(16)));

constexpr int MF_OFFP = 4 * 2 * SMAX;  // largest term offset in pieces
constexpr int MF_VLO = 1120;           // V pieces below 0 that a read can reach (35 blocks)
constexpr int MF_NTMAX = 4;            // output tiles of 1024 pieces held per wavefront

// Piece geometry for rows of nd digits.  The U row is stored reversed
// (piece x at byte ZU - x); a V row in blocks of 32 pieces at a stride of 36
// bytes (so that the 32 lanes of a read, one block each, hit 32 different
// LDS banks), logical piece P at block (P + MF_VLO) / 32.
struct MfGeo {
  int NP;   // pieces per row
  int MM;   // U blocks m = 0..MM-1 that can hold a piece
  int NT;   // output tiles (1024 pieces each) that can hold a nonzero sum
  int DQH;  // largest 32 q - m whose V blocks can hold a piece
  int ZU;   // byte of U piece 0 in its buffer (ZU = 3 mod 4)
  int UBs;  // bytes of the U buffer
  int VBLK; // 36-byte blocks of a V buffer
  int VBs;  // bytes of a V buffer
  int BUF;  // bytes of one staging buffer: U, V0, V1
  int FT;   // terms between flushes of the i32 accumulators
};

__host__ __device__ inline MfGeo mf_geo(int nd) {
  MfGeo g;
  g.NP = 4 * nd;
  g.MM = (g.NP + 30) / 32 + 1;
  g.NT = (2 * g.NP + MF_OFFP) / 1024 + 1;
  g.DQH = (g.NP + MF_OFFP - 1) / 32;
  g.ZU = 4 * ((g.NP + 61 + 3) / 4) + 3;
  g.UBs = (g.ZU + 32 + 15) & ~15;
  // logical pieces [-MF_VLO, NP + MF_OFFP + 1056) in 32-piece blocks
  g.VBLK = (MF_VLO + g.NP + MF_OFFP + 1056 + 31) / 32;
  g.VBs = (36 * g.VBLK + 15) & ~15;
  g.BUF = g.UBs + 2 * g.VBs;
  // one term adds at most NP products of magnitude <= 127^2 to an output
  const long long per_term = (long long)g.NP * 127 * 127;
  long long ft = per_term > 0 ? 2147483647LL / per_term : 1;
  g.FT = (int)(ft < 1 ? 1 : ft > 4096 ? 4096 : ft);
  return g;
}

// Staging bytes (two buffers) the MFMA path needs in LDS.
__host__ __device__ inline int mf_stage_bytes(int nd) { return 2 * mf_geo(nd).BUF; }

// Whether the MFMA path holds this size (all output tiles in one wavefront's
// accumulators).
__host__ __device__ inline bool mf_fits(int nd) { return mf_geo(nd).NT <= MF_NTMAX; }

// The four pieces s p0..s p3 of a 28-bit digit D, packed little-endian
// (forward = true: p0 in the low byte) or reversed (p3 in the low byte).
__device__ __forceinline__ uint32_t mf_pieces(int32_t D, bool forward) {
  const uint32_t M = (uint32_t)(D < 0 ? -D : D);
  uint32_t p[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int v = (int)((M >> (7 * q)) & 127u);
    p[q] = (uint32_t)(uint8_t)(int8_t)(D < 0 ? -v : v);
  }
  return forward ? (p[0] | (p[1] << 8) | (p[2] << 16) | (p[3] << 24))
                 : (p[3] | (p[2] << 8) | (p[1] << 16) | (p[0] << 24));
}

// Byte address in a V buffer of logical piece P (a multiple of 4 or the
// start of an 8-byte read at s0 + 8h within a block).
__device__ __forceinline__ int mf_vaddr(int P) {
  const int b = P + MF_VLO;
  return 36 * (b >> 5) + (b & 31);
}

// Zero both staging buffers (every thread of the workgroup).
__device__ __forceinline__ void mf_clear(uint8_t *stage, const MfGeo &g) {
  l_u32 *p = (l_u32 *)stage;
  for (int w = threadIdx.x; w < (2 * g.BUF) / 4; w += WGS) p[w] = 0u;
}

// Digits of one term's three rows, loaded by every thread (thread tid holds
// digits tid, tid + WGS, ... of each row; MF_PF per row at most).
constexpr int MF_PF = 3;  // nd <= 3 * WGS = 768 digits
struct MfPrefetch {
  int32_t u[MF_PF], v0[MF_PF], v1[MF_PF];
};

// (buffer loads: digits past nd read 0 without touching memory)
__device__ __forceinline__ void mf_load(MfPrefetch &r, const int32_t *U, const int32_t *V0,
                                        const int32_t *V1, int nd) {
  const __amdgpu_buffer_rsrc_t ru = dev_rsrc(U + HDR + RPAD, nd * 4);
  const __amdgpu_buffer_rsrc_t ra = dev_rsrc(V0 + HDR + RPAD, nd * 4);
  const __amdgpu_buffer_rsrc_t rb = dev_rsrc(V1 + HDR + RPAD, nd * 4);
#pragma unroll
  for (int j = 0; j < MF_PF; ++j) {
    const int o = 4 * (threadIdx.x + j * WGS);
    r.u[j] = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(ru, o, 0, 0);
    r.v0[j] = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(ra, o, 0, 0);
    r.v1[j] = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rb, o, 0, 0);
  }
}

// Store a prefetched term into staging buffer `buf`: U reversed, V0 and V1
// shifted up by their offsets (in digits; each V write also clears the
// pieces up to NP + MF_OFFP so that no piece of an earlier term with a
// larger offset survives).
__device__ __forceinline__ void mf_store(const MfPrefetch &r, uint8_t *buf, const MfGeo &g, int nd,
                                         int off0, int off1) {
  l_u8 *U = (l_u8 *)buf;
  l_u8 *V0 = U + g.UBs, *V1 = V0 + g.VBs;
  const int ndw = nd + 2 * SMAX;  // digit slots of a shifted V row
#pragma unroll
  for (int j = 0; j < MF_PF; ++j) {
    const int d = threadIdx.x + j * WGS;
    if (d < nd) *(l_u32 *)(U + g.ZU - 4 * d - 3) = mf_pieces(r.u[j], false);
  }
  // V slots s = 0..ndw-1 hold digit s - off (zero outside the row)
#pragma unroll
  for (int f = 0; f < 2; ++f) {
    l_u8 *V = f ? V1 : V0;
    const int off = f ? off1 : off0;
    // clear the slots below the shifted row and above it up to ndw
    for (int s = threadIdx.x; s < ndw; s += WGS) {
      if (s < off || s >= off + nd) *(l_u32 *)(V + mf_vaddr(4 * s)) = 0u;
    }
#pragma unroll
    for (int j = 0; j < MF_PF; ++j) {
      const int d = threadIdx.x + j * WGS;
      if (d < nd) *(l_u32 *)(V + mf_vaddr(4 * (d + off))) = mf_pieces(f ? r.v1[j] : r.v0[j], true);
    }
  }
}

// 8 bytes from LDS at any byte address (gfx950 reads unaligned LDS words
// in one ds_read_b64).
typedef __attribute__((address_space(3), aligned(1))) uint64_t l_u64u;
// 8 bytes from LDS at any byte address (gfx950 reads unaligned LDS words
// in one ds_read_b64).
typedef __attribute__((address_space(3), aligned(1))) uint64_t l_u64u;
// Stage a digit row held in LDS (header, RPAD zero digits, nd digits) as
// pieces: reversed into a U buffer, or at offset 0 into a V buffer (whose
// other slots must already be zero).  Every thread of the workgroup.
__device__ __forceinline__ void mf_stage_lds_row(const int32_t *row_, uint8_t *dst, bool as_u,
                                                 const MfGeo &g, int nd) {
  const l_i32 *row = (const l_i32 *)row_ + HDR + RPAD;
  l_u8 *D = (l_u8 *)dst;
  for (int d = threadIdx.x; d < nd; d += WGS) {
    const int32_t v = row[d];
    if (as_u) *(l_u32 *)(D + g.ZU - 4 * d - 3) = mf_pieces(v, false);
    else *(l_u32 *)(D + mf_vaddr(4 * d)) = mf_pieces(v, true);
  }
}

__device__ __forceinline__ uint64_t mf_ld64(const l_u8 *p) { return *(const l_u64u *)p; }

// The (m, tile) pairs of this wavefront: pairs in (m, q) order, q valid for
// m when 32 q - m lies in [-31, DQH] (a contiguous range of q for each m);
// wavefront w takes pairs [P w / 4, P (w+1) / 4).  All of it is uniform over
// the wavefront (scalar registers): `wave` comes through readfirstlane.
struct MfPairs {
  int m0, m1;    // first and last U block with pairs of this wavefront (m0 > m1: none)
  int qa0, qb1;  // first tile of block m0 and last tile of block m1 that are its pairs
};

__device__ __forceinline__ void mf_qrange(const MfGeo &g, int m, int *qlo, int *qhi) {
  // 32 q - m >= -31  <=>  q >= ceil((m - 31) / 32);  32 q - m <= DQH  <=>  q <= (m + DQH) / 32
  int lo = m >= 31 ? (m - 31 + 31) / 32 : 0;
  int hi = (m + g.DQH) / 32;
  if (hi > g.NT - 1) hi = g.NT - 1;
  *qlo = lo;
  *qhi = hi;
}

__device__ __forceinline__ MfPairs mf_pairs(const MfGeo &g, int wave) {
  int P = 0;
  for (int m = 0; m < g.MM; ++m) {
    int lo, hi;
    mf_qrange(g, m, &lo, &hi);
    P += hi >= lo ? hi - lo + 1 : 0;
  }
  const int plo = P * wave / 4, phi = P * (wave + 1) / 4;
  MfPairs r;
  r.m0 = 0;
  r.m1 = -1;
  r.qa0 = r.qb1 = 0;
  int pi = 0;
  for (int m = 0; m < g.MM; ++m) {
    int lo, hi;
    mf_qrange(g, m, &lo, &hi);
    for (int q = lo; q <= hi; ++q, ++pi) {
      if (pi == plo) {
        r.m0 = m;
        r.qa0 = q;
      }
      if (pi == phi - 1) {
        r.m1 = m;
        r.qb1 = q;
      }
    }
  }
  if (phi <= plo) r.m1 = -1;
  return r;
}

// One term on this wavefront's pairs: acc[f][q] += W (U's Toeplitz blocks)
// times X (V_f's blocks) for f < NF, one v_mfma_i32_32x32x32_i8 each:
// lane l (t = l % 32, h = l / 32) supplies the inner indices s = 16 h + u,
// u = 0..15, of both operands (the instruction sums over s, so any fixed
// assignment of s to the lane's bytes that both operands share is exact):
//   W bytes u: U[32 m + t - 16 h - u], 16 consecutive bytes of the reversed
//              U buffer from ZU - 32 m - t + 16 h;
//   X bytes u: V[32 (32 q + t - m) + 16 h + u], 16 bytes of block
//              32 q + t - m from offset 16 h.
// The operands of U block m + 1 are loaded while the products of block m
// are issued (two register stages).
typedef int mf_v4i __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3), aligned(1))) mf_v4i l_v4iu1;
typedef __attribute__((address_space(3), aligned(4))) mf_v4i l_v4iu4;
// 16 bytes at any byte address (the W reads) or at a multiple of 4 (X)
__device__ __forceinline__ mf_v4i mf_ld128(const l_u8 *p) { return *(const l_v4iu1 *)p; }
__device__ __forceinline__ mf_v4i mf_ld128a4(const l_u8 *p) { return *(const l_v4iu4 *)p; }

template <int NF>
struct MfStage {
  mf_v4i w;
  mf_v4i x[NF][MF_NTMAX];
  int qlo, qhi;
};

template <int NF>
__device__ __forceinline__ void mf_stage_load(MfStage<NF> &st, const l_u8 *wbase, const l_u8 *V0,
                                              const l_u8 *V1, int xl, int m, int qlo, int qhi) {
  st.qlo = qlo;
  st.qhi = qhi;
  st.w = mf_ld128(wbase - 32 * m);
  // every tile's operands are loaded (tiles outside [qlo, qhi] from tile
  // qlo's address, and not used), so that the number of LDS reads in flight
  // is fixed and the waits before the products can be exact
#pragma unroll
  for (int q = 0; q < MF_NTMAX; ++q) {
    const int qq = q < qlo ? qlo : q > qhi ? qlo : q;
    const int xo = xl + 36 * (32 * qq - m);
    st.x[0][q] = mf_ld128a4(V0 + xo);
    if constexpr (NF > 1) st.x[1][q] = mf_ld128a4(V1 + xo);
  }
}

template <int NF>
__device__ __forceinline__ void mf_stage_mma(mf_v16i (&acc)[NF][MF_NTMAX], const MfStage<NF> &st) {
#pragma unroll
  for (int q = 0; q < MF_NTMAX; ++q) {
    if (q < st.qlo || q > st.qhi) continue;
#pragma unroll
    for (int f = 0; f < NF; ++f)
      acc[f][q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(st.x[f][q], st.w, acc[f][q], 0, 0, 0);
  }
}

// Tiles of block m among this wavefront's pairs.
__device__ __forceinline__ void mf_qclip(const MfGeo &g, const MfPairs &pr, int m, int *qlo,
                                         int *qhi) {
  mf_qrange(g, m, qlo, qhi);
  if (m == pr.m0) *qlo = pr.qa0;
  if (m == pr.m1) *qhi = pr.qb1;
}

template <int NF>
__device__ __forceinline__ void mf_term(mf_v16i (&acc)[NF][MF_NTMAX], const uint8_t *buf,
                                        const MfGeo &g, const MfPairs &pr) {
  const int lane = threadIdx.x & 63, t = lane & 31, h = lane >> 5;
  const l_u8 *U = (const l_u8 *)buf;
  const l_u8 *V0 = U + g.UBs, *V1 = V0 + g.VBs;
  // per-lane parts of the addresses
  const l_u8 *wbase = U + g.ZU - t + 16 * h;
  const int xl = 36 * (t + MF_VLO / 32) + 16 * h;
  const int m0 = __builtin_amdgcn_readfirstlane(pr.m0), m1 = __builtin_amdgcn_readfirstlane(pr.m1);
  if (m0 > m1) return;
  // two register stages in turn: the operands of the next block are loaded
  // (unconditionally, the last block again at the end, so that the number of
  // reads in flight is fixed) while the current block's products issue
  MfStage<NF> A, B;
  int qa, qb;
  mf_qclip(g, pr, m0, &qa, &qb);
  mf_stage_load<NF>(A, wbase, V0, V1, xl, m0, qa, qb);
  for (int m = m0;; m += 2) {
    const int mb = m + 1 < m1 ? m + 1 : m1;
    mf_qclip(g, pr, mb, &qa, &qb);
    mf_stage_load<NF>(B, wbase, V0, V1, xl, mb, qa, qb);
    mf_stage_mma<NF>(acc, A);
    if (m + 1 > m1) break;
    const int ma = m + 2 < m1 ? m + 2 : m1;
    mf_qclip(g, pr, ma, &qa, &qb);
    mf_stage_load<NF>(A, wbase, V0, V1, xl, ma, qa, qb);
    mf_stage_mma<NF>(acc, B);
    if (m + 2 > m1) break;
  }
}

// Add the accumulators into the frames' 64-bit LDS columns lf[f * WB + c]
// and clear them.  The products are issued as X^T W^T (the transpose of
// O = W X), so lane l holds position t = l % 32 of the blocks
// R = 32 q + 8 b + 4 (l / 32) + r in its registers 4 b + r: output position
// pi = 32 R + t, column pi / 4 with weight 2^(7 (pi % 4)).  The four lanes
// t = 4c'..4c'+3 hold the four pieces of one column: they are weighted and
// added across the lane group (DPP row shifts), and the group's last lane
// adds the column into LDS, so each atomic instruction touches 16 columns
// in runs of 8 consecutive ones.
template <int NF>
__device__ __forceinline__ void mf_flush(mf_v16i (&acc)[NF][MF_NTMAX], long long *lf, int WB,
                                         const MfGeo &g) {
  const int lane = threadIdx.x & 63, t = lane & 31, h = lane >> 5;
  const int sh = 7 * (t & 3);
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int q = 0; q < MF_NTMAX; ++q) {
      if (q < g.NT) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          long long v = (long long)acc[f][q][r] * (long long)(1 << sh);
          v = dpp_sum4_64(v);
          const int R = 32 * q + 8 * (r >> 2) + 4 * h + (r & 3);
          const int c = 8 * R + (t >> 2);
          if ((t & 3) == 3 && v != 0 && c < WB)
            __hip_atomic_fetch_add((unsigned long long __attribute__((address_space(3))) *)
                                       ((l_i64 *)lf + (size_t)f * WB + c),
                                   (unsigned long long)v, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[f][q][r] = 0;
    }
}

}  // namespace mpts
