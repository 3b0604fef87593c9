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
// X depends on R - m only, so the blocks m = r and m = r + 32 use the same
// X operands (output tiles q and q + 1): a wavefront takes a range of r and
// for each loads two W operands and one X operand per tile and frame, which
// halves the LDS reads per product against one block at a time.
//
// One workgroup takes a contiguous range of terms of the two Cauchy frames
// of an index (they share U_k = a_{i-k}); for each term it stages the three
// rows as pieces in LDS, and its four wavefronts split the blocks r, each
// holding the accumulators of both frames for every output tile.
#pragma once
#include <hip/hip_runtime.h>
#include "mpts_common.h"
#include "mpts_rows.h"

namespace mpts {

typedef __attribute__((address_space(3))) uint8_t l_u8;
typedef __attribute__((address_space(3))) uint32_t l_u32;
typedef __attribute__((address_space(3), aligned(1))) uint32_t l_u32u;
typedef int mf_v16i __attribute__((ext_vector_type(16)));
typedef int mf_v4i __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3), aligned(4))) mf_v4i l_v4i4;
typedef __attribute__((address_space(3))) mf_v4i l_v4i16;

constexpr int MF_OFFP = 4 * 2 * SMAX;  // largest term offset in pieces
constexpr int MF_VLO = 1120;           // V pieces below 0 that a read can reach (35 blocks)
constexpr int MF_NTMAX = 4;            // output tiles of 1024 pieces held per wavefront
constexpr int MF_VB = 48;              // bytes per 32-piece V block (16-byte aligned reads)

// Piece geometry for rows of nd digits.  The U row is stored reversed (piece
// x at byte ZU - x) in four copies, copy c shifted up by c bytes, so that
// every lane's 16-byte W window starts on a 4-byte boundary of one copy; a
// V row in blocks of 32 pieces at a stride of MF_VB bytes, logical piece P
// at block (P + MF_VLO) / 32.
struct MfGeo {
  int NP;   // pieces per row
  int MM;   // U blocks m = 0..MM-1 that can hold a piece
  int NT;   // output tiles (1024 pieces each) that can hold a nonzero sum
  int DQH;  // last V block that can hold a piece
  int RR;   // blocks r = 0..RR-1 (r and r + 32)
  // X operands X(32 q - r), q < NQ(r), that can hold a piece, and the tiles
  // q + 1 < JQ(r) + 1 of the block r + 32: (NQA, JQA) for r < RS, (NQB, JQB)
  // from RS on (NQ(r) grows by at most one over the 32 blocks r)
  int NQA, JQA, NQB, JQB, RS;
  int ZU;   // byte of U piece 0 in a copy (ZU = 3 mod 4)
  int UCS;  // bytes of one U copy
  int VBLK; // blocks of a V buffer
  int VBs;  // bytes of a V buffer
  int BUF;  // bytes of one staging buffer: four U copies, V0, V1
  int FT;   // terms between flushes of the i32 accumulators
};

__host__ __device__ inline MfGeo mf_geo(int nd) {
  MfGeo g;
  g.NP = 4 * nd;
  g.MM = (g.NP + 30) / 32 + 1;
  g.NT = (2 * g.NP + MF_OFFP) / 1024 + 1;
  g.DQH = (g.NP + MF_OFFP - 1) / 32;
  g.RR = g.MM < 32 ? g.MM : 32;
  auto nq = [&](int r) { const int q = (r + g.DQH) / 32 + 1; return q < g.NT ? q : g.NT; };
  auto jq = [&](int q) { return g.MM > 32 ? (q < g.NT - 1 ? q : g.NT - 1) : 0; };
  g.NQA = nq(0);
  g.NQB = nq(g.RR - 1);
  g.JQA = jq(g.NQA);
  g.JQB = jq(g.NQB);
  // first r with NQ(r) = NQB: 32 NQA - DQH (tiles q < NQ(r) are those with
  // 32 q - r <= DQH)
  g.RS = g.NQB > g.NQA ? 32 * g.NQA - g.DQH : g.RR;
  if (g.RS < 0) g.RS = 0;
  if (g.RS > g.RR) g.RS = g.RR;
  g.ZU = 4 * ((g.NP + 64) / 4) + 3;
  // copies 64 bytes apart modulo 256 (16 LDS banks): the lanes of a W read
  // that take different copies then reach different banks
  g.UCS = (g.ZU + 64 + 15) & ~15;
  g.UCS += (64 - (g.UCS & 255) + 256) & 255;
  // logical pieces [-MF_VLO, NP + MF_OFFP + 1056) in 32-piece blocks
  g.VBLK = (MF_VLO + g.NP + MF_OFFP + 1056 + 31) / 32;
  g.VBs = (MF_VB * g.VBLK + 15) & ~15;
  g.BUF = 4 * g.UCS + 2 * g.VBs;
  // one term adds at most NP products of magnitude <= 127^2 to an output
  const long long per_term = (long long)g.NP * 127 * 127;
  long long ft = per_term > 0 ? 2147483647LL / per_term : 1;
  g.FT = (int)(ft < 1 ? 1 : ft > 4096 ? 4096 : ft);
  return g;
}

// Piece sums of one index, both frames: int32 P[f][pi], pi = 32 R + t <
// 1024 NT, after the two staging buffers.
__host__ __device__ inline int mf_parr_bytes(const MfGeo &g) { return 2 * g.NT * 1024 * 4; }

// Staging bytes (two buffers and the piece sums) the MFMA path needs in LDS.
__host__ __device__ inline int mf_stage_bytes(int nd) {
  const MfGeo g = mf_geo(nd);
  return 2 * g.BUF + mf_parr_bytes(g);
}

// Whether the MFMA path holds this size (all output tiles in one
// wavefront's accumulators, U blocks r and r + 32 only).
__host__ __device__ inline bool mf_fits(int nd) {
  const MfGeo g = mf_geo(nd);
  return g.NT <= MF_NTMAX && g.MM <= 64 && nd <= 2 * WGS;
}

// The four pieces s p0..s p3 of a 28-bit digit D, packed little-endian
// (forward = true: p0 in the low byte) or reversed (p3 in the low byte).
__device__ __forceinline__ uint32_t mf_pieces(int32_t D, bool forward) {
  const uint32_t M = (uint32_t)(D < 0 ? -D : D);
  // 7-bit fields of |D| spread one per byte (p0 in the low byte)
  uint32_t w = (M & 0x7fu) | ((M << 1) & 0x7f00u) | ((M << 2) & 0x7f0000u) | ((M << 3) & 0x7f000000u);
  // negative digit: every byte v becomes (256 - v) mod 256; bytes are at most
  // 127, so 128 - v per byte needs no borrow across bytes
  if (D < 0) w = (0x80808080u - w) ^ 0x80808080u;
  return forward ? w : __builtin_bswap32(w);
}

// Byte address in a V buffer of logical piece P.
__device__ __forceinline__ int mf_vaddr(int P) {
  const int b = P + MF_VLO;
  return MF_VB * (b >> 5) + (b & 31);
}

// Zero both staging buffers and the piece sums (every thread of the
// workgroup).
__device__ __forceinline__ void mf_clear(uint8_t *stage, const MfGeo &g) {
  l_u32 *p = (l_u32 *)stage;
  for (int w = threadIdx.x; w < (2 * g.BUF + mf_parr_bytes(g)) / 4; w += WGS) p[w] = 0u;
}

// Digits of one term's three rows, loaded by every thread (thread tid holds
// digits tid, tid + WGS, ... of each row; MF_PF per row at most).
constexpr int MF_PF = 2;  // nd <= 2 * WGS = 512 digits (mf_fits admits at most 487)
struct MfPrefetch {
  int32_t u[MF_PF], un[MF_PF], v0[MF_PF], v1[MF_PF];  // un: the U digit above u
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
    r.un[j] = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(ru, o + 4, 0, 0);
    r.v0[j] = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(ra, o, 0, 0);
    r.v1[j] = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rb, o, 0, 0);
  }
}

// Store a prefetched term into staging buffer `buf`: U reversed into its
// four copies, V0 and V1 shifted up by their offsets (in digits; each V
// write also clears the pieces up to NP + MF_OFFP so that no piece of an
// earlier term with a larger offset survives).
//
// Copy c holds piece x at byte ZU - x + c, so its aligned word at ZU - 3 - 4 D
// holds the pieces 4 D + c .. 4 D + c + 3: the reversed pieces of digit D
// shifted up by c bytes, below them the top c reversed pieces of digit D + 1
// (words D = -1 .. nd-1).  The U pieces of every term occupy the same
// bytes, so the copies' padding stays zero.
__device__ __forceinline__ void mf_store(const MfPrefetch &r, uint8_t *buf, const MfGeo &g, int nd,
                                         int off0, int off1) {
  l_u8 *U = (l_u8 *)buf;
  l_u8 *V0 = U + 4 * g.UCS, *V1 = V0 + g.VBs;
  const int ndw = nd + 2 * SMAX;  // digit slots of a shifted V row
#pragma unroll
  for (int j = 0; j < MF_PF; ++j) {
    const int d = threadIdx.x + j * WGS;
    if (d < nd) {
      const uint32_t w = mf_pieces(r.u[j], false), wn = mf_pieces(r.un[j], false);
      l_u8 *a = U + g.ZU - 3 - 4 * d;
      *(l_u32 *)a = w;
#pragma unroll
      for (int c = 1; c < 4; ++c) *(l_u32 *)(a + c * g.UCS) = (w << (8 * c)) | (wn >> (32 - 8 * c));
      if (d == 0) {
#pragma unroll
        for (int c = 1; c < 4; ++c) *(l_u32 *)(a + 4 + c * g.UCS) = w >> (32 - 8 * c);
      }
    }
  }
  // V slots s = 0..ndw-1 hold digit s - off (zero outside the row)
#pragma unroll
  for (int f = 0; f < 2; ++f) {
    l_u8 *V = f ? V1 : V0;
    const int off = f ? off1 : off0;
    // clear the slots below the shifted row ([0, off)) and above it up to
    // ndw ([off + nd, ndw)): at most 2 SMAX slots on each side
    for (int q = threadIdx.x; q < 4 * SMAX; q += WGS) {
      const int s = q < 2 * SMAX ? q : off + nd + (q - 2 * SMAX);
      if ((q < 2 * SMAX && s < off) || (q >= 2 * SMAX && s < ndw))
        *(l_u32 *)(V + mf_vaddr(4 * s)) = 0u;
    }
#pragma unroll
    for (int j = 0; j < MF_PF; ++j) {
      const int d = threadIdx.x + j * WGS;
      if (d < nd) *(l_u32 *)(V + mf_vaddr(4 * (d + off))) = mf_pieces(f ? r.v1[j] : r.v0[j], true);
    }
  }
}

// The operands of one block r: W of U blocks r and r + 32, and X(32 q - r)
// of both frames for q < NQX.  Lane l (t = l % 32, h = l / 32) supplies the
// inner indices s = 16 h + u, u = 0..15, of both operands (the instruction
// sums over s, so any fixed assignment of s to the lane's bytes that both
// operands share is exact):
//   W bytes u: U[32 m + t - 16 h - u], 16 consecutive bytes of the reversed
//              U from ZU - 32 m - t + 16 h, read from the copy c = (t + 1) % 4
//              whose shift makes that address a multiple of 4;
//   X bytes u: V[32 (32 q + t - r) + 16 h + u], 16 bytes of block
//              32 q + t - r from offset 16 h (16-byte aligned).
// Blocks past the V buffer read its last block, which holds no piece; tiles
// whose blocks hold no piece multiply zeros.
template <int NQX>
struct MfOps {
  mf_v4i w0, w1;
  mf_v4i x[2][NQX];
};

template <int NQX>
__device__ __forceinline__ void mf_ops_load(MfOps<NQX> &o, const l_u8 *wb, const l_u8 *V0,
                                            const l_u8 *V1, int xt, const MfGeo &g, int r, bool j1) {
  o.w0 = *(const l_v4i4 *)(wb - 32 * r);
  o.w1 = *(const l_v4i4 *)(wb - 32 * (j1 ? r + 32 : r));
#pragma unroll
  for (int q = 0; q < NQX; ++q) {
    int b = 32 * q - r + xt;
    b = b < g.VBLK - 1 ? b : g.VBLK - 1;
    o.x[0][q] = *(const l_v4i16 *)(V0 + MF_VB * b);
    o.x[1][q] = *(const l_v4i16 *)(V1 + MF_VB * b);
  }
}

// The products of block r: tiles q (U block r) and q + 1 (U block r + 32).
template <int NQX, int JQ>
__device__ __forceinline__ void mf_ops_mma(mf_v16i (&acc)[2][MF_NTMAX], const MfOps<NQX> &o,
                                           bool j1) {
#pragma unroll
  for (int q = 0; q < NQX; ++q)
#pragma unroll
    for (int f = 0; f < 2; ++f)
      acc[f][q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(o.x[f][q], o.w0, acc[f][q], 0, 0, 0);
  if (JQ > 0 && j1) {
#pragma unroll
    for (int q = 0; q < JQ; ++q)
#pragma unroll
      for (int f = 0; f < 2; ++f)
        acc[f][q + 1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(o.x[f][q], o.w1, acc[f][q + 1], 0, 0, 0);
  }
}

// The blocks r in [r0, r1) of one term, with NQX X operands per frame:
// acc[f][q] += the output tile q of frame f.  The operands of block r + 1
// are loaded while the products of block r are issued (two register
// stages; the last block is loaded again at the end, so that the number of
// reads in flight is fixed).
template <int NQX, int JQ>
__device__ __forceinline__ void mf_term_range(mf_v16i (&acc)[2][MF_NTMAX], const uint8_t *buf,
                                              const MfGeo &g, int r0, int r1) {
  const int lane = threadIdx.x & 63, t = lane & 31, h = lane >> 5, c = (t + 1) & 3;
  const l_u8 *wb = (const l_u8 *)buf + c * g.UCS + c + g.ZU - t + 16 * h;
  const l_u8 *V0 = (const l_u8 *)buf + 4 * g.UCS + 16 * h, *V1 = V0 + g.VBs;
  const int xt = t + MF_VLO / 32;
  MfOps<NQX> A, B;
  mf_ops_load<NQX>(A, wb, V0, V1, xt, g, r0, r0 + 32 < g.MM);
  for (int r = r0;; r += 2) {
    const int rb = r + 1 < r1 ? r + 1 : r1 - 1;
    mf_ops_load<NQX>(B, wb, V0, V1, xt, g, rb, rb + 32 < g.MM);
    mf_ops_mma<NQX, JQ>(acc, A, r + 32 < g.MM);
    if (r + 1 >= r1) break;
    const int ra = r + 2 < r1 ? r + 2 : r1 - 1;
    mf_ops_load<NQX>(A, wb, V0, V1, xt, g, ra, ra + 32 < g.MM);
    mf_ops_mma<NQX, JQ>(acc, B, r + 33 < g.MM);
    if (r + 2 >= r1) break;
  }
}

// One term on this wavefront's blocks r (a quarter of [0, RR)), each block
// with only the X operands that can hold a piece.
template <int NQA, int JQA, int NQB, int JQB>
__device__ __forceinline__ void mf_term(mf_v16i (&acc)[2][MF_NTMAX], const uint8_t *buf,
                                        const MfGeo &g) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r0 = g.RR * wave / 4, r1 = g.RR * (wave + 1) / 4;
  const int ra = r1 < g.RS ? r1 : g.RS, rb = r0 > g.RS ? r0 : g.RS;
  if (r0 < ra) mf_term_range<NQA, JQA>(acc, buf, g, r0, ra);
  if (NQB != NQA && rb < r1) mf_term_range<NQB, JQB>(acc, buf, g, rb, r1);
}

// Add the accumulators into the piece sums P and clear them.  The products
// are issued as X^T W^T (the transpose of O = W X), so lane l holds
// position t = l % 32 of the blocks R = 32 q + 8 b + 4 (l / 32) + r in its
// registers 4 b + r: output position pi = 32 R + t.  One LDS add per
// register and lane, 64 distinct positions per instruction (the wavefronts
// of the workgroup add into the same sums).
template <int NF>
__device__ __forceinline__ void mf_flush(mf_v16i (&acc)[NF][MF_NTMAX], int32_t *P, const MfGeo &g) {
  const int lane = threadIdx.x & 63, t = lane & 31, h = lane >> 5;
  l_i32 *lp = (l_i32 *)P;
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int q = 0; q < MF_NTMAX; ++q) {
      if (q < g.NT) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int R = 32 * q + 8 * (r >> 2) + 4 * h + (r & 3);
          __hip_atomic_fetch_add(lp + f * g.NT * 1024 + 32 * R + t, acc[f][q][r], __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[f][q][r] = 0;
    }
}

// Add the piece sums into the frames' 64-bit columns of the group's frames
// in global memory, gf[f * WB + c] (column c = pi / 4 with weight
// 2^(7 (pi % 4)); device-scope atomic adds), and clear them; every thread
// of the workgroup, after every wavefront's mf_flush.
__device__ __forceinline__ void mf_columns_global(int32_t *P, long long *gf, int WB, const MfGeo &g) {
  const int ncol = g.NT * 256;
  for (int w = threadIdx.x; w < 2 * ncol; w += WGS) {
    const int f = w >= ncol ? 1 : 0, c = w - f * ncol;
    l_v4i16 *pp = (l_v4i16 *)((l_i32 *)P + f * g.NT * 1024 + 4 * c);
    const mf_v4i v = *pp;
    if ((v.x | v.y | v.z | v.w) != 0) {
      const long long s = (long long)v.x + (long long)v.y * 128LL + (long long)v.z * 16384LL +
                          (long long)v.w * 2097152LL;
      if (c < WB && s != 0)
        __hip_atomic_fetch_add((unsigned long long *)(gf + (size_t)f * WB + c), (unsigned long long)s,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      *pp = mf_v4i{0, 0, 0, 0};
    }
  }
}

// Move the piece sums into the frames' 64-bit LDS columns lf[f * WB + c]
// (column c = pi / 4 with weight 2^(7 (pi % 4))) and clear them; every
// thread of the workgroup, after every wavefront's mf_flush.
__device__ __forceinline__ void mf_columns(int32_t *P, long long *lf, int WB, const MfGeo &g) {
  const int ncol = g.NT * 256;
  for (int w = threadIdx.x; w < 2 * ncol; w += WGS) {
    const int f = w >= ncol ? 1 : 0, c = w - f * ncol;
    l_v4i16 *pp = (l_v4i16 *)((l_i32 *)P + f * g.NT * 1024 + 4 * c);
    const mf_v4i v = *pp;
    if ((v.x | v.y | v.z | v.w) != 0) {
      const long long s = (long long)v.x + (long long)v.y * 128LL + (long long)v.z * 16384LL +
                          (long long)v.w * 2097152LL;
      if (c < WB)
        __hip_atomic_fetch_add((unsigned long long __attribute__((address_space(3))) *)
                                   ((l_i64 *)lf + (size_t)f * WB + c),
                               (unsigned long long)s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      *pp = mf_v4i{0, 0, 0, 0};
    }
  }
}

}  // namespace mpts
