// Rows (signed radix-2^28 digit vectors with a header) and the exact
// multi-term product accumulation over 8x8 digit tiles.
#pragma once
#include <hip/hip_runtime.h>
#include "mpts_common.h"
#include "mpts_wave.h"

namespace mpts {

__device__ __forceinline__ int32_t ld_relaxed(const int32_t *p) {
  return __hip_atomic_load(const_cast<int32_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ long long ld_relaxed(const long long *p) {
  return __hip_atomic_load(const_cast<long long *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_relaxed(const uint32_t *p) {
  return __hip_atomic_load(const_cast<uint32_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(int32_t *p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(long long *p, long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Device-coherent (sc1, L2-bypassing) 64-bit loads through a buffer
// resource: unlike atomic loads they are not ordered with each other, so a
// batch of them is in flight at once, and offsets outside [0, bytes) read 0.
typedef int mpts_v2i __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t dev_rsrc(const void *p, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, bytes, 0x00020000);
}
__device__ __forceinline__ long long ld_dev64(__amdgpu_buffer_rsrc_t rs, int byte_off) {
  mpts_v2i t = __builtin_amdgcn_raw_buffer_load_b64(rs, byte_off, 0, 16 /* sc1 */);
  return (long long)(((unsigned long long)(uint32_t)t.y << 32) | (uint32_t)t.x);
}
// All of this thread's outstanding global loads, stores and atomics are done.
__device__ __forceinline__ void wait_vmem() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

__device__ __forceinline__ int floordiv28(long long e, long long *rem) {
  long long q = e >= 0 ? e / DBITS : -((-e + DBITS - 1) / DBITS);
  *rem = e - q * DBITS;
  return (int)q;
}

// Bits [b, b+28) of the L-limb mantissa M (bits outside [0, 32 L) are zero).
__device__ __forceinline__ uint32_t mant_bits28(const int32_t *M, int L, long long b) {
  long long q = b >= 0 ? (b >> 5) : -((-b + 31) >> 5);
  int r = (int)(b - q * 32);
  unsigned long long lo = (q >= 0 && q < L) ? (uint32_t)M[q] : 0u;
  unsigned long long hi = (q + 1 >= 0 && q + 1 < L) ? (uint32_t)M[q + 1] : 0u;
  unsigned long long w = ((hi << 32) | lo) >> r;
  return (uint32_t)(w & (unsigned long long)DMASK);
}

// The same on mantissas in LDS or global memory, with int bit positions.
template <typename P>
__device__ __forceinline__ uint32_t mant_bits28_as(P M, int L, int b) {
  const int q = b >= 0 ? (b >> 5) : -((-b + 31) >> 5);
  const int r = b - q * 32;
  unsigned long long lo = (q >= 0 && q < L) ? (uint32_t)M[q] : 0u;
  unsigned long long hi = (q + 1 >= 0 && q + 1 < L) ? (uint32_t)M[q + 1] : 0u;
  unsigned long long w = ((hi << 32) | lo) >> r;
  return (uint32_t)(w & (unsigned long long)DMASK);
}
__device__ __forceinline__ uint32_t mant_bits28_l(const l_i32 *M, int L, int b) {
  return mant_bits28_as(M, L, b);
}
__device__ __forceinline__ uint32_t mant_bits28_g(const g_i32 *M, int L, int b) {
  return mant_bits28_as(M, L, b);
}

// Row of a normalised value nv = [sign, E, M[L]]: digit exponent e =
// floor(E / 28), digits of M * 2^(E - 28 e) with the sign applied.  Written
// by one wavefront (or any group of `nthr` threads indexed by `tid`), header
// and zero padding included.  `relaxed` selects L2-bypassing stores (for
// rows that other workgroups read).
__device__ void write_row(const int32_t *nv, int L, int nd, int RS, int32_t *row, bool relaxed,
                          int tid, int nthr, bool negate = false) {
  int s = negate ? -nv[0] : nv[0];
  long long E = nv[1];
  long long sh;
  int e = floordiv28(E, &sh);
  if (s == 0) e = 0;
  for (int w = tid; w < RS; w += nthr) {
    int32_t val = 0;
    if (w == 0) val = e;
    else if (w == 1) val = s;
    else if (w >= HDR + RPAD && w < HDR + RPAD + nd && s != 0) {
      int k = w - HDR - RPAD;
      uint32_t d = mant_bits28(nv + 2, L, (long long)DBITS * k - sh);
      val = s < 0 ? -(int32_t)d : (int32_t)d;
    }
    if (relaxed) st_relaxed(row + w, val);
    else row[w] = val;
  }
}

// ---------------------------------------------------------------------------
// Exact sums of products of rows ("frames").
//
// A frame is sum_t U_t * V_t over its terms.  With the terms' exponent sums
// e(U_t) + e(V_t) = base + off_t (0 <= off_t <= S), the frame's value is
// sum_c col[c] 2^(28 (base + c)), col[c] = sum_t sum_{m + n = c - off_t}
// U_t[m] V_t[n].  The (m, n') plane (n' = n + off_t) is cut into 8x8 tiles;
// a thread owning tile (mt, nt) accumulates its 15 anti-diagonal columns
// exactly in 64-bit integers over a share of the terms and adds them into
// the frame's column array.

// Terms of a frame come in up to three parts; part kinds:
//   CAUCHY: k = 0..n-1 -> U[idx - k] * V[k]   (rows of stride RS)
//   CORR:   k = 0..n-1 -> U[idx + k] * V[k]
//   DOT:    k = 0..n-1 -> U[k] * V[k]
//   ONE:    one term U * V
enum { PK_CAUCHY = 0, PK_CORR = 1, PK_DOT = 2, PK_ONE = 3 };

struct FramePart {
  int kind, n, idx, pad;
  const int32_t *U, *V;
  // optional exponent caches (LDS) indexed like the rows (row j of U ->
  // hU[j]): the row's digit exponent, or HZ for a zero row
  const int *hU, *hV;
  // parts without both caches: per-term digit offsets in LDS (frame_setup)
  const int8_t *ot;
};

struct FrameSrc {
  int nparts, n;  // n = total terms
  int mlo, mhi;   // digit range holding every nonzero digit of the parts' U rows
  int fbase;      // the frame's exponent base when given (else HZ: the terms' minimum)
  int pad;
  FramePart p[4];
};

// A frame's column c holds the digit weight 2^(28 (base + c)); term t sits at
// offset off_t = e(U_t) + e(V_t) - base in [0, S].  Tile rows mt0 .. mt0 +
// MTf - 1 and tile columns nt0 .. nt0 + NT - 1 can be nonzero.
struct FrameD {
  int n, base, S, NT, nz, mt0, MTf, nt0;
};

typedef __attribute__((address_space(3))) FrameSrc l_FrameSrc;
typedef __attribute__((address_space(3))) FrameD l_FrameD;

// Word copies between LDS descriptors and registers (descriptors in LDS are
// read and written through LDS addresses, not flat ones).  The words pass
// through an int array and memcpy: the descriptors hold pointers, which an
// int lvalue may not alias.
template <typename T>
__device__ __forceinline__ T lds_get(const T *p) {
  static_assert(sizeof(T) % 4 == 0, "descriptor of whole words");
  int w[sizeof(T) / 4];
  const l_i32 *s = (const l_i32 *)p;
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 4); ++k) w[k] = s[k];
  T v;
  __builtin_memcpy(&v, w, sizeof(T));
  return v;
}
template <typename T>
__device__ __forceinline__ void lds_put(T *p, const T &v) {
  static_assert(sizeof(T) % 4 == 0, "descriptor of whole words");
  int w[sizeof(T) / 4];
  __builtin_memcpy(w, &v, sizeof(T));
  l_i32 *d = (l_i32 *)p;
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 4); ++k) d[k] = w[k];
}

constexpr int HZ = (int)0x80000000;  // exponent cache entry of a zero row

__device__ __forceinline__ int row_exp(const int32_t *row) { return row[1] != 0 ? row[0] : HZ; }

__device__ __forceinline__ void part_rows(const FramePart &q, int k, int *iu, int *iv) {
  switch (q.kind) {
    case PK_CAUCHY: *iu = q.idx - k; *iv = k; break;
    case PK_CORR: *iu = q.idx + k; *iv = k; break;
    case PK_DOT: *iu = k; *iv = k; break;
    default: *iu = 0; *iv = 0;
  }
}

__device__ __forceinline__ void part_term(const FramePart &q, int k, int RS, const int32_t **U,
                                          const int32_t **V) {
  int iu, iv;
  part_rows(q, k, &iu, &iv);
  *U = q.U + (long long)iu * RS;
  *V = q.V + (long long)iv * RS;
}

__device__ __forceinline__ int row_exp_g(const g_i32 *row) { return row[1] != 0 ? row[0] : HZ; }

// Exponent sum of term k of a part (HZ when either row is zero).  The rows
// are in global memory, the caches in LDS.
__device__ __forceinline__ int part_esum(const FramePart &q, int k, int RS) {
  int iu, iv;
  part_rows(q, k, &iu, &iv);
  const int eu = q.hU ? ((const l_i32 *)q.hU)[iu] : row_exp_g((const g_i32 *)q.U + iu * RS);
  const int ev = q.hV ? ((const l_i32 *)q.hV)[iv] : row_exp_g((const g_i32 *)q.V + iv * RS);
  return (eu == HZ || ev == HZ) ? HZ : eu + ev;
}

__host__ __device__ inline FramePart mk_part(int kind, int n, int idx, const int32_t *U,
                                             const int32_t *V, const int *hU = nullptr,
                                             const int *hV = nullptr) {
  FramePart q;
  q.kind = kind;
  q.n = n;
  q.idx = idx;
  q.pad = 0;
  q.U = U;
  q.V = V;
  q.hU = hU;
  q.hV = hV;
  q.ot = nullptr;
  return q;
}

__host__ __device__ inline FrameSrc mk_frame1(FramePart a) {
  FrameSrc f;
  f.nparts = 1;
  f.n = a.n;
  f.mlo = 0;
  f.mhi = 0x7fffffff;
  f.fbase = (int)0x80000000;
  f.pad = 0;
  f.p[0] = a;
  f.p[1] = a;
  f.p[2] = a;
  f.p[3] = a;
  return f;
}

__host__ __device__ inline FrameSrc mk_frame2(FramePart a, FramePart b) {
  FrameSrc f = mk_frame1(a);
  f.nparts = 2;
  f.n = a.n + b.n;
  f.p[1] = b;
  return f;
}

__host__ __device__ inline FrameSrc mk_frame3(FramePart a, FramePart b, FramePart c) {
  FrameSrc f = mk_frame2(a, b);
  f.nparts = 3;
  f.n = a.n + b.n + c.n;
  f.p[2] = c;
  return f;
}

__host__ __device__ inline FrameSrc mk_frame4(FramePart a, FramePart b, FramePart c, FramePart d) {
  FrameSrc f = mk_frame3(a, b, c);
  f.nparts = 4;
  f.n = a.n + b.n + c.n + d.n;
  f.p[3] = d;
  return f;
}

// Tile (mt, nt) of the t-th tile in anti-diagonal order of an MT x NT grid
// (MT <= NT): diagonals d = mt + nt in increasing order, mt increasing along
// each diagonal.  Diagonals 0..MT-2 hold d+1 tiles, MT-1..NT-1 hold MT, and
// the last ones mirror the first (counted from the end).
__device__ __forceinline__ int tri_index(int t) {
  int d = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
  while ((d + 1) * (d + 2) / 2 <= t) ++d;
  while (d * (d + 1) / 2 > t) --d;
  return d;
}

__device__ __forceinline__ void tile_coords(int t, int MT, int NT, int *mt, int *nt) {
  const int T1 = MT * (MT - 1) / 2;
  const int T2 = MT * (NT - MT + 1);
  int d, m;
  if (t < T1) {
    d = tri_index(t);
    m = t - d * (d + 1) / 2;
  } else if (t < T1 + T2) {
    d = MT - 1 + (t - T1) / MT;
    m = (t - T1) % MT;
  } else {
    int t3 = MT * NT - 1 - t;
    int dd = tri_index(t3);
    d = MT + NT - 2 - dd;
    m = MT - 1 - (t3 - dd * (dd + 1) / 2);
  }
  *mt = m;
  *nt = d - m;
}

__device__ __forceinline__ void tile_normalize(long long (&acc)[16]) {
#pragma unroll
  for (int r = 0; r < 15; ++r) {
    acc[r + 1] += acc[r] >> DBITS;
    acc[r] &= DMASK;
  }
}

// The min / max slots of frame_setup's reduction, back to their neutral
// values (the next use is behind at least one workgroup barrier).
__device__ __forceinline__ void red_reset(int *red) {
  const int t = threadIdx.x;
  if (t < 2 * NFR) ((l_i32 *)red)[t] = (t & 1) ? -0x7fffffff : 0x7fffffff;
}

// Descriptor of a frame of n terms whose nonzero terms have exponent sums
// in [a, b] (a > b: no nonzero term), with the given base fbase (HZ: none)
// and the U operands' nonzero digits in [mlo, mhi].  A given base must lie
// at most 2 SMAX below every term; the spread of the terms is at most SMAX
// either way.
__device__ __forceinline__ FrameD make_desc(int n, int fbase, int mlo, int mhi, int a, int b,
                                           int nd, uint32_t *err) {
  FrameD d;
  d.n = n;
  d.nz = (a <= b) ? 1 : 0;
  int lo = 0, S = 0;
  if (d.nz) {
    d.base = fbase != HZ ? fbase : a;
    lo = a - d.base;
    S = b - d.base;
    if (b - a > SMAX || lo < 0 || S > 2 * SMAX) {
      atomicOr(err, 1u | 16u);
      lo = max(min(lo, 2 * SMAX), 0);
      S = max(min(S, 2 * SMAX), lo);
    }
  } else {
    d.base = fbase != HZ ? fbase : 0;
  }
  d.S = S;
  d.nt0 = lo / TQ;
  d.NT = (nd + S + TQ - 1) / TQ - d.nt0;
  const int MT = (nd + TQ - 1) / TQ;
  const int m0 = max(mlo, 0) / TQ;
  const int m1 = min(mhi, nd - 1) / TQ;
  d.mt0 = m0 < MT ? m0 : 0;
  d.MTf = m1 >= m0 && m0 < MT ? min(m1, MT - 1) - m0 + 1 : MT;
  return d;
}

// Per-workgroup frame setup: exponent base and spread of each frame's
// nonzero terms (one workgroup reduction for all frames).  Exponents come
// from the parts' caches (LDS) or, for parts without both caches, from the
// row headers; those parts get a table of per-term digit offsets in LDS
// (offs, maxn bytes), so that the product loop never waits on a header
// load.  The exponent sums are read twice (for the reduction, then for the
// table) rather than kept in a scratch array.  Every thread of the
// workgroup calls this; thread 0 stores the table slices into fs.
__device__ void frame_setup(FrameSrc *fs, FrameD *fd, int nf, int nd, int RS, int *red,
                            int8_t *offs, int maxn, uint32_t *err) {
  const int tid = threadIdx.x;
  int mn[NFR], mx[NFR];
  int ob = 0;  // table position of the next uncached part (same in every thread)
  bool fits = true;
#pragma unroll
  for (int f = 0; f < NFR; ++f) {
    mn[f] = 0x7fffffff;
    mx[f] = -0x7fffffff;
    if (f < nf) {
      const int np = ((const l_i32 *)&fs[f].nparts)[0];
      for (int j = 0; j < np; ++j) {
        const FramePart q = lds_get(&fs[f].p[j]);
        const bool cached = q.hU && q.hV;
        if (!cached && ob + q.n > maxn) fits = false;
        for (int k = tid; k < q.n; k += WGS) {
          const int e = part_esum(q, k, RS);
          if (e != HZ) {
            mn[f] = min(mn[f], e);
            mx[f] = max(mx[f], e);
          }
        }
        if (!cached) ob += (q.n + 15) & ~15;
      }
    }
    // workgroup min / max by LDS atomics on red (reset after every use)
    if (mn[f] <= mx[f]) {
      __hip_atomic_fetch_min((l_i32 *)red + 2 * f, mn[f], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
      __hip_atomic_fetch_max((l_i32 *)red + 2 * f + 1, mx[f], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
    }
  }
  __syncthreads();
  if (tid < nf) {
    const int f = tid;
    const int a = ((const l_i32 *)red)[2 * f], b = ((const l_i32 *)red)[2 * f + 1];
    const FrameSrc src = lds_get(fs + f);
    lds_put(fd + f, make_desc(src.n, src.fbase, src.mlo, src.mhi, a, b, nd, err));
  }
  if (tid == 0 && !fits) atomicOr(err, 8u);  // table too small: never expected
  __syncthreads();
  red_reset(red);
  if (ob == 0 || !fits) return;
  ob = 0;
  for (int f = 0; f < nf; ++f) {
    const int base = fd[f].base, S = fd[f].S;
    for (int j = 0; j < fs[f].nparts; ++j) {
      FramePart &q = fs[f].p[j];
      if (q.hU && q.hV) continue;
      for (int k = tid; k < q.n; k += WGS) {
        const int e = part_esum(q, k, RS);
        ((l_i8 *)offs)[ob + k] = (int8_t)(e == HZ ? 0 : min(max(e - base, 0), S));
      }
      if (tid == 0) q.ot = offs + ob;
      ob += (q.n + 15) & ~15;
    }
  }
  __syncthreads();
}

// Descriptor of the one-term frame U V whose rows are in LDS (the Horner
// and adjoint power products), from the two row headers.
__device__ __forceinline__ FrameD single_desc(const int32_t *U_, const int32_t *V_, int nd) {
  const l_i32 *U = (const l_i32 *)U_, *V = (const l_i32 *)V_;
  const int MT = (nd + TQ - 1) / TQ;
  FrameD d;
  const int e = (U[1] != 0 && V[1] != 0) ? U[0] + V[0] : HZ;
  d.n = 1;
  d.nz = e != HZ ? 1 : 0;
  d.base = d.nz ? e : 0;
  d.S = 0;
  d.NT = MT;
  d.mt0 = 0;
  d.MTf = MT;
  d.nt0 = 0;
  return d;
}

// Columns spanned by frame f's tiles: [0, (MT + NT) * 8 + 8).
__device__ __forceinline__ int frame_cols(const FrameD &d, int nd) {
  int MT = (nd + TQ - 1) / TQ;
  return (MT + d.nt0 + d.NT) * TQ + TQ;
}

__device__ __forceinline__ void tile_load_g(int32_t (&uu)[TQ], int32_t (&vv)[TQ], const g_i32 *U,
                                            const g_i32 *V, int mt, int nt, int off) {
  const g_i32 *u = U + HDR + RPAD + mt * TQ;
  const g_i32 *v = V + HDR + RPAD + nt * TQ - off;
#pragma unroll
  for (int r = 0; r < TQ; ++r) uu[r] = u[r];
#pragma unroll
  for (int r = 0; r < TQ; ++r) vv[r] = v[r];
}

__device__ __forceinline__ void tile_fma(long long (&acc)[16], const int32_t (&uu)[TQ],
                                         const int32_t (&vv)[TQ]) {
#pragma unroll
  for (int r = 0; r < TQ; ++r)
#pragma unroll
    for (int s = 0; s < TQ; ++s) acc[r + s] += (long long)uu[r] * (long long)vv[s];
}

__device__ __forceinline__ void acc_flush(long long (&acc)[16], long long *col) {
  tile_normalize(acc);
  l_i64 *c = (l_i64 *)col;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    if (acc[r] != 0) __hip_atomic_fetch_add((unsigned long long __attribute__((address_space(3))) *)(c + r),
                                            (unsigned long long)acc[r], __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_WORKGROUP);
    acc[r] = 0;
  }
}

// Terms per batch of the product loop: the digits of one batch are loaded
// while the previous batch's products are formed.
constexpr int PB = 4;
// Cost of a tile's own segment in the work partition, in terms.
constexpr int TILE_OVH = 6;

// Digits of term k of part pt for tile (mt, nt); the term's offset comes
// from the part's table (TAB) or from its exponent caches (LDS either way).
template <bool TAB>
__device__ __forceinline__ void term_load(int32_t (&u)[TQ], int32_t (&v)[TQ], const FramePart &pt,
                                          int k, int RS, int mt, int nt, int base, int S) {
  int iu, iv;
  part_rows(pt, k, &iu, &iv);
  const g_i32 *U = (const g_i32 *)pt.U + iu * RS, *V = (const g_i32 *)pt.V + iv * RS;
  int off;
  if (TAB) {
    off = ((const l_i8 *)pt.ot)[k];
  } else {
    const int eu = ((const l_i32 *)pt.hU)[iu], ev = ((const l_i32 *)pt.hV)[iv];
    off = (eu == HZ || ev == HZ) ? 0 : min(max(eu + ev - base, 0), S);
  }
  tile_load_g(u, v, U, V, mt, nt, off);
}

// Terms [k0, k1) of part pt (rows in global memory) into the 16 column sums
// of tile (mt, nt).  Two register batches of PB terms alternate: one is
// being loaded while the other's products are formed.  Loads are issued
// unconditionally (past the end they repeat the last term, whose products
// are then skipped), so that each wait covers exactly the batch it needs.
// The sums are carry-normalised after every 2 PB terms (2 PB <= FLUSH_TERMS
// keeps them inside 64 bits).
template <bool TAB>
__device__ __forceinline__ void part_tile_terms_t(long long (&acc)[16], const FramePart &pt,
                                                  int k0, int k1, int RS, int mt, int nt,
                                                  int base, int S) {
  int32_t ua[PB][TQ], va[PB][TQ], ub[PB][TQ], vb[PB][TQ];
  const int kl = k1 - 1;
#pragma unroll
  for (int j = 0; j < PB; ++j) term_load<TAB>(ua[j], va[j], pt, min(k0 + j, kl), RS, mt, nt, base, S);
  for (int k = k0; k < k1; k += 2 * PB) {
#pragma unroll
    for (int j = 0; j < PB; ++j)
      term_load<TAB>(ub[j], vb[j], pt, min(k + PB + j, kl), RS, mt, nt, base, S);
#pragma unroll
    for (int j = 0; j < PB; ++j)
      if (k + j < k1) tile_fma(acc, ua[j], va[j]);
#pragma unroll
    for (int j = 0; j < PB; ++j)
      term_load<TAB>(ua[j], va[j], pt, min(k + 2 * PB + j, kl), RS, mt, nt, base, S);
#pragma unroll
    for (int j = 0; j < PB; ++j)
      if (k + PB + j < k1) tile_fma(acc, ub[j], vb[j]);
    tile_normalize(acc);
  }
}

__device__ __forceinline__ void part_tile_terms(long long (&acc)[16], const FramePart &pt,
                                                int k0, int k1, int RS, int mt, int nt,
                                                int base, int S) {
  if (pt.ot) part_tile_terms_t<true>(acc, pt, k0, k1, RS, mt, nt, base, S);
  else if (pt.hU && pt.hV) part_tile_terms_t<false>(acc, pt, k0, k1, RS, mt, nt, base, S);
  // else: no offsets (a flagged table overflow); the frame is already wrong
}

// The workgroup `rank` of `G` accumulates its share of all frames' tiles
// into the LDS column arrays lf[f * WB + c]; every row is in global memory.
//
// With G a multiple of 8 (G >= 16) the group is split into 8 term groups,
// workgroup r in group r mod 8 (consecutive workgroups are dispatched to
// different XCDs, so a term group is one XCD's share): term group x takes
// the terms [n x / 8, n (x + 1) / 8) of every frame, so the rows it reads
// stay in its own L2.  Within a term group, the tiles (all of the group's
// terms each) are dealt to workgroups in contiguous ranges (anti-diagonal
// order) of equal cost.  Inside the workgroup the (tile, term) pairs are
// split evenly over the threads in tile-major order, so a thread walks
// consecutive terms of consecutive tiles; it keeps its 16 column sums in
// registers while it stays on one anti-diagonal and adds them into LDS
// when it leaves it.  Returns through span[2f], span[2f+1] the column range
// this workgroup touched in frame f (empty: lo >= hi).
__device__ __forceinline__ void frames_accumulate(const FrameSrc *fs_, const FrameD *fd_, int nf,
                                                  int nd, int RS,
                                  int WB, long long *lf, int rank, int G, int *span_,
                                  bool skip0 = false, unsigned long long *tprof = nullptr,
                                  unsigned long long *tmax = nullptr) {
  const int tid = threadIdx.x;
  const unsigned long long tp0 = tprof ? wall_clock64() : 0;
  // the descriptors live in LDS: read them as such (no flat accesses here)
  const l_FrameSrc *fs = (const l_FrameSrc *)fs_;
  const l_FrameD *fd = (const l_FrameD *)fd_;
  l_i32 *span = (l_i32 *)span_;
  const int X = (G >= 16 && (G & 7) == 0) ? 8 : 1;
  const int xg = rank % X;
  int sub = rank / X, GS = G / X;
  // skip0: workgroup 0 takes no share (the others split the work)
  int srank = rank, sG = G;
  if (skip0) {
    if (X == 1) {
      sub = rank - 1;
      GS = G - 1;
    } else if (xg == 0) {
      sub -= 1;
      GS -= 1;
    }
    srank = rank - 1;
    sG = G - 1;
  }
  // (tile, term) items of this term group: fewer than 2^31 for every
  // supported size, so the partition runs in 32-bit arithmetic
  // Frames with fewer terms than term groups (the single products of the
  // newest rows) are not split by terms: their tiles are dealt over all G
  // workgroups, one tile range each, apart from the term groups' shares.
  int ka[NFR], len[NFR], t0[NFR], t1[NFR];
  bool small[NFR];
  unsigned C = 0, Cs = 0;
#pragma unroll
  for (int f = 0; f < NFR; ++f) {
    ka[f] = len[f] = 0;
    small[f] = false;
    if (f >= nf || !fd[f].nz) continue;
    const unsigned n = (unsigned)fd[f].n;
    if (X > 1 && n < (unsigned)X) {
      small[f] = true;
      len[f] = (int)n;
      Cs += (unsigned)(fd[f].MTf * fd[f].NT);
      continue;
    }
    ka[f] = (int)(n * xg / X);
    len[f] = (int)(n * (xg + 1) / X) - ka[f];
    if (len[f] > 0) C += (unsigned)(fd[f].MTf * fd[f].NT) * (unsigned)(len[f] + TILE_OVH);
  }
  const unsigned cq = C / GS, cr = C - cq * GS;
  const unsigned lo = cq * sub + cr * sub / GS, hi = cq * (sub + 1) + cr * (sub + 1) / GS;
  const unsigned sq = Cs / sG, sr = Cs - sq * sG;
  const unsigned slo = sq * srank + sr * srank / sG, shi = sq * (srank + 1) + sr * (srank + 1) / sG;
  unsigned pre = 0, spre = 0, w = 0;
#pragma unroll
  for (int f = 0; f < NFR; ++f) {
    t0[f] = t1[f] = 0;
    if (f >= nf || len[f] == 0) continue;
    const unsigned n = (unsigned)len[f];
    const unsigned T = (unsigned)(fd[f].MTf * fd[f].NT);
    unsigned ta, tb;
    if (small[f]) {
      ta = slo <= spre ? 0u : slo - spre;
      tb = shi <= spre ? 0u : shi - spre;
      spre += T;
    } else {
      // a tile of this group costs its terms plus a fixed overhead (its own
      // segment: coordinates, first loads, flush)
      const unsigned nc = n + TILE_OVH;
      ta = lo <= pre ? 0u : (lo - pre + nc - 1) / nc;
      tb = hi <= pre ? 0u : (hi - pre + nc - 1) / nc;
      pre += T * nc;
    }
    if (ta > T) ta = T;
    if (tb > T) tb = T;
    t0[f] = (int)ta;
    t1[f] = (int)tb;
    w += (tb - ta) * n;
  }
  if (tid < 2 * nf) span[tid] = 0;
  __syncthreads();
  unsigned long long tp1 = 0;
  if (tprof) {
    tp1 = wall_clock64();
    if (tid == 0) atomicAdd(tprof, tp1 - tp0);  // partition (thread 0)
  }
  if (skip0 && rank == 0) return;
  if (tid < nf) {
    const int f = tid;
    if (t1[f] > t0[f]) {
      int mt, nt;
      tile_coords(t0[f], fd[f].MTf, fd[f].NT, &mt, &nt);
      int dlo = mt + nt + fd[f].mt0 + fd[f].nt0;
      tile_coords(t1[f] - 1, fd[f].MTf, fd[f].NT, &mt, &nt);
      int dhi = mt + nt + fd[f].mt0 + fd[f].nt0;
      span[2 * f] = min(dlo, dhi) * TQ;
      span[2 * f + 1] = max(dlo, dhi) * TQ + 2 * TQ;
    }
  }
  if (w == 0) return;
  unsigned q = (unsigned)(((unsigned long long)w * tid) / WGS);
  const unsigned qend = (unsigned)(((unsigned long long)w * (tid + 1)) / WGS);
  long long acc[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0;
  int cur_f = -1, cur_d = -1;
  int f = 0;
  unsigned fstart = 0;  // first item of frame f in the workgroup's list
  while (q < qend) {
    // frame of item q
    while (f < nf && q >= fstart + (unsigned)(t1[f] - t0[f]) * (unsigned)len[f]) {
      fstart += (unsigned)(t1[f] - t0[f]) * (unsigned)len[f];
      ++f;
    }
    const unsigned n = (unsigned)len[f];
    const unsigned rel = q - fstart;
    const unsigned tr = rel / n;
    const int t = t0[f] + (int)tr;
    const int kk0 = (int)(rel - tr * n);
    const unsigned seg_end = min(qend, fstart + (tr + 1) * n);
    int mt, nt;
    tile_coords(t, fd[f].MTf, fd[f].NT, &mt, &nt);
    mt += fd[f].mt0;
    nt += fd[f].nt0;
    const int d = mt + nt;
    if (f != cur_f || d != cur_d) {
      if (cur_f >= 0) acc_flush(acc, lf + (size_t)cur_f * WB + cur_d * TQ);
      cur_f = f;
      cur_d = d;
    }
    // frame terms [k, k1), walked part by part
    const l_FrameSrc &src = fs[f];
    const int nparts = src.nparts, fbase = fd[f].base, fS = fd[f].S;
    int k = ka[f] + kk0;
    const int k1 = k + (int)(seg_end - q);
    int j = 0, pbase = 0;
    while (k < k1) {
      while (j + 1 < nparts && k >= pbase + src.p[j].n) {
        pbase += src.p[j].n;
        ++j;
      }
      FramePart pt;
      pt.kind = src.p[j].kind;
      pt.n = src.p[j].n;
      pt.idx = src.p[j].idx;
      pt.pad = 0;
      pt.U = src.p[j].U;
      pt.V = src.p[j].V;
      pt.hU = src.p[j].hU;
      pt.hV = src.p[j].hV;
      pt.ot = src.p[j].ot;
      const int kend = min(k1, pbase + pt.n);
      part_tile_terms(acc, pt, k - pbase, kend - pbase, RS, mt, nt, fbase, fS);
      k = kend;
    }
    q = seg_end;
  }
  if (cur_f >= 0) acc_flush(acc, lf + (size_t)cur_f * WB + cur_d * TQ);
  if (tprof)
    __hip_atomic_fetch_max((unsigned long long __attribute__((address_space(3))) *)tmax,
                           wall_clock64() - tp1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

typedef int v4i __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) v4i l_v4i;

// Sum over each aligned group of 4 lanes, in the group's last lane (row
// shifts by 1 and 2 lanes: an inclusive scan over 4 lanes).  Every lane of
// the wavefront must be active.
__device__ __forceinline__ uint32_t dpp_sum4(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, true);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, true);
  return x;
}
template <int CTRL>
__device__ __forceinline__ long long dpp_shr_add64(long long v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, 0xf, 0xf, true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(
      0, (int)(uint32_t)((unsigned long long)v >> 32), CTRL, 0xf, 0xf, true);
  return v + (long long)(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ long long dpp_sum4_64(long long v) {
  return dpp_shr_add64<0x112>(dpp_shr_add64<0x111>(v));
}

// One-term frames f = 0..nf-1, U times the row V0 + f vstride, all in LDS
// (the Horner and adjoint power chains), computed by the whole workgroup
// into lf[f * WB + c]: each anti-diagonal of tiles goes to an aligned
// group of 4 lanes, lane c taking the tiles c, c + 4, ... of it (61
// diagonals at K=2000 fill one pass of the workgroup); the 4 run sums are
// added across the group in registers and one lane adds them into LDS, so
// no two lanes of a wavefront add into the same column at once.
__device__ void lds_products(const int32_t *U_, const int32_t *V0, int vstride, int nf, int nd,
                             int WB, long long *lf) {
  const int tid = threadIdx.x;
  const int MT = (nd + TQ - 1) / TQ;
  const int ND = 2 * MT - 1;                 // anti-diagonals
  const int slots = ND * 4;
  for (int f = 0; f < nf; ++f) {
    const l_i32 *Uh = (const l_i32 *)U_, *Vh = (const l_i32 *)(V0 + (size_t)f * vstride);
    if (Uh[1] == 0 || Vh[1] == 0) continue;  // a zero row: no products
    const l_i32 *U = Uh + HDR + RPAD;
    const l_i32 *V = Vh + HDR + RPAD;
    for (int sl0 = 0; sl0 < slots; sl0 += WGS) {
      const int sl = sl0 + tid;
      const int d = sl >> 2, c = sl & 3;
      const int mlo = d - MT + 1 > 0 ? d - MT + 1 : 0;
      const int mhi = d < ND ? (d < MT - 1 ? d : MT - 1) : -1;
      long long acc[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[r] = 0;
      for (int mt = mlo + c; mt <= mhi; mt += 4) {
        const int nt = d - mt;
        // 16-byte LDS reads: the rows' digits start 16-byte aligned
        const l_v4i *u4 = (const l_v4i *)(U + mt * TQ), *v4 = (const l_v4i *)(V + nt * TQ);
        const v4i ua = u4[0], ub = u4[1], va = v4[0], vb = v4[1];
        const int32_t uu[TQ] = {ua.x, ua.y, ua.z, ua.w, ub.x, ub.y, ub.z, ub.w};
        const int32_t vv[TQ] = {va.x, va.y, va.z, va.w, vb.x, vb.y, vb.z, vb.w};
        tile_fma(acc, uu, vv);
      }
      tile_normalize(acc);  // columns 0..14 in [0, 2^28): their 4-lane sums fit 32 bits
      uint32_t s32[15];
#pragma unroll
      for (int r = 0; r < 15; ++r) s32[r] = dpp_sum4((uint32_t)acc[r]);
      const long long top = dpp_sum4_64(acc[15]);
      if (c == 3 && d < ND) {
        l_i64 *col = (l_i64 *)lf + (size_t)f * WB + d * TQ;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const long long v = r < 15 ? (long long)s32[r] : top;
          if (v != 0)
            __hip_atomic_fetch_add((unsigned long long __attribute__((address_space(3))) *)(col + r),
                                   (unsigned long long)v, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
    }
  }
}

}  // namespace mpts
