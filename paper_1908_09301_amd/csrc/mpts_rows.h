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
};

struct FrameSrc {
  int nparts, n;  // n = total terms
  FramePart p[4];
};

struct FrameD {
  int n, base, S, NT, nz, obase;  // obase: first entry of this frame's offset slice
  long long cost0;                // first cost unit of this frame
};

__device__ __forceinline__ void part_term(const FramePart &q, int k, int RS, const int32_t **U,
                                          const int32_t **V) {
  switch (q.kind) {
    case PK_CAUCHY:
      *U = q.U + (long long)(q.idx - k) * RS;
      *V = q.V + (long long)k * RS;
      break;
    case PK_CORR:
      *U = q.U + (long long)(q.idx + k) * RS;
      *V = q.V + (long long)k * RS;
      break;
    case PK_DOT:
      *U = q.U + (long long)k * RS;
      *V = q.V + (long long)k * RS;
      break;
    default:
      *U = q.U;
      *V = q.V;
  }
}

__device__ __forceinline__ void frame_term(const FrameSrc &f, int k, int RS, const int32_t **U,
                                           const int32_t **V) {
  int j = 0;
  while (j + 1 < f.nparts && k >= f.p[j].n) {
    k -= f.p[j].n;
    ++j;
  }
  part_term(f.p[j], k, RS, U, V);
}

__host__ __device__ inline FramePart mk_part(int kind, int n, int idx, const int32_t *U,
                                             const int32_t *V) {
  FramePart q;
  q.kind = kind;
  q.n = n;
  q.idx = idx;
  q.pad = 0;
  q.U = U;
  q.V = V;
  return q;
}

__host__ __device__ inline FrameSrc mk_frame1(FramePart a) {
  FrameSrc f;
  f.nparts = 1;
  f.n = a.n;
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

// Per-workgroup frame setup: exponent base and spread of each frame's
// nonzero terms (one workgroup reduction for all frames), and the table of
// per-term digit offsets offs[obase_f + k] (0 for zero terms, whose rows
// are all-zero digits).  Every thread of the workgroup calls this.
// red: 4 waves x 2 NFR ints.
__device__ void frame_setup(const FrameSrc *fs, FrameD *fd, int nf, int nd, int RS, int *red,
                            int8_t *offs, int maxn, int *esum, int esum_cap, uint32_t *err) {
  const int tid = threadIdx.x;
  const int MT = (nd + TQ - 1) / TQ;
  int mn[NFR], mx[NFR];
  // one pass over the row headers: exponent sums kept in LDS (esum, laid
  // out frame after frame; INT_MIN marks a zero term) for the offset pass
  int eb = 0;
#pragma unroll
  for (int f = 0; f < NFR; ++f) {
    mn[f] = 0x7fffffff;
    mx[f] = -0x7fffffff;
    if (f < nf) {
      const bool keep = eb + fs[f].n <= esum_cap;
      for (int k = tid; k < fs[f].n; k += WGS) {
        const int32_t *U, *V;
        frame_term(fs[f], k, RS, &U, &V);
        int e = (int)0x80000000;
        if (U[1] != 0 && V[1] != 0) {
          e = U[0] + V[0];
          mn[f] = min(mn[f], e);
          mx[f] = max(mx[f], e);
        }
        if (keep) esum[eb + k] = e;
      }
      eb += fs[f].n;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      mn[f] = min(mn[f], __shfl_xor(mn[f], o, 64));
      mx[f] = max(mx[f], __shfl_xor(mx[f], o, 64));
    }
    if ((tid & 63) == 0) {
      red[(tid >> 6) * 2 * NFR + 2 * f] = mn[f];
      red[(tid >> 6) * 2 * NFR + 2 * f + 1] = mx[f];
    }
  }
  __syncthreads();
  if (tid < nf) {
    const int f = tid;
    int a = red[2 * f], b = red[2 * f + 1];
    for (int w = 1; w < WGS / 64; ++w) {
      a = min(a, red[w * 2 * NFR + 2 * f]);
      b = max(b, red[w * 2 * NFR + 2 * f + 1]);
    }
    FrameD d;
    d.n = fs[f].n;
    d.nz = (a <= b) ? 1 : 0;
    d.base = d.nz ? a : 0;
    int S = d.nz ? (b - a) : 0;
    if (S > SMAX) {
      atomicOr(err, 1u);
      S = SMAX;
    }
    d.S = S;
    d.NT = (nd + S + TQ - 1) / TQ;
    d.obase = 0;
    fd[f] = d;
  }
  __syncthreads();
  if (tid == 0) {
    long long c = 0;
    int ob = 0;
    for (int f = 0; f < nf; ++f) {
      fd[f].cost0 = c;
      if (fd[f].nz) c += (long long)MT * fd[f].NT * fd[f].n;
      fd[f].obase = ob;
      ob += (fs[f].n + 15) & ~15;
    }
    fd[nf].cost0 = c;
    if (ob > maxn) {  // cannot happen for the frames built here; never write past the table
      atomicOr(err, 1u);
      for (int f = 0; f <= nf; ++f) fd[f].cost0 = 0;
    }
  }
  __syncthreads();
  eb = 0;
  for (int f = 0; f < nf; ++f) {
    const int base = fd[f].base, S = fd[f].S;
    const bool keep = eb + fs[f].n <= esum_cap;
    if (fd[f].obase + fs[f].n <= maxn) {
      for (int k = tid; k < fs[f].n; k += WGS) {
        int e;
        if (keep) {
          e = esum[eb + k];
        } else {
          const int32_t *U, *V;
          frame_term(fs[f], k, RS, &U, &V);
          e = (U[1] != 0 && V[1] != 0) ? U[0] + V[0] : (int)0x80000000;
        }
        int off = 0;
        if (e != (int)0x80000000) {
          off = e - base;
          if (off < 0 || off > S) off = 0;  // only after a spread error (already flagged)
        }
        offs[fd[f].obase + k] = (int8_t)off;
      }
    }
    eb += fs[f].n;
  }
  __syncthreads();
}

// Frame setup for frames of exactly one term each (the Horner products):
// thread 0 only, no workgroup reduction.
__device__ void frame_setup_single(const FrameSrc *fs, FrameD *fd, int nf, int nd,
                                   int8_t *offs, int maxn) {
  const int MT = (nd + TQ - 1) / TQ;
  long long c = 0;
  for (int f = 0; f < nf; ++f) {
    FrameD d;
    const int32_t *U = fs[f].p[0].U, *V = fs[f].p[0].V;
    d.n = 1;
    d.nz = (U[1] != 0 && V[1] != 0) ? 1 : 0;
    d.base = d.nz ? U[0] + V[0] : 0;
    d.S = 0;
    d.NT = MT;
    d.obase = 16 * f;
    d.cost0 = c;
    if (d.nz) c += (long long)MT * MT;
    fd[f] = d;
    offs[16 * f] = 0;
  }
  fd[nf].cost0 = c;
}

// Columns spanned by frame f's tiles: [0, (MT + NT) * 8 + 8).
__device__ __forceinline__ int frame_cols(const FrameD &d, int nd) {
  int MT = (nd + TQ - 1) / TQ;
  return (MT + d.NT) * TQ + TQ;
}

__device__ __forceinline__ void tile_load(int32_t (&uu)[TQ], int32_t (&vv)[TQ], const int32_t *U,
                                          const int32_t *V, int mt, int nt, int off) {
  const int32_t *u = U + HDR + RPAD + mt * TQ;
  const int32_t *v = V + HDR + RPAD + nt * TQ - off;
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
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    if (acc[r] != 0) atomicAdd((unsigned long long *)(col + r), (unsigned long long)acc[r]);
    acc[r] = 0;
  }
}

// The workgroup `rank` of `G` accumulates its share of all frames' tiles
// into the LDS column arrays lf[f * WB + c].  Tiles are dealt to workgroups
// in contiguous ranges (anti-diagonal order) of equal cost (tiles x terms).
// Inside the workgroup the (tile, term) pairs are split evenly over the
// threads in tile-major order, so a thread walks consecutive terms of
// consecutive tiles; it keeps its 16 column sums in registers while it stays
// on one anti-diagonal and adds them into LDS when it leaves it.  The next
// term's digits are loaded before the current term's products are formed.
// Returns through span[2f], span[2f+1] the column range this workgroup
// touched in frame f (empty: lo >= hi).
__device__ void frames_accumulate(const FrameSrc *fs, const FrameD *fd, int nf, int nd, int RS,
                                  int WB, long long *lf, int rank, int G, int *span,
                                  const int8_t *offs, int maxn) {
  const int tid = threadIdx.x;
  const int MT = (nd + TQ - 1) / TQ;
  const long long C = fd[nf].cost0;
  const long long lo = C * rank / G, hi = C * (rank + 1) / G;
  int t0[NFR], t1[NFR];
  long long w = 0;
#pragma unroll
  for (int f = 0; f < NFR; ++f) {
    t0[f] = t1[f] = 0;
    if (f >= nf || !fd[f].nz || fd[f].n == 0) continue;
    long long pre = fd[f].cost0;
    long long n = fd[f].n;
    long long T = (long long)MT * fd[f].NT;
    long long a = lo - pre, b = hi - pre;
    long long ta = a <= 0 ? 0 : (a + n - 1) / n;
    long long tb = b <= 0 ? 0 : (b + n - 1) / n;
    if (ta > T) ta = T;
    if (tb > T) tb = T;
    t0[f] = (int)ta;
    t1[f] = (int)tb;
    w += (tb - ta) * n;
  }
  if (tid < 2 * nf) span[tid] = 0;
  __syncthreads();
  if (tid < nf) {
    const int f = tid;
    if (t1[f] > t0[f]) {
      int mt, nt;
      tile_coords(t0[f], MT, fd[f].NT, &mt, &nt);
      int dlo = mt + nt;
      tile_coords(t1[f] - 1, MT, fd[f].NT, &mt, &nt);
      int dhi = mt + nt;
      span[2 * f] = min(dlo, dhi) * TQ;
      span[2 * f + 1] = max(dlo, dhi) * TQ + 2 * TQ;
    }
  }
  if (w == 0) return;
  long long q = w * tid / WGS;
  const long long qend = w * (tid + 1) / WGS;
  long long acc[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0;
  int cur_f = -1, cur_d = -1;
  int since = 0;
  int f = 0;
  long long fstart = 0;  // first item of frame f in the workgroup's list
  while (q < qend) {
    // frame of item q
    while (f < nf && q >= fstart + (long long)(t1[f] - t0[f]) * fd[f].n) {
      fstart += (long long)(t1[f] - t0[f]) * fd[f].n;
      ++f;
    }
    const int n = fd[f].n;
    const long long rel = q - fstart;
    const int t = t0[f] + (int)(rel / n);
    const int k0 = (int)(rel % n);
    const long long seg_end = min(qend, fstart + (long long)(t - t0[f] + 1) * n);
    const int k1 = k0 + (int)(seg_end - q);
    int mt, nt;
    tile_coords(t, MT, fd[f].NT, &mt, &nt);
    const int d = mt + nt;
    if (f != cur_f || d != cur_d) {
      if (cur_f >= 0) acc_flush(acc, lf + (size_t)cur_f * WB + cur_d * TQ);
      cur_f = f;
      cur_d = d;
      since = 0;
    }
    const int8_t *of = offs + fd[f].obase;
    const int Sf = fd[f].S;
    const FrameSrc &src = fs[f];
    // walk the segment part by part with pointer strides (no per-term dispatch)
    int k = k0;
    while (k < k1) {
      int j = 0, kl = k;
      while (j + 1 < src.nparts && kl >= src.p[j].n) {
        kl -= src.p[j].n;
        ++j;
      }
      const FramePart &pt = src.p[j];
      const int kend = min(k1, k - kl + pt.n);
      const int32_t *U, *V;
      part_term(pt, kl, RS, &U, &V);
      const long long dU = pt.kind == PK_CAUCHY ? -(long long)RS : (pt.kind == PK_ONE ? 0 : RS);
      const long long dV = pt.kind == PK_ONE ? 0 : RS;
      int32_t ua[TQ], va[TQ], ub[TQ], vb[TQ];
      tile_load(ua, va, U, V, mt, nt, min(max((int)of[k], 0), Sf));
      while (k < kend) {
        if (k + 1 < kend) {
          U += dU;
          V += dV;
          tile_load(ub, vb, U, V, mt, nt, min(max((int)of[k + 1], 0), Sf));
        }
        tile_fma(acc, ua, va);
        if (++since == FLUSH_TERMS) {
          tile_normalize(acc);
          since = 0;
        }
        ++k;
        if (k >= kend) break;
        if (k + 1 < kend) {
          U += dU;
          V += dV;
          tile_load(ua, va, U, V, mt, nt, min(max((int)of[k + 1], 0), Sf));
        }
        tile_fma(acc, ub, vb);
        if (++since == FLUSH_TERMS) {
          tile_normalize(acc);
          since = 0;
        }
        ++k;
      }
    }
    q = seg_end;
  }
  if (cur_f >= 0) acc_flush(acc, lf + (size_t)cur_f * WB + cur_d * TQ);
}

}  // namespace mpts
