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
#include "mpts_rows.h"
#include "mpts_kernels.h"

namespace mpts {

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct Addend {
  const int32_t *p;  // row (is_row) or normalised value [sign, E, M]
  int is_row;
  int sgn;
};

// Exact sum of one product frame (columns from global memory or LDS) and up
// to three addends, resolved into sign and magnitude digits dig[0..64C).
// Each lane gathers its own chunk of columns straight into registers.
// Single wavefront.
template <int CM>
__device__ int combine_resolve(const long long *frame, bool frame_global, const FrameD *fd,
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
    if (adds[a].is_row) {
      e = adds[a].p[0];
      s = adds[a].p[1];
    } else {
      s = adds[a].p[0];
      e = floordiv28(adds[a].p[1], &ash[a]);
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
#pragma unroll
      for (int j = 0; j < CM; ++j) {
        if (j >= Cc) break;
        int fc = c0 + j - o;
        if (fc >= 0 && fc < fcols) v[j] = frame[fc];
      }
    }
  }
  for (int a = 0; a < nadd; ++a) {
    if (as[a] == 0) continue;
    const int o = (int)(ae[a] - lo);
    const long long sg = adds[a].sgn;
    if (adds[a].is_row) {
      const int32_t *row = adds[a].p + HDR + RPAD;
#pragma unroll
      for (int j = 0; j < CM; ++j) {
        if (j >= Cc) break;
        int k = c0 + j - o;
        if (k >= 0 && k < nd) v[j] += sg * row[k];
      }
    } else {
      const long long sgs = sg * as[a];
#pragma unroll
      for (int j = 0; j < CM; ++j) {
        if (j >= Cc) break;
        int k = c0 + j - o;
        if (k >= 0 && k < nd) v[j] += sgs * (long long)mant_bits28(adds[a].p + 2, L, (long long)DBITS * k - ash[a]);
      }
    }
  }
  bool ovf = false;
  int sgn = wave_resolve_regs<CM>(v, Cc, dig, &ovf);
  if (ovf && lane == 0) atomicOr(err, 1u);
  *dexp = lo;
  return sgn;
}

struct Carve {
  long long *lf;       // NFR * WB frame columns
  long long *tcols;    // 3 task column / digit buffers, 64*CM each
  int32_t *tq;         // 3 task quotient buffers, 64*CM each
  int32_t *tnorm;      // 3 tasks x 2 normalised values, NV each
  int32_t *hrow;       // 4 LDS rows (3 Horner accumulators, tau)
  FrameSrc *fs;        // NFR
  FrameD *fd;          // NFR + 1
  int *red;            // 64
  int *span;           // 2 NFR
  int8_t *offs;        // NFR x maxn per-term digit offsets
  int maxn;
  int NV;
};

__device__ Carve carve(unsigned char *smem, const Inst &I) {
  Carve c;
  const int NV = (I.L + 2 + 3) & ~3;
  c.NV = NV;
  unsigned char *p = smem;
  c.lf = (long long *)p;
  p += (size_t)NFR * I.WB * 8;
  c.tcols = (long long *)p;
  p += (size_t)3 * 64 * I.CM * 8;
  c.tq = (int32_t *)p;
  p += (size_t)3 * 64 * I.CM * 4;
  c.tnorm = (int32_t *)p;
  p += (size_t)6 * NV * 4;
  c.hrow = (int32_t *)p;
  p += (size_t)4 * I.RS * 4;
  c.fs = (FrameSrc *)p;
  p += sizeof(FrameSrc) * NFR;
  c.fd = (FrameD *)p;
  p += sizeof(FrameD) * (NFR + 1);
  c.red = (int *)p;
  p += 64 * 4;
  c.span = (int *)p;
  p += 2 * NFR * 4;
  c.maxn = max_terms(I.N);
  c.offs = (int8_t *)p;
  return c;
}

size_t lds_bytes(int L, int N, int RS, int WB, int CM) {
  const int NV = (L + 2 + 3) & ~3;
  const int maxn = max_terms(N);
  size_t b = (size_t)NFR * WB * 8 + (size_t)3 * 64 * CM * 8 + (size_t)3 * 64 * CM * 4 +
             (size_t)6 * NV * 4 + (size_t)4 * RS * 4 + sizeof(FrameSrc) * NFR +
             sizeof(FrameD) * (NFR + 1) + 64 * 4 + 2 * NFR * 4 + (size_t)maxn;
  return (b + 255) & ~(size_t)255;
}

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

// Spin until *flag >= target (thread 0 only); gives up after ~2 s, marking
// the error word so that the host reports it instead of hanging.
__device__ void spin_until(uint32_t *flag, uint32_t target, uint32_t *err) {
  long long polls = 0;
  // device-coherent (sc1) plain loads: they see the other workgroups'
  // atomics without turning every poll into a write at the coherence point
  const __amdgpu_buffer_rsrc_t rs = dev_rsrc(flag, 4);
  while ((uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, 0, 0, 16) < target) {
    __builtin_amdgcn_s_sleep(2);
    if (++polls > (1LL << 25)) {
      atomicOr(err, 4u);
      break;
    }
  }
}

// One finalisation task (one wavefront): which = 0 -> beta_{i+1},
// 1 -> gamma_{i+1}, 2 -> alpha_{i+1}.
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
  const int L = I.L, nd = I.nd, WB = I.WB;
  long long *cols = cv.tcols + (size_t)which * 64 * I.CM;
  int32_t *dig = (int32_t *)cols;
  int32_t *q = cv.tq + (size_t)which * 64 * I.CM;
  int32_t *tmp = cv.tnorm + (size_t)which * 2 * cv.NV;
  int32_t *res = tmp + cv.NV;
  int C;
  long long dexp;
  int sgn;
  int arr_out;
  bool ok = true;
  if (which == 0 || which == 1) {
    // s1 (which 0) or s2 (which 1): one rounding of the exact Cauchy sum
    sgn = combine_resolve<CM>(frames + (size_t)which * WB, frames_global, &cv.fd[which], nd, L,
                              nullptr, 0, dig, &C, &dexp, err);
    sub(8);
    ok &= wave_round(dig, C, sgn, dexp, false, L, tmp);
    sub(9);
    Addend ad[2];
    int nad;
    const FrameD *fr;
    const long long *fp;
    if (which == 0) {
      // R a_i - b_i - s1_i (b_i: this wave's previous result, still in LDS)
      ad[0] = Addend{res, 0, -1};
      ad[1] = Addend{tmp, 0, -1};
      nad = 2;
      fr = &cv.fd[3];
      fp = frames + (size_t)3 * WB;
      arr_out = 1;
    } else {
      // s2_i - b g_i
      ad[0] = Addend{tmp, 0, 1};
      nad = 1;
      fr = &cv.fd[4];
      fp = frames + (size_t)4 * WB;
      arr_out = 2;
    }
    sgn = combine_resolve<CM>(fp, frames_global, fr, nd, L, ad, nad, dig, &C, &dexp, err);
    sub(10);
  } else {
    // sigma (b_i - a_i)
    sgn = combine_resolve<CM>(frames + (size_t)2 * WB, frames_global, &cv.fd[2], nd, L, nullptr,
                              0, dig, &C, &dexp, err);
    arr_out = 0;
  }
  ok &= wave_div_round<CM>(dig, C, sgn, dexp, i + 1, L, nd, q, res);
  sub(11);
  if (!ok && lane == 0) atomicOr(err, 2u);
  write_row(res, L, nd, I.RS, row_ptr(I, arr_out, i + 1), I.G > 1, lane, 64);
  sub(12);
  if (I.coefs)
    copy_norm(res, I.coefs + ((long long)arr_out * (I.N + 1) + i + 1) * (L + 2), L, false, lane,
              64);
}

// ---------------------------------------------------------------------------
// Group protocol: one coefficient (or adjoint) index at a time.
struct GroupSync {
  uint32_t gen;
  unsigned long long nbulk;
};

// Leader: after writing rows that the group will read, publish them.
// Followers: wait for that publication.
__device__ void group_publish(const Inst &I, bool leader, GroupSync &gs, uint32_t *err) {
  const int tid = threadIdx.x;
  if (leader) {
    wait_vmem();
    __syncthreads();
    ++gs.gen;
    if (I.G > 1 && tid == 0) st_relaxed(I.sync + SY_FLAG, gs.gen);
  } else {
    ++gs.gen;
    if (tid == 0) spin_until(I.sync + SY_FLAG, gs.gen, err);
    __syncthreads();
  }
}

// Every workgroup of the group: frame descriptors, this workgroup's share
// of the products into LDS, and (G > 1) the L2-bypassing atomic adds of
// its columns into the group's global frames.  The leader then waits for
// every workgroup's adds.  Returns the frames the leader finalises from.
__device__ const long long *group_bulk(const Inst &I, const Carve &cv, int nf, int rank,
                                       GroupSync &gs, uint32_t *err) {
  const int tid = threadIdx.x;
  const int G = I.G, WB = I.WB;
  // the task buffers are idle during the bulk: they hold the exponent sums
  frame_setup(cv.fs, cv.fd, nf, I.nd, I.RS, cv.red, cv.offs, cv.maxn, (int *)cv.tcols,
              3 * 64 * I.CM * 2, err);
  frames_accumulate(cv.fs, cv.fd, nf, I.nd, I.RS, WB, cv.lf, rank, G, cv.span, cv.offs, cv.maxn);
  __syncthreads();
  ++gs.nbulk;
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
  if (tid == 0)
    __hip_atomic_fetch_add(I.sync + SY_ARRIVE, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (rank == 0) {
    if (tid == 0) spin_until(I.sync + SY_ARRIVE, (uint32_t)(G * gs.nbulk), err);
    __syncthreads();
  }
  return gf;
}

// Leader: clear the frames it finalised from, then publish its new rows.
// Followers: wait for the publication.
__device__ void group_release(const Inst &I, const Carve &cv, int nf, bool leader,
                              const long long *frames, GroupSync &gs, uint32_t *err) {
  const int tid = threadIdx.x;
  if (leader) {
    __syncthreads();
    for (int f = 0; f < nf; ++f) {
      int nc = cv.fd[f].nz ? frame_cols(cv.fd[f], I.nd) : 0;
      long long *fr = const_cast<long long *>(frames) + (size_t)f * I.WB;
      for (int c = tid; c < nc; c += WGS) {
        if (I.G > 1) st_relaxed(fr + c, 0LL);
        else fr[c] = 0;
      }
    }
  }
  group_publish(I, leader, gs, err);
}

// Rows 0 of the three coefficient arrays from a normalised state, published
// to the group; then, once per step, drop cached copies of rows that are
// about to be rewritten.
__device__ void start_step(const Inst &I, bool leader, const int32_t *state, GroupSync &gs,
                           uint32_t *err) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  if (leader && wave < 3)
    write_row(state + (size_t)wave * (I.L + 2), I.L, I.nd, I.RS, row_ptr(I, wave, 0), I.G > 1,
              lane, 64);
  group_publish(I, leader, gs, err);
  if (I.G > 1) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    __syncthreads();
  }
}

// The Taylor coefficients 1..N of one step (equation (3)), rows 0 given.
template <int CM>
__device__ void forward_coefficients(const Inst &I, const Carve &cv, int rank, GroupSync &gs,
                                     const int32_t *state, uint32_t *err) {
  const int tid = threadIdx.x, wave = tid >> 6;
  const bool leader = rank == 0;
  const int RS = I.RS;
  // the beta task keeps b_i in LDS (its result slot): start with b_0
  if (leader && wave == 0)
    copy_norm(state + (I.L + 2), cv.tnorm + cv.NV, I.L, false, threadIdx.x & 63, 64);
  for (int i = 0; i < I.N; ++i) {
    if (tid == 0) {
      FrameSrc *fs = cv.fs;
      fs[0] = mk_frame1(mk_part(PK_CAUCHY, i + 1, i, row_ptr(I, 0, 0), row_ptr(I, 2, 0)));
      fs[1] = mk_frame1(mk_part(PK_CAUCHY, i + 1, i, row_ptr(I, 0, 0), row_ptr(I, 1, 0)));
      fs[2] = mk_frame2(mk_part(PK_ONE, 1, 0, I.consts + (size_t)C_SIGMA * RS, row_ptr(I, 1, i)),
                        mk_part(PK_ONE, 1, 0, I.consts + (size_t)C_NSIGMA * RS, row_ptr(I, 0, i)));
      fs[3] = mk_frame1(mk_part(PK_ONE, 1, 0, I.consts + (size_t)C_R * RS, row_ptr(I, 0, i)));
      fs[4] = mk_frame1(mk_part(PK_ONE, 1, 0, I.consts + (size_t)C_NB * RS, row_ptr(I, 2, i)));
    }
    __syncthreads();
    const long long *frames = group_bulk(I, cv, NFR, rank, gs, err);
    if (leader && wave < 3) finalize_task<CM>(I, cv, wave, i, frames, I.G > 1, err);
    group_release(I, cv, NFR, leader, frames, gs, err);
  }
}

// Three single-workgroup chains at once on the leader: h_c <- round(tau h_c
// + addend_c(i)) for `count` iterations.  h_c starts as the row start_c (an
// LDS row in cv.hrow[c] must already hold it).  Used for the Horner sums of
// equation (2) (addend: coefficient rows) and for the adjoint's powers of tau
// (no addend; each result row is also stored to out rows).
template <int CM>
__device__ void tau_chains(const Inst &I, const Carve &cv, int count, int mode, uint32_t *err) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int L = I.L, nd = I.nd, RS = I.RS, WB = I.WB, N = I.N;
  const int32_t *tau_lds = cv.hrow + (size_t)3 * RS;
  for (int it = 0; it < count; ++it) {
    if (tid == 0) {
      for (int c = 0; c < 3; ++c)
        cv.fs[c] = mk_frame1(mk_part(PK_ONE, 1, 0, tau_lds, cv.hrow + (size_t)c * RS));
      frame_setup_single(cv.fs, cv.fd, 3, nd, cv.offs, cv.maxn);
    }
    __syncthreads();
    frames_accumulate(cv.fs, cv.fd, 3, nd, RS, WB, cv.lf, 0, 1, cv.span, cv.offs, cv.maxn);
    __syncthreads();
    if (wave < 3) {
      int32_t *dig = (int32_t *)(cv.tcols + (size_t)wave * 64 * I.CM);
      int32_t *h = cv.tnorm + (size_t)wave * 2 * cv.NV;
      Addend ad;
      int nad = 0;
      if (mode == 0) {  // Horner: i = N-1-it
        ad = Addend{row_ptr(I, wave, N - 1 - it), 1, 1};
        nad = 1;
      }
      int C;
      long long dexp;
      int sgn = combine_resolve<CM>(cv.lf + (size_t)wave * WB, false, &cv.fd[wave], nd, L, &ad,
                                    nad, dig, &C, &dexp, err);
      bool ok = wave_round(dig, C, sgn, dexp, false, L, h);
      if (!ok && lane == 0) atomicOr(err, 2u);
      write_row(h, L, nd, RS, cv.hrow + (size_t)wave * RS, false, lane, 64);
      if (mode == 1) write_row(h, L, nd, RS, q_row(I, wave, it + 1), I.G > 1, lane, 64);
      int nc = cv.fd[wave].nz ? frame_cols(cv.fd[wave], nd) : 0;
      for (int c = lane; c < nc; c += 64) cv.lf[(size_t)wave * WB + c] = 0;
    }
    __syncthreads();
  }
}

template <int CM>
__global__ void __launch_bounds__(WGS) k_run(const Inst *__restrict__ insts,
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
  const bool timed = I.prof != nullptr && tid == 0 && (rank == 0 || rank == 1);
  unsigned long long *prof = timed ? I.prof + (rank == 0 ? 0 : PH_NPHASE) : nullptr;
  unsigned long long tp = timed ? wall_clock64() : 0;
  auto mark = [&](int phase) {
    if (timed) {
      unsigned long long t = wall_clock64();
      atomicAdd(prof + phase, t - tp);
      tp = t;
    }
  };
  if (leader) {
    for (int c = wave; c < NCONST; c += 4)
      write_row(I.cnorm + (size_t)c * (L + 2), L, nd, RS, I.consts + (size_t)c * RS, G > 1, lane,
                64);
  }
  __syncthreads();

  for (long long step = 0; step < I.nsteps; ++step) {
    if (leader && wave < 3) {
      const int32_t *sv = I.state + (size_t)wave * (L + 2);
      if (step == 0 && I.ckpt) copy_norm(sv, I.ckpt + (size_t)wave * (L + 2), L, false, lane, 64);
      if (I.coefs) copy_norm(sv, I.coefs + (size_t)wave * (N + 1) * (L + 2), L, false, lane, 64);
    }
    start_step(I, leader, I.state, gs, err);
    mark(PH_STEP0);
    forward_coefficients<CM>(I, cv, rank, gs, I.state, err);
    mark(PH_ACCUM);
    if (I.mode == MODE_COEFFS) break;
    // Horner: h = c_N; h <- round(h tau + c_i), i = N-1..0, three chains at once
    if (leader) {
      for (int j = tid; j < 4 * RS; j += WGS) {
        int c = j / RS, w = j - c * RS;
        cv.hrow[j] = c < 3 ? row_ptr(I, c, N)[w] : (I.consts + (size_t)C_TAU * RS)[w];
      }
      __syncthreads();
      tau_chains<CM>(I, cv, N, 0, err);
      if (wave < 3) {
        const int32_t *h = cv.tnorm + (size_t)wave * 2 * cv.NV;
        copy_norm(h, I.state + (size_t)wave * (L + 2), L, false, lane, 64);
        if (I.ckpt)
          copy_norm(h, I.ckpt + ((size_t)(step + 1) * 3 + wave) * (L + 2), L, false, lane, 64);
      }
      __syncthreads();
      mark(PH_HORNER);
    }
  }
}

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
  if (leader) {
    for (int c = wave; c < NCONST; c += 4)
      write_row(I.cnorm + (size_t)c * (L + 2), L, nd, RS, I.consts + (size_t)c * RS, rel, lane, 64);
    // seed: the adjoint of ||x(T)||^2 is 2 x(T) (exact); parameter adjoints 0
    if (wave < 3) {
      const int32_t *xT = I.ckpt + ((size_t)I.nsteps * 3 + wave) * (L + 2);
      int32_t *b = bar_ptr(I, wave);
      for (int j = lane; j < L + 2; j += 64) b[j] = (j == 1 && xT[0] != 0) ? xT[1] + 1 : xT[j];
      int32_t *pb = bar_ptr(I, 3 + wave);
      for (int j = lane; j < L + 2; j += 64) pb[j] = 0;
    }
  }
  __syncthreads();
  const int32_t *cs = I.consts;
  for (long long n = I.nsteps - 1; n >= 0; --n) {
    // 1. the step's coefficients from its checkpoint
    start_step(I, leader, I.ckpt + (size_t)n * 3 * (L + 2), gs, err);
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
        fs[0] = mk_frame4(mk_part(PK_CORR, k, m, adj_row(I, A_NV, 0), row_ptr(I, 2, 0)),
                          mk_part(PK_CORR, k, m, adj_row(I, A_W, 0), row_ptr(I, 1, 0)),
                          mk_part(PK_ONE, one, 0, cs + (size_t)C_NSIGMA * RS, adj_row(I, A_U, mi)),
                          mk_part(PK_ONE, one, 0, cs + (size_t)C_R * RS, adj_row(I, A_V, mi)));
        fs[1] = mk_frame2(mk_part(PK_CORR, k, m, adj_row(I, A_W, 0), row_ptr(I, 0, 0)),
                          mk_part(PK_ONE, one, 0, cs + (size_t)C_SIGMA * RS, adj_row(I, A_U, mi)));
        fs[2] = mk_frame2(mk_part(PK_CORR, k, m, adj_row(I, A_NV, 0), row_ptr(I, 0, 0)),
                          mk_part(PK_ONE, one, 0, cs + (size_t)C_NB * RS, adj_row(I, A_W, mi)));
      }
      __syncthreads();
      const long long *frames = group_bulk(I, cv, 3, rank, gs, err);
      if (leader && wave < 3) {
        int32_t *dig = (int32_t *)(cv.tcols + (size_t)wave * 64 * I.CM);
        int32_t *q = cv.tq + (size_t)wave * 64 * I.CM;
        int32_t *res = cv.tnorm + (size_t)wave * 2 * cv.NV;
        int32_t *out = res + cv.NV;
        Addend ad[2];
        int nad = 1;
        ad[0] = Addend{q_row(I, wave, m), 1, 1};
        if (wave == 1 && m < N) {
          ad[1] = Addend{adj_row(I, A_NV, m), 1, 1};
          nad = 2;
        }
        int C;
        long long dexp;
        int sgn = combine_resolve<CM>(frames + (size_t)wave * WB, rel, &cv.fd[wave], nd, L, ad, nad,
                                      dig, &C, &dexp, err);
        bool ok = wave_round(dig, C, sgn, dexp, false, L, res);
        if (m > 0) {
          Addend a1 = Addend{res, 0, 1};
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
      fs[0] = mk_frame2(mk_part(PK_DOT, N, 0, adj_row(I, A_U, 0), row_ptr(I, 1, 0)),
                        mk_part(PK_DOT, N, 0, adj_row(I, A_NU, 0), row_ptr(I, 0, 0)));
      fs[1] = mk_frame1(mk_part(PK_DOT, N, 0, adj_row(I, A_V, 0), row_ptr(I, 0, 0)));
      fs[2] = mk_frame1(mk_part(PK_DOT, N, 0, adj_row(I, A_NW, 0), row_ptr(I, 2, 0)));
    }
    __syncthreads();
    const long long *frames = group_bulk(I, cv, 3, rank, gs, err);
    if (leader && wave < 3) {
      int32_t *dig = (int32_t *)(cv.tcols + (size_t)wave * 64 * I.CM);
      int32_t *res = cv.tnorm + (size_t)wave * 2 * cv.NV;
      Addend ad = Addend{bar_ptr(I, 3 + wave), 0, 1};
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

__global__ void k_clear(uint32_t *p, size_t nwords) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < nwords; i += stride) p[i] = 0u;
}

template <int CM>
static hipError_t launch_cm(const Inst *d_insts, const int *d_wg_inst, int nwg, size_t lds,
                            hipStream_t s) {
  auto kern = k_run<CM>;
  hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  void *args[] = {(void *)&d_insts, (void *)&d_wg_inst};
  return hipLaunchCooperativeKernel((const void *)kern, dim3(nwg), dim3(WGS), args, (unsigned)lds,
                                    s);
}

template <int CM>
static hipError_t launch_cm_plain(const Inst *d_insts, const int *d_wg_inst, int nwg, size_t lds,
                                  hipStream_t s) {
  auto kern = k_run<CM>;
  hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(nwg), dim3(WGS), lds, s, d_insts, d_wg_inst);
  return hipGetLastError();
}

hipError_t launch_run(const Inst *d_insts, const int *d_wg_inst, int nwg, int CM, size_t lds,
                      hipStream_t s, bool cooperative) {
  if (cooperative) {
    switch (CM) {
      case 4: return launch_cm<4>(d_insts, d_wg_inst, nwg, lds, s);
      case 8: return launch_cm<8>(d_insts, d_wg_inst, nwg, lds, s);
      case 16: return launch_cm<16>(d_insts, d_wg_inst, nwg, lds, s);
      case 32: return launch_cm<32>(d_insts, d_wg_inst, nwg, lds, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (CM) {
    case 4: return launch_cm_plain<4>(d_insts, d_wg_inst, nwg, lds, s);
    case 8: return launch_cm_plain<8>(d_insts, d_wg_inst, nwg, lds, s);
    case 16: return launch_cm_plain<16>(d_insts, d_wg_inst, nwg, lds, s);
    case 32: return launch_cm_plain<32>(d_insts, d_wg_inst, nwg, lds, s);
    default: return hipErrorInvalidValue;
  }
}

template <int CM>
static hipError_t launch_adj_cm(const Inst *d_insts, const int *d_wg_inst, int nwg, size_t lds,
                                hipStream_t s) {
  auto kern = k_adj<CM>;
  hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  void *args[] = {(void *)&d_insts, (void *)&d_wg_inst};
  return hipLaunchCooperativeKernel((const void *)kern, dim3(nwg), dim3(WGS), args, (unsigned)lds,
                                    s);
}

hipError_t launch_adj(const Inst *d_insts, const int *d_wg_inst, int nwg, int CM, size_t lds,
                      hipStream_t s) {
  switch (CM) {
    case 4: return launch_adj_cm<4>(d_insts, d_wg_inst, nwg, lds, s);
    case 8: return launch_adj_cm<8>(d_insts, d_wg_inst, nwg, lds, s);
    case 16: return launch_adj_cm<16>(d_insts, d_wg_inst, nwg, lds, s);
    case 32: return launch_adj_cm<32>(d_insts, d_wg_inst, nwg, lds, s);
    default: return hipErrorInvalidValue;
  }
}

template <int CM>
static hipError_t set_lds_cm(size_t lds) {
  hipError_t e = hipFuncSetAttribute((const void *)k_run<CM>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void *)k_adj<CM>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds);
}

hipError_t set_kernel_lds(int CM, size_t lds) {
  switch (CM) {
    case 4: return set_lds_cm<4>(lds);
    case 8: return set_lds_cm<8>(lds);
    case 16: return set_lds_cm<16>(lds);
    case 32: return set_lds_cm<32>(lds);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_clear(void *p, size_t bytes, hipStream_t s) {
  size_t words = bytes / 4;
  int blocks = (int)((words + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_clear, dim3(blocks), dim3(256), 0, s, (uint32_t *)p, words);
  return hipGetLastError();
}

int max_coresident(int CM, size_t lds, int *out) {
  int nb = 0;
  // the occupancy query honours the kernels' dynamic-LDS limit: raise it first
  hipError_t e = set_kernel_lds(CM, lds);
  if (e != hipSuccess) {
    (void)hipGetLastError();  // do not leave the failure for the next launch to report
    return -1;
  }
  int na = 0;
  switch (CM) {
    case 4:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_run<4>, WGS, lds);
      if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&na, k_adj<4>, WGS, lds);
      break;
    case 8:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_run<8>, WGS, lds);
      if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&na, k_adj<8>, WGS, lds);
      break;
    case 16:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_run<16>, WGS, lds);
      if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&na, k_adj<16>, WGS, lds);
      break;
    case 32:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_run<32>, WGS, lds);
      if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&na, k_adj<32>, WGS, lds);
      break;
    default: return -1;
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return -2;
  }
  *out = nb < na ? nb : na;
  return 0;
}

}  // namespace mpts
