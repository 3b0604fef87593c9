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
  c.maxn = (I.N + 1 + 15) & ~15;
  c.offs = (int8_t *)p;
  return c;
}

size_t lds_bytes(int L, int N, int RS, int WB, int CM) {
  const int NV = (L + 2 + 3) & ~3;
  const int maxn = (N + 1 + 15) & ~15;
  size_t b = (size_t)NFR * WB * 8 + (size_t)3 * 64 * CM * 8 + (size_t)3 * 64 * CM * 4 +
             (size_t)6 * NV * 4 + (size_t)4 * RS * 4 + sizeof(FrameSrc) * NFR +
             sizeof(FrameD) * (NFR + 1) + 64 * 4 + 2 * NFR * 4 + (size_t)NFR * maxn;
  return (b + 255) & ~(size_t)255;
}

__device__ __forceinline__ int32_t *row_ptr(const Inst &I, int arr, int idx) {
  return I.rows + ((long long)arr * (I.N + 1) + idx) * I.RS;
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
  // read-modify-write polls are answered at the coherence point
  while (__hip_atomic_fetch_add(flag, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
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
      // R a_i - b_i - s1_i
      ad[0] = Addend{row_ptr(I, 1, i), 1, -1};
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
  uint32_t *flag = I.sync + SY_FLAG;
  uint32_t *arrive = I.sync + SY_ARRIVE;
  Carve cv = carve(smem, I);
  for (int j = tid; j < NFR * WB; j += WGS) cv.lf[j] = 0;
  const int32_t *tau_row = I.consts + (size_t)C_TAU * RS;
  uint32_t gen = 0;
  unsigned long long nbulk = 0;
  // phase timers (thread 0 of the leader and of workgroup 1)
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
    // rows 0 of the three coefficient arrays are the current state
    if (leader) {
      if (wave < 3) {
        const int32_t *sv = I.state + (size_t)wave * (L + 2);
        write_row(sv, L, nd, RS, row_ptr(I, wave, 0), G > 1, lane, 64);
        if (step == 0 && I.ckpt) copy_norm(sv, I.ckpt + (size_t)wave * (L + 2), L, false, lane, 64);
        if (I.coefs) copy_norm(sv, I.coefs + (size_t)wave * (N + 1) * (L + 2), L, false, lane, 64);
      }
      wait_vmem();
      __syncthreads();
      ++gen;
      if (G > 1 && tid == 0) st_relaxed(flag, gen);
    } else {
      ++gen;
      if (tid == 0) spin_until(flag, gen, err);
      __syncthreads();
    }
    if (G > 1) {
      // rows are rewritten every step: drop cached copies once per step
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __syncthreads();
    }
    mark(PH_STEP0);

    for (int i = 0; i < N; ++i) {
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
      frame_setup(cv.fs, cv.fd, NFR, nd, RS, cv.red, cv.offs, cv.maxn, err);
      mark(PH_SETUP);
      frames_accumulate(cv.fs, cv.fd, NFR, nd, RS, WB, cv.lf, rank, G, cv.span, cv.offs, cv.maxn);
      __syncthreads();
      mark(PH_ACCUM);
      ++nbulk;
      long long *gf = I.gframes + (size_t)(nbulk & 1) * NFR * WB;
      if (G > 1) {
        for (int f = 0; f < NFR; ++f) {
          int c0 = cv.span[2 * f], c1 = cv.span[2 * f + 1];
          for (int c = c0 + tid; c < c1; c += WGS) {
            long long v = cv.lf[(size_t)f * WB + c];
            if (v != 0) {
              __hip_atomic_fetch_add((unsigned long long *)(gf + (size_t)f * WB + c),
                                     (unsigned long long)v, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
              cv.lf[(size_t)f * WB + c] = 0;
            }
          }
        }
        wait_vmem();
        __syncthreads();
        if (tid == 0)
          __hip_atomic_fetch_add(arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      mark(PH_FLUSH);
      if (leader) {
        if (G > 1) {
          if (tid == 0) spin_until(arrive, (uint32_t)(G * nbulk), err);
          __syncthreads();
        }
        mark(PH_WAIT);
        const long long *frames = G > 1 ? gf : cv.lf;
        if (wave < 3) finalize_task<(CM)>(I, cv, wave, i, frames, G > 1, err);
        __syncthreads();
        mark(PH_FINAL);
        // clear the frames for their next use
        for (int f = 0; f < NFR; ++f) {
          int nc = cv.fd[f].nz ? frame_cols(cv.fd[f], nd) : 0;
          for (int c = tid; c < nc; c += WGS) {
            if (G > 1) st_relaxed(gf + (size_t)f * WB + c, 0LL);
            else cv.lf[(size_t)f * WB + c] = 0;
          }
        }
        wait_vmem();
        __syncthreads();
        ++gen;
        if (G > 1 && tid == 0) st_relaxed(flag, gen);
        mark(PH_CLEAR);
      } else {
        ++gen;
        if (tid == 0) spin_until(flag, gen, err);
        __syncthreads();
        mark(PH_WAIT);
      }
    }
    if (I.mode == MODE_COEFFS) break;

    // Horner: h = c_N; h <- round(h tau + c_i), i = N-1..0, three chains at once
    if (leader) {
      // LDS copies of c_N (the three Horner accumulators) and of the tau row
      for (int j = tid; j < 4 * RS; j += WGS) {
        int c = j / RS, w = j - c * RS;
        cv.hrow[j] = c < 3 ? row_ptr(I, c, N)[w] : tau_row[w];
      }
      const int32_t *tau_lds = cv.hrow + (size_t)3 * RS;
      __syncthreads();
      for (int i = N - 1; i >= 0; --i) {
        if (tid == 0) {
          for (int c = 0; c < 3; ++c)
            cv.fs[c] = mk_frame1(mk_part(PK_ONE, 1, 0, tau_lds, cv.hrow + (size_t)c * RS));
          frame_setup_single(cv.fs, cv.fd, 3, nd, cv.offs, cv.maxn);
        }
        __syncthreads();
        frames_accumulate(cv.fs, cv.fd, 3, nd, RS, WB, cv.lf, 0, 1, cv.span, cv.offs, cv.maxn);
        __syncthreads();
        if (wave < 3) {
          long long *cols = cv.tcols + (size_t)wave * 64 * I.CM;
          int32_t *h = cv.tnorm + (size_t)wave * 2 * cv.NV;
          Addend ad = Addend{row_ptr(I, wave, i), 1, 1};
          int C;
          long long dexp;
          int sgn = combine_resolve<CM>(cv.lf + (size_t)wave * WB, false, &cv.fd[wave], nd, L, &ad,
                                        1, (int32_t *)cols, &C, &dexp, err);
          bool ok = wave_round((int32_t *)cols, C, sgn, dexp, false, L, h);
          if (!ok && lane == 0) atomicOr(err, 2u);
          write_row(h, L, nd, RS, cv.hrow + (size_t)wave * RS, false, lane, 64);
          int nc = cv.fd[wave].nz ? frame_cols(cv.fd[wave], nd) : 0;
          for (int c = lane; c < nc; c += 64) cv.lf[(size_t)wave * WB + c] = 0;
        }
        __syncthreads();
      }
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

hipError_t set_kernel_lds(int CM, size_t lds) {
  switch (CM) {
    case 4: return hipFuncSetAttribute((const void *)k_run<4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    case 8: return hipFuncSetAttribute((const void *)k_run<8>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    case 16: return hipFuncSetAttribute((const void *)k_run<16>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    case 32: return hipFuncSetAttribute((const void *)k_run<32>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
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
  hipError_t e;
  switch (CM) {
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_run<4>, WGS, lds); break;
    case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_run<8>, WGS, lds); break;
    case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_run<16>, WGS, lds); break;
    case 32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_run<32>, WGS, lds); break;
    default: return -1;
  }
  if (e != hipSuccess) return -1;
  *out = nb;
  return 0;
}

}  // namespace mpts
