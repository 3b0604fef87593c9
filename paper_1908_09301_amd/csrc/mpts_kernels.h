// Host-side entry points into the device code (launch wrappers).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include "mpts_common.h"

namespace mpts {

// Per-instance launchers (one translation unit per chunk size CM).
#define MPTS_DECLARE_CM(NS)                                                                     \
  namespace NS {                                                                                \
  hipError_t launch_run(const Inst *d_insts, const int *d_wg_inst, int nwg, size_t lds,         \
                        hipStream_t s, bool cooperative);                                       \
  hipError_t launch_adj(const Inst *d_insts, const int *d_wg_inst, int nwg, size_t lds,         \
                        hipStream_t s);                                                         \
  hipError_t launch_poly(const PolyInst *d_insts, int count, size_t lds, hipStream_t s);       \
  hipError_t set_lds(size_t lds, bool adjoint);                                                 \
  hipError_t occupancy(int *nb, size_t lds, bool adjoint);                                      \
  }
MPTS_DECLARE_CM(cm4)
MPTS_DECLARE_CM(cm8)
MPTS_DECLARE_CM(cm16)
MPTS_DECLARE_CM(cm32)
#undef MPTS_DECLARE_CM

// Bytes of dynamic LDS one workgroup of the forward (or adjoint) kernel needs.
size_t lds_bytes(int L, int N, int RS, int WB, int CM, bool adjoint, bool mfma);

// Launch of the persistent forward kernel over `nwg` workgroups; workgroup w
// runs trajectory d_insts[d_wg_inst[w]].  `cooperative` asks the runtime to
// guarantee that all workgroups are resident together; the plain launch
// (used under graph capture) relies on nwg not exceeding what fits at once.
hipError_t launch_run(const Inst *d_insts, const int *d_wg_inst, int nwg, int CM, size_t lds,
                      hipStream_t s, bool cooperative);

// Cooperative launch of the adjoint kernel (reverse sweep over checkpoints).
hipError_t launch_adj(const Inst *d_insts, const int *d_wg_inst, int nwg, int CM, size_t lds,
                      hipStream_t s);

// One workgroup per trajectory of a polynomial vector field (k_poly).
hipError_t launch_poly(const PolyInst *d_insts, int count, int CM, size_t lds, hipStream_t s);
// Bytes of dynamic LDS one workgroup of k_poly needs.
size_t poly_lds_bytes(int V, int Q, int RS, int WB, int CM, int maxn);

// Allow the forward (or adjoint) kernel instance for CM the given dynamic LDS size.
hipError_t set_kernel_lds(int CM, size_t lds, bool adjoint);

// Zero `bytes` of device memory with a kernel (usable under graph capture).
hipError_t launch_clear(void *p, size_t bytes, hipStream_t s);

// Workgroups of the forward (or adjoint) kernel that fit on one compute unit.
int max_coresident(int CM, size_t lds, int *out, bool adjoint);

}  // namespace mpts
