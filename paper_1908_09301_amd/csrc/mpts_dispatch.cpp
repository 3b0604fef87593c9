// Chunk-size dispatch of the kernel launchers: each instance (CM = 4, 8, 16,
// 32) lives in its own compilation of mpts_kernels.hip.
#include <hip/hip_runtime.h>
#include "mpts_kernels.h"

namespace mpts {

hipError_t launch_run(const Inst *d_insts, const int *d_wg_inst, int nwg, int CM, size_t lds,
                      hipStream_t s, bool cooperative) {
  switch (CM) {
    case 4: return cm4::launch_run(d_insts, d_wg_inst, nwg, lds, s, cooperative);
    case 8: return cm8::launch_run(d_insts, d_wg_inst, nwg, lds, s, cooperative);
    case 16: return cm16::launch_run(d_insts, d_wg_inst, nwg, lds, s, cooperative);
    case 32: return cm32::launch_run(d_insts, d_wg_inst, nwg, lds, s, cooperative);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_adj(const Inst *d_insts, const int *d_wg_inst, int nwg, int CM, size_t lds,
                      hipStream_t s) {
  switch (CM) {
    case 4: return cm4::launch_adj(d_insts, d_wg_inst, nwg, lds, s);
    case 8: return cm8::launch_adj(d_insts, d_wg_inst, nwg, lds, s);
    case 16: return cm16::launch_adj(d_insts, d_wg_inst, nwg, lds, s);
    case 32: return cm32::launch_adj(d_insts, d_wg_inst, nwg, lds, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_poly(const PolyInst *d_insts, int count, int CM, size_t lds, hipStream_t s) {
  switch (CM) {
    case 4: return cm4::launch_poly(d_insts, count, lds, s);
    case 8: return cm8::launch_poly(d_insts, count, lds, s);
    case 16: return cm16::launch_poly(d_insts, count, lds, s);
    case 32: return cm32::launch_poly(d_insts, count, lds, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t set_kernel_lds(int CM, size_t lds, bool adjoint) {
  switch (CM) {
    case 4: return cm4::set_lds(lds, adjoint);
    case 8: return cm8::set_lds(lds, adjoint);
    case 16: return cm16::set_lds(lds, adjoint);
    case 32: return cm32::set_lds(lds, adjoint);
    default: return hipErrorInvalidValue;
  }
}

int max_coresident(int CM, size_t lds, int *out, bool adjoint) {
  int nb = 0;
  // the occupancy query honours the kernel's dynamic-LDS limit: raise it first
  hipError_t e = set_kernel_lds(CM, lds, adjoint);
  if (e != hipSuccess) {
    (void)hipGetLastError();  // do not leave the failure for the next launch to report
    return -1;
  }
  switch (CM) {
    case 4: e = cm4::occupancy(&nb, lds, adjoint); break;
    case 8: e = cm8::occupancy(&nb, lds, adjoint); break;
    case 16: e = cm16::occupancy(&nb, lds, adjoint); break;
    case 32: e = cm32::occupancy(&nb, lds, adjoint); break;
    default: return -1;
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return -2;
  }
  *out = nb;
  return 0;
}

}  // namespace mpts
