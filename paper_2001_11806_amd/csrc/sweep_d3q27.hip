// Sweep instantiations for the D3Q27 stencil (one translation unit per
// stencil so the heavily unrolled kernels compile in parallel).
#include "sweep.h"

namespace lbm {

hipError_t launch_sweep_d3q27(int method, int dtype, int phase, const void* src, void* dst, const uint8_t* flags,
                          const void* force_y, const Geo& g, const Params& p, int has_mask, hipStream_t s) {
  switch (method) {
    case M_CUMULANT_GEN:
      return sweep_for_dtype<D3Q27, M_CUMULANT_GEN>(dtype, phase, src, dst, flags, force_y, g, p, has_mask, s);
    case M_SRT_SMAG:
      return sweep_for_dtype<D3Q27, M_SRT_SMAG>(dtype, phase, src, dst, flags, force_y, g, p, has_mask, s);
    case M_MRT_SMAG:
      return sweep_for_dtype<D3Q27, M_MRT_SMAG>(dtype, phase, src, dst, flags, force_y, g, p, has_mask, s);
    case M_KBC: return sweep_for_dtype<D3Q27, M_KBC>(dtype, phase, src, dst, flags, force_y, g, p, has_mask, s);
    case M_SRT: return sweep_for_dtype<D3Q27, M_SRT>(dtype, phase, src, dst, flags, force_y, g, p, has_mask, s);
    case M_TRT: return sweep_for_dtype<D3Q27, M_TRT>(dtype, phase, src, dst, flags, force_y, g, p, has_mask, s);
    case M_MRT: return sweep_for_dtype<D3Q27, M_MRT>(dtype, phase, src, dst, flags, force_y, g, p, has_mask, s);
    case M_MRT_UNIT:
      return sweep_for_dtype<D3Q27, M_MRT_UNIT>(dtype, phase, src, dst, flags, force_y, g, p, has_mask, s);
    case M_CUMULANT: return sweep_for_dtype<D3Q27, M_CUMULANT>(dtype, phase, src, dst, flags, force_y, g, p, has_mask, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace lbm
