// Fused encoding + FP16-MFMA decoder: forward (inference) launcher.
#include "fused_impl.h"

namespace fh {

using namespace fused_detail;

hipError_t launch_fused_fwd16(const GridDev& g, int H, int NH, const float* pos, int64_t n,
                              const void* table, fhash_dtype tdt, const float* params, float* y,
                              hipStream_t st) {
  FusedArgs A{};
  A.pos = reinterpret_cast<const float4*>(pos);
  A.n = n;
  A.table = table;
  A.params = params;
  A.y = y;
  A.in_w = g.L * g.F;
  return fused_dispatch<MODE_FWD16>(g, H, NH, tdt, A, nullptr, st);
}

}  // namespace fh
