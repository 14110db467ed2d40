// Fused encoding + 16-bit MFMA decoder (FP16 or BF16, FP32 accumulation):
// forward (inference) launcher.
#include "fused_impl.h"

namespace fh {

using namespace fused_detail;

hipError_t launch_fused_fwd16(const GridDev& g, int H, int NH, fhash_dtype ddt, const float* pos,
                              int64_t n, const void* table, fhash_dtype tdt, const float* params,
                              float* y, hipStream_t st) {
  FusedArgs A{};
  A.pos = reinterpret_cast<const float4*>(pos);
  A.n = n;
  A.table = table;
  A.params = params;
  A.y = y;
  A.in_w = g.L * g.F;
  if (ddt == FHASH_BF16)
    return fused_dispatch_f2<MODE_FWD16, __bf16>(g, H, NH, tdt, A, nullptr, st);
  return fused_dispatch<MODE_FWD16, _Float16>(g, H, NH, tdt, A, nullptr, st);
}

}  // namespace fh
