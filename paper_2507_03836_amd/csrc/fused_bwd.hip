// Fused encoding + MLP: backward given dL/dy, FP32 decoder.
#include "fused_impl.h"

namespace fh {

using namespace fused_detail;

hipError_t launch_fused_bwd(const GridDev& g, int H, int NH, fhash_dtype ddt, const float* pos,
                            int64_t n, const void* table, fhash_dtype tdt, const float* params,
                            const float* dy, float* d_table, float* d_params, void* ws, int64_t P,
                            hipStream_t st) {
  if (ddt != FHASH_F32)
    return launch_fused_bwd16(g, H, NH, ddt, pos, n, table, tdt, params, dy, d_table, d_params,
                              ws, P, st);
  FusedArgs A{};
  A.pos = reinterpret_cast<const float4*>(pos);
  A.dy = dy;
  A.n = n;
  A.table = table;
  A.params = params;
  A.d_table = d_table;
  A.part = static_cast<float*>(ws);
  A.P = P;
  A.in_w = g.L * g.F;
  return fused_dispatch<MODE_BWD, float>(g, H, NH, tdt, A, d_params, st);
}

}  // namespace fh
