// Fused encoding + MLP: forward + MSE loss + backward in one pass, 16-bit MFMA
// decoder (FP16 or BF16 operands, FP32 accumulation), two features per level.
#include "fused_impl.h"

namespace fh {

using namespace fused_detail;

hipError_t launch_fused_train16(const GridDev& g, int H, int NH, fhash_dtype ddt,
                                const float* pos, const float* target, int64_t n,
                                const void* table, fhash_dtype tdt, const float* params,
                                float loss_scale, float* d_table, float* d_params,
                                double* loss_sum, void* ws, int64_t P, hipStream_t st) {
  FusedArgs A{};
  A.pos = reinterpret_cast<const float4*>(pos);
  A.target = target;
  A.n = n;
  A.table = table;
  A.params = params;
  A.d_table = d_table;
  A.part = static_cast<float*>(ws);
  A.loss_sum = loss_sum;
  A.P = P;
  A.coef = (float)(2.0 * (double)loss_scale / (double)n);
  A.in_w = g.L * g.F;
  if (ddt == FHASH_BF16)
    return fused_dispatch_f2<MODE_TRAIN, __bf16>(g, H, NH, tdt, A, d_params, st);
  return fused_dispatch_f2<MODE_TRAIN, _Float16>(g, H, NH, tdt, A, d_params, st);
}

}  // namespace fh
