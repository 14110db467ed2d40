// Fused encoding + MLP: forward (inference) launcher and shape table.
#include "fused_impl.h"

namespace fh {

using namespace fused_detail;

bool fused_supported(int F, int in_w, int H, int NH) {
  if (F != 1 && F != 2 && F != 4) return false;
  const int inp = ((in_w + 15) / 16) * 16;
  if (NH < 1 || NH > 3) return false;
  return inp <= 32 && (H == 32 || H == 64);
}

size_t fused_ws_bytes(int64_t n, int64_t P) {
  return (size_t)fused_blocks(n, MODE_BWD) * (size_t)P * 4;
}

int64_t fused_partials(int64_t n) { return fused_blocks(n, MODE_BWD); }

hipError_t launch_fused_fwd(const GridDev& g, int H, int NH, const float* pos, int64_t n,
                            const void* table, fhash_dtype tdt, const float* params, float* y,
                            hipStream_t st) {
  FusedArgs A{};
  A.pos = reinterpret_cast<const float4*>(pos);
  A.n = n;
  A.table = table;
  A.params = params;
  A.y = y;
  A.in_w = g.L * g.F;
  return fused_dispatch<MODE_FWD, float>(g, H, NH, tdt, A, nullptr, st);
}

}  // namespace fh
