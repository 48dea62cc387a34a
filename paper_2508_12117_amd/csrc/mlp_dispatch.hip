// Matrix-core network kernel: shape support, weight packing, default launch.
#include "mlp_mfma.h"

namespace spider {

int mlp_variants(int precision, int H, int D, const MlpVariant** list) {
  return precision == 1 ? mlp_variants_bf16(H, D, list) : mlp_variants_f32(H, D, list);
}

bool mlp_mfma_supported(int precision, int H, int D) {
  const MlpVariant* l = nullptr;
  return mlp_variants(precision, H, D, &l) > 0;
}

size_t mfma_pack_bytes(int precision, int H) {
  return (size_t)H * H * (precision == 1 ? 2 : 4);
}

void mfma_pack_layer(int precision, int H, const float* W, void* fwd, void* bwd) {
  if (precision == 1)
    mfma::pack_layer<mfma::PolBF16>(H, W, kTanhScale, (unsigned char*)fwd, (unsigned char*)bwd);
  else
    mfma::pack_layer<mfma::PolF32>(H, W, kTanhScale, (unsigned char*)fwd, (unsigned char*)bwd);
}

hipError_t launch_mlp_mfma(int precision, const RowSource& src, const NetView& net, RowOut* out,
                           hipStream_t stream) {
  const MlpVariant* l = nullptr;
  if (mlp_variants(precision, net.H, net.D, &l) == 0) return hipErrorNotSupported;
  if (src.rows == 0) return hipSuccess;
  return l[0].launch(src, net, out, stream);
}

}  // namespace spider
