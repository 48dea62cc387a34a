// BF16 instantiations of the matrix-core network kernel and their tile
// variants (the autotuner in the host runtime picks one per network shape).
#include "mlp_mfma.h"
#include "mlp_pp.h"

namespace spider {

using mfma::launch_variant;
using mfma::PolBF16;

#define SPIDER_V(H, D, NW, RT) \
  MlpVariant { NW, RT, 0, &launch_variant<PolBF16, H, D, NW, RT> }
// shallower weight prefetch ring
#define SPIDER_VP(H, D, NW, RT, PF) \
  MlpVariant { NW, RT, 0, &launch_variant<PolBF16, H, D, NW, RT, PF, 1> }
// row halves in ping-pong, weight ring of one layer (schedule 1) or one and
// a half layers (schedule 2)
#define SPIDER_PP(H, D, NW, RT) \
  MlpVariant { NW, RT, 1, &mfma::launch_pp<PolBF16, H, D, NW, RT, H / 32> }
#define SPIDER_PP3(H, D, NW, RT) \
  MlpVariant { NW, RT, 2, &mfma::launch_pp<PolBF16, H, D, NW, RT, 3 * H / 64> }

int mlp_variants_bf16(int H, int D, const MlpVariant** list) {
  static const MlpVariant h32d2[] = {SPIDER_V(32, 2, 2, 4)};
  static const MlpVariant h32d3[] = {SPIDER_V(32, 3, 2, 4)};
  static const MlpVariant h32d4[] = {SPIDER_V(32, 4, 2, 4)};
  static const MlpVariant h64d3[] = {SPIDER_V(64, 3, 4, 4)};
  static const MlpVariant h64d4[] = {SPIDER_V(64, 4, 4, 4)};
  static const MlpVariant h128d3[] = {SPIDER_V(128, 3, 4, 4)};
  static const MlpVariant h128d4[] = {SPIDER_V(128, 4, 4, 4), SPIDER_PP(128, 4, 4, 4),
                                      SPIDER_V(128, 4, 4, 2)};
  static const MlpVariant h128d5[] = {SPIDER_V(128, 5, 4, 4)};
  static const MlpVariant h256d4[] = {SPIDER_V(256, 4, 8, 4), SPIDER_PP(256, 4, 8, 4)};
  static const MlpVariant h256d5[] = {SPIDER_V(256, 5, 8, 4), SPIDER_PP(256, 5, 8, 4)};
  static const MlpVariant h256d6[] = {SPIDER_V(256, 6, 8, 4), SPIDER_PP(256, 6, 8, 4),
                                      SPIDER_V(256, 6, 8, 2), SPIDER_VP(256, 6, 8, 4, 2),
                                      SPIDER_PP3(256, 6, 8, 4)};
  static const MlpVariant h256d7[] = {SPIDER_V(256, 7, 8, 4), SPIDER_PP(256, 7, 8, 4)};
  // eight layers: the 64-row tiles spill registers (seven stored derivative
  // layers); the 32-row ping-pong and the shallower ring do not
  static const MlpVariant h256d8[] = {SPIDER_V(256, 8, 8, 4), SPIDER_PP(256, 8, 8, 2),
                                      SPIDER_V(256, 8, 8, 2), SPIDER_VP(256, 8, 8, 4, 2)};
#define SPIDER_L(HH, DD, arr)                \
  if (H == HH && D == DD) {                  \
    *list = arr;                             \
    return (int)(sizeof(arr) / sizeof(arr[0])); \
  }
  SPIDER_L(32, 2, h32d2)
  SPIDER_L(32, 3, h32d3)
  SPIDER_L(32, 4, h32d4)
  SPIDER_L(64, 3, h64d3)
  SPIDER_L(64, 4, h64d4)
  SPIDER_L(128, 3, h128d3)
  SPIDER_L(128, 4, h128d4)
  SPIDER_L(128, 5, h128d5)
  SPIDER_L(256, 4, h256d4)
  SPIDER_L(256, 5, h256d5)
  SPIDER_L(256, 6, h256d6)
  SPIDER_L(256, 7, h256d7)
  SPIDER_L(256, 8, h256d8)
#undef SPIDER_L
  *list = nullptr;
  return 0;
}

}  // namespace spider
