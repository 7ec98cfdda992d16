// BF16 MFMA implicit-GEMM convolutions (not yet built: every shape reports
// unsupported and the ABI returns GW_EUNSUPPORTED for GW_BF16).
#include "internal.h"

namespace gw {

bool conv_bf16_supported(int, int, int, int, bool) { return false; }
size_t conv_bf16_packed_elems(int, int, int, bool) { return 0; }
hipError_t launch_pack_bf16(const float*, uint16_t*, int, int, int, bool, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_conv_bf16(const ConvP&, bool, int, int, hipStream_t) { return hipErrorNotSupported; }

}  // namespace gw
