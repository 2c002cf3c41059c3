// MFMA implicit-GEMM kernels for the wide layers (placeholder: not yet enabled).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace sc {

bool conv_mfma_supported(int, int, int, int, int) { return false; }
bool convt_mfma_supported(int, int, int, int) { return false; }
void pack_conv_mfma(const float*, int, int, int, int, std::vector<uint8_t>&, std::vector<float>&) {}
void pack_convt_mfma(const float*, int, int, int, int, std::vector<uint8_t>&, std::vector<float>&) {}
hipError_t launch_conv_mfma(const LayerArgs&, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_convt_mfma(const LayerArgs&, int, hipStream_t) { return hipErrorNotSupported; }

}  // namespace sc
