// K3: dense mode products with BF16 operands on MFMA (placeholder until the
// MFMA kernels land: reports "unsupported" so callers fall back to FP32).
#include "common.cuh"

namespace cpm {

bool chain_bf16_supported(const ChainGeom&) { return false; }

void launch_chain_bf16(const ChainArgs<float>&, const uint16_t*, uint16_t*, int, hipStream_t) {}

}  // namespace cpm
