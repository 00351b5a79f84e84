// Register-staged MFMA GEMM instantiations for float operands (the kernels are
// in gemm_kernels.h; one translation unit per element type).
#include "gemm_kernels.h"

namespace nnc {
NNC_GEMM_TYPED_ENTRY_POINTS(float, f32)
}  // namespace nnc
