// Register-staged MFMA GEMM instantiations for double operands (the kernels are
// in gemm_kernels.h; one translation unit per element type).
#include "gemm_kernels.h"

namespace nnc {
NNC_GEMM_TYPED_ENTRY_POINTS(double, f64)
}  // namespace nnc
