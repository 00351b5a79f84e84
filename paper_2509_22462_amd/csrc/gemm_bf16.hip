// Register-staged MFMA GEMM instantiations for bf16 operands (the kernels are
// in gemm_kernels.h; one translation unit per element type).
#include "gemm_kernels.h"

namespace nnc {
NNC_GEMM_TYPED_ENTRY_POINTS(bf16, bf16)
}  // namespace nnc
