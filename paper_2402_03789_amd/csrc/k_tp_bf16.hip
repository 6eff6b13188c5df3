// Tensor-product kernels of the BF16 form (float32 arithmetic, bfloat16 storage), in a translation unit
// of their own so that the three forms compile in parallel.
#include "k_tp.h"

namespace sn {
SN_TP_INST(float, bf16_t)
}  // namespace sn
