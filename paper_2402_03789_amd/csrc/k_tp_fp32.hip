// Tensor-product kernels of the FP32 form (float32 arithmetic and storage), in a translation unit
// of their own so that the three forms compile in parallel.
#include "k_tp.h"

namespace sn {
SN_TP_INST(float, float)
}  // namespace sn
