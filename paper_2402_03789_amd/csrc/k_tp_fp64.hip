// Tensor-product kernels of the FP64 form, in a translation unit
// of their own so that the three forms compile in parallel.
#include "k_tp.h"

namespace sn {
SN_TP_INST(double, double)
}  // namespace sn
