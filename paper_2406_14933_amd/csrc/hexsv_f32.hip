// FP32 step kernels (fused multiply-add allowed); the FP64 books and time
// step live in the control block and the per-tile partial records.
#include "hexsv_ensemble.h"
#include "hexsv_kernels.h"

namespace hexsv {
HEXSV_INSTANTIATE(float)
HEXSV_INSTANTIATE_ENSEMBLE(float)
}
