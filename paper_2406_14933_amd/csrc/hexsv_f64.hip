// FP64 step kernels: built with -ffp-contract=off so every operation rounds
// as written (the CPU reference is compiled the same way).
#include "hexsv_ensemble.h"
#include "hexsv_kernels.h"

namespace hexsv {
HEXSV_INSTANTIATE(double)
HEXSV_INSTANTIATE_ENSEMBLE(double)

}
