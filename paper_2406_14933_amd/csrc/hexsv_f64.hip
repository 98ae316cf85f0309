// FP64 step kernels: built with -ffp-contract=off so every operation rounds
// as written (the CPU reference is compiled the same way).
#include "hexsv_kernels.h"

namespace hexsv {
HEXSV_INSTANTIATE(double)
}
