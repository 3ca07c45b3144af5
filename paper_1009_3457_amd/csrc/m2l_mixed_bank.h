// Layout of the split-precision (BF16x3 / FP16x3) M2L operator banks.
#pragma once

#include <cstddef>

namespace fmm2d {

size_t mixed_bank_bytes(int p, int precision);

}  // namespace fmm2d
