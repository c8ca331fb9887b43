// FFT length 192 = 12 x 16: the alternative split the autotuner may pick per pass.
#include "lens.hpp"

VIE_REGISTER_SPLIT(12, 16)
