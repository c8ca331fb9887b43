// FFT length 216 = 12 x 18: the alternative split the autotuner may pick per pass.
#include "lens.hpp"

VIE_REGISTER_SPLIT(12, 18)
