// FFT length 256 = 32 x 8: the alternative split the autotuner may pick per pass.
#include "lens.hpp"

VIE_REGISTER_SPLIT(32, 8)
