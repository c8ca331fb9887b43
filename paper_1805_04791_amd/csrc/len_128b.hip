// FFT length 128 = 8 x 16: the alternative split the autotuner may pick per pass.
#include "lens.hpp"

VIE_REGISTER_SPLIT(8, 16)
