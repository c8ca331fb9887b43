// FFT length 384 = 24 x 16: kernel instantiations and registration.
#include "lens.hpp"

VIE_REGISTER_LEN(24, 16, 0, 1)
