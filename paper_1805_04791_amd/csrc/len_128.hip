// FFT length 128 = 16 x 8: kernel instantiations and registration.
#include "lens.hpp"

VIE_REGISTER_LEN(16, 8, 1, 1)
