// FFT length 192 = 16 x 12: kernel instantiations and registration.
#include "lens.hpp"

VIE_REGISTER_LEN(16, 12, 1, 1)
