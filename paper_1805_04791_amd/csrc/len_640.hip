// FFT length 640 = 32 x 20: kernel instantiations and registration.
#include "lens.hpp"

VIE_REGISTER_LEN(32, 20, 0, 1)
