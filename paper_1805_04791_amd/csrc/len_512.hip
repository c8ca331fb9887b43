// FFT length 512 = 32 x 16: kernel instantiations and registration.
#include "lens.hpp"

VIE_REGISTER_LEN(32, 16, 0, 1)
