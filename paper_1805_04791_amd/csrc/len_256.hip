// FFT length 256 = 16 x 16: kernel instantiations and registration.
#include "lens.hpp"

VIE_REGISTER_LEN(16, 16, 1, 1)
