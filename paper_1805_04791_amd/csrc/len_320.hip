// FFT length 320 = 20 x 16: kernel instantiations and registration.
#include "lens.hpp"

VIE_REGISTER_LEN(20, 16, 1, 0)
