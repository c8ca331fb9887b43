// FFT length 64 = 8 x 8: kernel instantiations and registration.
#include "lens.hpp"

VIE_REGISTER_LEN(8, 8, 1, 1)
