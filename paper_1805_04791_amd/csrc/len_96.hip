// FFT length 96 = 12 x 8: kernel instantiations and registration.
#include "lens.hpp"

VIE_REGISTER_LEN(12, 8, 1, 1)
