// FFT length 160 = 16 x 10: kernel instantiations and registration.
#include "lens.hpp"

VIE_REGISTER_LEN(16, 10, 1, 0)
