// FFT length 120 = 12 x 10: kernel instantiations and registration.
#include "lens.hpp"

VIE_REGISTER_LEN(12, 10, 1, 0)
