// FFT length 48 = 8 x 6: kernel instantiations and registration.
#include "lens.hpp"

VIE_REGISTER_LEN(8, 6, 1, 1)
