// FFT length 32 = 8 x 4: kernel instantiations and registration.
#include "lens.hpp"

VIE_REGISTER_LEN(8, 4, 1, 1)
