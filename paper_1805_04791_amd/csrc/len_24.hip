// FFT length 24 = 6 x 4: kernel instantiations and registration.
#include "lens.hpp"

VIE_REGISTER_LEN(6, 4, 1, 0)
