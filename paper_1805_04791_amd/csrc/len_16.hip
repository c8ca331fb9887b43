// FFT length 16 = 4 x 4: kernel instantiations and registration.
#include "lens.hpp"

VIE_REGISTER_LEN(4, 4, 1, 0)
