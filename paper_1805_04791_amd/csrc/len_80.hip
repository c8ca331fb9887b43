// FFT length 80 = 10 x 8: kernel instantiations and registration.
#include "lens.hpp"

VIE_REGISTER_LEN(10, 8, 1, 0)
