// FFT length 216 = 18 x 12: kernel instantiations and registration.
#include "lens.hpp"

VIE_REGISTER_LEN(18, 12, 1, 0)
