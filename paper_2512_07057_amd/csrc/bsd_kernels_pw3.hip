// Decoder kernels for columns of degree at most 6 (edge positions in 3 register word(s)).
#include "bsd_device.h"

BSD_DEFINE_PW(3)
