// Decoder kernels for columns of degree at most 2 (edge positions in 1 register word(s)).
#include "bsd_device.h"

BSD_DEFINE_PW(1)
