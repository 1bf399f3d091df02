// Decoder kernels for columns of degree at most 8 (edge positions in 4 register word(s)).
#include "bsd_device.h"

BSD_DEFINE_PW(4)
