// Decoder kernels for columns of degree at most 4 (edge positions in 2 register word(s)).
#include "bsd_device.h"

BSD_DEFINE_PW(2)
