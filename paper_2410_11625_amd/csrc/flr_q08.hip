// Kernel instantiations for 8 guide(s) and 1..4 channels.
#include "flr_device.hpp"
FLR_DEFINE_Q(8)
