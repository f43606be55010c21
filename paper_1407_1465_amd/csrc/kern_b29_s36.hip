// Kernel instances: radix 2^29, 36 limbs; lanes per exponentiation 2, 4.
#include "launch_impl.hpp"

RSAGPU_INSTANTIATE(29, 36, 2)
RSAGPU_INSTANTIATE(29, 36, 4)
