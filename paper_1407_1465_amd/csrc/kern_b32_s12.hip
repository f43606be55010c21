// Kernel instances: radix 2^32, 12 limbs; lanes per exponentiation 2, 4.
#include "launch_impl.hpp"

RSAGPU_INSTANTIATE(32, 12, 2)
RSAGPU_INSTANTIATE(32, 12, 4)
