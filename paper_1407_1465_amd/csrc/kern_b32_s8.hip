// Kernel instances: radix 2^32, 8 limbs; lanes per exponentiation 1, 2, 4.
#include "launch_impl.hpp"

RSAGPU_INSTANTIATE(32, 8, 1)
RSAGPU_INSTANTIATE(32, 8, 2)
RSAGPU_INSTANTIATE(32, 8, 4)
