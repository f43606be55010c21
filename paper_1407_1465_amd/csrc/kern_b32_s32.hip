// Kernel instances: radix 2^32, 32 limbs; lanes per exponentiation 2, 4, 8, 16.
#include "launch_impl.hpp"

RSAGPU_INSTANTIATE(32, 32, 2)
RSAGPU_INSTANTIATE(32, 32, 4)
RSAGPU_INSTANTIATE(32, 32, 8)
RSAGPU_INSTANTIATE(32, 32, 16)
