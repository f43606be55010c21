// Kernel instances: radix 2^32, 24 limbs; lanes per exponentiation 4, 8.
#include "launch_impl.hpp"

RSAGPU_INSTANTIATE(32, 24, 4)
RSAGPU_INSTANTIATE(32, 24, 8)
