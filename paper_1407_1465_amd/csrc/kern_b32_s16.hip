// Kernel instances: radix 2^32, 16 limbs; lanes per exponentiation 2, 4, 8.
#include "launch_impl.hpp"

RSAGPU_INSTANTIATE(32, 16, 2)
RSAGPU_INSTANTIATE(32, 16, 4)
RSAGPU_INSTANTIATE(32, 16, 8)
