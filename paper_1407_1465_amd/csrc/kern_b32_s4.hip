// Kernel instances: radix 2^32, 4 limbs; lanes per exponentiation 1, 2.
#include "launch_impl.hpp"

RSAGPU_INSTANTIATE(32, 4, 1)
RSAGPU_INSTANTIATE(32, 4, 2)
