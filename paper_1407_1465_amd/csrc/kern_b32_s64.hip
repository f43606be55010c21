// Kernel instances: radix 2^32, 64 limbs; lanes per exponentiation 4, 8, 16.
#include "launch_impl.hpp"

RSAGPU_INSTANTIATE(32, 64, 4)
RSAGPU_INSTANTIATE(32, 64, 8)
RSAGPU_INSTANTIATE(32, 64, 16)
