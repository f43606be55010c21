// Kernel instances: radix 2^32, 128 limbs; lanes per exponentiation 8, 16.
#include "launch_impl.hpp"

RSAGPU_INSTANTIATE(32, 128, 8)
RSAGPU_INSTANTIATE(32, 128, 16)
