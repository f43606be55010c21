// Kernel instances: radix 2^32, 2 limbs; lanes per exponentiation 1.
#include "launch_impl.hpp"

RSAGPU_INSTANTIATE(32, 2, 1)
