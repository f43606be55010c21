// Kernel instances: radix 2^29, 28 limbs; lanes per exponentiation 4.
#include "launch_impl.hpp"

RSAGPU_INSTANTIATE(29, 28, 4)
