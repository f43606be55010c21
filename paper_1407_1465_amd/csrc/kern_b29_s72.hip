// Kernel instances: radix 2^29, 72 limbs; lanes per exponentiation 4, 8.
#include "launch_impl.hpp"

RSAGPU_INSTANTIATE(29, 72, 4)
RSAGPU_INSTANTIATE(29, 72, 8)
