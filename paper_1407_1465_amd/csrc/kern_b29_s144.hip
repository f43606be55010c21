// Kernel instances: radix 2^29, 144 limbs; lanes per exponentiation 8, 16.
#include "launch_impl.hpp"

RSAGPU_INSTANTIATE(29, 144, 8)
RSAGPU_INSTANTIATE(29, 144, 16)
