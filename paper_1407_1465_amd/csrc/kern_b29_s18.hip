// Kernel instances: radix 2^29, 18 limbs; lanes per exponentiation 2.
#include "launch_impl.hpp"

RSAGPU_INSTANTIATE(29, 18, 2)
