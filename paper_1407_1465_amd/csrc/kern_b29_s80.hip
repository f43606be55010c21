// Kernel instances: radix 2^29, 80 limbs (the 72 of 2048-bit operands
// rounded up to a multiple of 16 lanes); lanes per exponentiation 16.
#include "launch_impl.hpp"

RSAGPU_INSTANTIATE(29, 80, 16)
