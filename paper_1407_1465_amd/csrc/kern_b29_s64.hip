// Kernel instances: radix 2^29, 64 limbs (the 56 of 1536-bit operands
// rounded up to a multiple of 16 lanes); lanes per exponentiation 16.
#include "launch_impl.hpp"

RSAGPU_INSTANTIATE(29, 64, 16)
