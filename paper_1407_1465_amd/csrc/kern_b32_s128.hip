// Kernel instances: radix 2^32, 128 limbs; exponentiation only (no CRT half is this wide); lanes per exponentiation 8, 16.
#include "launch_impl.hpp"

RSAGPU_INSTANTIATE_EXP(32, 128, 8)
RSAGPU_INSTANTIATE_EXP(32, 128, 16)
