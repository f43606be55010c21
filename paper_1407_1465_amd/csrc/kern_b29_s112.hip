// Kernel instances: radix 2^29, 112 limbs; exponentiation only (no CRT half is this wide); lanes per exponentiation 8, 16.
#include "launch_impl.hpp"

RSAGPU_INSTANTIATE_EXP(29, 112, 8)
RSAGPU_INSTANTIATE_EXP(29, 112, 16)
