// Kernel instances: radix 2^29, 144 limbs; exponentiation only (no CRT half is this wide); lanes per exponentiation 8, 16.
#include "launch_impl.hpp"

RSAGPU_INSTANTIATE_EXP(29, 144, 8)
RSAGPU_INSTANTIATE_EXP(29, 144, 16)
