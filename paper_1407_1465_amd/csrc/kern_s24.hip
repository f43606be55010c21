// Kernel instances of padded width 24 limbs (lanes per exponentiation: 4, 8).
#include "launch_impl.hpp"

RSAGPU_INSTANTIATE(24, 4)
RSAGPU_INSTANTIATE(24, 8)
