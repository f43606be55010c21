// Kernel instances of padded width 64 limbs (lanes per exponentiation: 4, 8, 16).
#include "launch_impl.hpp"

RSAGPU_INSTANTIATE(64, 4)
RSAGPU_INSTANTIATE(64, 8)
RSAGPU_INSTANTIATE(64, 16)
