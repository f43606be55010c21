// Kernel instances of padded width 96 limbs (lanes per exponentiation: 8, 16).
#include "launch_impl.hpp"

RSAGPU_INSTANTIATE(96, 8)
RSAGPU_INSTANTIATE(96, 16)
