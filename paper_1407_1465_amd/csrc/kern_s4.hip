// Kernel instances of padded width 4 limbs (lanes per exponentiation: 1, 2).
#include "launch_impl.hpp"

RSAGPU_INSTANTIATE(4, 1)
RSAGPU_INSTANTIATE(4, 2)
