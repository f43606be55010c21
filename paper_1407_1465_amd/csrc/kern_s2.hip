// Kernel instances of padded width 2 limbs (lanes per exponentiation: 1).
#include "launch_impl.hpp"

RSAGPU_INSTANTIATE(2, 1)
