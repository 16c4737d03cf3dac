// Autotuner cache lookup: tile width chosen for a (length, dtype, pass) on this device.
#pragma once

#include "common.hpp"

namespace tk {

// Tuned column-tile width W for pass (1 = Y, 2 = X) of length L, or 0 if none recorded.
int tuned_width(int L, tk_dtype dt, int pass);

}  // namespace tk
