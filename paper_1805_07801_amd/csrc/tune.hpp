// Autotuner cache: the tile shape chosen for a (length, dtype, pass) on this device.
#pragma once

#include "common.hpp"

namespace tk {

// Strided passes (pass 1 = Y, 2 = X): a = column width W; Z pass (pass 0): a = threads
// per workgroup.  E = points per thread.  a = 0 means no entry.
struct TileChoice {
    int a, E;
};

TileChoice tuned_tile(int L, tk_dtype dt, int pass);
void set_tuned_tile(int L, tk_dtype dt, int pass, TileChoice c);
void clear_tuned_tiles();

}  // namespace tk
