// Autotuner cache: the tile shape chosen for a (length, dtype, pass) on this device.
#pragma once

#include "common.hpp"

namespace tk {

// Strided passes (pass 1 = Y, 2 = X): a = column width W; Z pass (pass 0): a = threads
// per workgroup.  E = points per thread; v = kernel variant of a strided pass (0: one
// tile per workgroup, 1: persistent with loads issued one tile ahead).  a = 0 means no
// entry.
struct TileChoice {
    int a, E, v;
};

TileChoice tuned_tile(int L, tk_dtype dt, int pass);
void set_tuned_tile(int L, tk_dtype dt, int pass, TileChoice c);
void clear_tuned_tiles();

// Ensemble kernels compiled for grid size n with nt threads per workgroup (pass 8).
bool batch_tile_ok(int n, int nt);

}  // namespace tk
