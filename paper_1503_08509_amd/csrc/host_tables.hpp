// Create-time near-field screen-potential tables (see host_tables.cpp).
#pragma once

#include "host_fe.hpp"

namespace fep3m {

// T[a][D][m] (element units, h = 1): a in {0..d}^3 x fastest, D the offset of
// the target element from the source element in [-n_sr, n_sr]^3 (x fastest),
// m the order-p node of the target element (x fastest).  B: table box size
// in elements (odd, > 2 n_sr + 1).
void compute_tables(int p, const Screen1D &scr, int n_sr, int B, Vec &T);

}  // namespace fep3m
