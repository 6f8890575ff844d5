// tables.h -- host-side operator tables of the nodal DGSEM on LGL nodes.
#pragma once

namespace dgx {

// LGL nodes x[N+1] and weights w[N+1]; D[i*(N+1)+j] = l_j'(x_i); orthonormal Legendre
// Vandermonde inverse Vinv[a*(N+1)+i].  Returns false if N is out of range.
bool lgl_tables(int N, double* x, double* w, double* D, double* Vinv);

}  // namespace dgx
