// tables.h -- host-side operator tables of the nodal DGSEM on LGL nodes.
#pragma once

namespace dgx {

// LGL nodes x[N+1] and weights w[N+1]; D[i*(N+1)+j] = l_j'(x_i); orthonormal Legendre
// Vandermonde inverse Vinv[a*(N+1)+i].  Returns false if N is out of range.
bool lgl_tables(int N, double* x, double* w, double* D, double* Vinv);

// The per-handle operator tables of the kernels (layout TAB_* in kernels.h) for polydeg N
// and cell sizes h[3]: -(2/h_d) S with S = 2D - M^-1 B, lift factors +-(2/h_d)/w,
// FV factors -(2/h_d)/w_i, Legendre V^-1, LGL weights and nodes, 2/h_d.  For the weak form
// the first block holds (2/h_d) Dhat instead, Dhat_im = (w_m/w_i) D_mi.
bool stage_tables(int N, const double* h, double* T /* TAB_SIZE doubles, zeroed */,
                  bool weak = false);

}  // namespace dgx
