// Trefftz basis tables with a choice of spatial seed basis (Sec. 3, Sec. 6.3).
#pragma once

#include "tdg_internal.h"

namespace tdg {

// seed: 0 monomials x^beta, 1 products of Legendre polynomials, 2 products of
// Chebyshev polynomials of the first kind, in the scaled coordinates of
// Remark 3.1.  Every choice spans the same space U^p; only the basis differs.
Table build_table(int n, int p, int seed);

}  // namespace tdg
