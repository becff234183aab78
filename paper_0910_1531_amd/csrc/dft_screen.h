// Launch interface of the RFD screening-operator kernels (host side).
#pragma once

#include "dft_kernels.h"

namespace dft {

// Per-block minima and maxima of r[0 .. n) and counts of entries that are not positive and
// finite; returns the number of blocks written (at most cap).
int rsc_range(long long n, const double *r, double *pmin, double *pmax, int *pbad, int cap, hipStream_t s);

// Barycentric interpolation in the radius on the M first-kind Chebyshev points
// R_j = cc + dd cos((2 j + 1) pi / (2 M)) with weights (-1)^j sin((2 j + 1) pi / (2 M)):
// per point the reciprocal of sum_j w_j / (r - R_j), or the index j where r equals R_j.
void cheb_prep(long long n, const double *r, int M, double cc, double dd, double *inv_den, int *hit, hipStream_t s);
// out[i][x] (=, first node; += otherwise) l_m(r(x)) part[i][x] for the S fields.
void cheb_accum(long long n, int S, int m, int M, double cc, double dd, const double *r, const double *inv_den,
                const int *hit, const double *part, double *out, bool first, hipStream_t s);

}  // namespace dft
