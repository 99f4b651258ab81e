// Launchers of setup.hip.
#pragma once

#include "internal.h"

namespace eahp {

struct Lat {
  double B[9];  // reciprocal vectors as columns
};

void launch_vion_g(hipStream_t st, int n1, int n2, int n3, const Lat& L, int natoms, const double* R, const double* Z,
                   double r, double Omega, z64* box);
void launch_projectors(hipStream_t st, int64_t npw, const int* box, int n1, int n2, int n3, const Lat& L,
                       const double k[3], int natoms, const double* R, double rp, double Omega, z64* P, c32* P32);
void weighted_sum(hipStream_t st, int nk, int p, const double* vals, const double* kw, double scale, double* out);
void sum_strided(hipStream_t st, int m, int stride, int c, const double* part, double scale, double* out);
void border_mirror(hipStream_t st, int q, int r, z64* A, int64_t lda);
void copy2d(hipStream_t st, int rows, int cols, const z64* S, int64_t lds, z64* D, int64_t ldd);
void minval(hipStream_t st, int n, const double* v, double* out);
void maxval(hipStream_t st, int n, const double* v, double* out);
void minval_big(hipStream_t st, int64_t n, const double* v, double* out, DevMem& part);

}  // namespace eahp
