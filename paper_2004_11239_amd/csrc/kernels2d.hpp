// Launch wrappers of the two-dimensional operator (kernels2d.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace bzq {

// Real weights V[pair][c] of the half spectrum c <= ((N-1)^2 - 1)/2 (FP64
// arithmetic, stored as float or double); pd[pair] = {a, sigma_x, sigma_y,
// scale}, gj = Gauss-Jacobi nodes then weights (nj each).
hipError_t launch_table2d(void* V, const double* pd, const double* gj, int nj, int N, int npairs, bool fp32,
                          hipStream_t st);

// Q_hat = Q(f_hat) (both N^2 complex128, FFT order): compact copy into fc and
// f on the padded P^2 grid into fgrid, S workgroups over the npt pair-twos
// into Qpart[S][half spectrum], then the ordered sum (through
// tmp[kFinChunks = 16][half spectrum]) into Q_hat.
hipError_t launch_collision2d(const double* f_hat, double* Q_hat, void* fc, void* fgrid, const void* V,
                              const double* ph, const double* cp, const void* tw, double* Qpart, double* tmp, int N,
                              int P, int npt, int S, bool fp32, hipStream_t st);

}  // namespace bzq
