// Internal interface of the link-derivative and force kernels (force.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>

namespace eofa {

struct DerivArgs {
  int L[4];
  int Ls, Vh;
  const double2* links[2];  // packed FP64 links per parity (phases included)
  const double2* a;         // canonical complex128 5D field (one right-hand side)
  const double2* b;
  double2* y;               // canonical complex128 [4][V][3][3]
  double coef;              // y (+)= coef * (link derivative matrix)
  int g5r5_a;               // 1: use gamma_5 R5 a in place of a
  int accumulate;           // 1: add to y, 0: overwrite
};

void launch_dhop_deriv(const DerivArgs& d, hipStream_t st);
// y <- sum_a T^a Re Tr(T^a y) on nlinks 3 x 3 matrices, in place
void launch_force_project(size_t nlinks, void* y, hipStream_t st);
// G-parity in x: gauge [4][rows][Lx][3][3] -> x-doubled [4][rows][2Lx][3][3]
// (second half complex conjugated); rows = Lt*Lz*Ly
void launch_double_gauge(int Lx, size_t rows, const void* U, void* U2, hipStream_t st);
// physical force [4][rows][Lx] = F2(x) + conj(F2(x + Lx)) from the doubled one
void launch_fold_force(int Lx, size_t rows, const void* F2, void* F, hipStream_t st);

}  // namespace eofa
