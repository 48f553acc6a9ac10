// Banded Cholesky factors of the constant matrices and their substitution kernel
// (npfem_factor.hip): the paper's own route to the products with H~^-1 and h^2 M~^-1.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace npfem {

// Banded Cholesky factors of H~ (index 0) and M~/h^2 (index 1) in the reverse
// Cuthill-McKee order, laid out for the substitution kernels (npfem_factor.hip).
// Vector-unit layouts (FP64): rows in blocks of kFactorRows positions i0 .. i0+7, per
// block
//   F[jj][k] = -L[i0+k][i0-B+jj]     (0 outside the band or for negative columns)
//   G[jj][k] = -L[i0+8+jj][i0+k]     (0 outside the band or beyond n_pad)
//   T[k] = 1 / L[i0+k][i0+k],  T[8 + 8k + l] = L[i0+k][i0+l] for l < k (else 0)
// with B the half bandwidth b rounded up to a multiple of 16; padding positions carry
// the identity.
//
// Matrix-core layouts (FP32): blocks of kFactorMfmaRows = 16 positions i0 .. i0+15, k steps
// of 4 positions, one entry per lane l (row r = l & 15, k index q = l >> 4):
//   FA[st][l] = -L[i0+r][i0-B+4st+q]     GA[st][l] = -L[i0+16+4st+q][i0+r]
//   DA[st][l] = (L_D^-1)[r][4st+q]       DB[st][l] = (L_D^-1)[4st+q][r]
// with L_D the block's 16 x 16 diagonal block.
constexpr int kFactorRows = 8;
constexpr int kFactorMfmaRows = 16;
constexpr int kFactorDiag = kFactorRows + kFactorRows * kFactorRows;
constexpr size_t kBandSolveMaxLds = 160 * 1024;
template <typename Real>
struct BandFactorDev {
  int b, B, ring;              // half bandwidth, b rounded up to 16, LDS ring positions (B + 16)
  const int* iperm;            // [n_pad] position of vertex k in the order (identity on padding)
  const Real* F[2];
  const Real* G[2];
  const Real* T[2];
  const Real* FA[2];           // [n_pad / 16][B / 4][64]
  const Real* GA[2];
  const Real* DA[2];           // [n_pad / 16][4][64]
  const Real* DB[2];
};
template <typename Real>
size_t band_solve_lds_bytes(int ring);
size_t band_solve_work_bytes(int n_pad, int rows, int real_bytes);
template <typename Real>
hipError_t launch_band_solve(const BandFactorDev<Real>& f, int which, int n_pad, const Real* in, Real* out,
                             Real* work, int rows, hipStream_t s);

}  // namespace npfem
