// Batched banded Cholesky substitution: the paper's own route to the products with the
// constant matrices (section 2.1.1 factors H~ once and solves with the factor in every
// iteration).  A = H~ or M~/h^2 is factored on the host as P A P^T = L L^T, P the
// reverse Cuthill-McKee order of the mesh, so that L is banded (half bandwidth b); each
// right-hand side q then needs L y = P q and L^T z = y, out = P^T z.
//
// Both kernels give one wave 64 right-hand sides.  The right-hand sides are brought into
// the order and transposed to [position][right-hand side] once, through an LDS tile, into
// the caller's workspace, which then holds y and z; the result goes back the same way.
// The solved positions still inside the band sit in an LDS ring (one row of 64 values per
// position).
//   FP32: the matrix cores, blocks of 16 positions (band_solve_mfma_kernel).
//   FP64: the vector units, one lane per right-hand side, blocks of 8 positions; the
//         factor entries are uniform across the wave and are read through the scalar
//         unit, every ring read feeds eight FMAs and the 8 x 8 diagonal block is solved
//         in registers (band_solve_kernel).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "npfem_factor.h"

namespace npfem {
namespace {

constexpr int kRhs = 64;        // right-hand sides per wave (one per lane)
constexpr int kTileRow = 65;    // padded row of the 64 x 64 transpose tile

// acc[k] += sum over jj < B of C[jj][k] * ring[(base + jj) mod W] (the factor entries are
// stored negated; the ring holds W = B + 16 positions), one position at a time: the next
// position's factor entries (scalar loads) and ring value (LDS) are requested before the
// current position's FMAs.
template <typename Real>
__device__ __forceinline__ void band_dot(Real (&acc)[kFactorRows], const Real* __restrict__ C, const Real* win,
                                         int base, int W, int B, int lane) {
  int slot = ((base % W) + W) % W;
  Real c[kFactorRows], v = win[slot * kRhs + lane];
#pragma unroll
  for (int k = 0; k < kFactorRows; ++k) c[k] = C[k];
  for (int g = 0; g < B; ++g) {
    Real cc[kFactorRows], vv = v;
#pragma unroll
    for (int k = 0; k < kFactorRows; ++k) cc[k] = c[k];
    if (g + 1 < B) {
      slot = slot + 1 == W ? 0 : slot + 1;
      v = win[slot * kRhs + lane];
#pragma unroll
      for (int k = 0; k < kFactorRows; ++k) c[k] = C[(g + 1) * kFactorRows + k];
    }
#pragma unroll
    for (int k = 0; k < kFactorRows; ++k) acc[k] = fma(cc[k], vv, acc[k]);
  }
}

// in[r][k] -> Y[iperm[k]][r - r0] for the wave's 64 right-hand sides r0 .. r0+63, through
// the LDS tile `lds` ([64][65]): rows read whole, written back one position per row.
// Addresses are clamped into range (and the values past the end dropped) so that the
// loads carry no branches and issue back to back; the chunk's iperm entries are read
// once, one per lane, and handed out with readlane.
template <typename Real>
__device__ __forceinline__ void load_rhs(const Real* __restrict__ in, Real* __restrict__ Y, Real* lds,
                                         const int* __restrict__ iperm, int np, int rows, int64_t r0, int lane) {
  const int64_t r_last = rows - 1;
  for (int k0 = 0; k0 < np; k0 += kRhs) {
    const int k = min(k0 + lane, np - 1);
    const bool k_ok = k0 + lane < np;
    const int ip = iperm[k];
#pragma unroll 16
    for (int rr = 0; rr < kRhs; ++rr) {
      const int64_t r = r0 + rr;
      const Real val = in[min(r, r_last) * np + k];
      lds[rr * kTileRow + lane] = (r <= r_last && k_ok) ? val : Real(0);
    }
    __syncthreads();
    const int kn = min(kRhs, np - k0);
    for (int kk = 0; kk < kn; ++kk) {
      const int pos = __builtin_amdgcn_readlane(ip, kk);
      Y[(size_t)pos * kRhs + lane] = lds[lane * kTileRow + kk];
    }
    __syncthreads();
  }
}

// out[r][k] = Y[iperm[k]][r - r0], the same way back.
template <typename Real>
__device__ __forceinline__ void store_solution(const Real* __restrict__ Y, Real* lds, const int* __restrict__ iperm,
                                               Real* __restrict__ out, int np, int rows, int64_t r0, int lane) {
  for (int k0 = 0; k0 < np; k0 += kRhs) {
    const int ip = iperm[min(k0 + lane, np - 1)];
#pragma unroll 16
    for (int kk = 0; kk < kRhs; ++kk) {       // past np: a repeat of the last position, not stored
      const int pos = __builtin_amdgcn_readlane(ip, kk);
      lds[lane * kTileRow + kk] = Y[(size_t)pos * kRhs + lane];
    }
    __syncthreads();
    const int k = k0 + lane;
    if (k < np) {
      const int rn = (int)min((int64_t)kRhs, rows - r0);
      for (int rr = 0; rr < rn; ++rr) out[(r0 + rr) * np + k] = lds[rr * kTileRow + lane];
    }
    __syncthreads();
  }
}

// The pointers are kernel arguments (not struct members) so that their no-alias
// guarantee lets uniform entries (the FP64 factor, the diagonal blocks) be fetched by
// scalar loads.
template <typename Real>
__global__ __launch_bounds__(kRhs) void band_solve_kernel(const Real* __restrict__ F, const Real* __restrict__ G,
                                                          const Real* __restrict__ T, const int* __restrict__ iperm,
                                                          const Real* __restrict__ in, Real* __restrict__ out,
                                                          Real* __restrict__ work, int np, int B, int W,
                                                          int rows) {
  extern __shared__ __align__(16) unsigned char smem[];
  Real* lds = reinterpret_cast<Real*>(smem);
  const int lane = threadIdx.x;
  const int nblk = np / kFactorRows;
  const int64_t r0 = (int64_t)blockIdx.x * kRhs;
  Real* __restrict__ Y = work + (size_t)blockIdx.x * np * kRhs;

  load_rhs(in, Y, lds, iperm, np, rows, r0, lane);

  Real* win = lds;              // ring of the last solved positions, [W][64]
  Real nxt[kFactorRows], x[kFactorRows];

  // forward: L y = P q, positions ascending
  for (int s = 0; s < W; ++s) win[s * kRhs + lane] = Real(0);
#pragma unroll
  for (int k = 0; k < kFactorRows; ++k) nxt[k] = Y[(size_t)k * kRhs + lane];
  for (int blk = 0; blk < nblk; ++blk) {
    const int i0 = blk * kFactorRows;
    Real acc[kFactorRows];
#pragma unroll
    for (int k = 0; k < kFactorRows; ++k) acc[k] = nxt[k];
    if (blk + 1 < nblk) {
#pragma unroll
      for (int k = 0; k < kFactorRows; ++k) nxt[k] = Y[(size_t)(i0 + kFactorRows + k) * kRhs + lane];
    }
    band_dot(acc, F + (size_t)blk * B * kFactorRows, win, i0 - B, W, B, lane);
    const Real* __restrict__ Tb = T + (size_t)blk * kFactorDiag;
#pragma unroll
    for (int k = 0; k < kFactorRows; ++k) {
      Real s = acc[k];
#pragma unroll
      for (int l = 0; l < k; ++l) s = fma(-Tb[kFactorRows + k * kFactorRows + l], x[l], s);
      x[k] = s * Tb[k];
    }
    const int slot = i0 % W;                              // i0 and W are multiples of 8
#pragma unroll
    for (int k = 0; k < kFactorRows; ++k) {
      win[(slot + k) * kRhs + lane] = x[k];
      Y[(size_t)(i0 + k) * kRhs + lane] = x[k];
    }
  }

  // backward: L^T z = y, positions descending
  for (int s = 0; s < W; ++s) win[s * kRhs + lane] = Real(0);
#pragma unroll
  for (int k = 0; k < kFactorRows; ++k) nxt[k] = Y[(size_t)(np - kFactorRows + k) * kRhs + lane];
  for (int blk = nblk - 1; blk >= 0; --blk) {
    const int i0 = blk * kFactorRows;
    Real acc[kFactorRows];
#pragma unroll
    for (int k = 0; k < kFactorRows; ++k) acc[k] = nxt[k];
    if (blk > 0) {
#pragma unroll
      for (int k = 0; k < kFactorRows; ++k) nxt[k] = Y[(size_t)(i0 - kFactorRows + k) * kRhs + lane];
    }
    band_dot(acc, G + (size_t)blk * B * kFactorRows, win, i0 + kFactorRows, W, B, lane);
    const Real* __restrict__ Tb = T + (size_t)blk * kFactorDiag;
#pragma unroll
    for (int k = kFactorRows - 1; k >= 0; --k) {
      Real s = acc[k];
#pragma unroll
      for (int l = k + 1; l < kFactorRows; ++l) s = fma(-Tb[kFactorRows + l * kFactorRows + k], x[l], s);
      x[k] = s * Tb[k];
    }
    const int slot = i0 % W;                              // i0 and W are multiples of 8
#pragma unroll
    for (int k = 0; k < kFactorRows; ++k) {
      win[(slot + k) * kRhs + lane] = x[k];
      Y[(size_t)(i0 + k) * kRhs + lane] = x[k];
    }
  }
  __syncthreads();

  store_solution(Y, lds, iperm, out, np, rows, r0, lane);
}

// FP32 substitution on the matrix cores (v_mfma_f32_16x16x4_f32), blocks of 16 positions.
// A block's update from the solved window, acc -= L[block][window] x[window], is a 16 x B
// by B x 64 product: A operand the factor (one entry per lane, so no broadcast), B operand
// the ring (position x right-hand side), four accumulator tiles of 16 right-hand sides
// (lane l holds rows 4 (l >> 4) .. +3 of column l & 15).  The 16 x 16 diagonal block is
// applied as its inverse, 16 more matrix instructions; the right-hand sides reach the B
// layout through the ring slots the block is about to fill.  The factor stream runs one
// 16-position group ahead across blocks, the ring values one group ahead within a block;
// Y rows and the diagonal inverse one block ahead.
typedef float floatx4_t __attribute__((ext_vector_type(4)));

template <bool kFwd>
__device__ __forceinline__ void mfma_pass(const float* __restrict__ A, const float* __restrict__ D,
                                          float* __restrict__ Y, float* win, int np, int B, int W, int lane) {
  const int l16 = lane & 15, kq = lane >> 4;
  const int nb = np / kFactorMfmaRows, ks = B / 4, ng = B / 16;
  for (int s = 0; s < W; ++s) win[s * kRhs + lane] = 0.f;
  const int b_first = kFwd ? 0 : nb - 1;
  floatx4_t nxt[4];
  float an[4], dn[4];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) nxt[t][r] = Y[(size_t)(b_first * 16 + 4 * kq + r) * kRhs + t * 16 + l16];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    an[q] = A[((size_t)b_first * ks + q) * 64 + lane];
    dn[q] = D[((size_t)b_first * 4 + q) * 64 + lane];
  }
  // ring values of a 16-position group starting at slot sb (a multiple of 16, as are B
  // and W, so the group does not wrap), in the B-operand layout
  auto ring_group = [&](int sb, float (&bv)[4][4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int t = 0; t < 4; ++t) bv[q][t] = win[(sb + 4 * q + kq) * kRhs + t * 16 + l16];
  };
  auto first_slot = [&](int i0) {
    const int base = kFwd ? i0 - B : i0 + kFactorMfmaRows;
    return ((base % W) + W) % W;
  };
  float bn_[4][4];
  ring_group(first_slot(b_first * kFactorMfmaRows), bn_);
  for (int it = 0; it < nb; ++it) {
    const int bi = kFwd ? it : nb - 1 - it;
    const bool more = it + 1 < nb;
    const int bn = kFwd ? bi + 1 : bi - 1;
    const int i0 = bi * kFactorMfmaRows;
    floatx4_t acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = nxt[t];
    if (more) {
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) nxt[t][r] = Y[(size_t)(bn * 16 + 4 * kq + r) * kRhs + t * 16 + l16];
    }
    const float* __restrict__ Ab = A + (size_t)bi * ks * 64;
    const float* __restrict__ An = more ? A + (size_t)bn * ks * 64 : nullptr;
    int sb = first_slot(i0);
    for (int g = 0; g < ng; ++g) {
      float a[4], bv[4][4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = an[q];
#pragma unroll
        for (int t = 0; t < 4; ++t) bv[q][t] = bn_[q][t];
      }
      const float* __restrict__ src = g + 1 < ng ? Ab + (g + 1) * 256 : An;
      if (src) {
#pragma unroll
        for (int q = 0; q < 4; ++q) an[q] = src[q * 64 + lane];
      }
      sb = sb + 16 == W ? 0 : sb + 16;
      if (g + 1 < ng) ring_group(sb, bn_);           // the next group: solved positions only
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q], bv[q][t], acc[t], 0, 0, 0);
    }
    // the diagonal block: x = L_D^-1 acc (forward) or L_D^-T acc (backward)
    float d[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) d[q] = dn[q];
    if (more) {
#pragma unroll
      for (int q = 0; q < 4; ++q) dn[q] = D[((size_t)bn * 4 + q) * 64 + lane];
    }
    const int sd = i0 % W;                           // multiples of 16: no wrap inside the block
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) win[(sd + 4 * kq + r) * kRhs + t * 16 + l16] = acc[t][r];
    floatx4_t x[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) x[t] = floatx4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int t = 0; t < 4; ++t)
        x[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(d[q], win[(sd + 4 * q + kq) * kRhs + t * 16 + l16], x[t], 0, 0, 0);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        win[(sd + 4 * kq + r) * kRhs + t * 16 + l16] = x[t][r];
        Y[(size_t)(i0 + 4 * kq + r) * kRhs + t * 16 + l16] = x[t][r];
      }
    // the next block's first group, which may hold the positions just solved
    if (more) ring_group(first_slot(bn * kFactorMfmaRows), bn_);
  }
}

__global__ __launch_bounds__(kRhs) void band_solve_mfma_kernel(const float* __restrict__ FA,
                                                               const float* __restrict__ GA,
                                                               const float* __restrict__ DA,
                                                               const float* __restrict__ DB,
                                                               const int* __restrict__ iperm,
                                                               const float* __restrict__ in, float* __restrict__ out,
                                                               float* __restrict__ work, int np, int B, int W,
                                                               int rows) {
  extern __shared__ __align__(16) unsigned char smem[];
  float* lds = reinterpret_cast<float*>(smem);
  const int lane = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * kRhs;
  float* __restrict__ Y = work + (size_t)blockIdx.x * np * kRhs;
  load_rhs(in, Y, lds, iperm, np, rows, r0, lane);       // ends with a barrier: Y visible to all lanes
  mfma_pass<true>(FA, DA, Y, lds, np, B, W, lane);
  mfma_pass<false>(GA, DB, Y, lds, np, B, W, lane);
  __syncthreads();
  store_solution(Y, lds, iperm, out, np, rows, r0, lane);
}

}  // namespace

template <typename Real>
size_t band_solve_lds_bytes(int ring) {
  return (size_t)std::max(ring, kTileRow) * kRhs * sizeof(Real);
}

size_t band_solve_work_bytes(int n_pad, int rows, int real_bytes) {
  return (size_t)((rows + kRhs - 1) / kRhs) * kRhs * n_pad * real_bytes;
}

template <typename Real>
hipError_t launch_band_solve(const BandFactorDev<Real>& f, int which, int n_pad, const Real* in, Real* out,
                             Real* work, int rows, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  const size_t lds = band_solve_lds_bytes<Real>(f.ring);
  if (lds > kBandSolveMaxLds) return hipErrorInvalidValue;
  const int grid = (rows + kRhs - 1) / kRhs;
  const void* fn;
  if constexpr (std::is_same<Real, float>::value) fn = reinterpret_cast<const void*>(&band_solve_mfma_kernel);
  else fn = reinterpret_cast<const void*>(&band_solve_kernel<double>);
  if (lds > 64 * 1024) {          // above the default dynamic LDS limit (set on the current device)
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if constexpr (std::is_same<Real, float>::value)
    hipLaunchKernelGGL(band_solve_mfma_kernel, dim3(grid), dim3(kRhs), lds, s, f.FA[which], f.GA[which],
                       f.DA[which], f.DB[which], f.iperm, in, out, work, n_pad, f.B, f.ring, rows);
  else
    hipLaunchKernelGGL(band_solve_kernel<double>, dim3(grid), dim3(kRhs), lds, s, f.F[which], f.G[which],
                       f.T[which], f.iperm, in, out, work, n_pad, f.B, f.ring, rows);
  return hipGetLastError();
}

template size_t band_solve_lds_bytes<float>(int);
template size_t band_solve_lds_bytes<double>(int);
template hipError_t launch_band_solve<float>(const BandFactorDev<float>&, int, int, const float*, float*, float*,
                                             int, hipStream_t);
template hipError_t launch_band_solve<double>(const BandFactorDev<double>&, int, int, const double*, double*,
                                              double*, int, hipStream_t);

}  // namespace npfem
