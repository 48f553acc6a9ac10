// gfx950 kernels of the learned warm start: per-cell frame and features, network
// inference and training (forward, loss, backward, gradient reduction, Adam).
//
// One workgroup (4 wave64) carries one cell at a time.  Node-wise products with the
// 64 x 64 (or 64 x 128) weight blocks run on the matrix cores
// (v_mfma_f32_16x16x32_bf16): each wave takes 16-node row blocks; the A operand of a
// layer is [h_i | mean_{j in N(i)} h_j] built on the fly from the activations in
// memory (8 consecutive features per lane, gathered over the neighbour list), the B
// operand is the weight block held in registers.  Weight gradients are sums over
// nodes: 32-node chunks are staged transposed in LDS so that the node index becomes
// the contiguous k dimension of the matrix instruction.  Every per-workgroup gradient
// sum goes to its own slot and the slots are reduced in a fixed order, so training is
// deterministic.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "npfem_internal.h"
#include "npfem_net_internal.h"

namespace npfem {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kRS = 16;     // reduction stride (values per wave)
constexpr int kTP = 40;     // LDS row pitch (BF16) of the transposed 32-node chunks
constexpr int kNetUnrollDeg = 6;   // neighbour gathers issued together (the icosphere degree)

__device__ inline int tid() { return threadIdx.x; }

__device__ inline float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ inline uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ inline bf16x8 ld8(const uint16_t* p) { return *reinterpret_cast<const bf16x8*>(p); }
__device__ inline bf16x8 zero8() {
  const __bf16 z = (__bf16)0.f;
  return bf16x8{z, z, z, z, z, z, z, z};
}

template <int N, int NW = 4>
__device__ inline void wg_sum(double (&v)[N], double* red) {
  static_assert(N <= kRS, "wg_sum: too many values");
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double x = v[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    v[i] = x;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) red[wave * kRS + i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) t += red[w * kRS + i];
    v[i] = t;
  }
}

// Orthogonal polar factor of a 3x3 matrix with positive determinant (scaled Newton
// iteration X <- (g X + X^-T / g) / 2, g = (|X^-1|_F / |X|_F)^(1/2); Higham 1986).
// This is the Kabsch rotation: C = U S V^T -> U V^T.  Identity for det <= 0.
__device__ void polar3(const double* C, double* R) {
  double X[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) X[k] = C[k];
  const double d0 = X[0] * (X[4] * X[8] - X[5] * X[7]) - X[1] * (X[3] * X[8] - X[5] * X[6]) +
                    X[2] * (X[3] * X[7] - X[4] * X[6]);
  if (!(d0 > 0.0) || !isfinite(d0)) {
#pragma unroll
    for (int k = 0; k < 9; ++k) R[k] = (k % 4 == 0) ? 1.0 : 0.0;
    return;
  }
  for (int it = 0; it < 60; ++it) {
    double cof[9];
    cof[0] = X[4] * X[8] - X[5] * X[7];
    cof[1] = X[5] * X[6] - X[3] * X[8];
    cof[2] = X[3] * X[7] - X[4] * X[6];
    cof[3] = X[2] * X[7] - X[1] * X[8];
    cof[4] = X[0] * X[8] - X[2] * X[6];
    cof[5] = X[1] * X[6] - X[0] * X[7];
    cof[6] = X[1] * X[5] - X[2] * X[4];
    cof[7] = X[2] * X[3] - X[0] * X[5];
    cof[8] = X[0] * X[4] - X[1] * X[3];
    const double d = X[0] * cof[0] + X[1] * cof[1] + X[2] * cof[2];
    const double id = 1.0 / d;
    double nx = 0.0, nc = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      nx += X[k] * X[k];
      nc += cof[k] * cof[k];
    }
    const double g = sqrt(sqrt(nc * id * id / nx));          // (|X^-1|_F / |X|_F)^(1/2)
    const double cg = 0.5 * id / g, xg = 0.5 * g;
    double diff = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const double xn = xg * X[k] + cg * cof[k];
      diff += (xn - X[k]) * (xn - X[k]);
      X[k] = xn;
    }
    if (diff <= 1e-30) break;
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = X[k];
}

// ---------------------------------------------------------------------------------
// Forward: frame, features, encoder, message-passing layers, decoder.
// ---------------------------------------------------------------------------------

// Frame (mass-weighted centroids, covariance with the rest shape, Kabsch) and the node
// features of cell k, written as BF16 rows of 32 (zero padded) to feat.  Leaves R and
// s in fr[0..9] (LDS) and ends with a barrier.
template <typename Real, int NT>
__device__ void cell_features(const NetFwdArgs<Real>& A, const NetMeshDev& M, int k, const Real* x, const Real* v,
                              const Real* f, uint16_t* feat, uint16_t* feat2, double* red, double* fr) {
  const int n = M.n, np = M.n_pad;
  double s1[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int i = tid(); i < n; i += NT) {
    const double m = M.mass[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      s1[c] += m * (double)x[3 * i + c];
      s1[3 + c] += m * (double)v[3 * i + c];
      s1[6 + c] += (double)f[3 * i + c];
    }
  }
  wg_sum<9, NT / 64>(s1, red);
  const double ims = 1.0 / M.mass_sum;
  const double xc[3] = {s1[0] * ims, s1[1] * ims, s1[2] * ims};
  const double vc[3] = {s1[3] * ims, s1[4] * ims, s1[5] * ims};
  const double ac[3] = {s1[6] * ims, s1[7] * ims, s1[8] * ims};
  double s2[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int i = tid(); i < n; i += NT) {
    const double m = M.mass[i];
    double d[3], fd[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      d[c] = (double)x[3 * i + c] - xc[c];
      fd[c] = (double)f[3 * i + c] - m * ac[c];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) s2[3 * a + b] += m * d[a] * M.Xc[3 * i + b];
    s2[9] += fd[0] * fd[0] + fd[1] * fd[1] + fd[2] * fd[2];
  }
  wg_sum<10, NT / 64>(s2, red);
  if (tid() == 0) {
    double R[9];
    polar3(s2, R);
    const double s = A.h * A.h * (sqrt(s2[9] / n) + A.W.force_floor) / M.mass_mean;
#pragma unroll
    for (int q = 0; q < 9; ++q) fr[q] = R[q];
    fr[9] = s;
    if (A.S.frame) {
#pragma unroll
      for (int q = 0; q < 10; ++q) A.S.frame[(size_t)k * 12 + q] = fr[q];
    }
  }
  __syncthreads();
  double R[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) R[q] = fr[q];
  const double s = fr[9];
  const double hs = A.h / s, h2s = A.h * A.h / s, iq = 1.0 / A.W.shape_scale;
  for (int i = tid(); i < np; i += NT) {
    float fv[kNetFeat];
#pragma unroll
    for (int q = 0; q < kNetFeat; ++q) fv[q] = 0.f;
    if (i < n) {
      const double m = M.mass[i];
      double d[3], dv[3], df[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        d[c] = (double)x[3 * i + c] - xc[c];
        dv[c] = (double)v[3 * i + c] - vc[c];
        df[c] = (double)f[3 * i + c] - m * ac[c];
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        double rd = 0.0, rv = 0.0, rf = 0.0;                 // (R^T w)_a = sum_b R[b][a] w_b
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          rd += R[3 * b + a] * d[b];
          rv += R[3 * b + a] * dv[b];
          rf += R[3 * b + a] * df[b];
        }
        const double Xa = M.Xc[3 * i + a];
        fv[a] = (float)((rd - Xa) * iq);
        fv[3 + a] = (float)(rv * hs);
        fv[6 + a] = (float)(rf * h2s / m);
        fv[9 + a] = (float)(Xa * M.inv_rho);
      }
    }
    bf16x8 w0, w1;
#pragma unroll
    for (int e = 0; e < 8; ++e) w0[e] = (__bf16)fv[e];
#pragma unroll
    for (int e = 0; e < 8; ++e) w1[e] = (__bf16)(e < 4 ? fv[8 + e] : 0.f);
    for (uint16_t* base : {feat, feat2}) {
      if (!base) continue;
      uint16_t* fp = base + (size_t)i * kNetFeatPad;
      *reinterpret_cast<bf16x8*>(fp) = w0;
      *reinterpret_cast<bf16x8*>(fp + 8) = w1;
      *reinterpret_cast<bf16x8*>(fp + 16) = zero8();
      *reinterpret_cast<bf16x8*>(fp + 24) = zero8();
    }
  }
  __syncthreads();
}

// Encoder rows of the waves w = wave, wave + NWV, ...: h0 = relu(W_e f + b_e) into
// H (row pitch hp); training also stores h0 and z0 (pitch kNetH) to Hg / Zg.
template <int NWV>
__device__ void encoder_rows(const NetWeights& W, const uint16_t* feat, int n, int np, uint16_t* H, int hp,
                             uint16_t* Hg, uint16_t* Zg) {
  const int lane = tid() & 63, wave = tid() >> 6, l16 = lane & 15, kq = lane >> 4;
  bf16x8 bq[4];
  float bias[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    bq[cb] = ld8(W.We + (size_t)(cb * 16 + l16) * kNetFeatPad + 8 * kq);
    bias[cb] = W.theta[W.lay.off_be + cb * 16 + l16];
  }
  for (int rb = wave; rb < (np >> 4); rb += NWV) {
    const bf16x8 aq = ld8(feat + (size_t)(rb * 16 + l16) * kNetFeatPad + 8 * kq);
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const floatx4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aq, bq[cb], floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = rb * 16 + 4 * kq + i, col = cb * 16 + l16;
        const float z = row < n ? acc[i] + bias[cb] : 0.f;
        const uint16_t hb = f2bf(fmaxf(z, 0.f));
        H[(size_t)row * hp + col] = hb;
        if (Hg) {
          Hg[(size_t)row * kNetH + col] = hb;
          Zg[(size_t)row * kNetH + col] = f2bf(z);
        }
      }
    }
  }
}

// Decoder on the matrix cores: o = W_d h + b_d (3 outputs padded to one 16-column
// block); lanes l16 = 0, 1, 2 of each 16-lane group hold the components of a row and
// exchange them to form the correction s R o (world frame) and/or store o.
template <typename Real, int NWV>
__device__ void decoder_rows(const NetFwdArgs<Real>& A, int k, int64_t voff, int n, int np, const uint16_t* H,
                             int hp, const double* fr) {
  const int lane = tid() & 63, wave = tid() >> 6, l16 = lane & 15, kq = lane >> 4;
  double R[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) R[q] = fr[q];
  const double s = fr[9];
  bf16x8 bq[2];
#pragma unroll
  for (int s2 = 0; s2 < 2; ++s2) bq[s2] = l16 < 3 ? ld8(A.W.Wd + (size_t)l16 * kNetH + 32 * s2 + 8 * kq) : zero8();
  const float bias = l16 < 3 ? A.W.theta[A.W.lay.off_bd + l16] : 0.f;
  for (int rb = wave; rb < (np >> 4); rb += NWV) {
    const int row = rb * 16 + l16;
    floatx4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ld8(H + (size_t)row * hp + 8 * kq), bq[0],
                                                          floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ld8(H + (size_t)row * hp + 32 + 8 * kq), bq[1], acc, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float o = acc[i] + bias;                    // o[4kq + i][l16]
      const float o0 = __shfl(o, kq * 16, 64), o1 = __shfl(o, kq * 16 + 1, 64), o2 = __shfl(o, kq * 16 + 2, 64);
      const int r2 = rb * 16 + 4 * kq + i;
      if (r2 < n && l16 < 3) {
        if (A.delta) {
          const double da = s * (R[3 * l16] * o0 + R[3 * l16 + 1] * o1 + R[3 * l16 + 2] * o2);
          A.delta[3 * (voff + r2) + l16] = (Real)da;
        }
        if (A.S.out) A.S.out[((size_t)k * A.S.n_pad_max + r2) * 3 + l16] = o;
      }
    }
  }
}

// One message-passing layer over the row blocks of this wave: reads h (row pitch hp)
// and its neighbour means, writes h + relu(z) to Hout (pitch kNetH) and z to Zout.
// Neighbour j of row i: nbr(q, i) for q < deg(i).
template <int NWV, typename NbrF, typename DegF>
__device__ void layer_rows(const NetWeights& W, int l, int n, int np, int width, const uint16_t* Hin, int hp,
                           uint16_t* Hout, uint16_t* Zout, NbrF nbr, DegF deg) {
  const int lane = tid() & 63, wave = tid() >> 6, l16 = lane & 15, kq = lane >> 4;
  const uint16_t* Wl = W.Wl + (size_t)l * kNetH * 2 * kNetH;
  bf16x8 bq[4][4];
  float bias[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) bq[s4][cb] = ld8(Wl + (size_t)(cb * 16 + l16) * 2 * kNetH + 32 * s4 + 8 * kq);
    bias[cb] = W.theta[W.lay.b(l) + cb * 16 + l16];
  }
  for (int rb = wave; rb < (np >> 4); rb += NWV) {
    const int row = rb * 16 + l16;
    bf16x8 aq[4];
    if (row < n) {
      aq[0] = ld8(Hin + (size_t)row * hp + 8 * kq);
      aq[1] = ld8(Hin + (size_t)row * hp + 32 + 8 * kq);
      float g0[8], g1[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) g0[e] = g1[e] = 0.f;
      const int dg = deg(row);
      // the first kNetUnrollDeg ELL columns are loaded unconditionally (ELL padding points
      // at the row itself, so every address is valid) and masked by the degree; wider
      // meshes continue in a rolled loop
#pragma unroll
      for (int q = 0; q < kNetUnrollDeg; ++q) {
        const int j = q < width ? nbr(q, row) : row;
        const float w = q < dg ? 1.f : 0.f;
        const bf16x8 h0 = ld8(Hin + (size_t)j * hp + 8 * kq);
        const bf16x8 h1 = ld8(Hin + (size_t)j * hp + 32 + 8 * kq);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          g0[e] += w * (float)h0[e];
          g1[e] += w * (float)h1[e];
        }
      }
      for (int q = kNetUnrollDeg; q < dg; ++q) {
        const int j = nbr(q, row);
        const bf16x8 h0 = ld8(Hin + (size_t)j * hp + 8 * kq);
        const bf16x8 h1 = ld8(Hin + (size_t)j * hp + 32 + 8 * kq);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          g0[e] += (float)h0[e];
          g1[e] += (float)h1[e];
        }
      }
      const float inv = 1.0f / (float)dg;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        aq[2][e] = (__bf16)(g0[e] * inv);
        aq[3][e] = (__bf16)(g1[e] * inv);
      }
    } else {
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) aq[s4] = zero8();
    }
    floatx4 acc[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[cb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aq[s4], bq[s4][cb], acc[cb], 0, 0, 0);
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r2 = rb * 16 + 4 * kq + i, col = cb * 16 + l16;
        const float z = r2 < n ? acc[cb][i] + bias[cb] : 0.f;
        const float hn = r2 < n ? bf2f(Hin[(size_t)r2 * hp + col]) + fmaxf(z, 0.f) : 0.f;
        Hout[(size_t)r2 * kNetH + col] = f2bf(hn);
        if (Zout) Zout[(size_t)r2 * kNetH + col] = f2bf(z);
      }
    }
  }
}

// Variant for any mesh size: activations ping-pong in memory, neighbours from CSR.
template <typename Real>
__global__ void __launch_bounds__(kBlock) net_forward_kernel(NetFwdArgs<Real> A) {
  __shared__ double red[4 * kRS];
  __shared__ double fr[10];
  const NetLayout L = A.W.lay;
  const bool train = A.S.train != 0;
  const size_t plane = (size_t)A.S.n_pad_max * kNetH;
  const int nh = train ? L.layers + 1 : 2;
  for (int k = blockIdx.x; k < A.n_cells; k += gridDim.x) {
    const int cell = A.cells ? A.cells[k] : k;
    const NetMeshDev& M = A.meshes[A.cell_mesh[cell]];
    const int n = M.n, np = M.n_pad;
    const int64_t voff = A.cell_voff[cell];
    const size_t slot = train ? (size_t)k : (size_t)blockIdx.x;
    uint16_t* feat = A.S.feat + slot * A.S.n_pad_max * kNetFeatPad;
    uint16_t* Hs = A.S.H + slot * nh * plane;
    uint16_t* Zs = train ? A.S.Z + slot * (L.layers + 1) * plane : nullptr;
    cell_features<Real, kBlock>(A, M, k, A.x + 3 * voff, A.v + 3 * voff, A.f + 3 * voff, feat, nullptr, red, fr);
    encoder_rows<kBlock / 64>(A.W, feat, n, np, Hs, kNetH, nullptr, nullptr);
    if (train) {                              // z0 for the backward pass
      __syncthreads();
      encoder_rows<kBlock / 64>(A.W, feat, n, np, Hs, kNetH, Hs, Zs);
    }
    __syncthreads();
    auto nbr = [&](int q, int i) { return M.nb_ell[q * np + i]; };
    auto deg = [&](int i) { return M.nb_ptr[i + 1] - M.nb_ptr[i]; };
    for (int l = 0; l < L.layers; ++l) {
      const uint16_t* Hin = Hs + (size_t)(train ? l : (l & 1)) * plane;
      uint16_t* Hout = Hs + (size_t)(train ? l + 1 : ((l + 1) & 1)) * plane;
      layer_rows<kBlock / 64>(A.W, l, n, np, M.nb_deg, Hin, kNetH, Hout, train ? Zs + (size_t)(l + 1) * plane : nullptr,
                              nbr, deg);
      __syncthreads();
    }
    const uint16_t* HL = Hs + (size_t)(train ? L.layers : (L.layers & 1)) * plane;
    decoder_rows<Real, kBlock / 64>(A, k, voff, n, np, HL, kNetH, fr);
    __syncthreads();
  }
}

// LDS-resident variant (meshes whose activations fit a compute unit): 512 threads; the
// cell's activations live in LDS (row pitch kHP, so 16-byte operand reads of 8
// consecutive rows fall in distinct banks) together with the mesh's neighbour lists;
// each layer's output goes to memory (L2) and is copied back after a barrier.
constexpr int kNetLdsBlock = 512;
constexpr int kHP = 72;
constexpr int kNetLdsHeader = 8 * kRS * 8 + 16 * 8;   // reduction, frame

template <typename Real>
__global__ void __launch_bounds__(kNetLdsBlock) net_forward_lds_kernel(NetFwdArgs<Real> A) {
  const int np_max = A.S.n_pad_max, deg_max = A.nb_deg_max;
  extern __shared__ __align__(16) unsigned char lds[];
  double* red = reinterpret_cast<double*>(lds);
  double* fr = red + 8 * kRS;
  uint16_t* Hl = reinterpret_cast<uint16_t*>(lds + kNetLdsHeader);
  uint16_t* Fl = Hl + (size_t)np_max * kHP;                    // features [np_max][32]
  uint16_t* nbl = Fl + (size_t)np_max * kNetFeatPad;
  uint8_t* degl = reinterpret_cast<uint8_t*>(nbl + (size_t)deg_max * np_max);
  constexpr int NT = kNetLdsBlock, NWV = kNetLdsBlock / 64;
  const NetLayout L = A.W.lay;
  const bool train = A.S.train != 0;
  const size_t plane = (size_t)A.S.n_pad_max * kNetH;
  const int nh = train ? L.layers + 1 : 2;
  int staged = -1;
  for (int k = blockIdx.x; k < A.n_cells; k += gridDim.x) {
    const int cell = A.cells ? A.cells[k] : k;
    const int mi = A.cell_mesh[cell];
    const NetMeshDev& M = A.meshes[mi];
    const int n = M.n, np = M.n_pad;
    const int64_t voff = A.cell_voff[cell];
    if (mi != staged) {                       // neighbour lists of this mesh type into LDS
      __syncthreads();
      for (int e = tid(); e < M.nb_deg * np; e += NT) nbl[e] = (uint16_t)M.nb_ell[e];
      for (int i = tid(); i < np; i += NT) degl[i] = (uint8_t)(i < n ? M.nb_ptr[i + 1] - M.nb_ptr[i] : 0);
      staged = mi;
    }
    const size_t slot = train ? (size_t)k : (size_t)blockIdx.x;
    uint16_t* feat = A.S.feat + slot * A.S.n_pad_max * kNetFeatPad;
    uint16_t* Hs = A.S.H + slot * nh * plane;
    uint16_t* Zs = train ? A.S.Z + slot * (L.layers + 1) * plane : nullptr;
    cell_features<Real, NT>(A, M, k, A.x + 3 * voff, A.v + 3 * voff, A.f + 3 * voff, Fl, train ? feat : nullptr,
                            red, fr);
    encoder_rows<NWV>(A.W, Fl, n, np, Hl, kHP, train ? Hs : nullptr, Zs);
    __syncthreads();
    auto nbr = [&](int q, int i) { return (int)nbl[q * np + i]; };
    auto deg = [&](int i) { return (int)degl[i]; };
    for (int l = 0; l < L.layers; ++l) {
      uint16_t* Hout = Hs + (size_t)(train ? l + 1 : 0) * plane;
      layer_rows<NWV>(A.W, l, n, np, M.nb_deg, Hl, kHP, Hout, train ? Zs + (size_t)(l + 1) * plane : nullptr, nbr,
                      deg);
      __syncthreads();
      const int chunks = np * (kNetH / 8);
      for (int c0 = tid(); c0 < chunks; c0 += 4 * NT) {
        bf16x8 t[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {                   // loads issued together (clamped, always valid)
          const int c = min(c0 + u * NT, chunks - 1);
          t[u] = ld8(Hout + (size_t)(c >> 3) * kNetH + 8 * (c & 7));
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int c = c0 + u * NT;
          if (c < chunks) *reinterpret_cast<bf16x8*>(Hl + (size_t)(c >> 3) * kHP + 8 * (c & 7)) = t[u];
        }
      }
      __syncthreads();
    }
    decoder_rows<Real, NWV>(A, k, voff, n, np, Hl, kHP, fr);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------
// Inference: the frame of every cell first (one wave per cell), then the network with
// the cell's activations resident in LDS and updated in place.
// ---------------------------------------------------------------------------------

__device__ inline double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Per cell k: R (rest -> world, row-major), the displacement scale s, and the centroid,
// mean velocity and mean acceleration used by the features (kNetFrame doubles).
template <typename Real>
__global__ void __launch_bounds__(256) net_frame_kernel(NetFwdArgs<Real> A) {
  const int lane = tid() & 63;
  const int k = blockIdx.x * 4 + (tid() >> 6);
  if (k >= A.n_cells) return;
  const int cell = A.cells ? A.cells[k] : k;
  const NetMeshDev& M = A.meshes[A.cell_mesh[cell]];
  const int n = M.n;
  const int64_t voff = A.cell_voff[cell];
  const Real* x = A.x + 3 * voff;
  const Real* v = A.v + 3 * voff;
  const Real* f = A.f + 3 * voff;
  double s1[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int i = lane; i < n; i += 64) {
    const double m = M.mass[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      s1[c] += m * (double)x[3 * i + c];
      s1[3 + c] += m * (double)v[3 * i + c];
      s1[6 + c] += (double)f[3 * i + c];
    }
  }
#pragma unroll
  for (int q = 0; q < 9; ++q) s1[q] = wave_sum(s1[q]);
  const double ims = 1.0 / M.mass_sum;
  double fr[kNetFrame];
#pragma unroll
  for (int q = 0; q < 9; ++q) fr[10 + q] = s1[q] * ims;      // x_c, v_c, a_c
  double s2[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int i = lane; i < n; i += 64) {
    const double m = M.mass[i];
    double d[3], fd[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      d[c] = (double)x[3 * i + c] - fr[10 + c];
      fd[c] = (double)f[3 * i + c] - m * fr[16 + c];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) s2[3 * a + b] += m * d[a] * M.Xc[3 * i + b];
    s2[9] += fd[0] * fd[0] + fd[1] * fd[1] + fd[2] * fd[2];
  }
#pragma unroll
  for (int q = 0; q < 10; ++q) s2[q] = wave_sum(s2[q]);
  polar3(s2, fr);                                          // every lane, the same values
  fr[9] = A.h * A.h * (sqrt(s2[9] / n) + A.W.force_floor) / M.mass_mean;
  fr[19] = 0.0;
  double* out = A.cframe + (size_t)k * kNetFrame;
#pragma unroll
  for (int q = 0; q < kNetFrame; ++q)
    if (lane == q) out[q] = fr[q];
}

constexpr int kInfBlock = 512;
constexpr int kInfWaves = kInfBlock / 64;
constexpr int kInfMaxRegRounds = 3;            // row-block rounds whose results stay in registers

// LDS of the resident inference: h [n_pad][kHP] bf16, the neighbour lists, the degrees,
// then the staging of the rounds beyond kInfMaxRegRounds (16 KB per round).
__host__ __device__ inline size_t infer_lds_base(int n_pad, int nb_deg) {
  return ((size_t)n_pad * kHP * 2 + (size_t)nb_deg * n_pad * 2 + (size_t)n_pad + 15) / 16 * 16;
}

// One message-passing layer of the resident variant.  Every wave computes h + relu(z)
// for its row blocks rb = wave + kInfWaves r: the first RL rounds into the LDS staging
// area Ob (per block, 8 packed dwords per lane), the last RR rounds into registers;
// after a barrier all of them are written over h in LDS (the layer reads every
// neighbour's old h before any row is overwritten).  The neighbour sums take one bf16
// half of a dword per dot2 instruction (the other half weighted 0), so activations are
// added in FP32 without being unpacked first.
template <int RR>
__device__ __attribute__((always_inline)) inline void infer_layer(const NetWeights& W, int l, int n, int np,
                                                                  int width, uint16_t* H, const uint16_t* nbl,
                                                                  const uint8_t* degl, uint32_t* Ob, int RL) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  const int lane = tid() & 63, wave = tid() >> 6, l16 = lane & 15, kq = lane >> 4;
  const uint16_t* Wl = W.Wl + (size_t)l * kNetH * 2 * kNetH;
  bf16x8 bq[4][4];
  float bias[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) bq[s4][cb] = ld8(Wl + (size_t)(cb * 16 + l16) * 2 * kNetH + 32 * s4 + 8 * kq);
    bias[cb] = W.theta[W.lay.b(l) + cb * 16 + l16];
  }
  const bf16x2 one_lo = {(__bf16)1.f, (__bf16)0.f}, one_hi = {(__bf16)0.f, (__bf16)1.f};
  const bf16x2 zero2 = {(__bf16)0.f, (__bf16)0.f};
  const int nrb = np >> 4;
  // new h of row block rb: rows rb*16 + 4kq + i, column cb*16 + l16, as bf16 pairs over i
  auto block = [&](int rb, uint32_t (&o)[8]) {
    const int row = rb * 16 + l16;
    bf16x8 aq[4];
    aq[0] = ld8(H + (size_t)row * kHP + 8 * kq);
    aq[1] = ld8(H + (size_t)row * kHP + 32 + 8 * kq);
    float g[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) g[e] = 0.f;
    const int dg = degl[row];                              // 0 for padding rows
    auto add = [&](int j, bf16x2 wl, bf16x2 wh) {
      const uint4 h0 = *reinterpret_cast<const uint4*>(H + (size_t)j * kHP + 8 * kq);
      const uint4 h1 = *reinterpret_cast<const uint4*>(H + (size_t)j * kHP + 32 + 8 * kq);
      const uint32_t w[8] = {h0.x, h0.y, h0.z, h0.w, h1.x, h1.y, h1.z, h1.w};
#pragma unroll
      for (int d = 0; d < 8; ++d) {
        const bf16x2 p = __builtin_bit_cast(bf16x2, w[d]);
        g[2 * d] = __builtin_amdgcn_fdot2_f32_bf16(p, wl, g[2 * d], false);
        g[2 * d + 1] = __builtin_amdgcn_fdot2_f32_bf16(p, wh, g[2 * d + 1], false);
      }
    };
    // the first kNetUnrollDeg ELL columns are read unconditionally (ELL padding points
    // at the row itself) and weighted by q < degree; wider meshes go on in a loop
#pragma unroll
    for (int q = 0; q < kNetUnrollDeg; ++q) {
      const int j = q < width ? (int)nbl[q * np + row] : row;
      const bool on = q < dg;
      add(j, on ? one_lo : zero2, on ? one_hi : zero2);
    }
    for (int q = kNetUnrollDeg; q < dg; ++q) add((int)nbl[q * np + row], one_lo, one_hi);
    const float inv = dg > 0 ? 1.0f / (float)dg : 0.f;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      aq[2][e] = (__bf16)(g[e] * inv);
      aq[3][e] = (__bf16)(g[8 + e] * inv);
    }
    floatx4 acc[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[cb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aq[s4], bq[s4][cb], acc[cb], 0, 0, 0);
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      float hv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r2 = rb * 16 + 4 * kq + i;
        const float z = acc[cb][i] + bias[cb];
        hv[i] = r2 < n ? bf2f(H[(size_t)r2 * kHP + cb * 16 + l16]) + fmaxf(z, 0.f) : 0.f;
      }
      o[2 * cb] = __builtin_bit_cast(uint32_t, bf16x2{(__bf16)hv[0], (__bf16)hv[1]});
      o[2 * cb + 1] = __builtin_bit_cast(uint32_t, bf16x2{(__bf16)hv[2], (__bf16)hv[3]});
    }
  };
  auto put = [&](int rb, const uint32_t (&o)[8]) {
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r2 = rb * 16 + 4 * kq + i;
        const uint32_t w = o[2 * cb + (i >> 1)];
        H[(size_t)r2 * kHP + cb * 16 + l16] = (uint16_t)((i & 1) ? (w >> 16) : (w & 0xffffu));
      }
  };
  uint32_t* ob = Ob + (size_t)wave * 8 * 64 + lane;        // this lane's dwords of round r: ob[r * kInfWaves * 512 + 64 d]
  for (int r = 0; r < RL; ++r) {
    const int rb = wave + kInfWaves * r;
    if (rb >= nrb) break;                                  // uniform over the wave
    uint32_t o[8];
    block(rb, o);
#pragma unroll
    for (int d = 0; d < 8; ++d) ob[(size_t)r * kInfWaves * 512 + 64 * d] = o[d];
  }
  uint32_t out[RR][8];
#pragma unroll
  for (int r = 0; r < RR; ++r) {
    const int rb = wave + kInfWaves * (RL + r);
    if (rb >= nrb) break;
    block(rb, out[r]);
  }
  __syncthreads();
  for (int r = 0; r < RL; ++r) {
    const int rb = wave + kInfWaves * r;
    if (rb >= nrb) break;
    uint32_t o[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) o[d] = ob[(size_t)r * kInfWaves * 512 + 64 * d];
    put(rb, o);
  }
#pragma unroll
  for (int r = 0; r < RR; ++r) {
    const int rb = wave + kInfWaves * (RL + r);
    if (rb >= nrb) break;
    put(rb, out[r]);
  }
  __syncthreads();
}

// Resident inference: one cell at a time per workgroup (512 threads), its activations
// [n_pad][kHP] and its mesh's neighbour lists in LDS.  The encoder computes each row's
// features from x_n, v_n, F_ext and the cell's frame as it forms its operand.
template <typename Real, int RR>
__global__ void __launch_bounds__(kInfBlock) net_infer_kernel(NetFwdArgs<Real> A, int RL) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int np_max = A.S.n_pad_max;
  uint16_t* H = reinterpret_cast<uint16_t*>(lds);
  uint16_t* nbl = H + (size_t)np_max * kHP;
  uint8_t* degl = reinterpret_cast<uint8_t*>(nbl + (size_t)A.nb_deg_max * np_max);
  uint32_t* Ob = reinterpret_cast<uint32_t*>(lds + infer_lds_base(np_max, A.nb_deg_max));
  const int lane = tid() & 63, wave = tid() >> 6, l16 = lane & 15, kq = lane >> 4;
  const NetLayout L = A.W.lay;
  int staged = -1;
  for (int k = blockIdx.x; k < A.n_cells; k += gridDim.x) {
    const int cell = A.cells ? A.cells[k] : k;
    const int mi = A.cell_mesh[cell];
    const NetMeshDev& M = A.meshes[mi];
    const int n = M.n, np = M.n_pad, nrb = np >> 4;
    const int64_t voff = A.cell_voff[cell];
    __syncthreads();                                       // the previous cell's decoder is done with H
    if (mi != staged) {                                    // neighbour lists of this mesh type
      for (int e = tid(); e < M.nb_deg * np; e += kInfBlock) nbl[e] = (uint16_t)M.nb_ell[e];
      for (int i = tid(); i < np; i += kInfBlock) degl[i] = (uint8_t)(i < n ? M.nb_ptr[i + 1] - M.nb_ptr[i] : 0);
      staged = mi;
    }
    const double* fr = A.cframe + (size_t)k * kNetFrame;
    // ---- encoder: features of row l16 (lanes kq = 0, 1 hold features 0-7, 8-11) --------
    {
      bf16x8 be[4];
      float bias_e[4];
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        be[cb] = ld8(A.W.We + (size_t)(cb * 16 + l16) * kNetFeatPad + 8 * kq);
        bias_e[cb] = A.W.theta[L.off_be + cb * 16 + l16];
      }
      float R[9];
#pragma unroll
      for (int q = 0; q < 9; ++q) R[q] = (float)fr[q];
      const double s = fr[9];
      const float hs = (float)(A.h / s), h2s = (float)(A.h * A.h / s), iq = (float)(1.0 / A.W.shape_scale);
      const float irho = (float)M.inv_rho;
      for (int rb = wave; rb < nrb; rb += kInfWaves) {
        const int row = rb * 16 + l16;
        float fv[kNetFeat];
#pragma unroll
        for (int q = 0; q < kNetFeat; ++q) fv[q] = 0.f;
        if (row < n && kq < 2) {
          const Real* xr = A.x + 3 * (voff + row);
          const Real* vr = A.v + 3 * (voff + row);
          const Real* fq = A.f + 3 * (voff + row);
          const double m = M.mass[row];
          float d[3], dv[3], df[3], Xa[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            d[c] = (float)((double)xr[c] - fr[10 + c]);
            dv[c] = (float)((double)vr[c] - fr[13 + c]);
            df[c] = (float)((double)fq[c] - m * fr[16 + c]);
            Xa[c] = (float)M.Xc[3 * row + c];
          }
          const float im = (float)(1.0 / m);
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            float rd = 0.f, rv = 0.f, rf = 0.f;            // (R^T w)_a = sum_b R[b][a] w_b
#pragma unroll
            for (int b = 0; b < 3; ++b) {
              rd += R[3 * b + a] * d[b];
              rv += R[3 * b + a] * dv[b];
              rf += R[3 * b + a] * df[b];
            }
            fv[a] = (rd - Xa[a]) * iq;
            fv[3 + a] = rv * hs;
            fv[6 + a] = rf * h2s * im;
            fv[9 + a] = Xa[a] * irho;
          }
        }
        bf16x8 aq;
#pragma unroll
        for (int e = 0; e < 8; ++e) aq[e] = (__bf16)(kq == 0 ? fv[e] : (kq == 1 && e < 4 ? fv[8 + e] : 0.f));
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          const floatx4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aq, be[cb], floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int r2 = rb * 16 + 4 * kq + i;
            const float z = r2 < n ? acc[i] + bias_e[cb] : 0.f;
            H[(size_t)r2 * kHP + cb * 16 + l16] = f2bf(fmaxf(z, 0.f));
          }
        }
      }
    }
    __syncthreads();
    for (int l = 0; l < L.layers; ++l) infer_layer<RR>(A.W, l, n, np, M.nb_deg, H, nbl, degl, Ob, RL);
    // ---- decoder (the frame's R and s, read from memory) --------------------------------
    double fr2[10];
#pragma unroll
    for (int q = 0; q < 10; ++q) fr2[q] = fr[q];
    decoder_rows<Real, kInfWaves>(A, k, voff, n, np, H, kHP, fr2);
  }
}

// ---------------------------------------------------------------------------------
// Loss: target t = R^T delta* / s with delta* = x_{n+1} - x_n - u0 = x_{n+1} - y_n,
// squared error, dLoss/do.
// ---------------------------------------------------------------------------------
template <typename Real>
__global__ void __launch_bounds__(kBlock) net_loss_kernel(NetLossArgs<Real> A) {
  __shared__ double red[4 * kRS];
  for (int k = blockIdx.x; k < A.n_cells; k += gridDim.x) {
    const int cell = A.cells ? A.cells[k] : k;
    const NetMeshDev& M = A.meshes[A.cell_mesh[cell]];
    const int n = M.n, np = M.n_pad;
    const int64_t voff = A.cell_voff[cell];
    const double* fr = A.S.frame + (size_t)k * 12;
    double R[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) R[q] = fr[q];
    const double is = 1.0 / fr[9];
    double acc[1] = {0.0};
    for (int i = tid(); i < np; i += kBlock) {
      float* dO = A.dout + ((size_t)k * A.S.n_pad_max + i) * 3;
      if (i < n) {
        const int64_t g = 3 * (voff + i);
        double d[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) d[c] = ((double)A.x_next[g + c] - (double)A.x[g + c]) - (double)A.u0[g + c];
        const float* o = A.S.out + ((size_t)k * A.S.n_pad_max + i) * 3;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const double t = (R[a] * d[0] + R[3 + a] * d[1] + R[6 + a] * d[2]) * is;
          const double r = (double)o[a] - t;
          acc[0] += r * r;
          dO[a] = (float)(2.0 * r * A.inv_count);
        }
      } else {
        dO[0] = dO[1] = dO[2] = 0.f;
      }
    }
    wg_sum<1>(acc, red);
    if (tid() == 0) A.cell_loss[k] = acc[0];
  }
}

// ---------------------------------------------------------------------------------
// Backward: per cell, decoder then layers in reverse then encoder; weight gradients
// added to this workgroup's slot of the partial sums.
// ---------------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) net_backward_kernel(NetBwdArgs A) {
  __shared__ __align__(16) uint16_t tz[kNetH * kTP];   // dz^T of a 32-node chunk
  __shared__ __align__(16) uint16_t th[kNetH * kTP];   // h^T (or features^T)
  __shared__ __align__(16) uint16_t ta[kNetH * kTP];   // (neighbour mean of h)^T
  const NetLayout L = A.W.lay;
  const int lane = tid() & 63, wave = tid() >> 6, l16 = lane & 15, kq = lane >> 4;
  const size_t plane = (size_t)A.S.n_pad_max * kNetH;
  float* part = A.partial + (size_t)blockIdx.x * L.count;
  float* dHa = A.dH + (size_t)blockIdx.x * 2 * plane;
  float* dHb = dHa + plane;
  float* Qb = A.Q + (size_t)blockIdx.x * plane;
  uint16_t* dZ = A.dZ + (size_t)blockIdx.x * plane;

  for (int k = blockIdx.x; k < A.n_cells; k += gridDim.x) {
    const int cell = A.cells ? A.cells[k] : k;
    const NetMeshDev& M = A.meshes[A.cell_mesh[cell]];
    const int n = M.n, np = M.n_pad;
    const uint16_t* Hs = A.S.H + (size_t)k * (L.layers + 1) * plane;
    const uint16_t* Zs = A.S.Z + (size_t)k * (L.layers + 1) * plane;
    const uint16_t* feat = A.S.feat + (size_t)k * A.S.n_pad_max * kNetFeatPad;
    const float* dO = A.dout + (size_t)k * A.S.n_pad_max * 3;

    // ---- decoder ---------------------------------------------------------------------
    const uint16_t* HL = Hs + (size_t)L.layers * plane;
    if (tid() < 3 * kNetH) {
      const int c = tid() / kNetH, q = tid() % kNetH;
      float acc = 0.f;
      for (int i = 0; i < n; ++i) acc += dO[3 * i + c] * bf2f(HL[(size_t)i * kNetH + q]);
      part[L.off_Wd + tid()] += acc;
    } else if (tid() < 3 * kNetH + 3) {
      const int c = tid() - 3 * kNetH;
      float acc = 0.f;
      for (int i = 0; i < n; ++i) acc += dO[3 * i + c];
      part[L.off_bd + c] += acc;
    }
    for (int e = tid(); e < np * kNetH; e += kBlock) {
      const int i = e / kNetH, q = e % kNetH;
      float g = 0.f;
      if (i < n)
        g = dO[3 * i] * bf2f(A.W.Wd[q]) + dO[3 * i + 1] * bf2f(A.W.Wd[kNetH + q]) +
            dO[3 * i + 2] * bf2f(A.W.Wd[2 * kNetH + q]);
      dHa[e] = g;
    }
    __syncthreads();

    float* dcur = dHa;
    float* dnext = dHb;
    for (int l = L.layers - 1; l >= -1; --l) {            // l = -1: the encoder
      const uint16_t* Z = Zs + (size_t)(l + 1) * plane;
      const uint16_t* Hin = l >= 0 ? Hs + (size_t)l * plane : nullptr;
      // dz = dh * [z > 0], and the bias gradient
      for (int e = tid(); e < np * kNetH; e += kBlock) {
        const int i = e / kNetH;
        const float dz = (i < n && bf2f(Z[e]) > 0.f) ? dcur[e] : 0.f;
        dZ[e] = f2bf(dz);
      }
      if (tid() < kNetH) {
        float acc = 0.f;
        for (int i = 0; i < n; ++i) {
          const size_t e = (size_t)i * kNetH + tid();
          if (bf2f(Z[e]) > 0.f) acc += dcur[e];
        }
        part[(l >= 0 ? L.b(l) : L.off_be) + tid()] += acc;
      }
      __syncthreads();
      // weight gradients: dW_s = dz^T h, dW_n = dz^T mean_N(h)  (dW_e = dz^T f)
      floatx4 gs[4], gn[4];
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) gs[kb] = gn[kb] = floatx4{0.f, 0.f, 0.f, 0.f};
      for (int c0 = 0; c0 < np; c0 += 32) {
        for (int e = tid(); e < 32 * kNetH; e += kBlock) {
          const int nd = e >> 6, q = e & 63, i = c0 + nd;
          tz[q * kTP + nd] = dZ[(size_t)i * kNetH + q];
          if (l >= 0) {
            th[q * kTP + nd] = Hin[(size_t)i * kNetH + q];
            float a = 0.f;
            if (i < n) {
              const int p0 = M.nb_ptr[i], p1 = M.nb_ptr[i + 1];
              for (int p = p0; p < p1; ++p) a += bf2f(Hin[(size_t)M.nb_idx[p] * kNetH + q]);
              a /= (float)(p1 - p0);
            }
            ta[q * kTP + nd] = f2bf(a);
          } else if (q < kNetFeatPad) {
            th[q * kTP + nd] = feat[(size_t)i * kNetFeatPad + q];
          }
        }
        __syncthreads();
        const bf16x8 aq = ld8(tz + (wave * 16 + l16) * kTP + 8 * kq);
        if (l >= 0) {
#pragma unroll
          for (int kb = 0; kb < 4; ++kb) {
            gs[kb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aq, ld8(th + (kb * 16 + l16) * kTP + 8 * kq), gs[kb], 0, 0, 0);
            gn[kb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aq, ld8(ta + (kb * 16 + l16) * kTP + 8 * kq), gn[kb], 0, 0, 0);
          }
        } else {
#pragma unroll
          for (int kb = 0; kb < 2; ++kb)
            gs[kb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aq, ld8(th + (kb * 16 + l16) * kTP + 8 * kq), gs[kb], 0, 0, 0);
        }
        __syncthreads();
      }
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int o = wave * 16 + 4 * kq + i, q = kb * 16 + l16;
          if (l >= 0) {
            part[L.Ws(l) + o * kNetH + q] += gs[kb][i];
            part[L.Wn(l) + o * kNetH + q] += gn[kb][i];
          } else if (kb < 2 && q < kNetFeat) {
            part[L.off_We + o * kNetFeat + q] += gs[kb][i];
          }
        }
      }
      if (l < 0) break;
      // dh_prev = dh + W_s^T dz + (mean_N)^T (W_n^T dz)
      {
        const uint16_t* WsT = A.W.WsT + (size_t)l * kNetH * kNetH;
        const uint16_t* WnT = A.W.WnT + (size_t)l * kNetH * kNetH;
        bf16x8 bs[2][4], bn[2][4];
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
          for (int cb = 0; cb < 4; ++cb) {
            bs[s2][cb] = ld8(WsT + (size_t)(cb * 16 + l16) * kNetH + 32 * s2 + 8 * kq);
            bn[s2][cb] = ld8(WnT + (size_t)(cb * 16 + l16) * kNetH + 32 * s2 + 8 * kq);
          }
        for (int rb = wave; rb < (np >> 4); rb += 4) {
          const int row = rb * 16 + l16;
          const bf16x8 a0 = ld8(dZ + (size_t)row * kNetH + 8 * kq);
          const bf16x8 a1 = ld8(dZ + (size_t)row * kNetH + 32 + 8 * kq);
          floatx4 ap[4], an[4];
#pragma unroll
          for (int cb = 0; cb < 4; ++cb) {
            ap[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bs[0][cb], floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
            ap[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bs[1][cb], ap[cb], 0, 0, 0);
            an[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bn[0][cb], floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
            an[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bn[1][cb], an[cb], 0, 0, 0);
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int r2 = rb * 16 + 4 * kq + i;
            const float ideg = r2 < n ? 1.0f / (float)(M.nb_ptr[r2 + 1] - M.nb_ptr[r2]) : 0.f;
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
              const size_t o = (size_t)r2 * kNetH + cb * 16 + l16;
              dnext[o] = r2 < n ? dcur[o] + ap[cb][i] : 0.f;
              Qb[o] = an[cb][i] * ideg;
            }
          }
        }
      }
      __syncthreads();
      for (int e = tid(); e < n * kNetH; e += kBlock) {
        const int j = e / kNetH, q = e % kNetH;
        float acc = 0.f;
        for (int p = M.nb_ptr[j]; p < M.nb_ptr[j + 1]; ++p) acc += Qb[(size_t)M.nb_idx[p] * kNetH + q];
        dnext[e] += acc;
      }
      __syncthreads();
      float* t = dcur;
      dcur = dnext;
      dnext = t;
    }
    __syncthreads();
  }
}

__global__ void net_reduce_kernel(const float* __restrict__ partial, int grid, int64_t count, float* grad) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= count) return;
  double s = 0.0;
  for (int g = 0; g < grid; ++g) s += (double)partial[(size_t)g * count + p];
  grad[p] = (float)s;
}

__global__ void net_adam_kernel(float* theta, float* m, float* v, const float* grad, int64_t count, float lr,
                                float b1, float b2, float eps, float c1, float c2) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= count) return;
  const float g = grad[p];
  const float mn = b1 * m[p] + (1.f - b1) * g;
  const float vn = b2 * v[p] + (1.f - b2) * g * g;
  m[p] = mn;
  v[p] = vn;
  theta[p] -= lr * (mn / c1) / (sqrtf(vn / c2) + eps);
}

// BF16 copies of the weight blocks in the layouts the kernels read.
__global__ void net_pack_kernel(NetWeights w, uint16_t* We, uint16_t* Wl, uint16_t* WsT, uint16_t* WnT,
                                uint16_t* Wd) {
  const NetLayout L = w.lay;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nWe = (int64_t)kNetH * kNetFeatPad, nL = (int64_t)L.layers * kNetH * kNetH;
  if (e < nWe) {
    const int o = (int)(e / kNetFeatPad), c = (int)(e % kNetFeatPad);
    We[e] = c < kNetFeat ? f2bf(w.theta[L.off_We + o * kNetFeat + c]) : (uint16_t)0;
  }
  if (e < nL) {
    const int l = (int)(e / (kNetH * kNetH)), r = (int)(e % (kNetH * kNetH));
    const int o = r / kNetH, q = r % kNetH;
    const float ws = w.theta[L.Ws(l) + r], wn = w.theta[L.Wn(l) + r];
    Wl[(size_t)l * kNetH * 2 * kNetH + (size_t)o * 2 * kNetH + q] = f2bf(ws);
    Wl[(size_t)l * kNetH * 2 * kNetH + (size_t)o * 2 * kNetH + kNetH + q] = f2bf(wn);
    WsT[(size_t)l * kNetH * kNetH + (size_t)q * kNetH + o] = f2bf(ws);
    WnT[(size_t)l * kNetH * kNetH + (size_t)q * kNetH + o] = f2bf(wn);
  }
  if (e < 3 * kNetH) Wd[e] = f2bf(w.theta[L.off_Wd + e]);
}

__global__ void fill_zero_kernel(float* p, int64_t count) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) p[e] = 0.f;
}

inline int blocks_for(int64_t count, int threads) { return (int)((count + threads - 1) / threads); }

}  // namespace

size_t net_forward_lds_bytes(int n_pad, int nb_deg) {
  const size_t b = kNetLdsHeader + (size_t)n_pad * (kHP + kNetFeatPad) * 2 + (size_t)nb_deg * n_pad * 2 +
                   (size_t)n_pad;
  return (b + 15) / 16 * 16 <= 160 * 1024 && nb_deg <= 255 ? (b + 15) / 16 * 16 : 0;
}

template <typename Real>
hipError_t launch_net_forward(const NetFwdArgs<Real>& a, int grid, size_t lds_bytes, hipStream_t s) {
  (void)hipGetLastError();
  if (lds_bytes > 0) {
    if (lds_bytes < net_forward_lds_bytes(a.S.n_pad_max, a.nb_deg_max)) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&net_forward_lds_kernel<Real>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(net_forward_lds_kernel<Real>, dim3(grid), dim3(kNetLdsBlock), lds_bytes, s, a);
  } else {
    hipLaunchKernelGGL(net_forward_kernel<Real>, dim3(grid), dim3(kBlock), 0, s, a);
  }
  return hipGetLastError();
}

namespace {
int infer_rounds(int n_pad) { return (n_pad / 16 + kInfWaves - 1) / kInfWaves; }
}  // namespace

size_t net_infer_lds_bytes(int n_pad, int nb_deg) {
  const int lds_rounds = std::max(0, infer_rounds(n_pad) - kInfMaxRegRounds);
  const size_t r = infer_lds_base(n_pad, nb_deg) + (size_t)lds_rounds * kInfWaves * 512 * 4;
  return r <= 160 * 1024 && nb_deg <= 255 && n_pad <= 65535 ? r : 0;
}

template <typename Real, int RR>
hipError_t launch_infer_rr(const NetFwdArgs<Real>& a, int grid, size_t lds, int RL, hipStream_t s) {
  const void* fn = reinterpret_cast<const void*>(&net_infer_kernel<Real, RR>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((net_infer_kernel<Real, RR>), dim3(grid), dim3(kInfBlock), lds, s, a, RL);
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_net_infer(const NetFwdArgs<Real>& a, int grid, size_t lds_bytes, hipStream_t s) {
  (void)hipGetLastError();
  if (!a.cframe || a.n_cells < 1 || grid < 1) return hipErrorInvalidValue;
  const size_t need = net_infer_lds_bytes(a.S.n_pad_max, a.nb_deg_max);
  if (need == 0 || lds_bytes < need) return hipErrorInvalidValue;
  hipLaunchKernelGGL(net_frame_kernel<Real>, dim3((a.n_cells + 3) / 4), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int rounds = infer_rounds(a.S.n_pad_max);
  const int RL = std::max(0, rounds - kInfMaxRegRounds);   // rounds staged in LDS
  if (rounds <= 1) return launch_infer_rr<Real, 1>(a, grid, lds_bytes, 0, s);
  if (rounds == 2) return launch_infer_rr<Real, 2>(a, grid, lds_bytes, 0, s);
  return launch_infer_rr<Real, kInfMaxRegRounds>(a, grid, lds_bytes, RL, s);
}

template <typename Real>
hipError_t launch_net_loss(const NetLossArgs<Real>& a, hipStream_t s) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(net_loss_kernel<Real>, dim3(a.n_cells), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_net_backward(const NetBwdArgs& a, int grid, hipStream_t s) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(net_backward_kernel, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_net_reduce(const float* partial, int grid, int64_t count, float* grad, hipStream_t s) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(net_reduce_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, s, partial, grid, count, grad);
  return hipGetLastError();
}

hipError_t launch_net_adam(float* theta, float* m, float* v, const float* grad, int64_t count, double lr,
                           double b1, double b2, double eps, int t, hipStream_t s) {
  (void)hipGetLastError();
  const float c1 = (float)(1.0 - std::pow(b1, t)), c2 = (float)(1.0 - std::pow(b2, t));
  hipLaunchKernelGGL(net_adam_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, s, theta, m, v, grad, count,
                     (float)lr, (float)b1, (float)b2, (float)eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_net_pack(const NetWeights& w, uint16_t* We, uint16_t* Wl, uint16_t* WsT, uint16_t* WnT,
                           uint16_t* Wd, hipStream_t s) {
  (void)hipGetLastError();
  const int64_t n = std::max<int64_t>((int64_t)w.lay.layers * kNetH * kNetH, (int64_t)kNetH * kNetFeatPad);
  hipLaunchKernelGGL(net_pack_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, w, We, Wl, WsT, WnT, Wd);
  return hipGetLastError();
}

hipError_t launch_fill_zero(float* p, int64_t count, hipStream_t s) {
  (void)hipGetLastError();
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

template hipError_t launch_net_forward<float>(const NetFwdArgs<float>&, int, size_t, hipStream_t);
template hipError_t launch_net_forward<double>(const NetFwdArgs<double>&, int, size_t, hipStream_t);
template hipError_t launch_net_infer<float>(const NetFwdArgs<float>&, int, size_t, hipStream_t);
template hipError_t launch_net_infer<double>(const NetFwdArgs<double>&, int, size_t, hipStream_t);
template hipError_t launch_net_loss<float>(const NetLossArgs<float>&, hipStream_t);
template hipError_t launch_net_loss<double>(const NetLossArgs<double>&, hipStream_t);

}  // namespace npfem
