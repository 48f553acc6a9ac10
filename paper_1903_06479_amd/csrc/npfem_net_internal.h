// Internal structures of the learned warm start (host library and gfx950 kernels).
//
// The network predicts, per mesh vertex, the correction delta = x_{n+1} - y_n from
// the first guess y_n of the step to the converged positions.  It works in each
// cell's best-fit rest frame (mass-weighted Kabsch rotation R against the rest mesh)
// on 12 node features, with a residual GraphSAGE network of hidden width 64 and mean
// aggregation over mesh neighbours: BF16 weights and activations on the matrix cores,
// FP32 accumulation, FP64 frame and reductions.
#pragma once

#include <cstdint>

#include "npfem.h"

namespace npfem {

constexpr int kNetH = 64;          // hidden width (fixed: four 16-wide MFMA column blocks)
constexpr int kNetFeat = 12;       // node features
constexpr int kNetFeatPad = 32;    // features padded to one BF16 MFMA k step
constexpr int kNetMaxLayers = 8;
constexpr int kNetFrame = 20;      // per-cell frame of inference: R (9), s, x_c (3), v_c (3), a_c (3), unused

// Per mesh type: what the network needs of the rest mesh.
struct NetMeshDev {
  int n, n_pad;                // vertices, rows padded to a multiple of 32
  const int* nb_ptr;           // [n+1] CSR neighbours
  const int* nb_idx;
  const int* nb_ell;           // [nb_deg][n_pad] the same lists padded (ELL), column q at q * n_pad
  int nb_deg;                  // ELL width (maximum degree)
  const double* Xc;            // [n][3] rest positions minus their mass-weighted centroid
  const double* mass;          // [n]
  double inv_rho;              // 1 / max |X_i - X_c|
  double mass_sum, mass_mean;
};

// Parameter offsets in the flat FP32 vector (row-major blocks):
// W_e [H][12], b_e [H]; per layer W_s [H][H], W_n [H][H], b [H]; W_d [3][H], b_d [3].
struct NetLayout {
  int layers;
  int64_t off_We, off_be, off_Ws0, layer_stride, off_Wd, off_bd, count;
  __host__ __device__ int64_t Ws(int l) const { return off_Ws0 + l * layer_stride; }
  __host__ __device__ int64_t Wn(int l) const { return Ws(l) + kNetH * kNetH; }
  __host__ __device__ int64_t b(int l) const { return Wn(l) + kNetH * kNetH; }
};

inline NetLayout net_layout(int layers) {
  NetLayout L;
  L.layers = layers;
  L.off_We = 0;
  L.off_be = (int64_t)kNetH * kNetFeat;
  L.off_Ws0 = L.off_be + kNetH;
  L.layer_stride = 2 * kNetH * kNetH + kNetH;
  L.off_Wd = L.off_Ws0 + layers * L.layer_stride;
  L.off_bd = L.off_Wd + 3 * kNetH;
  L.count = L.off_bd + 3;
  return L;
}

// Weights as the kernels read them (BF16 bits), derived from the FP32 parameters.
struct NetWeights {
  NetLayout lay;
  double force_floor, shape_scale;
  const float* theta;          // [count] FP32 parameters (biases are read from here)
  const uint16_t* We;          // [H][32]       W_e, features zero-padded to 32
  const uint16_t* Wl;          // [L][H][2H]    [W_s | W_n] by output row
  const uint16_t* WsT;         // [L][H][H]     W_s transposed (input-major)
  const uint16_t* WnT;         // [L][H][H]     W_n transposed
  const uint16_t* Wd;          // [3][H]
};

// Activation storage.  In training every layer is kept per cell (slot = cell of the
// minibatch); in inference each workgroup reuses two buffers (slot = workgroup).
struct NetActs {
  uint16_t* feat;              // [slots][n_pad][32]
  uint16_t* H;                 // [slots][n_h][n_pad][H]  n_h = L + 1 (training) or 2
  uint16_t* Z;                 // [slots][L + 1][n_pad][H] pre-activations (training only)
  double* frame;               // [cells][12]: R (9, row-major, rest -> world), s, unused
  float* out;                  // [cells][n_pad][3] network outputs o (training only)
  int n_pad_max;
  int train;
};

template <typename Real>
struct NetFwdArgs {
  NetWeights W;
  NetActs S;
  const NetMeshDev* meshes;
  const int64_t* cell_voff;
  const int* cell_mesh;
  const int* cells;            // nullable list of batch cells; else cell k of the batch
  int n_cells;
  int nb_deg_max;              // largest ELL width of the plan's meshes
  double h;
  const Real* x;               // [V][3]
  const Real* v;
  const Real* f;
  Real* delta;                 // [V][3] world-frame correction (inference), or null
  double* cframe;              // [n_cells][kNetFrame] frames of the resident inference
};

template <typename Real>
struct NetLossArgs {
  NetActs S;
  const NetMeshDev* meshes;
  const int64_t* cell_voff;
  const int* cell_mesh;
  const int* cells;
  int n_cells;
  double inv_count;            // 1 / (3 * nodes in the minibatch)
  const Real* x;               // [V][3] x_n
  const Real* x_next;          // [V][3] converged x_{n+1}
  const Real* u0;              // [V][3] first guess y_n - x_n: the target is x_{n+1} - x_n - u0
  float* dout;                 // [cells][n_pad][3] dLoss/do
  double* cell_loss;           // [cells]
};

struct NetBwdArgs {
  NetWeights W;
  NetActs S;
  const NetMeshDev* meshes;
  const int* cell_mesh;
  const int* cells;
  int n_cells;
  const float* dout;           // [cells][n_pad][3]
  float* dH;                   // [grid][2][n_pad][H] scratch
  float* Q;                    // [grid][n_pad][H]
  uint16_t* dZ;                // [grid][n_pad][H]
  float* partial;              // [grid][count] per-workgroup gradient sums
};

// Forward launch: with lds_bytes > 0 the LDS-resident variant (512 threads, the cell's
// activations and neighbour lists in LDS) is used, else the variant that gathers from
// memory (any mesh size).
template <typename Real>
hipError_t launch_net_forward(const NetFwdArgs<Real>& a, int grid, size_t lds_bytes, hipStream_t s);
// LDS the resident variant needs for meshes up to n_pad rows and degree nb_deg (0 if it
// does not fit a compute unit).
size_t net_forward_lds_bytes(int n_pad, int nb_deg);
// Inference with the cell's activations resident in LDS (meshes with n_pad <= 1024): a
// frame kernel (one wave per cell, into a.cframe), then the network (512 threads per
// cell, one workgroup per CU).  lds_bytes from net_infer_lds_bytes, 0 if it does not fit.
template <typename Real>
hipError_t launch_net_infer(const NetFwdArgs<Real>& a, int grid, size_t lds_bytes, hipStream_t s);
size_t net_infer_lds_bytes(int n_pad, int nb_deg);
template <typename Real>
hipError_t launch_net_loss(const NetLossArgs<Real>& a, hipStream_t s);
hipError_t launch_net_backward(const NetBwdArgs& a, int grid, hipStream_t s);
hipError_t launch_net_reduce(const float* partial, int grid, int64_t count, float* grad, hipStream_t s);
hipError_t launch_net_adam(float* theta, float* m, float* v, const float* grad, int64_t count, double lr,
                           double b1, double b2, double eps, int t, hipStream_t s);
hipError_t launch_net_pack(const NetWeights& w, uint16_t* We, uint16_t* Wl, uint16_t* WsT, uint16_t* WnT,
                           uint16_t* Wd, hipStream_t s);
hipError_t launch_fill_zero(float* p, int64_t count, hipStream_t s);

}  // namespace npfem
