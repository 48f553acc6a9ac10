// gfx950 kernels of the batched npFEM step.
//
// One workgroup (4 wave64) owns a tile of up to kMaxTile cells of one mesh type and
// carries them through a whole time step (Algorithm 1 of the paper): first guess,
// quasi-Newton iterations with line search, velocity update and dissipation.  Cells
// are worked on one at a time by the whole workgroup, with the cell's rest positions
// and trial displacement staged in LDS; the one operation that couples cells, the
// product with the shared dense inverse H~^-1 (section 2.1.1), is done for the whole
// tile at once on the matrix cores.  Workgroups are persistent and pull tiles from a
// queue, so one launch covers an uneven batch.
//
// Per-cell vectors in the workspace are structure-of-arrays [3][n_pad] so that the
// tile's vectors form the row-major (3T x n_pad) operand of the MFMA product.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <type_traits>
#include <vector>

#include "npfem_internal.h"

namespace npfem {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <typename Real> struct Eps;
template <> struct Eps<float> { static constexpr double v = 1.1920928955078125e-07; };
template <> struct Eps<double> { static constexpr double v = 2.220446049250313e-16; };

// LDS: [red: 4 waves x 32 doubles][32 doubles, spare][ints: 32][mesh descriptor][cell vectors ...];
// during the BF16 tile product the region from the cell vectors on holds the tile's rows
// in BF16.  The current tile's mesh descriptor is copied to LDS so that reading its table
// pointers waits on the LDS counter only, never on global loads in flight.
constexpr int kRedStride = 32;
constexpr int kRedDoubles = 4 * kRedStride;
constexpr int kMeshLds = 256;
constexpr int kLdsMesh = kRedDoubles * 8 + 32 * 8 + 32 * 4;
constexpr int kLdsHeader = kLdsMesh + kMeshLds;   // reduction, 32 spare doubles, ints, mesh
static_assert(sizeof(MeshDev<double>) <= kMeshLds && sizeof(MeshDev<float>) <= kMeshLds, "mesh descriptor");
static_assert(sizeof(MeshDev<double>) % 4 == 0 && sizeof(MeshDev<float>) % 4 == 0, "mesh descriptor");

__device__ inline int tid() { return threadIdx.x; }

// 16-byte vectors of the plan's precision for the per-cell vector passes (the SoA
// vectors have 3 n_pad elements, a multiple of 96, so every pass is whole vectors).
template <typename Real> struct Vec16;
template <> struct Vec16<float> { typedef float type __attribute__((ext_vector_type(4))); static constexpr int W = 4; };
template <> struct Vec16<double> { typedef double type __attribute__((ext_vector_type(2))); static constexpr int W = 2; };
template <typename Real>
__device__ inline typename Vec16<Real>::type vload(const Real* p, int e) {
  return *reinterpret_cast<const typename Vec16<Real>::type*>(p + e);
}
template <typename Real>
__device__ inline void vstore(Real* p, int e, typename Vec16<Real>::type v) {
  *reinterpret_cast<typename Vec16<Real>::type*>(p + e) = v;
}
template <typename Real>
__device__ inline void vcopy(Real* dst, const Real* src, int len) {
  constexpr int W = Vec16<Real>::W;
#pragma unroll 2
  for (int e = W * tid(); e < len; e += W * kBlock) vstore(dst, e, vload(src, e));
}

// Reads of the per-mesh tables (global memory shared by every cell): with the address
// space explicit the compiler emits global loads with a scalar base and a 32-bit offset,
// not flat loads, which would also hold up every wait on the LDS.
template <typename T>
__device__ inline T gld(const T* p, int i) {
  typedef const T __attribute__((address_space(1))) GT;
  return ((GT*)p)[(unsigned)i];
}

// Entries of a vertex's ELL lists (neighbours, incident corners) fetched per group.
constexpr int kEllGroup = 6;

// Lane permutation of a double within rows of 16 lanes (DPP, on the vector ALU).
template <int CTRL>
__device__ inline double dpp_row(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ inline double read_lane(double x, int lane) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)v, lane), hi = __builtin_amdgcn_readlane((int)(v >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// Sum of a double over the wave: within each row of 16 lanes by DPP (pairs, quads, half
// rows, rows), then the four row sums; the same on every lane, fixed order.
__device__ inline double wave_sum(double x) {
  x += dpp_row<0xB1>(x);    // quad_perm [1,0,3,2]
  x += dpp_row<0x4E>(x);    // quad_perm [2,3,0,1]
  x += dpp_row<0x141>(x);   // row_half_mirror
  x += dpp_row<0x140>(x);   // row_mirror
  return (read_lane(x, 0) + read_lane(x, 16)) + (read_lane(x, 32) + read_lane(x, 48));
}

// Sum N (<= 32) doubles over the workgroup; fixed order, so deterministic.
template <int N>
__device__ inline void block_sum(double (&v)[N], double* red) {
  static_assert(N <= kRedStride, "block_sum: too many values");
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = wave_sum(v[i]);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) red[wave * kRedStride + i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i)
    v[i] = (red[i] + red[kRedStride + i]) + (red[2 * kRedStride + i] + red[3 * kRedStride + i]);
}

template <typename Real>
__device__ inline double dot_vec(const Real* a, const Real* b, int len, double* red) {
  double s[1] = {0.0};
  for (int e = tid(); e < len; e += kBlock) s[0] += (double)a[e] * (double)b[e];
  block_sum<1>(s, red);
  return s[0];
}

// ---------------------------------------------------------------------------------
// LDS staging
// ---------------------------------------------------------------------------------

// One cell's AoS [n][3] values -> SoA [3][np] (padding zero); load(e) yields AoS element
// e = 3 i + c.  Each thread issues the loads of up to kStageBatch elements before its
// first store, so staging a cell costs one memory latency rather than one per element.
constexpr int kStageBatch = 8;
template <typename Real, typename Load>
__device__ inline void aos_to_soa(Real* dst, int n, int np, Load load) {
  const int len = 3 * n;
  for (int base = 0; base < len; base += kStageBatch * kBlock) {
    Real v[kStageBatch];
#pragma unroll
    for (int k = 0; k < kStageBatch; ++k) {
      const int e = base + k * kBlock + tid();
      v[k] = e < len ? load(e) : Real(0);
    }
#pragma unroll
    for (int k = 0; k < kStageBatch; ++k) {
      const int e = base + k * kBlock + tid();
      if (e < len) {
        const int i = e / 3, c = e - 3 * i;
        dst[c * np + i] = v[k];
      }
    }
  }
  const int pad = np - n;
  for (int e = tid(); e < 3 * pad; e += kBlock) {
    const int c = e / pad, i = n + (e - c * pad);
    dst[c * np + i] = Real(0);
  }
}

// x_n of one cell: global AoS [n][3] -> LDS SoA [3][np].
template <typename Real>
__device__ inline void stage_aos(Real* dst, const Real* src, int n, int np) {
  aos_to_soa(dst, n, np, [&](int e) { return src[e]; });
}

// Reciprocal and square root of the FP32 bulk arithmetic: the hardware instructions
// (v_rcp_f32, v_sqrt_f32, about 1 ulp) instead of the correctly rounded sequences; the
// FP64 path keeps the exact operations.
template <typename Real> __device__ inline Real rcp_(Real x) { return Real(1) / x; }
template <> __device__ inline float rcp_<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <typename Real> __device__ inline Real sqrt_(Real x) { return sqrt(x); }
template <> __device__ inline float sqrt_<float>(float x) { return __builtin_amdgcn_sqrtf(x); }

// ---------------------------------------------------------------------------------
// Normalisers of the global terms (section 2.1.2): |grad V|^2 with grad V_k = nbar_k / 3,
// and (when accA is given) |grad A|^2 with grad A = sum over the incident triangles of
// n x (the edge opposite the vertex) / 2, at x = x_n (+ u when ut is given).  Per chunk,
// each triangle's contributions go to `work` (9 per triangle: the volume normal / 6 and
// the area gradients of corners a and b, corner c taking minus their sum), then every
// vertex gathers its corners into accV (and accA).
// ---------------------------------------------------------------------------------
template <typename Real>
__device__ void normalisers(const MeshDev<Real>& M, const Real* xn, const Real* ut, Real* accV, Real* accA,
                            Real* work, double* red, double& GV, double& GA) {
  const int n = M.n, np = M.n_pad, nt = M.nt, ch = M.chunk;
  const bool area = accA != nullptr;
  for (int e = tid(); e < 3 * np; e += kBlock) {
    accV[e] = Real(0);
    if (area) accA[e] = Real(0);
  }
  for (int t0 = 0; t0 < nt; t0 += ch) {
    __syncthreads();
    const int tn = min(ch, nt - t0);
    for (int tt = tid(); tt < tn; tt += kBlock) {
      const int t = t0 + tt;
      const int a = gld(M.tri, 3 * t), b = gld(M.tri, 3 * t + 1), c = gld(M.tri, 3 * t + 2);
      Real e1x = xn[a] - xn[c], e1y = xn[np + a] - xn[np + c], e1z = xn[2 * np + a] - xn[2 * np + c];
      Real e2x = xn[b] - xn[c], e2y = xn[np + b] - xn[np + c], e2z = xn[2 * np + b] - xn[2 * np + c];
      if (ut) {
        e1x += ut[a] - ut[c]; e1y += ut[np + a] - ut[np + c]; e1z += ut[2 * np + a] - ut[2 * np + c];
        e2x += ut[b] - ut[c]; e2y += ut[np + b] - ut[np + c]; e2z += ut[2 * np + b] - ut[2 * np + c];
      }
      const Real nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
      work[tt] = nx / Real(6);
      work[ch + tt] = ny / Real(6);
      work[2 * ch + tt] = nz / Real(6);
      if (area) {
        // a collapsed triangle (area below 1e-6 of its rest area) has no normal and adds
        // nothing to the area gradient
        const Real nn2 = nx * nx + ny * ny + nz * nz;
        const bool collapsed = (double)nn2 * gld(M.inv4a2, t) < 1e-12;   // (area ratio)^2
        const Real nn = sqrt_(nn2);
        const Real s = nn > Real(0) && !collapsed ? Real(0.5) * rcp_(nn) : Real(0);
        const Real hx = s * nx, hy = s * ny, hz = s * nz;       // n / 2
        work[3 * ch + tt] = -(hy * e2z - hz * e2y);              // corner a: -(n/2) x e2
        work[4 * ch + tt] = -(hz * e2x - hx * e2z);
        work[5 * ch + tt] = -(hx * e2y - hy * e2x);
        work[6 * ch + tt] = hy * e1z - hz * e1y;                 // corner b: (n/2) x e1
        work[7 * ch + tt] = hz * e1x - hx * e1z;
        work[8 * ch + tt] = hx * e1y - hy * e1x;
      }
    }
    __syncthreads();
    for (int i = tid(); i < n; i += kBlock) {
      Real gx = 0, gy = 0, gz = 0, ax = 0, ay = 0, az = 0;
      // incident corners from the ELL list, a group of indices in flight together;
      // padding and corners outside this chunk add zero
      for (int q0 = 0; q0 < M.vc_deg; q0 += kEllGroup) {
        int cc[kEllGroup];
#pragma unroll
        for (int u = 0; u < kEllGroup; ++u) cc[u] = q0 + u < M.vc_deg ? gld(M.vc_ell, (q0 + u) * np + i) : -1;
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < kEllGroup; ++u) {
          const int cid = cc[u];
          const int tri = cid / 3, k = cid - 3 * tri, t = tri - t0;
          const bool ok = cid >= 0 && t >= 0 && t < tn;
          const int tc = ok ? t : 0;
          gx += ok ? work[tc] : Real(0);
          gy += ok ? work[ch + tc] : Real(0);
          gz += ok ? work[2 * ch + tc] : Real(0);
          if (area) {
            const Real sg = ok ? (k == 2 ? Real(-1) : Real(1)) : Real(0);
            const Real pax = work[3 * ch + tc], pay = work[4 * ch + tc], paz = work[5 * ch + tc];
            const Real pbx = work[6 * ch + tc], pby = work[7 * ch + tc], pbz = work[8 * ch + tc];
            ax += sg * (k == 0 ? pax : (k == 1 ? pbx : pax + pbx));
            ay += sg * (k == 0 ? pay : (k == 1 ? pby : pay + pby));
            az += sg * (k == 0 ? paz : (k == 1 ? pbz : paz + pbz));
          }
        }
      }
      accV[i] += gx;
      accV[np + i] += gy;
      accV[2 * np + i] += gz;
      if (area) {
        accA[i] += ax;
        accA[np + i] += ay;
        accA[2 * np + i] += az;
      }
    }
  }
  __syncthreads();
  double sm[2] = {0.0, 0.0};
  for (int i = tid(); i < n; i += kBlock) {
    sm[0] += (double)accV[i] * accV[i] + (double)accV[np + i] * accV[np + i] + (double)accV[2 * np + i] * accV[2 * np + i];
    if (area)
      sm[1] += (double)accA[i] * accA[i] + (double)accA[np + i] * accA[np + i] + (double)accA[2 * np + i] * accA[2 * np + i];
  }
  block_sum<2>(sm, red);
  GV = sm[0];
  GA = area ? sm[1] : 1.0;
}

// ---------------------------------------------------------------------------------
// Objective and gradient at x = x_n + u (eq. GeneralizedObjectiveFunctionDerivative)
// ---------------------------------------------------------------------------------
struct EvalResult {
  double E, noise, resid, vol, area, degen;
  double terms[8];   // inertial, area, Skalak, bending(+Rayleigh), volume, triangle Rayleigh, global area, collision
};

// Collision term of one cell (section 4.7): per vertex the partner q and its normal n
// found at the start of the step (AoS [n][3], global; n = 0 where there is none), weight w.
template <typename Real>
struct Contacts {
  const Real* q;
  const Real* n;
  double w;
};

// SL(2) projection of the singular values (section 2.1.2): t = 1 + tau, the largest
// root of t^4 - s1 t^3 + s2 t - 1, written in deviations s_i = 1 + a_i so that small
// strains lose no digits:  f(tau) = (1+tau)^3 (tau - a1) + tau (1 + a2) + a2.
// f is convex for t >= s1/2 and f(s1/2) <= 0, so Newton from any start right of the
// root decreases monotonically onto it.
template <typename Real>
__device__ inline Real sl2_tau(Real a1, Real a2, Real sig1, Real J) {
  Real tau;
  if (J >= Real(1)) {
    tau = a1;                                             // f(s1) = J - 1 >= 0
  } else {
    const Real s3 = sig1 * sig1 * sig1;
    tau = a1 + fmin((Real(1) - J) * rcp_(fmax(s3, Real(1e-30))), Real(1));
  }
  const Real tol = Real(Eps<Real>::v) * Real(4);
  for (int it = 0; it < 60; ++it) {
    const Real t = Real(1) + tau;
    const Real t2 = t * t;
    const Real f = t2 * t * (tau - a1) + tau * (Real(1) + a2) + a2;
    const Real df = t2 * (Real(1) + Real(4) * tau - Real(3) * a1) + Real(1) + a2;
    const Real step = f * rcp_(df);
    tau -= step;
    if (!(fabs(step) > tol * (Real(1) + fabs(tau)))) break;
  }
  return tau;
}

// EXT: the optional terms (global area, the literal volume normaliser, contacts) are
// compiled in; without them the evaluation carries none of their code.
template <typename Real, bool EXT>
__device__ void evaluate(const MeshDev<Real>& M, const MaterialDev& mat, bool literal, double h, double Gn,
                         double GA, const Contacts<Real>& col, const Real* xn, const Real* ut, const Real* bvec,
                         Real* work, Real* gout, double* red, EvalResult& res) {
  const int n = M.n, np = M.n_pad, nt = M.nt, ch = M.chunk;
  const Real inv_h2 = Real(1.0 / (h * h));
  const Real beta = Real(mat.beta), kb = Real(mat.k_bend);
  const Real Cst = Real(mat.C), Bsk = Real(mat.B), Dsk = Real(mat.D);

  // xn, ut, bvec and gout are the cell's vectors (in LDS unless the mesh is too large).
  // The corner buffer holds, per triangle, the in-plane gradient of corners a and b (6
  // values; corner c gets minus their sum; with the global-area term switched on it
  // includes that term's gradient) and the normal e1 x e2 (3 values; the volume
  // gradient of each corner is a sixth of it).  When all triangles fit one chunk and no
  // global-area term needs the total area beforehand, the enclosed volume and area are
  // summed in the triangle pass itself; otherwise first, in a pass of their own.
  const bool single = nt <= ch;
  const bool area_on = EXT && mat.k_area_global > 0.0;
  const bool pre = !single || area_on;
  // ---- literal volume normaliser: |grad V|^2 at the trial point (gout as scratch) ---
  if (EXT && literal) {
    double gv, ga;
    normalisers(M, xn, ut, gout, static_cast<Real*>(nullptr), work, red, gv, ga);
    Gn = gv;
  }
  // ---- pass A: (volume and area when needed first) and bending residuals -> work ----
  double accA[4] = {0.0, 0.0, 0.0, 0.0};   // 6 volume, bending energy, bending Rayleigh energy, 2 area
  if (pre) {
    for (int t = tid(); t < nt; t += kBlock) {
      const int a = gld(M.tri, 3 * t), b = gld(M.tri, 3 * t + 1), c = gld(M.tri, 3 * t + 2);
      const double E1x = ((double)xn[a] - (double)xn[c]) + ((double)ut[a] - (double)ut[c]);
      const double E1y = ((double)xn[np + a] - (double)xn[np + c]) + ((double)ut[np + a] - (double)ut[np + c]);
      const double E1z = ((double)xn[2 * np + a] - (double)xn[2 * np + c]) + ((double)ut[2 * np + a] - (double)ut[2 * np + c]);
      const double E2x = ((double)xn[b] - (double)xn[c]) + ((double)ut[b] - (double)ut[c]);
      const double E2y = ((double)xn[np + b] - (double)xn[np + c]) + ((double)ut[np + b] - (double)ut[np + c]);
      const double E2z = ((double)xn[2 * np + b] - (double)xn[2 * np + c]) + ((double)ut[2 * np + b] - (double)ut[2 * np + c]);
      const double cx = (double)xn[c] + ut[c], cy = (double)xn[np + c] + ut[np + c], cz = (double)xn[2 * np + c] + ut[2 * np + c];
      accA[0] += E1x * (E2y * cz - E2z * cy) + E1y * (E2z * cx - E2x * cz) + E1z * (E2x * cy - E2y * cx);
      const double Nx = E1y * E2z - E1z * E2y, Ny = E1z * E2x - E1x * E2z, Nz = E1x * E2y - E1y * E2x;
      accA[3] += sqrt(Nx * Nx + Ny * Ny + Nz * Nz);
    }
  }
  for (int i = tid(); i < n; i += kBlock) {
    Real lx = 0, ly = 0, lz = 0, ux = 0, uy = 0, uz = 0;
    const Real xix = xn[i], xiy = xn[np + i], xiz = xn[2 * np + i];
    const Real uix = ut[i], uiy = ut[np + i], uiz = ut[2 * np + i];
    Real Ai = 0, l0 = 0;
    for (int q0 = 0; q0 < M.nb_deg; q0 += kEllGroup) {
      // a group's neighbours and weights (padding: the vertex itself, weight 0) are all
      // requested before the first is used; the scheduling barrier keeps them together
      int jj[kEllGroup];
      Real ww[kEllGroup];
#pragma unroll
      for (int u = 0; u < kEllGroup; ++u) {
        const bool in = q0 + u < M.nb_deg;
        jj[u] = in ? gld(M.nb_ell, (q0 + u) * np + i) : i;
        ww[u] = in ? gld(M.nbw_ell, (q0 + u) * np + i) : Real(0);
      }
      if (q0 == 0) {
        Ai = gld(M.vor_area, i);
        l0 = gld(M.ell0, i);
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < kEllGroup; ++u) {
        const int j = jj[u];
        const Real w = ww[u];
        const Real dux = ut[j] - uix, duy = ut[np + j] - uiy, duz = ut[2 * np + j] - uiz;
        lx += w * ((xn[j] - xix) + dux);
        ly += w * ((xn[np + j] - xiy) + duy);
        lz += w * ((xn[2 * np + j] - xiz) + duz);
        ux += w * dux;
        uy += w * duy;
        uz += w * duz;
      }
    }
    const Real inv_A = rcp_(Ai);
    lx *= inv_A; ly *= inv_A; lz *= inv_A;
    ux *= inv_A; uy *= inv_A; uz *= inv_A;
    const Real nrm = sqrt_(lx * lx + ly * ly + lz * lz);
    const Real sc = nrm > Real(1e-30) ? l0 * rcp_(nrm) : Real(0);
    const Real rx = lx - sc * lx, ry = ly - sc * ly, rz = lz - sc * lz;
    accA[1] += 0.5 * (double)(kb * Ai) * ((double)rx * rx + (double)ry * ry + (double)rz * rz);
    accA[2] += 0.5 * (double)(beta * kb * Ai) * ((double)ux * ux + (double)uy * uy + (double)uz * uz);
    work[i] = rx + beta * ux;
    work[np + i] = ry + beta * uy;
    work[2 * np + i] = rz + beta * uz;
  }
  double coefd = 0.0, vol = 0.0, area = 0.0, coefa = 0.0;
  if (pre) {
    block_sum<4>(accA, red);
    vol = accA[0] / 6.0;
    area = 0.5 * accA[3];
    coefd = mat.k_volume * (vol - M.V0) / Gn;               // k C / G_n
    coefa = area_on ? mat.k_area_global * (area - M.A0) / GA : 0.0;
  } else {
    double ab[2] = {accA[1], accA[2]};
    block_sum<2>(ab, red);                                   // also the barrier before pass B
    accA[1] = ab[0];
    accA[2] = ab[1];
  }

  // ---- pass B: bending gradient + inertia - b (+ collision) -> gout -----------------
  // collision: (w/2) min(d, 0)^2 per vertex with d = (x - q) . n, gradient w min(d, 0) n;
  // the term drops out wherever the vertex no longer penetrates
  double accB[2] = {0.0, 0.0};
  const Real wc = Real(col.w);
  for (int i = tid(); i < n; i += kBlock) {
    Real gx = 0, gy = 0, gz = 0;
    const Real rix = work[i], riy = work[np + i], riz = work[2 * np + i];
    Real mass = 0;
    for (int q0 = 0; q0 < M.nb_deg; q0 += kEllGroup) {
      // as in pass A: the group's neighbours and weights (and the mass) are requested
      // before the first is used
      int jj[kEllGroup];
      Real ww[kEllGroup];
#pragma unroll
      for (int u = 0; u < kEllGroup; ++u) {
        const bool in = q0 + u < M.nb_deg;
        jj[u] = in ? gld(M.nb_ell, (q0 + u) * np + i) : i;
        ww[u] = in ? gld(M.nbw_ell, (q0 + u) * np + i) : Real(0);
      }
      if (q0 == 0) mass = gld(M.mass, i);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < kEllGroup; ++u) {
        const int j = jj[u];
        const Real w = ww[u];
        gx += w * (work[j] - rix);
        gy += w * (work[np + j] - riy);
        gz += w * (work[2 * np + j] - riz);
      }
    }
    const Real mi = mass * inv_h2;
    const Real ux = ut[i], uy = ut[np + i], uz = ut[2 * np + i];
    const Real bx = bvec[i], by = bvec[np + i], bz = bvec[2 * np + i];
    Real ox = kb * gx + (mi * ux - bx), oy = kb * gy + (mi * uy - by), oz = kb * gz + (mi * uz - bz);
    if (EXT && col.n) {
      const Real cnx = gld(col.n, 3 * i), cny = gld(col.n, 3 * i + 1), cnz = gld(col.n, 3 * i + 2);
      const Real cqx = gld(col.q, 3 * i), cqy = gld(col.q, 3 * i + 1), cqz = gld(col.q, 3 * i + 2);
      const Real dd = ((xn[i] - cqx) + ux) * cnx + ((xn[np + i] - cqy) + uy) * cny + ((xn[2 * np + i] - cqz) + uz) * cnz;
      const Real dm = dd < Real(0) ? dd : Real(0);
      ox += wc * dm * cnx;
      oy += wc * dm * cny;
      oz += wc * dm * cnz;
      accB[1] += 0.5 * col.w * (double)dm * dm;
    }
    gout[i] = ox;
    gout[np + i] = oy;
    gout[2 * np + i] = oz;
    accB[0] += 0.5 * (double)mi * ((double)ux * ux + (double)uy * uy + (double)uz * uz)
               - ((double)ux * bx + (double)uy * by + (double)uz * bz);
  }
  for (int i = n + tid(); i < np; i += kBlock) gout[i] = gout[np + i] = gout[2 * np + i] = Real(0);
  __syncthreads();   // work (R) is reused for the corner chunks below

  // ---- passes C/D: triangle in-plane terms + volume, per chunk --------------------
  // area PD, Skalak, triangle Rayleigh, |u.b|, 6 volume, 2 area, collapsed triangles
  double accC[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const Real ca = Real(0.5 * coefa);               // global area: k_A (A - A0) / G_A / 2
  double accD[4] = {0.0, 0.0, 0.0, 0.0};   // |grad|^2, |M u/h^2|^2, |b|^2, |F_int|^2
  for (int t0 = 0; t0 < nt; t0 += ch) {
    const int tn = min(ch, nt - t0);
    for (int tt = tid(); tt < tn; tt += kBlock) {
      const int t = t0 + tt;
      // The triangle's table entries are all requested before the first is used, then
      // its corners' coordinates from LDS; scheduling barriers keep each group together.
      const int a = gld(M.tri, 3 * t), b = gld(M.tri, 3 * t + 1), c = gld(M.tri, 3 * t + 2);
      const double D00 = gld(M.dminv, 4 * t), D01 = gld(M.dminv, 4 * t + 1), D10 = gld(M.dminv, 4 * t + 2), D11 = gld(M.dminv, 4 * t + 3);
      const double area_t = gld(M.area, t), i4a2_t = gld(M.inv4a2, t);
      __builtin_amdgcn_sched_barrier(0);
      const Real xa = xn[a], ya = xn[np + a], za = xn[2 * np + a];
      const Real xb = xn[b], yb = xn[np + b], zb = xn[2 * np + b];
      const Real xc = xn[c], yc = xn[np + c], zc = xn[2 * np + c];
      const Real uax = ut[a], uay = ut[np + a], uaz = ut[2 * np + a];
      const Real ubx = ut[b], uby = ut[np + b], ubz = ut[2 * np + b];
      const Real ucx = ut[c], ucy = ut[np + c], ucz = ut[2 * np + c];
      __builtin_amdgcn_sched_barrier(0);
      const Real d00 = Real(D00), d01 = Real(D01), d10 = Real(D10), d11 = Real(D11);
      const Real A0 = Real(area_t);
      // The strain measures (sigma - 1, area ratio - 1) are small differences of O(1)
      // quantities, so the edges, F = [e1 e2] D_m^-1, F^T F and |e1 x e2|^2 are formed
      // in FP64 from the stored values (exact differences); everything after that works
      // on the small differences and keeps its relative precision in FP32.
      const double E1x = ((double)xa - (double)xc) + ((double)uax - (double)ucx);
      const double E1y = ((double)ya - (double)yc) + ((double)uay - (double)ucy);
      const double E1z = ((double)za - (double)zc) + ((double)uaz - (double)ucz);
      const double E2x = ((double)xb - (double)xc) + ((double)ubx - (double)ucx);
      const double E2y = ((double)yb - (double)yc) + ((double)uby - (double)ucy);
      const double E2z = ((double)zb - (double)zc) + ((double)ubz - (double)ucz);
      const double F0x = E1x * D00 + E2x * D10, F0y = E1y * D00 + E2y * D10, F0z = E1z * D00 + E2z * D10;
      const double F1x = E1x * D01 + E2x * D11, F1y = E1y * D01 + E2y * D11, F1z = E1z * D01 + E2z * D11;
      const double C00 = F0x * F0x + F0y * F0y + F0z * F0z;
      const double C01 = F0x * F1x + F0y * F1y + F0z * F1z;
      const double C11 = F1x * F1x + F1y * F1y + F1z * F1z;
      const double Nx = E1y * E2z - E1z * E2y, Ny = E1z * E2x - E1x * E2z, Nz = E1x * E2y - E1y * E2x;
      const double NN = Nx * Nx + Ny * Ny + Nz * Nz;
      // displacement part of F for the Rayleigh term
      const Real eu1x = uax - ucx, eu1y = uay - ucy, eu1z = uaz - ucz;
      const Real eu2x = ubx - ucx, eu2y = uby - ucy, eu2z = ubz - ucz;
      const Real f0x = Real(F0x), f0y = Real(F0y), f0z = Real(F0z);
      const Real f1x = Real(F1x), f1y = Real(F1y), f1z = Real(F1z);
      const Real g0x = eu1x * d00 + eu2x * d10, g0y = eu1y * d00 + eu2y * d10, g0z = eu1z * d00 + eu2z * d10;
      const Real g1x = eu1x * d01 + eu2x * d11, g1y = eu1y * d01 + eu2y * d11, g1z = eu1z * d01 + eu2z * d11;
      const Real c01 = Real(C01);
      const Real nx = Real(Nx), ny = Real(Ny), nz = Real(Nz);
      const Real nn = sqrt_(Real(NN));
      // a collapsed triangle (area below 1e-6 of its rest area) has no second in-plane
      // direction: u2 below is taken as zero, so that direction carries no force
      const bool collapsed = NN * i4a2_t < 1e-12;
      // area ratio J = sigma1 sigma2 = |e1 x e2| / (2 A0)
      const Real Jsq_m1 = Real(NN * i4a2_t - 1.0);
      const Real J = sqrt_(fmax(Real(1) + Jsq_m1, Real(0)));
      const Real Jm1 = Jsq_m1 * rcp_(J + Real(1));
      const Real half = Real(0.5 * (C00 - C11));
      const Real disc = sqrt_(half * half + c01 * c01);
      const Real s1m = Real(0.5 * ((C00 - 1.0) + (C11 - 1.0))) + disc;          // sigma1^2 - 1
      const Real sig1 = sqrt_(fmax(Real(1) + s1m, Real(0)));
      const Real a1 = s1m * rcp_(sig1 + Real(1));                              // sigma1 - 1
      const Real inv_s1 = sig1 > Real(1e-30) ? rcp_(sig1) : Real(0);
      const Real a2 = (Jm1 - a1) * inv_s1;                                     // sigma2 - 1
      const Real sig2 = Real(1) + a2;
      // right singular vectors v1, v2 = perp(v1); left u1 = F v1 / sigma1, u2 = nhat x u1
      Real vx, vy;
      if (half >= Real(0)) { vx = half + disc; vy = c01; } else { vx = c01; vy = disc - half; }
      const Real vn = sqrt_(vx * vx + vy * vy);
      if (vn > Real(0)) {
        const Real ivn = rcp_(vn);
        vx *= ivn;
        vy *= ivn;
      } else {
        vx = Real(1);
        vy = Real(0);
      }
      const Real u1x = (f0x * vx + f1x * vy) * inv_s1, u1y = (f0y * vx + f1y * vy) * inv_s1, u1z = (f0z * vx + f1z * vy) * inv_s1;
      const Real inv_nn = nn > Real(1e-30) ? rcp_(nn) : Real(0);
      const Real hx = collapsed ? Real(0) : nx * inv_nn, hy = collapsed ? Real(0) : ny * inv_nn,
                 hz = collapsed ? Real(0) : nz * inv_nn;
      const Real u2x = hy * u1z - hz * u1y, u2y = hz * u1x - hx * u1z, u2z = hx * u1y - hy * u1x;
      // area PD: closest SL(2) element diag(t, 1/t)
      const Real tau = sl2_tau<Real>(a1, a2, sig1, J);
      const Real dA1 = a1 - tau, dA2 = a2 + tau * rcp_(Real(1) + tau);
      // modified Skalak: f'(s) = B/2 s (s^2 - 1) + D (s - 1)^3
      const Real s2m = a2 * (Real(2) + a2);                                    // sigma2^2 - 1
      const Real fp1 = Real(0.5) * Bsk * sig1 * s1m + Dsk * a1 * a1 * a1;
      const Real fp2 = Real(0.5) * Bsk * sig2 * s2m + Dsk * a2 * a2 * a2;
      const Real w1 = A0 * (Cst * dA1 + fp1), w2 = A0 * (Cst * dA2 + fp2), wr = beta * Cst * A0;
      // dE/dF = w1 u1 v1^T + w2 u2 v2^T + wr F_u, with v2 = (-vy, vx)
      const Real G0x = w1 * u1x * vx - w2 * u2x * vy + wr * g0x;
      const Real G0y = w1 * u1y * vx - w2 * u2y * vy + wr * g0y;
      const Real G0z = w1 * u1z * vx - w2 * u2z * vy + wr * g0z;
      const Real G1x = w1 * u1x * vy + w2 * u2x * vx + wr * g1x;
      const Real G1y = w1 * u1y * vy + w2 * u2y * vx + wr * g1y;
      const Real G1z = w1 * u1z * vy + w2 * u2z * vx + wr * g1z;
      // corner gradients [g_a g_b] = dE/dF D_m^-T, g_c = -g_a - g_b, plus the volume
      // gradient k C / G_n * (e1 x e2) / 6 on each corner
      Real gax = G0x * d00 + G1x * d01, gay = G0y * d00 + G1y * d01, gaz = G0z * d00 + G1z * d01;
      Real gbx = G0x * d10 + G1x * d11, gby = G0y * d10 + G1y * d11, gbz = G0z * d10 + G1z * d11;
      if (area_on) {
        // global area: k_A (A - A0) / G_A times grad A_t, which is -(n/2) x e2 at corner a
        // and (n/2) x e1 at corner b (n the unit normal, from the raw cross product)
        const Real e1x = Real(E1x), e1y = Real(E1y), e1z = Real(E1z);
        const Real e2x = Real(E2x), e2y = Real(E2y), e2z = Real(E2z);
        const Real mx = ca * hx, my = ca * hy, mz = ca * hz;      // zero for a collapsed triangle
        gax -= my * e2z - mz * e2y;
        gay -= mz * e2x - mx * e2z;
        gaz -= mx * e2y - my * e2x;
        gbx += my * e1z - mz * e1y;
        gby += mz * e1x - mx * e1z;
        gbz += mx * e1y - my * e1x;
      }
      work[0 * ch + tt] = gax;
      work[1 * ch + tt] = gay;
      work[2 * ch + tt] = gaz;
      work[3 * ch + tt] = gbx;
      work[4 * ch + tt] = gby;
      work[5 * ch + tt] = gbz;
      work[6 * ch + tt] = nx;
      work[7 * ch + tt] = ny;
      work[8 * ch + tt] = nz;
      if (!pre) {
        // x_a . (x_b x x_c) = E1 . (E2 x x_c) with E1 = x_a - x_c, E2 = x_b - x_c (FP64)
        const double cx = (double)xc + (double)ucx, cy = (double)yc + (double)ucy, cz = (double)zc + (double)ucz;
        accC[4] += E1x * (E2y * cz - E2z * cy) + E1y * (E2z * cx - E2x * cz) + E1z * (E2x * cy - E2y * cx);
        accC[5] += (double)J * area_t;                      // deformed area = J A0
      }
      accC[6] += collapsed ? 1.0 : 0.0;
      accC[0] += 0.5 * (double)(Cst * A0) * ((double)dA1 * dA1 + (double)dA2 * dA2);
      accC[1] += (double)A0 * (0.125 * (double)Bsk * ((double)s1m * s1m + (double)s2m * s2m)
                               + 0.25 * (double)Dsk * ((double)a1 * a1 * a1 * a1 + (double)a2 * a2 * a2 * a2));
      accC[2] += 0.5 * (double)wr * ((double)g0x * g0x + (double)g0y * g0y + (double)g0z * g0z
                                     + (double)g1x * g1x + (double)g1y * g1y + (double)g1z * g1z);
    }
    if (!pre) {
      double vv[2] = {accC[4], accC[5]};
      block_sum<2>(vv, red);                  // also the barrier before the gather
      vol = vv[0] / 6.0;
      area = vv[1];
      coefd = mat.k_volume * (vol - M.V0) / Gn;
    } else {
      __syncthreads();
    }
    const Real coef = Real(coefd / 6.0);         // per corner: k C / G_n * (e1 x e2) / 6
    const bool last = t0 + ch >= nt;
    for (int i = tid(); i < n; i += kBlock) {
      Real gx = 0, gy = 0, gz = 0, vx = 0, vy = 0, vz = 0;
      // Branch-free, so that the reads of all corners are in flight together: a padding
      // entry, or a corner outside this chunk, reads the chunk's first triangle and adds
      // zero; corner k adds g_a, g_b or -(g_a + g_b) (the same roundings as adding each
      // case on its own).
      Real mass = 0;
      for (int q0 = 0; q0 < M.vc_deg; q0 += kEllGroup) {
        int cc[kEllGroup];
#pragma unroll
        for (int u = 0; u < kEllGroup; ++u) cc[u] = q0 + u < M.vc_deg ? gld(M.vc_ell, (q0 + u) * np + i) : -1;
        if (q0 == 0 && last) mass = gld(M.mass, i);      // with the first group
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < kEllGroup; ++u) {
          const int cid = cc[u];
          const int tri = cid / 3, k = cid - 3 * tri, t = tri - t0;
          const bool ok = cid >= 0 && t >= 0 && t < tn;
          const int tc = ok ? t : 0;
          const Real ax = work[tc], ay = work[ch + tc], az = work[2 * ch + tc];
          const Real bx = work[3 * ch + tc], by = work[4 * ch + tc], bz = work[5 * ch + tc];
          const Real nx = work[6 * ch + tc], ny = work[7 * ch + tc], nz = work[8 * ch + tc];
          const Real sg = ok ? (k == 2 ? Real(-1) : Real(1)) : Real(0);
          gx += sg * (k == 0 ? ax : (k == 1 ? bx : ax + bx));
          gy += sg * (k == 0 ? ay : (k == 1 ? by : ay + by));
          gz += sg * (k == 0 ? az : (k == 1 ? bz : az + bz));
          vx += ok ? nx : Real(0);
          vy += ok ? ny : Real(0);
          vz += ok ? nz : Real(0);
        }
      }
      gx += coef * vx;
      gy += coef * vy;
      gz += coef * vz;
      gx += gout[i];
      gy += gout[np + i];
      gz += gout[2 * np + i];
      gout[i] = gx;
      gout[np + i] = gy;
      gout[2 * np + i] = gz;
      if (last) {
        const Real mi = mass * inv_h2;
        const Real ux = ut[i], uy = ut[np + i], uz = ut[2 * np + i];
        const Real bx = bvec[i], by = bvec[np + i], bz = bvec[2 * np + i];
        const double mux = (double)mi * ux, muy = (double)mi * uy, muz = (double)mi * uz;
        const double fx = gx - (mux - bx), fy = gy - (muy - by), fz = gz - (muz - bz);
        accD[0] += (double)gx * gx + (double)gy * gy + (double)gz * gz;
        accD[1] += mux * mux + muy * muy + muz * muz;
        accD[2] += (double)bx * bx + (double)by * by + (double)bz * bz;
        accD[3] += fx * fx + fy * fy + fz * fz;
        accC[3] += fabs((double)ux * bx + (double)uy * by + (double)uz * bz);
      }
    }
    __syncthreads();
  }
  const double Cv = vol - M.V0, Ca = area - M.A0;
  const double e_vol = 0.5 * mat.k_volume * Cv * Cv / Gn;
  const double e_area = area_on ? 0.5 * mat.k_area_global * Ca * Ca / GA : 0.0;
  double acc[11] = {accB[0], accC[0], accC[1], accC[2], accC[3], accD[0], accD[1], accD[2], accD[3], accC[6], accB[1]};
  block_sum<11>(acc, red);
  const double e_col = acc[10];
  const double inertial = acc[0];
  res.vol = vol;
  res.area = area;
  res.degen = acc[9];
  res.terms[0] = inertial;
  res.terms[1] = acc[1];
  res.terms[2] = acc[2];
  res.terms[3] = accA[1] + accA[2];
  res.terms[4] = e_vol;
  res.terms[5] = acc[3];
  res.terms[6] = e_area;
  res.terms[7] = e_col;
  res.E = inertial + acc[1] + acc[2] + accA[1] + accA[2] + e_vol + acc[3] + e_area + e_col;
  // rounding scale of E: the sum of the magnitudes of its terms
  res.noise = fabs(inertial) + 2.0 * acc[4] + acc[1] + acc[2] + accA[1] + accA[2] + e_vol + acc[3] + e_area + e_col;
  const double num = sqrt(acc[5]);
  const double den = sqrt(acc[6]) + sqrt(acc[7]) + sqrt(acc[8]) + M.floor_force;
  res.resid = num == 0.0 ? 0.0 : num / den;
  if (!isfinite(res.E) || !isfinite(num)) res.resid = INFINITY;
}

// ---------------------------------------------------------------------------------
// Tile product Out^T = In^T A with A = A^T (n_pad x n_pad), In^T / Out^T (rows x n_pad)
// on the matrix cores.  16x16 output blocks; each wave owns every fourth column block
// and all (<= 4) row blocks, so an A fragment is loaded once per wave and reused.
// Both operands are read as vectors along k (A is symmetric, so its column fragment is
// a row fragment).  Operand lanes: lane l supplies row l%16, k-slot l/16 of A_op and
// k-slot l/16, column l%16 of B_op; result slot i of lane l is row 4(l/16) + i (f32)
// or row 4i + l/16 (f64), column l%16 (measured on gfx950).
// ---------------------------------------------------------------------------------
__device__ inline void tile_gemm(const float* __restrict__ A, int np, const float* __restrict__ In,
                                 float* __restrict__ Out, int rows) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  const int mb_n = (rows + 15) >> 4;
  for (int nb = wave; nb < (np >> 4); nb += 4) {
    const int n0 = nb << 4;
    floatx4 acc[4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) acc[mb] = floatx4{0.f, 0.f, 0.f, 0.f};
    const float* arow = A + (size_t)(n0 + l16) * np + 4 * kq;
    for (int k0 = 0; k0 < np; k0 += 16) {
      const floatx4 bq = *reinterpret_cast<const floatx4*>(arow + k0);
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) {
        if (mb < mb_n) {
          const int r = mb * 16 + l16;
          const floatx4 aq = r < rows ? *reinterpret_cast<const floatx4*>(In + (size_t)r * np + k0 + 4 * kq)
                                      : floatx4{0.f, 0.f, 0.f, 0.f};
          acc[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(aq.x, bq.x, acc[mb], 0, 0, 0);
          acc[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(aq.y, bq.y, acc[mb], 0, 0, 0);
          acc[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(aq.z, bq.z, acc[mb], 0, 0, 0);
          acc[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(aq.w, bq.w, acc[mb], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      if (mb < mb_n) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = mb * 16 + 4 * kq + i;
          if (r < rows) Out[(size_t)r * np + n0 + l16] = acc[mb][i];
        }
      }
    }
  }
}

__device__ inline void tile_gemm(const double* __restrict__ A, int np, const double* __restrict__ In,
                                 double* __restrict__ Out, int rows) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  const int mb_n = (rows + 15) >> 4;
  for (int nb = wave; nb < (np >> 4); nb += 4) {
    const int n0 = nb << 4;
    doublex4 acc[4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) acc[mb] = doublex4{0.0, 0.0, 0.0, 0.0};
    const double* arow = A + (size_t)(n0 + l16) * np + 4 * kq;
    for (int k0 = 0; k0 < np; k0 += 16) {
      const doublex4 bq = *reinterpret_cast<const doublex4*>(arow + k0);
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) {
        if (mb < mb_n) {
          const int r = mb * 16 + l16;
          const doublex4 aq = r < rows ? *reinterpret_cast<const doublex4*>(In + (size_t)r * np + k0 + 4 * kq)
                                       : doublex4{0.0, 0.0, 0.0, 0.0};
          acc[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(aq.x, bq.x, acc[mb], 0, 0, 0);
          acc[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(aq.y, bq.y, acc[mb], 0, 0, 0);
          acc[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(aq.z, bq.z, acc[mb], 0, 0, 0);
          acc[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(aq.w, bq.w, acc[mb], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      if (mb < mb_n) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = mb * 16 + 4 * i + kq;   // f64 result: slot i of lane l is row 4i + l/16
          if (r < rows) Out[(size_t)r * np + n0 + l16] = acc[mb][i];
        }
      }
    }
  }
}

// BF16 variant for FP32 plans: Out^T = In^T (diag(a) + A_off) with the off-diagonal part
// A_off in BF16 on the matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation) and
// the diagonal applied exactly in FP32 in the epilogue.  In is rounded to BF16 on the
// fly (8 consecutive k per lane, the same k order for both operands).
__device__ inline void tile_gemm_bf16(const uint16_t* __restrict__ Abits, const float* __restrict__ diag,
                                      int np, const float* __restrict__ In, float* __restrict__ Out,
                                      int rows) {
  const __bf16* A = reinterpret_cast<const __bf16*>(Abits);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  const int mb_n = (rows + 15) >> 4;
  for (int nb = wave; nb < (np >> 4); nb += 4) {
    const int n0 = nb << 4;
    floatx4 acc[4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) acc[mb] = floatx4{0.f, 0.f, 0.f, 0.f};
    const __bf16* arow = A + (size_t)(n0 + l16) * np + 8 * kq;
    for (int k0 = 0; k0 < np; k0 += 32) {
      const bf16x8 bq = *reinterpret_cast<const bf16x8*>(arow + k0);
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) {
        if (mb < mb_n) {
          const int r = mb * 16 + l16;
          bf16x8 aq;
          if (r < rows) {
            const floatx4 lo = *reinterpret_cast<const floatx4*>(In + (size_t)r * np + k0 + 8 * kq);
            const floatx4 hi = *reinterpret_cast<const floatx4*>(In + (size_t)r * np + k0 + 8 * kq + 4);
            aq = bf16x8{(__bf16)lo.x, (__bf16)lo.y, (__bf16)lo.z, (__bf16)lo.w,
                        (__bf16)hi.x, (__bf16)hi.y, (__bf16)hi.z, (__bf16)hi.w};
          } else {
            aq = bf16x8{(__bf16)0.f, (__bf16)0.f, (__bf16)0.f, (__bf16)0.f,
                        (__bf16)0.f, (__bf16)0.f, (__bf16)0.f, (__bf16)0.f};
          }
          acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aq, bq, acc[mb], 0, 0, 0);
        }
      }
    }
    const float dn = diag[n0 + l16];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      if (mb < mb_n) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = mb * 16 + 4 * kq + i;
          if (r < rows) {
            const size_t o = (size_t)r * np + n0 + l16;
            Out[o] = acc[mb][i] + dn * In[o];
          }
        }
      }
    }
  }
}

// n_pad up to which the whole k range of the staged BF16 product fits one chunk.
constexpr int kStageMaxPad = 1024;

// The same product with the tile's rows staged in LDS as BF16 (rows padded to 16), in
// chunks of at most kc_max columns of k (one chunk when the rows fit the LDS region; a
// chunk needs 16 ceil(rows/16) (kc + 8) BF16 of LDS at `stage`; the partial products of
// later chunks are added to Out by the lane that wrote it), each wave carrying four
// column blocks at a time, so that four independent B fragments are in flight per k step
// and every A fragment read from LDS feeds four matrix instructions.
// The off-diagonal part is stored in an order of the vertices (position k' holds vertex
// perm[k']) and each 16-column block is applied over the k' range band[2 cb],
// band[2 cb + 1] only: with inverse_bf16 = 2 a reverse Cuthill-McKee order, in which the
// inverse's significant entries lie near the diagonal, and the range that holds them;
// with inverse_bf16 = 1 the identity (perm null) and the whole range.  The input rows
// are gathered through the permutation as they are staged, and each output column n' goes to vertex
// perm[n'], with the exact FP32 diagonal of that vertex.  A wave's four column blocks
// are consecutive, so their ranges nearly coincide; it runs over their union (the stored
// matrix is zero outside each block's own range).
__device__ inline void tile_gemm_bf16_band(const uint16_t* __restrict__ Abits, const float* __restrict__ diag,
                                           const int* __restrict__ perm, const int* __restrict__ band, int np,
                                           const float* __restrict__ In, float* __restrict__ Out, int rows,
                                           __bf16* stage, int kc_max) {
  const __bf16* A = reinterpret_cast<const __bf16*>(Abits);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  const int mb_n = (rows + 15) >> 4;
  constexpr int NB = 4;
  const int ncb = np >> 4;
  for (int kb0 = 0; kb0 < np; kb0 += kc_max) {
    const int kc = min(kc_max, np - kb0);               // a multiple of 32
    const int ldk = kc + 8;
    const int k8n = kc >> 3;
    __syncthreads();
    if (perm) {                                         // gathered through the order
#pragma unroll 4
      for (int e = tid(); e < mb_n * 16 * k8n; e += kBlock) {
        const int r = e / k8n, k8 = (e - r * k8n) << 3;
        const int4 p0 = *reinterpret_cast<const int4*>(perm + kb0 + k8);
        const int4 p1 = *reinterpret_cast<const int4*>(perm + kb0 + k8 + 4);
        const float* row = In + (size_t)(r < rows ? r : 0) * np;
        const float z = r < rows ? 1.f : 0.f;
        const bf16x8 v = {(__bf16)(z * row[p0.x]), (__bf16)(z * row[p0.y]), (__bf16)(z * row[p0.z]),
                          (__bf16)(z * row[p0.w]), (__bf16)(z * row[p1.x]), (__bf16)(z * row[p1.y]),
                          (__bf16)(z * row[p1.z]), (__bf16)(z * row[p1.w])};
        *reinterpret_cast<bf16x8*>(stage + r * ldk + k8) = v;
      }
    } else {                                            // the identity order: 16-byte loads
      for (int e = tid(); e < mb_n * 16 * k8n; e += kBlock) {
        const int r = e / k8n, k8 = (e - r * k8n) << 3;
        bf16x8 v;
        if (r < rows) {
          const floatx4 lo = *reinterpret_cast<const floatx4*>(In + (size_t)r * np + kb0 + k8);
          const floatx4 hi = *reinterpret_cast<const floatx4*>(In + (size_t)r * np + kb0 + k8 + 4);
          v = bf16x8{(__bf16)lo.x, (__bf16)lo.y, (__bf16)lo.z, (__bf16)lo.w,
                     (__bf16)hi.x, (__bf16)hi.y, (__bf16)hi.z, (__bf16)hi.w};
        } else {
          v = bf16x8{(__bf16)0.f, (__bf16)0.f, (__bf16)0.f, (__bf16)0.f,
                     (__bf16)0.f, (__bf16)0.f, (__bf16)0.f, (__bf16)0.f};
        }
        *reinterpret_cast<bf16x8*>(stage + r * ldk + k8) = v;
      }
    }
    __syncthreads();
    // one 16-row block of the tile at a time (a 5-cell tile has one): the accumulators of
    // one row block by NB column blocks stay small next to the step's other live values
    for (int mb = 0; mb < mb_n; ++mb) {
      for (int g0 = NB * wave; g0 < ncb; g0 += 4 * NB) {
        floatx4 acc[NB];
        const __bf16* arow[NB];
        bool valid[NB];
        int lo = np, hi = 0;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          const int cb = g0 + q;
          valid[q] = cb < ncb;
          arow[q] = A + (size_t)((valid[q] ? cb : 0) * 16 + l16) * np + kb0 + 8 * kq;
          if (valid[q]) {
            lo = min(lo, band[2 * cb]);
            hi = max(hi, band[2 * cb + 1]);
          }
          acc[q] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
        const int k_lo = max(lo, kb0) - kb0, k_hi = min(hi, kb0 + kc) - kb0;   // this chunk's part
        const __bf16* srow = stage + (mb * 16 + l16) * ldk + 8 * kq;
        for (int k0 = k_lo; k0 < k_hi; k0 += 32) {
          bf16x8 bq[NB];
#pragma unroll
          for (int q = 0; q < NB; ++q) bq[q] = *reinterpret_cast<const bf16x8*>(arow[q] + k0);
          const bf16x8 aq = *reinterpret_cast<const bf16x8*>(srow + k0);
#pragma unroll
          for (int q = 0; q < NB; ++q) acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aq, bq[q], acc[q], 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          if (!valid[q]) continue;
          const int n = perm ? perm[(g0 + q) * 16 + l16] : (g0 + q) * 16 + l16;
          const float dn = diag[n];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int r = mb * 16 + 4 * kq + i;
            if (r < rows) {
              const size_t o = (size_t)r * np + n;
              Out[o] = acc[q][i] + (kb0 == 0 ? dn * In[o] : Out[o]);
            }
          }
        }
      }
    }
  }
}

// The tile's product with H~^-1 (which 0) or h^2 M~^-1 (which 1) in the plan's format.
// Kept out of line: inlined into the step, its accumulators and staging add to the
// register pressure of the whole iteration loop and the step kernel spills more.
template <typename Real>
__device__ __attribute__((noinline)) void tile_product(const MeshDev<Real>& M, const SolverDev& sol, int which, const Real* In,
                                    Real* Out, int rows, unsigned char* stage, int stage_k) {
  if constexpr (std::is_same<Real, float>::value) {
    if (sol.bf16) {
      const uint16_t* Ab = which == 0 ? M.hinv_bf : M.minv_bf;
      const float* dg = which == 0 ? M.hinv_diag : M.minv_diag;
      // staged (banded, or dense with the identity order); unstaged only for dense storage
      // (the host guarantees stage_k >= 32 for banded storage)
      if (stage_k >= 32)
        tile_gemm_bf16_band(Ab, dg, M.bperm, M.bband + which * 2 * (M.n_pad >> 4), M.n_pad, In, Out, rows,
                            reinterpret_cast<__bf16*>(stage), stage_k);
      else
        tile_gemm_bf16(Ab, dg, M.n_pad, In, Out, rows);
      return;
    }
  }
  tile_gemm(which == 0 ? M.hinv : M.minv, M.n_pad, In, Out, rows);
}

// ---------------------------------------------------------------------------------
// The step
// ---------------------------------------------------------------------------------
enum { VB = 0, VU, VG, VD, VQ, VS0 };   // per-cell workspace vectors (history from VS0)

template <typename Real>
struct Tile {
  Real* W;
  int np, T;
  __device__ Real* vec(int v, int j) const { return W + ((size_t)v * T + j) * 3 * np; }
  __device__ Real* mat(int v) const { return W + (size_t)v * T * 3 * np; }
};

template <typename Real, typename CST>
__device__ void finalize_cell(const StepArgs<Real>& A, const MeshDev<Real>& M, int cell, int64_t voff, CST& cs,
                              const Real* xn, const Real* U, double* red, double* bc) {
  const int n = M.n, np = M.n_pad;
  const double h = A.sol.h;
  Real* xo = A.x_out + 3 * voff;
  Real* vo = A.v_out + 3 * voff;
  if (cs.status & NPFEM_NONFINITE) {
    for (int e = tid(); e < 3 * n; e += kBlock) {
      const int i = e / 3, c = e - 3 * i;
      xo[e] = xn[c * np + i];
      vo[e] = A.v[3 * voff + e];
    }
  } else {
    // v = u / h, then damp its departure from the best-fit rigid motion (section 2.1.4)
    double s1[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int i = tid(); i < n; i += kBlock) {
      const double m = gld(M.mass, i);
      s1[0] += m;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double x = (double)xn[c * np + i] + (double)U[c * np + i];
        s1[1 + c] += m * x;
        s1[4 + c] += m * ((double)U[c * np + i] / h);
      }
    }
    block_sum<7>(s1, red);
    const double xc[3] = {s1[1] / s1[0], s1[2] / s1[0], s1[3] / s1[0]};
    const double vc[3] = {s1[4] / s1[0], s1[5] / s1[0], s1[6] / s1[0]};
    double s2[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};   // L (3), I_xx I_yy I_zz I_xy I_xz I_yz
    for (int i = tid(); i < n; i += kBlock) {
      const double m = gld(M.mass, i);
      const double rx = (double)xn[i] + (double)U[i] - xc[0];
      const double ry = (double)xn[np + i] + (double)U[np + i] - xc[1];
      const double rz = (double)xn[2 * np + i] + (double)U[2 * np + i] - xc[2];
      const double vx = (double)U[i] / h, vy = (double)U[np + i] / h, vz = (double)U[2 * np + i] / h;
      s2[0] += m * (ry * vz - rz * vy);
      s2[1] += m * (rz * vx - rx * vz);
      s2[2] += m * (rx * vy - ry * vx);
      s2[3] += m * (ry * ry + rz * rz);
      s2[4] += m * (rx * rx + rz * rz);
      s2[5] += m * (rx * rx + ry * ry);
      s2[6] -= m * rx * ry;
      s2[7] -= m * rx * rz;
      s2[8] -= m * ry * rz;
    }
    block_sum<9>(s2, red);
    // omega = I^-1 L (3x3 symmetric, adjugate)
    const double Ixx = s2[3], Iyy = s2[4], Izz = s2[5], Ixy = s2[6], Ixz = s2[7], Iyz = s2[8];
    const double c00 = Iyy * Izz - Iyz * Iyz, c01 = Ixz * Iyz - Ixy * Izz, c02 = Ixy * Iyz - Ixz * Iyy;
    const double c11 = Ixx * Izz - Ixz * Ixz, c12 = Ixy * Ixz - Ixx * Iyz, c22 = Ixx * Iyy - Ixy * Ixy;
    const double det = Ixx * c00 + Ixy * c01 + Ixz * c02;
    double w[3] = {0, 0, 0};
    if (det > 0) {
      w[0] = (c00 * s2[0] + c01 * s2[1] + c02 * s2[2]) / det;
      w[1] = (c01 * s2[0] + c11 * s2[1] + c12 * s2[2]) / det;
      w[2] = (c02 * s2[0] + c12 * s2[1] + c22 * s2[2]) / det;
    }
    const double kap = A.mat.kappa;
    for (int i = tid(); i < n; i += kBlock) {
      const double rx = (double)xn[i] + (double)U[i] - xc[0];
      const double ry = (double)xn[np + i] + (double)U[np + i] - xc[1];
      const double rz = (double)xn[2 * np + i] + (double)U[2 * np + i] - xc[2];
      const double vx = (double)U[i] / h, vy = (double)U[np + i] / h, vz = (double)U[2 * np + i] / h;
      const double dvx = vc[0] + (w[1] * rz - w[2] * ry) - vx;
      const double dvy = vc[1] + (w[2] * rx - w[0] * rz) - vy;
      const double dvz = vc[2] + (w[0] * ry - w[1] * rx) - vz;
      vo[3 * i] = (Real)(vx + kap * dvx);
      vo[3 * i + 1] = (Real)(vy + kap * dvy);
      vo[3 * i + 2] = (Real)(vz + kap * dvz);
      xo[3 * i] = xn[i] + U[i];
      xo[3 * i + 1] = xn[np + i] + U[np + i];
      xo[3 * i + 2] = xn[2 * np + i] + U[2 * np + i];
    }
  }
  if (A.stats && tid() == 0) {
    npfem_cell_stats st;
    st.iterations = cs.iter;
    st.evaluations = cs.evals;
    st.status = (uint32_t)cs.status | ((cs.degen && !(cs.status & NPFEM_NONFINITE)) ? NPFEM_DEGENERATE_TRI : 0u) |
                (cs.fallback ? NPFEM_START_FALLBACK : 0u);
    st.halvings = cs.halvings;
    st.residual = cs.resid;
    st.objective = cs.E;
    st.volume = bc[0];
    st.area = bc[1];
    A.stats[cell] = st;
  }
}

template <typename Real, int H, bool EXT, int LAY, typename CST>
__device__ __attribute__((always_inline)) inline void run_tile(const StepArgs<Real>& A, int tile, Real* W, CST* CS, double* red,
                         int* sint, unsigned char* lds) {
  const TileDesc td = A.tiles[tile];
  MeshDev<Real>* Ml = reinterpret_cast<MeshDev<Real>*>(lds + kLdsMesh);
  // the tile's cells and their vertex offsets, looked up once per tile
  __shared__ int s_cell[kMaxTile];
  __shared__ int64_t s_voff[kMaxTile];
  {
    constexpr int nw = sizeof(MeshDev<Real>) / 4;
    static_assert(nw <= 128, "mesh descriptor copy");
    const int* src = reinterpret_cast<const int*>(A.meshes + td.mesh);
    if (tid() < nw) reinterpret_cast<int*>(Ml)[tid()] = src[tid()];
    const int jt = tid() - 128;
    if (jt >= 0 && jt < td.count) {
      const int c = A.tile_cells[td.first + jt];
      s_cell[jt] = c;
      s_voff[jt] = A.cell_voff[c];
    }
    __syncthreads();
  }
  const MeshDev<Real>& M = *Ml;
  const int n = M.n, np = M.n_pad, cnt = td.count, len = 3 * np;
  Tile<Real> tl{W, np, A.tile_cells_max};
  // the current cell's x_n and trial u (and gradient and b) in LDS, then the corner
  // chunks; for meshes too large for that, x_n and u follow the tile's vectors in the
  // workspace and the LDS holds the corner chunks only
  // (LAY is the batch's layout, the largest over its meshes: 0 all in LDS, 1 gradient
  // and b in the workspace, 2 x_n and u too; below it the placement is known at compile
  // time and every access to these vectors is an LDS instruction)
  const bool vl = LAY == 0 || M.vec_lds != 0, xl = LAY < 2 || M.xu_lds != 0;
  unsigned char* stage = lds + kLdsHeader;                   // BF16 staging of the tile product
  Real* xn = xl ? reinterpret_cast<Real*>(lds + kLdsHeader) : W + (size_t)A.n_vec_slot * A.tile_cells_max * 3 * np;
  Real* ut = xn + 3 * np;
  Real* gl = ut + 3 * np;
  Real* bl = gl + 3 * np;
  Real* work = reinterpret_cast<Real*>(lds + kLdsHeader) + (xl ? (vl ? 12 : 6) * np : 0);
  const double h = A.sol.h;
  const int m = A.sol.m;
  const double eps = Eps<Real>::v;
  __shared__ double s_vol[kMaxTile], s_area[kMaxTile];
  const bool area_on = EXT && A.mat.k_area_global > 0.0, literal = EXT && A.sol.literal != 0;
  auto contacts = [&](int j) {
    return EXT && A.col_n ? Contacts<Real>{A.col_q + 3 * s_voff[j], A.col_n + 3 * s_voff[j], A.w_col}
                   : Contacts<Real>{nullptr, nullptr, 0.0};
  };
  // per cell: gradient and b in LDS, or (meshes too large for that) in the workspace
  auto gvec = [&](int j) { return vl ? gl : tl.vec(VS0 + 2 * m, j); };
  auto bvec = [&](int j) { return vl ? bl : tl.vec(VB, j); };

  // ---- initial state: b = M v_n / h + F_ext, |grad V(x_n)|^2, first guess --------
  for (int j = 0; j < cnt; ++j) {
    const int64_t voff = s_voff[j];
    stage_aos(xn, A.x + 3 * voff, n, np);
    const Real* vs = A.v + 3 * voff;
    const Real* fs = A.f + 3 * voff;
    aos_to_soa(tl.vec(VB, j), n, np, [&](int e) { return gld(M.mass, e / 3) * vs[e] / Real(h) + fs[e]; });
    if (A.u_guess) {
      const Real* gs = A.u_guess + 3 * voff;
      aos_to_soa(tl.vec(VU, j), n, np, [&](int e) { return gs[e]; });
    }
    __syncthreads();
    // normalisers at x_n (ut and, for the area term, the cell's gradient vector are free
    // until the first evaluation)
    double Gn, GA;
    normalisers(M, xn, static_cast<const Real*>(nullptr), ut, area_on ? gvec(j) : static_cast<Real*>(nullptr),
                work, red, Gn, GA);
    if (tid() == 0) {
      auto& cs = CS[j];
      cs.Gn = Gn;
      cs.GA = GA;
      cs.hist_n = cs.hist_head = cs.iter = cs.evals = cs.status = cs.retry = cs.halvings = cs.degen = cs.fallback = 0;
      cs.active = 1;
    }
    __syncthreads();
  }
  if (!A.u_guess) {
    tile_product(M, A.sol, 1, tl.mat(VB), tl.mat(VU), 3 * cnt, stage, A.stage_k);                                              // u = h^2 M~^-1 b
    __syncthreads();
    if (A.guess_only) {
      for (int j = 0; j < cnt; ++j) {
        const int64_t voff = s_voff[j];
        const Real* U = tl.vec(VU, j);
        for (int e = tid(); e < len; e += kBlock) {
          const int c = e / np, i = e - c * np;
          if (i < n) A.x_out[3 * (voff + i) + c] = U[e];
        }
      }
      return;
    }
  }

  // ---- first evaluation ---------------------------------------------------------
  // With a learned correction delta the cell is evaluated at y_n and at y_n + delta and
  // goes on from y_n + delta only if that does not raise the objective; otherwise it
  // starts from y_n as the plain step does (status bit NPFEM_START_FALLBACK).
  for (int j = 0; j < cnt; ++j) {
    stage_aos(xn, A.x + 3 * s_voff[j], n, np);
    vcopy(ut, tl.vec(VU, j), len);
    if (vl) vcopy(bl, tl.vec(VB, j), len);
    __syncthreads();
    EvalResult r;
    evaluate<Real, EXT>(M, A.mat, literal, h, CS[j].Gn, CS[j].GA, contacts(j), xn, ut, bvec(j), work, gvec(j), red, r);
    bool fallback = false;
    vcopy(tl.vec(VG, j), gvec(j), len);
    if (A.u_delta) {
      const int64_t voff = s_voff[j];
      for (int e = tid(); e < len; e += kBlock) {
        const int c = e / np, i = e - c * np;
        if (i < n) ut[e] += A.u_delta[3 * (voff + i) + c];
      }
      __syncthreads();                                           // VG holds grad g(y_n); ut = u0 + delta
      EvalResult r1;
      evaluate<Real, EXT>(M, A.mat, literal, h, CS[j].Gn, CS[j].GA, contacts(j), xn, ut, bvec(j), work, gvec(j), red,
                          r1);
      if (isfinite(r1.E) && isfinite(r1.resid) && r1.E <= r.E) {
        r = r1;
        vcopy(tl.vec(VU, j), ut, len);
        vcopy(tl.vec(VG, j), gvec(j), len);
      } else {
        fallback = true;
      }
    }
    const bool bad = !isfinite(r.E) || !isfinite(r.resid);
    const bool done = bad || r.resid <= A.sol.tol;
    if (!done) vcopy(tl.vec(VQ, j), fallback ? tl.vec(VG, j) : gvec(j), len);
    if (tid() == 0) {
      auto& cs = CS[j];
      cs.E = r.E;
      cs.noise = r.noise;
      cs.resid = r.resid;
      cs.evals = A.u_delta ? 2 : 1;
      cs.degen = r.degen > 0.0;
      cs.fallback = fallback;
      s_vol[j] = r.vol;
      s_area[j] = r.area;
      if (bad) { cs.status = NPFEM_NONFINITE; cs.active = 0; }
      else if (done) { cs.status = NPFEM_CONVERGED; cs.active = 0; }
    }
    __syncthreads();
  }

  // ---- quasi-Newton iterations (Algorithm 1, while loop) --------------------------
  // L-BFGS two-loop recursion (Nocedal & Wright Alg. 7.4) written with the matrix
  // SY[i][j] = s_i . y_j of the stored pairs: with q_i = g - sum_{j newer} alpha_j y_j,
  //   alpha_i = rho_i (s_i . g - sum_{j newer} alpha_j SY[i][j]),
  // and with z_i = r + sum_{j older} (alpha_j - beta_j) s_j, r = H~^-1 q,
  //   beta_i = rho_i (y_i . r + sum_{j older} (alpha_j - beta_j) SY[j][i]),
  // so each half of the recursion is one pass of dot products plus one pass that
  // combines vectors.  The dot products the first half needs are accumulated while
  // the step is accepted.
  //
  // Every round an active cell accepts a step (iter + 1, bounded by max_iter) or clears
  // its history for one retry, so 2 max_iter + 2 rounds always suffice.
  const int max_rounds = 2 * A.sol.max_iter + 2;
  for (int round = 0;; ++round) {
    if (tid() == 0) {
      int act = 0;
      for (int j = 0; j < cnt; ++j) {
        if (round >= max_rounds && CS[j].active) {
          CS[j].active = 0;
          CS[j].status = NPFEM_MAXITER;
        }
        act += CS[j].active;
      }
      sint[1] = act;
    }
    __syncthreads();
    if (sint[1] == 0) break;
    tile_product(M, A.sol, 0, tl.mat(VQ), tl.mat(VD), 3 * cnt, stage, A.stage_k);                                              // r = H~^-1 q
    __syncthreads();
    for (int j = 0; j < cnt; ++j) {
      auto& cs = CS[j];
      if (!cs.active) continue;                                  // uniform: read after a barrier
      Real* U = tl.vec(VU, j);
      Real* G = tl.vec(VG, j);
      Real* GT = gvec(j);                                        // trial gradient
      Real* D = tl.vec(VD, j);
      Real* Q = tl.vec(VQ, j);
      const int hn = cs.hist_n, head = cs.hist_head;
      // ring slot of stored pair p (0 oldest .. hn-1 newest); with no history (m = 0)
      // nothing is stored and no slot is ever read
      auto slot = [&](int p) { return m > 0 ? (head - hn + p + m) % m : 0; };
      constexpr int W = Vec16<Real>::W;
      typedef typename Vec16<Real>::type V;
      // When a vector takes at most two 16-byte slots per thread, r and the stored y_p are
      // loaded in one batch together with the staging of x_n and b and kept in registers
      // until the direction is formed, so the two halves below cost two memory round
      // trips instead of four.  The sums run in the same order either way.
      const bool fused = len <= 2 * W * kBlock;
      const V zero = {};
      V rr[2], ys[H][2];
      const int ek[2] = {W * tid(), W * tid() + W * kBlock};
      if (fused) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const bool in = ek[k] < len;
          rr[k] = in ? vload(D, ek[k]) : zero;
#pragma unroll
          for (int p = 0; p < H; ++p) {
            ys[p][k] = in && hn > 0 ? vload(tl.vec(VS0 + m + slot(p), j), ek[k]) : zero;
          }
        }
      }
      stage_aos(xn, A.x + 3 * s_voff[j], n, np);
      if (vl) vcopy(bl, tl.vec(VB, j), len);
      // second half: y_p . r for every stored pair (one pass)
      double yr[H];
#pragma unroll
      for (int p = 0; p < H; ++p) yr[p] = 0.0;
      if (hn > 0) {
        if (fused) {
#pragma unroll
          for (int k = 0; k < 2; ++k) {
            if (ek[k] < len) {
#pragma unroll
              for (int p = 0; p < H; ++p) {
#pragma unroll
                for (int w = 0; w < W; ++w) yr[p] += (double)(p < hn ? ys[p][k][w] : Real(0)) * rr[k][w];
              }
            }
          }
        } else {
#pragma unroll 2
          for (int e = W * tid(); e < len; e += W * kBlock) {
            const auto rv = vload(D, e);
#pragma unroll
            for (int p = 0; p < H; ++p) {
              if (p < hn) {
                const auto yv = vload(tl.vec(VS0 + m + slot(p), j), e);
#pragma unroll
                for (int w = 0; w < W; ++w) yr[p] += (double)yv[w] * rv[w];
              }
            }
          }
        }
        block_sum<H>(yr, red);
      }
      double cf[H];                                    // alpha_p - beta_p
#pragma unroll
      for (int p = 0; p < H; ++p) {
        cf[p] = 0.0;
        if (p < hn) {
          double acc = yr[p];
#pragma unroll
          for (int q = 0; q < H; ++q)
            if (q < p) acc += cf[q] * cs.SY[slot(q)][slot(p)];
          cf[p] = cs.alpha[slot(p)] - cs.rho[slot(p)] * acc;
        }
      }
      // d = -(r + sum_p cf_p s_p), g . d, and the first trial point u + d staged in LDS
      // (one pass)
      double gdv[1] = {0.0};
      auto d_slot = [&](int e, const V& rv, const V& gv, const V& uv, auto&& s_of) {
        double z[W];
#pragma unroll
        for (int w = 0; w < W; ++w) z[w] = rv[w];
#pragma unroll
        for (int p = 0; p < H; ++p) {
          const V sv = s_of(p);
#pragma unroll
          for (int w = 0; w < W; ++w) z[w] += cf[p] * (double)(p < hn ? sv[w] : Real(0));
        }
        V dv, tv;
#pragma unroll
        for (int w = 0; w < W; ++w) {
          dv[w] = Real(-z[w]);
          tv[w] = uv[w] + dv[w];
          gdv[0] += (double)gv[w] * dv[w];
        }
        vstore(D, e, dv);
        vstore(ut, e, tv);
      };
      if (fused) {
#pragma unroll
        for (int k = 0; k < 2; ++k)
          if (ek[k] < len)
            d_slot(ek[k], rr[k], vload(G, ek[k]), vload(U, ek[k]),
                   [&](int p) { return hn > 0 ? vload(tl.vec(VS0 + slot(p), j), ek[k]) : zero; });
      } else {
#pragma unroll 2
        for (int e = W * tid(); e < len; e += W * kBlock)
          d_slot(e, vload(D, e), vload(G, e), vload(U, e), [&](int p) { return hn > 0 ? vload(tl.vec(VS0 + slot(p), j), e) : zero; });
      }
      block_sum<1>(gdv, red);
      const double gd = gdv[0];
      // line search: alpha = 1, 1/2, ... until sufficient decrease (Algorithm 1)
      double alpha = 1.0;
      bool accepted = false;
      EvalResult r;
      int hv = 0;
      for (; hv <= A.sol.max_halvings; ++hv) {
        if (hv > 0) {
          const Real al = Real(alpha);
#pragma unroll 2
          for (int e = W * tid(); e < len; e += W * kBlock) {
            const auto uv = vload(U, e), dv = vload(D, e);
            vstore(ut, e, uv + al * dv);
          }
          __syncthreads();
        }
        evaluate<Real, EXT>(M, A.mat, literal, h, cs.Gn, cs.GA, contacts(j), xn, ut, bvec(j), work, GT, red, r);
        const double slack = A.sol.noise * fmax(cs.noise, r.noise);
        accepted = isfinite(r.E) && (r.E <= cs.E + A.sol.c1 * alpha * gd + slack);
        if (accepted) break;
        alpha *= 0.5;
      }
      const int evals_add = accepted ? hv + 1 : hv;
      if (!accepted) {
        if (hn > 0) {
          vcopy(Q, G, len);
          __syncthreads();
          if (tid() == 0) {
            cs.hist_n = 0;
            cs.evals += evals_add;
            cs.halvings += evals_add;
          }
        } else if (tid() == 0) {
          cs.status = NPFEM_LS_FAIL;
          cs.active = 0;
          cs.evals += evals_add;
          cs.halvings += evals_add;
        }
        __syncthreads();
        continue;
      }
      // accept: s = alpha d, y = grad_t - grad, u += s, grad = grad_t; in the same pass the
      // dot products of the new pair with itself, with the kept pairs and with the new
      // gradient.  With a full ring the new pair goes into the oldest pair's slot.
      const Real al = Real(alpha);
      const bool full = m > 0 && hn == m;
      const int ns = head;                                       // slot written
      // acc: [0] s.y  [1] s.s  [2] y.y  [3] s.g'  [4+p] s_p.g'  [4+H+p] s.y_p  [4+2H+p] y.s_p
      double acc[4 + 3 * H];
#pragma unroll
      for (int k = 0; k < 4 + 3 * H; ++k) acc[k] = 0.0;
      if (m > 0) {
        Real* Sn = tl.vec(VS0 + ns, j);
        Real* Yn = tl.vec(VS0 + m + ns, j);
#pragma unroll 2
        for (int e = W * tid(); e < len; e += W * kBlock) {
          const auto gt = vload(GT, e), gv = vload(G, e), dv = vload(D, e), uv = vload(U, e);
          const auto sv = al * dv;
          const auto yv = gt - gv;
#pragma unroll
          for (int p = 0; p < H; ++p) {
            // every slot is read (its index is always inside the ring) and the terms of
            // pairs not in use are switched off, so that all reads are in flight together;
            // p = 0 is the slot being replaced when the ring is full
            const bool use = p < hn && !(full && p == 0);
            const auto so = vload(tl.vec(VS0 + slot(p), j), e), yo = vload(tl.vec(VS0 + m + slot(p), j), e);
#pragma unroll
            for (int w = 0; w < W; ++w) {
              const double sw = use ? (double)so[w] : 0.0, yw = use ? (double)yo[w] : 0.0;
              acc[4 + p] += sw * gt[w];
              acc[4 + H + p] += (double)sv[w] * yw;
              acc[4 + 2 * H + p] += (double)yv[w] * sw;
            }
          }
          vstore(Sn, e, sv);
          vstore(Yn, e, yv);
          vstore(U, e, uv + sv);
          vstore(G, e, gt);
#pragma unroll
          for (int w = 0; w < W; ++w) {
            acc[0] += (double)sv[w] * yv[w];
            acc[1] += (double)sv[w] * sv[w];
            acc[2] += (double)yv[w] * yv[w];
            acc[3] += (double)sv[w] * gt[w];
          }
        }
      } else {
#pragma unroll 2
        for (int e = W * tid(); e < len; e += W * kBlock) {
          vstore(U, e, vload(U, e) + al * vload(D, e));
          vstore(G, e, vload(GT, e));
        }
      }
      block_sum<4 + 3 * H>(acc, red);
      // the reduced dot products (the same in every lane) picked by pair index o < H
      auto pick = [&](int base, int o) {
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < H; ++k)
          if (k == o) v = acc[base + k];
        return v;
      };
      const bool store = m > 0 && acc[0] > 1e-12 * sqrt(acc[1] * acc[2]);
      // new history (p = 0 oldest): the kept old pairs (old index p + first_kept), then the
      // new pair in slot ns if it is stored
      const int first_kept = full ? 1 : 0;
      const int n_kept = hn - first_kept;
      const int hn2 = n_kept + (store ? 1 : 0);
      const int head2 = store ? (head + 1) % m : head;
      auto slot2 = [&](int p) { return p < n_kept && m > 0 ? (head - hn + first_kept + p + m) % m : ns; };
      const bool conv = r.resid <= A.sol.tol;
      const bool out_of_iters = cs.iter + 1 >= A.sol.max_iter;
      // first half of the next recursion: alpha_p, newest first
      double al_new[H];
#pragma unroll
      for (int p = H - 1; p >= 0; --p) {
        al_new[p] = 0.0;
        if (p < hn2) {
          const bool isnew = p >= n_kept;
          const double rho = isnew ? 1.0 / acc[0] : cs.rho[slot2(p)];
          double sg = isnew ? acc[3] : pick(4, p + first_kept);
#pragma unroll
          for (int q = H - 1; q >= 0; --q) {
            if (q > p && q < hn2) {
              // SY[slot p][slot q] = s_p . y_q; the new pair is the newest, so p is old here
              const double syq = q >= n_kept ? pick(4 + 2 * H, p + first_kept)   // s_p . y_new
                                             : cs.SY[slot2(p)][slot2(q)];
              sg -= al_new[q] * syq;
            }
          }
          al_new[p] = rho * sg;
        }
      }
      __syncthreads();
      if (tid() == 0) {
        if (store) {
          cs.rho[ns] = 1.0 / acc[0];
          cs.SY[ns][ns] = acc[0];
          for (int p = 0; p < n_kept; ++p) {
            const int sp = slot2(p), o = p + first_kept;
            cs.SY[ns][sp] = pick(4 + H, o);         // s_new . y_p
            cs.SY[sp][ns] = pick(4 + 2 * H, o);     // s_p . y_new
          }
        }
#pragma unroll
        for (int p = 0; p < H; ++p)
          if (p < hn2) cs.alpha[slot2(p)] = al_new[p];
        cs.hist_n = hn2;
        cs.hist_head = head2;
        cs.E = r.E;
        cs.noise = r.noise;
        cs.resid = r.resid;
        cs.iter += 1;
        cs.evals += evals_add;
        cs.halvings += hv;
        cs.degen = r.degen > 0.0;
        s_vol[j] = r.vol;
        s_area[j] = r.area;
        if (conv) { cs.status = NPFEM_CONVERGED; cs.active = 0; }
        else if (out_of_iters) { cs.status = NPFEM_MAXITER; cs.active = 0; }
      }
      if (conv || out_of_iters) { __syncthreads(); continue; }
      // q = g - sum_p alpha_p y_p (one pass)
#pragma unroll 2
      for (int e = W * tid(); e < len; e += W * kBlock) {
        const auto gv = vload(G, e);
        double qv[W];
#pragma unroll
        for (int w = 0; w < W; ++w) qv[w] = gv[w];
#pragma unroll
        for (int p = 0; p < H; ++p) {
          const auto yv = m > 0 ? vload(tl.vec(VS0 + m + slot2(p), j), e) : gv;
#pragma unroll
          for (int w = 0; w < W; ++w) qv[w] -= al_new[p] * (double)(p < hn2 ? yv[w] : Real(0));
        }
        typename Vec16<Real>::type o;
#pragma unroll
        for (int w = 0; w < W; ++w) o[w] = Real(qv[w]);
        vstore(Q, e, o);
      }
      __syncthreads();
    }
    __syncthreads();
  }

  // ---- velocity update and dissipation --------------------------------------------
  for (int j = 0; j < cnt; ++j) {
    stage_aos(xn, A.x + 3 * s_voff[j], n, np);
    vcopy(ut, tl.vec(VU, j), len);
    __syncthreads();
    double bc[2] = {s_vol[j], s_area[j]};
    auto cs = CS[j];
    finalize_cell(A, M, s_cell[j], s_voff[j], cs, xn, ut, red, bc);
    __syncthreads();
  }
}

#ifndef NPFEM_STEP_WAVES_PER_SIMD
#define NPFEM_STEP_WAVES_PER_SIMD 2
#endif
// H: compile-time bound on the L-BFGS history (the loops over pairs are unrolled to H);
// CSL: the tile's cell states live in LDS at byte offset A.cs_lds (else in the workspace);
// EXT: the optional terms of the objective are compiled in; LAY: the batch's vector
// layout (0: every mesh keeps the current cell's vectors in LDS, 1: some mesh keeps the
// gradient and b in the workspace, 2: some mesh keeps x_n and u there too).
template <typename Real, int H, bool CSL, bool EXT, int LAY>
__global__ void __launch_bounds__(kBlock, NPFEM_STEP_WAVES_PER_SIMD) step_kernel(StepArgs<Real> A) {
  extern __shared__ __align__(16) unsigned char lds[];
  double* red = reinterpret_cast<double*>(lds);
  int* sint = reinterpret_cast<int*>(lds + kRedDoubles * 8 + 32 * 8);
  Real* W = A.work + (size_t)blockIdx.x * A.slot_stride;
  CellStateT<H>* CS = CSL ? reinterpret_cast<CellStateT<H>*>(lds + A.cs_lds)
                          : reinterpret_cast<CellStateT<H>*>(A.cstate) + (size_t)blockIdx.x * A.tile_cells_max;
  for (;;) {
    if (tid() == 0) sint[0] = atomicAdd(A.tile_counter, 1);
    __syncthreads();
    const int tile = sint[0];
    __syncthreads();
    if (tile >= A.n_tiles) break;
    run_tile<Real, H, EXT, LAY>(A, tile, W, CS, red, sint, lds);
    __syncthreads();
  }
}

__global__ void reset_counter(int* c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0;
}

// One workgroup per cell: objective and gradient at x_n + u (no iteration).
template <typename Real, int LAY>
__global__ void __launch_bounds__(kBlock) eval_kernel(StepArgs<Real> A, const Real* u, Real* grad,
                                                      double* terms, Real* scratch) {
  extern __shared__ __align__(16) unsigned char lds[];
  double* red = reinterpret_cast<double*>(lds);
  const int cell = blockIdx.x;
  const MeshDev<Real>& M = A.meshes[A.cell_mesh[cell]];
  const int n = M.n, np = M.n_pad, len = 3 * np;
  const int64_t voff = A.cell_voff[cell];
  // per cell in the scratch: gradient, b, x_n, u (3 n_pad_max each), where not in LDS
  const bool vl = LAY == 0 || M.vec_lds != 0, xl = LAY < 2 || M.xu_lds != 0;
  Real* cs = scratch + (size_t)cell * 4 * 3 * A.n_pad_max;
  Real* xn = xl ? reinterpret_cast<Real*>(lds + kLdsHeader) : cs + 2 * 3 * A.n_pad_max;
  Real* ut = xl ? xn + 3 * np : cs + 3 * 3 * A.n_pad_max;
  Real* G = vl ? ut + 3 * np : cs;
  Real* B = vl ? G + 3 * np : cs + 3 * A.n_pad_max;
  Real* work = reinterpret_cast<Real*>(lds + kLdsHeader) + (xl ? (vl ? 12 : 6) * np : 0);
  stage_aos(xn, A.x + 3 * voff, n, np);
  const Real* vs = A.v + 3 * voff;
  const Real* fs = A.f + 3 * voff;
  aos_to_soa(B, n, np, [&](int e) { return gld(M.mass, e / 3) * vs[e] / Real(A.sol.h) + fs[e]; });
  __syncthreads();
  double Gn, GA;
  normalisers(M, xn, static_cast<const Real*>(nullptr), ut, A.mat.k_area_global > 0.0 ? G : static_cast<Real*>(nullptr),
              work, red, Gn, GA);
  __syncthreads();
  stage_aos(ut, u + 3 * voff, n, np);
  __syncthreads();
  EvalResult r;
  evaluate<Real, true>(M, A.mat, A.sol.literal != 0, A.sol.h, Gn, GA, Contacts<Real>{nullptr, nullptr, 0.0}, xn, ut, B, work, G,
           red, r);
  for (int e = tid(); e < 3 * n; e += kBlock) {
    const int i = e / 3, c = e - 3 * i;
    grad[3 * voff + e] = G[c * np + i];
  }
  if (tid() == 0) {
    double* o = terms + (size_t)kTerms * cell;
    o[0] = r.E;
    for (int k = 0; k < 6; ++k) o[1 + k] = r.terms[k];
    o[7] = r.resid;
    o[8] = r.terms[6];
    o[9] = r.area;
    o[10] = r.degen;
  }
}

template <typename Real>
__global__ void __launch_bounds__(kBlock) apply_inverse_kernel(const Real* A, int np, const Real* in,
                                                               Real* out, int rows) {
  const int r0 = blockIdx.x * 48;
  tile_gemm(A, np, in + (size_t)r0 * np, out + (size_t)r0 * np, min(48, rows - r0));
}

// 48 rows per workgroup, staged in LDS in chunks of kc columns (48 (kc + 8) BF16).
__global__ void __launch_bounds__(kBlock) apply_inverse_band_kernel(const uint16_t* A, const float* diag,
                                                                    const int* perm, const int* band, int np,
                                                                    const float* in, float* out, int rows, int kc) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int r0 = blockIdx.x * 48;
  tile_gemm_bf16_band(A, diag, perm, band, np, in + (size_t)r0 * np, out + (size_t)r0 * np, min(48, rows - r0),
                      reinterpret_cast<__bf16*>(lds), kc);
}

__global__ void __launch_bounds__(kBlock) apply_inverse_bf16_kernel(const uint16_t* A, const float* diag, int np,
                                                                    const float* in, float* out, int rows) {
  const int r0 = blockIdx.x * 48;
  tile_gemm_bf16(A, diag, np, in + (size_t)r0 * np, out + (size_t)r0 * np, min(48, rows - r0));
}

template <typename Real>
__global__ void drag_kernel(const Real* x, const Real* v, const int64_t* cell_voff, const int* cell_mesh,
                            const int* mesh_n, const double* zeta, const double* rate,
                            const double* origin, double umax, double radius, double ay, double az,
                            Real* f) {
  const int cell = blockIdx.x;
  const int n = mesh_n[cell_mesh[cell]];
  const int64_t voff = cell_voff[cell];
  const double z0 = zeta[cell], g = rate[cell];
  const double oy = origin[3 * cell + 1], oz = origin[3 * cell + 2];
  for (int i = tid(); i < n; i += blockDim.x) {
    const int64_t k = 3 * (voff + i);
    const double y = x[k + 1], z = x[k + 2];
    double ux = g * z;
    if (umax != 0.0) {
      const double wy = oy + y - ay, wz = oz + z - az;
      const double rho2 = wy * wy + wz * wz;
      if (rho2 < radius * radius) ux += umax * (1.0 - rho2 / (radius * radius));
    }
    f[k] = (Real)(z0 * (ux - (double)v[k]));
    f[k + 1] = (Real)(-z0 * (double)v[k + 1]);
    f[k + 2] = (Real)(-z0 * (double)v[k + 2]);
  }
}

// Totals of per-cell step results: per-thread sums over a strided range of cells, a
// workgroup reduction through LDS, then one set of device-scope atomics per workgroup
// (integer sums, so the result does not depend on the order).
__global__ void __launch_bounds__(kBlock) stats_accumulate_kernel(const npfem_cell_stats* st, int64_t n,
                                                                  npfem_stats_total* tot) {
  __shared__ long long s_sum[kBlock / 64][9];
  __shared__ int s_max[kBlock / 64], s_fb[kBlock / 64];
  __shared__ double s_res[kBlock / 64];
  long long v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};   // cells, iterations, evaluations, halvings, not converged, 4 status bits
  int mx = 0, fb = 0;
  double rmax = 0.0;
  for (int64_t c = (int64_t)blockIdx.x * kBlock + tid(); c < n; c += (int64_t)gridDim.x * kBlock) {
    const npfem_cell_stats a = st[c];
    v[0] += 1;
    v[1] += a.iterations;
    v[2] += a.evaluations;
    v[3] += a.halvings;
    v[4] += (a.status & NPFEM_CONVERGED) ? 0 : 1;
    v[5] += (a.status & NPFEM_MAXITER) ? 1 : 0;
    v[6] += (a.status & NPFEM_LS_FAIL) ? 1 : 0;
    v[7] += (a.status & NPFEM_NONFINITE) ? 1 : 0;
    v[8] += (a.status & NPFEM_DEGENERATE_TRI) ? 1 : 0;
    fb += (a.status & NPFEM_START_FALLBACK) ? 1 : 0;
    mx = max(mx, a.iterations);
    rmax = fmax(rmax, a.residual);
  }
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int k = 0; k < 9; ++k) v[k] += __shfl_xor(v[k], off);
    mx = max(mx, __shfl_xor(mx, off));
    fb += __shfl_xor(fb, off);
    rmax = fmax(rmax, __shfl_xor(rmax, off));
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 9; ++k) s_sum[wave][k] = v[k];
    s_max[wave] = mx;
    s_fb[wave] = fb;
    s_res[wave] = rmax;
  }
  __syncthreads();
  if (tid() == 0) {
    for (int w = 1; w < kBlock / 64; ++w) {
#pragma unroll
      for (int k = 0; k < 9; ++k) v[k] += s_sum[w][k];
      mx = max(mx, s_max[w]);
      fb += s_fb[w];
      rmax = fmax(rmax, s_res[w]);
    }
    unsigned long long* t = reinterpret_cast<unsigned long long*>(tot);
    atomicAdd(&t[0], (unsigned long long)v[0]);
    atomicAdd(&t[1], (unsigned long long)v[1]);
    atomicAdd(&t[2], (unsigned long long)v[2]);
    atomicAdd(&t[3], (unsigned long long)v[3]);
    atomicAdd(&t[4], (unsigned long long)v[4]);
    for (int k = 0; k < 4; ++k) atomicAdd(&t[5 + k], (unsigned long long)v[5 + k]);
    atomicMax(&tot->max_iterations, mx);
    atomicAdd(&tot->start_fallback, fb);
    // residuals are >= 0 (or +inf / NaN), so their bit patterns order like the values
    atomicMax(reinterpret_cast<unsigned long long*>(&tot->max_residual), (unsigned long long)__double_as_longlong(rmax));
  }
}

__global__ void stats_reset_kernel(npfem_stats_total* tot) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *tot = npfem_stats_total{};
}

}  // namespace

// The library builds this file as two objects, NPFEM_PART 1 (the FP32 instantiations and
// everything that is not a template) and NPFEM_PART 2 (the FP64 instantiations), so that
// they compile in parallel; without NPFEM_PART it holds both.
#if !defined(NPFEM_PART) || NPFEM_PART == 1
// Device scratch of the allocation-free step (npfem_step_noalloc): the tile counter,
// the cell states and the workspace of the persistent workgroups.  One copy per device,
// held until the process ends.  Host code never uses this name as an address: it takes
// the per-device address from scratch_address() and passes that to the kernels.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(void** ptr) { return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch)); }

hipError_t launch_stats_accumulate(const npfem_cell_stats* st, int64_t n, npfem_stats_total* tot, hipStream_t s) {
  (void)hipGetLastError();   // drop an error left behind by unrelated earlier calls
  const int64_t want = (n + kBlock - 1) / kBlock;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(want, 512));
  hipLaunchKernelGGL(stats_accumulate_kernel, dim3(grid), dim3(kBlock), 0, s, st, n, tot);
  return hipGetLastError();
}

hipError_t launch_stats_reset(npfem_stats_total* tot, hipStream_t s) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(stats_reset_kernel, dim3(1), dim3(64), 0, s, tot);
  return hipGetLastError();
}

// k columns of the BF16 tile product staged per chunk: what the LDS region of `lds`
// bytes holds for stage_rows rows (a multiple of 32, capped at n_pad; 0: not staged).
int stage_cols(size_t lds, int stage_rows, int n_pad) {
  if (stage_rows <= 0 || lds <= (size_t)kLdsHeader) return 0;
  const long kc = (long)((lds - kLdsHeader) / (2 * (size_t)stage_rows)) - 8;
  const long k32 = kc / 32 * 32;
  return (int)(k32 >= n_pad ? n_pad : (k32 >= 32 ? k32 : 0));
}
#endif

template <typename Real>
size_t lds_bytes(int n_pad, int chunk, int stage_rows, int vec_lds, int xu_lds) {
  // x_n, trial u (and, with vec_lds, the gradient and b), 3 n_pad each, unless they live
  // in the workspace, then the corner chunks (9 per triangle, at least 3 n_pad: the
  // bending pass keeps its residuals there)
  const size_t work = (size_t)(3 * n_pad > 9 * chunk ? 3 * n_pad : 9 * chunk);
  const size_t vecs = xu_lds ? (vec_lds ? 12 : 6) * (size_t)n_pad : 0;
  size_t region = sizeof(Real) * (vecs + work);
  if (stage_rows > 0 && n_pad <= kStageMaxPad) {
    const size_t st = (size_t)stage_rows * (n_pad + 8) * 2;
    region = region > st ? region : st;
  }
  return kLdsHeader + region;
}

// Layout 2 (x_n and u in the workspace) exists for FP64 plans only: FP32 plans of the
// supported meshes always keep them in LDS (the host refuses an FP32 mesh that would not).
template <typename Real> constexpr int kMaxLayout = std::is_same<Real, double>::value ? 2 : 1;

template <typename Real, int LAY>
void step_kernel_ptrs(std::vector<const void*>& out) {
  out.push_back(reinterpret_cast<const void*>(&step_kernel<Real, 2, false, false, LAY>));
  out.push_back(reinterpret_cast<const void*>(&step_kernel<Real, 5, false, false, LAY>));
  out.push_back(reinterpret_cast<const void*>(&step_kernel<Real, kMaxHistory, false, false, LAY>));
  out.push_back(reinterpret_cast<const void*>(&step_kernel<Real, 2, true, false, LAY>));
  out.push_back(reinterpret_cast<const void*>(&step_kernel<Real, 5, true, false, LAY>));
  out.push_back(reinterpret_cast<const void*>(&step_kernel<Real, kMaxHistory, true, false, LAY>));
  out.push_back(reinterpret_cast<const void*>(&step_kernel<Real, 2, false, true, LAY>));
  out.push_back(reinterpret_cast<const void*>(&step_kernel<Real, 5, false, true, LAY>));
  out.push_back(reinterpret_cast<const void*>(&step_kernel<Real, kMaxHistory, false, true, LAY>));
  out.push_back(reinterpret_cast<const void*>(&step_kernel<Real, 2, true, true, LAY>));
  out.push_back(reinterpret_cast<const void*>(&step_kernel<Real, 5, true, true, LAY>));
  out.push_back(reinterpret_cast<const void*>(&step_kernel<Real, kMaxHistory, true, true, LAY>));
  out.push_back(reinterpret_cast<const void*>(&eval_kernel<Real, LAY>));
}

template <typename Real>
hipError_t set_lds_limit(size_t bytes) {
  std::vector<const void*> fns;
  step_kernel_ptrs<Real, 0>(fns);
  step_kernel_ptrs<Real, 1>(fns);
  if constexpr (kMaxLayout<Real> >= 2) step_kernel_ptrs<Real, 2>(fns);
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename Real>
hipError_t occupancy(int* blocks_per_cu, size_t lds) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(
      blocks_per_cu, step_kernel<Real, kMaxHistory, false, true, kMaxLayout<Real>>, kBlock, lds);
}

template <typename Real, int H, bool EXT, int LAY>
void launch_step_h(const StepArgs<Real>& a, int grid, size_t lds, hipStream_t s) {
  if (a.cs_lds >= 0) hipLaunchKernelGGL((step_kernel<Real, H, true, EXT, LAY>), dim3(grid), dim3(kBlock), lds, s, a);
  else hipLaunchKernelGGL((step_kernel<Real, H, false, EXT, LAY>), dim3(grid), dim3(kBlock), lds, s, a);
}

template <typename Real, bool EXT, int LAY>
void launch_step_e(const StepArgs<Real>& a, int grid, size_t lds, hipStream_t s) {
  if (a.sol.m <= 2) launch_step_h<Real, 2, EXT, LAY>(a, grid, lds, s);
  else if (a.sol.m <= 5) launch_step_h<Real, 5, EXT, LAY>(a, grid, lds, s);
  else launch_step_h<Real, kMaxHistory, EXT, LAY>(a, grid, lds, s);
}

template <typename Real, int LAY>
void launch_step_x(const StepArgs<Real>& a, int grid, size_t lds, hipStream_t s) {
  // the optional terms' code only where they are used
  const bool ext = a.mat.k_area_global > 0.0 || a.sol.literal != 0 || a.col_n != nullptr;
  if (ext) launch_step_e<Real, true, LAY>(a, grid, lds, s);
  else launch_step_e<Real, false, LAY>(a, grid, lds, s);
}

template <typename Real>
hipError_t launch_step(const StepArgs<Real>& a, int grid, size_t lds, hipStream_t s, int* counter) {
  (void)hipGetLastError();   // drop an error left behind by unrelated earlier calls
  if (a.layout < 0 || a.layout > kMaxLayout<Real>) return hipErrorInvalidValue;
  hipLaunchKernelGGL(reset_counter, dim3(1), dim3(64), 0, s, counter);
  if (a.layout == 0) launch_step_x<Real, 0>(a, grid, lds, s);
  else if (a.layout == 1) launch_step_x<Real, 1>(a, grid, lds, s);
  else if constexpr (kMaxLayout<Real> >= 2) launch_step_x<Real, kMaxLayout<Real>>(a, grid, lds, s);
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_eval(const StepArgs<Real>& a, int n_cells, const Real* u, Real* grad, double* terms,
                       size_t lds, hipStream_t s) {
  (void)hipGetLastError();   // drop an error left behind by unrelated earlier calls
  if (a.layout < 0 || a.layout > kMaxLayout<Real>) return hipErrorInvalidValue;
  if (a.layout == 0)
    hipLaunchKernelGGL((eval_kernel<Real, 0>), dim3(n_cells), dim3(kBlock), lds, s, a, u, grad, terms, a.work);
  else if (a.layout == 1)
    hipLaunchKernelGGL((eval_kernel<Real, 1>), dim3(n_cells), dim3(kBlock), lds, s, a, u, grad, terms, a.work);
  else if constexpr (kMaxLayout<Real> >= 2)
    hipLaunchKernelGGL((eval_kernel<Real, kMaxLayout<Real>>), dim3(n_cells), dim3(kBlock), lds, s, a, u, grad, terms, a.work);
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_apply_inverse(const Real* A, int n_pad, const Real* in, Real* out, int rows,
                                hipStream_t s) {
  (void)hipGetLastError();   // drop an error left behind by unrelated earlier calls
  hipLaunchKernelGGL(apply_inverse_kernel<Real>, dim3((rows + 47) / 48), dim3(kBlock), 0, s, A, n_pad,
                     in, out, rows);
  return hipGetLastError();
}

#if !defined(NPFEM_PART) || NPFEM_PART == 1
hipError_t launch_apply_inverse_band(const uint16_t* A, const float* diag, const int* perm, const int* band,
                                     int n_pad, const float* in, float* out, int rows, hipStream_t s) {
  (void)hipGetLastError();   // drop an error left behind by unrelated earlier calls
  const int kc = std::min(n_pad, (65536 / (2 * 48) - 8) / 32 * 32);
  const size_t lds = (size_t)48 * (kc + 8) * 2;
  hipLaunchKernelGGL(apply_inverse_band_kernel, dim3((rows + 47) / 48), dim3(kBlock), lds, s, A, diag, perm, band,
                     n_pad, in, out, rows, kc);
  return hipGetLastError();
}

hipError_t launch_apply_inverse_bf16(const uint16_t* A, const float* diag, int n_pad, const float* in,
                                     float* out, int rows, hipStream_t s) {
  (void)hipGetLastError();   // drop an error left behind by unrelated earlier calls
  hipLaunchKernelGGL(apply_inverse_bf16_kernel, dim3((rows + 47) / 48), dim3(kBlock), 0, s, A, diag, n_pad, in,
                     out, rows);
  return hipGetLastError();
}
#endif

template <typename Real>
hipError_t launch_drag(const Real* x, const Real* v, const int64_t* cell_voff, const int* cell_mesh,
                       const int* mesh_n, int n_cells, const double* zeta, const double* rate,
                       const double* origin, double umax, double radius, double ay, double az, Real* f,
                       hipStream_t s) {
  (void)hipGetLastError();   // drop an error left behind by unrelated earlier calls
  hipLaunchKernelGGL(drag_kernel<Real>, dim3(n_cells), dim3(kBlock), 0, s, x, v, cell_voff, cell_mesh,
                     mesh_n, zeta, rate, origin, umax, radius, ay, az, f);
  return hipGetLastError();
}

#define NPFEM_INSTANTIATE(R)                                                                       \
  template size_t lds_bytes<R>(int, int, int, int, int);                                                     \
  template hipError_t set_lds_limit<R>(size_t);                                                    \
  template hipError_t occupancy<R>(int*, size_t);                                                  \
  template hipError_t launch_step<R>(const StepArgs<R>&, int, size_t, hipStream_t, int*);          \
  template hipError_t launch_eval<R>(const StepArgs<R>&, int, const R*, R*, double*, size_t,       \
                                     hipStream_t);                                                 \
  template hipError_t launch_apply_inverse<R>(const R*, int, const R*, R*, int, hipStream_t);      \
  template hipError_t launch_drag<R>(const R*, const R*, const int64_t*, const int*, const int*,   \
                                     int, const double*, const double*, const double*, double,     \
                                     double, double, double, R*, hipStream_t);
#if !defined(NPFEM_PART) || NPFEM_PART == 1
NPFEM_INSTANTIATE(float)
#endif
#if !defined(NPFEM_PART) || NPFEM_PART == 2
NPFEM_INSTANTIATE(double)
#endif

}  // namespace npfem
