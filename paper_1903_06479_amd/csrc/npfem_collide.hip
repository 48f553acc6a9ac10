// Contact search between cells for the collision term (section 4.7 of the paper).
//
// The paper finds, for every vertex, the neighbouring vertices of other cells through
// the fluid lattice and a k-d tree, and gives a colliding vertex a desired position from
// its neighbours and their normals.  Here the search is a uniform grid of cell size
// equal to the cutoff, hashed into a table and filled by a counting sort (per-bucket
// counts by atomics, an exclusive scan, a scatter); each vertex then scans the 27 grid
// cells around it for the nearest vertex of another cell.  The partner's position in the
// vertex's own cell frame and the partner's unit area-weighted normal are written for
// the step, which adds (w/2) min((x - q) . n, 0)^2 per vertex.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "npfem_internal.h"

namespace npfem {

namespace {

constexpr int kCB = 256;            // threads per workgroup
constexpr int kScanPerThread = 16;  // table entries per thread in the scan
constexpr int kScanBlock = kCB * kScanPerThread;

__device__ inline unsigned grid_hash(int ix, int iy, int iz, unsigned mask) {
  return ((unsigned)ix * 73856093u ^ (unsigned)iy * 19349663u ^ (unsigned)iz * 83492791u) & mask;
}

// Unit area-weighted vertex normals of every cell at x (FP64), one workgroup per cell:
// each vertex sums (x_b - x_a) x (x_c - x_a) over its incident triangles.
template <typename Real>
__global__ void __launch_bounds__(kCB) vertex_normals_kernel(CollideArgs<Real> A) {
  const int cell = blockIdx.x;
  const MeshDev<Real>& M = A.meshes[A.cell_mesh[cell]];
  const int64_t voff = A.cell_voff[cell];
  const Real* x = A.x + 3 * voff;
  for (int i = threadIdx.x; i < M.n; i += kCB) {
    double sx = 0, sy = 0, sz = 0;
    for (int q = 0; q < M.vc_deg; ++q) {
      const int cid = M.vc_ell[q * M.n_pad + i];
      if (cid < 0) continue;
      const int t = cid / 3;
      const int a = M.tri[3 * t], b = M.tri[3 * t + 1], c = M.tri[3 * t + 2];
      const double ux = (double)x[3 * b] - x[3 * a], uy = (double)x[3 * b + 1] - x[3 * a + 1], uz = (double)x[3 * b + 2] - x[3 * a + 2];
      const double vx = (double)x[3 * c] - x[3 * a], vy = (double)x[3 * c + 1] - x[3 * a + 1], vz = (double)x[3 * c + 2] - x[3 * a + 2];
      sx += uy * vz - uz * vy;
      sy += uz * vx - ux * vz;
      sz += ux * vy - uy * vx;
    }
    const double ln = sqrt(sx * sx + sy * sy + sz * sz);
    const double s = ln > 0 ? 1.0 / ln : 0.0;
    double* o = A.normals + 3 * (voff + i);
    o[0] = sx * s;
    o[1] = sy * s;
    o[2] = sz * s;
  }
}

// Grid keys of every vertex (world position origin + x), the vertex's cell, and the
// per-bucket counts.
template <typename Real>
__global__ void __launch_bounds__(kCB) grid_keys_kernel(CollideArgs<Real> A) {
  const int cell = blockIdx.x;
  const int n = A.mesh_n[A.cell_mesh[cell]];
  const int64_t voff = A.cell_voff[cell];
  const double ox = A.origin[3 * cell], oy = A.origin[3 * cell + 1], oz = A.origin[3 * cell + 2];
  for (int i = threadIdx.x; i < n; i += kCB) {
    const int64_t v = voff + i;
    const double px = ox + (double)A.x[3 * v], py = oy + (double)A.x[3 * v + 1], pz = oz + (double)A.x[3 * v + 2];
    const unsigned key = grid_hash((int)floor(px * A.inv_h), (int)floor(py * A.inv_h), (int)floor(pz * A.inv_h), A.mask);
    A.vkey[v] = key;
    A.vcell[v] = cell;
    atomicAdd(&A.count[key], 1u);
  }
}

__global__ void __launch_bounds__(kCB) fill_zero_u32_kernel(unsigned* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kCB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kCB) p[i] = 0u;
}

// Exclusive scan of the bucket counts in three passes: block sums, a scan of the block
// sums by one workgroup, then each block's scan plus its offset.
__device__ inline unsigned block_exclusive_scan(unsigned v, unsigned* sh, unsigned* total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kCB; off <<= 1) {
    const unsigned a = t >= off ? sh[t - off] : 0u;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  const unsigned incl = sh[t];
  if (total) *total = sh[kCB - 1];
  __syncthreads();
  return incl - v;
}

__global__ void __launch_bounds__(kCB) scan_block_sums_kernel(const unsigned* in, int64_t n, unsigned* bsum) {
  __shared__ unsigned sh[kCB];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPerThread;
  unsigned s = 0;
  for (int k = 0; k < kScanPerThread; ++k)
    if (base + k < n) s += in[base + k];
  unsigned tot;
  block_exclusive_scan(s, sh, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kCB) scan_sums_kernel(unsigned* bsum, int nb) {
  __shared__ unsigned sh[kCB];
  unsigned carry = 0;
  for (int b0 = 0; b0 < nb; b0 += kCB) {
    const int i = b0 + threadIdx.x;
    const unsigned v = i < nb ? bsum[i] : 0u;
    unsigned tot;
    const unsigned ex = block_exclusive_scan(v, sh, &tot);
    if (i < nb) bsum[i] = carry + ex;
    carry += tot;
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kCB) scan_apply_kernel(const unsigned* in, int64_t n, const unsigned* bsum,
                                                         unsigned* out) {
  __shared__ unsigned sh[kCB];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPerThread;
  unsigned s = 0;
  for (int k = 0; k < kScanPerThread; ++k)
    if (base + k < n) s += in[base + k];
  unsigned run = bsum[blockIdx.x] + block_exclusive_scan(s, sh, nullptr);
  for (int k = 0; k < kScanPerThread; ++k)
    if (base + k < n) {
      out[base + k] = run;
      run += in[base + k];
    }
}

// Scatter every vertex into its bucket's range (the order within a bucket does not
// matter: the search below keeps the lexicographically smallest (distance, index)).
__global__ void __launch_bounds__(kCB) grid_fill_kernel(const unsigned* vkey, int64_t nv, const unsigned* start,
                                                        unsigned* fill, unsigned* sorted) {
  for (int64_t v = (int64_t)blockIdx.x * kCB + threadIdx.x; v < nv; v += (int64_t)gridDim.x * kCB) {
    const unsigned key = vkey[v];
    const unsigned pos = start[key] + atomicAdd(&fill[key], 1u);
    sorted[pos] = (unsigned)v;
  }
}

// Nearest vertex of another cell within the cutoff: its position in the cell frame of
// the searching vertex and its normal, or zeros.
template <typename Real>
__global__ void __launch_bounds__(kCB) contact_kernel(CollideArgs<Real> A) {
  const int cell = blockIdx.x;
  const int n = A.mesh_n[A.cell_mesh[cell]];
  const int64_t voff = A.cell_voff[cell];
  const double ox = A.origin[3 * cell], oy = A.origin[3 * cell + 1], oz = A.origin[3 * cell + 2];
  const double c2 = A.cutoff * A.cutoff;
  for (int i = threadIdx.x; i < n; i += kCB) {
    const int64_t v = voff + i;
    const double px = ox + (double)A.x[3 * v], py = oy + (double)A.x[3 * v + 1], pz = oz + (double)A.x[3 * v + 2];
    const int ix = (int)floor(px * A.inv_h), iy = (int)floor(py * A.inv_h), iz = (int)floor(pz * A.inv_h);
    double best = c2;
    int64_t bj = -1;
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const unsigned key = grid_hash(ix + dx, iy + dy, iz + dz, A.mask);
          const unsigned s0 = A.start[key], s1 = s0 + A.count[key];
          for (unsigned e = s0; e < s1; ++e) {
            const int64_t j = A.sorted[e];
            const int cj = A.vcell[j];
            if (cj == cell) continue;
            const double jx = A.origin[3 * cj] + (double)A.x[3 * j];
            const double jy = A.origin[3 * cj + 1] + (double)A.x[3 * j + 1];
            const double jz = A.origin[3 * cj + 2] + (double)A.x[3 * j + 2];
            const double ex = jx - px, ey = jy - py, ez = jz - pz;
            const double d2 = ex * ex + ey * ey + ez * ez;
            if (d2 < best || (d2 == best && bj >= 0 && j < bj)) {
              best = d2;
              bj = j;
            }
          }
        }
    Real* q = A.q + 3 * v;
    Real* nn = A.n + 3 * v;
    if (bj >= 0) {
      const int cj = A.vcell[bj];
      q[0] = (Real)((A.origin[3 * cj] - ox) + (double)A.x[3 * bj]);
      q[1] = (Real)((A.origin[3 * cj + 1] - oy) + (double)A.x[3 * bj + 1]);
      q[2] = (Real)((A.origin[3 * cj + 2] - oz) + (double)A.x[3 * bj + 2]);
      nn[0] = (Real)A.normals[3 * bj];
      nn[1] = (Real)A.normals[3 * bj + 1];
      nn[2] = (Real)A.normals[3 * bj + 2];
      atomicAdd(A.n_contacts, 1ull);
    } else {
      q[0] = q[1] = q[2] = Real(0);
      nn[0] = nn[1] = nn[2] = Real(0);
    }
  }
}

}  // namespace

template <typename Real>
hipError_t launch_collide(const CollideArgs<Real>& a, int n_cells, int64_t n_vert, hipStream_t s) {
  (void)hipGetLastError();   // drop an error left behind by unrelated earlier calls
  const int64_t table = (int64_t)a.mask + 1;
  const int zg = (int)std::min<int64_t>((table + kCB - 1) / kCB, 4096);
  hipLaunchKernelGGL(fill_zero_u32_kernel, dim3(zg), dim3(kCB), 0, s, a.count, table);
  hipLaunchKernelGGL(fill_zero_u32_kernel, dim3(zg), dim3(kCB), 0, s, a.fill, table);
  hipLaunchKernelGGL(fill_zero_u32_kernel, dim3(1), dim3(kCB), 0, s, reinterpret_cast<unsigned*>(a.n_contacts), (int64_t)2);
  hipLaunchKernelGGL((vertex_normals_kernel<Real>), dim3(n_cells), dim3(kCB), 0, s, a);
  hipLaunchKernelGGL((grid_keys_kernel<Real>), dim3(n_cells), dim3(kCB), 0, s, a);
  const int nb = (int)((table + kScanBlock - 1) / kScanBlock);
  hipLaunchKernelGGL(scan_block_sums_kernel, dim3(nb), dim3(kCB), 0, s, a.count, table, a.bsum);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(kCB), 0, s, a.bsum, nb);
  hipLaunchKernelGGL(scan_apply_kernel, dim3(nb), dim3(kCB), 0, s, a.count, table, a.bsum, a.start);
  const int vg = (int)std::min<int64_t>((n_vert + kCB - 1) / kCB, 8192);
  hipLaunchKernelGGL(grid_fill_kernel, dim3(vg), dim3(kCB), 0, s, a.vkey, n_vert, a.start, a.fill, a.sorted);
  hipLaunchKernelGGL((contact_kernel<Real>), dim3(n_cells), dim3(kCB), 0, s, a);
  return hipGetLastError();
}

int collide_scan_blocks(int64_t table) { return (int)((table + kScanBlock - 1) / kScanBlock); }

template hipError_t launch_collide<float>(const CollideArgs<float>&, int, int64_t, hipStream_t);
template hipError_t launch_collide<double>(const CollideArgs<double>&, int, int64_t, hipStream_t);

}  // namespace npfem
