// Internal structures shared by the host library and the gfx950 kernels.
#pragma once

#include <cstdint>

#include "npfem.h"

namespace npfem {

constexpr int kBlock = 256;        // threads per workgroup (4 wave64)
constexpr int kMaxHistory = 8;     // L-BFGS pairs
constexpr int kMaxTile = 21;       // cells per tile: 3*21 = 63 rows <= 4 MFMA row blocks
constexpr int kTerms = 11;         // objective terms reported by npfem_eval

// Rest data of one mesh type on the device (precision Real).
template <typename Real>
struct MeshDev {
  int n, nt, n_pad;            // vertices, triangles, n rounded up to 32
  int chunk;                   // triangles per LDS corner chunk
  int vec_lds;                 // 1: the current cell's gradient and b live in LDS (else in the workspace)
  int xu_lds;                  // 1: the current cell's x_n and trial u live in LDS (else in the
                               //    workspace, after the per-cell vectors; implies vec_lds = 0)
  const int* tri;              // [nt][3]
  const double* dminv;         // [nt][4] D_m^-1 row-major (FP64 in every precision: the
  const double* area;          // [nt] rest area            triangle geometry is formed in FP64)
  const double* inv4a2;        // [nt] 1 / (2 A_t)^2
  const int* vc_ptr;           // [n+1] vertex -> incident corners (tri*3 + k), by triangle
  const int* vc_idx;
  const int* nb_ptr;           // [n+1] vertex -> neighbours
  const int* nb_idx;
  const Real* nb_w;            // cotangent weight (cot a + cot b)/2 of each neighbour edge
  int nb_deg, vc_deg;          // padded widths of the ELL lists below (max degree / valence)
  const int* nb_ell;           // [nb_deg][n_pad] neighbour of vertex i (i itself as padding)
  const Real* nbw_ell;         // [nb_deg][n_pad] its cotangent weight (0 as padding)
  const int* vc_ell;           // [vc_deg][n_pad] incident corner 3t + k (-1 as padding)
  const Real* vor_area;        // [n] mixed Voronoi area A_i
  const Real* ell0;            // [n] |l0_i|
  const Real* mass;            // [n]
  const Real* hinv;            // [n_pad][n_pad] H~^-1
  const Real* minv;            // [n_pad][n_pad] h^2 M~^-1
  const uint16_t* hinv_bf;     // [n_pad][n_pad] off-diagonal part of H~^-1, BF16 bits (or null)
  const uint16_t* minv_bf;     // [n_pad][n_pad] off-diagonal part of h^2 M~^-1, BF16 bits
  const float* hinv_diag;      // [n_pad] diagonal of H~^-1
  const float* minv_diag;      // [n_pad] diagonal of h^2 M~^-1
  // staged BF16 products: hinv_bf / minv_bf hold, in row n' and column k',
  // A[perm[n']][perm[k']] within the band of n''s 16-column block, 0 outside (inverse_bf16
  // = 2: a reverse Cuthill-McKee order and the significant entries' range; 1: the
  // identity and the whole range)
  const int* bperm;            // [n_pad] vertex at position k' of the order (identity on padding);
                               // null for the identity order
  const int* bband;            // [2][n_pad / 16][2] per matrix (H~^-1, h^2 M~^-1) and 16-column block:
                               // k' range [lo, hi), multiples of 32
  double V0;                   // rest volume
  double A0;                   // rest area
  double floor_force;          // B sqrt(A0): force floor of the residual
};

struct MaterialDev {
  double B, C, D, k_bend, k_volume, beta, kappa, k_area_global;
};

struct SolverDev {
  double h, tol, c1, noise;    // noise = noise_factor * machine epsilon
  int m, max_iter, max_halvings;
  int bf16;                    // products with the inverses on the BF16 matrix cores (2: banded)
  int literal;                 // volume normaliser at the current x (else frozen at x_n)
};

// Per-cell scalar state of the step for a history of at most H pairs (the arrays are
// indexed by history slot < m <= H).  The step kernel keeps a tile's states in LDS when
// that costs no workgroups per CU, else in the workspace.
template <int H>
struct CellStateT {
  double E;                    // objective at the current iterate
  double noise;                // sum of |terms| of E (line-search rounding scale)
  double Gn;                   // |grad V(x_n)|^2
  double GA;                   // |grad A(x_n)|^2 (global-area term)
  double resid;
  double rho[H];
  double alpha[H];
  double SY[H][H];             // s_i . y_j over the history slots
  int hist_n, hist_head, iter, evals, status, active, retry, halvings;
  int degen;                   // the current iterate has a collapsed triangle
  int fallback;                // the learned start raised the objective: started from y_n
};
using CellState = CellStateT<kMaxHistory>;

// History bound of the step kernel variant that runs a history of m pairs.
inline int history_bound(int m) { return m <= 2 ? 2 : (m <= 5 ? 5 : kMaxHistory); }
inline size_t cell_state_bytes(int m) {
  const int H = history_bound(m);
  return H == 2 ? sizeof(CellStateT<2>) : (H == 5 ? sizeof(CellStateT<5>) : sizeof(CellStateT<kMaxHistory>));
}

struct TileDesc {
  int mesh;                    // mesh type
  int count;                   // cells in this tile (<= cells_per_tile)
  int first;                   // index into the tile_cells list
  int pad;
};

template <typename Real>
struct StepArgs {
  const MeshDev<Real>* meshes; // [n_meshes] (device)
  MaterialDev mat;
  SolverDev sol;
  const TileDesc* tiles;       // [n_tiles]
  const int* tile_cells;       // cell ids, tiles[t].first .. first + count
  const int64_t* cell_voff;    // [n_cells] first vertex of each cell
  const int* cell_mesh;        // [n_cells]
  int n_tiles, tile_cells_max; // cells_per_tile
  int* tile_counter;           // work queue head
  int n_vec_slot;              // vectors per workspace slot
  int64_t slot_stride;         // Reals per slot
  Real* work;                  // [slots][n_vec_slot][T][3][n_pad_max]
  CellState* cstate;           // [slots][T] (read as CellStateT<H>) when cs_lds < 0
  int cs_lds;                  // byte offset of the tile's cell states in LDS, or -1
  int n_pad_max;
  int layout;                  // largest over the batch's meshes: 0 current cell's vectors in LDS,
                               // 1 gradient and b in the workspace, 2 x_n and u there too
  int stage_k;                 // k columns per LDS chunk of the BF16 tile product (0: unstaged)
  const Real* x;               // [V][3]
  const Real* v;
  const Real* f;
  const Real* u_guess;         // nullable: start from x_n + u_guess instead of the first guess
  const Real* u_delta;         // nullable: start from the first guess + u_delta (learned correction)
  const Real* col_q;           // nullable: [V][3] contact partner of each vertex (cell frame)
  const Real* col_n;           //           [V][3] its normal (zero: no contact)
  double w_col;                //           weight of the collision term
  int guess_only;              // write the first guess y_n - x_n to x_out and stop
  Real* x_out;
  Real* v_out;
  npfem_cell_stats* stats;     // nullable
};

// Contact search between cells (npfem_collide.hip).
template <typename Real>
struct CollideArgs {
  const MeshDev<Real>* meshes;
  const int64_t* cell_voff;
  const int* cell_mesh;
  const int* mesh_n;
  const double* origin;        // [n_cells][3] world origin of each cell
  const Real* x;               // [V][3] cell-local positions
  double cutoff, inv_h;        // contact distance; 1 / grid cell size (= 1 / cutoff)
  unsigned mask;               // hash table size - 1 (a power of two)
  unsigned* count;             // [table] vertices per bucket
  unsigned* start;             // [table] first slot of each bucket
  unsigned* fill;              // [table] slots filled so far
  unsigned* bsum;              // [scan blocks] block sums of the scan
  unsigned* vkey;              // [V] bucket of each vertex
  int* vcell;                  // [V] cell of each vertex
  unsigned* sorted;            // [V] vertices ordered by bucket
  double* normals;             // [V][3] unit area-weighted vertex normals
  Real* q;                     // [V][3] out: partner position in the vertex's cell frame
  Real* n;                     // [V][3] out: partner normal (zero: no contact)
  unsigned long long* n_contacts;  // out: number of vertices with a contact
};
template <typename Real>
hipError_t launch_collide(const CollideArgs<Real>& a, int n_cells, int64_t n_vert, hipStream_t s);
int collide_scan_blocks(int64_t table);

// Launch wrappers (npfem_kernels.hip).
template <typename Real>
hipError_t launch_step(const StepArgs<Real>& a, int grid, size_t lds, hipStream_t s, int* counter);
template <typename Real>
hipError_t launch_eval(const StepArgs<Real>& a, int n_cells, const Real* u, Real* grad,
                       double* terms, size_t lds, hipStream_t s);
template <typename Real>
hipError_t launch_apply_inverse(const Real* A, int n_pad, const Real* in, Real* out, int rows,
                                hipStream_t s);
hipError_t launch_apply_inverse_band(const uint16_t* A, const float* diag, const int* perm, const int* band,
                                     int n_pad, const float* in, float* out, int rows, hipStream_t s);
hipError_t launch_apply_inverse_bf16(const uint16_t* A, const float* diag, int n_pad, const float* in,
                                     float* out, int rows, hipStream_t s);
template <typename Real>
hipError_t launch_drag(const Real* x, const Real* v, const int64_t* cell_voff, const int* cell_mesh,
                       const int* mesh_n, int n_cells, const double* zeta, const double* rate,
                       const double* origin, double umax, double radius, double ay, double az,
                       Real* f, hipStream_t s);
// Allocation-free step: size of the per-device scratch array and its device address
// (the address must be looked up with the device current).
constexpr size_t kScratchBytes = size_t(64) << 20;
hipError_t scratch_address(void** ptr);
hipError_t launch_stats_accumulate(const npfem_cell_stats* st, int64_t n, npfem_stats_total* tot, hipStream_t s);
hipError_t launch_stats_reset(npfem_stats_total* tot, hipStream_t s);
// LDS of the step kernel; stage_rows > 0: rows of the BF16 tile product staged in LDS;
// xu_lds: x_n and the trial u of the current cell are kept in LDS; vec_lds: so are its
// gradient and b.
template <typename Real>
size_t lds_bytes(int n_pad, int chunk, int stage_rows, int vec_lds, int xu_lds);
int stage_cols(size_t lds, int stage_rows, int n_pad);
template <typename Real>
hipError_t set_lds_limit(size_t bytes);
template <typename Real>
hipError_t occupancy(int* blocks_per_cu, size_t lds);

}  // namespace npfem
