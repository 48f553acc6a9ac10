// Host side of the npFEM library: argument checking, FP64 rest data and constant
// matrices, the batch schedule, and the C ABI declared in include/npfem.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "npfem.h"
#include "npfem_factor.h"
#include "npfem_internal.h"
#include "npfem_net_internal.h"

using namespace npfem;

namespace {

// LDS a step workgroup may use (the CU's 160 KB less the kernel's static arrays and a
// margin).
constexpr size_t kStepLdsCap = 160 * 1024 - 1024;

thread_local std::string g_err;

npfem_status fail(npfem_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(e_ == hipErrorOutOfMemory ? NPFEM_E_OOM : NPFEM_E_HIP,                \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                   \
  } while (0)

struct V3 {
  double x, y, z;
};
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline double norm(V3 a) { return std::sqrt(dot(a, a)); }

// Run f(i) for i in [0, n) on the host cores.
template <typename F>
void parallel_for(int n, F f) {
  int nt = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 64) nt = 1;
  std::vector<std::thread> th;
  for (int w = 0; w < nt; ++w)
    th.emplace_back([&, w] {
      for (int i = w; i < n; i += nt) f(i);
    });
  for (auto& t : th) t.join();
}

// In-place lower Cholesky of a dense SPD matrix (row-major); false if not SPD.
bool cholesky(std::vector<double>& A, int n) {
  for (int j = 0; j < n; ++j) {
    double* rj = &A[(size_t)j * n];
    double s = rj[j];
    for (int k = 0; k < j; ++k) s -= rj[k] * rj[k];
    if (!(s > 0.0) || !std::isfinite(s)) return false;
    const double d = std::sqrt(s);
    rj[j] = d;
    const int rem = n - j - 1;
    parallel_for(rem, [&](int q) {
      const int i = j + 1 + q;
      double* ri = &A[(size_t)i * n];
      double t = ri[j];
      for (int k = 0; k < j; ++k) t -= ri[k] * rj[k];
      ri[j] = t / d;
    });
  }
  return true;
}

// Inverse of an SPD matrix from its Cholesky factor L (lower, row-major):
// A^-1 = L^-T L^-1.  W^T (row j = column j of L^-1) is built by forward substitution.
std::vector<double> spd_inverse(const std::vector<double>& L, int n) {
  std::vector<double> WT((size_t)n * n, 0.0);
  parallel_for(n, [&](int j) {
    double* w = &WT[(size_t)j * n];
    w[j] = 1.0 / L[(size_t)j * n + j];
    for (int i = j + 1; i < n; ++i) {
      const double* li = &L[(size_t)i * n];
      double s = 0.0;
      for (int k = j; k < i; ++k) s += li[k] * w[k];
      w[i] = -s / li[i];
    }
  });
  std::vector<double> inv((size_t)n * n, 0.0);
  parallel_for(n, [&](int a) {
    const double* wa = &WT[(size_t)a * n];
    for (int b = a; b < n; ++b) {
      const double* wb = &WT[(size_t)b * n];
      double s = 0.0;
      for (int k = b; k < n; ++k) s += wa[k] * wb[k];
      inv[(size_t)a * n + b] = s;
    }
  });
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < a; ++b) inv[(size_t)a * n + b] = inv[(size_t)b * n + a];
  return inv;
}

int round_up(int v, int m) { return (v + m - 1) / m * m; }

// Per-device address of the allocation-free step's scratch array, looked up once per
// device (with that device current) when the first plan on it is created.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

npfem_status init_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(NPFEM_E_UNSUPPORTED, "scratch: device index too large");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return NPFEM_OK;
  void* ptr = nullptr;
  HIP_TRY(scratch_address(&ptr));
  if (!ptr) return fail(NPFEM_E_HIP, "scratch: hipGetSymbolAddress returned NULL");
  g_scratch_ptr[device] = ptr;
  return NPFEM_OK;
}

void* scratch_of(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return device >= 0 && device < kMaxDevices ? g_scratch_ptr[device] : nullptr;
}

// FP32 -> BF16 bits, round to nearest even (finite inputs).
uint16_t to_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

}  // namespace

// ---------------------------------------------------------------------------------
// Mesh
// ---------------------------------------------------------------------------------
struct npfem_mesh {
  int n = 0, nt = 0, ne = 0;
  std::vector<double> X;          // [n][3]
  std::vector<int> tri;           // [nt][3]
  std::vector<double> dminv;      // [nt][4]
  std::vector<double> area;       // [nt]
  std::vector<int> vc_ptr, vc_idx;
  std::vector<int> nb_ptr, nb_idx;
  std::vector<double> nb_w;       // (cot a + cot b) / 2
  std::vector<double> vor_area, ell0, bary_area;
  double V0 = 0.0, A0 = 0.0;
};

extern "C" {

const char* npfem_status_string(npfem_status s) {
  switch (s) {
    case NPFEM_OK: return "ok";
    case NPFEM_E_INVALID: return "invalid argument";
    case NPFEM_E_MESH: return "invalid mesh";
    case NPFEM_E_NOT_SPD: return "matrix not symmetric positive definite";
    case NPFEM_E_HIP: return "HIP runtime error";
    case NPFEM_E_OOM: return "out of memory";
    case NPFEM_E_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* npfem_last_error(void) { return g_err.c_str(); }

void npfem_material_default(npfem_material* m) {
  if (!m) return;
  m->B = 10.6;
  m->C = 530.0;
  m->D = 35.0;
  m->k_bend = 0.2;
  m->k_volume = 250.0;
  m->beta = 0.01;
  m->kappa = 0.6;
  m->density = 1100.0;
  m->k_mat = -1.0;
  m->k_area_global = 0.0;
}

void npfem_solver_params_default(npfem_solver_params* p) {
  if (!p) return;
  p->precision = NPFEM_FP32;
  p->lbfgs_m = 5;
  p->max_iter = 200;
  p->max_halvings = 30;
  p->tol = 1e-6;
  p->c1 = 1e-4;
  p->noise_factor = 8.0;
  p->cells_per_tile = 0;
  p->grid_blocks = 0;
  p->inverse_bf16 = 0;
  p->volume_normaliser = NPFEM_VOLUME_STEP_FROZEN;
}

npfem_status npfem_mesh_create(int32_t n, const double* xyz, int32_t nt, const int32_t* tris,
                               npfem_mesh** out) {
  if (!out || !xyz || !tris) return fail(NPFEM_E_INVALID, "mesh_create: NULL pointer");
  *out = nullptr;
  if (n < 4 || nt < 4) return fail(NPFEM_E_MESH, "mesh_create: need at least 4 vertices and 4 triangles");
  auto m = std::make_unique<npfem_mesh>();
  m->n = n;
  m->nt = nt;
  m->X.assign(xyz, xyz + 3 * (size_t)n);
  m->tri.assign(tris, tris + 3 * (size_t)nt);
  for (double v : m->X)
    if (!std::isfinite(v)) return fail(NPFEM_E_MESH, "mesh_create: non-finite vertex coordinate");
  // closed, consistently oriented: every directed edge once, its reverse once
  std::unordered_map<int64_t, int> dir;
  dir.reserve(3 * (size_t)nt);
  for (int t = 0; t < nt; ++t) {
    const int* f = &m->tri[3 * t];
    for (int k = 0; k < 3; ++k) {
      if (f[k] < 0 || f[k] >= n) return fail(NPFEM_E_MESH, "mesh_create: vertex index out of range");
    }
    if (f[0] == f[1] || f[1] == f[2] || f[0] == f[2])
      return fail(NPFEM_E_MESH, "mesh_create: triangle with a repeated vertex");
    for (int k = 0; k < 3; ++k) {
      const int64_t key = (int64_t)f[k] * n + f[(k + 1) % 3];
      if (dir.count(key)) return fail(NPFEM_E_MESH, "mesh_create: directed edge used twice (non-manifold or inconsistent orientation)");
      dir[key] = t;
    }
  }
  for (const auto& kv : dir) {
    const int64_t a = kv.first / n, b = kv.first % n;
    if (!dir.count(b * n + a)) return fail(NPFEM_E_MESH, "mesh_create: open boundary edge");
  }
  m->ne = (int)(dir.size() / 2);
  auto P = [&](int i) { return V3{m->X[3 * i], m->X[3 * i + 1], m->X[3 * i + 2]}; };

  // per-triangle rest data in the triangle's own 2D frame, third vertex as reference
  m->dminv.resize(4 * (size_t)nt);
  m->area.resize(nt);
  double vol6 = 0.0;
  for (int t = 0; t < nt; ++t) {
    const V3 Xa = P(m->tri[3 * t]), Xb = P(m->tri[3 * t + 1]), Xc = P(m->tri[3 * t + 2]);
    const V3 E1 = sub(Xa, Xc), E2 = sub(Xb, Xc);
    const V3 nr = cross(E1, E2);
    const double nn = norm(nr), l1 = norm(E1);
    if (!(nn > 0.0) || !(l1 > 0.0)) return fail(NPFEM_E_MESH, "mesh_create: degenerate rest triangle");
    const V3 e1 = {E1.x / l1, E1.y / l1, E1.z / l1};
    const V3 nh = {nr.x / nn, nr.y / nn, nr.z / nn};
    const V3 e2 = cross(nh, e1);
    const double d00 = dot(e1, E1), d01 = dot(e1, E2), d10 = dot(e2, E1), d11 = dot(e2, E2);
    const double det = d00 * d11 - d01 * d10;
    m->dminv[4 * t + 0] = d11 / det;
    m->dminv[4 * t + 1] = -d01 / det;
    m->dminv[4 * t + 2] = -d10 / det;
    m->dminv[4 * t + 3] = d00 / det;
    m->area[t] = 0.5 * nn;
    vol6 += dot(Xa, cross(Xb, Xc));
  }
  m->V0 = vol6 / 6.0;
  if (!(m->V0 > 0.0)) return fail(NPFEM_E_MESH, "mesh_create: enclosed volume not positive (triangles must be counter-clockwise seen from outside)");
  for (double a : m->area) m->A0 += a;

  // cotangent weights omega_ij = (cot a + cot b)/2 and mixed Voronoi areas (Meyer et al.)
  std::unordered_map<int64_t, double> omega;
  m->vor_area.assign(n, 0.0);
  m->bary_area.assign(n, 0.0);
  for (int t = 0; t < nt; ++t) {
    const int* f = &m->tri[3 * t];
    V3 p[3] = {P(f[0]), P(f[1]), P(f[2])};
    double ang[3], cot[3];
    for (int k = 0; k < 3; ++k) {
      const V3 u = sub(p[(k + 1) % 3], p[k]), v = sub(p[(k + 2) % 3], p[k]);
      cot[k] = dot(u, v) / norm(cross(u, v));
      ang[k] = std::atan2(norm(cross(u, v)), dot(u, v));
    }
    for (int k = 0; k < 3; ++k) {
      const int i = f[(k + 1) % 3], j = f[(k + 2) % 3];   // edge opposite corner k
      const int64_t key = (int64_t)std::min(i, j) * n + std::max(i, j);
      omega[key] += 0.5 * cot[k];
      m->bary_area[f[k]] += m->area[t] / 3.0;
    }
    const bool obtuse = ang[0] > M_PI / 2 || ang[1] > M_PI / 2 || ang[2] > M_PI / 2;
    for (int k = 0; k < 3; ++k) {
      const int j = (k + 1) % 3, l = (k + 2) % 3;
      if (!obtuse) {
        const V3 pj = sub(p[k], p[j]), pl = sub(p[k], p[l]);
        m->vor_area[f[k]] += (dot(pj, pj) * cot[l] + dot(pl, pl) * cot[j]) / 8.0;
      } else if (ang[k] > M_PI / 2) {
        m->vor_area[f[k]] += m->area[t] / 2.0;
      } else {
        m->vor_area[f[k]] += m->area[t] / 4.0;
      }
    }
  }
  // neighbour lists (CSR) and |l0_i|
  std::vector<std::vector<std::pair<int, double>>> nbs(n);
  for (const auto& kv : omega) {
    const int i = (int)(kv.first / n), j = (int)(kv.first % n);
    nbs[i].push_back({j, kv.second});
    nbs[j].push_back({i, kv.second});
  }
  m->nb_ptr.assign(n + 1, 0);
  m->ell0.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    if (nbs[i].empty()) return fail(NPFEM_E_MESH, "mesh_create: unreferenced vertex");
    std::sort(nbs[i].begin(), nbs[i].end());
    m->nb_ptr[i + 1] = m->nb_ptr[i] + (int)nbs[i].size();
    V3 l = {0, 0, 0};
    for (auto& [j, w] : nbs[i]) {
      m->nb_idx.push_back(j);
      m->nb_w.push_back(w);
      const V3 d = sub(P(j), P(i));
      l.x += w * d.x;
      l.y += w * d.y;
      l.z += w * d.z;
    }
    m->ell0[i] = norm(l) / m->vor_area[i];
  }
  // vertex -> incident corners, in triangle order
  std::vector<std::vector<int>> vc(n);
  for (int t = 0; t < nt; ++t)
    for (int k = 0; k < 3; ++k) vc[m->tri[3 * t + k]].push_back(3 * t + k);
  m->vc_ptr.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    m->vc_ptr[i + 1] = m->vc_ptr[i] + (int)vc[i].size();
    m->vc_idx.insert(m->vc_idx.end(), vc[i].begin(), vc[i].end());
  }
  *out = m.release();
  return NPFEM_OK;
}

void npfem_mesh_destroy(npfem_mesh* m) { delete m; }

npfem_status npfem_mesh_query(const npfem_mesh* m, int32_t* n, int32_t* nt, int32_t* ne, double* V0,
                              double* A0) {
  if (!m) return fail(NPFEM_E_INVALID, "mesh_query: NULL mesh");
  if (n) *n = m->n;
  if (nt) *nt = m->nt;
  if (ne) *ne = m->ne;
  if (V0) *V0 = m->V0;
  if (A0) *A0 = m->A0;
  return NPFEM_OK;
}

npfem_status npfem_mesh_rest_data(const npfem_mesh* m, double* vor_area, double* ell0, double* tri_area,
                                  double* dminv) {
  if (!m) return fail(NPFEM_E_INVALID, "mesh_rest_data: NULL mesh");
  if (vor_area) std::copy(m->vor_area.begin(), m->vor_area.end(), vor_area);
  if (ell0) std::copy(m->ell0.begin(), m->ell0.end(), ell0);
  if (tri_area) std::copy(m->area.begin(), m->area.end(), tri_area);
  if (dminv) std::copy(m->dminv.begin(), m->dminv.end(), dminv);
  return NPFEM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------
// Plan
// ---------------------------------------------------------------------------------
namespace {

struct DeviceBuffers {
  std::vector<void*> ptrs;
  ~DeviceBuffers() { release(); }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
  template <typename T>
  npfem_status upload(const T* src, size_t count, const T** out) {
    void* p = nullptr;
    HIP_TRY(hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T)));
    ptrs.push_back(p);
    if (count) HIP_TRY(hipMemcpy(p, src, count * sizeof(T), hipMemcpyHostToDevice));
    *out = static_cast<const T*>(p);
    return NPFEM_OK;
  }
  npfem_status alloc(size_t bytes, void** out) {
    void* p = nullptr;
    HIP_TRY(hipMalloc(&p, std::max<size_t>(bytes, 16)));
    ptrs.push_back(p);
    *out = p;
    return NPFEM_OK;
  }
};

struct MeshPlan {
  const npfem_mesh* mesh;
  int n_pad, chunk, vec_lds = 1, xu_lds = 1;
  std::vector<double> mass;
  double floor_force;
  MeshDev<float> dev32;
  MeshDev<double> dev64;
  BandFactorDev<float> fac32{};      // banded Cholesky factors of H~ and M~/h^2 (F null: not available)
  BandFactorDev<double> fac64{};
};

template <typename Real>
std::vector<Real> pad_matrix(const std::vector<double>& A, int n, int np, double scale) {
  std::vector<Real> P((size_t)np * np, Real(0));
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) P[(size_t)i * np + j] = Real(scale * A[(size_t)i * n + j]);
  return P;
}

}  // namespace

struct npfem_plan {
  int device = 0, precision = NPFEM_FP32, cu_count = 0;
  double dt = 0.0;
  npfem_material mat{};
  npfem_solver_params prm{};
  std::vector<MeshPlan> meshes;
  DeviceBuffers buf;
  const void* d_meshdev = nullptr;
};

namespace {

// Reverse Cuthill-McKee order of the mesh's vertex graph (George & Liu 1981): per
// connected component, a breadth-first search from a pseudo-peripheral vertex (the
// smallest-degree vertex of the last level of a search from the previous start, twice),
// visiting neighbours by increasing degree; the whole order reversed.
constexpr double kBandRel = 1e-4;   // banded BF16 products: entries kept above this, relative

std::vector<int> rcm_order(const npfem_mesh* m) {
  const int n = m->n;
  auto deg = [&](int i) { return m->nb_ptr[i + 1] - m->nb_ptr[i]; };
  std::vector<int> order;
  order.reserve(n);
  std::vector<char> placed(n, 0);
  std::vector<int> stamp(n, -1), queue, nbrs;
  int pass = 0;
  // breadth-first search over unplaced vertices; returns the order of the visit
  auto bfs = [&](int s0, bool sorted) {
    queue.assign(1, s0);
    stamp[s0] = ++pass;
    for (size_t h = 0; h < queue.size(); ++h) {
      const int v = queue[h];
      nbrs.clear();
      for (int q = m->nb_ptr[v]; q < m->nb_ptr[v + 1]; ++q) {
        const int w = m->nb_idx[q];
        if (!placed[w] && stamp[w] != pass) {
          stamp[w] = pass;
          nbrs.push_back(w);
        }
      }
      if (sorted)
        std::stable_sort(nbrs.begin(), nbrs.end(), [&](int a, int b) { return deg(a) < deg(b); });
      queue.insert(queue.end(), nbrs.begin(), nbrs.end());
    }
    return queue;
  };
  for (;;) {
    int start = -1;
    for (int i = 0; i < n; ++i)
      if (!placed[i] && (start < 0 || deg(i) < deg(start))) start = i;
    if (start < 0) break;
    for (int it = 0; it < 2; ++it) {                 // move the start towards the periphery
      const std::vector<int> q = bfs(start, false);
      // the last level: vertices at the largest distance (re-derived from a level sweep)
      std::vector<int> level(n, -1);
      level[start] = 0;
      int far = 0;
      for (int v : q)
        for (int k = m->nb_ptr[v]; k < m->nb_ptr[v + 1]; ++k) {
          const int w = m->nb_idx[k];
          if (!placed[w] && level[w] < 0) {
            level[w] = level[v] + 1;
            far = std::max(far, level[w]);
          }
        }
      int best = start;
      for (int v : q)
        if (level[v] == far && (best == start || deg(v) < deg(best))) best = v;
      start = best;
    }
    for (int v : bfs(start, true)) {
      placed[v] = 1;
      order.push_back(v);
    }
  }
  std::reverse(order.begin(), order.end());
  return order;
}

// Banded Cholesky factor of P A P^T (P: the order `perm`, A dense FP64 n x n), computed
// within the band of the permuted matrix only (a banded matrix's Cholesky factor keeps
// its band); false if A is not positive definite.
struct BandFactorHost {
  int n = 0, b = 0;
  std::vector<double> L;               // [n][n], zero outside the band
  // entry (i, j) of the factor padded to n_pad: the identity on the padding positions
  double at(int i, int j) const {
    if (i < n && j < n) return (j <= i && i - j <= b) ? L[(size_t)i * n + j] : 0.0;
    return i == j ? 1.0 : 0.0;
  }
};

bool band_factor(const std::vector<double>& A, int n, const std::vector<int>& perm, BandFactorHost& out) {
  std::vector<double> Ap((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Ap[(size_t)i * n + j] = A[(size_t)perm[i] * n + perm[j]];
  int b = 0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j)
      if (Ap[(size_t)i * n + j] != 0.0) {
        b = std::max(b, i - j);
        break;
      }
  std::vector<double>& L = out.L;
  L.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    const int lo = std::max(0, i - b);
    for (int j = lo; j <= i; ++j) {
      double s = Ap[(size_t)i * n + j];
      for (int k = lo; k < j; ++k) s -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      if (j < i) {
        L[(size_t)i * n + j] = s / L[(size_t)j * n + j];
      } else {
        if (!(s > 0.0) || !std::isfinite(s)) return false;
        L[(size_t)i * n + i] = std::sqrt(s);
      }
    }
  }
  out.n = n;
  out.b = b;
  return true;
}

// The factor in the layouts of the substitution kernels (see BandFactorDev) for a band
// width B (a multiple of 16, at least b) and n_pad positions.
template <typename Real>
void factor_layouts(const BandFactorHost& f, int np, int B, std::vector<Real>& F, std::vector<Real>& G,
                    std::vector<Real>& T, std::vector<Real>& FA, std::vector<Real>& GA, std::vector<Real>& DA,
                    std::vector<Real>& DB) {
  const int R = kFactorRows, nblk = np / R;
  F.assign((size_t)nblk * B * R, Real(0));
  G.assign((size_t)nblk * B * R, Real(0));
  T.assign((size_t)nblk * kFactorDiag, Real(0));
  for (int blk = 0; blk < nblk; ++blk) {
    const int i0 = blk * R;
    for (int jj = 0; jj < B; ++jj)
      for (int k = 0; k < R; ++k) {
        const int jf = i0 - B + jj, jg = i0 + R + jj;
        if (jf >= 0) F[((size_t)blk * B + jj) * R + k] = Real(-f.at(i0 + k, jf));
        if (jg < np) G[((size_t)blk * B + jj) * R + k] = Real(-f.at(jg, i0 + k));
      }
    Real* Tb = &T[(size_t)blk * kFactorDiag];
    for (int k = 0; k < R; ++k) {
      Tb[k] = Real(1.0 / f.at(i0 + k, i0 + k));
      for (int l = 0; l < k; ++l) Tb[R + k * R + l] = Real(f.at(i0 + k, i0 + l));
    }
  }
  // matrix-core layouts: blocks of 16 positions, k steps of 4, one entry per lane
  // (lane l: row l & 15, k index l >> 4)
  const int M = kFactorMfmaRows, nb = np / M, ks = B / 4;
  FA.assign((size_t)nb * ks * 64, Real(0));
  GA.assign((size_t)nb * ks * 64, Real(0));
  DA.assign((size_t)nb * 4 * 64, Real(0));
  DB.assign((size_t)nb * 4 * 64, Real(0));
  for (int bi = 0; bi < nb; ++bi) {
    const int i0 = bi * M;
    for (int st = 0; st < ks; ++st)
      for (int l = 0; l < 64; ++l) {
        const int row = i0 + (l & 15), kq = l >> 4;
        const int jf = i0 - B + 4 * st + kq, jg = i0 + M + 4 * st + kq;
        if (jf >= 0) FA[((size_t)bi * ks + st) * 64 + l] = Real(-f.at(row, jf));
        if (jg < np) GA[((size_t)bi * ks + st) * 64 + l] = Real(-f.at(jg, row));
      }
    // inverse of the 16 x 16 lower-triangular diagonal block, by forward substitution
    double Dinv[16][16] = {};
    for (int c = 0; c < M; ++c)
      for (int r = c; r < M; ++r) {
        double t = r == c ? 1.0 : 0.0;
        for (int q = c; q < r; ++q) t -= f.at(i0 + r, i0 + q) * Dinv[q][c];
        Dinv[r][c] = t / f.at(i0 + r, i0 + r);
      }
    for (int st = 0; st < 4; ++st)
      for (int l = 0; l < 64; ++l) {
        const int r = l & 15, k = 4 * st + (l >> 4);
        DA[((size_t)bi * 4 + st) * 64 + l] = Real(Dinv[r][k]);     // L_D^-1
        DB[((size_t)bi * 4 + st) * 64 + l] = Real(Dinv[k][r]);     // L_D^-T
      }
  }
}

// Uploads both factors (H~ and M~/h^2) in precision Real, in one band width B (the wider
// of the two), with the order's inverse permutation, in the layout of the plan's kernel
// (FP32: FA, GA, DA, DB; FP64: F, G, T); leaves them null when the kernel's LDS ring
// would not fit a compute unit.
template <typename Real>
npfem_status upload_factor(npfem_plan* p, int np, const std::vector<int>& perm, const BandFactorHost (&fh)[2],
                           BandFactorDev<Real>& f) {
  f = BandFactorDev<Real>{};
  f.b = std::max(fh[0].b, fh[1].b);
  const int B = std::max(16, (f.b + 15) / 16 * 16);
  f.ring = B + 16;
  if (band_solve_lds_bytes<Real>(f.ring) > kBandSolveMaxLds) return NPFEM_OK;
  std::vector<int> ip(np);
  for (int k = 0; k < np; ++k) ip[k] = k;
  for (size_t a = 0; a < perm.size(); ++a) ip[perm[a]] = (int)a;
  npfem_status s;
  if ((s = p->buf.upload(ip.data(), ip.size(), &f.iperm))) return s;
  f.B = B;
  for (int w = 0; w < 2; ++w) {
    std::vector<Real> F, G, T, FA, GA, DA, DB;
    factor_layouts<Real>(fh[w], np, B, F, G, T, FA, GA, DA, DB);
    if constexpr (std::is_same<Real, float>::value) {       // FP32: the matrix-core kernel
      if ((s = p->buf.upload(FA.data(), FA.size(), &f.FA[w]))) return s;
      if ((s = p->buf.upload(GA.data(), GA.size(), &f.GA[w]))) return s;
      if ((s = p->buf.upload(DA.data(), DA.size(), &f.DA[w]))) return s;
      if ((s = p->buf.upload(DB.data(), DB.size(), &f.DB[w]))) return s;
    } else {                                                // FP64: the vector-unit kernel
      if ((s = p->buf.upload(F.data(), F.size(), &f.F[w]))) return s;
      if ((s = p->buf.upload(G.data(), G.size(), &f.G[w]))) return s;
      if ((s = p->buf.upload(T.data(), T.size(), &f.T[w]))) return s;
    }
  }
  return NPFEM_OK;
}

template <typename Real>
npfem_status upload_mesh(npfem_plan* p, MeshPlan& mp, const std::vector<double>& hinv,
                         const std::vector<double>& minv_h2, MeshDev<Real>& d) {
  const npfem_mesh* m = mp.mesh;
  const int n = m->n, np = mp.n_pad;
  auto conv = [](const std::vector<double>& v) { return std::vector<Real>(v.begin(), v.end()); };
  d.n = n;
  d.nt = m->nt;
  d.n_pad = np;
  d.chunk = mp.chunk;
  d.vec_lds = mp.vec_lds;
  d.xu_lds = mp.xu_lds;
  npfem_status s;
  if ((s = p->buf.upload(m->tri.data(), m->tri.size(), &d.tri))) return s;
  auto w = conv(m->nb_w), va = conv(m->vor_area), e0 = conv(m->ell0), ms = conv(mp.mass);
  std::vector<double> i4(m->nt);
  for (int t = 0; t < m->nt; ++t) i4[t] = 0.25 / (m->area[t] * m->area[t]);
  if ((s = p->buf.upload(m->dminv.data(), m->dminv.size(), &d.dminv))) return s;
  if ((s = p->buf.upload(m->area.data(), m->area.size(), &d.area))) return s;
  if ((s = p->buf.upload(i4.data(), i4.size(), &d.inv4a2))) return s;
  if ((s = p->buf.upload(m->vc_ptr.data(), m->vc_ptr.size(), &d.vc_ptr))) return s;
  if ((s = p->buf.upload(m->vc_idx.data(), m->vc_idx.size(), &d.vc_idx))) return s;
  if ((s = p->buf.upload(m->nb_ptr.data(), m->nb_ptr.size(), &d.nb_ptr))) return s;
  if ((s = p->buf.upload(m->nb_idx.data(), m->nb_idx.size(), &d.nb_idx))) return s;
  if ((s = p->buf.upload(w.data(), w.size(), &d.nb_w))) return s;
  // padded (ELL) copies of the neighbour and corner lists, column q of vertex i at q*n_pad + i
  int nbd = 0, vcd = 0;
  for (int i = 0; i < n; ++i) {
    nbd = std::max(nbd, m->nb_ptr[i + 1] - m->nb_ptr[i]);
    vcd = std::max(vcd, m->vc_ptr[i + 1] - m->vc_ptr[i]);
  }
  std::vector<int> nbe((size_t)nbd * np), vce((size_t)vcd * np, -1);
  std::vector<Real> nbwe((size_t)nbd * np, Real(0));
  for (int i = 0; i < np; ++i)
    for (int q = 0; q < nbd; ++q) nbe[(size_t)q * np + i] = i < n ? i : 0;
  for (int i = 0; i < n; ++i) {
    for (int q = m->nb_ptr[i]; q < m->nb_ptr[i + 1]; ++q) {
      const size_t o = (size_t)(q - m->nb_ptr[i]) * np + i;
      nbe[o] = m->nb_idx[q];
      nbwe[o] = Real(m->nb_w[q]);
    }
    for (int q = m->vc_ptr[i]; q < m->vc_ptr[i + 1]; ++q) vce[(size_t)(q - m->vc_ptr[i]) * np + i] = m->vc_idx[q];
  }
  d.nb_deg = nbd;
  d.vc_deg = vcd;
  if ((s = p->buf.upload(nbe.data(), nbe.size(), &d.nb_ell))) return s;
  if ((s = p->buf.upload(nbwe.data(), nbwe.size(), &d.nbw_ell))) return s;
  if ((s = p->buf.upload(vce.data(), vce.size(), &d.vc_ell))) return s;
  if ((s = p->buf.upload(va.data(), va.size(), &d.vor_area))) return s;
  if ((s = p->buf.upload(e0.data(), e0.size(), &d.ell0))) return s;
  if ((s = p->buf.upload(ms.data(), ms.size(), &d.mass))) return s;
  auto H = pad_matrix<Real>(hinv, n, np, 1.0);
  auto Mi = pad_matrix<Real>(minv_h2, n, np, 1.0);
  if ((s = p->buf.upload(H.data(), H.size(), &d.hinv))) return s;
  if ((s = p->buf.upload(Mi.data(), Mi.size(), &d.minv))) return s;
  d.hinv_bf = d.minv_bf = nullptr;
  d.hinv_diag = d.minv_diag = nullptr;
  d.bperm = d.bband = nullptr;
  if (p->prm.inverse_bf16 && p->precision == NPFEM_FP32) {
    // exact FP32 diagonal + BF16 off-diagonal part (zero diagonal, zero padding); banded:
    // the off-diagonal part in the reverse Cuthill-McKee order, each 16-column block kept
    // over the k' range of its entries above kBandRel sqrt(A_ii A_jj)
    const bool banded = p->prm.inverse_bf16 == 2;
    std::vector<int> perm(np);
    for (int i = 0; i < np; ++i) perm[i] = i;
    if (banded) {
      const std::vector<int> ord = rcm_order(m);
      std::copy(ord.begin(), ord.end(), perm.begin());
    }
    const int ncb = np / 16;
    std::vector<int> band((size_t)2 * ncb * 2, 0);
    for (int which = 0; which < 2; ++which) {
      const std::vector<double>& A = which == 0 ? hinv : minv_h2;
      std::vector<uint16_t> off((size_t)np * np, 0);
      std::vector<float> dg(np, 0.0f);
      for (int i = 0; i < n; ++i) dg[i] = (float)A[(size_t)i * n + i];
      if (!banded) {
        for (int i = 0; i < n; ++i)
          for (int j = 0; j < n; ++j)
            if (j != i) off[(size_t)i * np + j] = to_bf16((float)A[(size_t)i * n + j]);
      } else {
        std::vector<double> sd(n);
        for (int i = 0; i < n; ++i) sd[i] = std::sqrt(std::fabs(A[(size_t)i * n + i]));
        for (int cb = 0; cb < ncb; ++cb) {
          int lo = np, hi = 0;
          for (int a = 16 * cb; a < 16 * cb + 16 && a < n; ++a)
            for (int k = 0; k < n; ++k) {
              const int i = perm[a], j = perm[k];
              if (i != j && std::fabs(A[(size_t)i * n + j]) > kBandRel * sd[i] * sd[j]) {
                lo = std::min(lo, k);
                hi = std::max(hi, k + 1);
              }
            }
          if (lo >= hi) lo = hi = 0;
          lo = lo / 32 * 32;
          hi = std::min(np, (hi + 31) / 32 * 32);
          band[((size_t)which * ncb + cb) * 2] = lo;
          band[((size_t)which * ncb + cb) * 2 + 1] = hi;
          for (int a = 16 * cb; a < 16 * cb + 16 && a < n; ++a)
            for (int k = lo; k < hi && k < n; ++k)
              if (k != a) off[(size_t)a * np + k] = to_bf16((float)A[(size_t)perm[a] * n + perm[k]]);
        }
      }
      const uint16_t** po = which == 0 ? &d.hinv_bf : &d.minv_bf;
      const float** pd = which == 0 ? &d.hinv_diag : &d.minv_diag;
      if ((s = p->buf.upload(off.data(), off.size(), po))) return s;
      if ((s = p->buf.upload(dg.data(), dg.size(), pd))) return s;
    }
    if (!banded)                                   // the identity order, whole ranges
      for (size_t k = 0; k < band.size(); k += 2) {
        band[k] = 0;
        band[k + 1] = np;
      }
    if (banded && (s = p->buf.upload(perm.data(), perm.size(), &d.bperm))) return s;   // null: identity
    if ((s = p->buf.upload(band.data(), band.size(), &d.bband))) return s;
  }
  d.V0 = m->V0;
  d.A0 = m->A0;
  d.floor_force = mp.floor_force;
  return NPFEM_OK;
}

// Largest triangle chunk for which the step's LDS fits the budget.
template <typename Real>
int choose_chunk(int np, int nt, size_t budget, int vec_lds, int xu_lds) {
  if (lds_bytes<Real>(np, nt, 0, vec_lds, xu_lds) <= budget) return nt;
  int lo = 0;
  for (int ch = nt; ch >= 64; ch -= 64)
    if (lds_bytes<Real>(np, ch, 0, vec_lds, xu_lds) <= budget) { lo = ch; break; }
  return lo;
}

// LDS layout of a mesh: the first fit of (gradient and b in LDS, whole triangle list in
// one chunk, two workgroups per CU), (in the workspace, one chunk, two per CU), (in LDS,
// one chunk, one per CU), (in the workspace, largest chunk, one per CU), and finally
// (x_n and u in the workspace too, the LDS holding only the largest triangle chunk).
template <typename Real>
void choose_layout(int np, int nt, size_t half, size_t cap, int* chunk, int* vec_lds, int* xu_lds) {
  const size_t budgets[5] = {half, half, cap, cap, cap};
  const int vls[5] = {1, 0, 1, 0, 0};
  const int xus[5] = {1, 1, 1, 1, 0};
  for (int k = 0; k < 5; ++k) {
    const int ch = choose_chunk<Real>(np, nt, budgets[k], vls[k], xus[k]);
    if (ch == nt || (k >= 3 && ch > 0)) {
      *chunk = ch;
      *vec_lds = vls[k];
      *xu_lds = xus[k];
      return;
    }
  }
  *chunk = 0;
  *vec_lds = 0;
  *xu_lds = 0;
}

}  // namespace

extern "C" {

npfem_status npfem_plan_create(int32_t device, const npfem_mesh* const* meshes, int32_t n_meshes,
                               const npfem_material* mat, double dt, const npfem_solver_params* prm,
                               npfem_plan** out) {
  if (!out || !meshes || !mat || !prm) return fail(NPFEM_E_INVALID, "plan_create: NULL pointer");
  *out = nullptr;
  if (n_meshes < 1) return fail(NPFEM_E_INVALID, "plan_create: need at least one mesh");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(NPFEM_E_INVALID, "plan_create: dt must be positive");
  if (prm->precision != NPFEM_FP32 && prm->precision != NPFEM_FP64)
    return fail(NPFEM_E_INVALID, "plan_create: unknown precision");
  if (prm->lbfgs_m < 0 || prm->lbfgs_m > kMaxHistory)
    return fail(NPFEM_E_INVALID, "plan_create: lbfgs_m must be in [0, 8]");
  if (prm->max_iter < 1 || prm->max_halvings < 0 || !(prm->tol >= 0.0) || !(prm->c1 >= 0.0))
    return fail(NPFEM_E_INVALID, "plan_create: bad solver controls");
  if (prm->cells_per_tile < 0 || prm->cells_per_tile > kMaxTile)
    return fail(NPFEM_E_INVALID, "plan_create: cells_per_tile must be in [0, 21]");
  if (prm->inverse_bf16 < 0 || prm->inverse_bf16 > 2)
    return fail(NPFEM_E_INVALID, "plan_create: inverse_bf16 must be 0, 1 or 2");
  if (prm->volume_normaliser != NPFEM_VOLUME_STEP_FROZEN && prm->volume_normaliser != NPFEM_VOLUME_PAPER_LITERAL)
    return fail(NPFEM_E_INVALID, "plan_create: unknown volume_normaliser");
  const double mats[] = {mat->B, mat->C, mat->D, mat->k_bend, mat->k_volume, mat->beta, mat->density, mat->k_area_global};
  for (double v : mats)
    if (!(v >= 0.0) || !std::isfinite(v)) return fail(NPFEM_E_INVALID, "plan_create: material constants must be finite and >= 0");
  if (!(mat->density > 0.0)) return fail(NPFEM_E_INVALID, "plan_create: density must be positive");
  if (!(mat->kappa >= 0.0 && mat->kappa <= 1.0)) return fail(NPFEM_E_INVALID, "plan_create: kappa must be in [0, 1]");
  for (int i = 0; i < n_meshes; ++i)
    if (!meshes[i]) return fail(NPFEM_E_INVALID, "plan_create: NULL mesh");

  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(NPFEM_E_INVALID, "plan_create: no such HIP device");
  HIP_TRY(hipSetDevice(device));
  if (npfem_status se = init_scratch(device)) return se;
  auto p = std::make_unique<npfem_plan>();
  p->device = device;
  p->precision = prm->precision;
  p->dt = dt;
  p->mat = *mat;
  p->prm = *prm;
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device));
  p->cu_count = prop.multiProcessorCount;
  const double h = dt, kmat = mat->k_mat < 0 ? mat->B : mat->k_mat;
  const bool fp64 = prm->precision == NPFEM_FP64;
  const size_t lds_cap = kStepLdsCap;
  p->meshes.resize(n_meshes);
  for (int mi = 0; mi < n_meshes; ++mi) {
    const npfem_mesh* m = meshes[mi];
    MeshPlan& mp = p->meshes[mi];
    mp.mesh = m;
    const int n = m->n;
    mp.n_pad = round_up(n, 32);
    // two workgroups per CU when the whole triangle list fits in half the LDS
    const size_t half = 80 * 1024 - 512;
    if (fp64)
      choose_layout<double>(mp.n_pad, m->nt, half, lds_cap, &mp.chunk, &mp.vec_lds, &mp.xu_lds);
    else
      choose_layout<float>(mp.n_pad, m->nt, half, lds_cap, &mp.chunk, &mp.vec_lds, &mp.xu_lds);
    if (mp.chunk <= 0)
      return fail(NPFEM_E_UNSUPPORTED, "plan_create: mesh too large for the LDS in this precision");
    if (!fp64 && !mp.xu_lds)
      return fail(NPFEM_E_UNSUPPORTED, "plan_create: FP32 plans keep each cell's x_n and u in LDS; this mesh is too large for that");
    // lumped mass by barycentric area (section 2.1)
    double bsum = 0.0;
    for (double a : m->bary_area) bsum += a;
    mp.mass.resize(n);
    for (int i = 0; i < n; ++i) mp.mass[i] = mat->density * m->V0 * m->bary_area[i] / bsum;
    mp.floor_force = mat->B * std::sqrt(m->A0);
    // L' (area + bending PD), K_mat (material term of H~), dense n x n per coordinate
    std::vector<double> Lp((size_t)n * n, 0.0), Km((size_t)n * n, 0.0);
    for (int t = 0; t < m->nt; ++t) {
      const int* f = &m->tri[3 * t];
      const double* d = &m->dminv[4 * t];
      const double g[3][2] = {{d[0], d[1]}, {d[2], d[3]}, {-d[0] - d[2], -d[1] - d[3]}};
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          const double gg = g[a][0] * g[b][0] + g[a][1] * g[b][1];
          Lp[(size_t)f[a] * n + f[b]] += m->area[t] * mat->C * gg;
          Km[(size_t)f[a] * n + f[b]] += m->area[t] * kmat * gg;
        }
    }
    for (int i = 0; i < n; ++i) {
      // bending row G_i: omega_ij / A_i at j, -sum at i; weight k_b A_i
      std::vector<std::pair<int, double>> row;
      double diag = 0.0;
      for (int q = m->nb_ptr[i]; q < m->nb_ptr[i + 1]; ++q) {
        const double c = m->nb_w[q] / m->vor_area[i];
        row.push_back({m->nb_idx[q], c});
        diag -= c;
      }
      row.push_back({i, diag});
      const double w = mat->k_bend * m->vor_area[i];
      for (auto& [a, ca] : row)
        for (auto& [b, cb] : row) Lp[(size_t)a * n + b] += w * ca * cb;
    }
    // M~ = M + beta h^2 L';  H~ = M~/h^2 + L' + (k_volume + k_area_global) I + K_mat
    std::vector<double> Mt((size_t)n * n), Ht((size_t)n * n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const size_t k = (size_t)i * n + j;
        Mt[k] = mat->beta * h * h * Lp[k] + (i == j ? mp.mass[i] : 0.0);
        Ht[k] = Mt[k] / (h * h) + Lp[k] + Km[k] + (i == j ? mat->k_volume + mat->k_area_global : 0.0);
      }
    // the paper's route: banded factors of H~ and M~/h^2 in the reverse Cuthill-McKee order
    {
      const std::vector<int> perm = rcm_order(m);
      std::vector<double> Ms(Mt);
      for (double& v : Ms) v /= h * h;
      BandFactorHost fh[2];
      if (!band_factor(Ht, n, perm, fh[0]))
        return fail(NPFEM_E_NOT_SPD, "plan_create: H~ is not positive definite");
      if (!band_factor(Ms, n, perm, fh[1]))
        return fail(NPFEM_E_NOT_SPD, "plan_create: M~ is not positive definite");
      npfem_status fs = fp64 ? upload_factor<double>(p.get(), mp.n_pad, perm, fh, mp.fac64)
                             : upload_factor<float>(p.get(), mp.n_pad, perm, fh, mp.fac32);
      if (fs) return fs;
    }
    if (!cholesky(Mt, n)) return fail(NPFEM_E_NOT_SPD, "plan_create: M~ is not positive definite");
    if (!cholesky(Ht, n)) return fail(NPFEM_E_NOT_SPD, "plan_create: H~ is not positive definite");
    const std::vector<double> Hinv = spd_inverse(Ht, n);
    std::vector<double> Minv = spd_inverse(Mt, n);
    for (double& v : Minv) v *= h * h;
    npfem_status s = fp64 ? upload_mesh<double>(p.get(), mp, Hinv, Minv, mp.dev64)
                          : upload_mesh<float>(p.get(), mp, Hinv, Minv, mp.dev32);
    if (s) return s;
  }
  // device array of mesh descriptors
  npfem_status s;
  if (fp64) {
    std::vector<MeshDev<double>> v;
    for (auto& mp : p->meshes) v.push_back(mp.dev64);
    const MeshDev<double>* d;
    if ((s = p->buf.upload(v.data(), v.size(), &d))) return s;
    p->d_meshdev = d;
  } else {
    std::vector<MeshDev<float>> v;
    for (auto& mp : p->meshes) v.push_back(mp.dev32);
    const MeshDev<float>* d;
    if ((s = p->buf.upload(v.data(), v.size(), &d))) return s;
    p->d_meshdev = d;
  }
  *out = p.release();
  return NPFEM_OK;
}

void npfem_plan_destroy(npfem_plan* p) {
  if (!p) return;
  (void)hipSetDevice(p->device);
  delete p;
}

npfem_status npfem_plan_masses(const npfem_plan* p, int32_t mi, double* out) {
  if (!p || !out) return fail(NPFEM_E_INVALID, "plan_masses: NULL pointer");
  if (mi < 0 || mi >= (int)p->meshes.size()) return fail(NPFEM_E_INVALID, "plan_masses: bad mesh index");
  std::copy(p->meshes[mi].mass.begin(), p->meshes[mi].mass.end(), out);
  return NPFEM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------
// Batch
// ---------------------------------------------------------------------------------
struct npfem_batch {
  npfem_plan* plan = nullptr;
  int64_t n_cells = 0, n_vert = 0;
  int n_pad_max = 0;
  std::vector<std::vector<int>> by_mesh;   // cells of each mesh type, in batch order
  DeviceBuffers buf;                       // cell layout (fixed)
  const int64_t* cell_voff = nullptr;
  const int* cell_mesh = nullptr;
  const int* mesh_n = nullptr;
  void* eval_scratch = nullptr;
  // schedule: tiling, history length and workspace (rebuilt by the autotuner)
  int T = 0, m = 0, n_tiles = 0, grid = 0, n_vec = 0, stage_k = 0, cs_lds = -1;
  size_t lds = 0;
  int64_t slot_stride = 0;
  DeviceBuffers sched;
  const TileDesc* tiles = nullptr;
  const int* tile_cells = nullptr;
  int* counter = nullptr;
  void* work = nullptr;
  CellState* cstate = nullptr;
  // captured steps (hipGraph), each keyed by the buffers, stream and network it was
  // captured with; a few are kept so that callers alternating between buffer sets (the
  // usual ping-pong of x and x_out) replay instead of capturing again
  static constexpr int kGraphCache = 4;
  struct GraphEntry {
    const void* key[9];
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;
  };
  int use_graph = 0;
  std::vector<GraphEntry> graphs;
  uint64_t graph_clock = 0;
  int64_t graph_captures = 0, graph_replays = 0;
  // learned warm start: the predicted correction of every vertex (allocated on first use)
  DeviceBuffers dbuf;
  void* delta = nullptr;
  double* net_frames = nullptr;             // [n_cells][kNetFrame] frames of the resident inference
  // contact search: hashed grid buffers (allocated on first use)
  DeviceBuffers cbuf;
  int64_t c_table = 0;
  unsigned *c_count = nullptr, *c_start = nullptr, *c_fill = nullptr, *c_bsum = nullptr, *c_vkey = nullptr,
           *c_sorted = nullptr;
  int* c_vcell = nullptr;
  double* c_normals = nullptr;
  unsigned long long* c_ncontacts = nullptr;
  void drop_graph() {
    for (auto& g : graphs) {
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
      if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    graphs.clear();
  }
  ~npfem_batch() { drop_graph(); }
};

namespace {

template <typename Real>
StepArgs<Real> make_args(npfem_batch* b) {
  npfem_plan* p = b->plan;
  StepArgs<Real> a{};
  a.meshes = static_cast<const MeshDev<Real>*>(p->d_meshdev);
  a.mat = {p->mat.B, p->mat.C, p->mat.D, p->mat.k_bend, p->mat.k_volume, p->mat.beta, p->mat.kappa,
           p->mat.k_area_global};
  const double eps = std::is_same<Real, float>::value ? 1.1920928955078125e-07 : 2.220446049250313e-16;
  a.sol = {p->dt, p->prm.tol, p->prm.c1, p->prm.noise_factor * eps, b->m, p->prm.max_iter,
           p->prm.max_halvings, std::is_same<Real, float>::value ? p->prm.inverse_bf16 : 0,
           p->prm.volume_normaliser == NPFEM_VOLUME_PAPER_LITERAL ? 1 : 0};
  a.tiles = b->tiles;
  a.tile_cells = b->tile_cells;
  a.cell_voff = b->cell_voff;
  a.cell_mesh = b->cell_mesh;
  a.n_tiles = b->n_tiles;
  a.tile_cells_max = b->T;
  a.tile_counter = b->counter;
  a.n_vec_slot = b->n_vec;
  a.slot_stride = b->slot_stride;
  a.work = static_cast<Real*>(b->work);
  a.cstate = b->cstate;
  a.cs_lds = b->cs_lds;
  a.n_pad_max = b->n_pad_max;
  a.layout = 0;
  for (size_t mi = 0; mi < p->meshes.size(); ++mi)
    if (!b->by_mesh[mi].empty())
      a.layout = std::max(a.layout, !p->meshes[mi].xu_lds ? 2 : (!p->meshes[mi].vec_lds ? 1 : 0));
  a.stage_k = b->stage_k;
  return a;
}

// (Re)build the schedule for T cells per tile and history length m: the tile list
// (cells of one mesh type, largest meshes first since the cost grows like n^2), the
// LDS size, the persistent grid and the workspace.
template <typename Real>
npfem_status batch_schedule(npfem_batch* b, int T, int m) {
  npfem_plan* p = b->plan;
  b->drop_graph();
  b->sched.release();
  b->T = T;
  b->m = m;
  const int nm = (int)p->meshes.size();
  std::vector<int> order(nm);
  for (int i = 0; i < nm; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int a, int c) { return p->meshes[a].mesh->n > p->meshes[c].mesh->n; });
  std::vector<TileDesc> tiles;
  std::vector<int> tcells;
  for (int mi : order) {
    const auto& cl = b->by_mesh[mi];
    for (size_t s0 = 0; s0 < cl.size(); s0 += T) {
      TileDesc td;
      td.mesh = mi;
      td.count = (int)std::min<size_t>(T, cl.size() - s0);
      td.first = (int)tcells.size();
      td.pad = 0;
      tcells.insert(tcells.end(), cl.begin() + s0, cl.begin() + s0 + td.count);
      tiles.push_back(td);
    }
  }
  b->n_tiles = (int)tiles.size();
  npfem_status s;
  if ((s = b->sched.upload(tiles.data(), tiles.size(), &b->tiles))) return s;
  if ((s = b->sched.upload(tcells.data(), tcells.size(), &b->tile_cells))) return s;
  size_t lds = 0;
  const int stage_rows = (p->prm.inverse_bf16 && std::is_same<Real, float>::value) ? 16 * ((3 * T + 15) / 16) : 0;
  for (int mi = 0; mi < nm; ++mi)
    if (!b->by_mesh[mi].empty())
      lds = std::max(lds, lds_bytes<Real>(p->meshes[mi].n_pad, p->meshes[mi].chunk, stage_rows,
                                          p->meshes[mi].vec_lds, p->meshes[mi].xu_lds));
  b->stage_k = stage_cols(lds, stage_rows, b->n_pad_max);   // the staging stays below the cell states
  if (p->prm.inverse_bf16 == 2 && std::is_same<Real, float>::value && b->stage_k < 32)
    return fail(NPFEM_E_UNSUPPORTED, "batch_schedule: banded products need an LDS staging area");
  // the tile's cell states go to LDS (after everything else) when they fit the LDS a
  // workgroup may have and cost no workgroups per CU
  {
    const size_t base = (lds + 15) / 16 * 16, with_cs = base + (size_t)T * cell_state_bytes(m);
    b->cs_lds = -1;
    if (with_cs <= kStepLdsCap) {
      HIP_TRY(set_lds_limit<Real>(with_cs));
      int per_base = 0, per_cs = 0;
      HIP_TRY(occupancy<Real>(&per_base, lds));
      HIP_TRY(occupancy<Real>(&per_cs, with_cs));
      if (per_cs >= per_base && per_cs > 0) {
        b->cs_lds = (int)base;
        lds = with_cs;
      }
    }
  }
  b->lds = lds;
  HIP_TRY(set_lds_limit<Real>(lds));
  int per_cu = 0;
  HIP_TRY(occupancy<Real>(&per_cu, lds));
  if (per_cu < 1) return fail(NPFEM_E_UNSUPPORTED, "batch: step kernel does not fit on a compute unit");
  const int slots = p->cu_count * per_cu;
  b->grid = p->prm.grid_blocks > 0 ? p->prm.grid_blocks : slots;
  b->grid = std::max(1, std::min(b->grid, b->n_tiles));
  // b, u, grad, d, q, the history, and a trial gradient if some mesh keeps it out of LDS
  bool any_global = false, any_xu_global = false;
  for (int mi = 0; mi < nm; ++mi) {
    if (!b->by_mesh[mi].empty() && !p->meshes[mi].vec_lds) any_global = true;
    if (!b->by_mesh[mi].empty() && !p->meshes[mi].xu_lds) any_xu_global = true;
  }
  b->n_vec = 5 + 2 * m + (any_global ? 1 : 0);
  // per slot: the tile's vectors, then (if some mesh keeps them out of LDS) the current
  // cell's x_n and trial u
  b->slot_stride = ((int64_t)b->n_vec * T + (any_xu_global ? 2 : 0)) * 3 * b->n_pad_max;
  const size_t wbytes = (size_t)b->grid * b->slot_stride * sizeof(Real);
  if ((s = b->sched.alloc(wbytes, &b->work))) return s;
  HIP_TRY(hipMemset(b->work, 0, wbytes));
  void* cs;
  if ((s = b->sched.alloc((size_t)b->grid * T * sizeof(CellState), &cs))) return s;
  b->cstate = static_cast<CellState*>(cs);
  void* c;
  if ((s = b->sched.alloc(sizeof(int), &c))) return s;
  b->counter = static_cast<int*>(c);
  return NPFEM_OK;
}

npfem_status schedule(npfem_batch* b, int T, int m) {
  return b->plan->precision == NPFEM_FP64 ? batch_schedule<double>(b, T, m) : batch_schedule<float>(b, T, m);
}

int default_tile(const npfem_batch* b) {
  // as many cells per tile as keep every compute unit busy (the matrix product runs 3T
  // rows; T = 5, 10, 16 fill 16, 32, 48 rows)
  const int64_t want = 2 * (int64_t)b->plan->cu_count;
  return b->n_cells / 16 >= want ? 16 : (b->n_cells / 10 >= want ? 10 : 5);
}

}  // namespace

extern "C" {

npfem_status npfem_batch_create(npfem_plan* p, int64_t n_cells, const int32_t* cell_mesh,
                                npfem_batch** out, int64_t* n_vert_out) {
  if (!p || !out || (!cell_mesh && n_cells > 0)) return fail(NPFEM_E_INVALID, "batch_create: NULL pointer");
  *out = nullptr;
  if (n_cells < 1 || n_cells > (1ll << 30)) return fail(NPFEM_E_INVALID, "batch_create: n_cells out of range");
  HIP_TRY(hipSetDevice(p->device));
  auto b = std::make_unique<npfem_batch>();
  b->plan = p;
  b->n_cells = n_cells;
  const int nm = (int)p->meshes.size();
  std::vector<int64_t> voff(n_cells);
  std::vector<std::vector<int>> by_mesh(nm);
  int64_t v = 0;
  for (int64_t c = 0; c < n_cells; ++c) {
    const int mi = cell_mesh[c];
    if (mi < 0 || mi >= nm) return fail(NPFEM_E_INVALID, "batch_create: mesh index out of range");
    voff[c] = v;
    v += p->meshes[mi].mesh->n;
    by_mesh[mi].push_back((int)c);
  }
  b->n_vert = v;
  b->by_mesh = by_mesh;
  b->n_pad_max = 0;
  std::vector<int> mesh_n(nm);
  for (int i = 0; i < nm; ++i) {
    mesh_n[i] = p->meshes[i].mesh->n;
    if (!by_mesh[i].empty()) b->n_pad_max = std::max(b->n_pad_max, p->meshes[i].n_pad);
  }
  npfem_status s;
  std::vector<int> cm(cell_mesh, cell_mesh + n_cells);
  if ((s = b->buf.upload(voff.data(), voff.size(), &b->cell_voff))) return s;
  if ((s = b->buf.upload(cm.data(), cm.size(), &b->cell_mesh))) return s;
  if ((s = b->buf.upload(mesh_n.data(), mesh_n.size(), &b->mesh_n))) return s;
  const int T = p->prm.cells_per_tile > 0 ? p->prm.cells_per_tile : default_tile(b.get());
  if ((s = schedule(b.get(), T, p->prm.lbfgs_m))) return s;
  if (n_vert_out) *n_vert_out = v;
  *out = b.release();
  return NPFEM_OK;
}

void npfem_batch_destroy(npfem_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->plan->device);
  delete b;
}

}  // extern "C"

namespace {

npfem_status launch_step_now(npfem_batch* b, const void* x, const void* v, const void* f, void* x_out,
                             void* v_out, const void* u_guess, npfem_cell_stats* stats, hipStream_t s,
                             const void* u_delta = nullptr, int guess_only = 0, const void* col_q = nullptr,
                             const void* col_n = nullptr, double w_col = 0.0) {
  if (b->plan->precision == NPFEM_FP64) {
    auto a = make_args<double>(b);
    a.col_q = static_cast<const double*>(col_q);
    a.col_n = static_cast<const double*>(col_n);
    a.w_col = w_col;
    a.x = static_cast<const double*>(x);
    a.v = static_cast<const double*>(v);
    a.f = static_cast<const double*>(f);
    a.u_guess = static_cast<const double*>(u_guess);
    a.u_delta = static_cast<const double*>(u_delta);
    a.guess_only = guess_only;
    a.x_out = static_cast<double*>(x_out);
    a.v_out = static_cast<double*>(v_out);
    a.stats = stats;
    HIP_TRY(launch_step<double>(a, b->grid, b->lds, s, b->counter));
  } else {
    auto a = make_args<float>(b);
    a.col_q = static_cast<const float*>(col_q);
    a.col_n = static_cast<const float*>(col_n);
    a.w_col = w_col;
    a.x = static_cast<const float*>(x);
    a.v = static_cast<const float*>(v);
    a.f = static_cast<const float*>(f);
    a.u_guess = static_cast<const float*>(u_guess);
    a.u_delta = static_cast<const float*>(u_delta);
    a.guess_only = guess_only;
    a.x_out = static_cast<float*>(x_out);
    a.v_out = static_cast<float*>(v_out);
    a.stats = stats;
    HIP_TRY(launch_step<float>(a, b->grid, b->lds, s, b->counter));
  }
  return NPFEM_OK;
}

// Run `launch` on stream s, directly or through one of the batch's captured graphs: a
// graph is captured for a key (buffers, stream, network generation) not seen before,
// replacing the least recently used one when the cache is full, and replayed otherwise.
// The NULL stream cannot be captured, so launches on it are always direct.
template <typename F>
npfem_status run_maybe_graph(npfem_batch* b, const void* const (&key)[9], hipStream_t s, F launch) {
  if (!b->use_graph || s == nullptr) return launch();
  npfem_batch::GraphEntry* hit = nullptr;
  for (auto& g : b->graphs) {
    bool same = true;
    for (int k = 0; k < 9; ++k) same = same && key[k] == g.key[k];
    if (same) hit = &g;
  }
  if (!hit) {
    if ((int)b->graphs.size() >= npfem_batch::kGraphCache) {
      auto lru = std::min_element(b->graphs.begin(), b->graphs.end(),
                                  [](const auto& a, const auto& c) { return a.last_use < c.last_use; });
      (void)hipGraphExecDestroy(lru->exec);
      (void)hipGraphDestroy(lru->graph);
      b->graphs.erase(lru);
    }
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    npfem_status st = launch();
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &g);
    if (st) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    HIP_TRY(e);
    npfem_batch::GraphEntry ent;
    ent.graph = g;
    const hipError_t ei = hipGraphInstantiate(&ent.exec, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      (void)hipGraphDestroy(g);
      HIP_TRY(ei);
    }
    for (int k = 0; k < 9; ++k) ent.key[k] = key[k];
    b->graphs.push_back(ent);
    hit = &b->graphs.back();
    b->graph_captures += 1;
  } else {
    b->graph_replays += 1;
  }
  hit->last_use = ++b->graph_clock;
  HIP_TRY(hipGraphLaunch(hit->exec, s));
  return NPFEM_OK;
}

}  // namespace

extern "C" {

npfem_status npfem_step(npfem_batch* b, const void* x, const void* v, const void* f, void* x_out,
                        void* v_out, const void* u_guess, npfem_cell_stats* stats, void* stream) {
  if (!b || !x || !v || !f || !x_out || !v_out) return fail(NPFEM_E_INVALID, "step: NULL pointer");
  HIP_TRY(hipSetDevice(b->plan->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const void* const key[9] = {x, v, f, x_out, v_out, u_guess, stats, stream, nullptr};
  return run_maybe_graph(b, key, s, [&] { return launch_step_now(b, x, v, f, x_out, v_out, u_guess, stats, s); });
}

npfem_status npfem_step_contacts(npfem_batch* b, const void* x, const void* v, const void* f,
                                 const void* contact_q, const void* contact_n, double w_col, void* x_out,
                                 void* v_out, npfem_cell_stats* stats, void* stream) {
  if (!b || !x || !v || !f || !contact_q || !contact_n || !x_out || !v_out)
    return fail(NPFEM_E_INVALID, "step_contacts: NULL pointer");
  if (!(w_col >= 0.0) || !std::isfinite(w_col)) return fail(NPFEM_E_INVALID, "step_contacts: w_col must be >= 0");
  HIP_TRY(hipSetDevice(b->plan->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  return launch_step_now(b, x, v, f, x_out, v_out, nullptr, stats, s, nullptr, 0, contact_q, contact_n, w_col);
}

}  // extern "C"

namespace {

template <typename Real>
npfem_status collide_now(npfem_batch* b, const double* origin, const void* x, double cutoff, void* q, void* n,
                         hipStream_t s) {
  CollideArgs<Real> a{};
  a.meshes = static_cast<const MeshDev<Real>*>(b->plan->d_meshdev);
  a.cell_voff = b->cell_voff;
  a.cell_mesh = b->cell_mesh;
  a.mesh_n = b->mesh_n;
  a.origin = origin;
  a.x = static_cast<const Real*>(x);
  a.cutoff = cutoff;
  a.inv_h = 1.0 / cutoff;
  a.mask = (unsigned)(b->c_table - 1);
  a.count = b->c_count;
  a.start = b->c_start;
  a.fill = b->c_fill;
  a.bsum = b->c_bsum;
  a.vkey = b->c_vkey;
  a.vcell = b->c_vcell;
  a.sorted = b->c_sorted;
  a.normals = b->c_normals;
  a.q = static_cast<Real*>(q);
  a.n = static_cast<Real*>(n);
  a.n_contacts = b->c_ncontacts;
  HIP_TRY(launch_collide<Real>(a, (int)b->n_cells, b->n_vert, s));
  return NPFEM_OK;
}

}  // namespace

extern "C" {

npfem_status npfem_collisions_detect(npfem_batch* b, const double* cell_origin, const void* x, double cutoff,
                                     void* contact_q, void* contact_n, int64_t* n_contacts, void* stream) {
  if (!b || !cell_origin || !x || !contact_q || !contact_n) return fail(NPFEM_E_INVALID, "collisions_detect: NULL pointer");
  if (!(cutoff > 0.0) || !std::isfinite(cutoff)) return fail(NPFEM_E_INVALID, "collisions_detect: cutoff must be > 0");
  if (b->n_vert > (int64_t)1 << 31) return fail(NPFEM_E_UNSUPPORTED, "collisions_detect: more than 2^31 vertices");
  HIP_TRY(hipSetDevice(b->plan->device));
  if (!b->c_count) {
    int64_t table = 1024;
    while (table < 2 * b->n_vert) table *= 2;
    const int nb = collide_scan_blocks(table);
    void* p;
    npfem_status st;
    if ((st = b->cbuf.alloc(table * sizeof(unsigned), &p))) return st;
    b->c_count = static_cast<unsigned*>(p);
    if ((st = b->cbuf.alloc(table * sizeof(unsigned), &p))) return st;
    b->c_start = static_cast<unsigned*>(p);
    if ((st = b->cbuf.alloc(table * sizeof(unsigned), &p))) return st;
    b->c_fill = static_cast<unsigned*>(p);
    if ((st = b->cbuf.alloc((size_t)nb * sizeof(unsigned), &p))) return st;
    b->c_bsum = static_cast<unsigned*>(p);
    if ((st = b->cbuf.alloc(b->n_vert * sizeof(unsigned), &p))) return st;
    b->c_vkey = static_cast<unsigned*>(p);
    if ((st = b->cbuf.alloc(b->n_vert * sizeof(unsigned), &p))) return st;
    b->c_sorted = static_cast<unsigned*>(p);
    if ((st = b->cbuf.alloc(b->n_vert * sizeof(int), &p))) return st;
    b->c_vcell = static_cast<int*>(p);
    if ((st = b->cbuf.alloc(b->n_vert * 3 * sizeof(double), &p))) return st;
    b->c_normals = static_cast<double*>(p);
    if ((st = b->cbuf.alloc(sizeof(unsigned long long), &p))) return st;
    b->c_ncontacts = static_cast<unsigned long long*>(p);
    b->c_table = table;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  npfem_status st = b->plan->precision == NPFEM_FP64 ? collide_now<double>(b, cell_origin, x, cutoff, contact_q, contact_n, s)
                                                     : collide_now<float>(b, cell_origin, x, cutoff, contact_q, contact_n, s);
  if (st) return st;
  if (n_contacts) {
    unsigned long long c = 0;
    HIP_TRY(hipMemcpyAsync(&c, b->c_ncontacts, sizeof(c), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *n_contacts = (int64_t)c;
  }
  return NPFEM_OK;
}

npfem_status npfem_step_noalloc(npfem_batch* b, const void* x, const void* v, const void* f, void* x_out,
                                void* v_out, const void* u_guess, npfem_cell_stats* stats, void* stream) {
  if (!b || !x || !v || !f || !x_out || !v_out) return fail(NPFEM_E_INVALID, "step_noalloc: NULL pointer");
  HIP_TRY(hipSetDevice(b->plan->device));
  unsigned char* base = static_cast<unsigned char*>(scratch_of(b->plan->device));
  if (!base) return fail(NPFEM_E_HIP, "step_noalloc: no scratch address for this device");
  // layout: [tile counter: 256 B][cell states of the grid, 256-aligned][workspace slots]
  const size_t rs = b->plan->precision == NPFEM_FP64 ? sizeof(double) : sizeof(float);
  const size_t slot_bytes = (size_t)b->slot_stride * rs;
  const size_t cs_bytes = (size_t)b->T * sizeof(CellState);
  auto need = [&](int g) { return (size_t)256 + ((size_t)g * cs_bytes + 255) / 256 * 256 + (size_t)g * slot_bytes; };
  int grid = b->grid;
  while (grid > 0 && need(grid) > kScratchBytes) --grid;
  if (grid < 1)
    return fail(NPFEM_E_UNSUPPORTED, "step_noalloc: one workgroup's workspace (" + std::to_string(need(1)) +
                                         " B) exceeds the " + std::to_string(kScratchBytes) + " B scratch");
  int* counter = reinterpret_cast<int*>(base);
  CellState* cstate = reinterpret_cast<CellState*>(base + 256);
  unsigned char* work = base + 256 + ((size_t)grid * cs_bytes + 255) / 256 * 256;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (b->plan->precision == NPFEM_FP64) {
    auto a = make_args<double>(b);
    a.tile_counter = counter;
    a.cstate = cstate;
    a.work = reinterpret_cast<double*>(work);
    a.x = static_cast<const double*>(x);
    a.v = static_cast<const double*>(v);
    a.f = static_cast<const double*>(f);
    a.u_guess = static_cast<const double*>(u_guess);
    a.x_out = static_cast<double*>(x_out);
    a.v_out = static_cast<double*>(v_out);
    a.stats = stats;
    HIP_TRY(launch_step<double>(a, grid, b->lds, s, counter));
  } else {
    auto a = make_args<float>(b);
    a.tile_counter = counter;
    a.cstate = cstate;
    a.work = reinterpret_cast<float*>(work);
    a.x = static_cast<const float*>(x);
    a.v = static_cast<const float*>(v);
    a.f = static_cast<const float*>(f);
    a.u_guess = static_cast<const float*>(u_guess);
    a.x_out = static_cast<float*>(x_out);
    a.v_out = static_cast<float*>(v_out);
    a.stats = stats;
    HIP_TRY(launch_step<float>(a, grid, b->lds, s, counter));
  }
  return NPFEM_OK;
}

npfem_status npfem_first_guess(npfem_batch* b, const void* x, const void* v, const void* f, void* u_out,
                               void* stream) {
  if (!b || !x || !v || !f || !u_out) return fail(NPFEM_E_INVALID, "first_guess: NULL pointer");
  HIP_TRY(hipSetDevice(b->plan->device));
  return launch_step_now(b, x, v, f, u_out, u_out, nullptr, nullptr, static_cast<hipStream_t>(stream), nullptr, 1);
}

npfem_status npfem_batch_set_graph(npfem_batch* b, int32_t use_graph) {
  if (!b) return fail(NPFEM_E_INVALID, "batch_set_graph: NULL batch");
  b->use_graph = use_graph ? 1 : 0;
  if (!b->use_graph) b->drop_graph();
  return NPFEM_OK;
}

npfem_status npfem_batch_graph_counts(const npfem_batch* b, int64_t* captures, int64_t* replays) {
  if (!b) return fail(NPFEM_E_INVALID, "batch_graph_counts: NULL batch");
  if (captures) *captures = b->graph_captures;
  if (replays) *replays = b->graph_replays;
  return NPFEM_OK;
}

npfem_status npfem_batch_schedule(npfem_batch* b, int32_t cells_per_tile, int32_t lbfgs_m) {
  if (!b) return fail(NPFEM_E_INVALID, "batch_schedule: NULL batch");
  if (cells_per_tile < 1 || cells_per_tile > kMaxTile) return fail(NPFEM_E_INVALID, "batch_schedule: cells_per_tile must be in [1, 21]");
  if (lbfgs_m < 0 || lbfgs_m > kMaxHistory) return fail(NPFEM_E_INVALID, "batch_schedule: lbfgs_m must be in [0, 8]");
  HIP_TRY(hipSetDevice(b->plan->device));
  return schedule(b, cells_per_tile, lbfgs_m);
}

npfem_status npfem_batch_get_schedule(const npfem_batch* b, int32_t* cells_per_tile, int32_t* lbfgs_m,
                                      int32_t* grid_blocks, int32_t* n_tiles) {
  if (!b) return fail(NPFEM_E_INVALID, "batch_get_schedule: NULL batch");
  if (cells_per_tile) *cells_per_tile = b->T;
  if (lbfgs_m) *lbfgs_m = b->m;
  if (grid_blocks) *grid_blocks = b->grid;
  if (n_tiles) *n_tiles = b->n_tiles;
  return NPFEM_OK;
}

npfem_status npfem_batch_autotune(npfem_batch* b, const void* x, const void* v, const void* f, void* x_scratch,
                                  void* v_scratch, int32_t max_lbfgs_m, void* stream, double* best_ms) {
  if (!b || !x || !v || !f || !x_scratch || !v_scratch) return fail(NPFEM_E_INVALID, "batch_autotune: NULL pointer");
  if (max_lbfgs_m < 0 || max_lbfgs_m > kMaxHistory) return fail(NPFEM_E_INVALID, "batch_autotune: bad max_lbfgs_m");
  HIP_TRY(hipSetDevice(b->plan->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int use_graph = b->use_graph;
  b->use_graph = 0;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  double best = 1e300;
  const int T0 = b->T, m0 = b->m;
  int bT = T0, bm = m0;
  // tiles of 2 or 3 cells only for batches that leave workgroups idle at 5 cells per tile
  const int Ts[] = {2, 3, 5, 10, 16, 21};
  const int ms[] = {2, 3, 5, 8};
  const bool small = b->n_cells < 5 * 2 * (int64_t)b->plan->cu_count;
  npfem_status st = NPFEM_OK;
  for (int T : Ts) {
    if (T < 5 && !small) continue;
    if ((int64_t)T > b->n_cells && T != 5) continue;
    for (int m : ms) {
      if (m > max_lbfgs_m && !(m == 2 && max_lbfgs_m < 2)) continue;
      const int mm = std::min(m, max_lbfgs_m);
      if ((st = schedule(b, T, mm))) break;
      // one step to warm up, one timed
      if ((st = launch_step_now(b, x, v, f, x_scratch, v_scratch, nullptr, nullptr, s))) break;
      (void)hipEventRecord(e0, s);
      if ((st = launch_step_now(b, x, v, f, x_scratch, v_scratch, nullptr, nullptr, s))) break;
      (void)hipEventRecord(e1, s);
      if (hipEventSynchronize(e1) != hipSuccess) { st = fail(NPFEM_E_HIP, "batch_autotune: event sync failed"); break; }
      float ms_ = 0.f;
      (void)hipEventElapsedTime(&ms_, e0, e1);
      if (ms_ < best) {
        best = ms_;
        bT = T;
        bm = mm;
      }
      if (mm != m) break;
    }
    if (st) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->use_graph = use_graph;
  if (st) {
    const std::string msg = g_err;
    (void)schedule(b, T0, m0);               // leave the batch on the schedule it had
    g_err = msg;
    return st;
  }
  if (best_ms) *best_ms = best;
  return schedule(b, bT, bm);
}

npfem_status npfem_stats_accumulate(const npfem_cell_stats* st, int64_t n, npfem_stats_total* tot, void* stream) {
  if (!st || !tot || n < 0) return fail(NPFEM_E_INVALID, "stats_accumulate: NULL pointer or negative count");
  if (n == 0) return NPFEM_OK;
  HIP_TRY(launch_stats_accumulate(st, n, tot, static_cast<hipStream_t>(stream)));
  return NPFEM_OK;
}

npfem_status npfem_stats_reset(npfem_stats_total* tot, void* stream) {
  if (!tot) return fail(NPFEM_E_INVALID, "stats_reset: NULL pointer");
  HIP_TRY(launch_stats_reset(tot, static_cast<hipStream_t>(stream)));
  return NPFEM_OK;
}

npfem_status npfem_eval(npfem_batch* b, const void* x, const void* v, const void* f, const void* u,
                        void* grad, double* terms, void* stream) {
  if (!b || !x || !v || !f || !u || !grad || !terms) return fail(NPFEM_E_INVALID, "eval: NULL pointer");
  HIP_TRY(hipSetDevice(b->plan->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool fp64 = b->plan->precision == NPFEM_FP64;
  const size_t rs = fp64 ? 8 : 4;
  if (!b->eval_scratch) {
    npfem_status st = b->buf.alloc((size_t)b->n_cells * 12 * b->n_pad_max * rs, &b->eval_scratch);
    if (st) return st;
  }
  if (fp64) {
    auto a = make_args<double>(b);
    a.x = static_cast<const double*>(x);
    a.v = static_cast<const double*>(v);
    a.f = static_cast<const double*>(f);
    a.work = static_cast<double*>(b->eval_scratch);
    HIP_TRY(launch_eval<double>(a, (int)b->n_cells, static_cast<const double*>(u), static_cast<double*>(grad),
                                terms, b->lds, s));
  } else {
    auto a = make_args<float>(b);
    a.x = static_cast<const float*>(x);
    a.v = static_cast<const float*>(v);
    a.f = static_cast<const float*>(f);
    a.work = static_cast<float*>(b->eval_scratch);
    HIP_TRY(launch_eval<float>(a, (int)b->n_cells, static_cast<const float*>(u), static_cast<float*>(grad),
                               terms, b->lds, s));
  }
  return NPFEM_OK;
}

npfem_status npfem_apply_inverse(npfem_plan* p, int32_t mi, int32_t which, const void* in, void* out,
                                 int32_t rows, int32_t* n_pad_out, void* stream) {
  if (!p) return fail(NPFEM_E_INVALID, "apply_inverse: NULL plan");
  if (mi < 0 || mi >= (int)p->meshes.size()) return fail(NPFEM_E_INVALID, "apply_inverse: bad mesh index");
  if (which != 0 && which != 1) return fail(NPFEM_E_INVALID, "apply_inverse: which must be 0 or 1");
  const MeshPlan& mp = p->meshes[mi];
  if (n_pad_out) *n_pad_out = mp.n_pad;
  if (rows == 0) return NPFEM_OK;
  if (!in || !out || rows < 0) return fail(NPFEM_E_INVALID, "apply_inverse: bad buffers or rows");
  HIP_TRY(hipSetDevice(p->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (p->precision == NPFEM_FP64) {
    const double* A = which == 0 ? mp.dev64.hinv : mp.dev64.minv;
    HIP_TRY(launch_apply_inverse<double>(A, mp.n_pad, static_cast<const double*>(in), static_cast<double*>(out),
                                         rows, s));
  } else if (p->prm.inverse_bf16 == 2) {
    const uint16_t* A = which == 0 ? mp.dev32.hinv_bf : mp.dev32.minv_bf;
    const float* dg = which == 0 ? mp.dev32.hinv_diag : mp.dev32.minv_diag;
    HIP_TRY(launch_apply_inverse_band(A, dg, mp.dev32.bperm, mp.dev32.bband + (size_t)which * 2 * (mp.n_pad / 16),
                                      mp.n_pad, static_cast<const float*>(in), static_cast<float*>(out), rows, s));
  } else if (p->prm.inverse_bf16) {
    const uint16_t* A = which == 0 ? mp.dev32.hinv_bf : mp.dev32.minv_bf;
    const float* dg = which == 0 ? mp.dev32.hinv_diag : mp.dev32.minv_diag;
    HIP_TRY(launch_apply_inverse_bf16(A, dg, mp.n_pad, static_cast<const float*>(in), static_cast<float*>(out),
                                      rows, s));
  } else {
    const float* A = which == 0 ? mp.dev32.hinv : mp.dev32.minv;
    HIP_TRY(launch_apply_inverse<float>(A, mp.n_pad, static_cast<const float*>(in), static_cast<float*>(out),
                                        rows, s));
  }
  return NPFEM_OK;
}

int64_t npfem_solve_factor_workspace(const npfem_plan* p, int32_t mi, int32_t rows) {
  if (!p || mi < 0 || mi >= (int)p->meshes.size() || rows < 0) return -1;
  const int rb = p->precision == NPFEM_FP64 ? (int)sizeof(double) : (int)sizeof(float);
  return (int64_t)band_solve_work_bytes(p->meshes[mi].n_pad, rows, rb);
}

npfem_status npfem_solve_factor(npfem_plan* p, int32_t mi, int32_t which, const void* in, void* out, int32_t rows,
                                void* work, int64_t work_bytes, int32_t* bandwidth_out, void* stream) {
  if (!p) return fail(NPFEM_E_INVALID, "solve_factor: NULL plan");
  if (mi < 0 || mi >= (int)p->meshes.size()) return fail(NPFEM_E_INVALID, "solve_factor: bad mesh index");
  if (which != 0 && which != 1) return fail(NPFEM_E_INVALID, "solve_factor: which must be 0 or 1");
  const MeshPlan& mp = p->meshes[mi];
  const bool fp64 = p->precision == NPFEM_FP64;
  if (bandwidth_out) *bandwidth_out = fp64 ? mp.fac64.b : mp.fac32.b;
  if (!(fp64 ? (const void*)mp.fac64.F[0] : (const void*)mp.fac32.FA[0]))
    return fail(NPFEM_E_UNSUPPORTED, "solve_factor: the factor's band is too wide for the substitution kernel");
  if (rows == 0) return NPFEM_OK;
  if (!in || !out || !work || rows < 0) return fail(NPFEM_E_INVALID, "solve_factor: bad buffers or rows");
  if (work_bytes < npfem_solve_factor_workspace(p, mi, rows))
    return fail(NPFEM_E_INVALID, "solve_factor: workspace too small");
  HIP_TRY(hipSetDevice(p->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (fp64)
    HIP_TRY(launch_band_solve<double>(mp.fac64, which, mp.n_pad, static_cast<const double*>(in),
                                      static_cast<double*>(out), static_cast<double*>(work), rows, s));
  else
    HIP_TRY(launch_band_solve<float>(mp.fac32, which, mp.n_pad, static_cast<const float*>(in),
                                     static_cast<float*>(out), static_cast<float*>(work), rows, s));
  return NPFEM_OK;
}

npfem_status npfem_drag_forces(npfem_batch* b, const void* x, const void* v, const double* zeta,
                               const double* rate, const double* origin, double umax, double radius,
                               double ay, double az, void* f, void* stream) {
  if (!b || !x || !v || !zeta || !rate || !origin || !f) return fail(NPFEM_E_INVALID, "drag_forces: NULL pointer");
  HIP_TRY(hipSetDevice(b->plan->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (b->plan->precision == NPFEM_FP64)
    HIP_TRY(launch_drag<double>(static_cast<const double*>(x), static_cast<const double*>(v), b->cell_voff,
                                b->cell_mesh, b->mesh_n, (int)b->n_cells, zeta, rate, origin, umax, radius,
                                ay, az, static_cast<double*>(f), s));
  else
    HIP_TRY(launch_drag<float>(static_cast<const float*>(x), static_cast<const float*>(v), b->cell_voff,
                               b->cell_mesh, b->mesh_n, (int)b->n_cells, zeta, rate, origin, umax, radius, ay,
                               az, static_cast<float*>(f), s));
  return NPFEM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------
// Learned warm start
// ---------------------------------------------------------------------------------

struct npfem_net {
  npfem_plan* plan = nullptr;
  uint64_t generation = 0;                  // unique per network created (keys captured graphs)
  NetLayout lay{};
  double force_floor = 1.0, shape_scale = 0.1;
  DeviceBuffers buf;                        // parameters, optimiser state, BF16 weights, meshes
  float* theta = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  uint16_t *We = nullptr, *Wl = nullptr, *WsT = nullptr, *WnT = nullptr, *Wd = nullptr;
  const NetMeshDev* d_meshes = nullptr;
  int n_pad_max = 0, nb_deg_max = 0;
  size_t fwd_lds = 0;                       // LDS of the resident forward variant (0: not used)
  size_t inf_lds = 0;                       // LDS of the resident inference (0: not used)
  int adam_t = 0;
  // inference scratch: per workgroup, features and two activation planes
  DeviceBuffers ibuf;
  int igrid = 0;
  uint16_t *ifeat = nullptr, *iH = nullptr;
  // training scratch, sized for the largest minibatch seen
  DeviceBuffers tbuf;
  int tcap = 0, bgrid = 0;
  uint16_t *tfeat = nullptr, *tH = nullptr, *tZ = nullptr, *dZ = nullptr;
  double *tframe = nullptr, *tloss = nullptr;
  float *tout = nullptr, *tdout = nullptr, *dH = nullptr, *Q = nullptr, *partial = nullptr;

  NetWeights weights() const {
    NetWeights w;
    w.lay = lay;
    w.force_floor = force_floor;
    w.shape_scale = shape_scale;
    w.theta = theta;
    w.We = We;
    w.Wl = Wl;
    w.WsT = WsT;
    w.WnT = WnT;
    w.Wd = Wd;
    return w;
  }
};

namespace {

bool net_config_ok(const npfem_net_config* c) {
  return c && c->hidden == kNetH && c->layers >= 1 && c->layers <= kNetMaxLayers && c->force_floor > 0.0 &&
         c->shape_scale > 0.0 && std::isfinite(c->force_floor) && std::isfinite(c->shape_scale);
}

npfem_status net_upload_params(npfem_net* net, const float* theta, hipStream_t s) {
  for (int64_t i = 0; i < net->lay.count; ++i)
    if (!std::isfinite(theta[i])) return fail(NPFEM_E_INVALID, "net: non-finite parameter");
  HIP_TRY(hipMemcpy(net->theta, theta, net->lay.count * sizeof(float), hipMemcpyHostToDevice));
  HIP_TRY(launch_fill_zero(net->adam_m, net->lay.count, s));
  HIP_TRY(launch_fill_zero(net->adam_v, net->lay.count, s));
  HIP_TRY(launch_net_pack(net->weights(), net->We, net->Wl, net->WsT, net->WnT, net->Wd, s));
  HIP_TRY(hipStreamSynchronize(s));
  net->adam_t = 0;
  return NPFEM_OK;
}

npfem_status net_check_batch(const npfem_net* net, const npfem_batch* b) {
  if (net->plan != b->plan) return fail(NPFEM_E_INVALID, "net: batch belongs to another plan");
  return NPFEM_OK;
}

npfem_status net_inference_scratch(npfem_net* net) {
  if (net->ibuf.ptrs.size()) return NPFEM_OK;
  net->igrid = 4 * net->plan->cu_count;
  const size_t np = (size_t)net->n_pad_max;
  void* p;
  npfem_status s;
  if ((s = net->ibuf.alloc((size_t)net->igrid * np * kNetFeatPad * 2, &p))) return s;
  net->ifeat = static_cast<uint16_t*>(p);
  if ((s = net->ibuf.alloc((size_t)net->igrid * 2 * np * kNetH * 2, &p))) return s;
  net->iH = static_cast<uint16_t*>(p);
  return NPFEM_OK;
}

npfem_status net_training_scratch(npfem_net* net, int cells) {
  if (cells <= net->tcap) return NPFEM_OK;
  net->tbuf.release();
  net->tcap = 0;
  const size_t np = (size_t)net->n_pad_max, L1 = (size_t)net->lay.layers + 1, C = (size_t)cells;
  net->bgrid = std::max(1, std::min(cells, net->plan->cu_count));
  const size_t G = (size_t)net->bgrid;
  void* p;
  npfem_status s;
  if ((s = net->tbuf.alloc(C * np * kNetFeatPad * 2, &p))) return s;
  net->tfeat = static_cast<uint16_t*>(p);
  if ((s = net->tbuf.alloc(C * L1 * np * kNetH * 2, &p))) return s;
  net->tH = static_cast<uint16_t*>(p);
  if ((s = net->tbuf.alloc(C * L1 * np * kNetH * 2, &p))) return s;
  net->tZ = static_cast<uint16_t*>(p);
  if ((s = net->tbuf.alloc(C * 12 * sizeof(double), &p))) return s;
  net->tframe = static_cast<double*>(p);
  if ((s = net->tbuf.alloc(C * sizeof(double), &p))) return s;
  net->tloss = static_cast<double*>(p);
  if ((s = net->tbuf.alloc(C * np * 3 * sizeof(float), &p))) return s;
  net->tout = static_cast<float*>(p);
  if ((s = net->tbuf.alloc(C * np * 3 * sizeof(float), &p))) return s;
  net->tdout = static_cast<float*>(p);
  if ((s = net->tbuf.alloc(G * 2 * np * kNetH * sizeof(float), &p))) return s;
  net->dH = static_cast<float*>(p);
  if ((s = net->tbuf.alloc(G * np * kNetH * sizeof(float), &p))) return s;
  net->Q = static_cast<float*>(p);
  if ((s = net->tbuf.alloc(G * np * kNetH * 2, &p))) return s;
  net->dZ = static_cast<uint16_t*>(p);
  if ((s = net->tbuf.alloc(G * (size_t)net->lay.count * sizeof(float), &p))) return s;
  net->partial = static_cast<float*>(p);
  net->tcap = cells;
  return NPFEM_OK;
}

template <typename Real>
NetFwdArgs<Real> net_fwd_args(const npfem_net* net, const npfem_batch* b, const void* x, const void* v,
                              const void* f) {
  NetFwdArgs<Real> a{};
  a.W = net->weights();
  a.meshes = net->d_meshes;
  a.cell_voff = b->cell_voff;
  a.cell_mesh = b->cell_mesh;
  a.h = b->plan->dt;
  a.x = static_cast<const Real*>(x);
  a.v = static_cast<const Real*>(v);
  a.f = static_cast<const Real*>(f);
  a.S.n_pad_max = net->n_pad_max;
  a.nb_deg_max = net->nb_deg_max;
  return a;
}

// persistent workgroups of the forward launch: the LDS-resident variant runs one per CU
int net_fwd_grid(const npfem_net* net, int n_cells) {
  const int g = net->fwd_lds ? net->plan->cu_count : 4 * net->plan->cu_count;
  return std::max(1, std::min(g, n_cells));
}

template <typename Real>
npfem_status net_infer_now(npfem_net* net, npfem_batch* b, const void* x, const void* v, const void* f,
                           void* delta, hipStream_t s) {
  auto a = net_fwd_args<Real>(net, b, x, v, f);
  a.S.feat = net->ifeat;
  a.S.H = net->iH;
  a.S.train = 0;
  a.n_cells = (int)b->n_cells;
  a.delta = static_cast<Real*>(delta);
  if (net->inf_lds) {                       // resident inference: one workgroup per CU
    a.cframe = b->net_frames;
    HIP_TRY(launch_net_infer<Real>(a, std::max(1, std::min(net->plan->cu_count, (int)b->n_cells)), net->inf_lds, s));
    return NPFEM_OK;
  }
  HIP_TRY(launch_net_forward<Real>(a, std::min(net->igrid, net_fwd_grid(net, (int)b->n_cells)), net->fwd_lds, s));
  return NPFEM_OK;
}

// the batch's frame buffer of the resident inference, allocated before any launch (and
// so before a graph capture)
npfem_status net_batch_frames(const npfem_net* net, npfem_batch* b) {
  if (!net->inf_lds || b->net_frames) return NPFEM_OK;
  void* p;
  npfem_status s;
  if ((s = b->dbuf.alloc((size_t)b->n_cells * kNetFrame * sizeof(double), &p))) return s;
  b->net_frames = static_cast<double*>(p);
  return NPFEM_OK;
}

npfem_status net_infer_any(npfem_net* net, npfem_batch* b, const void* x, const void* v, const void* f,
                           void* delta, hipStream_t s) {
  return b->plan->precision == NPFEM_FP64 ? net_infer_now<double>(net, b, x, v, f, delta, s)
                                          : net_infer_now<float>(net, b, x, v, f, delta, s);
}

template <typename Real>
npfem_status net_loss_grad_now(npfem_net* net, npfem_batch* b, const int32_t* cells, int n_cells,
                               const void* x, const void* v, const void* f, const void* x_next, const void* u0,
                               double* loss_out, float* grad_out, hipStream_t s) {
  // The listed cells are copied to the host and range-checked before any kernel reads
  // them; their vertex count gives the mean.
  int64_t nodes = 0;
  if (cells) {
    std::vector<int32_t> hc(n_cells);
    HIP_TRY(hipMemcpyAsync(hc.data(), cells, n_cells * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int k = 0; k < n_cells; ++k) {
      if (hc[k] < 0 || hc[k] >= b->n_cells) return fail(NPFEM_E_INVALID, "net_loss_grad: cell index out of range");
    }
    std::vector<int> cm(b->n_cells);
    for (size_t mi = 0; mi < b->by_mesh.size(); ++mi)
      for (int c : b->by_mesh[mi]) cm[c] = (int)mi;
    for (int k = 0; k < n_cells; ++k) nodes += b->plan->meshes[cm[hc[k]]].mesh->n;
  } else {
    for (size_t mi = 0; mi < b->by_mesh.size(); ++mi)
      for (int c : b->by_mesh[mi])
        if (c < n_cells) nodes += b->plan->meshes[mi].mesh->n;
  }
  auto a = net_fwd_args<Real>(net, b, x, v, f);
  a.S.feat = net->tfeat;
  a.S.H = net->tH;
  a.S.Z = net->tZ;
  a.S.frame = net->tframe;
  a.S.out = net->tout;
  a.S.train = 1;
  a.cells = cells;
  a.n_cells = n_cells;
  HIP_TRY(launch_net_forward<Real>(a, net_fwd_grid(net, n_cells), net->fwd_lds, s));
  NetLossArgs<Real> la{};
  la.S = a.S;
  la.meshes = net->d_meshes;
  la.cell_voff = b->cell_voff;
  la.cell_mesh = b->cell_mesh;
  la.cells = cells;
  la.n_cells = n_cells;
  la.inv_count = 1.0 / (3.0 * (double)nodes);
  la.x = static_cast<const Real*>(x);
  la.x_next = static_cast<const Real*>(x_next);
  la.u0 = static_cast<const Real*>(u0);
  la.dout = net->tdout;
  la.cell_loss = net->tloss;
  HIP_TRY(launch_net_loss<Real>(la, s));
  NetBwdArgs ba{};
  ba.W = net->weights();
  ba.S = a.S;
  ba.meshes = net->d_meshes;
  ba.cell_mesh = b->cell_mesh;
  ba.cells = cells;
  ba.n_cells = n_cells;
  ba.dout = net->tdout;
  ba.dH = net->dH;
  ba.Q = net->Q;
  ba.dZ = net->dZ;
  ba.partial = net->partial;
  const int g = std::max(1, std::min(net->bgrid, n_cells));
  HIP_TRY(launch_fill_zero(net->partial, (int64_t)g * net->lay.count, s));
  HIP_TRY(launch_net_backward(ba, g, s));
  HIP_TRY(launch_net_reduce(net->partial, g, net->lay.count, grad_out, s));
  if (loss_out) {
    std::vector<double> cl(n_cells);
    HIP_TRY(hipMemcpyAsync(cl.data(), net->tloss, n_cells * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    double t = 0.0;
    for (double c : cl) t += c;
    *loss_out = t * la.inv_count;
  }
  return NPFEM_OK;
}

}  // namespace

extern "C" {

void npfem_net_config_default(npfem_net_config* c) {
  if (!c) return;
  c->hidden = kNetH;
  c->layers = 4;
  c->force_floor = 1.0;
  c->shape_scale = 0.1;
}

int64_t npfem_net_param_count(const npfem_net_config* c) {
  if (!net_config_ok(c)) return -1;
  return net_layout(c->layers).count;
}

npfem_status npfem_net_create(npfem_plan* p, const npfem_net_config* cfg, const float* theta, npfem_net** out) {
  if (!p || !cfg || !theta || !out) return fail(NPFEM_E_INVALID, "net_create: NULL pointer");
  *out = nullptr;
  if (!net_config_ok(cfg)) return fail(NPFEM_E_INVALID, "net_create: hidden must be 64, layers 1..8, scales > 0");
  HIP_TRY(hipSetDevice(p->device));
  auto net = std::make_unique<npfem_net>();
  net->plan = p;
  static std::atomic<uint64_t> next_generation{1};
  net->generation = next_generation.fetch_add(1);
  net->lay = net_layout(cfg->layers);
  net->force_floor = cfg->force_floor;
  net->shape_scale = cfg->shape_scale;
  const int64_t P = net->lay.count;
  void* q;
  npfem_status s;
  for (float** dst : {&net->theta, &net->adam_m, &net->adam_v}) {
    if ((s = net->buf.alloc(P * sizeof(float), &q))) return s;
    *dst = static_cast<float*>(q);
  }
  const size_t nL = (size_t)cfg->layers * kNetH * kNetH;
  if ((s = net->buf.alloc((size_t)kNetH * kNetFeatPad * 2, &q))) return s;
  net->We = static_cast<uint16_t*>(q);
  if ((s = net->buf.alloc(2 * nL * 2, &q))) return s;
  net->Wl = static_cast<uint16_t*>(q);
  if ((s = net->buf.alloc(nL * 2, &q))) return s;
  net->WsT = static_cast<uint16_t*>(q);
  if ((s = net->buf.alloc(nL * 2, &q))) return s;
  net->WnT = static_cast<uint16_t*>(q);
  if ((s = net->buf.alloc(3 * kNetH * 2, &q))) return s;
  net->Wd = static_cast<uint16_t*>(q);
  // per mesh type: rest positions about the mass-weighted centroid, masses, neighbours
  std::vector<NetMeshDev> md(p->meshes.size());
  for (size_t mi = 0; mi < p->meshes.size(); ++mi) {
    const MeshPlan& mp = p->meshes[mi];
    const npfem_mesh* m = mp.mesh;
    NetMeshDev& d = md[mi];
    d.n = m->n;
    d.n_pad = mp.n_pad;
    net->n_pad_max = std::max(net->n_pad_max, mp.n_pad);
    double ms = 0.0, c[3] = {0, 0, 0};
    for (int i = 0; i < m->n; ++i) {
      ms += mp.mass[i];
      for (int k = 0; k < 3; ++k) c[k] += mp.mass[i] * m->X[3 * i + k];
    }
    std::vector<double> Xc(3 * (size_t)m->n);
    double rho = 0.0;
    for (int i = 0; i < m->n; ++i) {
      double r2 = 0.0;
      for (int k = 0; k < 3; ++k) {
        Xc[3 * i + k] = m->X[3 * i + k] - c[k] / ms;
        r2 += Xc[3 * i + k] * Xc[3 * i + k];
      }
      rho = std::max(rho, std::sqrt(r2));
    }
    for (int i = 0; i < m->n; ++i)
      if (m->nb_ptr[i + 1] == m->nb_ptr[i]) return fail(NPFEM_E_MESH, "net_create: vertex without neighbours");
    d.inv_rho = 1.0 / rho;
    d.mass_sum = ms;
    d.mass_mean = ms / m->n;
    d.nb_ptr = p->precision == NPFEM_FP64 ? mp.dev64.nb_ptr : mp.dev32.nb_ptr;
    d.nb_idx = p->precision == NPFEM_FP64 ? mp.dev64.nb_idx : mp.dev32.nb_idx;
    d.nb_ell = p->precision == NPFEM_FP64 ? mp.dev64.nb_ell : mp.dev32.nb_ell;
    d.nb_deg = p->precision == NPFEM_FP64 ? mp.dev64.nb_deg : mp.dev32.nb_deg;
    net->nb_deg_max = std::max(net->nb_deg_max, d.nb_deg);
    if ((s = net->buf.upload(Xc.data(), Xc.size(), &d.Xc))) return s;
    if ((s = net->buf.upload(mp.mass.data(), mp.mass.size(), &d.mass))) return s;
  }
  if ((s = net->buf.upload(md.data(), md.size(), &net->d_meshes))) return s;
  net->fwd_lds = std::getenv("NPFEM_NET_NO_LDS") ? 0 : net_forward_lds_bytes(net->n_pad_max, net->nb_deg_max);
  net->inf_lds = std::getenv("NPFEM_NET_NO_LDS") ? 0 : net_infer_lds_bytes(net->n_pad_max, net->nb_deg_max);
  if ((s = net_upload_params(net.get(), theta, nullptr))) return s;
  *out = net.release();
  return NPFEM_OK;
}

void npfem_net_destroy(npfem_net* net) {
  if (!net) return;
  (void)hipSetDevice(net->plan->device);
  delete net;
}

npfem_status npfem_net_set_params(npfem_net* net, const float* theta) {
  if (!net || !theta) return fail(NPFEM_E_INVALID, "net_set_params: NULL pointer");
  HIP_TRY(hipSetDevice(net->plan->device));
  HIP_TRY(hipDeviceSynchronize());
  return net_upload_params(net, theta, nullptr);
}

npfem_status npfem_net_get_params(const npfem_net* net, float* theta) {
  if (!net || !theta) return fail(NPFEM_E_INVALID, "net_get_params: NULL pointer");
  HIP_TRY(hipSetDevice(net->plan->device));
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(theta, net->theta, net->lay.count * sizeof(float), hipMemcpyDeviceToHost));
  return NPFEM_OK;
}

npfem_status npfem_net_infer(npfem_net* net, npfem_batch* b, const void* x, const void* v, const void* f,
                             void* delta, void* stream) {
  if (!net || !b || !x || !v || !f || !delta) return fail(NPFEM_E_INVALID, "net_infer: NULL pointer");
  npfem_status s;
  if ((s = net_check_batch(net, b))) return s;
  HIP_TRY(hipSetDevice(b->plan->device));
  if ((s = net_inference_scratch(net))) return s;
  if ((s = net_batch_frames(net, b))) return s;
  return net_infer_any(net, b, x, v, f, delta, static_cast<hipStream_t>(stream));
}

npfem_status npfem_step_learned(npfem_batch* b, npfem_net* net, const void* x, const void* v, const void* f,
                                void* x_out, void* v_out, npfem_cell_stats* stats, void* stream) {
  if (!net || !b || !x || !v || !f || !x_out || !v_out) return fail(NPFEM_E_INVALID, "step_learned: NULL pointer");
  npfem_status s;
  if ((s = net_check_batch(net, b))) return s;
  HIP_TRY(hipSetDevice(b->plan->device));
  if ((s = net_inference_scratch(net))) return s;
  if ((s = net_batch_frames(net, b))) return s;
  if (!b->delta) {
    const size_t bytes = (size_t)b->n_vert * 3 * (b->plan->precision == NPFEM_FP64 ? 8 : 4);
    if ((s = b->dbuf.alloc(bytes, &b->delta))) return s;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  // the network enters the key by its generation, never by its address (a new network may
  // be allocated where a destroyed one was)
  const void* const key[9] = {x, v, f, x_out, v_out, b->delta, stats, stream,
                              reinterpret_cast<const void*>(static_cast<uintptr_t>(net->generation))};
  return run_maybe_graph(b, key, st, [&]() -> npfem_status {
    npfem_status r;
    if ((r = net_infer_any(net, b, x, v, f, b->delta, st))) return r;
    return launch_step_now(b, x, v, f, x_out, v_out, nullptr, stats, st, b->delta, 0);
  });
}

npfem_status npfem_net_loss_grad(npfem_net* net, npfem_batch* b, const int32_t* cells, int32_t n_cells,
                                 const void* x, const void* v, const void* f, const void* x_next, const void* u0,
                                 double* loss_out, float* grad_out, void* stream) {
  if (!net || !b || !x || !v || !f || !x_next || !u0 || !grad_out)
    return fail(NPFEM_E_INVALID, "net_loss_grad: NULL pointer");
  if (n_cells < 1 || (!cells && n_cells > b->n_cells)) return fail(NPFEM_E_INVALID, "net_loss_grad: bad cell count");
  npfem_status s;
  if ((s = net_check_batch(net, b))) return s;
  HIP_TRY(hipSetDevice(b->plan->device));
  if ((s = net_training_scratch(net, n_cells))) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  return b->plan->precision == NPFEM_FP64
             ? net_loss_grad_now<double>(net, b, cells, n_cells, x, v, f, x_next, u0, loss_out, grad_out, st)
             : net_loss_grad_now<float>(net, b, cells, n_cells, x, v, f, x_next, u0, loss_out, grad_out, st);
}

npfem_status npfem_net_adam_step(npfem_net* net, const float* grad, double lr, double b1, double b2, double eps,
                                 void* stream) {
  if (!net || !grad) return fail(NPFEM_E_INVALID, "net_adam_step: NULL pointer");
  if (!(lr > 0.0) || !(b1 >= 0.0 && b1 < 1.0) || !(b2 >= 0.0 && b2 < 1.0) || !(eps > 0.0))
    return fail(NPFEM_E_INVALID, "net_adam_step: bad hyper-parameters");
  HIP_TRY(hipSetDevice(net->plan->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  net->adam_t += 1;
  HIP_TRY(launch_net_adam(net->theta, net->adam_m, net->adam_v, grad, net->lay.count, lr, b1, b2, eps,
                          net->adam_t, s));
  HIP_TRY(launch_net_pack(net->weights(), net->We, net->Wl, net->WsT, net->WnT, net->Wd, s));
  return NPFEM_OK;
}

}  // extern "C"
