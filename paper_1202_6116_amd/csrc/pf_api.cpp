// Host layer of the C ABI in include/pf.h: configuration checks, workspace
// carving, the FEM operator tables, the conjugate-gradient drivers and the
// time-step loop.  All arithmetic on fields runs in the HIP kernels of
// pf_kernels.hip; this file only orders launches and reads back the
// convergence scalars.
#include "pf.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <condition_variable>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "pf_internal.h"

namespace pf {

MgHierarchy build_mg(const pf_config& cfg, const FemTables& tb);
MgHierarchy build_mg_phi(const pf_config& cfg);
std::vector<MgLevel> mg_plan(const pf_config& cfg);
std::vector<MgLevel> mg_plan_phi(const pf_config& cfg);
template <typename T>
hipError_t launch_mg_fine(const Dims& d, const TileMap& tm, const FemTables* tb, bool gen, const double* dinv, int mode,
                          double omega, const T* x, const T* b, T* out, const MgCoarse<T>& mc, const CgScalars* sc,
                          double* partials, int pstride, int poff, hipStream_t s);
template <typename T>
hipError_t launch_mg_level(const Dims& d, int nc, const double* tab, const double* dinv, int mode, double omega,
                           const T* x, const T* b, T* out, const CgScalars* sc, int top_fixed, hipStream_t s);
template <typename T>
hipError_t launch_mg_scale(const Dims& d, int nc, const double* dinv, double omega, const T* b, T* x,
                           const CgScalars* sc, hipStream_t s);
template <typename T>
hipError_t launch_mg_restrict(const Dims& df, const Dims& dc, int nc, int cx, int cy, const MgZ* zmap,
                              const int* zfine, const T* rf, T* bc, const CgScalars* sc, int zoff, int fnz,
                              int ftop_fixed, int ctop_fixed, hipStream_t s);
template <typename T>
hipError_t launch_mg_prolong(const Dims& df, const Dims& dc, int nc, int cx, int cy, const MgZ* zmap, const T* xc,
                             T* xf, const CgScalars* sc, int zoff, int ftop_fixed, int ctop_fixed, const T* bf,
                             const double* dinv, double omega, hipStream_t s);
template <typename T>
hipError_t launch_mg_dense(const Dims& d, int nc, int n, const double* M, const T* b, T* x, const CgScalars* sc,
                           hipStream_t s);
template <typename T>
hipError_t launch_mgp_fine(const Dims& d, const TileMap& tm, const Coefs<T>& cf, const double* dinv, int mode,
                           double omega, const T* x, const T* b, T* out, const MgCoarse<T>& mc,
                           const uint8_t* emask, const CgScalars* sc, double* partials, int pstride, int poff,
                           hipStream_t s);

// kernel launchers (pf_kernels.hip)
int node_blocks(const Dims& d);
TileMap make_tile_map(const Dims& d, int ty, int target);
template <typename T> hipError_t launch_fill(T* a, int64_t n, T v, hipStream_t s);
template <typename T, typename U> hipError_t launch_convert(const T* a, U* b, int64_t n, hipStream_t s);
template <typename T> hipError_t launch_cg_finish(T* x, const T* p, int64_t n, const CgScalars* sc, hipStream_t s);
hipError_t launch_cg_reduce(const double* partials, int nblocks, int nv, CgScalars* sc, int mode, double tol,
                            int maxit, hipStream_t s, double tol2, double* out);
hipError_t launch_refine_update(double* x64, float* x32, const float* d, const float* p, const CgScalars* sc,
                                int64_t n, hipStream_t s);
hipError_t launch_extrapolate(double* x, const ExtrapRing& ring, int64_t n, hipStream_t s);
hipError_t launch_extrap_score(const double* x, const ExtrapRing& ring, const ExtrapScore& sc, int64_t n,
                               hipStream_t s);
template <typename T, typename S, typename R>
hipError_t launch_poisson_setup(const Dims& d, const TileMap& tm, const Coefs<T>& cf, const S* P, const S* V, T cdt,
                                int with_P, int with_bc, const T* ghost_top, T phi_bottom, const uint8_t* emask,
                                T* x, R* r, R* p, R* dz, double* partials, hipStream_t s);
template <typename T>
hipError_t launch_poisson_cg_a(const Dims& d, const TileMap& tm, const Coefs<T>& cf, const T* r, const T* p_old,
                               T* p_new, T* x, const CgScalars* sc, double* partials, int unit_w, hipStream_t s);
template <typename T>
hipError_t launch_poisson_cg_b(const Dims& d, const TileMap& tm, const Coefs<T>& cf, const T* p, T* r,
                               const uint8_t* emask, const CgScalars* sc, double* partials, hipStream_t s);
template <typename T, typename S, typename R>
hipError_t launch_fem_setup(const Dims& d, const TileMap& tm, const Coefs<T>& cf, const FemTables* tb, bool gen,
                            const S* P, const S* V, T cdt, const T* W, T* x, R* r, R* p0, R* p1, R* dz,
                            T* fout, double* partials, hipStream_t s);
template <typename T, typename R>
hipError_t launch_fem_resid(const Dims& d, const TileMap& tm, const FemTables* tb, bool gen, const T* f, T* x, R* r,
                            R* p0, R* p1, R* dz, double* partials, hipStream_t s);
template <typename T>
hipError_t launch_fem_cg_a(const Dims& d, const TileMap& tm, const FemTables* tb, bool gen, const T* r,
                           const T* p_old, T* p_new, T* x, const CgScalars* sc, double* partials, int unit_w,
                           hipStream_t s);
template <typename T>
hipError_t launch_fem_cg_b(const Dims& d, const TileMap& tm, const FemTables* tb, bool gen, const T* p, T* r,
                           const CgScalars* sc, double* partials, hipStream_t s);
template <typename T>
hipError_t launch_force(const Dims& d, const TileMap& tm, const Coefs<T>& cf, const FemTables* tb, const T* P,
                        const T* V, T cdt, const T* phi, const T* ghost_top, const T* u, int mode,
                        const NoiseSpec& ns, T* Pn, T* Vn, T* Fout, hipStream_t s);
hipError_t launch_noise(const NoiseSpec& ns, int64_t N, double* xi, hipStream_t s);
template <typename S>
hipError_t launch_elec_quad(const Dims& dp, const Coefs<double>& cf, const S* P, const double* phi,
                            const double* phi_bc, const uint8_t* emask, double* partials, hipStream_t s);
template <typename S>
hipError_t launch_energy(const Dims& d, const Coefs<double>& cf, const FemTables* tb, const S* P, const double* phi,
                         const double* phi_bc, const double* ghost_top, const double* u, double* partials,
                         hipStream_t s);
template <typename S>
hipError_t launch_hvp(const Dims& d, const Coefs<double>& cf, const FemTables* tb, const S* P, const S* V,
                      double cdt, const double* w, const double* u, const double* psi, const double* du, double* Hw,
                      hipStream_t s);
template <typename S>
hipError_t launch_adjoint_axpy(int mode, double dt, S* lamP, S* lamV, double* w, const double* Hw, int64_t n,
                               hipStream_t s);
template <typename S>
hipError_t launch_theta_dot(const Dims& d, const Coefs<double>& cf, const double* w, const double* phi_e, int x0,
                            int x1, int y0, int y1, const S* P, const S* V, double cdt, double* partials,
                            hipStream_t s);

enum { kAdjPrepPc = 0, kAdjPrepEuler, kAdjPrepInit, kAdjUpdPc, kAdjUpdEuler, kAdjUpdInit };

// ---------------------------------------------------------------------------
// FEM operator tables from 1D element integrals
// ---------------------------------------------------------------------------
// The trilinear shape functions are products of 1D hat functions and the
// 2x2x2 Gauss rule of Eq. 14 integrates every product exactly, so each
// entry of the assembled stiffness, body-force and stress operators is a
// sum of products of three 1D integrals, one per axis.  For a node with
// neighbour offset d in {-1, 0, +1} along an axis the assembled 1D rows are
//   m = int N_n N_m,  s = int N_n' N_m',  g = int N_n N_m',  gt = int N_n' N_m,
// summed over the (one or two) 1D elements holding both nodes.

namespace {

enum End { kEndInterior = 0, kEndLow = 1, kEndHigh = 2 };

struct Row1D {
  double m[3], s[3], g[3], gt[3];
};

Row1D row1d(double h, int end) {
  // element integrals on [0, h]; local node 0 at 0, node 1 at h
  const double me[2][2] = {{h / 3, h / 6}, {h / 6, h / 3}};
  const double se[2][2] = {{1 / h, -1 / h}, {-1 / h, 1 / h}};
  const double ge[2][2] = {{-0.5, 0.5}, {-0.5, 0.5}};  // int N_a N_b'
  Row1D r;
  std::memset(&r, 0, sizeof(r));
  auto add = [&](int a, int b, int o) {  // row node = local a, column = local b at offset o
    r.m[o + 1] += me[a][b];
    r.s[o + 1] += se[a][b];
    r.g[o + 1] += ge[a][b];
    r.gt[o + 1] += ge[b][a];
  };
  if (end != kEndLow) {  // element on the minus side: row node is its local 1
    add(1, 0, -1);
    add(1, 1, 0);
  }
  if (end != kEndHigh) {  // element on the plus side: row node is its local 0
    add(0, 0, 0);
    add(0, 1, 1);
  }
  return r;
}

int voigt(int a, int b) {
  if (a == b) return a;
  if ((a == 0 && b == 1) || (a == 1 && b == 0)) return 3;
  if ((a == 1 && b == 2) || (a == 2 && b == 1)) return 4;
  return 5;
}

}  // namespace

// ---------------------------------------------------------------------------
// Crystal frame: grid-frame stiffness and electrostriction
// ---------------------------------------------------------------------------
// C, Q and the Landau coefficients are given on the crystal axes; the
// crystal-to-grid rotation R (all zeros: identity) maps them to the grid.

Material make_material(const pf_config& c) {
  Material m;
  bool zero = true;
  for (int t = 0; t < 9; t++) zero = zero && c.rotation[t] == 0.0;
  for (int t = 0; t < 9; t++) m.R[t] = zero ? (t % 4 == 0 ? 1.0 : 0.0) : c.rotation[t];
  m.rotated = false;
  for (int t = 0; t < 9; t++) m.rotated = m.rotated || m.R[t] != (t % 4 == 0 ? 1.0 : 0.0);
  // Bond's stress transformation in the Voigt order (xx, yy, zz, xy, yz, zx):
  // sigma' = M sigma, and with engineering strain C' = M C M^T.
  static const int vi[6] = {0, 1, 2, 0, 1, 2}, vj[6] = {0, 1, 2, 1, 2, 0};
  const double* a = m.R;
  double M[6][6];
  for (int r = 0; r < 6; r++)
    for (int q = 0; q < 6; q++) {
      const int i = vi[r], j = vj[r], k = vi[q], l = vj[q];
      M[r][q] = q < 3 ? a[3 * i + k] * a[3 * j + k] : a[3 * i + k] * a[3 * j + l] + a[3 * i + l] * a[3 * j + k];
    }
  double C0[6][6] = {};
  for (int r = 0; r < 3; r++)
    for (int q = 0; q < 3; q++) C0[r][q] = r == q ? c.C11 : c.C12;
  C0[3][3] = C0[4][4] = C0[5][5] = c.C44;
  for (int r = 0; r < 6; r++)
    for (int q = 0; q < 6; q++) {
      double sum = 0;
      for (int s = 0; s < 6; s++)
        for (int t = 0; t < 6; t++) sum += M[r][s] * C0[s][t] * M[q][t];
      m.C[r][q] = m.rotated ? sum : C0[r][q];
    }
  // Eq. 15 as a quadratic form on the grid components: eps0(P) is the
  // rotated crystal eigenstrain of p = R^T P; its coefficients follow from
  // evaluations at e_a and e_a + e_b (polarisation identity).
  auto eps_grid = [&](const double P[3], double e[6]) {
    double p[3], ec[3][3], eg[3][3];
    for (int k = 0; k < 3; k++) p[k] = a[k] * P[0] + a[3 + k] * P[1] + a[6 + k] * P[2];
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++)
        ec[i][j] = i == j ? c.Q11 * p[i] * p[i] + c.Q12 * (p[(i + 1) % 3] * p[(i + 1) % 3] + p[(i + 2) % 3] * p[(i + 2) % 3])
                          : c.Q44 * p[i] * p[j];
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) {
        double sum = 0;
        for (int k = 0; k < 3; k++)
          for (int l = 0; l < 3; l++) sum += a[3 * i + k] * ec[k][l] * a[3 * j + l];
        eg[i][j] = sum;
      }
    for (int v = 0; v < 6; v++) e[v] = (v < 3 ? 1.0 : 2.0) * eg[vi[v]][vj[v]];
  };
  double ea[3][6];
  for (int q = 0; q < 3; q++) {
    double P[3] = {0, 0, 0};
    P[q] = 1;
    eps_grid(P, ea[q]);
    for (int v = 0; v < 6; v++) m.Qv[v][q] = ea[q][v];
  }
  static const int pa[3] = {0, 1, 2}, pb[3] = {1, 2, 0};  // pairs xy, yz, zx
  for (int t = 0; t < 3; t++) {
    double P[3] = {0, 0, 0}, e[6];
    P[pa[t]] = P[pb[t]] = 1;
    eps_grid(P, e);
    for (int v = 0; v < 6; v++) m.Qv[v][3 + t] = 0.5 * (e[v] - ea[pa[t]][v] - ea[pb[t]][v]);
  }
  // cubic structure on the grid axes: no normal/shear or shear/shear coupling
  m.cubic = true;
  for (int r = 0; r < 6; r++)
    for (int q = 0; q < 6; q++)
      if ((r < 3) != (q < 3) || (r >= 3 && q >= 3 && r != q)) m.cubic = m.cubic && m.C[r][q] == 0.0;
  return m;
}

namespace {

// elastic tensor C_{ijkl} on the grid axes
double cijkl(const Material& m, int i, int j, int k, int l) { return m.C[voigt(i, j)][voigt(k, l)]; }

void build_tables(const pf_config& c, FemTables* t) {
  std::memset(t, 0, sizeof(*t));
  const Material mat = make_material(c);
  const Row1D in = row1d(c.h, kEndInterior);
  const Row1D zrow[3] = {row1d(c.h, kEndLow), row1d(c.h, kEndInterior), row1d(c.h, kEndHigh)};
  auto factor = [](const Row1D& r, bool d_row, bool d_col, int o) {
    if (d_row && d_col) return r.s[o];
    if (d_row) return r.gt[o];
    if (d_col) return r.g[o];
    return r.m[o];
  };
  for (int dz = -1; dz <= 1; dz++)
    for (int dy = -1; dy <= 1; dy++)
      for (int dx = -1; dx <= 1; dx++) {
        const int o = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
        const int off[3] = {dx + 1, dy + 1, dz + 1};
        for (int zt = 0; zt < 3; zt++) {
          const Row1D* ax[3] = {&in, &in, &zrow[zt]};
          // stiffness: K^{ce} = sum_{j,l} C_{cjel} int d_j N_n d_l N_m
          if (zt != kLow) {
            const int kt = (zt == kInterior) ? 0 : 1;
            for (int cc = 0; cc < 3; cc++)
              for (int e = 0; e < 3; e++) {
                double sum = 0;
                for (int j = 0; j < 3; j++)
                  for (int l = 0; l < 3; l++) {
                    const double cf = cijkl(mat, cc, j, e, l);
                    if (cf == 0.0) continue;
                    double p = cf;
                    for (int a = 0; a < 3; a++) p *= factor(*ax[a], a == j, a == l, off[a]);
                    sum += p;
                  }
                t->K[kt][cc][e][o] = sum;
              }
            // body force: f_c = sum_j int d_j N_n N_m sigma0_{cj}
            for (int cc = 0; cc < 3; cc++)
              for (int j = 0; j < 3; j++) {
                double p = 1;
                for (int a = 0; a < 3; a++) p *= factor(*ax[a], a == j, false, off[a]);
                t->Bf[kt][cc][voigt(cc, j)][o] += p;
              }
          }
          // weighted strain: int N_n eps_v(u), eps_ab = (d_b u_a + d_a u_b) (engineering shear)
          for (int a = 0; a < 3; a++)
            for (int b = a; b < 3; b++) {
              const int v = voigt(a, b);
              for (int pass = 0; pass < (a == b ? 1 : 2); pass++) {
                const int comp = pass ? b : a, der = pass ? a : b;  // d_der u_comp
                double p = 1;
                for (int x = 0; x < 3; x++) p *= factor(*ax[x], false, x == der, off[x]);
                t->Su[zt][v][comp][o] += p;
              }
            }
          t->Ms[zt][o] = ax[0]->m[off[0]] * ax[1]->m[off[1]] * ax[2]->m[off[2]];
        }
      }
  // compact form for a stiffness cubic on the grid axes, checked entry by entry
  {
    double kmax = 0.0;
    for (int kt = 0; kt < 2; kt++)
      for (int cc = 0; cc < 3; cc++)
        for (int e = 0; e < 3; e++)
          for (int o = 0; o < kTaps; o++) kmax = std::max(kmax, std::fabs(t->K[kt][cc][e][o]));
    const double tol = 1e-12 * kmax;
    bool seen_i[8] = {}, seen_t[24] = {};
    bool ok = true;
    for (int kt = 0; kt < 2 && ok; kt++)
      for (int cc = 0; cc < 3 && ok; cc++)
        for (int e = 0; e < 3 && ok; e++)
          for (int o = 0; o < kTaps && ok; o++) {
            const int off[3] = {o % 3 - 1, (o / 3) % 3 - 1, o / 9 - 1};
            int sg = 1;
            const int cl = kc_class(kt, cc, e, off, &sg);
            const double v = t->K[kt][cc][e][o];
            if (cl < 0) {
              ok = std::fabs(v) <= tol;
              continue;
            }
            double* slot = kt == 0 ? &t->kc_int[cl] : &t->kc_top[cl];
            bool* seen = kt == 0 ? &seen_i[cl] : &seen_t[cl];
            if (!*seen) {
              *slot = sg * v;
              *seen = true;
            } else {
              ok = std::fabs(v - sg * *slot) <= tol;
            }
          }
    for (int q = 0; q < 8; q++) ok = ok && seen_i[q];
    for (int q = 0; q < 24; q++) ok = ok && seen_t[q];
    t->compact = ok ? 1 : 0;
  }
  for (int zt = 0; zt < 3; zt++)
    for (int o = 0; o < 3; o++) {
      t->m1[zt][o] = zrow[zt].m[o];
      t->g1[zt][o] = zrow[zt].g[o];
      t->gt1[zt][o] = zrow[zt].gt[o];
    }
  for (int cc = 0; cc < 3; cc++) {
    t->inv_diag[0][cc] = 1.0 / t->K[0][cc][cc][13];
    t->inv_diag[1][cc] = 1.0 / t->K[1][cc][cc][13];
  }
}


// ---------------------------------------------------------------------------
// Context and workspace
// ---------------------------------------------------------------------------

constexpr size_t kAlign = 256;

// The film grid and the potential grid (the film plus, with the open top,
// n_air air planes above it).
int phi_planes(const pf_config& c) { return c.nz + (c.top_bc == PF_TOP_OPEN ? c.n_air : 0); }
Dims film_dims(const pf_config& c) {
  const int64_t plane = (int64_t)c.nx * c.ny;
  return Dims{c.nx, c.ny, c.nz, plane * c.nz, plane, c.nz, plane * c.nz, phi_planes(c)};
}
Dims potential_dims(const pf_config& c) {
  const int64_t plane = (int64_t)c.nx * c.ny;
  const int nzp = phi_planes(c);
  return Dims{c.nx, c.ny, nzp, plane * nzp, plane, c.nz, plane * c.nz, nzp};
}
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Workspace of the multigrid of one operator (PF_PRECOND_MG with at least two
// levels): the solver-grid z, pre-smoothed iterate and residual; per coarser
// level b, v, t, o; per level the inverse diagonal, per coarser level its
// stencils and z maps; the dense inverse of the coarsest level.  Vectors hold
// nc components of doubles.
struct MgLayout {
  size_t z = 0, v0 = 0, t0 = 0;
  std::vector<size_t> b, v, t, o, dinv, tab, zmap, zfine;
  std::vector<size_t> tabw;    // coarser levels: the stencils times omega D^-1 (the first sweep folded in)
  size_t dense = 0, dense_n = 0;  // the dense inverse and its order
  size_t first = 0, end = 0;   // the range of all multigrid vectors (cleared at init)
};

struct Layout {
  // byte offsets into the workspace
  size_t P[2], V[2];           // state (state precision), double-buffered
  size_t phi, u;               // solutions (FP64 masters); phi on the potential grid
  size_t phi32, u32;           // FP32 working copies (FP32_REFINE)
  size_t ghost64, ghost32, ghost_unit;
  size_t emask;                // open top: electrode nodes of the first air plane (bytes)
  size_t phi_bc, basis;        // boundary potential and electrode basis (FP64)
  size_t pr, pp[2], fr, fp[2]; // CG vectors, sized for FP64 (FP32 solves use half)
  size_t dphi, du;             // refinement corrections (FP32)
  size_t fbody;                // FP32_REFINE: the FEM body force of the first sweep (FP64)
  size_t escore;               // warm_start 3: the score partials of phi and u
  size_t hist;                 // ring of earlier solutions for extrapolated warm starts
                               // (extrap_order slots of Np (phi) then extrap_order of 3N (u))
  size_t adj_hist;             // the same for the adjoint solutions: psi (Np) and the adjoint
                               // displacement (3N), then the displacement at the
                               // linearisation point (3N, a ring of its own)
  size_t scratch[8];           // max(3N, Np) doubles each: adjoint, energy, conversions
  size_t tables, scalars, result, partials;
  MgLayout mg[2];              // multigrid of the Poisson (0) and the FEM (1) operator
  size_t total;
};

// Multigrid levels of one operator (0: Poisson, 1: FEM) for this
// configuration (empty: Jacobi).
std::vector<MgLevel> mg_levels_for(const pf_config& c, int field) {
  if (c.precond != PF_PRECOND_MG) return {};
  std::vector<MgLevel> lv = field == 0 ? mg_plan_phi(c) : mg_plan(c);
  if (lv.size() < 2) lv.clear();
  return lv;
}

// Scalar slots: 0 Poisson CG, 1 FEM CG, 2 sums (energy, adjoint); partial
// slots likewise, plus 3 and 4 for the multigrid setups of the FEM and the
// Poisson solve (which may run at the same time).
constexpr int kNumScalars = 5;
constexpr int kPartialsPerBlock = 4;
constexpr int kResultSlots = 128;

// Slots of the ring of earlier solutions: extrap_order, one more with
// warm_start 3 (its orders are scored on the solutions before the newest).
int ring_slots(const pf_config& c) { return c.extrap_order + (c.warm_start == 3 ? 1 : 0); }

Layout make_layout(const pf_config& c, int npartials) {
  const size_t N = (size_t)c.nx * c.ny * c.nz;
  const size_t Np = (size_t)c.nx * c.ny * phi_planes(c);  // potential grid
  const size_t S = std::max(3 * N, Np);
  const size_t es = c.precision == PF_FP32_REFINE ? 4 : 8;
  const size_t plane = (size_t)c.nx * c.ny;
  Layout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align_up(bytes);
    return at;
  };
  for (int b = 0; b < 2; b++) L.P[b] = take(3 * N * es);
  for (int b = 0; b < 2; b++) L.V[b] = take(3 * N * es);
  L.phi = take(Np * 8);
  L.u = take(3 * N * 8);
  L.phi32 = take(Np * 4);
  L.u32 = take(3 * N * 4);
  L.ghost64 = take(plane * 8);
  L.ghost32 = take(plane * 4);
  L.ghost_unit = take(plane * 8);
  L.emask = take(plane);
  L.phi_bc = take(Np * 8);
  L.basis = take((size_t)std::max(c.n_electrodes, 1) * Np * 8);
  L.pr = take(Np * 8);
  for (int b = 0; b < 2; b++) L.pp[b] = take(Np * 8);
  L.fr = take(3 * N * 8);
  for (int b = 0; b < 2; b++) L.fp[b] = take(3 * N * 8);
  L.dphi = take(Np * 4);
  L.du = take(3 * N * 4);
  L.fbody = c.precision != PF_FP64 ? take(3 * N * 8) : 0;
  L.hist = c.warm_start >= 2 && c.extrap_order > 0 ? take((Np + 3 * N) * 8 * (size_t)ring_slots(c)) : 0;
  L.adj_hist = c.warm_start >= 2 && c.extrap_order > 0 ? take((Np + 6 * N) * 8 * (size_t)c.extrap_order) : 0;
  L.escore = take((size_t)2 * kScoreBlocks * (kMaxExtrap + 1) * 8);
  for (int t = 0; t < 8; t++) L.scratch[t] = take(S * 8);
  for (int f = 0; f < 2; f++) {
    const std::vector<MgLevel> mg = mg_levels_for(c, f);
    if (mg.empty()) continue;
    MgLayout& M = L.mg[f];
    const size_t nc = f == 0 ? 1 : 3;
    const size_t N0 = f == 0 ? Np : N;
    const size_t top = f == 0 && c.top_bc == PF_TOP_METAL ? 1 : 0;
    M.first = o;
    M.z = take(nc * N0 * 8);
    M.v0 = take(nc * N0 * 8);
    M.t0 = take(nc * N0 * 8);
    for (size_t l = 0; l < mg.size(); l++) {
      const size_t Nl = (size_t)mg[l].nx * mg[l].ny * mg[l].nz;
      const bool c1 = l > 0;
      M.b.push_back(c1 ? take(nc * Nl * 8) : 0);
      M.v.push_back(c1 ? take(nc * Nl * 8) : 0);
      M.t.push_back(c1 ? take(nc * Nl * 8) : 0);
      M.o.push_back(c1 ? take(nc * Nl * 8) : 0);
    }
    M.end = o;
    for (size_t l = 0; l < mg.size(); l++) {
      M.dinv.push_back(take((size_t)mg[l].nz * nc * 8));
      M.tab.push_back(l > 0 ? take((size_t)mg[l].nz * nc * nc * 27 * 8) : 0);
      M.tabw.push_back(l > 0 ? take((size_t)mg[l].nz * nc * nc * 27 * 8) : 0);
      M.zmap.push_back(l > 0 ? take((size_t)mg[l - 1].nz * sizeof(MgZ)) : 0);
      M.zfine.push_back(l > 0 ? take((size_t)mg[l].nz * sizeof(int)) : 0);
    }
    const MgLevel& C = mg.back();
    const size_t n = nc * (size_t)C.nx * C.ny * (C.nz - 1 - top);
    if ((int64_t)n <= kMgDenseMax) {
      M.dense = take(n * n * 8);
      M.dense_n = n;
    }
  }
  L.tables = take(sizeof(FemTables));
  L.scalars = take(sizeof(CgScalars) * kNumScalars);
  L.result = take(kResultSlots * 8);
  L.partials = take((size_t)npartials * kPartialsPerBlock * 8 * kNumScalars);
  L.total = o;
  return L;
}

// Scratch slots (3N doubles each).
enum {
  kScrW = 0,      // adjoint direction w
  kScrHw,         // H w
  kScrULin,       // displacement at the linearisation point
  kScrDu,         // adjoint displacement
  kScrPsi,        // adjoint potential (Np)
  kScrPhiE,       // energy: phi at P (Np)
  kScrUE,         // energy: u at P
  kScrTmp,        // conversions
};

// Iteration-count predictions (one per kind of solve), used to size the
// first batch of iterations enqueued before the first read-back.
enum { kPredPhi = 0, kPredU, kPredPhiIn, kPredUIn, kPredAux, kPredAdjPsi, kPredAdjU, kPredAdjDu, kPredCount };

// Floor of the relative tolerance of the FP32 inner solves (FP32 CG with
// FP64 dot products tracks FP64 CG to about 1e-6 of its right-hand side).
constexpr double kInnerTol = 1e-6;
constexpr int kMaxOuter = 30;

}  // namespace

}  // namespace pf

struct pf_ctx {
  pf_config cfg;
  std::vector<pf_electrode> electrodes;
  pf::Material mat;          // grid-frame stiffness and electrostriction
  bool gen;                  // FEM kernels take the general stencil (the stiffness is not cubic on the grid axes)
  pf::MgHierarchy mg[2];     // multigrid of the Poisson (0) and FEM (1) operator (no levels: Jacobi)
  std::vector<pf::Dims> mg_dims[2];
  pf::Dims dims;             // film grid
  pf::Dims dims_p;           // potential grid
  pf::Layout lay;
  char* ws;
  size_t ws_bytes;
  int static_device;         // pf_init_static: the device whose static workspace this is (-1: caller's workspace)
  // The coarse part of each V-cycle (restriction from the solver grid down
  // to the coarsest level and back up to level 1) has fixed arguments for a
  // field (0 Poisson, 1 FEM) and vector type ([1]: float): it is captured
  // once into a graph of kernel nodes and replayed (with per-launch events,
  // one pair around each replay).  graphs: off for static contexts and
  // after a failed capture.
  bool graphs;
  hipStream_t capture_stream[2];
  hipGraphExec_t mg_graph[2][2];
  double mg_graph_bytes[2][2];
  hipStream_t stream;        // the caller's stream
  // The FEM solve of a step runs on a worker thread with a stream of its
  // own, concurrently with the Poisson solve (forked from and joined back
  // into the caller's stream by events).
  int device;
  hipStream_t stream2;
  hipEvent_t ev_fork, ev_join;
  struct Worker {
    std::thread th;
    std::mutex mu;
    std::condition_variable cv;
    std::function<void()> job;
    bool busy = false, quit = false;
  };
  std::unique_ptr<Worker> worker;
  std::mutex err_mu;
  int nblocks;              // node-kernel blocks (film grid)
  int nblocks_p;            // node-kernel blocks (potential grid)
  pf::TileMap tm_p;         // tiles of the Poisson iteration kernels (64 x 4)
  pf::TileMap tm_f;         // tiles of the FEM iteration kernels (64 x 4)
  int npartials;            // partial slots per solver (max of both block counts)
  pf::CgScalars* host_sc;   // pinned read-back buffers, one per scalar slot
  double* host_res;         // pinned read-back of reduction results
  std::string err;
  bool have_state;
  bool phi_bc_valid;
  bool basis_valid;
  bool adj_warm;            // adjoint scratch holds earlier adjoint solutions
  int hist_valid;           // solutions held for extrapolated warm starts (0..ring slots)
  std::vector<double> escore_host[2];  // warm_start 3: the score partials of phi and u read back
  int extrap_chosen[2] = {0, 0};       // warm_start 3: the order of the last refresh of phi and u
  int hist_head;            // ring slot that the next stored solution goes to
  int adj_valid, adj_head;  // the same for the adjoint solutions psi and du
  int lin_valid, lin_head;  // and for the displacement at the linearisation point
  int64_t step;
  int cur;                  // which P/V buffer is current
  int pred[pf::kPredCount];
  // per-kernel-class accounting: PF_TIMING_EVENTS records events around
  // every launch (solves sequential), PF_TIMING_BYTES only counts launches
  // and their algorithmic bytes (solves stay concurrent)
  int timing;
  std::vector<hipEvent_t> events;
  struct TimedLaunch {
    int cls, slot, solver, k;
    double bytes;
  };
  // launches awaiting their solve's iteration count: [0] the caller's
  // thread, [1] the worker's
  std::vector<TimedLaunch> pending[2];
  std::mutex kc_mu;
  double kc_ms[PF_KC_COUNT];
  int64_t kc_n[PF_KC_COUNT];
  double kc_bytes[PF_KC_COUNT];
};

namespace pf {
namespace {

// The stream the calling host thread enqueues on: the caller's stream, or
// the context's second stream on its worker thread.
thread_local hipStream_t tl_stream = nullptr;
inline hipStream_t strm(const pf_ctx* c) { return tl_stream ? tl_stream : c->stream; }

template <typename T>
T* at(pf_ctx* c, size_t off) {
  return reinterpret_cast<T*>(c->ws + off);
}

template <typename T>
T* scratch(pf_ctx* c, int slot) {
  return at<T>(c, c->lay.scratch[slot]);
}

pf_status fail(pf_ctx* c, pf_status s, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    std::lock_guard<std::mutex> g(c->err_mu);
    c->err = buf;
  }
  return s;
}

// The worker thread: runs one posted job at a time on the context's second
// stream (its device made current first).
void worker_main(pf_ctx* c) {
  (void)hipSetDevice(c->device);
  tl_stream = c->stream2;
  pf_ctx::Worker& w = *c->worker;
  std::unique_lock<std::mutex> lk(w.mu);
  for (;;) {
    w.cv.wait(lk, [&] { return w.quit || static_cast<bool>(w.job); });
    if (w.quit) return;
    std::function<void()> job = std::move(w.job);
    w.job = nullptr;
    lk.unlock();
    job();
    lk.lock();
    w.busy = false;
    w.cv.notify_all();
  }
}

void worker_post(pf_ctx* c, std::function<void()> job) {
  pf_ctx::Worker& w = *c->worker;
  std::lock_guard<std::mutex> g(w.mu);
  w.job = std::move(job);
  w.busy = true;
  w.cv.notify_all();
}

void worker_wait(pf_ctx* c) {
  pf_ctx::Worker& w = *c->worker;
  std::unique_lock<std::mutex> lk(w.mu);
  w.cv.wait(lk, [&] { return !w.busy; });
}

#define PF_HIP(ctx, ...)                                                                         \
  do {                                                                                           \
    hipError_t e_ = (__VA_ARGS__);                                                               \
    if (e_ != hipSuccess)                                                                        \
      return fail(ctx, PF_EHIP, "%s: %s (%s:%d)", #__VA_ARGS__, hipGetErrorString(e_), __FILE__, \
                  __LINE__);                                                                     \
  } while (0)

#define PF_TRY(expr)                          \
  do {                                        \
    pf_status s_ = (expr);                    \
    if (s_ != PF_OK) return s_;               \
  } while (0)

pf_status validate(const pf_config* c, std::string* why) {
  auto bad = [&](const char* m) {
    if (why) *why = m;
    return PF_EINVAL;
  };
  if (!c) return bad("null config");
  if (c->nx < 3 || c->ny < 3 || c->nz < 3) return bad("nx, ny, nz must be >= 3");
  if ((int64_t)c->nx * c->ny * c->nz > ((int64_t)1 << 34)) return bad("grid too large");
  if (!(c->h > 0) || !std::isfinite(c->h)) return bad("h must be > 0");
  if (!(c->dt > 0) || !std::isfinite(c->dt)) return bad("dt must be > 0");
  if (!(c->eps_b > 0)) return bad("eps_b must be > 0");
  if (c->n_electrodes < 0 || c->n_electrodes > 64) return bad("n_electrodes must be in [0, 64]");
  if (c->n_electrodes > 0 && !c->electrodes) return bad("electrodes is NULL");
  for (int e = 0; e < c->n_electrodes; e++) {
    const pf_electrode& a = c->electrodes[e];
    if (a.x0 < 0 || a.x1 > c->nx || a.x0 >= a.x1 || a.y0 < 0 || a.y1 > c->ny || a.y0 >= a.y1)
      return bad("electrode rectangle out of range or empty");
    if (!std::isfinite(a.volts)) return bad("electrode voltage not finite");
    for (int f = 0; f < e; f++) {
      const pf_electrode& b = c->electrodes[f];
      if (a.x0 < b.x1 && b.x0 < a.x1 && a.y0 < b.y1 && b.y0 < a.y1) return bad("electrodes overlap");
    }
  }
  if (c->integrator != PF_INT_PC && c->integrator != PF_INT_EULER) return bad("unknown integrator");
  if (c->precision != PF_FP64 && c->precision != PF_FP32_REFINE && c->precision != PF_FP32_SOLVES)
    return bad("unknown precision");
  if (!(c->tol_phi > 0) || !(c->tol_u > 0)) return bad("tolerances must be > 0");
  if (c->maxit <= 0) return bad("maxit must be > 0");
  if (c->warm_start < 0 || c->warm_start > 3) return bad("warm_start must be 0, 1, 2 or 3");
  if (c->extrap_order < 0 || c->extrap_order > kMaxExtrap) return bad("extrap_order must be in 0..8");
  if (!(c->noise_sigma >= 0) || !std::isfinite(c->noise_sigma)) return bad("noise_sigma must be finite and >= 0");
  if (c->top_bc != PF_TOP_METAL && c->top_bc != PF_TOP_OPEN) return bad("unknown top_bc");
  if (c->precond != PF_PRECOND_JACOBI && c->precond != PF_PRECOND_MG) return bad("unknown precond");
  for (int t = 0; t < 3; t++)
    if (!std::isfinite(c->misfit[t])) return bad("misfit not finite");
  {
    bool zero = true;
    for (int t = 0; t < 9; t++) zero = zero && c->rotation[t] == 0.0;
    if (!zero) {
      const double* R = c->rotation;
      for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
          const double d = R[3 * i] * R[3 * j] + R[3 * i + 1] * R[3 * j + 1] + R[3 * i + 2] * R[3 * j + 2];
          if (!(std::fabs(d - (i == j ? 1.0 : 0.0)) <= 1e-10)) return bad("rotation is not orthonormal");
        }
      const double det = R[0] * (R[4] * R[8] - R[5] * R[7]) - R[1] * (R[3] * R[8] - R[5] * R[6]) +
                         R[2] * (R[3] * R[7] - R[4] * R[6]);
      if (!(det > 0)) return bad("rotation must have determinant +1");
    }
  }
  if (c->top_bc == PF_TOP_OPEN) {
    if (c->n_air < 1 || c->n_air > 4 * c->nz) return bad("n_air must be in [1, 4 nz] with the open top");
    if (!(c->eps_air > 0) || !std::isfinite(c->eps_air)) return bad("eps_air must be > 0");
  }
  if (c->terms & ~(uint32_t)PF_TERM_ALL) return bad("unknown term bits");
  if (!(c->C11 > 0) || !(c->C44 > 0) || !(c->C11 > std::fabs(c->C12)) || !(c->C11 + 2 * c->C12 > 0))
    return bad("stiffness must be positive definite");
  return PF_OK;
}

template <typename T>
Coefs<T> make_coefs(const pf_ctx* c) {
  const pf_config& g = c->cfg;
  Coefs<T> k;
  k.a1 = (T)g.a1;
  k.a11 = (T)g.a11;
  k.a12 = (T)g.a12;
  k.G = (T)g.G;
  k.L = (T)g.L;
  k.dt = (T)g.dt;
  k.h = (T)g.h;
  k.inv_h2 = (T)(1.0 / (g.h * g.h));
  k.inv_2h = (T)(0.5 / g.h);
  k.inv_h3 = (T)(1.0 / (g.h * g.h * g.h));
  k.eps_over_h2 = (T)(g.eps_b / (g.h * g.h));
  k.inv_diag_poisson = (T)(g.h * g.h / (6.0 * g.eps_b));
  const bool open = g.top_bc == PF_TOP_OPEN;
  const double ea = open ? g.eps_air : g.eps_b;
  const double ei = ea == g.eps_b ? g.eps_b : 2 * g.eps_b * ea / (g.eps_b + ea);
  k.eps_air_over_h2 = (T)(ea / (g.h * g.h));
  k.eps_iface_over_h2 = (T)(ei / (g.h * g.h));
  k.open = open ? 1 : 0;
  const Material& m = c->mat;
  k.rotated = m.rotated ? 1 : 0;
  for (int t = 0; t < 9; t++) k.R[t] = (T)m.R[t];
  for (int r = 0; r < 6; r++)
    for (int q = 0; q < 6; q++) {
      k.Cg[6 * r + q] = (T)m.C[r][q];
      k.Qv[r][q] = (T)m.Qv[r][q];
    }
  const double es[6] = {g.misfit[0], g.misfit[1], 0.0, g.misfit[2], 0.0, 0.0};
  for (int v = 0; v < 6; v++) k.es[v] = (T)es[v];
  k.C11 = (T)g.C11;
  k.C12 = (T)g.C12;
  k.C44 = (T)g.C44;
  k.Q11 = (T)g.Q11;
  k.Q12 = (T)g.Q12;
  k.Q44 = (T)g.Q44;
  k.phi_bottom = (T)g.phi_bottom;
  k.terms = g.terms;
  return k;
}

// fp32: the state (P, V) and the force are float; refined: the solves run
// in float with double refinement (PF_FP32_REFINE and PF_FP32_SOLVES)
bool fp32(const pf_ctx* c) { return c->cfg.precision == PF_FP32_REFINE; }
bool refined(const pf_ctx* c) { return c->cfg.precision != PF_FP64; }
size_t state_bytes(const pf_ctx* c) { return fp32(c) ? 4 : 8; }

CgScalars* dev_sc(pf_ctx* c, int which) { return at<CgScalars>(c, c->lay.scalars) + which; }
double* dev_partials(pf_ctx* c, int which) {
  return at<double>(c, c->lay.partials) + (size_t)which * c->npartials * kPartialsPerBlock;
}
double* dev_result(pf_ctx* c) { return at<double>(c, c->lay.result); }
const uint8_t* emask(pf_ctx* c) { return c->cfg.top_bc == PF_TOP_OPEN ? at<uint8_t>(c, c->lay.emask) : nullptr; }

// ---------------------------------------------------------------------------
// Event timing of launches
// ---------------------------------------------------------------------------

// bytes: the launch's algorithmic HBM traffic (compulsory reads and writes,
// stencil neighbours counted once), accumulated per class.
template <typename F>
hipError_t timed(pf_ctx* c, int cls, int solver, int k, double bytes, F&& launch) {
  if (c->timing == PF_TIMING_OFF) return launch();
  if (c->timing == PF_TIMING_BYTES) {
    hipError_t err = launch();
    if (err == hipSuccess) c->pending[tl_stream ? 1 : 0].push_back({cls, -1, solver, k, bytes});
    return err;
  }
  const int slot = (int)c->pending[0].size();
  while ((int)c->events.size() < 2 * (slot + 1)) {
    hipEvent_t e;
    hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) return err;
    c->events.push_back(e);
  }
  hipError_t err = hipEventRecord(c->events[2 * slot], strm(c));
  if (err != hipSuccess) return err;
  err = launch();
  if (err != hipSuccess) return err;
  err = hipEventRecord(c->events[2 * slot + 1], strm(c));
  if (err != hipSuccess) return err;
  c->pending[0].push_back({cls, slot, solver, k, bytes});
  return hipSuccess;
}

// After a stream synchronisation: accumulates the pending launches.  CG
// iterations at or beyond `iters` of `solver` returned at entry and are
// dropped.
void collect_timing(pf_ctx* c, int solver, int iters, int list) {
  std::lock_guard<std::mutex> g(c->kc_mu);
  for (const auto& t : c->pending[list]) {
    if (t.solver >= 0 && t.solver == solver && t.k >= iters) continue;
    float ms = 0.f;
    if (t.slot >= 0 && hipEventElapsedTime(&ms, c->events[2 * t.slot], c->events[2 * t.slot + 1]) != hipSuccess)
      continue;
    c->kc_ms[t.cls] += ms;
    c->kc_n[t.cls] += 1;
    c->kc_bytes[t.cls] += t.bytes;
  }
  c->pending[list].clear();
}

pf_status read_scalars(pf_ctx* c, int which, CgScalars* out) {
  PF_HIP(c, hipMemcpyAsync(c->host_sc + which, dev_sc(c, which), sizeof(CgScalars), hipMemcpyDeviceToHost, strm(c)));
  PF_HIP(c, hipStreamSynchronize(strm(c)));
  *out = c->host_sc[which];
  if (c->timing) collect_timing(c, which, out->iter, tl_stream ? 1 : 0);
  return PF_OK;
}

pf_status sync(pf_ctx* c) {
  PF_HIP(c, hipStreamSynchronize(strm(c)));
  if (c->timing) collect_timing(c, -1, 0, tl_stream ? 1 : 0);
  return PF_OK;
}

hipError_t reduce(pf_ctx* c, const double* part, int nb, int nv, int which, int mode, double tol, double tol2,
                  double* out, int solver = -1, int k = -1) {
  const int maxit = c->cfg.maxit;
  return timed(c, PF_KC_REDUCE, solver, k, (double)nb * nv * 8 + sizeof(CgScalars), [&] {
    return launch_cg_reduce(part, nb, nv, dev_sc(c, which), mode, tol, maxit, strm(c), tol2, out);
  });
}

// ---------------------------------------------------------------------------
// Conjugate-gradient drivers
// ---------------------------------------------------------------------------
// The setup kernel forms r = b - A x and the first direction; each iteration
// is two fused kernels (direction update + operator + p.q; residual update
// + r.z), each followed by a single-block reduce that advances the scalars
// on the device.  The host enqueues iterations in batches and reads the
// scalars once per batch; kernels enqueued after convergence return at
// entry.  A last kernel applies the deferred update of x.

struct SolveResult {
  int iters;
  int outer;
  double relres;
  int done;
};

template <typename T>
// defer (non-null): the deferred last update x += alpha p is left to the
// caller, who receives p.
pf_status run_cg(pf_ctx* c, int which, int predicted, T* x, T* const pbuf[2], int64_t n,
                 const std::function<hipError_t(int)>& iteration, CgScalars* hout, const char* what,
                 const T** defer = nullptr) {
  CgScalars h;
  int k = 0;
  int batch = std::max(2, predicted);
  const int maxit = c->cfg.maxit;
  for (;;) {
    const int nb = std::min(batch, maxit - k);
    for (int t = 0; t < nb; t++, k++) PF_HIP(c, iteration(k));
    PF_TRY(read_scalars(c, which, &h));
    if (h.done != kRunning) break;
    if (k >= maxit) return fail(c, PF_EHIP, "%s: solver state did not advance", what);
    // one more iteration usually suffices after the predicted count: small
    // follow-up batches waste no iterations (each is ~35 launches with the
    // multigrid cycle) for one more read-back
    batch = std::max(1, predicted / 8);
  }
  // no iteration (the setup met the test): no deferred update, and the
  // first direction buffer was never written
  if (h.done != kNonFinite && h.iter == 0) {
    if (defer) *defer = nullptr;
  } else if (h.done != kNonFinite) {
    if (defer) *defer = pbuf[h.iter & 1];
    else
      PF_HIP(c, timed(c, PF_KC_FINISH, -1, -1, 3.0 * n * sizeof(T),
                      [&] { return launch_cg_finish<T>(x, pbuf[h.iter & 1], n, dev_sc(c, which), strm(c)); }));
  }
  *hout = h;
  if (h.done == kNonFinite) return fail(c, PF_ENONFINITE, "%s: non-finite value in the CG reductions", what);
  return PF_OK;
}

pf_status cg_status(pf_ctx* c, const CgScalars& h, SolveResult* res, const char* what) {
  res->iters = h.iter;
  res->outer = 1;
  res->done = h.done;
  res->relres = h.zero_rhs ? 0.0 : std::sqrt(h.rnorm2 / h.bnorm2);
  if (h.done == kMaxIt)
    return fail(c, PF_ENOCONV, "%s: no convergence in %d iterations (relres %.3e)", what, h.iter, res->relres);
  return PF_OK;
}

bool mg_on(const pf_ctx* c, int f) { return !c->mg[f].levels.empty(); }

// One multigrid V-cycle z0 = M r0 of the Poisson (f = 0) or the FEM (f = 1)
// operator (pre-smoothing: one damped Jacobi sweep from zero; residual,
// restriction, the coarser levels, prolongation; post-smoothing: one sweep),
// symmetric, so CG may use it.  When level 1 halves x and y, the last
// prolongation happens inside the post-smoothing kernel (kMgCorrect).  The first sweep is never stored: on the
// solver grid the residual kernel applies A to omega D^-1 b on the fly
// (kMgFirst), on the coarser levels it runs with the stencils of
// A omega D^-1 (folded on the host), and the prolongation forms
// omega D^-1 b + P e.  The Poisson cycle runs on the operator of all
// potential-grid nodes and zeroes z0 on the electrode nodes of the open top,
// a projection that keeps the preconditioner symmetric on the unknowns.  The
// last sweep also writes the tiles' r0 . z0 to part[lid * pstride + poff].
// k: the CG iteration (for the event timing), -1 in a setup.
template <typename T>
hipError_t mg_vcycle(pf_ctx* c, int f, const T* r0, T* z0, CgScalars* sc, double* part, int pstride, int poff,
                     int k) {
  const MgHierarchy& h = c->mg[f];
  const MgLayout& L = c->lay.mg[f];
  const std::vector<Dims>& D = c->mg_dims[f];
  const int nl = (int)h.levels.size();
  const int nc = h.nc;
  const int top = h.top_fixed ? 1 : 0;
  const FemTables* tb = at<FemTables>(c, c->lay.tables);
  const bool gen = c->gen;
  const Coefs<T> cf = make_coefs<T>(c);
  hipStream_t st = strm(c);
  auto V = [&](size_t off) { return at<T>(c, off); };
  auto Dv = [&](int l) { return at<double>(c, L.dinv[l]); };
  auto Zm = [&](int l) { return at<MgZ>(c, L.zmap[l]); };
  auto Zf = [&](int l) { return at<int>(c, L.zfine[l]); };
  // while the coarse part is captured into a graph, launches are recorded
  // (not run) and their bytes summed for the graph's accounting
  bool capturing = false;
  double cap_bytes = 0.0;
  auto run = [&](double bytes, auto&& fn) -> hipError_t {
    if (capturing) {
      cap_bytes += bytes;
      return fn();
    }
    return timed(c, PF_KC_MG, f, k, bytes, fn);
  };
  // algorithmic bytes: nc values of T per node of level l, times `reps`
  auto lb = [&](int l, double reps) { return reps * nc * (double)D[l].N * sizeof(T); };
  // the solver grid: the Poisson levels count a fixed bottom plane below it
  const int zoff0 = f == 0 ? 1 : 0;
  // the correction of level 1 as the kMgCorrect kernels read it
  MgCoarse<T> mc{};
  mc.e = V(L.o[1]);
  mc.zmap = Zm(1);
  mc.N = D[1].N;
  mc.plane = D[1].plane;
  mc.nx = D[1].nx, mc.ny = D[1].ny, mc.nz = D[1].nz;
  mc.zoff = zoff0;
  mc.top_fixed = top;
  auto fine = [&](int mode, double omega, const T* x, T* out, double* pp) {
    if (f == 0)
      return launch_mgp_fine<T>(D[0], c->tm_p, cf, Dv(0), mode, omega, x, r0, out, mc,
                                mode != kMgFirst ? emask(c) : nullptr, sc, pp, pstride, poff, st);
    return launch_mg_fine<T>(D[0], c->tm_f, tb, gen, Dv(0), mode, omega, x, r0, out, mc, sc, pp, pstride, poff, st);
  };
  // level 1 halves x and y: the last prolongation is fused into the sweep
  const bool fused = h.levels[1].cx && h.levels[1].cy && D[0].nx == 2 * D[1].nx && D[0].ny == 2 * D[1].ny;
  const Dims& d0 = D[0];
  const double om0 = h.levels[0].omega;
  T* v0 = V(L.v0);
  T* t0 = V(L.t0);
  auto run0 = [&](double bytes, auto&& fn) { return timed(c, f == 0 ? PF_KC_MG_PHI0 : PF_KC_MG_U0, f, k, bytes, fn); };
  // the solver grid's unknowns: the FEM's clamped plane is not one
  const double n0 = f == 0 ? (double)c->dims_p.N : (double)(c->dims.N - c->dims.plane);
  const double v0b = nc * n0 * sizeof(T);
  // first sweep's residual: b read, t written
  hipError_t e = run0(2 * v0b, [&] { return fine(kMgFirst, om0, nullptr, t0, nullptr); });
  // the coarse part: restriction to level 1, the coarser levels, and the
  // prolongations and sweeps back up to level 1
  auto coarse_part = [&]() -> hipError_t {
  hipError_t e = run(lb(0, 1) + lb(1, 1), [&] {
      // the solver grid stores no fixed planes (the Poisson ghost planes
      // lie outside its storage)
      return launch_mg_restrict<T>(d0, D[1], nc, h.levels[1].cx, h.levels[1].cy, Zm(1), Zf(1), t0, V(L.b[1]), sc,
                                   zoff0, h.levels[0].nz, 0, top, st);
    });
  for (int l = 1; l < nl - 1 && e == hipSuccess; l++) {
    const Dims& d = D[l];
    // residual of the first sweep: b - (A omega D^-1) b with the folded stencils
    const double* tabw = at<double>(c, L.tabw[l]);
    e = run(lb(l, 2), [&] {
      return launch_mg_level<T>(d, nc, tabw, Dv(l), kMgResidual, 0.0, V(L.b[l]), V(L.b[l]), V(L.t[l]), sc, top, st);
    });
    if (e == hipSuccess)
      e = run(lb(l, 1) + lb(l + 1, 1), [&] {
        return launch_mg_restrict<T>(d, D[l + 1], nc, h.levels[l + 1].cx, h.levels[l + 1].cy, Zm(l + 1), Zf(l + 1),
                                     V(L.t[l]), V(L.b[l + 1]), sc, 0, d.nz, top, top, st);
      });
  }
  // coarsest level
  const int lc = nl - 1;
  if (e == hipSuccess) {
    const Dims& d = D[lc];
    if (h.dense_n > 0) {
      e = run(8.0 * h.dense_n * h.dense_n + lb(lc, 2), [&] {
        return launch_mg_dense<T>(d, nc, h.dense_n, at<double>(c, L.dense), V(L.b[lc]), V(L.o[lc]), sc, st);
      });
    } else {
      // damped Jacobi sweeps from zero, ping-pong between v and t, last into o
      const double* tab = at<double>(c, L.tab[lc]);
      const int ns = std::max(1, h.coarse_sweeps);
      T* cur = V(ns == 1 ? L.o[lc] : L.v[lc]);
      e = run(lb(lc, 2), [&] { return launch_mg_scale<T>(d, nc, Dv(lc), h.levels[lc].omega, V(L.b[lc]), cur, sc, st); });
      for (int t = 1; t < ns && e == hipSuccess; t++) {
        T* nxt = t == ns - 1 ? V(L.o[lc]) : (cur == V(L.v[lc]) ? V(L.t[lc]) : V(L.v[lc]));
        e = run(lb(lc, 3), [&] {
          return launch_mg_level<T>(d, nc, tab, Dv(lc), kMgSweep, h.levels[lc].omega, cur, V(L.b[lc]), nxt, sc, top,
                                    st);
        });
        cur = nxt;
      }
    }
  }
  for (int l = nl - 2; l >= 1 && e == hipSuccess; l--) {
    const Dims& d = D[l];
    const double* tab = at<double>(c, L.tab[l]);
    e = run(lb(l, 2) + lb(l + 1, 1), [&] {
      return launch_mg_prolong<T>(d, D[l + 1], nc, h.levels[l + 1].cx, h.levels[l + 1].cy, Zm(l + 1), V(L.o[l + 1]),
                                  V(L.v[l]), sc, 0, top, top, V(L.b[l]), Dv(l), h.levels[l].omega, st);
    });
    if (e == hipSuccess)
      e = run(lb(l, 3), [&] {
        return launch_mg_level<T>(d, nc, tab, Dv(l), kMgSweep, h.levels[l].omega, V(L.v[l]), V(L.b[l]), V(L.o[l]),
                                  sc, top, st);
      });
  }
  return e;
  };
  if (e == hipSuccess) {
    const int ti = sizeof(T) == 4 ? 1 : 0;
    if (c->graphs && !c->mg_graph[f][ti]) {
      // capture on the field's own stream (the caller's may be the null
      // stream, which cannot capture); nothing runs while capturing
      const hipStream_t keep = st;
      st = c->capture_stream[f];
      capturing = true;
      cap_bytes = 0.0;
      hipGraph_t g = nullptr;
      hipError_t ce = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
      if (ce == hipSuccess) {
        const hipError_t le = coarse_part();
        ce = hipStreamEndCapture(st, &g);
        if (ce == hipSuccess) ce = le;
      }
      hipGraphExec_t ex = nullptr;
      if (ce == hipSuccess && g) ce = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      if (g) (void)hipGraphDestroy(g);
      st = keep;
      capturing = false;
      if (ce == hipSuccess && ex) {
        c->mg_graph[f][ti] = ex;
        c->mg_graph_bytes[f][ti] = cap_bytes;
      } else {
        c->graphs = false;  // launch kernel by kernel from now on
        (void)hipGetLastError();
      }
    }
    if (c->graphs && c->mg_graph[f][ti]) {
      hipGraphExec_t ex = c->mg_graph[f][ti];
      e = timed(c, PF_KC_MG, f, k, c->mg_graph_bytes[f][ti], [&] { return hipGraphLaunch(ex, st); });
    } else {
      e = coarse_part();
    }
  }
  if (fused) {
    // b and the level-1 correction read, z written
    if (e == hipSuccess) e = run0(2 * v0b + lb(1, 1), [&] { return fine(kMgCorrect, om0, nullptr, z0, part); });
    return e;
  }
  if (e == hipSuccess)
    e = run(lb(0, 2) + lb(1, 1), [&] {
      return launch_mg_prolong<T>(d0, D[1], nc, h.levels[1].cx, h.levels[1].cy, Zm(1), V(L.o[1]), v0, sc, zoff0, 0,
                                  top, r0, Dv(0), om0, st);
    });
  if (e == hipSuccess) e = run0(3 * v0b, [&] { return fine(kMgSweep, om0, v0, z0, part); });
  return e;
}

// After a setup with the multigrid preconditioner: z = M r and rho = r.z.
template <typename T>
hipError_t mg_setup(pf_ctx* c, int f, const T* r) {
  CgScalars* sc = dev_sc(c, f);
  double* part = dev_partials(c, f == 0 ? 4 : 3);
  hipError_t e = mg_vcycle<T>(c, f, r, at<T>(c, c->lay.mg[f].z), sc, part, 1, 0, -1);
  const int nb = f == 0 ? c->tm_p.nblocks : c->tm_f.nblocks;
  if (e == hipSuccess) e = reduce(c, part, nb, 1, f, kRedRho, 0.0, 0.0, nullptr);
  return e;
}

template <typename T>
std::function<hipError_t(int)> poisson_iteration(pf_ctx* c, const Coefs<T>& cf, T* r, T* const pb[2], T* x,
                                                 double tol) {
  return [=](int k) -> hipError_t {
    const Dims& d = c->dims_p;
    const uint8_t* em = emask(c);
    CgScalars* sc = dev_sc(c, 0);
    double* part = dev_partials(c, 0);
    const bool mg = mg_on(c, 0);
    T* z = mg ? at<T>(c, c->lay.mg[0].z) : nullptr;
    const double vb = (double)d.N * sizeof(T);
    // A: r or z, p_old, x read; p_new, x written (the first iteration: r or
    // z read, p_new written).  B: p, r read; r written.
    hipError_t e = timed(c, PF_KC_POISSON_A, 0, k, (k == 0 ? 2 : 5) * vb, [&] {
      return launch_poisson_cg_a<T>(d, c->tm_p, cf, mg ? z : r, k == 0 ? nullptr : pb[k & 1], pb[(k + 1) & 1], x,
                                    sc, part, mg ? 1 : 0, strm(c));
    });
    if (e == hipSuccess) e = reduce(c, part, c->tm_p.nblocks, 1, 0, kRedAlpha, tol, 0, nullptr, 0, k);
    if (e == hipSuccess)
      e = timed(c, PF_KC_POISSON_B, 0, k, 3 * vb,
                [&] { return launch_poisson_cg_b<T>(d, c->tm_p, cf, pb[(k + 1) & 1], r, em, sc, part, strm(c)); });
    // multigrid: z = M r replaces the Jacobi-weighted r.z of kernel B
    // (with multigrid the convergence test comes first, so the last iteration runs no V-cycle)
    if (e == hipSuccess && mg) e = reduce(c, part, c->tm_p.nblocks, 2, 0, kRedCheck, tol, 0, nullptr, 0, k);
    if (e == hipSuccess && mg) e = mg_vcycle<T>(c, 0, r, z, sc, part, 2, 0, k);
    if (e == hipSuccess) e = reduce(c, part, c->tm_p.nblocks, 2, 0, mg ? kRedConj : kRedBeta, tol, 0, nullptr, 0, k);
    return e;
  };
}

template <typename T>
std::function<hipError_t(int)> fem_iteration(pf_ctx* c, T* r, T* const pb[2], T* x, double tol) {
  return [=](int k) -> hipError_t {
    const Dims& d = c->dims;
    const FemTables* tb = at<FemTables>(c, c->lay.tables);
    CgScalars* sc = dev_sc(c, 1);
    double* part = dev_partials(c, 1);
    const bool mg = mg_on(c, 1);
    T* z = mg ? at<T>(c, c->lay.mg[1].z) : nullptr;
    // the clamped plane holds no unknowns
    const double vb = 3.0 * (d.N - d.plane) * sizeof(T);
    // the first iteration reads no p_old and leaves x alone
    hipError_t e = timed(c, PF_KC_FEM_A, 1, k, (k == 0 ? 2 : 5) * vb, [&] {
      return launch_fem_cg_a<T>(d, c->tm_f, tb, c->gen, mg ? z : r, k == 0 ? nullptr : pb[k & 1], pb[(k + 1) & 1],
                                x, sc, part, mg ? 1 : 0, strm(c));
    });
    if (e == hipSuccess) e = reduce(c, part, c->tm_f.nblocks, 1, 1, kRedAlpha, tol, 0, nullptr, 1, k);
    if (e == hipSuccess)
      e = timed(c, PF_KC_FEM_B, 1, k, 3 * vb,
                [&] {
                  return launch_fem_cg_b<T>(d, c->tm_f, tb, c->gen, pb[(k + 1) & 1], r, sc, part, strm(c));
                });
    // multigrid: z = M r replaces the Jacobi-weighted r.z of kernel B
    // (with multigrid the convergence test comes first, so the last iteration runs no V-cycle)
    if (e == hipSuccess && mg) e = reduce(c, part, c->tm_f.nblocks, 2, 1, kRedCheck, tol, 0, nullptr, 1, k);
    if (e == hipSuccess && mg) e = mg_vcycle<T>(c, 1, r, z, sc, part, 2, 0, k);
    if (e == hipSuccess) e = reduce(c, part, c->tm_f.nblocks, 2, 1, mg ? kRedConj : kRedBeta, tol, 0, nullptr, 1, k);
    return e;
  };
}

// FP64 Poisson solve of A x = -D_h Pp + ghost terms, Pp = P + cdt V (P of
// storage S; V may be null; P unused when with_P = 0).
template <typename S>
pf_status solve_poisson64(pf_ctx* c, int pred, const S* P, const S* V, double cdt, int with_P, int with_bc,
                          const double* ghost, double phi_bottom, double* x, double tol, bool warm,
                          SolveResult* res) {
  const Dims& d = c->dims_p;
  const Coefs<double> cf = make_coefs<double>(c);
  double* part = dev_partials(c, 0);
  double* r = at<double>(c, c->lay.pr);
  double* const pb[2] = {at<double>(c, c->lay.pp[0]), at<double>(c, c->lay.pp[1])};
  if (!warm) PF_HIP(c, launch_fill<double>(x, d.N, 0.0, strm(c)));
  // P (and V) read when with_P; x read; r written
  const double sb = (with_P ? 3.0 * c->dims.N * sizeof(S) * (V ? 2 : 1) : 0.0) + 2.0 * d.N * 8;
  PF_HIP(c, timed(c, PF_KC_POISSON_SETUP, -1, -1, sb, [&] {
    return launch_poisson_setup<double, S, double>(d, c->tm_p, cf, P, V, cdt, with_P, with_bc, ghost, phi_bottom, emask(c),
                                                   x, r, pb[0], nullptr, part, strm(c));
  }));
  PF_HIP(c, reduce(c, part, c->tm_p.nblocks, 3, 0, kRedSetup, tol, 0, nullptr));
  if (mg_on(c, 0)) PF_HIP(c, mg_setup<double>(c, 0, r));
  CgScalars h;
  PF_TRY(run_cg<double>(c, 0, c->pred[pred], x, pb, d.N, poisson_iteration<double>(c, cf, r, pb, x, tol), &h,
                        "Poisson solve"));
  c->pred[pred] = h.iter;
  return cg_status(c, h, res, "Poisson solve");
}

// FP64 FEM solve of K x = f(eps0(Pp)) (W null) or K x = f(deps0/dP(Pp) W).
template <typename S>
pf_status solve_fem64(pf_ctx* c, int pred, const S* P, const S* V, double cdt, const double* W, double* x,
                      double tol, bool warm, SolveResult* res) {
  const Dims& d = c->dims;
  const Coefs<double> cf = make_coefs<double>(c);
  const FemTables* tb = at<FemTables>(c, c->lay.tables);
  double* part = dev_partials(c, 1);
  double* r = at<double>(c, c->lay.fr);
  double* const pb[2] = {at<double>(c, c->lay.fp[0]), at<double>(c, c->lay.fp[1])};
  if (!warm) PF_HIP(c, launch_fill<double>(x, 3 * d.N, 0.0, strm(c)));
  // P (and V), or W, read; x read; r written
  const double n3 = 3.0 * d.N;
  const double sb = (W ? n3 * 8 : n3 * sizeof(S) * (V ? 2 : 1)) + 2 * n3 * 8;
  PF_HIP(c, timed(c, PF_KC_FEM_SETUP, -1, -1, sb, [&] {
    return launch_fem_setup<double, S, double>(d, c->tm_f, cf, tb, c->gen, P, V, cdt, W, x, r, pb[0], pb[1], nullptr,
                                               nullptr, part, strm(c));
  }));
  PF_HIP(c, reduce(c, part, c->tm_f.nblocks, 3, 1, kRedSetup, tol, 0, nullptr));
  if (mg_on(c, 1)) PF_HIP(c, mg_setup<double>(c, 1, r));
  CgScalars h;
  PF_TRY(run_cg<double>(c, 1, c->pred[pred], x, pb, 3 * d.N, fem_iteration<double>(c, r, pb, x, tol), &h,
                        "FEM solve"));
  c->pred[pred] = h.iter;
  return cg_status(c, h, res, "FEM solve");
}

// Iterative refinement (FP32_REFINE): each sweep forms the FP64 residual of
// the FP64 iterate x64 (the outer test ||b - A x64|| <= tol ||b||), solves
// the correction equation in FP32 (FP64 dot products) to the accuracy the
// outer test still needs (no tighter than kInnerTol), adds the correction to
// x64 and refreshes the FP32 working copy x32.  One sweep usually suffices,
// so the Krylov space is rarely thrown away by a restart.  The FEM setup of
// the first sweep stores the body force (FP64); later sweeps form b - K x64
// from it without evaluating the eigenstress again.
// S: the state's type (float for PF_FP32_REFINE, double for PF_FP32_SOLVES).
template <typename S>
pf_status solve_refined(pf_ctx* c, bool fem, const S* P, const S* V, double cdt, double* x64, float* x32,
                        double tol, bool warm, SolveResult* res) {
  const Dims& d = fem ? c->dims : c->dims_p;
  const int which = fem ? 1 : 0;
  const int64_t n = fem ? 3 * d.N : d.N;
  const int setup_blocks = fem ? c->tm_f.nblocks : c->tm_p.nblocks;
  const Coefs<double> cf64 = make_coefs<double>(c);
  const Coefs<float> cf32 = make_coefs<float>(c);
  const FemTables* tb = at<FemTables>(c, c->lay.tables);
  double* part = dev_partials(c, which);
  float* r = at<float>(c, fem ? c->lay.fr : c->lay.pr);
  float* const pb[2] = {at<float>(c, fem ? c->lay.fp[0] : c->lay.pp[0]),
                        at<float>(c, fem ? c->lay.fp[1] : c->lay.pp[1])};
  float* dz = at<float>(c, fem ? c->lay.du : c->lay.dphi);
  const char* what = fem ? "FEM solve (refined)" : "Poisson solve (refined)";
  const int pred = fem ? kPredUIn : kPredPhiIn;
  if (!warm) PF_HIP(c, launch_fill<double>(x64, n, 0.0, strm(c)));
  res->iters = 0;
  res->outer = 0;
  res->relres = 0;
  auto iteration = fem ? fem_iteration<float>(c, r, pb, dz, kInnerTol)
                       : poisson_iteration<float>(c, cf32, r, pb, dz, kInnerTol);
  double* fbody = at<double>(c, c->lay.fbody);
  bool synced = false;  // x32 == (float) x64, as the last refinement update left it
  for (;;) {
    // per unknown: the first FEM sweep reads P, V and x64 and writes r, p,
    // d (FP32) and the FP64 body force; later sweeps read the body force
    // and x64 instead of P, V; the Poisson setup reads P, V of the film and
    // x64 and writes r, p, d
    const double n3 = 3.0 * c->dims.N;
    const double sv = 2.0 * sizeof(S);
    if (fem && res->outer == 0) {
      PF_HIP(c, timed(c, PF_KC_FEM_SETUP, -1, -1, n3 * (sv + 8 + 2 * 4 + 8), [&] {
        return launch_fem_setup<double, S, float>(d, c->tm_f, cf64, tb, c->gen, P, V, cdt, nullptr, x64, r, pb[0],
                                                  pb[1], dz, fbody, part, strm(c));
      }));
    } else if (fem) {
      PF_HIP(c, timed(c, PF_KC_FEM_SETUP, -1, -1, n3 * (8 + 8 + 2 * 4), [&] {
        return launch_fem_resid<double, float>(d, c->tm_f, tb, c->gen, fbody, x64, r, pb[0], pb[1], dz, part,
                                               strm(c));
      }));
    } else {
      PF_HIP(c, timed(c, PF_KC_POISSON_SETUP, -1, -1, n3 * sv + (double)d.N * (8 + 2 * 4), [&] {
        return launch_poisson_setup<double, S, float>(d, c->tm_p, cf64, P, V, cdt, 1, 1, at<double>(c, c->lay.ghost64),
                                                          c->cfg.phi_bottom, emask(c), x64, r, pb[0], dz, part,
                                                          strm(c));
      }));
    }
    PF_HIP(c, reduce(c, part, setup_blocks, 3, which, kRedOuter, tol, kInnerTol, nullptr));
    CgScalars h;
    const float* pfin = nullptr;  // the inner solve's deferred last update (applied by the refinement update)
    bool inner = true;
    if (res->outer > 0) {
      // a later sweep mostly finds the outer test met: read it back before
      // launching the inner solve, whose batch would otherwise only return
      // at entry
      PF_TRY(read_scalars(c, which, &h));
      if (h.done == kNonFinite) return fail(c, PF_ENONFINITE, "%s: non-finite value in the CG reductions", what);
      inner = !h.outer_done;
    }
    if (inner) {
      if (mg_on(c, which)) PF_HIP(c, mg_setup<float>(c, which, r));
      PF_TRY(run_cg<float>(c, which, c->pred[pred], dz, pb, n, iteration, &h, what, &pfin));
      res->iters += h.iter;
    }
    res->relres = h.outer_b2 > 0 ? std::sqrt(h.outer_r2 / h.outer_b2) : 0.0;
    if (h.outer_done) {
      if (h.zero_rhs) {
        PF_HIP(c, launch_fill<double>(x64, n, 0.0, strm(c)));
        synced = false;
      }
      if (!synced)
        PF_HIP(c, timed(c, PF_KC_OTHER, -1, -1, 12.0 * n,
                        [&] { return launch_convert<double, float>(x64, x32, n, strm(c)); }));
      return PF_OK;
    }
    if (h.iter > 0) c->pred[pred] = h.iter;
    // x64 read and written, x32 written, d (and the last direction) read
    PF_HIP(c, timed(c, PF_KC_OTHER, -1, -1, (double)n * (16 + 4 + 4 + (pfin ? 4 : 0)), [&] {
      return launch_refine_update(x64, x32, dz, pfin, pfin ? dev_sc(c, which) : nullptr, n, strm(c));
    }));
    synced = true;
    res->outer++;
    if (res->outer >= kMaxOuter) {
      return fail(c, PF_ENOCONV, "%s: %d refinement sweeps, relres %.3e", what, res->outer, res->relres);
    }
  }
}

pf_status worst(pf_status a, pf_status b) {
  if (a == PF_OK) return b;
  if (b == PF_OK) return a;
  if (a == PF_ENOCONV) return b;
  return a;
}

bool fatal(pf_status s) { return s != PF_OK && s != PF_ENOCONV; }

void stats_add(pf_step_stats* st, int which, const SolveResult& r) {
  if (!st) return;
  if (which == 0) {
    st->iters_phi += r.iters;
    st->last_iters_phi = r.iters;
    st->solves_phi++;
    st->relres_phi = std::max(st->relres_phi, r.relres);
  } else {
    st->iters_u += r.iters;
    st->last_iters_u = r.iters;
    st->solves_u++;
    st->relres_u = std::max(st->relres_u, r.relres);
  }
}

// warm_start 2: replaces the state's phi and u by their extrapolation from
// the last solutions (the first solves after a state change use what is
// available: the order grows by one per refresh up to extrap_order).  The
// weights of the polynomial through m + 1 equally spaced values, evaluated
// one step past the newest, are (-1)^t C(m+1, t+1), t = 0..m.
// warm_start 3: the order of each refresh is the one among 0..extrap_order
// whose extrapolation from the solutions before the newest would have come
// closest to the newest (squared error summed over a fixed sample of the
// field, 1/64 of its values in chunks of 256); the order that predicts best
// changes along a trajectory (high while the fields move smoothly, low once
// the step-to-step changes approach the solver tolerance, which the weights
// amplify).
// extrapolate_plan does the host side (ring descriptors of phi and u, ring
// head advanced; false: order 0, nothing to launch); extrapolate_field
// launches one field's kernels on the calling thread's stream, so each solve
// extrapolates its own field on its own stream.
// ring_plan: the descriptors of nf fields of lengths len[] whose rings of
// `slots` values lie one after the other at byte offset off; valid and head
// are the ring's fill and next slot; cap the highest order.
void extrap_weights(int m, double* c) {
  for (int t = 0; t <= m; t++) {
    double b = 1;
    for (int q = 1; q <= t + 1; q++) b = b * (m + 2 - q) / q;
    c[t] = (t & 1) ? -b : b;
  }
}

bool ring_plan(pf_ctx* c, size_t off, int nf, const int64_t* len, int& valid, int& head, ExtrapRing* ring, int slots,
               int cap) {
  const int m = std::min(valid, cap);
  const int nh = std::min(valid, slots);
  int64_t first = 0;
  for (int f = 0; f < nf; f++) {
    ExtrapRing& r = ring[f];
    double* base = slots > 0 ? at<double>(c, off) + first : nullptr;
    first += (int64_t)slots * len[f];
    r.m = m;
    r.nh = nh;
    extrap_weights(m, r.c);
    for (int t = 0; t <= kMaxExtrap; t++)
      r.h[t] = t < nh ? base + (int64_t)((head - 1 - t + 2 * slots) % slots) * len[f] : nullptr;
    r.dest = slots > 0 ? base + (int64_t)head * len[f] : nullptr;
  }
  if (cap == 0) return false;  // the previous solution is the guess
  head = (head + 1) % slots;
  if (valid < slots) valid++;
  return true;
}

bool extrapolate_plan(pf_ctx* c, ExtrapRing ring[2]) {
  const int64_t len[2] = {c->dims_p.N, 3 * c->dims.N};
  return ring_plan(c, c->lay.hist, 2, len, c->hist_valid, c->hist_head, ring, ring_slots(c->cfg),
                   c->cfg.extrap_order);
}

// Replaces x (n values, the previous solution) by its extrapolation and
// stores the previous solution in the ring, on the calling thread's stream.
pf_status extrapolate_into(pf_ctx* c, double* x, int64_t n, const ExtrapRing& ring) {
  // x and m history slots read; x and the ring slot written
  PF_HIP(c, timed(c, PF_KC_OTHER, -1, -1, 8.0 * n * (ring.m + 3),
                  [&] { return launch_extrapolate(x, ring, n, strm(c)); }));
  return PF_OK;
}

pf_status extrapolate_field(pf_ctx* c, int f, const ExtrapRing& ring0) {
  const int64_t n = f == 0 ? c->dims_p.N : 3 * c->dims.N;
  double* x = at<double>(c, f == 0 ? c->lay.phi : c->lay.u);
  ExtrapRing ring = ring0;
  if (c->cfg.warm_start == 3) {
    // score the orders the history allows, then extrapolate with the best
    ExtrapScore sc{};
    sc.mmax = std::min(c->cfg.extrap_order, ring.nh - 1);
    int best = 0;
    if (sc.mmax >= 1) {
      for (int m = 0; m <= sc.mmax; m++) extrap_weights(m, sc.c[m]);
      const int nv = kMaxExtrap + 1;
      sc.partials = at<double>(c, c->lay.escore) + (size_t)f * kScoreBlocks * nv;
      // the sampled values of x and of the mmax + 1 earlier solutions read
      const double sb = 8.0 * (sc.mmax + 2) * (double)n / kScoreStride;
      PF_HIP(c, timed(c, PF_KC_OTHER, -1, -1, sb, [&] { return launch_extrap_score(x, ring, sc, n, strm(c)); }));
      std::vector<double>& hp = c->escore_host[f];
      PF_HIP(c, hipMemcpyAsync(hp.data(), sc.partials, hp.size() * sizeof(double), hipMemcpyDeviceToHost, strm(c)));
      PF_HIP(c, hipStreamSynchronize(strm(c)));
      double emin = 0.0;
      for (int m = 0; m <= sc.mmax; m++) {
        double e = 0.0;
        for (int b = 0; b < kScoreBlocks; b++) e += hp[(size_t)b * nv + m];
        if (m == 0 || e < emin) emin = e, best = m;
      }
    } else {
      best = ring.m;  // no choice yet: what the history holds (order 0 or 1)
    }
    ring.m = best;
    extrap_weights(best, ring.c);
    c->extrap_chosen[f] = best;
  }
  // x and m history slots read; x and the ring slot written
  PF_HIP(c, timed(c, PF_KC_OTHER, -1, -1, 8.0 * n * (ring.m + 3),
                  [&] { return launch_extrapolate(x, ring, n, strm(c)); }));
  return PF_OK;
}

// Solves phi and u of the state at Pp = P + cdt V (state precision).  With
// both fields and no per-launch timing the FEM solve runs on the worker's
// stream concurrently with the Poisson solve on the caller's: the two touch
// disjoint buffers and scalar slots, so the results do not depend on how
// their kernels interleave.
// ring (non-null): first replace each field by its extrapolation.
pf_status solve_nonlocal(pf_ctx* c, const void* P, const void* V, double cdt, bool warm, pf_step_stats* st,
                         const ExtrapRing* ring = nullptr) {
  double* phi = at<double>(c, c->lay.phi);
  double* u = at<double>(c, c->lay.u);
  auto poisson = [&](SolveResult* r) -> pf_status {
    if (ring) PF_TRY(extrapolate_field(c, 0, ring[0]));
    if (fp32(c))
      return solve_refined<float>(c, false, static_cast<const float*>(P), static_cast<const float*>(V), cdt, phi,
                                  at<float>(c, c->lay.phi32), c->cfg.tol_phi, warm, r);
    if (refined(c))
      return solve_refined<double>(c, false, static_cast<const double*>(P), static_cast<const double*>(V), cdt, phi,
                                   at<float>(c, c->lay.phi32), c->cfg.tol_phi, warm, r);
    return solve_poisson64<double>(c, kPredPhi, static_cast<const double*>(P), static_cast<const double*>(V), cdt, 1,
                                   1, at<double>(c, c->lay.ghost64), c->cfg.phi_bottom, phi, c->cfg.tol_phi, warm, r);
  };
  auto fem = [&](SolveResult* r) -> pf_status {
    if (ring) PF_TRY(extrapolate_field(c, 1, ring[1]));
    if (fp32(c))
      return solve_refined<float>(c, true, static_cast<const float*>(P), static_cast<const float*>(V), cdt, u,
                                  at<float>(c, c->lay.u32), c->cfg.tol_u, warm, r);
    if (refined(c))
      return solve_refined<double>(c, true, static_cast<const double*>(P), static_cast<const double*>(V), cdt, u,
                                   at<float>(c, c->lay.u32), c->cfg.tol_u, warm, r);
    return solve_fem64<double>(c, kPredU, static_cast<const double*>(P), static_cast<const double*>(V), cdt, nullptr,
                               u, c->cfg.tol_u, warm, r);
  };
  const bool elec = c->cfg.terms & PF_TERM_ELEC, elas = c->cfg.terms & PF_TERM_ELAS;
  if (elec && elas && c->worker && c->timing != PF_TIMING_EVENTS) {
    PF_HIP(c, hipEventRecord(c->ev_fork, strm(c)));
    SolveResult rf{};
    pf_status sf = PF_OK;
    worker_post(c, [&] {
      const hipError_t e = hipStreamWaitEvent(c->stream2, c->ev_fork, 0);
      sf = e == hipSuccess ? fem(&rf) : fail(c, PF_EHIP, "fork: %s", hipGetErrorString(e));
      const hipError_t e2 = hipEventRecord(c->ev_join, c->stream2);
      if (e2 != hipSuccess && !fatal(sf)) sf = fail(c, PF_EHIP, "join: %s", hipGetErrorString(e2));
    });
    SolveResult rp{};
    const pf_status sp = poisson(&rp);
    worker_wait(c);
    PF_HIP(c, hipStreamWaitEvent(strm(c), c->ev_join, 0));
    if (fatal(sp)) return sp;
    if (fatal(sf)) return sf;
    stats_add(st, 0, rp);
    stats_add(st, 1, rf);
    return worst(sp, sf);
  }
  pf_status out = PF_OK;
  if (elec) {
    SolveResult r{};
    const pf_status s = poisson(&r);
    if (fatal(s)) return s;
    stats_add(st, 0, r);
    out = worst(out, s);
  }
  if (elas) {
    SolveResult r{};
    const pf_status s = fem(&r);
    if (fatal(s)) return s;
    stats_add(st, 1, r);
    out = worst(out, s);
  }
  return out;
}

// Force sweep on the state's buffers (state precision).
// The noise of step `step` (amp = 0 when the configuration has none).
NoiseSpec noise_spec(const pf_ctx* c, int64_t step, bool on) {
  NoiseSpec ns;
  ns.amp = on ? c->cfg.noise_sigma / std::sqrt(c->cfg.dt) : 0.0;
  ns.key0 = (uint32_t)c->cfg.noise_seed;
  ns.key1 = (uint32_t)(c->cfg.noise_seed >> 32);
  ns.step0 = (uint32_t)(uint64_t)step;
  ns.step1 = (uint32_t)((uint64_t)step >> 32);
  return ns;
}

// Force at P (+ cdt V) and the update `mode`; the step modes add the thermal
// noise of the current step.
pf_status launch_state_force(pf_ctx* c, const void* P, const void* V, double cdt, int mode, void* Pn, void* Vn,
                             void* F, const void* phi_override = nullptr, const void* u_override = nullptr) {
  const FemTables* tb = at<FemTables>(c, c->lay.tables);
  const NoiseSpec ns = noise_spec(c, c->step, mode == kPcStep || mode == kEulerStep);
  // P (and V), phi, u read; the new P and V (predictor-corrector step) or
  // one of V, P, F written
  const size_t es = fp32(c) ? 4 : 8;
  const double n3 = 3.0 * c->dims.N;
  const double fb = es * (n3 * (V ? 2 : 1) + (double)c->dims_p.N + n3 + n3 * (mode == kPcStep ? 2 : 1));
  if (fp32(c)) {
    const Coefs<float> cf = make_coefs<float>(c);
    const float* phi = phi_override ? static_cast<const float*>(phi_override) : at<float>(c, c->lay.phi32);
    const float* u = u_override ? static_cast<const float*>(u_override) : at<float>(c, c->lay.u32);
    PF_HIP(c, timed(c, PF_KC_FORCE, -1, -1, fb, [&] {
      return launch_force<float>(c->dims, c->tm_f, cf, tb, static_cast<const float*>(P), static_cast<const float*>(V),
                                 (float)cdt, phi, at<float>(c, c->lay.ghost32), u, mode, ns, static_cast<float*>(Pn),
                                 static_cast<float*>(Vn), static_cast<float*>(F), strm(c));
    }));
  } else {
    const Coefs<double> cf = make_coefs<double>(c);
    const double* phi = phi_override ? static_cast<const double*>(phi_override) : at<double>(c, c->lay.phi);
    const double* u = u_override ? static_cast<const double*>(u_override) : at<double>(c, c->lay.u);
    PF_HIP(c, timed(c, PF_KC_FORCE, -1, -1, fb, [&] {
      return launch_force<double>(c->dims, c->tm_f, cf, tb, static_cast<const double*>(P), static_cast<const double*>(V), cdt,
                                  phi, at<double>(c, c->lay.ghost64), u, mode, ns, static_cast<double*>(Pn),
                                  static_cast<double*>(Vn), static_cast<double*>(F), strm(c));
    }));
  }
  return PF_OK;
}

// Builds the multigrid hierarchy of one operator (0: Poisson, 1: FEM) and
// uploads it; clears the multigrid vectors (their fixed planes stay zero).
// The Poisson solver grid stores no bottom ghost plane, so the inverse
// diagonal of its level 0 is uploaded from its second plane on.
// Synchronises.
pf_status upload_mg(pf_ctx* c, int f, const FemTables& tb) {
  c->mg[f] = f == 0 ? build_mg_phi(c->cfg) : build_mg(c->cfg, tb);
  MgHierarchy& h = c->mg[f];
  h.tables_w.clear();
  const MgLayout& L = c->lay.mg[f];
  if (h.levels.size() != L.dinv.size()) return fail(c, PF_EINVAL, "multigrid plan changed between layout and init");
  std::vector<Dims>& D = c->mg_dims[f];
  D.clear();
  for (size_t l = 0; l < h.levels.size(); l++) {
    const MgLevel& m = h.levels[l];
    const int64_t plane = (int64_t)m.nx * m.ny;
    D.push_back(l == 0 ? (f == 0 ? c->dims_p : c->dims)
                       : Dims{m.nx, m.ny, m.nz, plane * m.nz, plane, m.nz, plane * m.nz, m.nz});
    const size_t skip = l == 0 && f == 0 ? (size_t)h.nc : 0;
    const size_t count = (size_t)D.back().nz * h.nc;
    if (skip + count > m.dinv.size()) return fail(c, PF_EINVAL, "multigrid: level %zu does not match its grid", l);
    PF_HIP(c, hipMemcpyAsync(c->ws + L.dinv[l], m.dinv.data() + skip, count * 8, hipMemcpyHostToDevice, strm(c)));
    if (l > 0) {
      if (h.tables[l].size() != (size_t)m.nz * h.nc * h.nc * 27 || h.zmaps[l].size() != (size_t)h.levels[l - 1].nz ||
          h.zfine[l].size() != (size_t)m.nz)
        return fail(c, PF_EINVAL, "multigrid: level %zu tables do not match its grid", l);
      PF_HIP(c, hipMemcpyAsync(c->ws + L.tab[l], h.tables[l].data(), h.tables[l].size() * 8, hipMemcpyHostToDevice,
                               strm(c)));
      // A omega D^-1: column (plane k + dz, component e) scaled by omega / diag
      std::vector<double> tw(h.tables[l].size(), 0.0);
      const int nc = h.nc;
      for (int k = 0; k < m.nz; k++)
        for (int cc = 0; cc < nc; cc++)
          for (int e = 0; e < nc; e++)
            for (int o = 0; o < 27; o++) {
              const int kk = k + o / 9 - 1;
              if (kk < 0 || kk >= m.nz) continue;
              const size_t at_ = (((size_t)k * nc + cc) * nc + e) * 27 + o;
              tw[at_] = h.tables[l][at_] * m.omega * m.dinv[(size_t)kk * nc + e];
            }
      h.tables_w.push_back(std::move(tw));
      PF_HIP(c, hipMemcpyAsync(c->ws + L.tabw[l], h.tables_w.back().data(), h.tables_w.back().size() * 8,
                               hipMemcpyHostToDevice, strm(c)));
      PF_HIP(c, hipMemcpyAsync(c->ws + L.zmap[l], h.zmaps[l].data(), h.zmaps[l].size() * sizeof(MgZ),
                               hipMemcpyHostToDevice, strm(c)));
      PF_HIP(c, hipMemcpyAsync(c->ws + L.zfine[l], h.zfine[l].data(), h.zfine[l].size() * sizeof(int),
                               hipMemcpyHostToDevice, strm(c)));
    }
  }
  if (h.dense_n > 0) {
    if (L.dense == 0 || (size_t)h.dense_n != L.dense_n)
      return fail(c, PF_EINVAL, "multigrid: no room for the coarsest inverse");
    PF_HIP(c, hipMemcpyAsync(c->ws + L.dense, h.dense_inv.data(), h.dense_inv.size() * 8, hipMemcpyHostToDevice,
                             strm(c)));
  }
  PF_HIP(c, launch_fill<double>(at<double>(c, L.first), (int64_t)((L.end - L.first) / 8), 0.0, strm(c)));
  PF_HIP(c, hipStreamSynchronize(strm(c)));
  return PF_OK;
}

// Uploads the top ghost plane for the current electrode voltages.
pf_status upload_ghosts(pf_ctx* c) {
  const pf_config& g = c->cfg;
  std::vector<double> g64((size_t)g.nx * g.ny, g.phi_top);
  for (auto& e : c->electrodes)
    for (int j = e.y0; j < e.y1; j++)
      for (int i = e.x0; i < e.x1; i++) g64[(size_t)i + (size_t)g.nx * j] = e.volts;
  std::vector<float> g32(g64.begin(), g64.end());
  // open top: the electrode nodes of the first air plane are the Dirichlet nodes
  std::vector<uint8_t> mask((size_t)g.nx * g.ny, 0);
  for (auto& e : c->electrodes)
    for (int j = e.y0; j < e.y1; j++)
      for (int i = e.x0; i < e.x1; i++) mask[(size_t)i + (size_t)g.nx * j] = 1;
  PF_HIP(c, hipMemcpyAsync(c->ws + c->lay.ghost64, g64.data(), g64.size() * 8, hipMemcpyHostToDevice, strm(c)));
  PF_HIP(c, hipMemcpyAsync(c->ws + c->lay.ghost32, g32.data(), g32.size() * 4, hipMemcpyHostToDevice, strm(c)));
  PF_HIP(c, hipMemcpyAsync(c->ws + c->lay.emask, mask.data(), mask.size(), hipMemcpyHostToDevice, strm(c)));
  PF_HIP(c, hipStreamSynchronize(strm(c)));
  return PF_OK;
}

double aux_tol(const pf_ctx* c) { return std::min(c->cfg.tol_phi, 1e-12); }

// phi_bc: the potential of the boundary values with P = 0 (linear-dielectric
// superposition of the applied field).
pf_status ensure_phi_bc(pf_ctx* c) {
  if (c->phi_bc_valid) return PF_OK;
  SolveResult r{};
  pf_status s = solve_poisson64<double>(c, kPredAux, nullptr, nullptr, 0.0, 0, 1, at<double>(c, c->lay.ghost64),
                                        c->cfg.phi_bottom, at<double>(c, c->lay.phi_bc), aux_tol(c), false, &r);
  if (fatal(s)) return s;
  c->phi_bc_valid = true;
  return s;
}

// Electrode basis: phi^(e) for unit voltage on electrode e, every other
// boundary value zero, P = 0.
pf_status ensure_basis(pf_ctx* c) {
  if (c->basis_valid || c->cfg.n_electrodes == 0) return PF_OK;
  const pf_config& g = c->cfg;
  pf_status out = PF_OK;
  for (int e = 0; e < g.n_electrodes; e++) {
    std::vector<double> unit((size_t)g.nx * g.ny, 0.0);
    const pf_electrode& el = c->electrodes[e];
    for (int j = el.y0; j < el.y1; j++)
      for (int i = el.x0; i < el.x1; i++) unit[(size_t)i + (size_t)g.nx * j] = 1.0;
    PF_HIP(c, hipMemcpyAsync(c->ws + c->lay.ghost_unit, unit.data(), unit.size() * 8, hipMemcpyHostToDevice,
                             strm(c)));
    SolveResult r{};
    pf_status s = solve_poisson64<double>(c, kPredAux, nullptr, nullptr, 0.0, 0, 1, at<double>(c, c->lay.ghost_unit),
                                          0.0, at<double>(c, c->lay.basis) + (size_t)e * c->dims_p.N, aux_tol(c), false,
                                          &r);
    if (fatal(s)) return s;
    out = worst(out, s);
  }
  c->basis_valid = true;
  return out;
}

// ---------------------------------------------------------------------------
// Adjoint
// ---------------------------------------------------------------------------

// Hw = (dF/dP)(X) w, X = P + cdt V (storage S), w in scratch kScrW.
template <typename S>
pf_status hvp(pf_ctx* c, const S* P, const S* V, double cdt, const double* ulin_in = nullptr) {
  const Dims& d = c->dims;
  const Coefs<double> cf = make_coefs<double>(c);
  const FemTables* tb = at<FemTables>(c, c->lay.tables);
  double* w = scratch<double>(c, kScrW);
  double* ulin = scratch<double>(c, kScrULin);
  double* du = scratch<double>(c, kScrDu);
  double* psi = scratch<double>(c, kScrPsi);
  // warm_start 2 and 3: the adjoint solutions of the previous adjoint steps
  // are extrapolated like the forward ones with warm_start 2 (rings of psi
  // and du; ulin has a ring of its own, which restarts after steps that were
  // given ulin)
  ExtrapRing ring[2], lring[1];
  const int64_t len[2] = {c->dims_p.N, 3 * d.N};
  const int64_t llen[1] = {3 * d.N};
  const bool xw = c->adj_warm && c->cfg.warm_start >= 2;
  const int cap = c->cfg.extrap_order;
  const bool ex = xw && ring_plan(c, c->lay.adj_hist, 2, len, c->adj_valid, c->adj_head, ring, cap, cap);
  const size_t loff = c->lay.adj_hist + (size_t)c->cfg.extrap_order * (size_t)(len[0] + len[1]) * 8;
  const bool lex = xw && !ulin_in && ring_plan(c, loff, 1, llen, c->lin_valid, c->lin_head, lring, cap, cap);
  if (ulin_in) {
    // the scratch keeps the latest displacement, a valid warm start should a
    // later step have to solve for it
    c->lin_valid = 0;
    PF_HIP(c, hipMemcpyAsync(ulin, ulin_in, (size_t)llen[0] * sizeof(double), hipMemcpyDeviceToDevice, strm(c)));
  }
  // the displacement at the linearisation point and the adjoint displacement
  // (given: the forward step's own solution, no solve)
  auto fem = [&]() -> pf_status {
    SolveResult r{};
    if (lex) PF_TRY(extrapolate_into(c, ulin, llen[0], lring[0]));
    if (ex) PF_TRY(extrapolate_into(c, du, len[1], ring[1]));
    pf_status s = PF_OK;
    if (!ulin_in) {
      s = solve_fem64<S>(c, kPredAdjU, P, V, cdt, nullptr, ulin, c->cfg.tol_u, c->adj_warm, &r);
      if (fatal(s)) return s;
    }
    const pf_status s2 = solve_fem64<S>(c, kPredAdjDu, P, V, cdt, w, du, c->cfg.tol_u, c->adj_warm, &r);
    return fatal(s2) ? s2 : worst(s, s2);
  };
  // the adjoint potential
  auto poisson = [&]() -> pf_status {
    SolveResult r{};
    if (ex) PF_TRY(extrapolate_into(c, psi, len[0], ring[0]));
    return solve_poisson64<double>(c, kPredAdjPsi, w, nullptr, 0.0, 1, 0, at<double>(c, c->lay.ghost64), 0.0, psi,
                                   c->cfg.tol_phi, c->adj_warm, &r);
  };
  const bool elec = c->cfg.terms & PF_TERM_ELEC, elas = c->cfg.terms & PF_TERM_ELAS;
  pf_status out = PF_OK;
  if (elec && elas && c->worker && c->timing != PF_TIMING_EVENTS) {
    // concurrent, as the forward solves
    PF_HIP(c, hipEventRecord(c->ev_fork, strm(c)));
    pf_status sf = PF_OK;
    worker_post(c, [&] {
      const hipError_t e = hipStreamWaitEvent(c->stream2, c->ev_fork, 0);
      sf = e == hipSuccess ? fem() : fail(c, PF_EHIP, "fork: %s", hipGetErrorString(e));
      const hipError_t e2 = hipEventRecord(c->ev_join, c->stream2);
      if (e2 != hipSuccess && !fatal(sf)) sf = fail(c, PF_EHIP, "join: %s", hipGetErrorString(e2));
    });
    const pf_status sp = poisson();
    worker_wait(c);
    PF_HIP(c, hipStreamWaitEvent(strm(c), c->ev_join, 0));
    if (fatal(sp)) return sp;
    if (fatal(sf)) return sf;
    out = worst(sp, sf);
  } else {
    if (elas) {
      const pf_status s = fem();
      if (fatal(s)) return s;
      out = worst(out, s);
    }
    if (elec) {
      const pf_status s = poisson();
      if (fatal(s)) return s;
      out = worst(out, s);
    }
  }
  // P (and V), w, the linearisation point's u, psi and du read; H w written
  const double hb = 3.0 * d.N * (sizeof(S) * (V ? 2 : 1) + 4 * 8) + 8.0 * c->dims_p.N;
  PF_HIP(c, timed(c, PF_KC_OTHER, -1, -1, hb, [&] {
    return launch_hvp<S>(d, cf, tb, P, V, cdt, w, ulin_in ? ulin_in : ulin, psi, du, scratch<double>(c, kScrHw),
                         strm(c));
  }));
  c->adj_warm = true;
  return out;
}

// dtheta += scale * w . dF/dtheta(X), theta = (V_1..V_ne, a1).
template <typename S>
pf_status theta_accumulate(pf_ctx* c, const S* P, const S* V, double cdt, double scale, double* dtheta) {
  const Dims& d = c->dims;
  const Coefs<double> cf = make_coefs<double>(c);
  const double* w = scratch<double>(c, kScrW);
  double* part = dev_partials(c, 2);
  const int ne = c->cfg.n_electrodes;
  if ((c->cfg.terms & PF_TERM_ELEC) && ne > 0) {
    PF_TRY(ensure_basis(c));
    for (int e = 0; e < ne; e++) {
      const pf_electrode& el = c->electrodes[e];
      const double* phe = at<double>(c, c->lay.basis) + (size_t)e * c->dims_p.N;
      PF_HIP(c, timed(c, PF_KC_OTHER, -1, -1, 3.0 * d.N * 8 + 8.0 * c->dims_p.N, [&] {
        return launch_theta_dot<S>(d, cf, w, phe, el.x0, el.x1, el.y0, el.y1, P, V, cdt, part, strm(c));
      }));
      PF_HIP(c, reduce(c, part, c->nblocks, 1, 2, kRedSum, 0, 0, dev_result(c) + e));
    }
  }
  if (c->cfg.terms & PF_TERM_LANDAU) {
    PF_HIP(c, timed(c, PF_KC_OTHER, -1, -1, 3.0 * d.N * (8 + sizeof(S) * (V ? 2 : 1)), [&] {
      return launch_theta_dot<S>(d, cf, w, nullptr, 0, 0, 0, 0, P, V, cdt, part, strm(c));
    }));
    PF_HIP(c, reduce(c, part, c->nblocks, 1, 2, kRedSum, 0, 0, dev_result(c) + ne));
  }
  PF_HIP(c, hipMemcpyAsync(c->host_res, dev_result(c), (ne + 1) * 8, hipMemcpyDeviceToHost, strm(c)));
  PF_TRY(sync(c));
  for (int e = 0; e < ne; e++)
    if ((c->cfg.terms & PF_TERM_ELEC)) dtheta[e] += scale * c->host_res[e];
  if (c->cfg.terms & PF_TERM_LANDAU) dtheta[ne] += scale * c->host_res[ne];
  return PF_OK;
}

template <typename S>
pf_status adjoint_step_t(pf_ctx* c, const S* Pn, const S* Vn, S* lamP, S* lamV, double* dtheta,
                         const double* un = nullptr) {
  const bool pc = c->cfg.integrator == PF_INT_PC;
  const int64_t n3 = 3 * c->dims.N;
  const double dt = c->cfg.dt;
  double* w = scratch<double>(c, kScrW);
  double* Hw = scratch<double>(c, kScrHw);
  const S* V = pc ? Vn : nullptr;
  const double cdt = pc ? dt : 0.0;
  PF_HIP(c, launch_adjoint_axpy<S>(pc ? kAdjPrepPc : kAdjPrepEuler, dt, lamP, lamV, w, Hw, n3, strm(c)));
  pf_status s = hvp<S>(c, Pn, V, cdt, un);
  if (fatal(s)) return s;
  PF_TRY(theta_accumulate<S>(c, Pn, V, cdt, pc ? 1.0 : dt, dtheta));
  PF_HIP(c, launch_adjoint_axpy<S>(pc ? kAdjUpdPc : kAdjUpdEuler, dt, lamP, lamV, w, Hw, n3, strm(c)));
  PF_TRY(sync(c));
  return s;
}

template <typename S>
pf_status adjoint_initial_t(pf_ctx* c, const S* P0, S* lamP, S* lamV, double* dtheta) {
  const int64_t n3 = 3 * c->dims.N;
  double* w = scratch<double>(c, kScrW);
  double* Hw = scratch<double>(c, kScrHw);
  PF_HIP(c, launch_adjoint_axpy<S>(kAdjPrepInit, 0.0, lamP, lamV, w, Hw, n3, strm(c)));
  pf_status s = hvp<S>(c, P0, nullptr, 0.0);
  if (fatal(s)) return s;
  PF_TRY(theta_accumulate<S>(c, P0, nullptr, 0.0, 1.0, dtheta));
  PF_HIP(c, launch_adjoint_axpy<S>(kAdjUpdInit, 0.0, lamP, lamV, w, Hw, n3, strm(c)));
  PF_TRY(sync(c));
  return s;
}

// ---------------------------------------------------------------------------
// Energy
// ---------------------------------------------------------------------------

template <typename S>
pf_status energy_t(pf_ctx* c, const S* P, double out[5]) {
  const Dims& d = c->dims;
  const Coefs<double> cf = make_coefs<double>(c);
  pf_status st = PF_OK;
  double* phi = scratch<double>(c, kScrPhiE);
  double* u = scratch<double>(c, kScrUE);
  if (c->cfg.terms & PF_TERM_ELEC) {
    PF_TRY(ensure_phi_bc(c));
    PF_HIP(c, hipMemcpyAsync(phi, at<double>(c, c->lay.phi), c->dims_p.N * 8, hipMemcpyDeviceToDevice, strm(c)));
    SolveResult r{};
    pf_status s = solve_poisson64<S>(c, kPredAux, P, nullptr, 0.0, 1, 1, at<double>(c, c->lay.ghost64),
                                     c->cfg.phi_bottom, phi, c->cfg.tol_phi, true, &r);
    if (fatal(s)) return s;
    st = worst(st, s);
  }
  if (c->cfg.terms & PF_TERM_ELAS) {
    PF_HIP(c, hipMemcpyAsync(u, at<double>(c, c->lay.u), 3 * d.N * 8, hipMemcpyDeviceToDevice, strm(c)));
    SolveResult r{};
    pf_status s = solve_fem64<S>(c, kPredAux, P, nullptr, 0.0, nullptr, u, c->cfg.tol_u, true, &r);
    if (fatal(s)) return s;
    st = worst(st, s);
  }
  double* part = dev_partials(c, 2);
  PF_HIP(c, timed(c, PF_KC_OTHER, -1, -1, 3.0 * d.N * (sizeof(S) + 8) + 16.0 * c->dims_p.N, [&] {
    return launch_energy<S>(d, cf, at<FemTables>(c, c->lay.tables), P, phi, at<double>(c, c->lay.phi_bc),
                            at<double>(c, c->lay.ghost64), u, part, strm(c));
  }));
  PF_HIP(c, reduce(c, part, c->nblocks, 4, 2, kRedSum, 0, 0, dev_result(c)));
  if (c->cfg.terms & PF_TERM_ELEC) {
    PF_HIP(c, timed(c, PF_KC_OTHER, -1, -1, 3.0 * d.N * sizeof(S) + 16.0 * c->dims_p.N, [&] {
      return launch_elec_quad<S>(c->dims_p, cf, P, phi, at<double>(c, c->lay.phi_bc), emask(c), part, strm(c));
    }));
    PF_HIP(c, reduce(c, part, c->nblocks_p, 1, 2, kRedSum, 0, 0, dev_result(c) + 4));
  }
  PF_HIP(c, hipMemcpyAsync(c->host_res, dev_result(c), 5 * 8, hipMemcpyDeviceToHost, strm(c)));
  PF_TRY(sync(c));
  for (int t = 0; t < 4; t++) out[t] = c->host_res[t];
  if (c->cfg.terms & PF_TERM_ELEC) out[2] += c->host_res[4];
  out[4] = out[0] + out[1] + out[2] + out[3];
  return st;
}

}  // namespace
}  // namespace pf

namespace pf {
namespace {
// Tile grids of 64 x 4-node tiles sized to what stays resident at once, four
// 256-thread blocks per CU (the FEM iteration kernels are capped at 128
// VGPRs for that; their FP64 ring takes 28.5 KB of LDS).
// Tiles of the solver-grid kernels: z-chunks short enough for about 4096
// blocks (16 per CU: the small kernels keep 8 resident) while a chunk keeps
// at least 16 planes (its two halo planes cost at most 1/8 more reads);
// otherwise chunks for about 1024 blocks.
TileMap solver_tiles(const Dims& d) {
  const TileMap t = make_tile_map(d, kBY, 4096);
  return t.kz >= 16 ? t : make_tile_map(d, kBY, 1024);
}
TileMap poisson_tiles(const pf_config&, const Dims& d) { return solver_tiles(d); }
TileMap fem_tiles(const pf_config&, const Dims& d) { return solver_tiles(d); }
int partial_slots(const pf_config& c) {
  const Dims d = film_dims(c), dp = potential_dims(c);
  return std::max(std::max(node_blocks(d), node_blocks(dp)),
                  std::max(poisson_tiles(c, dp).nblocks, fem_tiles(c, d).nblocks));
}
}  // namespace
}  // namespace pf

namespace pf {
namespace {
MgHierarchy diag_hierarchy(const pf_config* cfg, int32_t field) {
  if (field == 0) return build_mg_phi(*cfg);
  FemTables t;
  build_tables(*cfg, &t);
  return build_mg(*cfg, t);
}
}  // namespace
}  // namespace pf

using namespace pf;

extern "C" {

const char* pf_status_str(pf_status s) {
  switch (s) {
    case PF_OK: return "ok";
    case PF_EINVAL: return "invalid argument";
    case PF_ENOMEM: return "workspace too small";
    case PF_EHIP: return "HIP runtime error";
    case PF_ENOCONV: return "CG did not converge";
    case PF_ENONFINITE: return "non-finite value";
    case PF_ESTATE: return "call out of order";
  }
  return "unknown status";
}

const char* pf_last_error(const pf_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

pf_status pf_workspace_size(const pf_config* cfg, size_t* bytes) {
  if (!bytes) return PF_EINVAL;
  pf_status s = validate(cfg, nullptr);
  if (s != PF_OK) return s;
  *bytes = make_layout(*cfg, partial_slots(*cfg)).total;
  return PF_OK;
}

namespace {

// pf_init and pf_init_static.  static_device >= 0: the workspace is that
// device's static array (claimed by the caller); the context then takes no
// pinned host memory, second stream or worker thread (its solves run one
// after the other on the caller's stream), so making it allocates no
// device memory.
pf_status init_ctx(const char* who, const pf_config* cfg, void* ws, size_t bytes, void* stream, int static_device,
                   pf_ctx** out) {
  pf_ctx* c = new pf_ctx();
  c->static_device = static_device;
  c->cfg = *cfg;
  c->electrodes.assign(cfg->electrodes, cfg->electrodes + cfg->n_electrodes);
  c->cfg.electrodes = c->electrodes.data();
  c->mat = make_material(*cfg);
  c->dims = film_dims(*cfg);
  c->dims_p = potential_dims(*cfg);
  c->nblocks = node_blocks(c->dims);
  c->nblocks_p = node_blocks(c->dims_p);
  c->tm_p = poisson_tiles(*cfg, c->dims_p);
  c->tm_f = fem_tiles(*cfg, c->dims);
  c->npartials = partial_slots(*cfg);
  c->lay = make_layout(*cfg, c->npartials);
  if (bytes < c->lay.total) {
    fprintf(stderr, "%s: workspace of %zu bytes, %zu needed\n", who, bytes, c->lay.total);
    delete c;
    return PF_ENOMEM;
  }
  c->ws = static_cast<char*>(ws);
  c->ws_bytes = bytes;
  c->stream = static_cast<hipStream_t>(stream);
  c->have_state = c->phi_bc_valid = c->basis_valid = c->adj_warm = false;
  c->hist_valid = 0;
  c->hist_head = 0;
  c->adj_valid = 0;
  c->adj_head = 0;
  c->lin_valid = 0;
  c->lin_head = 0;
  for (int f = 0; f < 2; f++) c->escore_host[f].assign((size_t)kScoreBlocks * (kMaxExtrap + 1), 0.0);
  c->step = 0;
  c->cur = 0;
  for (int t = 0; t < kPredCount; t++) c->pred[t] = 16;
  c->timing = PF_TIMING_OFF;
  std::memset(c->kc_ms, 0, sizeof(c->kc_ms));
  std::memset(c->kc_n, 0, sizeof(c->kc_n));
  std::memset(c->kc_bytes, 0, sizeof(c->kc_bytes));
  c->host_sc = nullptr;
  c->host_res = nullptr;
  if (static_device >= 0) {
    // read-backs into ordinary host memory, solves on the caller's stream
    c->device = static_device;
    c->host_sc = new CgScalars[kNumScalars];
    c->host_res = new double[kResultSlots];
  } else {
    if (hipHostMalloc(reinterpret_cast<void**>(&c->host_sc), sizeof(CgScalars) * kNumScalars,
                      hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&c->host_res), kResultSlots * 8, hipHostMallocDefault) != hipSuccess) {
      fprintf(stderr, "%s: pinned host allocation failed\n", who);
      pf_destroy(c);
      return PF_EHIP;
    }
    // the second stream (default priority) and the worker thread that uses it
    if (hipGetDevice(&c->device) != hipSuccess ||
        hipStreamCreateWithFlags(&c->stream2, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess ||
        hipStreamCreateWithFlags(&c->capture_stream[0], hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&c->capture_stream[1], hipStreamNonBlocking) != hipSuccess) {
      fprintf(stderr, "%s: stream or event creation failed\n", who);
      pf_destroy(c);
      return PF_EHIP;
    }
    c->graphs = true;
    c->worker.reset(new pf_ctx::Worker());
    c->worker->th = std::thread(worker_main, c);
  }
  FemTables tb;
  build_tables(c->cfg, &tb);
  c->gen = !c->mat.cubic || !tb.compact;
  pf_status st = PF_OK;
  hipError_t e = hipMemcpyAsync(c->ws + c->lay.tables, &tb, sizeof(tb), hipMemcpyHostToDevice, strm(c));
  if (e != hipSuccess) st = fail(c, PF_EHIP, "table upload: %s", hipGetErrorString(e));
  for (int f = 0; f < 2 && st == PF_OK; f++)
    if (!c->lay.mg[f].dinv.empty()) st = upload_mg(c, f, tb);
  if (st == PF_OK) st = upload_ghosts(c);
  if (st == PF_OK) {
    static_assert(sizeof(CgScalars) % 8 == 0, "scalars are cleared as doubles");
    e = launch_fill<double>(reinterpret_cast<double*>(c->ws + c->lay.scalars),
                            (int64_t)(sizeof(CgScalars) * kNumScalars / 8), 0.0, strm(c));
    if (e == hipSuccess) e = hipStreamSynchronize(strm(c));
    if (e != hipSuccess) st = fail(c, PF_EHIP, "init: %s", hipGetErrorString(e));
  }
  if (st != PF_OK) {
    fprintf(stderr, "%s: %s\n", who, c->err.c_str());
    pf_destroy(c);
    return st;
  }
  *out = c;
  return PF_OK;
}

}  // namespace

pf_status pf_init(const pf_config* cfg, void* ws, size_t bytes, void* stream, pf_ctx** out) {
  if (!out) return PF_EINVAL;
  *out = nullptr;
  std::string why;
  if (validate(cfg, &why) != PF_OK) {
    fprintf(stderr, "pf_init: %s\n", why.c_str());
    return PF_EINVAL;
  }
  if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) {
    fprintf(stderr, "pf_init: workspace must be non-null and 256-byte aligned\n");
    return PF_EINVAL;
  }
  return init_ctx("pf_init", cfg, ws, bytes, stream, -1, out);
}

pf_status pf_init_static(const pf_config* cfg, void* stream, pf_ctx** out) {
  if (!out) return PF_EINVAL;
  *out = nullptr;
  std::string why;
  if (validate(cfg, &why) != PF_OK) {
    fprintf(stderr, "pf_init_static: %s\n", why.c_str());
    return PF_EINVAL;
  }
  size_t need = 0;
  if (pf_workspace_size(cfg, &need) != PF_OK) return PF_EINVAL;
  if (need > kStaticWorkspaceBytes) {
    fprintf(stderr, "pf_init_static: the configuration needs a workspace of %zu bytes; the static workspace holds "
            "%zu (use pf_init with a workspace of the caller's)\n", need, kStaticWorkspaceBytes);
    return PF_EINVAL;
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) {
    fprintf(stderr, "pf_init_static: no current device\n");
    return PF_EHIP;
  }
  void* ws = nullptr;
  const hipError_t e = static_workspace_acquire(dev, &ws);
  if (e == hipErrorAlreadyAcquired) {
    fprintf(stderr, "pf_init_static: another context uses the static workspace of device %d\n", dev);
    return PF_ESTATE;
  }
  if (e != hipSuccess) {
    fprintf(stderr, "pf_init_static: static workspace of device %d: %s\n", dev, hipGetErrorString(e));
    return PF_EHIP;
  }
  const pf_status st = init_ctx("pf_init_static", cfg, ws, kStaticWorkspaceBytes, stream, dev, out);
  if (st != PF_OK) static_workspace_release(dev);
  return st;
}

void pf_destroy(pf_ctx* c) {
  if (!c) return;
  if (c->worker) {
    {
      std::lock_guard<std::mutex> g(c->worker->mu);
      c->worker->quit = true;
      c->worker->cv.notify_all();
    }
    c->worker->th.join();
    c->worker.reset();
  }
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  if (c->stream2) (void)hipStreamDestroy(c->stream2);
  if (c->mg_graph[0][0] || c->mg_graph[0][1] || c->mg_graph[1][0] || c->mg_graph[1][1]) {
    // no replay may still be queued when its graph goes
    if (c->stream2) (void)hipStreamSynchronize(c->stream2);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
  }
  for (int f = 0; f < 2; f++) {
    for (int t = 0; t < 2; t++)
      if (c->mg_graph[f][t]) (void)hipGraphExecDestroy(c->mg_graph[f][t]);
    if (c->capture_stream[f]) (void)hipStreamDestroy(c->capture_stream[f]);
  }
  for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
  if (c->static_device >= 0) {
    // the static workspace is free for the device's next context once the
    // work queued on it has finished
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    delete[] c->host_sc;
    delete[] c->host_res;
    static_workspace_release(c->static_device);
  } else {
    if (c->host_sc) (void)hipHostFree(c->host_sc);
    if (c->host_res) (void)hipHostFree(c->host_res);
  }
  delete c;
}

pf_status pf_set_state(pf_ctx* c, const void* P, const void* phi0, const void* u0) {
  if (!c || !P) return fail(c, PF_EINVAL, "pf_set_state: null argument");
  const int64_t N = c->dims.N, Np = c->dims_p.N;
  const size_t es = state_bytes(c);
  c->cur = 0;
  c->step = 0;
  c->hist_valid = 0;
  c->hist_head = 0;
  void* Pc = c->ws + c->lay.P[0];
  void* Vc = c->ws + c->lay.V[0];
  double* phi = at<double>(c, c->lay.phi);
  double* u = at<double>(c, c->lay.u);
  PF_HIP(c, hipMemcpyAsync(Pc, P, 3 * N * es, hipMemcpyDeviceToDevice, strm(c)));
  if (phi0) PF_HIP(c, hipMemcpyAsync(phi, phi0, Np * 8, hipMemcpyDeviceToDevice, strm(c)));
  else PF_HIP(c, launch_fill<double>(phi, Np, 0.0, strm(c)));
  if (u0) PF_HIP(c, hipMemcpyAsync(u, u0, 3 * N * 8, hipMemcpyDeviceToDevice, strm(c)));
  else PF_HIP(c, launch_fill<double>(u, 3 * N, 0.0, strm(c)));
  if (fp32(c)) {
    PF_HIP(c, launch_convert<double, float>(phi, at<float>(c, c->lay.phi32), Np, strm(c)));
    PF_HIP(c, launch_convert<double, float>(u, at<float>(c, c->lay.u32), 3 * N, strm(c)));
    PF_HIP(c, launch_fill<float>(static_cast<float*>(Vc), 3 * N, 0.0f, strm(c)));
  } else {
    PF_HIP(c, launch_fill<double>(static_cast<double*>(Vc), 3 * N, 0.0, strm(c)));
  }
  pf_status s = PF_OK;
  if (c->cfg.integrator == PF_INT_PC) {
    s = solve_nonlocal(c, Pc, nullptr, 0.0, true, nullptr);
    if (fatal(s)) return s;
    PF_TRY(launch_state_force(c, Pc, nullptr, 0.0, kPcInit, nullptr, Vc, nullptr));
  }
  PF_TRY(sync(c));
  c->have_state = true;
  return s;
}

pf_status pf_restore_state(pf_ctx* c, const void* P, const void* V, const void* phi, const void* u, int64_t step) {
  if (!c || !P || !V || !phi || !u) return fail(c, PF_EINVAL, "pf_restore_state: null argument");
  const int64_t N = c->dims.N, Np = c->dims_p.N;
  const size_t es = state_bytes(c);
  c->cur = 0;
  c->hist_valid = 0;
  c->hist_head = 0;
  PF_HIP(c, hipMemcpyAsync(c->ws + c->lay.P[0], P, 3 * N * es, hipMemcpyDeviceToDevice, strm(c)));
  PF_HIP(c, hipMemcpyAsync(c->ws + c->lay.V[0], V, 3 * N * es, hipMemcpyDeviceToDevice, strm(c)));
  PF_HIP(c, hipMemcpyAsync(at<double>(c, c->lay.phi), phi, Np * 8, hipMemcpyDeviceToDevice, strm(c)));
  PF_HIP(c, hipMemcpyAsync(at<double>(c, c->lay.u), u, 3 * N * 8, hipMemcpyDeviceToDevice, strm(c)));
  if (fp32(c)) {
    PF_HIP(c, launch_convert<double, float>(at<double>(c, c->lay.phi), at<float>(c, c->lay.phi32), Np, strm(c)));
    PF_HIP(c, launch_convert<double, float>(at<double>(c, c->lay.u), at<float>(c, c->lay.u32), 3 * N, strm(c)));
  }
  c->step = step;
  c->have_state = true;
  return PF_OK;
}

pf_status pf_get_state(const pf_ctx* cc, void* P, void* V, void* phi, void* u, int64_t* step) {
  pf_ctx* c = const_cast<pf_ctx*>(cc);
  if (!c) return PF_EINVAL;
  if (!c->have_state) return fail(c, PF_ESTATE, "pf_get_state: no state (call pf_set_state first)");
  const int64_t N = c->dims.N, Np = c->dims_p.N;
  const size_t es = state_bytes(c);
  if (P) PF_HIP(c, hipMemcpyAsync(P, c->ws + c->lay.P[c->cur], 3 * N * es, hipMemcpyDeviceToDevice, strm(c)));
  if (V) PF_HIP(c, hipMemcpyAsync(V, c->ws + c->lay.V[c->cur], 3 * N * es, hipMemcpyDeviceToDevice, strm(c)));
  if (phi) PF_HIP(c, hipMemcpyAsync(phi, at<double>(c, c->lay.phi), Np * 8, hipMemcpyDeviceToDevice, strm(c)));
  if (u) PF_HIP(c, hipMemcpyAsync(u, at<double>(c, c->lay.u), 3 * N * 8, hipMemcpyDeviceToDevice, strm(c)));
  if (step) *step = c->step;
  return PF_OK;
}

pf_status pf_step(pf_ctx* c, int32_t nsteps, pf_step_stats* st) {
  if (!c) return PF_EINVAL;
  if (nsteps < 0) return fail(c, PF_EINVAL, "pf_step: nsteps < 0");
  if (!c->have_state) return fail(c, PF_ESTATE, "pf_step: no state (call pf_set_state first)");
  if (st) std::memset(st, 0, sizeof(*st));
  const bool pc = c->cfg.integrator == PF_INT_PC;
  const int every = c->cfg.nonlocal_every <= 1 ? 1 : c->cfg.nonlocal_every;
  pf_status out = PF_OK;
  for (int s = 0; s < nsteps; s++) {
    void* P = c->ws + c->lay.P[c->cur];
    void* V = c->ws + c->lay.V[c->cur];
    void* Pn = c->ws + c->lay.P[c->cur ^ 1];
    void* Vn = c->ws + c->lay.V[c->cur ^ 1];
    if (c->step % every == 0) {
      ExtrapRing ring[2];
      const bool ex = c->cfg.warm_start >= 2 && extrapolate_plan(c, ring);
      pf_status r = solve_nonlocal(c, P, pc ? V : nullptr, pc ? c->cfg.dt : 0.0, c->cfg.warm_start != 0, st,
                                   ex ? ring : nullptr);
      if (fatal(r)) return r;
      out = worst(out, r);
    }
    PF_TRY(launch_state_force(c, P, pc ? V : nullptr, pc ? c->cfg.dt : 0.0, pc ? kPcStep : kEulerStep, Pn, Vn,
                              nullptr));
    c->cur ^= 1;
    c->step++;
    if (st) st->steps++;
  }
  PF_TRY(sync(c));
  return out;
}

pf_status pf_solve_phi(pf_ctx* c, const void* P, void* phi, pf_solve_stats* st) {
  if (!c || !P || !phi) return fail(c, PF_EINVAL, "pf_solve_phi: null argument");
  SolveResult r{};
  pf_status s;
  if (fp32(c))
    s = solve_refined<float>(c, false, static_cast<const float*>(P), nullptr, 0.0, static_cast<double*>(phi),
                             scratch<float>(c, kScrTmp), c->cfg.tol_phi, c->cfg.warm_start != 0, &r);
  else if (refined(c))
    s = solve_refined<double>(c, false, static_cast<const double*>(P), nullptr, 0.0, static_cast<double*>(phi),
                              scratch<float>(c, kScrTmp), c->cfg.tol_phi, c->cfg.warm_start != 0, &r);
  else
    s = solve_poisson64<double>(c, kPredAux, static_cast<const double*>(P), nullptr, 0.0, 1, 1,
                                at<double>(c, c->lay.ghost64), c->cfg.phi_bottom, static_cast<double*>(phi),
                                c->cfg.tol_phi, c->cfg.warm_start != 0, &r);
  if (st) {
    st->iters = r.iters;
    st->outer = r.outer;
    st->relres = r.relres;
  }
  pf_status e = sync(c);
  return fatal(e) ? e : s;
}

pf_status pf_solve_u(pf_ctx* c, const void* P, void* u, pf_solve_stats* st) {
  if (!c || !P || !u) return fail(c, PF_EINVAL, "pf_solve_u: null argument");
  SolveResult r{};
  pf_status s;
  if (fp32(c))
    s = solve_refined<float>(c, true, static_cast<const float*>(P), nullptr, 0.0, static_cast<double*>(u),
                             scratch<float>(c, kScrTmp), c->cfg.tol_u, c->cfg.warm_start != 0, &r);
  else if (refined(c))
    s = solve_refined<double>(c, true, static_cast<const double*>(P), nullptr, 0.0, static_cast<double*>(u),
                              scratch<float>(c, kScrTmp), c->cfg.tol_u, c->cfg.warm_start != 0, &r);
  else
    s = solve_fem64<double>(c, kPredAux, static_cast<const double*>(P), nullptr, 0.0, nullptr,
                            static_cast<double*>(u), c->cfg.tol_u, c->cfg.warm_start != 0, &r);
  if (st) {
    st->iters = r.iters;
    st->outer = r.outer;
    st->relres = r.relres;
  }
  pf_status e = sync(c);
  return fatal(e) ? e : s;
}

pf_status pf_noise(pf_ctx* c, int64_t step, double* xi) {
  if (!c || !xi) return fail(c, PF_EINVAL, "pf_noise: null argument");
  PF_HIP(c, launch_noise(noise_spec(c, step, true), c->dims.N, xi, strm(c)));
  return PF_OK;
}

pf_status pf_force(pf_ctx* c, const void* P, const void* phi, const void* u, void* F) {
  if (!c || !P || !F) return fail(c, PF_EINVAL, "pf_force: null argument");
  if ((c->cfg.terms & PF_TERM_ELEC) && !phi) return fail(c, PF_EINVAL, "pf_force: phi needed");
  if ((c->cfg.terms & PF_TERM_ELAS) && !u) return fail(c, PF_EINVAL, "pf_force: u needed");
  const int64_t N = c->dims.N;
  if (fp32(c)) {
    // rounded copies in two scratch slots (free outside pf_energy): phi
    // spans the potential grid, air planes of the open top included
    float* phi32 = scratch<float>(c, kScrTmp);
    float* u32 = scratch<float>(c, kScrUE);
    if (phi) PF_HIP(c, launch_convert<double, float>(static_cast<const double*>(phi), phi32, c->dims_p.N, strm(c)));
    if (u) PF_HIP(c, launch_convert<double, float>(static_cast<const double*>(u), u32, 3 * N, strm(c)));
    return launch_state_force(c, P, nullptr, 0.0, kForceOut, nullptr, nullptr, F, phi32, u32);
  }
  return launch_state_force(c, P, nullptr, 0.0, kForceOut, nullptr, nullptr, F, phi, u);
}

pf_status pf_energy(pf_ctx* c, double out[5]) {
  if (!c || !out) return fail(c, PF_EINVAL, "pf_energy: null argument");
  if (!c->have_state) return fail(c, PF_ESTATE, "pf_energy: no state (call pf_set_state first)");
  const void* P = c->ws + c->lay.P[c->cur];
  if (fp32(c)) return energy_t<float>(c, static_cast<const float*>(P), out);
  return energy_t<double>(c, static_cast<const double*>(P), out);
}

pf_status pf_set_params(pf_ctx* c, const double* volts, double a1) {
  if (!c) return PF_EINVAL;
  // validate everything before changing anything: a rejected call leaves the
  // parameters as they were
  if (!std::isfinite(a1)) return fail(c, PF_EINVAL, "pf_set_params: a1 not finite");
  if (volts)
    for (int e = 0; e < c->cfg.n_electrodes; e++)
      if (!std::isfinite(volts[e])) return fail(c, PF_EINVAL, "pf_set_params: voltage not finite");
  c->cfg.a1 = a1;
  if (volts) {
    for (int e = 0; e < c->cfg.n_electrodes; e++) c->electrodes[e].volts = volts[e];
    c->phi_bc_valid = false;
    c->hist_valid = 0;
    c->hist_head = 0;
    PF_TRY(upload_ghosts(c));
  }
  return PF_OK;
}

pf_status pf_adjoint_step_u(pf_ctx* c, const void* P_n, const void* V_n, const void* u_n, void* lamP, void* lamV,
                            double* dtheta) {
  if (!c || !P_n || !lamP || !lamV || !dtheta) return fail(c, PF_EINVAL, "pf_adjoint_step: null argument");
  if (c->cfg.integrator == PF_INT_PC && !V_n) return fail(c, PF_EINVAL, "pf_adjoint_step: V_n needed");
  if (c->cfg.nonlocal_every > 1)
    return fail(c, PF_EINVAL, "pf_adjoint_step: the adjoint needs phi and u refreshed every step");
  const double* un = static_cast<const double*>(u_n);
  if (fp32(c))
    return adjoint_step_t<float>(c, static_cast<const float*>(P_n), static_cast<const float*>(V_n),
                                 static_cast<float*>(lamP), static_cast<float*>(lamV), dtheta, un);
  return adjoint_step_t<double>(c, static_cast<const double*>(P_n), static_cast<const double*>(V_n),
                                static_cast<double*>(lamP), static_cast<double*>(lamV), dtheta, un);
}

pf_status pf_adjoint_step(pf_ctx* c, const void* P_n, const void* V_n, void* lamP, void* lamV, double* dtheta) {
  return pf_adjoint_step_u(c, P_n, V_n, nullptr, lamP, lamV, dtheta);
}

pf_status pf_adjoint_initial_rate(pf_ctx* c, const void* P0, void* lamP, void* lamV, double* dtheta) {
  if (!c || !P0 || !lamP || !lamV || !dtheta) return fail(c, PF_EINVAL, "pf_adjoint_initial_rate: null argument");
  pf_status s = PF_OK;
  if (c->cfg.integrator == PF_INT_PC) {
    if (fp32(c))
      s = adjoint_initial_t<float>(c, static_cast<const float*>(P0), static_cast<float*>(lamP),
                                   static_cast<float*>(lamV), dtheta);
    else
      s = adjoint_initial_t<double>(c, static_cast<const double*>(P0), static_cast<double*>(lamP),
                                    static_cast<double*>(lamV), dtheta);
  }
  // The reverse sweep ends here: the next adjoint step starts its solves from
  // zero, so a sweep does not depend on the solutions of an earlier one.
  c->adj_warm = false;
  c->adj_valid = c->adj_head = 0;
  c->lin_valid = c->lin_head = 0;
  return s;
}

pf_status pf_timing(pf_ctx* c, int mode, double* ms, int64_t* launches, double* bytes) {
  if (!c) return PF_EINVAL;
  if (mode != PF_TIMING_OFF && mode != PF_TIMING_EVENTS && mode != PF_TIMING_BYTES)
    return fail(c, PF_EINVAL, "pf_timing: unknown mode %d", mode);
  PF_TRY(sync(c));
  // every solve has read back its iteration count by now: what is still
  // pending (the worker's last launches) counts in full
  if (c->timing) {
    collect_timing(c, -1, 0, 0);
    collect_timing(c, -1, 0, 1);
  }
  for (int t = 0; t < PF_KC_COUNT; t++) {
    if (ms) ms[t] = c->kc_ms[t];
    if (launches) launches[t] = c->kc_n[t];
    if (bytes) bytes[t] = c->kc_bytes[t];
    c->kc_ms[t] = 0;
    c->kc_n[t] = 0;
    c->kc_bytes[t] = 0;
  }
  c->timing = mode;
  return PF_OK;
}

pf_status pf_mg_levels(const pf_config* cfg, int32_t field, int32_t* nlevels, int32_t* dims, double* omega,
                       int32_t max_levels) {
  if (!nlevels || (field != 0 && field != 1) || validate(cfg, nullptr) != PF_OK) return PF_EINVAL;
  const MgHierarchy h = diag_hierarchy(cfg, field);
  *nlevels = (int32_t)h.levels.size();
  for (int l = 0; l < (int)h.levels.size() && l < max_levels; l++) {
    if (dims) {
      dims[3 * l] = h.levels[l].nx;
      dims[3 * l + 1] = h.levels[l].ny;
      dims[3 * l + 2] = h.levels[l].nz;
    }
    if (omega) omega[l] = h.levels[l].omega;
  }
  return PF_OK;
}

pf_status pf_mg_table(const pf_config* cfg, int32_t field, int32_t level, double* out, size_t count) {
  if (!out || (field != 0 && field != 1) || validate(cfg, nullptr) != PF_OK) return PF_EINVAL;
  const MgHierarchy h = diag_hierarchy(cfg, field);
  if (level < 0 || level >= (int32_t)h.levels.size()) return PF_EINVAL;
  const std::vector<double>& T = h.tables[level];
  if (count < T.size()) return PF_EINVAL;
  std::memcpy(out, T.data(), T.size() * 8);
  return PF_OK;
}

size_t pf_fem_table_size(void) {
  FemTables* t = nullptr;
  return sizeof(t->K) / 8 + sizeof(t->Bf) / 8 + sizeof(t->Su) / 8 + sizeof(t->Ms) / 8;
}

pf_status pf_fem_tables(const pf_config* cfg, double* out, size_t count) {
  if (!out || count < pf_fem_table_size()) return PF_EINVAL;
  if (validate(cfg, nullptr) != PF_OK) return PF_EINVAL;
  FemTables t;
  build_tables(*cfg, &t);
  double* o = out;
  std::memcpy(o, t.K, sizeof(t.K));
  o += sizeof(t.K) / 8;
  std::memcpy(o, t.Bf, sizeof(t.Bf));
  o += sizeof(t.Bf) / 8;
  std::memcpy(o, t.Su, sizeof(t.Su));
  o += sizeof(t.Su) / 8;
  std::memcpy(o, t.Ms, sizeof(t.Ms));
  return PF_OK;
}

}  // extern "C"
