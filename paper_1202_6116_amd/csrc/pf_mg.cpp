// Multigrid hierarchy of the FEM operator (host): grid levels, Galerkin
// coarse operators A_{l+1} = P^T A_l P as per-plane 27-point block stencils,
// Jacobi weights, smoother damping and the coarsest level's inverse.
//
// The film is periodic in x and y, clamped on plane 0 and free on top, so
// every level operator is invariant under x/y translations and varies only
// with the plane.  Prolongation P is trilinear: in x and y coarse node I sits
// on fine node 2I (a level is halved while it is even and at least 8 wide);
// in z the coarse planes are the even fine planes plus the top plane, so the
// free surface stays on every level.  The coarse stencils are read off
// A_{l+1} applied to unit vectors on small periodic probe domains, which is
// exact because P, A_l and P^T all have a support of one coarse cell.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "pf.h"
#include "pf_internal.h"

namespace pf {

namespace {

inline int tap_index(int dx, int dy, int dz) { return (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1); }
inline int wrap_host(int i, int n) { return ((i % n) + n) % n; }

// A level operator on a periodic probe domain (wx x wy x nz, nc components,
// component-major) from per-plane stencils T[k][c][e][o].  Plane 0, and the
// top plane when it is fixed, hold no unknowns: their rows and columns are
// zero.
struct ProbeOp {
  int wx, wy, nz, nc;
  bool top_fixed;
  const std::vector<double>* planes;
  int64_t plane() const { return (int64_t)wx * wy; }
  int64_t n() const { return plane() * nz; }
  bool active(int k) const { return k >= 1 && k < nz - (top_fixed ? 1 : 0); }
  double coef(int k, int c, int e, int o) const {
    return (*planes)[(((size_t)k * nc + c) * nc + e) * 27 + o];
  }
  void apply(const std::vector<double>& x, std::vector<double>& y) const {
    const int64_t N = n();
    y.assign((size_t)nc * N, 0.0);
    for (int k = 0; k < nz; k++) {
      if (!active(k)) continue;
      for (int j = 0; j < wy; j++)
        for (int i = 0; i < wx; i++) {
          const int64_t r = i + (int64_t)wx * (j + (int64_t)wy * k);
          for (int dz = -1; dz <= 1; dz++) {
            const int kk = k + dz;
            if (kk < 0 || kk >= nz || !active(kk)) continue;
            for (int dy = -1; dy <= 1; dy++)
              for (int dx = -1; dx <= 1; dx++) {
                const int o = tap_index(dx, dy, dz);
                const int64_t m = wrap_host(i + dx, wx) + (int64_t)wx * (wrap_host(j + dy, wy) + (int64_t)wy * kk);
                for (int c = 0; c < nc; c++)
                  for (int e = 0; e < nc; e++) y[c * N + r] += coef(k, c, e, o) * x[e * N + m];
              }
          }
        }
    }
  }
  double diag(int k, int c) const { return coef(k, c, c, 13); }
};

// Prolongation between a fine domain (fx, fy, fz) and a coarse one; fixed
// planes (0, and the tops when fixed) carry zero.
struct ProbeTransfer {
  int fx, fy, fz, cx_, cy_, cz, nc;
  bool cx, cy, top_fixed;
  const std::vector<MgZ>* zmap;  // per fine plane
  bool fine_active(int k) const { return k >= 1 && k < fz - (top_fixed ? 1 : 0); }
  bool coarse_active(int k) const { return k >= 1 && k < cz - (top_fixed ? 1 : 0); }
  template <typename F>
  void for_parents(int i, int j, int k, F f) const {
    int xi[2], yi[2];
    double xw[2], yw[2];
    int nxp, nyp;
    if (cx) {
      if (i % 2 == 0) {
        xi[0] = i / 2, xw[0] = 1.0, nxp = 1;
      } else {
        xi[0] = (i - 1) / 2, xi[1] = wrap_host((i + 1) / 2, cx_), xw[0] = xw[1] = 0.5, nxp = 2;
      }
    } else {
      xi[0] = i, xw[0] = 1.0, nxp = 1;
    }
    if (cy) {
      if (j % 2 == 0) {
        yi[0] = j / 2, yw[0] = 1.0, nyp = 1;
      } else {
        yi[0] = (j - 1) / 2, yi[1] = wrap_host((j + 1) / 2, cy_), yw[0] = yw[1] = 0.5, nyp = 2;
      }
    } else {
      yi[0] = j, yw[0] = 1.0, nyp = 1;
    }
    const MgZ& z = (*zmap)[k];
    const int zi[2] = {z.lo, z.hi};
    const double zw[2] = {z.wlo, z.whi};
    for (int a = 0; a < 2; a++) {
      if (zw[a] == 0.0 || !coarse_active(zi[a])) continue;
      for (int b = 0; b < nyp; b++)
        for (int q = 0; q < nxp; q++) f(xi[q], yi[b], zi[a], zw[a] * yw[b] * xw[q]);
    }
  }
  void prolong(const std::vector<double>& xc, std::vector<double>& xf) const {
    const int64_t Nf = (int64_t)fx * fy * fz, Nc = (int64_t)cx_ * cy_ * cz;
    xf.assign((size_t)nc * Nf, 0.0);
    for (int k = 0; k < fz; k++) {
      if (!fine_active(k)) continue;
      for (int j = 0; j < fy; j++)
        for (int i = 0; i < fx; i++) {
          const int64_t r = i + (int64_t)fx * (j + (int64_t)fy * k);
          for_parents(i, j, k, [&](int I, int J, int K, double w) {
            const int64_t m = I + (int64_t)cx_ * (J + (int64_t)cy_ * K);
            for (int c = 0; c < nc; c++) xf[c * Nf + r] += w * xc[c * Nc + m];
          });
        }
    }
  }
  void restrict_(const std::vector<double>& yf, std::vector<double>& yc) const {
    const int64_t Nf = (int64_t)fx * fy * fz, Nc = (int64_t)cx_ * cy_ * cz;
    yc.assign((size_t)nc * Nc, 0.0);
    for (int k = 0; k < fz; k++) {
      if (!fine_active(k)) continue;
      for (int j = 0; j < fy; j++)
        for (int i = 0; i < fx; i++) {
          const int64_t r = i + (int64_t)fx * (j + (int64_t)fy * k);
          for_parents(i, j, k, [&](int I, int J, int K, double w) {
            const int64_t m = I + (int64_t)cx_ * (J + (int64_t)cy_ * K);
            for (int c = 0; c < nc; c++) yc[c * Nc + m] += w * yf[c * Nf + r];
          });
        }
    }
  }
};

// Coarse planes in z: the even fine planes and the top plane.
std::vector<int> coarse_planes(int nz) {
  std::vector<int> z;
  for (int k = 0; k < nz; k += 2) z.push_back(k);
  if (z.back() != nz - 1) z.push_back(nz - 1);
  return z;
}

std::vector<MgZ> zmap_for(int nz, const std::vector<int>& zc) {
  std::vector<MgZ> m(nz);
  for (int k = 0; k < nz; k++) {
    MgZ& e = m[k];
    auto it = std::lower_bound(zc.begin(), zc.end(), k);
    if (*it == k) {
      e.lo = e.hi = (int)(it - zc.begin());
      e.wlo = 1.0;
      e.whi = 0.0;
    } else {
      const int b = (int)(it - zc.begin()), a = b - 1;
      const double span = zc[b] - zc[a];
      e.lo = a;
      e.hi = b;
      e.wlo = (zc[b] - k) / span;
      e.whi = (k - zc[a]) / span;
    }
  }
  return m;
}

// Largest eigenvalue of D^-1 A on an 8 x 8 periodic probe (power iteration).
double jacobi_lambda_max(int nz, int nc, bool top_fixed, const std::vector<double>* planes) {
  ProbeOp op{8, 8, nz, nc, top_fixed, planes};
  const int64_t N = op.n();
  std::vector<double> x((size_t)nc * N), y;
  uint32_t s = 12345u;
  for (int64_t t = 0; t < nc * N; t++) {
    s = s * 1664525u + 1013904223u;
    x[t] = op.active((int)((t % N) / op.plane())) ? (double)(s >> 8) / (double)(1u << 24) - 0.5 : 0.0;
  }
  double lam = 0.0;
  for (int it = 0; it < 60; it++) {
    op.apply(x, y);
    double nrm = 0.0;
    for (int c = 0; c < nc; c++)
      for (int64_t m = 0; m < N; m++) {
        const int k = (int)(m / op.plane());
        if (!op.active(k)) continue;
        y[c * N + m] /= op.diag(k, c);
        nrm += y[c * N + m] * y[c * N + m];
      }
    nrm = std::sqrt(nrm);
    if (!(nrm > 0)) break;
    lam = nrm;
    for (int64_t t = 0; t < nc * N; t++) x[t] = y[t] / nrm;
  }
  return lam;
}

// In-place inverse of a symmetric positive definite matrix (Cholesky).
bool spd_inverse(std::vector<double>& A, int n) {
  std::vector<double> L(A.size(), 0.0);
  for (int j = 0; j < n; j++) {
    double d = A[(size_t)j * n + j];
    for (int k = 0; k < j; k++) d -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
    if (!(d > 0)) return false;
    const double ljj = std::sqrt(d);
    L[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; i++) {
      double s = A[(size_t)i * n + j];
      for (int k = 0; k < j; k++) s -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      L[(size_t)i * n + j] = s / ljj;
    }
  }
  // inverse = L^-T L^-1, column by column
  std::vector<double> col(n);
  for (int c = 0; c < n; c++) {
    for (int i = 0; i < n; i++) {
      double s = i == c ? 1.0 : 0.0;
      for (int k = 0; k < i; k++) s -= L[(size_t)i * n + k] * col[k];
      col[i] = s / L[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; i--) {
      double s = col[i];
      for (int k = i + 1; k < n; k++) s -= L[(size_t)k * n + i] * col[k];
      col[i] = s / L[(size_t)i * n + i];
    }
    for (int i = 0; i < n; i++) A[(size_t)i * n + c] = col[i];
  }
  return true;
}

int64_t unknowns(const MgLevel& l, int nc, bool top_fixed) {
  return (int64_t)nc * l.nx * l.ny * (l.nz - 1 - (top_fixed ? 1 : 0));
}

// Grid levels: halve x and y while even and at least 8 wide, keep every
// other plane and the top in z, until the coarsest level has at most
// kMgDenseMax unknowns or nothing can be coarsened.
std::vector<MgLevel> plan_levels(int nx, int ny, int nz, int nc, bool top_fixed) {
  std::vector<MgLevel> lv;
  MgLevel l0;
  l0.nx = nx, l0.ny = ny, l0.nz = nz;
  l0.cx = l0.cy = false;
  l0.omega = 0.0;
  lv.push_back(l0);
  for (;;) {
    const MgLevel f = lv.back();
    if (unknowns(f, nc, top_fixed) <= kMgDenseMax) break;
    const bool cx = f.nx % 2 == 0 && f.nx >= 8, cy = f.ny % 2 == 0 && f.ny >= 8;
    const int nzc = (int)coarse_planes(f.nz).size();
    if (!cx && !cy && nzc == f.nz) break;
    if ((int)lv.size() >= kMgMaxLevels) break;
    MgLevel c;
    c.nx = cx ? f.nx / 2 : f.nx;
    c.ny = cy ? f.ny / 2 : f.ny;
    c.nz = nzc;
    c.cx = cx, c.cy = cy;
    c.omega = 0.0;
    lv.push_back(c);
  }
  return lv;
}

// The hierarchy for a level-0 operator given as per-plane stencils.
MgHierarchy build_generic(int nx, int ny, int nz, int nc, bool top_fixed, std::vector<double> level0) {
  MgHierarchy h;
  h.nc = nc;
  h.top_fixed = top_fixed;
  const std::vector<MgLevel> plan = plan_levels(nx, ny, nz, nc, top_fixed);
  h.levels.push_back(plan[0]);
  h.tables.push_back(std::move(level0));
  h.zmaps.emplace_back();
  h.zfine.emplace_back();
  const size_t blk = (size_t)nc * nc * 27;
  for (size_t l = 1; l < plan.size(); l++) {
    const MgLevel& f = h.levels.back();
    const MgLevel& c = plan[l];
    const bool cx = c.cx, cy = c.cy;
    const std::vector<int> zc = coarse_planes(f.nz);
    const std::vector<MgZ> zm = zmap_for(f.nz, zc);
    // Galerkin operator by probing on periodic domains of 4 (coarsened) or
    // 3 (kept) coarse nodes per direction.
    const int wcx = cx ? 4 : 3, wcy = cy ? 4 : 3;
    const int wfx = cx ? 8 : 3, wfy = cy ? 8 : 3;
    const size_t lf = h.levels.size() - 1;
    ProbeOp fine_op{wfx, wfy, f.nz, nc, top_fixed, &h.tables[lf]};
    ProbeTransfer tr{wfx, wfy, f.nz, wcx, wcy, c.nz, nc, cx, cy, top_fixed, &zm};
    std::vector<double> T((size_t)c.nz * blk, 0.0);
    const int64_t Nc = (int64_t)wcx * wcy * c.nz;
    std::vector<double> u((size_t)nc * Nc), v, w, y;
    for (int K = 1; K < c.nz - (top_fixed ? 1 : 0); K++)
      for (int e = 0; e < nc; e++) {
        std::fill(u.begin(), u.end(), 0.0);
        u[e * Nc + (int64_t)wcx * wcy * K] = 1.0;
        tr.prolong(u, v);
        fine_op.apply(v, w);
        tr.restrict_(w, y);
        // column (e, K) at the origin: row (c, K') at (-dx, -dy) is the
        // coefficient of offset (dx, dy, K - K')
        for (int Kr = std::max(1, K - 1); Kr <= std::min(c.nz - 1, K + 1); Kr++)
          for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
              const int64_t m = wrap_host(-dx, wcx) + (int64_t)wcx * (wrap_host(-dy, wcy) + (int64_t)wcy * Kr);
              for (int cc = 0; cc < nc; cc++)
                T[(((size_t)Kr * nc + cc) * nc + e) * 27 + tap_index(dx, dy, K - Kr)] = y[cc * Nc + m];
            }
      }
    h.levels.push_back(c);
    h.tables.push_back(std::move(T));
    h.zmaps.push_back(zm);
    h.zfine.push_back(zc);
  }
  // Jacobi weights and smoother damping per level
  for (size_t l = 0; l < h.levels.size(); l++) {
    MgLevel& L = h.levels[l];
    ProbeOp op{8, 8, L.nz, nc, top_fixed, &h.tables[l]};
    L.dinv.assign((size_t)L.nz * nc, 0.0);
    for (int k = 0; k < L.nz; k++)
      if (op.active(k))
        for (int c = 0; c < nc; c++) L.dinv[(size_t)k * nc + c] = 1.0 / op.diag(k, c);
    const double lam = jacobi_lambda_max(L.nz, nc, top_fixed, &h.tables[l]);
    // damping of the Jacobi smoother: 4 / (3 lambda_max(D^-1 A)) is the
    // classic choice for smoothing alone; as the preconditioner of CG the
    // cycle converges fastest at about 1.3 times it (the benchmark films: 11%
    // fewer iterations; at 1.5 times on every level, where omega lambda_max
    // nears 2 and the cycle nears indefiniteness, slower than at 1), and the
    // coarse levels of the FEM hierarchy at 1.15 times that again (5% fewer
    // FEM iterations; the Poisson levels gain nothing from it), with the
    // estimate of lambda_max taken 5% high.  omega lambda_max stays at 1.65
    // (1.90 on the coarse FEM levels), below 2, so the symmetric cycle stays
    // positive definite.
    L.omega = (nc == 3 && l > 0 ? 1.15 : 1.0) * 1.3 * 4.0 / (3.0 * 1.05 * lam);
  }
  // Coarsest level: dense inverse over its unknowns, or damped Jacobi sweeps
  // when it is too large for that.
  const MgLevel& C = h.levels.back();
  const int64_t n = unknowns(C, nc, top_fixed);
  h.dense_n = 0;
  h.coarse_sweeps = 0;
  if (n <= kMgDenseMax) {
    ProbeOp op{C.nx, C.ny, C.nz, nc, top_fixed, &h.tables.back()};
    const int64_t N = op.n(), pl = op.plane();
    const int64_t nu = n / nc;  // unknowns per component: planes 1 .. active top
    std::vector<double> A((size_t)n * n, 0.0), x((size_t)nc * N, 0.0), y;
    auto idx = [&](int c, int64_t m) { return (int64_t)c * nu + (m - pl); };
    for (int e = 0; e < nc; e++)
      for (int64_t m = pl; m < pl + nu; m++) {
        std::fill(x.begin(), x.end(), 0.0);
        x[e * N + m] = 1.0;
        op.apply(x, y);
        for (int c = 0; c < nc; c++)
          for (int64_t r = pl; r < pl + nu; r++) A[(size_t)idx(c, r) * n + idx(e, m)] = y[c * N + r];
      }
    if (spd_inverse(A, (int)n)) {
      h.dense_n = (int)n;
      h.dense_inv = std::move(A);
    }
  }
  if (h.dense_n == 0) h.coarse_sweeps = 2 * std::max(C.nz, 8);
  return h;
}

// Poisson: the potential grid extended by the bottom ghost plane (plane 0,
// fixed) and, with the metal top, the top ghost plane (fixed); stored plane
// k is extended plane k + 1.
int phi_ext_planes(const pf_config& c) {
  const bool open = c.top_bc == PF_TOP_OPEN;
  const int nzp = c.nz + (open ? c.n_air : 0);
  return nzp + 1 + (open ? 0 : 1);
}

}  // namespace

std::vector<MgLevel> mg_plan(const pf_config& cfg);
std::vector<MgLevel> mg_plan_phi(const pf_config& cfg);
MgHierarchy build_mg(const pf_config& cfg, const FemTables& tb);
MgHierarchy build_mg_phi(const pf_config& cfg);

std::vector<MgLevel> mg_plan(const pf_config& cfg) { return plan_levels(cfg.nx, cfg.ny, cfg.nz, 3, false); }

std::vector<MgLevel> mg_plan_phi(const pf_config& cfg) {
  return plan_levels(cfg.nx, cfg.ny, phi_ext_planes(cfg), 1, cfg.top_bc != PF_TOP_OPEN);
}

// FEM: level 0 is the assembled stiffness (interior rows, the top row; plane
// 0 clamped).
MgHierarchy build_mg(const pf_config& cfg, const FemTables& tb) {
  std::vector<double> T0((size_t)cfg.nz * 243, 0.0);
  for (int k = 1; k < cfg.nz; k++)
    for (int c = 0; c < 3; c++)
      for (int e = 0; e < 3; e++)
        for (int o = 0; o < 27; o++)
          T0[(((size_t)k * 3 + c) * 3 + e) * 27 + o] = tb.K[k == cfg.nz - 1 ? 1 : 0][c][e][o];
  return build_generic(cfg.nx, cfg.ny, cfg.nz, 3, false, std::move(T0));
}

// Poisson: level 0 is the 7-point operator -div(eps grad) / h^2 of the
// potential grid on the extended planes, with the electrode nodes of the
// open top counted as unknowns (the preconditioner's output is zeroed there).
MgHierarchy build_mg_phi(const pf_config& cfg) {
  const bool open = cfg.top_bc == PF_TOP_OPEN;
  const int nze = phi_ext_planes(cfg);
  const int nzf = cfg.nz, nzp = nze - 1 - (open ? 0 : 1);
  const double ih2 = 1.0 / (cfg.h * cfg.h);
  const double ef = cfg.eps_b * ih2, ea = (open ? cfg.eps_air : cfg.eps_b) * ih2;
  const double ei = (open && cfg.eps_air != cfg.eps_b) ? 2 * cfg.eps_b * cfg.eps_air / (cfg.eps_b + cfg.eps_air) * ih2 : ef;
  std::vector<double> T0((size_t)nze * 27, 0.0);
  for (int k = 0; k < nzp; k++) {  // stored plane k, extended k + 1
    const double xy = k < nzf ? ef : ea;
    const double dn = k < nzf ? ef : (k == nzf ? ei : ea);
    const double up = (k + 1 >= nzp) ? (open ? 0.0 : xy) : (k + 1 < nzf ? ef : (k + 1 == nzf ? ei : ea));
    double* t = &T0[(size_t)(k + 1) * 27];
    t[tap_index(0, 0, 0)] = 4 * xy + up + dn;
    t[tap_index(1, 0, 0)] = t[tap_index(-1, 0, 0)] = t[tap_index(0, 1, 0)] = t[tap_index(0, -1, 0)] = -xy;
    t[tap_index(0, 0, 1)] = -up;
    t[tap_index(0, 0, -1)] = -dn;
  }
  return build_generic(cfg.nx, cfg.ny, nze, 1, !open, std::move(T0));
}

}  // namespace pf
