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
#include <functional>
#include <string>
#include <vector>

#include "pf_internal.h"

namespace pf {

// kernel launchers (pf_kernels.hip)
int node_blocks(const Dims& d);
TileMap make_tile_map(const Dims& d);
template <typename T> hipError_t launch_fill(T* a, int64_t n, T v, hipStream_t s);
template <typename T, typename U> hipError_t launch_convert(const T* a, U* b, int64_t n, hipStream_t s);
template <typename T> hipError_t launch_cg_finish(T* x, const T* p, int64_t n, const CgScalars* sc, hipStream_t s);
hipError_t launch_cg_reduce(const double* partials, int nblocks, int nv, CgScalars* sc, int mode, double tol,
                            int maxit, hipStream_t s);
template <typename T, typename S>
hipError_t launch_poisson_setup(const Dims& d, const Coefs<T>& cf, const S* P, const S* V, T cdt, int with_P,
                                int with_bc, const T* ghost_top, T phi_bottom, const T* x, T* r, T* p,
                                double* partials, hipStream_t s);
template <typename T>
hipError_t launch_poisson_cg_a(const Dims& d, const TileMap& tm, const Coefs<T>& cf, const T* r, const T* p_old,
                               T* p_new, T* x, const CgScalars* sc, double* partials, hipStream_t s);
template <typename T>
hipError_t launch_poisson_cg_b(const Dims& d, const TileMap& tm, const Coefs<T>& cf, const T* p, T* r,
                               const CgScalars* sc, double* partials, hipStream_t s);
template <typename T, typename S>
hipError_t launch_fem_setup(const Dims& d, const Coefs<T>& cf, const FemTables* tb, const S* P, const S* V, T cdt,
                            T* x, T* r, T* p0, T* p1, double* partials, hipStream_t s);
template <typename T>
hipError_t launch_fem_cg_a(const Dims& d, const TileMap& tm, const FemTables* tb, const T* r, const T* p_old,
                           T* p_new, T* x, const CgScalars* sc, double* partials, hipStream_t s);
template <typename T>
hipError_t launch_fem_cg_b(const Dims& d, const TileMap& tm, const FemTables* tb, const T* p, T* r,
                           const CgScalars* sc, double* partials, hipStream_t s);
template <typename T>
hipError_t launch_force(const Dims& d, const Coefs<T>& cf, const FemTables* tb, const T* P, const T* V, T cdt,
                        const T* phi, const T* ghost_top, const T* u, int mode, T* Pn, T* Vn, T* Fout,
                        hipStream_t s);

enum { kRedSetup = 0, kRedAlpha = 1, kRedBeta = 2 };

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

// cubic elastic tensor C_{ijkl} (Voigt C11, C12, C44)
double cijkl(const pf_config& c, int i, int j, int k, int l) {
  if (i == j && k == l) return i == k ? c.C11 : c.C12;
  if ((i == k && j == l) || (i == l && j == k)) return c.C44;
  return 0.0;
}

int voigt(int a, int b) {
  if (a == b) return a;
  if ((a == 0 && b == 1) || (a == 1 && b == 0)) return 3;
  if ((a == 1 && b == 2) || (a == 2 && b == 1)) return 4;
  return 5;
}

void build_tables(const pf_config& c, FemTables* t) {
  std::memset(t, 0, sizeof(*t));
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
                    const double cf = cijkl(c, cc, j, e, l);
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
  t->inv_diag[0] = 1.0 / t->K[0][0][0][13];
  t->inv_diag[1] = 1.0 / t->K[1][0][0][13];
}

// ---------------------------------------------------------------------------
// Context and workspace
// ---------------------------------------------------------------------------

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  // byte offsets into the workspace
  size_t P[2], V[2], phi, u, phi32, u32, ghost64, ghost32, ghost_unit64, phi_bc, basis;
  size_t pr, pp[2], fr, fp[2];          // Poisson / FEM CG vectors (state precision)
  size_t rr64, fr64, dphi64, du64;       // FP32_REFINE outer residuals and corrections
  size_t adj[8];                         // adjoint / energy scratch
  size_t tables, scalars, partials;
  size_t total;
};

constexpr int kNumScalars = 4;   // Poisson, FEM, two spares
constexpr int kPartialsPerBlock = 4;

Layout make_layout(const pf_config& c, int npartials) {
  const size_t N = (size_t)c.nx * c.ny * c.nz;
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
  L.phi = take(N * 8);
  L.u = take(3 * N * 8);
  L.phi32 = c.precision == PF_FP32_REFINE ? take(N * 4) : 0;
  L.u32 = c.precision == PF_FP32_REFINE ? take(3 * N * 4) : 0;
  L.ghost64 = take(plane * 8);
  L.ghost32 = take(plane * 4);
  L.ghost_unit64 = take(plane * 8);
  L.phi_bc = take(N * 8);
  L.basis = take((size_t)std::max(c.n_electrodes, 1) * N * 8);
  L.pr = take(N * es);
  for (int b = 0; b < 2; b++) L.pp[b] = take(N * es);
  L.fr = take(3 * N * es);
  for (int b = 0; b < 2; b++) L.fp[b] = take(3 * N * es);
  if (c.precision == PF_FP32_REFINE) {
    L.rr64 = take(N * 8);
    L.fr64 = take(3 * N * 8);
    L.dphi64 = take(N * 8);
    L.du64 = take(3 * N * 8);
  } else {
    L.rr64 = L.fr64 = L.dphi64 = L.du64 = 0;
  }
  for (int t = 0; t < 8; t++) L.adj[t] = take(3 * N * 8);
  L.tables = take(sizeof(FemTables));
  L.scalars = take(sizeof(CgScalars) * kNumScalars);
  L.partials = take((size_t)npartials * kPartialsPerBlock * 8 * kNumScalars);
  L.total = o;
  return L;
}

}  // namespace

}  // namespace pf

struct pf_ctx {
  pf_config cfg;
  std::vector<pf_electrode> electrodes;
  std::vector<double> volts;
  pf::Dims dims;
  pf::Layout lay;
  char* ws;
  size_t ws_bytes;
  hipStream_t stream;
  int nblocks;              // node-kernel blocks
  pf::TileMap tm;           // tile-kernel geometry
  int npartials;            // partial slots per solver (max of both block counts)
  pf::CgScalars* host_sc;   // pinned read-back buffer
  std::string err;
  bool have_state;
  bool have_basis;
  int64_t step;
  int cur;                  // which P/V buffer is current
  int last_iters_phi, last_iters_u;
  // per-kernel-class event timing
  bool timing;
  std::vector<hipEvent_t> events;
  struct TimedLaunch {
    int cls, slot, solver, k;
  };
  std::vector<TimedLaunch> pending;
  double kc_ms[PF_KC_COUNT];
  int64_t kc_n[PF_KC_COUNT];
};

namespace pf {
namespace {

template <typename T>
T* at(pf_ctx* c, size_t off) {
  return reinterpret_cast<T*>(c->ws + off);
}

pf_status fail(pf_ctx* c, pf_status s, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return s;
}

#define PF_HIP(ctx, call)                                                                 \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(ctx, PF_EHIP, "%s: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                  __LINE__);                                                              \
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
  if (c->precision != PF_FP64 && c->precision != PF_FP32_REFINE) return bad("unknown precision");
  if (!(c->tol_phi > 0) || !(c->tol_u > 0)) return bad("tolerances must be > 0");
  if (c->maxit <= 0) return bad("maxit must be > 0");
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

CgScalars* dev_sc(pf_ctx* c, int which) { return at<CgScalars>(c, c->lay.scalars) + which; }
double* dev_partials(pf_ctx* c, int which) {
  return at<double>(c, c->lay.partials) + (size_t)which * c->npartials * kPartialsPerBlock;
}

// Event timing of one launch: `launch` is called between two event records
// when timing is on.  solver/k tag CG iterations (solver -1: always counted).
template <typename F>
hipError_t timed(pf_ctx* c, int cls, int solver, int k, F&& launch) {
  if (!c->timing) return launch();
  const int slot = (int)c->pending.size();
  while ((int)c->events.size() < 2 * (slot + 1)) {
    hipEvent_t e;
    hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) return err;
    c->events.push_back(e);
  }
  hipError_t err = hipEventRecord(c->events[2 * slot], c->stream);
  if (err != hipSuccess) return err;
  err = launch();
  if (err != hipSuccess) return err;
  err = hipEventRecord(c->events[2 * slot + 1], c->stream);
  if (err != hipSuccess) return err;
  c->pending.push_back({cls, slot, solver, k});
  return hipSuccess;
}

// After a stream synchronisation: accumulates the pending launches.  CG
// iterations at or beyond `iters` of `solver` returned at entry and are
// dropped.
void collect_timing(pf_ctx* c, int solver, int iters) {
  for (const auto& t : c->pending) {
    if (t.solver >= 0 && t.solver == solver && t.k >= iters) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->events[2 * t.slot], c->events[2 * t.slot + 1]) == hipSuccess) {
      c->kc_ms[t.cls] += ms;
      c->kc_n[t.cls] += 1;
    }
  }
  c->pending.clear();
}

// Reads back the scalars of one solver (synchronises the stream).
pf_status read_scalars(pf_ctx* c, int which, CgScalars* out) {
  PF_HIP(c, hipMemcpyAsync(c->host_sc, dev_sc(c, which), sizeof(CgScalars), hipMemcpyDeviceToHost, c->stream));
  PF_HIP(c, hipStreamSynchronize(c->stream));
  *out = *c->host_sc;
  if (c->timing) collect_timing(c, which, out->iter);
  return PF_OK;
}

pf_status sync(pf_ctx* c) {
  PF_HIP(c, hipStreamSynchronize(c->stream));
  if (c->timing) collect_timing(c, -1, 0);
  return PF_OK;
}

// ---------------------------------------------------------------------------
// Conjugate-gradient drivers
// ---------------------------------------------------------------------------
// The setup kernel forms r = b - A x and the first direction; each iteration
// is two fused kernels (direction update + operator + p.q; residual update
// + r.z + convergence).  Step lengths live on the device; the host enqueues
// iterations in batches and reads the scalars once per batch, kernels
// enqueued after convergence return at entry.  A last kernel applies the
// deferred update of x.

struct SolveResult {
  int iters;
  double relres;
  int done;
};

pf_status finish_solve(pf_ctx* c, int which, const CgScalars& h, SolveResult* res, const char* what) {
  res->iters = h.iter;
  res->done = h.done;
  res->relres = h.zero_rhs ? 0.0 : std::sqrt(h.rnorm2 / h.bnorm2);
  if (h.done == kNonFinite) return fail(c, PF_ENONFINITE, "%s: non-finite value in the CG reductions", what);
  if (h.done == kMaxIt)
    return fail(c, PF_ENOCONV, "%s: no convergence in %d iterations (relres %.3e)", what, h.iter, res->relres);
  (void)which;
  return PF_OK;
}

template <typename T>
pf_status run_cg(pf_ctx* c, int which, int predicted, T* x, T* const pbuf[2], int64_t n,
                 const std::function<hipError_t(int)>& iteration, SolveResult* res, const char* what) {
  CgScalars h;
  int k = 0;
  int batch = std::max(2, predicted);
  const int maxit = c->cfg.maxit;
  for (;;) {
    const int nb = std::min(batch, maxit - k);
    for (int t = 0; t < nb; t++, k++) PF_HIP(c, iteration(k));
    pf_status st = read_scalars(c, which, &h);
    if (st != PF_OK) return st;
    if (h.done != kRunning) break;
    if (k >= maxit) return fail(c, PF_EHIP, "%s: solver state did not advance", what);
    batch = std::max(4, predicted / 8);
  }
  if (h.done != kNonFinite)
    PF_HIP(c, timed(c, PF_KC_FINISH, -1, -1,
                    [&] { return launch_cg_finish<T>(x, pbuf[h.iter & 1], n, dev_sc(c, which), c->stream); }));
  return finish_solve(c, which, h, res, what);
}

// Poisson solve for Pp = P + cdt V (V may be null); boundary values from
// ghost (top) and phi_bottom when with_bc.
template <typename T>
pf_status solve_poisson(pf_ctx* c, const T* P, const T* V, T cdt, int with_P, int with_bc, const T* ghost,
                        T phi_bottom, T* x, double tol, bool warm, SolveResult* res) {
  const Dims& d = c->dims;
  const Coefs<T> cf = make_coefs<T>(c);
  CgScalars* sc = dev_sc(c, 0);
  double* part = dev_partials(c, 0);
  T* r = at<T>(c, c->lay.pr);
  T* pb[2] = {at<T>(c, c->lay.pp[0]), at<T>(c, c->lay.pp[1])};
  if (!warm) PF_HIP(c, launch_fill<T>(x, d.N, (T)0, c->stream));
  const TileMap& tm = c->tm;
  const int nb = c->nblocks, tb_ = tm.nblocks, maxit = c->cfg.maxit;
  PF_HIP(c, timed(c, PF_KC_POISSON_SETUP, -1, -1, [&] {
    return launch_poisson_setup<T, T>(d, cf, P, V, cdt, with_P, with_bc, ghost, phi_bottom, x, r, pb[0], part,
                                      c->stream);
  }));
  PF_HIP(c, timed(c, PF_KC_REDUCE, -1, -1,
                  [&] { return launch_cg_reduce(part, nb, 3, sc, kRedSetup, tol, maxit, c->stream); }));
  auto iteration = [&](int k) -> hipError_t {
    hipError_t e = timed(c, PF_KC_POISSON_A, 0, k, [&] {
      return launch_poisson_cg_a<T>(d, tm, cf, r, pb[k & 1], pb[(k + 1) & 1], x, sc, part, c->stream);
    });
    if (e == hipSuccess)
      e = timed(c, PF_KC_REDUCE, 0, k,
                [&] { return launch_cg_reduce(part, tb_, 1, sc, kRedAlpha, tol, maxit, c->stream); });
    if (e == hipSuccess)
      e = timed(c, PF_KC_POISSON_B, 0, k,
                [&] { return launch_poisson_cg_b<T>(d, tm, cf, pb[(k + 1) & 1], r, sc, part, c->stream); });
    if (e == hipSuccess)
      e = timed(c, PF_KC_REDUCE, 0, k,
                [&] { return launch_cg_reduce(part, tb_, 2, sc, kRedBeta, tol, maxit, c->stream); });
    return e;
  };
  return run_cg<T>(c, 0, c->last_iters_phi, x, pb, d.N, iteration, res, "Poisson solve");
}

template <typename T>
pf_status solve_fem(pf_ctx* c, const T* P, const T* V, T cdt, T* x, double tol, bool warm, SolveResult* res) {
  const Dims& d = c->dims;
  const Coefs<T> cf = make_coefs<T>(c);
  const FemTables* tb = at<FemTables>(c, c->lay.tables);
  CgScalars* sc = dev_sc(c, 1);
  double* part = dev_partials(c, 1);
  T* r = at<T>(c, c->lay.fr);
  T* pb[2] = {at<T>(c, c->lay.fp[0]), at<T>(c, c->lay.fp[1])};
  if (!warm) PF_HIP(c, launch_fill<T>(x, 3 * d.N, (T)0, c->stream));
  const TileMap& tm = c->tm;
  const int nb = c->nblocks, tb_ = tm.nblocks, maxit = c->cfg.maxit;
  PF_HIP(c, timed(c, PF_KC_FEM_SETUP, -1, -1, [&] {
    return launch_fem_setup<T, T>(d, cf, tb, P, V, cdt, x, r, pb[0], pb[1], part, c->stream);
  }));
  PF_HIP(c, timed(c, PF_KC_REDUCE, -1, -1,
                  [&] { return launch_cg_reduce(part, nb, 3, sc, kRedSetup, tol, maxit, c->stream); }));
  auto iteration = [&](int k) -> hipError_t {
    hipError_t e = timed(c, PF_KC_FEM_A, 1, k, [&] {
      return launch_fem_cg_a<T>(d, tm, tb, r, pb[k & 1], pb[(k + 1) & 1], x, sc, part, c->stream);
    });
    if (e == hipSuccess)
      e = timed(c, PF_KC_REDUCE, 1, k,
                [&] { return launch_cg_reduce(part, tb_, 1, sc, kRedAlpha, tol, maxit, c->stream); });
    if (e == hipSuccess)
      e = timed(c, PF_KC_FEM_B, 1, k,
                [&] { return launch_fem_cg_b<T>(d, tm, tb, pb[(k + 1) & 1], r, sc, part, c->stream); });
    if (e == hipSuccess)
      e = timed(c, PF_KC_REDUCE, 1, k,
                [&] { return launch_cg_reduce(part, tb_, 2, sc, kRedBeta, tol, maxit, c->stream); });
    return e;
  };
  return run_cg<T>(c, 1, c->last_iters_u, x, pb, 3 * d.N, iteration, res, "FEM solve");
}

pf_status worst(pf_status a, pf_status b) {
  if (a == PF_OK) return b;
  if (b == PF_OK) return a;
  if (a == PF_ENOCONV) return b;
  return a;
}

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

// Solves phi and u at Pp = P + cdt V into the state's phi and u.
pf_status solve_nonlocal64(pf_ctx* c, const double* P, const double* V, double cdt, bool warm, pf_step_stats* st) {
  pf_status out = PF_OK;
  if (c->cfg.terms & PF_TERM_ELEC) {
    SolveResult r{};
    pf_status s = solve_poisson<double>(c, P, V, cdt, 1, 1, at<double>(c, c->lay.ghost64), c->cfg.phi_bottom,
                                        at<double>(c, c->lay.phi), c->cfg.tol_phi, warm, &r);
    if (s != PF_OK && s != PF_ENOCONV) return s;
    c->last_iters_phi = r.iters;
    stats_add(st, 0, r);
    out = worst(out, s);
  }
  if (c->cfg.terms & PF_TERM_ELAS) {
    SolveResult r{};
    pf_status s = solve_fem<double>(c, P, V, cdt, at<double>(c, c->lay.u), c->cfg.tol_u, warm, &r);
    if (s != PF_OK && s != PF_ENOCONV) return s;
    c->last_iters_u = r.iters;
    stats_add(st, 1, r);
    out = worst(out, s);
  }
  return out;
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
  Dims d{cfg->nx, cfg->ny, cfg->nz, (int64_t)cfg->nx * cfg->ny * cfg->nz, (int64_t)cfg->nx * cfg->ny};
  *bytes = make_layout(*cfg, std::max(node_blocks(d), make_tile_map(d).nblocks)).total;
  return PF_OK;
}

pf_status pf_init(const pf_config* cfg, void* ws, size_t bytes, void* stream, pf_ctx** out) {
  if (!out) return PF_EINVAL;
  *out = nullptr;
  std::string why;
  if (validate(cfg, &why) != PF_OK) {
    fprintf(stderr, "pf_init: %s\n", why.c_str());
    return PF_EINVAL;
  }
  if (cfg->precision != PF_FP64) {
    fprintf(stderr, "pf_init: this build supports PF_FP64 only\n");
    return PF_EINVAL;
  }
  if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) {
    fprintf(stderr, "pf_init: workspace must be non-null and 256-byte aligned\n");
    return PF_EINVAL;
  }
  pf_ctx* c = new pf_ctx();
  c->cfg = *cfg;
  c->electrodes.assign(cfg->electrodes, cfg->electrodes + cfg->n_electrodes);
  c->cfg.electrodes = c->electrodes.data();
  for (auto& e : c->electrodes) c->volts.push_back(e.volts);
  c->dims = Dims{cfg->nx, cfg->ny, cfg->nz, (int64_t)cfg->nx * cfg->ny * cfg->nz, (int64_t)cfg->nx * cfg->ny};
  c->nblocks = node_blocks(c->dims);
  c->tm = make_tile_map(c->dims);
  c->npartials = std::max(c->nblocks, c->tm.nblocks);
  c->lay = make_layout(*cfg, c->npartials);
  if (bytes < c->lay.total) {
    fprintf(stderr, "pf_init: workspace of %zu bytes, %zu needed\n", bytes, c->lay.total);
    delete c;
    return PF_ENOMEM;
  }
  c->ws = static_cast<char*>(ws);
  c->ws_bytes = bytes;
  c->stream = static_cast<hipStream_t>(stream);
  c->have_state = false;
  c->have_basis = false;
  c->step = 0;
  c->cur = 0;
  c->last_iters_phi = c->last_iters_u = 16;
  c->timing = false;
  std::memset(c->kc_ms, 0, sizeof(c->kc_ms));
  std::memset(c->kc_n, 0, sizeof(c->kc_n));
  if (hipHostMalloc(reinterpret_cast<void**>(&c->host_sc), sizeof(CgScalars), hipHostMallocDefault) != hipSuccess) {
    fprintf(stderr, "pf_init: pinned host allocation failed\n");
    delete c;
    return PF_EHIP;
  }
  // tables and ghost planes (host-built, copied once)
  FemTables tb;
  build_tables(c->cfg, &tb);
  std::vector<double> g64((size_t)cfg->nx * cfg->ny, cfg->phi_top);
  for (auto& e : c->electrodes)
    for (int j = e.y0; j < e.y1; j++)
      for (int i = e.x0; i < e.x1; i++) g64[(size_t)i + (size_t)cfg->nx * j] = e.volts;
  std::vector<float> g32(g64.begin(), g64.end());
  pf_status st = PF_OK;
  auto cp = [&](size_t off, const void* src, size_t n) {
    if (st != PF_OK) return;
    hipError_t e = hipMemcpyAsync(c->ws + off, src, n, hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) st = fail(c, PF_EHIP, "table upload: %s", hipGetErrorString(e));
  };
  cp(c->lay.tables, &tb, sizeof(tb));
  cp(c->lay.ghost64, g64.data(), g64.size() * 8);
  cp(c->lay.ghost32, g32.data(), g32.size() * 4);
  if (st == PF_OK) {
    static_assert(sizeof(CgScalars) % 8 == 0, "scalars are cleared as doubles");
    hipError_t e = launch_fill<double>(reinterpret_cast<double*>(c->ws + c->lay.scalars),
                                       (int64_t)(sizeof(CgScalars) * kNumScalars / 8), 0.0, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) st = fail(c, PF_EHIP, "init: %s", hipGetErrorString(e));
  }
  if (st != PF_OK) {
    fprintf(stderr, "pf_init: %s\n", c->err.c_str());
    (void)hipHostFree(c->host_sc);
    delete c;
    return st;
  }
  *out = c;
  return PF_OK;
}

void pf_destroy(pf_ctx* c) {
  if (!c) return;
  for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
  if (c->host_sc) (void)hipHostFree(c->host_sc);
  delete c;
}

pf_status pf_set_state(pf_ctx* c, const void* P, const void* phi0, const void* u0) {
  if (!c || !P) return fail(c, PF_EINVAL, "pf_set_state: null argument");
  const int64_t N = c->dims.N;
  c->cur = 0;
  c->step = 0;
  double* Pc = at<double>(c, c->lay.P[0]);
  double* Vc = at<double>(c, c->lay.V[0]);
  double* phi = at<double>(c, c->lay.phi);
  double* u = at<double>(c, c->lay.u);
  PF_HIP(c, hipMemcpyAsync(Pc, P, 3 * N * 8, hipMemcpyDeviceToDevice, c->stream));
  if (phi0) PF_HIP(c, hipMemcpyAsync(phi, phi0, N * 8, hipMemcpyDeviceToDevice, c->stream));
  else PF_HIP(c, launch_fill<double>(phi, N, 0.0, c->stream));
  if (u0) PF_HIP(c, hipMemcpyAsync(u, u0, 3 * N * 8, hipMemcpyDeviceToDevice, c->stream));
  else PF_HIP(c, launch_fill<double>(u, 3 * N, 0.0, c->stream));
  PF_HIP(c, launch_fill<double>(Vc, 3 * N, 0.0, c->stream));
  pf_status s = PF_OK;
  if (c->cfg.integrator == PF_INT_PC) {
    s = solve_nonlocal64(c, Pc, nullptr, 0.0, true, nullptr);
    if (s != PF_OK && s != PF_ENOCONV) return s;
    const Coefs<double> cf = make_coefs<double>(c);
    PF_HIP(c, launch_force<double>(c->dims, cf, at<FemTables>(c, c->lay.tables), Pc, nullptr, 0.0, phi,
                                   at<double>(c, c->lay.ghost64), u, kPcInit, nullptr, Vc, nullptr, c->stream));
  }
  PF_HIP(c, hipStreamSynchronize(c->stream));
  c->have_state = true;
  return s;
}

pf_status pf_restore_state(pf_ctx* c, const void* P, const void* V, const void* phi, const void* u, int64_t step) {
  if (!c || !P || !V || !phi || !u) return fail(c, PF_EINVAL, "pf_restore_state: null argument");
  const int64_t N = c->dims.N;
  c->cur = 0;
  PF_HIP(c, hipMemcpyAsync(at<double>(c, c->lay.P[0]), P, 3 * N * 8, hipMemcpyDeviceToDevice, c->stream));
  PF_HIP(c, hipMemcpyAsync(at<double>(c, c->lay.V[0]), V, 3 * N * 8, hipMemcpyDeviceToDevice, c->stream));
  PF_HIP(c, hipMemcpyAsync(at<double>(c, c->lay.phi), phi, N * 8, hipMemcpyDeviceToDevice, c->stream));
  PF_HIP(c, hipMemcpyAsync(at<double>(c, c->lay.u), u, 3 * N * 8, hipMemcpyDeviceToDevice, c->stream));
  c->step = step;
  c->have_state = true;
  return PF_OK;
}

pf_status pf_get_state(const pf_ctx* cc, void* P, void* V, void* phi, void* u, int64_t* step) {
  pf_ctx* c = const_cast<pf_ctx*>(cc);
  if (!c) return PF_EINVAL;
  if (!c->have_state) return fail(c, PF_ESTATE, "pf_get_state: no state (call pf_set_state first)");
  const int64_t N = c->dims.N;
  if (P) PF_HIP(c, hipMemcpyAsync(P, at<double>(c, c->lay.P[c->cur]), 3 * N * 8, hipMemcpyDeviceToDevice, c->stream));
  if (V) PF_HIP(c, hipMemcpyAsync(V, at<double>(c, c->lay.V[c->cur]), 3 * N * 8, hipMemcpyDeviceToDevice, c->stream));
  if (phi) PF_HIP(c, hipMemcpyAsync(phi, at<double>(c, c->lay.phi), N * 8, hipMemcpyDeviceToDevice, c->stream));
  if (u) PF_HIP(c, hipMemcpyAsync(u, at<double>(c, c->lay.u), 3 * N * 8, hipMemcpyDeviceToDevice, c->stream));
  if (step) *step = c->step;
  return PF_OK;
}

pf_status pf_step(pf_ctx* c, int32_t nsteps, pf_step_stats* st) {
  if (!c) return PF_EINVAL;
  if (nsteps < 0) return fail(c, PF_EINVAL, "pf_step: nsteps < 0");
  if (!c->have_state) return fail(c, PF_ESTATE, "pf_step: no state (call pf_set_state first)");
  if (st) std::memset(st, 0, sizeof(*st));
  const Coefs<double> cf = make_coefs<double>(c);
  const FemTables* tb = at<FemTables>(c, c->lay.tables);
  const bool pc = c->cfg.integrator == PF_INT_PC;
  const int every = c->cfg.nonlocal_every <= 1 ? 1 : c->cfg.nonlocal_every;
  pf_status out = PF_OK;
  for (int s = 0; s < nsteps; s++) {
    double* P = at<double>(c, c->lay.P[c->cur]);
    double* V = at<double>(c, c->lay.V[c->cur]);
    double* Pn = at<double>(c, c->lay.P[c->cur ^ 1]);
    double* Vn = at<double>(c, c->lay.V[c->cur ^ 1]);
    if (c->step % every == 0) {
      pf_status r = solve_nonlocal64(c, P, pc ? V : nullptr, pc ? c->cfg.dt : 0.0, c->cfg.warm_start != 0, st);
      if (r != PF_OK && r != PF_ENOCONV) return r;
      out = worst(out, r);
    }
    PF_HIP(c, timed(c, PF_KC_FORCE, -1, -1, [&] {
      return launch_force<double>(c->dims, cf, tb, P, pc ? V : nullptr, pc ? c->cfg.dt : 0.0,
                                  at<double>(c, c->lay.phi), at<double>(c, c->lay.ghost64), at<double>(c, c->lay.u),
                                  pc ? kPcStep : kEulerStep, Pn, Vn, nullptr, c->stream);
    }));
    c->cur ^= 1;
    c->step++;
    if (st) st->steps++;
  }
  pf_status ss = sync(c);
  if (ss != PF_OK) return ss;
  return out;
}

pf_status pf_solve_phi(pf_ctx* c, const void* P, void* phi, pf_solve_stats* st) {
  if (!c || !P || !phi) return fail(c, PF_EINVAL, "pf_solve_phi: null argument");
  SolveResult r{};
  pf_status s = solve_poisson<double>(c, static_cast<const double*>(P), nullptr, 0.0, 1, 1,
                                      at<double>(c, c->lay.ghost64), c->cfg.phi_bottom, static_cast<double*>(phi),
                                      c->cfg.tol_phi, c->cfg.warm_start != 0, &r);
  if (st) {
    st->iters = r.iters;
    st->outer = 1;
    st->relres = r.relres;
  }
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail(c, PF_EHIP, "pf_solve_phi: %s", hipGetErrorString(e));
  return s;
}

pf_status pf_solve_u(pf_ctx* c, const void* P, void* u, pf_solve_stats* st) {
  if (!c || !P || !u) return fail(c, PF_EINVAL, "pf_solve_u: null argument");
  SolveResult r{};
  pf_status s = solve_fem<double>(c, static_cast<const double*>(P), nullptr, 0.0, static_cast<double*>(u),
                                  c->cfg.tol_u, c->cfg.warm_start != 0, &r);
  if (st) {
    st->iters = r.iters;
    st->outer = 1;
    st->relres = r.relres;
  }
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail(c, PF_EHIP, "pf_solve_u: %s", hipGetErrorString(e));
  return s;
}

pf_status pf_force(pf_ctx* c, const void* P, const void* phi, const void* u, void* F) {
  if (!c || !P || !F) return fail(c, PF_EINVAL, "pf_force: null argument");
  if ((c->cfg.terms & PF_TERM_ELEC) && !phi) return fail(c, PF_EINVAL, "pf_force: phi needed");
  if ((c->cfg.terms & PF_TERM_ELAS) && !u) return fail(c, PF_EINVAL, "pf_force: u needed");
  const Coefs<double> cf = make_coefs<double>(c);
  PF_HIP(c, launch_force<double>(c->dims, cf, at<FemTables>(c, c->lay.tables), static_cast<const double*>(P),
                                 nullptr, 0.0, static_cast<const double*>(phi), at<double>(c, c->lay.ghost64),
                                 static_cast<const double*>(u), kForceOut, nullptr, nullptr,
                                 static_cast<double*>(F), c->stream));
  return PF_OK;
}

pf_status pf_timing(pf_ctx* c, int enable, double* ms, int64_t* launches) {
  if (!c) return PF_EINVAL;
  pf_status s = sync(c);
  if (s != PF_OK) return s;
  for (int t = 0; t < PF_KC_COUNT; t++) {
    if (ms) ms[t] = c->kc_ms[t];
    if (launches) launches[t] = c->kc_n[t];
    c->kc_ms[t] = 0;
    c->kc_n[t] = 0;
  }
  c->timing = enable != 0;
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

pf_status pf_energy(pf_ctx* c, double out[5]) {
  (void)out;
  return fail(c, PF_EINVAL, "pf_energy: not available in this build");
}

pf_status pf_set_params(pf_ctx* c, const double* volts, double a1) {
  if (!c) return PF_EINVAL;
  (void)volts;
  (void)a1;
  return fail(c, PF_EINVAL, "pf_set_params: not available in this build");
}

pf_status pf_adjoint_step(pf_ctx* c, const void*, const void*, void*, void*, double*) {
  return fail(c, PF_EINVAL, "pf_adjoint_step: not available in this build");
}

pf_status pf_adjoint_initial_rate(pf_ctx* c, const void*, void*, void*, double*) {
  return fail(c, PF_EINVAL, "pf_adjoint_initial_rate: not available in this build");
}

}  // extern "C"
