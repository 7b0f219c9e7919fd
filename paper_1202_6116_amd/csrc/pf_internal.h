// Internal declarations shared by the host layer (pf_api.cpp) and the HIP
// kernels (pf_kernels.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace pf {

// Threads per block of the node kernels: 64 along x (one wavefront per
// x-row segment, coalesced), 4 rows along y.  Grid: (ceil(nx/64),
// ceil(ny/4), nz), one thread per node.
constexpr int kBX = 64;
constexpr int kBY = 4;
constexpr int kThreads = kBX * kBY;

// Offsets of a 27-point stencil are numbered o = (dx+1) + 3 (dy+1) + 9 (dz+1).
constexpr int kTaps = 27;

// Row types along z.  The clamped plane k = 0 has only the element above it
// (kLow), planes 1..nz-2 are interior, the free top plane k = nz-1 has only
// the element below it (kHigh).
enum ZType { kLow = 0, kInterior = 1, kHigh = 2 };

// Constant operator tables of the trilinear-hex FEM on the uniform grid,
// built on the host from 1D element integrals.  Stored in the workspace and
// read by the kernels with uniform (scalar) loads.
struct FemTables {
  // Stiffness stencil K^{cd}(o): rows of interior planes [0], top plane [1].
  double K[2][3][3][kTaps];
  // Body force of a nodal stress field sigma0 = C eps0 (Voigt v):
  // f_c = sum_v Bf[.][c][v](o) sigma0_v; interior [0], top [1].
  double Bf[2][3][6][kTaps];
  // Weighted strain of a displacement field: (int N_n eps_v(u)) =
  // sum_c Su[z][v][c](o) u_c, z in {kLow, kInterior, kHigh}.
  double Su[3][6][3][kTaps];
  // Consistent mass M x M x M, z in {kLow, kInterior, kHigh}.
  double Ms[3][kTaps];
  // Inverse Jacobi diagonal of K for interior and top rows, per component.
  double inv_diag[2][3];
  // The 1D element integrals the 3D stencils above are products of (row
  // kind z in {kLow, kInterior, kHigh}, tap dz + 1): mass int N_n N_m,
  // int N_n N_m' (g) and int N_n' N_m (gt).  The x and y axes use kInterior.
  double m1[3][3], g1[3][3], gt1[3][3];
  // With a stiffness cubic on the grid axes, K takes few distinct values:
  // K[zt][c][e](o) = sign * kc[class] (kc_class below); compact = 1 when
  // every coefficient of K was checked to have that form.
  double kc_int[8], kc_top[24];
  int32_t compact;
};

__host__ __device__ __forceinline__ int kc_abs(int v) { return v < 0 ? -v : v; }
__host__ __device__ __forceinline__ int kc_sgn(int v) { return v < 0 ? -1 : 1; }

// Class of the stiffness coefficient K[zt][c][e] at offset off for a
// stiffness cubic on the grid axes (-1: structurally zero), and its sign.
// Interior rows (zt 0) depend on which offsets are non-zero (the element
// integrals are even in the offset, their derivative rows odd); top rows
// (zt 1) also on whether the neighbour is in the plane below.
__host__ __device__ __forceinline__ int kc_class(int zt, int c, int e, const int off[3], int* sign) {
  *sign = 1;
  if (zt == 0) {
    if (c == e) return kc_abs(off[c]) * 3 + kc_abs(off[(c + 1) % 3]) + kc_abs(off[(c + 2) % 3]);
    if (off[c] == 0 || off[e] == 0) return -1;
    *sign = kc_sgn(off[c]) * kc_sgn(off[e]);
    return 6 + kc_abs(off[3 - c - e]);
  }
  if (off[2] > 0) return -1;  // no element above the top plane
  const int zi = off[2] == 0 ? 1 : 0;
  if (c < 2 && e < 2) {
    if (c == e) return kc_abs(off[c]) * 4 + kc_abs(off[1 - c]) * 2 + zi;
    if (off[c] == 0 || off[e] == 0) return -1;
    *sign = kc_sgn(off[c]) * kc_sgn(off[e]);
    return 14 + zi;
  }
  if (c == 2 && e == 2) return 8 + zi * 3 + kc_abs(off[0]) + kc_abs(off[1]);
  if (e == 2) {  // in-plane row, z column
    if (off[c] == 0) return -1;
    *sign = kc_sgn(off[c]);
    return 16 + kc_abs(off[1 - c]) * 2 + zi;
  }
  if (off[e] == 0) return -1;  // z row, in-plane column
  *sign = kc_sgn(off[e]);
  return 20 + kc_abs(off[1 - e]) * 2 + zi;
}

// Scalars of one conjugate-gradient solve, resident in device memory.  The
// last block of each reduction kernel updates them; every kernel of a solve
// reads them at entry and returns at once when `done` is set.
struct CgScalars {
  double rho;            // r.z of the current residual
  double alpha;          // step length, applied to x lazily by the next kernel
  double beta;           // conjugation factor for the next direction
  double bnorm2;         // ||b||^2
  double rnorm2;         // ||r||^2 of the current residual
  double tol;            // relative tolerance
  int32_t iter;          // iterations completed
  int32_t maxit;
  int32_t done;          // 0 running, 1 converged, 2 iteration cap, 3 non-finite
  int32_t zero_rhs;      // b == 0: the solution is x = 0
  int32_t outer_done;    // refinement: the FP64 residual met the tolerance
  double outer_b2;       // refinement: ||b||^2 of the FP64 system
  double outer_r2;       // refinement: ||b - A x||^2 of the FP64 iterate
  double pad;
};

enum CgDone { kRunning = 0, kConverged = 1, kMaxIt = 2, kNonFinite = 3 };

// Tiles of the z-marching kernels: ntx x nty columns of 64 x ty nodes, each
// cut into nkz chunks of kz planes; one block per (column, chunk).
struct TileMap {
  int ty, ntx, nty, kz, nkz, nblocks;
  int gy;  // tile rows per group of the block order (see tile_coord)
};

// Polynomial extrapolation of a solution to the next step from the current
// value and up to kMaxExtrap earlier ones (newest first), with the
// coefficients of the interpolating polynomial evaluated one step ahead;
// the current value then replaces the oldest (or the next free) ring slot.
constexpr int kMaxExtrap = 8;
struct ExtrapRing {
  const double* h[kMaxExtrap + 1];  // earlier solutions, newest first (m used, nh valid)
  double* dest;                     // ring slot that receives the current value
  double c[kMaxExtrap + 1];         // c[0] for the current value, c[t] for h[t-1]
  int m;
  int nh;                           // earlier solutions held (warm_start 3 scores orders < nh)
};

// warm_start 3: sampled one-step prediction errors of the extrapolation
// orders 0..mmax (every kScoreStride-th chunk of 256 values of a field),
// per block of extrap_score_kernel; c[m][t] are the weights of order m.
constexpr int kScoreBlocks = 1024;
constexpr int kScoreStride = 64;
struct ExtrapScore {
  double c[kMaxExtrap + 1][kMaxExtrap + 1];
  double* partials;  // kScoreBlocks x (kMaxExtrap + 1)
  int mmax;
};

// Material on the grid axes (host): rotation R (crystal to grid), the Voigt
// stiffness C (engineering strain) and the electrostriction quadratic forms,
// eps0_v = sum_q Qv[v][q] m_q with m = (x^2, y^2, z^2, 2xy, 2yz, 2zx).
struct Material {
  double R[9];
  double C[6][6];
  double Qv[6][6];
  bool rotated;  // R is not the identity
  bool cubic;    // C has the cubic zero pattern on the grid axes
};

// Modes of the single-block reduce kernel.
enum { kRedSetup = 0, kRedAlpha = 1, kRedBeta = 2, kRedOuter = 3, kRedSum = 4, kRedRho = 5, kRedCheck = 6, kRedConj = 7 };

// Multigrid hierarchy of the FEM operator (built on the host, pf_mg.cpp).
// Level kernels: out = b - A x (kMgResidual), one damped Jacobi sweep
// out = x + omega D^-1 (b - A x) (kMgSweep), or (solver-grid kernels only)
// the residual of the first sweep from zero, out = b - A (omega D^-1 b), with
// x not read (kMgFirst), or the sweep of kMgSweep from x = omega D^-1 b + P e,
// x formed on the fly from b and the correction e of the next level, when
// that level halves x and y (kMgCorrect: the prolongation is never stored).
enum { kMgResidual = 0, kMgSweep = 1, kMgFirst = 2, kMgCorrect = 3 };
// Size of the static device workspace of pf_init_static (per GPU).
constexpr size_t kStaticWorkspaceBytes = size_t(64) << 20;
hipError_t static_workspace_acquire(int device, void** ptr);
void static_workspace_release(int device);

constexpr int kMgMaxLevels = 12;
constexpr int64_t kMgDenseMax = 512;  // coarsest level solved by a dense inverse up to this many unknowns

// Linear interpolation in z from the coarse planes lo, hi (clamp plane 0
// carries zero) to one fine plane.
struct MgZ {
  int lo, hi;
  double wlo, whi;
};

// The correction e of the next coarser level, read by the kMgCorrect
// solver-grid kernels: NC components of N values each; zmap gives the coarse
// z parents of the fine plane with extended index k + zoff (k the stored
// plane); the plane 0 and, with top_fixed, the top plane carry zero.
template <typename T>
struct MgCoarse {
  const T* e;
  const MgZ* zmap;
  int64_t N, plane;
  int nx, ny, nz;
  int zoff, top_fixed;
};

struct MgLevel {
  int nx, ny, nz;            // nodes per direction (plane 0 is the clamp)
  bool cx, cy;               // halved in x / y from the finer level
  double omega;              // damping of the Jacobi smoother
  std::vector<double> dinv;  // inverse diagonal per plane and component (nz x 3)
};

struct MgHierarchy {
  int nc;                                     // components: 3 (FEM) or 1 (Poisson)
  bool top_fixed;                             // the top plane of every level is fixed (metal top)
  std::vector<MgLevel> levels;                // 0 = the solver's grid
  std::vector<std::vector<double>> tables;    // nz x nc x nc x 27 stencils (level 0: the operator itself)
  std::vector<std::vector<double>> tables_w;  // level >= 1 (from index 0 up): stencils times omega D^-1
  std::vector<std::vector<MgZ>> zmaps;        // level >= 1: per plane of the finer level
  std::vector<std::vector<int>> zfine;        // level >= 1: finer-level plane of each plane
  int dense_n;                                // coarsest: unknowns of the dense inverse (0: none)
  std::vector<double> dense_inv;              // dense_n x dense_n
  int coarse_sweeps;                          // coarsest: Jacobi sweeps when there is no inverse
};

// Per-call description of a node grid: the film grid (nz = nzf) or the
// potential grid (nz = nzp: the film plus, with the open top, the air planes
// above it).  nzf, Nf and nzp are the same in both.
struct Dims {
  int nx, ny, nz;
  int64_t N;        // nodes
  int64_t plane;    // nx * ny
  int nzf;          // film planes
  int64_t Nf;       // film nodes
  int nzp;          // planes of the potential grid
};

// Material and model coefficients used inside kernels.
template <typename T>
struct Coefs {
  T a1, a11, a12;       // Landau
  T G, L, dt;           // gradient, mobility, time step
  T h, inv_h2, inv_2h, inv_h3;
  T eps_over_h2;        // eps_b / h^2
  T inv_diag_poisson;   // h^2 / (6 eps_b)
  T eps_air_over_h2;    // open top: eps_air / h^2
  T eps_iface_over_h2;  // open top: harmonic mean of eps_b and eps_air / h^2
  int open;             // open top: air planes, zero normal field on top
  // Rotated crystal frame (rotated != 0): R maps crystal axes to grid axes;
  // Cg is the grid-frame Voigt stiffness and eps0_v = sum Qv[v][.] of the
  // products (xx, yy, zz, 2xy, 2yz, 2zx) of the grid components of P.
  int rotated;
  T R[9];
  T Cg[36];
  T Qv[6][6];
  T es[6];              // substrate strain (Voigt, engineering shear), subtracted from eps0
  T C11, C12, C44, Q11, Q12, Q44;
  T phi_bottom;
  uint32_t terms;
};

enum Terms { kLandau = 1, kGrad = 2, kElec = 4, kElas = 8 };

// Thermal noise of one step: the force gains amp * xi, xi the standard
// normal variates keyed by (seed, step, node).  amp = 0: no noise.
struct NoiseSpec {
  double amp;
  uint32_t key0, key1;      // seed words
  uint32_t step0, step1;    // step words
};

// What the force kernel does with the force F at the evaluation point.
enum ForceMode {
  kForceOut = 0,     // F written to an output array
  kPcInit = 1,       // V = F
  kPcStep = 2,       // V' = (V + F)/2, P' = P + dt V'
  kEulerStep = 3,    // P' = P + dt F
};

}  // namespace pf
