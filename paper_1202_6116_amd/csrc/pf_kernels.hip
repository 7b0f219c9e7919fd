// HIP kernels of the TDGL step on gfx950.
//
// Numbering: node n = i + nx (j + ny k), fields are structure-of-arrays
// (component c of node n at c*N + n), periodic in x and y, k = 0 the clamped
// substrate side, k = nz-1 the free top (Sec. III.A-B of the paper).
//
// Two launch shapes:
//  * node kernels (right-hand sides, force sweep, reductions over fields):
//    one thread per node, blocks of 64 x 4 nodes of one z-plane;
//  * tile kernels (the conjugate-gradient iterations, which carry all the
//    time): a block owns a 64 x 4 column of nodes and marches it through a
//    chunk of z-planes, staging each plane with a one-node halo in LDS (a
//    ring of three planes), so every stencil neighbour is read from HBM/L2
//    about once.  Blocks are numbered so that consecutive tiles run on the
//    same XCD (work-groups are dealt round-robin to the 8 XCDs), keeping
//    neighbouring tiles' halos in one L2.
//
// Reductions are deterministic: a fixed shuffle tree per wavefront, waves
// in order, one partial per block written with plain stores, then a
// single-block reduce kernel that sums the partials in a fixed order and
// updates the conjugate-gradient scalars on the device.
#include "pf_internal.h"

#include <math.h>
#include <stdlib.h>

namespace pf {

namespace {

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ __forceinline__ int tid_flat() { return threadIdx.x + threadIdx.y * blockDim.x; }

template <typename T>
struct Vec2;
template <>
struct Vec2<double> {
  using type = double2;
};
template <>
struct Vec2<float> {
  using type = float2;
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block partial sums of NV values into partials[bid*NV + t].
template <int NV, int NT>
__device__ __forceinline__ void block_partials(double (&v)[NV], double* partials, int bid) {
  __shared__ double red[NV][NT / 64];
  const int tid = tid_flat();
  const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int t = 0; t < NV; t++) {
    double s = wave_sum(v[t]);
    if (lane == 0) red[t][wv] = s;
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int t = 0; t < NV; t++) {
      double s = 0.0;
      for (int w = 0; w < NT / 64; w++) s += red[t][w];
      partials[(int64_t)bid * NV + t] = s;
    }
  }
}

__device__ __forceinline__ int node_block_id() { return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z); }

__device__ __forceinline__ bool finite(double x) { return isfinite(x); }

// ||r|| <= tol ||b||
__device__ __forceinline__ bool converged(double rnorm2, double bnorm2, double tol) {
  return sqrt(rnorm2) <= tol * sqrt(bnorm2);
}

// ---------------------------------------------------------------------------
// Tile geometry of the z-marching kernels
// ---------------------------------------------------------------------------
// A tile is 64 x TY nodes of a plane (TY = 4: one node per thread; TY = 8:
// two consecutive rows per thread), staged with a one-node halo.
constexpr int kHX = kBX + 2;
template <int TY>
struct Halo {
  static constexpr int HY = TY + 2;                        // halo rows
  static constexpr int HP = kHX * HY;                      // halo points
  static constexpr int NPT = (HP + kThreads - 1) / kThreads;  // points per thread
};

// Logical tile of this block: work-groups go round-robin to the 8 XCDs, so
// XCD x receives physical blocks x, x+8, ...; they are given the contiguous
// logical range [start_x, start_x + count_x).
__device__ __forceinline__ int logical_block(int nblocks) {
  const int b = blockIdx.x;
  const int q = nblocks >> 3, r = nblocks & 7;
  const int x = b & 7, w = b >> 3;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + w;
}

struct TileCoord {
  int i0, j0, k0, k1, lid;
};

// Within a z-chunk, tiles go in groups of gy tile rows: the rows of a group
// fastest, then x, then the groups, so that the blocks that share a y halo
// row start one after the other (x neighbours gy apart) and read it while it
// is still in the XCD's L2; the last group may hold fewer rows.
__device__ __forceinline__ TileCoord tile_coord(const Dims& d, const TileMap& tm) {
  const int lid = logical_block(tm.nblocks);
  TileCoord t;
  const int cols = tm.ntx * tm.nty;
  const int kc = lid / cols;
  const int c = lid - kc * cols;
  const int gsz = tm.gy * tm.ntx;
  const int g = c / gsz;
  const int r = c - g * gsz;
  const int rows = min(tm.gy, tm.nty - g * tm.gy);
  const int tx = r / rows;
  const int ty = g * tm.gy + (r - tx * rows);
  t.i0 = tx * kBX;
  t.j0 = ty * tm.ty;
  t.k0 = kc * tm.kz;
  t.k1 = min(d.nz, t.k0 + tm.kz);
  t.lid = lid;
  return t;
}

__device__ __forceinline__ int slot_of(int k) { return (k + 3) % 3; }

// Jacobi weights of the FEM rows (interior and top plane, per component)
// held in scalars: a run-time choice between two arrays would put the arrays
// in scratch memory.  Without GEN the components share one weight.
template <typename T, bool GEN>
struct JacobiW {
  T i0, i1, i2, t0, t1, t2;
  __device__ __forceinline__ explicit JacobiW(const FemTables* __restrict__ tb)
      : i0((T)tb->inv_diag[0][0]), i1((T)tb->inv_diag[0][GEN ? 1 : 0]), i2((T)tb->inv_diag[0][GEN ? 2 : 0]),
        t0((T)tb->inv_diag[1][0]), t1((T)tb->inv_diag[1][GEN ? 1 : 0]), t2((T)tb->inv_diag[1][GEN ? 2 : 0]) {}
  __device__ __forceinline__ T operator()(bool top, int c) const {
    const T wi = c == 0 ? i0 : (c == 1 ? i1 : i2);
    const T wt = c == 0 ? t0 : (c == 1 ? t1 : t2);
    return top ? wt : wi;
  }
};

// Software-pipelined staging of tile planes.  Each thread owns NPT of the
// halo-plane points.  stage_fetch issues the global loads of a plane into
// registers (raw values, RAW per point); stage_store combines them into the
// staged values (NC per point) and writes the ring slot.  The z-march
// fetches plane k+2 while plane k is being computed, so the loads of a block
// overlap its own arithmetic (the barrier waits for LDS only).
template <typename T, int RAW, int NPT>
struct Stage {
  T v[NPT][RAW];
};

template <int TY, typename T, int RAW, int NPT, typename Fetch>
__device__ __forceinline__ void stage_fetch(Stage<T, RAW, NPT>& st, const Dims& d, int i0, int j0, int k,
                                            Fetch f) {
  using H = Halo<TY>;
#pragma unroll
  for (int q = 0; q < NPT; q++) {
    const int t = tid_flat() + q * kThreads;
#pragma unroll
    for (int c = 0; c < RAW; c++) st.v[q][c] = 0;
    if (t < H::HP) {
      const int hx = t % kHX, hy = t / kHX;
      int gi = i0 + hx - 1, gj = j0 + hy - 1;
      if (k >= 0 && k < d.nz && gi >= -1 && gi <= d.nx && gj >= -1 && gj <= d.ny) {
        gi = wrap(gi, d.nx);
        gj = wrap(gj, d.ny);
        f(gi + (int64_t)d.nx * gj + d.plane * k, k, st.v[q]);
      }
    }
  }
}

template <int TY, typename T, int NC, int RAW, int NPT, typename Comb>
__device__ __forceinline__ void stage_store(T (&ring)[3][NC][TY + 2][kHX], const Stage<T, RAW, NPT>& st, int k,
                                            Comb comb) {
  using H = Halo<TY>;
  const int s = slot_of(k);
#pragma unroll
  for (int q = 0; q < NPT; q++) {
    const int t = tid_flat() + q * kThreads;
    if (t < H::HP) {
      const int hx = t % kHX, hy = t / kHX;
      T out[NC];
      comb(k, st.v[q], out);
#pragma unroll
      for (int c = 0; c < NC; c++) ring[s][c][hy][hx] = out[c];
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Reduce kernel: sums the block partials in a fixed order and advances the
// conjugate-gradient scalars.
//   kRedSetup  (b.b, r.z, r.r) of the initial residual
//   kRedAlpha  p.q            -> alpha = rho / p.q
//   kRedBeta   (r.z, r.r)     -> beta, iteration count, convergence
// ---------------------------------------------------------------------------
//   kRedOuter  (b.b, r.z, r.r) of the FP64 residual of an iterative
//              refinement sweep: records the outer test and starts the
//              inner (FP32) solve for the correction, asked to reach what
//              the outer test still needs, max(tol2, tol ||b|| / (2 ||r||)),
//              tol2 being the floor that FP32 arithmetic can reach
//   kRedSum    plain sums written to out[0..NV-1]
//   kRedCheck  r.r (second value) after the residual update: iteration
//              count and convergence, decided before the preconditioner
//              runs (so the last iteration applies none)
//   kRedConj   r.z (first value) of the preconditioned residual -> beta
constexpr int kRedThreads = 1024;

template <int NV>
__global__ __launch_bounds__(kRedThreads) void cg_reduce_kernel(const double* __restrict__ partials, int nblocks,
                                                                CgScalars* sc, int mode, double tol, int maxit,
                                                                double tol2, double* out) {
  if ((mode == kRedAlpha || mode == kRedBeta || mode == kRedRho || mode == kRedCheck || mode == kRedConj) &&
      sc->done)
    return;
  __shared__ double red[NV][kRedThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double s[NV];
#pragma unroll
  for (int t = 0; t < NV; t++) s[t] = 0.0;
  for (int b = tid; b < nblocks; b += kRedThreads) {
#pragma unroll
    for (int t = 0; t < NV; t++) s[t] += partials[(int64_t)b * NV + t];
  }
#pragma unroll
  for (int t = 0; t < NV; t++) {
    double w = wave_sum(s[t]);
    if (lane == 0) red[t][wv] = w;
  }
  __syncthreads();
  if (tid != 0) return;
  double a[NV];
#pragma unroll
  for (int t = 0; t < NV; t++) {
    a[t] = 0.0;
    for (int w = 0; w < kRedThreads / 64; w++) a[t] += red[t][w];
  }
  if (mode == kRedSum) {
#pragma unroll
    for (int t = 0; t < NV; t++) out[t] = a[t];
    return;
  }
  if (mode == kRedRho) {  // r.z of a preconditioner applied after the setup
    if (!finite(a[0]) || !(a[0] > 0.0)) sc->done = kNonFinite;
    else sc->rho = a[0];
    return;
  }
  if (mode == kRedOuter) {
    const double b2 = a[0], rz = a[NV > 1 ? 1 : 0], r2 = a[NV > 2 ? 2 : 0];
    sc->outer_b2 = b2;
    sc->outer_r2 = r2;
    sc->alpha = 0.0;
    sc->beta = 0.0;
    sc->iter = 0;
    sc->maxit = maxit;
    sc->zero_rhs = 0;
    sc->bnorm2 = r2;  // the inner system's right-hand side is the residual
    sc->rho = rz;
    sc->rnorm2 = r2;
    sc->tol = (r2 > 0.0) ? fmax(tol2, 0.5 * tol * sqrt(b2 / r2)) : tol2;
    if (!finite(b2) || !finite(rz) || !finite(r2)) {
      sc->done = kNonFinite;
      sc->outer_done = 0;
    } else if (b2 == 0.0) {
      sc->done = kConverged;
      sc->outer_done = 1;
      sc->zero_rhs = 1;
    } else if (converged(r2, b2, tol)) {
      sc->done = kConverged;
      sc->outer_done = 1;
    } else {
      sc->done = kRunning;
      sc->outer_done = 0;
    }
    return;
  }
  if (mode == kRedSetup) {
    // a = (b.b, r.z, r.r)
    sc->bnorm2 = a[0];
    sc->rho = a[NV > 1 ? 1 : 0];
    sc->rnorm2 = a[NV > 2 ? 2 : 0];
    sc->alpha = 0.0;
    sc->beta = 0.0;
    sc->iter = 0;
    sc->tol = tol;
    sc->maxit = maxit;
    sc->zero_rhs = 0;
    sc->outer_done = 0;
    const double rn2 = sc->rnorm2;
    if (!finite(a[0]) || !finite(sc->rho) || !finite(rn2)) sc->done = kNonFinite;
    else if (a[0] == 0.0) {
      sc->done = kConverged;
      sc->zero_rhs = 1;
      sc->rnorm2 = 0.0;
    } else if (converged(rn2, a[0], tol)) sc->done = kConverged;
    else sc->done = maxit <= 0 ? kMaxIt : kRunning;
  } else if (mode == kRedAlpha) {
    if (!finite(a[0]) || !(a[0] > 0.0)) sc->done = kNonFinite;
    else sc->alpha = sc->rho / a[0];
  } else if (mode == kRedCheck) {
    const double rr = a[NV > 1 ? 1 : 0];
    const int it = sc->iter + 1;
    sc->iter = it;
    sc->rnorm2 = rr;
    if (!finite(rr)) sc->done = kNonFinite;
    else if (converged(rr, sc->bnorm2, sc->tol)) sc->done = kConverged;
    else if (it >= sc->maxit) sc->done = kMaxIt;
  } else if (mode == kRedConj) {
    const double rz = a[0];
    if (!finite(rz) || !(rz > 0.0)) {
      sc->done = kNonFinite;
    } else {
      sc->beta = rz / sc->rho;
      sc->rho = rz;
    }
  } else {
    const double rz = a[0], rr = a[NV > 1 ? 1 : 0];
    const int it = sc->iter + 1;
    sc->iter = it;
    sc->beta = rz / sc->rho;
    sc->rho = rz;
    sc->rnorm2 = rr;
    if (!finite(rz) || !finite(rr)) sc->done = kNonFinite;
    else if (converged(rr, sc->bnorm2, sc->tol)) sc->done = kConverged;
    else if (it >= sc->maxit) sc->done = kMaxIt;
  }
}

// ---------------------------------------------------------------------------
// Utility kernels
// ---------------------------------------------------------------------------

template <typename T>
__global__ void fill_kernel(T* a, int64_t n, T v) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; t < n; t += stride) a[t] = v;
}

template <typename T, typename U>
__global__ void convert_kernel(const T* a, U* b, int64_t n) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; t < n; t += stride) b[t] = (U)a[t];
}

// x += alpha p with alpha from the solver scalars; x = 0 for a zero rhs.
template <typename T>
__global__ void cg_finish_kernel(T* x, const T* p, int64_t n, const CgScalars* sc) {
  const T alpha = (T)sc->alpha;
  const bool zero = sc->zero_rhs != 0;
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; t < n; t += stride) x[t] = zero ? (T)0 : x[t] + alpha * p[t];
}

// Initial guess for the next solve: x (the last solution) becomes the value
// one step ahead of the polynomial through x and the M earlier solutions of
// the ring (weights from the host), and x is stored into the ring slot that
// drops out.  One read of x and of each history field, two writes.
template <int M>
__global__ void extrapolate_kernel(double* x, ExtrapRing ring, int64_t n) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; t < n; t += stride) {
    const double a = x[t];
    double g = ring.c[0] * a;
#pragma unroll
    for (int k = 0; k < M; k++) g += ring.c[k + 1] * ring.h[k][t];
    ring.dest[t] = a;
    x[t] = g;
  }
}

// warm_start 3: how well each extrapolation order 0..mmax would have
// predicted the newest solution x from the solutions before it (ring.h[0]
// newest), measured on every kScoreStride-th chunk of 256 values by the
// squared second difference along x of the prediction error (the solves
// start from the residual b - A x0 = A (x - x0), and A weighs an error by
// its second differences, so rough errors cost more than smooth ones of the
// same size): per block, the sums go to partials[block][m].
__global__ __launch_bounds__(256) void extrap_score_kernel(const double* __restrict__ x, ExtrapRing ring,
                                                           ExtrapScore sc, int64_t n) {
  double e[kMaxExtrap + 1];
#pragma unroll
  for (int m = 0; m <= kMaxExtrap; m++) e[m] = 0.0;
  const int lane = threadIdx.x & 63;
  const int64_t chunks = (n + 255) / 256;
  // uniform over the block: every lane takes part in the shuffles
  for (int64_t q = (int64_t)blockIdx.x * kScoreStride; q < chunks; q += (int64_t)gridDim.x * kScoreStride) {
    const int64_t i = q * 256 + threadIdx.x;
    const bool in = i < n;
    double h[kMaxExtrap + 1];
#pragma unroll
    for (int t = 0; t <= kMaxExtrap; t++) h[t] = in && t <= sc.mmax ? ring.h[t][i] : 0.0;
    const double xv = in ? x[i] : 0.0;
    // the neighbours along the chunk are the lanes beside (its interior lanes count)
    const bool inner = in && lane > 0 && lane < 63 && i + 1 < n;
#pragma unroll
    for (int m = 0; m <= kMaxExtrap; m++) {
      if (m <= sc.mmax) {  // uniform over the block
        double pr = 0.0;
#pragma unroll
        for (int t = 0; t <= m; t++) pr += sc.c[m][t] * h[t];
        const double er = pr - xv;
        const double lo = __shfl_up(er, 1, 64), hi = __shfl_down(er, 1, 64);
        const double d2 = hi - 2.0 * er + lo;
        if (inner) e[m] += d2 * d2;
      }
    }
  }
  __shared__ double red[kMaxExtrap + 1][256 / 64];
  const int wv = threadIdx.x >> 6;
#pragma unroll
  for (int m = 0; m <= kMaxExtrap; m++) {
    const double w = wave_sum(e[m]);
    if (lane == 0) red[m][wv] = w;
  }
  __syncthreads();
  if (threadIdx.x <= kMaxExtrap) {
    double t = 0.0;
    for (int w = 0; w < 256 / 64; w++) t += red[threadIdx.x][w];
    sc.partials[(int64_t)blockIdx.x * (kMaxExtrap + 1) + threadIdx.x] = t;
  }
}

// Iterative refinement: x64 += d, x32 = x64 (rounded working copy).
// x64 += d, x32 = (float) x64.  With p, the inner solve's deferred last
// update is applied first, d + alpha p, as cg_finish_kernel would have
// (zero when the inner right-hand side was zero).
__global__ void refine_update_kernel(double* x64, float* x32, const float* d, const float* p, const CgScalars* sc,
                                     int64_t n) {
  const float alpha = p ? (float)sc->alpha : 0.f;
  const bool zero = p && sc->zero_rhs != 0;
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; t < n; t += stride) {
    const float dz = p ? (zero ? 0.f : d[t] + alpha * p[t]) : d[t];
    const double v = x64[t] + (double)dz;
    x64[t] = v;
    x32[t] = (float)v;
  }
}

// ---------------------------------------------------------------------------
// Poisson: A phi = -eps_b Lap_h phi (zero ghosts), b = -D_h P + ghost terms
// ---------------------------------------------------------------------------

// Coupling weights of plane k of the potential grid, divided by h^2: in-plane
// faces (the plane's permittivity), the z-faces above and below (harmonic
// means across the film/air interface; none above the open top) and the
// Jacobi weight 1 / (4 xy + up + dn).  The metal top has eps_b everywhere.
template <typename T>
struct PlaneEps {
  T xy, up, dn, w;
};

template <typename T>
__device__ __forceinline__ PlaneEps<T> plane_eps(const Dims& d, const Coefs<T>& cf, int k) {
  PlaneEps<T> e;
  if (!cf.open) {
    e.xy = e.up = e.dn = cf.eps_over_h2;
    e.w = cf.inv_diag_poisson;
    return e;
  }
  const T ef = cf.eps_over_h2, ea = cf.eps_air_over_h2, ei = cf.eps_iface_over_h2;
  e.xy = k < d.nzf ? ef : ea;
  e.dn = k < d.nzf ? ef : (k == d.nzf ? ei : ea);
  e.up = k + 1 >= d.nzp ? (T)0 : (k + 1 < d.nzf ? ef : (k + 1 == d.nzf ? ei : ea));
  e.w = (T)1 / (4 * e.xy + e.up + e.dn);
  return e;
}

// b from Pp = P + cdt V (V may be null) and the ghost planes; r = b - A x;
// partial (b.b, r.z, r.r) with z = r / diag.  The first direction is not
// stored (the first iteration forms it from r); p gets zeros on the
// electrode nodes only.  T: arithmetic and x; S: storage
// of P and V; R: storage of r and p (FP32 for the inner solve of a
// refinement sweep, which also clears its correction dz).  Each block
// marches a 64 x 4 tile up its z-chunk: the values of its own column at the
// planes below and above (x and Pp_z) are carried in registers, so every
// plane is read once; the in-plane neighbours come from the plane in hand.
template <typename T, typename S, typename R>
__global__ __launch_bounds__(kThreads) void poisson_setup_kernel(
    Dims d, TileMap tm, Coefs<T> cf, const S* __restrict__ P, const S* __restrict__ V, T cdt, int with_P,
    int with_bc, const T* __restrict__ ghost_top, T phi_bottom, const uint8_t* __restrict__ emask,
    T* __restrict__ x, R* __restrict__ r, R* __restrict__ p, R* __restrict__ dz, double* partials) {
  const TileCoord tc = tile_coord(d, tm);
  const int i = tc.i0 + threadIdx.x, j = tc.j0 + threadIdx.y;
  double v[3] = {0.0, 0.0, 0.0};
  if (i < d.nx && j < d.ny) {
    const int64_t Nf = d.Nf, pl = d.plane;
    const int64_t col = i + (int64_t)d.nx * j;
    const int64_t cxp = wrap(i + 1, d.nx) + (int64_t)d.nx * j, cxm = wrap(i - 1, d.nx) + (int64_t)d.nx * j;
    const int64_t cyp = i + (int64_t)d.nx * wrap(j + 1, d.ny), cym = i + (int64_t)d.nx * wrap(j - 1, d.ny);
    // electrode nodes of the open top (Dirichlet, first air plane)
    auto is_el = [&](int kk, int64_t c) { return emask != nullptr && kk == d.nzf && emask[c] != 0; };
    auto dval = [&](int64_t c) -> T { return with_bc ? ghost_top[c] : (T)0; };
    auto pp = [&](int c, int64_t m) -> T { return (T)P[c * Nf + m] + (V ? cdt * (T)V[c * Nf + m] : (T)0); };
    // own column: Pp_z of the film planes and x of planes k - 1, k, k + 1
    // (x is not read at electrode nodes: this kernel writes it there)
    auto pz = [&](int kk) -> T { return with_P && kk >= 0 && kk < d.nzf ? pp(2, col + pl * kk) : (T)0; };
    auto xcol = [&](int kk) -> T {
      return kk >= 0 && kk < d.nz && !is_el(kk, col) ? x[col + pl * kk] : (T)0;
    };
    const int k0 = tc.k0;
    T pz_m = pz(k0 - 1), pz_c = pz(k0);
    T x_m = xcol(k0 - 1), x_c = xcol(k0);
    for (int k = k0; k < tc.k1; k++) {
      const int64_t n = col + pl * k;
      const bool up = k + 1 < d.nz, dn = k > 0;
      const T pz_p = pz(k + 1);
      const T x_p = xcol(k + 1);
      if (is_el(k, col)) {
        x[n] = dval(col);
        r[n] = 0;
        p[n] = 0;
        if (dz) dz[n] = 0;
      } else {
        const int64_t nxp = cxp + pl * k, nxm = cxm + pl * k, nyp = cyp + pl * k, nym = cym + pl * k;
        T b = 0;
        if (with_P) {
          const T dx = k < d.nzf ? pp(0, nxp) - pp(0, nxm) : (T)0;
          const T dy = k < d.nzf ? pp(1, nyp) - pp(1, nym) : (T)0;
          b = -(dx + dy + (pz_p - pz_m)) * cf.inv_2h;
        }
        const PlaneEps<T> e = plane_eps(d, cf, k);
        if (with_bc) {
          if (k == 0) b += e.dn * phi_bottom;
          if (!cf.open && k == d.nz - 1) b += e.up * ghost_top[col];
          if (cf.open) {
            if (is_el(k, cxp)) b += e.xy * ghost_top[cxp];
            if (is_el(k, cxm)) b += e.xy * ghost_top[cxm];
            if (is_el(k, cyp)) b += e.xy * ghost_top[cyp];
            if (is_el(k, cym)) b += e.xy * ghost_top[cym];
            if (is_el(k + 1, col)) b += e.up * ghost_top[col];
            if (is_el(k - 1, col)) b += e.dn * ghost_top[col];
          }
        }
        T Ax;
        if (!cf.open) {
          T s = x[nxp] + x[nxm] + x[nyp] + x[nym];
          if (up) s += x_p;
          if (dn) s += x_m;
          Ax = cf.eps_over_h2 * (6 * x_c - s);
        } else {
          auto xu = [&](int kk, int64_t c, int64_t m) -> T { return is_el(kk, c) ? (T)0 : x[m]; };
          const T sxy = xu(k, cxp, nxp) + xu(k, cxm, nxm) + xu(k, cyp, nyp) + xu(k, cym, nym);
          const T xup = up ? x_p : (T)0;
          const T xdn = dn ? x_m : (T)0;
          Ax = e.xy * (4 * x_c - sxy) + e.up * (x_c - xup) + e.dn * (x_c - xdn);
        }
        const T rr = b - Ax;
        const T z = rr * e.w;
        r[n] = (R)rr;
        if (dz) dz[n] = 0;
        v[0] += (double)b * b;
        v[1] += (double)rr * z;
        v[2] += (double)rr * rr;
      }
      pz_m = pz_c;
      pz_c = pz_p;
      x_m = x_c;
      x_c = x_p;
    }
  }
  block_partials<3, kThreads>(v, partials, tc.lid);
}

// Iteration kernel A: p_new = z + beta p_old on the tile and its halo, q =
// A p_new, x += alpha_prev p_old (the deferred update of the previous
// iteration); partial p_new . q.  p_old null: the first iteration, p_new = z.
// unit_w: r holds the preconditioned residual z itself (multigrid).
template <typename T>
__global__ __launch_bounds__(kThreads) void poisson_cg_a_kernel(Dims d, TileMap tm, Coefs<T> cf,
                                                                const T* __restrict__ r, const T* __restrict__ p_old,
                                                                T* __restrict__ p_new, T* __restrict__ x,
                                                                const CgScalars* sc, double* partials, int unit_w) {
  if (sc->done) return;
  constexpr int TY = kBY;
  __shared__ T ring[3][1][TY + 2][kHX];
  const T beta = (T)sc->beta, alpha = (T)sc->alpha, c6 = cf.eps_over_h2;
  // the first iteration (p_old null): p = z, x untouched (alpha, beta zero)
  const bool first = p_old == nullptr;
  const TileCoord tc = tile_coord(d, tm);
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int i = tc.i0 + lx, j = tc.j0 + ly;
  const bool valid = i < d.nx && j < d.ny;
  const int64_t col = valid ? i + (int64_t)d.nx * j : 0;
  auto fetch = [&](int64_t m, int, T* raw) {
    raw[0] = r[m];
    if (!first) raw[1] = p_old[m];
  };
  auto comb = [&](int kk, const T* raw, T* out) {
    out[0] = raw[0] * (unit_w ? (T)1 : plane_eps(d, cf, kk).w) + beta * raw[1];
  };
  Stage<T, 2, Halo<TY>::NPT> st;
  stage_fetch<TY>(st, d, tc.i0, tc.j0, tc.k0 - 1, fetch);
  stage_store<TY>(ring, st, tc.k0 - 1, comb);
  stage_fetch<TY>(st, d, tc.i0, tc.j0, tc.k0, fetch);
  stage_store<TY>(ring, st, tc.k0, comb);
  stage_fetch<TY>(st, d, tc.i0, tc.j0, tc.k0 + 1, fetch);
  T cpo = 0, cx = 0;  // centre p_old, x of the plane being computed
  if (valid && !first) {
    cpo = p_old[col + d.plane * tc.k0];
    cx = x[col + d.plane * tc.k0];
  }
  double acc = 0.0;
  for (int k = tc.k0; k < tc.k1; k++) {
    stage_store<TY>(ring, st, k + 1, comb);
    if (k + 2 <= tc.k1) stage_fetch<TY>(st, d, tc.i0, tc.j0, k + 2, fetch);
    T npo = 0, nx_ = 0;
    if (valid && !first && k + 1 < tc.k1) {
      npo = p_old[col + d.plane * (k + 1)];
      nx_ = x[col + d.plane * (k + 1)];
    }
    __syncthreads();
    if (valid) {
      const int sm = slot_of(k - 1), s0 = slot_of(k), sp = slot_of(k + 1);
      const T pc = ring[s0][0][ly + 1][lx + 1];
      const T sxy = ring[s0][0][ly + 1][lx] + ring[s0][0][ly + 1][lx + 2] + ring[s0][0][ly][lx + 1] +
                    ring[s0][0][ly + 2][lx + 1];
      const T pdn = ring[sm][0][ly + 1][lx + 1], pup = ring[sp][0][ly + 1][lx + 1];
      T q;
      if (!cf.open) {
        q = c6 * (6 * pc - (sxy + pdn + pup));
      } else {
        const PlaneEps<T> e = plane_eps(d, cf, k);
        q = e.xy * (4 * pc - sxy) + e.up * (pc - pup) + e.dn * (pc - pdn);
      }
      const int64_t n = col + d.plane * k;
      p_new[n] = pc;
      if (!first) x[n] = cx + alpha * cpo;
      acc += (double)pc * q;
    }
    cpo = npo;
    cx = nx_;
    __syncthreads();
  }
  double v[1] = {acc};
  block_partials<1, kThreads>(v, partials, tc.lid);
}

// Iteration kernel B: r -= alpha A p (operator recomputed); partial (r.z, r.r).
template <typename T>
__global__ __launch_bounds__(kThreads) void poisson_cg_b_kernel(Dims d, TileMap tm, Coefs<T> cf,
                                                                const T* __restrict__ p, T* __restrict__ r,
                                                                const uint8_t* __restrict__ emask,
                                                                const CgScalars* sc, double* partials) {
  if (sc->done) return;
  constexpr int TY = kBY;
  __shared__ T ring[3][1][TY + 2][kHX];
  const T alpha = (T)sc->alpha, c6 = cf.eps_over_h2;
  const TileCoord tc = tile_coord(d, tm);
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int i = tc.i0 + lx, j = tc.j0 + ly;
  const bool valid = i < d.nx && j < d.ny;
  const int64_t col = valid ? i + (int64_t)d.nx * j : 0;
  auto fetch = [&](int64_t m, int, T* raw) { raw[0] = p[m]; };
  auto comb = [&](int, const T* raw, T* out) { out[0] = raw[0]; };
  Stage<T, 1, Halo<TY>::NPT> st;
  stage_fetch<TY>(st, d, tc.i0, tc.j0, tc.k0 - 1, fetch);
  stage_store<TY>(ring, st, tc.k0 - 1, comb);
  stage_fetch<TY>(st, d, tc.i0, tc.j0, tc.k0, fetch);
  stage_store<TY>(ring, st, tc.k0, comb);
  stage_fetch<TY>(st, d, tc.i0, tc.j0, tc.k0 + 1, fetch);
  T cr = valid ? r[col + d.plane * tc.k0] : (T)0;
  double a0 = 0.0, a1 = 0.0;
  for (int k = tc.k0; k < tc.k1; k++) {
    stage_store<TY>(ring, st, k + 1, comb);
    if (k + 2 <= tc.k1) stage_fetch<TY>(st, d, tc.i0, tc.j0, k + 2, fetch);
    const T nr = (valid && k + 1 < tc.k1) ? r[col + d.plane * (k + 1)] : (T)0;
    __syncthreads();
    if (valid) {
      const int sm = slot_of(k - 1), s0 = slot_of(k), sp = slot_of(k + 1);
      const T pc = ring[s0][0][ly + 1][lx + 1];
      const T sxy = ring[s0][0][ly + 1][lx] + ring[s0][0][ly + 1][lx + 2] + ring[s0][0][ly][lx + 1] +
                    ring[s0][0][ly + 2][lx + 1];
      const T pdn = ring[sm][0][ly + 1][lx + 1], pup = ring[sp][0][ly + 1][lx + 1];
      const PlaneEps<T> e = plane_eps(d, cf, k);
      T q;
      if (!cf.open) q = c6 * (6 * pc - (sxy + pdn + pup));
      else q = e.xy * (4 * pc - sxy) + e.up * (pc - pup) + e.dn * (pc - pdn);
      T rn = cr - alpha * q;
      if (emask != nullptr && k == d.nzf && emask[col] != 0) rn = 0;  // electrode rows stay zero
      r[col + d.plane * k] = rn;
      a0 += (double)rn * (rn * e.w);
      a1 += (double)rn * rn;
    }
    cr = nr;
    __syncthreads();
  }
  double v[2] = {a0, a1};
  block_partials<2, kThreads>(v, partials, tc.lid);
}

// ---------------------------------------------------------------------------
// FEM: 27-point block stencils of the trilinear hex element
// ---------------------------------------------------------------------------

namespace {

// K u at a row of type zt (0 interior, 1 top) for a neighbour loader
// ld(dx, dy, dz, out[3]).  GEN: the general stencil of the tables.  Else the
// stiffness is cubic on the grid axes and each coefficient is one of 8
// (interior) or 24 (top) values, indexed at compile time by kc_class: they
// fit the scalar registers (the 153 and 243 table values do not, and
// spilled coefficients cost v_readlane instructions per row of nodes), and
// the structurally zero taps are skipped.
template <typename T, bool GEN, typename Load>
__device__ __forceinline__ void fem_K_apply(const FemTables* __restrict__ tb, int zt, Load ld, T out[3]) {
  out[0] = out[1] = out[2] = 0;
  if (!GEN) {
    if (zt == 0) {
#pragma unroll
      for (int dz = -1; dz <= 1; dz++)
#pragma unroll
        for (int dy = -1; dy <= 1; dy++)
#pragma unroll
          for (int dx = -1; dx <= 1; dx++) {
            const int off[3] = {dx, dy, dz};
            T u[3];
            ld(dx, dy, dz, u);
#pragma unroll
            for (int c = 0; c < 3; c++)
#pragma unroll
              for (int e = 0; e < 3; e++) {
                int sg = 1;
                const int cl = kc_class(0, c, e, off, &sg);
                if (cl < 0) continue;
                const T k = (T)tb->kc_int[cl];
                out[c] += (sg > 0 ? k : -k) * u[e];
              }
          }
    } else {
#pragma unroll
      for (int dz = -1; dz <= 0; dz++)
#pragma unroll
        for (int dy = -1; dy <= 1; dy++)
#pragma unroll
          for (int dx = -1; dx <= 1; dx++) {
            const int off[3] = {dx, dy, dz};
            T u[3];
            ld(dx, dy, dz, u);
#pragma unroll
            for (int c = 0; c < 3; c++)
#pragma unroll
              for (int e = 0; e < 3; e++) {
                int sg = 1;
                const int cl = kc_class(1, c, e, off, &sg);
                if (cl < 0) continue;
                const T k = (T)tb->kc_top[cl];
                out[c] += (sg > 0 ? k : -k) * u[e];
              }
          }
    }
    return;
  }
  if (zt == 0) {
#pragma unroll
    for (int dz = -1; dz <= 1; dz++)
#pragma unroll
      for (int dy = -1; dy <= 1; dy++)
#pragma unroll
        for (int dx = -1; dx <= 1; dx++) {
          const int o = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
          T u[3];
          ld(dx, dy, dz, u);
#pragma unroll
          for (int c = 0; c < 3; c++)
#pragma unroll
            for (int e = 0; e < 3; e++) out[c] += (T)tb->K[0][c][e][o] * u[e];
        }
  } else {
#pragma unroll
    for (int dz = -1; dz <= 0; dz++)
#pragma unroll
      for (int dy = -1; dy <= 1; dy++)
#pragma unroll
        for (int dx = -1; dx <= 1; dx++) {
          const int o = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
          T u[3];
          ld(dx, dy, dz, u);
#pragma unroll
          for (int c = 0; c < 3; c++)
#pragma unroll
            for (int e = 0; e < 3; e++) out[c] += (T)tb->K[1][c][e][o] * u[e];
        }
  }
}

// Linear index of the neighbour (i+dx, j+dy, k+dz), periodic in x and y.
__device__ __forceinline__ int64_t nbr(const Dims& d, int i, int j, int k, int dx, int dy, int dz) {
  return wrap(i + dx, d.nx) + (int64_t)d.nx * wrap(j + dy, d.ny) + d.plane * (k + dz);
}

// Nodal eigenstrain of P relative to the substrate strain (Eq. 15; Voigt,
// engineering shear): the cubic form on crystal-aligned grids, else the
// grid-frame quadratic forms Qv.
template <bool ROT = true, typename T>
__device__ __forceinline__ void eigenstrain(const Coefs<T>& cf, T x, T y, T z, T e[6]) {
  if (ROT && cf.rotated) {
    const T m[6] = {x * x, y * y, z * z, 2 * x * y, 2 * y * z, 2 * z * x};
#pragma unroll
    for (int v = 0; v < 6; v++) {
      T a = 0;
#pragma unroll
      for (int q = 0; q < 6; q++) a += cf.Qv[v][q] * m[q];
      e[v] = a - cf.es[v];
    }
    return;
  }
  const T x2 = x * x, y2 = y * y, z2 = z * z;
  e[0] = cf.Q11 * x2 + cf.Q12 * (y2 + z2) - cf.es[0];
  e[1] = cf.Q11 * y2 + cf.Q12 * (z2 + x2) - cf.es[1];
  e[2] = cf.Q11 * z2 + cf.Q12 * (x2 + y2) - cf.es[2];
  e[3] = 2 * cf.Q44 * x * y - cf.es[3];
  e[4] = 2 * cf.Q44 * y * z - cf.es[4];
  e[5] = 2 * cf.Q44 * z * x - cf.es[5];
}

// sigma = C e for the Voigt stiffness (engineering shear).
template <bool ROT = true, typename T>
__device__ __forceinline__ void cubic_stress(const Coefs<T>& cf, const T e[6], T s[6]) {
  if (ROT && cf.rotated) {
#pragma unroll
    for (int v = 0; v < 6; v++) {
      T a = 0;
#pragma unroll
      for (int w = 0; w < 6; w++) a += cf.Cg[6 * v + w] * e[w];
      s[v] = a;
    }
    return;
  }
  s[0] = cf.C11 * e[0] + cf.C12 * (e[1] + e[2]);
  s[1] = cf.C11 * e[1] + cf.C12 * (e[2] + e[0]);
  s[2] = cf.C11 * e[2] + cf.C12 * (e[0] + e[1]);
  s[3] = cf.C44 * e[3];
  s[4] = cf.C44 * e[4];
  s[5] = cf.C44 * e[5];
}

// (d eps0/dP)(p) w: the eigenstrain linearised at p in direction w.
template <bool ROT = true, typename T>
__device__ __forceinline__ void eigenstrain_lin(const Coefs<T>& cf, T x, T y, T z, T wx, T wy, T wz, T e[6]) {
  if (ROT && cf.rotated) {
    const T m[6] = {2 * x * wx, 2 * y * wy, 2 * z * wz, 2 * (x * wy + y * wx), 2 * (y * wz + z * wy),
                    2 * (z * wx + x * wz)};
#pragma unroll
    for (int v = 0; v < 6; v++) {
      T a = 0;
#pragma unroll
      for (int q = 0; q < 6; q++) a += cf.Qv[v][q] * m[q];
      e[v] = a;
    }
    return;
  }
  e[0] = 2 * (cf.Q11 * x * wx + cf.Q12 * (y * wy + z * wz));
  e[1] = 2 * (cf.Q11 * y * wy + cf.Q12 * (z * wz + x * wx));
  e[2] = 2 * (cf.Q11 * z * wz + cf.Q12 * (x * wx + y * wy));
  e[3] = 2 * cf.Q44 * (x * wy + y * wx);
  e[4] = 2 * cf.Q44 * (y * wz + z * wy);
  e[5] = 2 * cf.Q44 * (z * wx + x * wz);
}

// s . (d eps0/dP)(p): the elastic driving force of a nodal stress s.  Also
// s . (d2 eps0/dP2) w, which is the same contraction at p = w.
template <bool ROT = true, typename T>
__device__ __forceinline__ void stress_pull(const Coefs<T>& cf, const T p[3], const T s[6], T g[3]) {
  if (ROT && cf.rotated) {
    // sum_v s_v Qv[v] as a symmetric 3x3 matrix, times 2 p
    T A[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int v = 0; v < 6; v++)
#pragma unroll
      for (int q = 0; q < 6; q++) A[q] += s[v] * cf.Qv[v][q];
    g[0] = 2 * (A[0] * p[0] + A[3] * p[1] + A[5] * p[2]);
    g[1] = 2 * (A[3] * p[0] + A[1] * p[1] + A[4] * p[2]);
    g[2] = 2 * (A[5] * p[0] + A[4] * p[1] + A[2] * p[2]);
    return;
  }
  g[0] = 2 * p[0] * (cf.Q11 * s[0] + cf.Q12 * (s[1] + s[2])) + 2 * cf.Q44 * (p[1] * s[3] + p[2] * s[5]);
  g[1] = 2 * p[1] * (cf.Q11 * s[1] + cf.Q12 * (s[2] + s[0])) + 2 * cf.Q44 * (p[0] * s[3] + p[2] * s[4]);
  g[2] = 2 * p[2] * (cf.Q11 * s[2] + cf.Q12 * (s[0] + s[1])) + 2 * cf.Q44 * (p[1] * s[4] + p[0] * s[5]);
}

// Landau energy density, gradient and Hessian (Eq. 1) of the crystal
// components p = R^T P; gradient and Hessian are returned on the grid axes.
// ROT = false compiles the crystal-aligned forms only (the caller knows the
// frame is not rotated); ROT = true decides at run time.
template <bool ROT = true, typename T>
__device__ __forceinline__ void to_crystal(const Coefs<T>& cf, const T P[3], T c[3]) {
  if (!(ROT && cf.rotated)) {
    c[0] = P[0], c[1] = P[1], c[2] = P[2];
    return;
  }
#pragma unroll
  for (int a = 0; a < 3; a++) c[a] = cf.R[a] * P[0] + cf.R[3 + a] * P[1] + cf.R[6 + a] * P[2];
}

template <bool ROT = true, typename T>
__device__ __forceinline__ void to_grid(const Coefs<T>& cf, const T c[3], T P[3]) {
  if (!(ROT && cf.rotated)) {
    P[0] = c[0], P[1] = c[1], P[2] = c[2];
    return;
  }
#pragma unroll
  for (int a = 0; a < 3; a++) P[a] = cf.R[3 * a] * c[0] + cf.R[3 * a + 1] * c[1] + cf.R[3 * a + 2] * c[2];
}

template <bool ROT = true, typename T>
__device__ __forceinline__ T landau_density(const Coefs<T>& cf, const T P[3]) {
  T c[3];
  to_crystal<ROT>(cf, P, c);
  const T x2 = c[0] * c[0], y2 = c[1] * c[1], z2 = c[2] * c[2];
  return cf.a1 * (x2 + y2 + z2) + cf.a11 * (x2 * x2 + y2 * y2 + z2 * z2) + cf.a12 * (x2 * y2 + y2 * z2 + z2 * x2);
}

template <bool ROT = true, typename T>
__device__ __forceinline__ void landau_gradient(const Coefs<T>& cf, const T P[3], T g[3]) {
  T c[3], gc[3];
  to_crystal<ROT>(cf, P, c);
  const T x2 = c[0] * c[0], y2 = c[1] * c[1], z2 = c[2] * c[2];
  gc[0] = 2 * cf.a1 * c[0] + 4 * cf.a11 * x2 * c[0] + 2 * cf.a12 * c[0] * (y2 + z2);
  gc[1] = 2 * cf.a1 * c[1] + 4 * cf.a11 * y2 * c[1] + 2 * cf.a12 * c[1] * (z2 + x2);
  gc[2] = 2 * cf.a1 * c[2] + 4 * cf.a11 * z2 * c[2] + 2 * cf.a12 * c[2] * (x2 + y2);
  to_grid<ROT>(cf, gc, g);
}

template <bool ROT = true, typename T>
__device__ __forceinline__ void landau_hessian_apply(const Coefs<T>& cf, const T P[3], const T w[3], T out[3]) {
  T c[3], wc[3], oc[3];
  to_crystal<ROT>(cf, P, c);
  to_crystal<ROT>(cf, w, wc);
  const T x2 = c[0] * c[0], y2 = c[1] * c[1], z2 = c[2] * c[2];
  const T H00 = 2 * cf.a1 + 12 * cf.a11 * x2 + 2 * cf.a12 * (y2 + z2);
  const T H11 = 2 * cf.a1 + 12 * cf.a11 * y2 + 2 * cf.a12 * (z2 + x2);
  const T H22 = 2 * cf.a1 + 12 * cf.a11 * z2 + 2 * cf.a12 * (x2 + y2);
  const T H01 = 4 * cf.a12 * c[0] * c[1], H12 = 4 * cf.a12 * c[1] * c[2], H02 = 4 * cf.a12 * c[0] * c[2];
  oc[0] = H00 * wc[0] + H01 * wc[1] + H02 * wc[2];
  oc[1] = H01 * wc[0] + H11 * wc[1] + H12 * wc[2];
  oc[2] = H02 * wc[0] + H12 * wc[1] + H22 * wc[2];
  to_grid<ROT>(cf, oc, out);
}

}  // namespace

// f = body force of the eigenstrain of Pp = P + cdt V (Eq. 15); r = f - K x;
// partials with z = r / diag (the first iteration forms the first direction
// itself, so it is not stored).  The clamped plane k = 0 has x = r = p = 0 (both direction
// buffers).  Partial (f.f, r.z, r.r) per tile.
// With W non-null the eigenstrain is replaced by its linearisation at Pp in
// the direction W, deps0 = (d eps0/dP)(Pp) W (the right-hand side of the
// adjoint FEM solve).
// A tile kernel like the force: the body-force stencils are products of 1D
// element integrals (rows m, gt = int N_n' N_m), so with the nodal
// eigenstress sigma = C eps0 staged per plane in LDS, each node forms
//   A_c = (gt x m) sigma_cx + (m x gt) sigma_cy,   B_c = (m x m) sigma_cz
// in x and y and sums f_c(t) = sum_dz mz_t(dz) A_c + gtz_t(dz) B_c over its
// column in registers; x is staged in the usual three-plane ring for K x.
// ROT compiles the rotated-frame eigenstrain and stress (run-time check);
// without it the crystal-aligned forms only, which keeps the 78 coefficients
// of the rotated forms out of the scalar registers.
template <typename T, typename S, typename R, bool GEN, bool ROT>
__global__ __launch_bounds__(kThreads, 3) void fem_setup_kernel(
    Dims d, TileMap tm, Coefs<T> cf, const FemTables* __restrict__ tb, const S* __restrict__ P,
    const S* __restrict__ V, T cdt, const T* __restrict__ W, T* __restrict__ x, R* __restrict__ r,
    R* __restrict__ p0, R* __restrict__ p1, R* __restrict__ dz, T* __restrict__ fout, double* partials) {
  constexpr int TY = kBY;
  using H = Halo<TY>;
  __shared__ T sgm[6][TY + 2][kHX];
  __shared__ T ring[3][3][TY + 2][kHX];
  const TileCoord tc = tile_coord(d, tm);
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int i = tc.i0 + lx, j = tc.j0 + ly;
  const bool valid = i < d.nx && j < d.ny;
  const int64_t N = d.N, pl = d.plane;
  const int64_t col = valid ? i + (int64_t)d.nx * j : 0;
  const bool hasV = V != nullptr, hasW = W != nullptr;
  // the prefetch keeps P and V in the state precision: converting a loaded
  // value would wait for the load; they are converted when staged
  Stage<S, 6, H::NPT> sp;  // P, V of the next source plane
  Stage<T, 3, H::NPT> sw;  // W of the next source plane (with hasW)
  Stage<T, 3, H::NPT> sx;  // x of the next plane
  auto fetch_p = [&](int64_t m, int, S* raw) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
      raw[c] = P[c * N + m];
      raw[3 + c] = hasV ? V[c * N + m] : (S)0;
    }
  };
  auto fetch_w = [&](int64_t m, int, T* raw) {
#pragma unroll
    for (int c = 0; c < 3; c++) raw[c] = W[c * N + m];
  };
  auto fetch_x = [&](int64_t m, int k, T* raw) {
    if (k == 0) return;  // the clamp
#pragma unroll
    for (int c = 0; c < 3; c++) raw[c] = x[c * N + m];
  };
  auto comb_x = [&](int, const T* raw, T* o) {
#pragma unroll
    for (int c = 0; c < 3; c++) o[c] = raw[c];
  };
  auto fetch = [&](int k) {
    stage_fetch<TY>(sp, d, tc.i0, tc.j0, k, fetch_p);
    if (hasW) stage_fetch<TY>(sw, d, tc.i0, tc.j0, k, fetch_w);
    stage_fetch<TY>(sx, d, tc.i0, tc.j0, k, fetch_x);
  };
  // stage plane s: eigenstress into sgm, x into the ring
  auto stage = [&](int s) {
#pragma unroll
    for (int q = 0; q < H::NPT; q++) {
      const int t = tid_flat() + q * kThreads;
      if (t >= H::HP) continue;
      const int hx = t % kHX, hy = t / kHX;
      const int gi = tc.i0 + hx - 1, gj = tc.j0 + hy - 1;
      const bool live = s >= 0 && s < d.nz && gi >= -1 && gi <= d.nx && gj >= -1 && gj <= d.ny;
      T sg[6] = {0, 0, 0, 0, 0, 0};
      if (live) {
        const S* raw = sp.v[q];
        const T px = (T)raw[0] + cdt * (T)raw[3], py = (T)raw[1] + cdt * (T)raw[4], pz = (T)raw[2] + cdt * (T)raw[5];
        T e[6];
        if (hasW) eigenstrain_lin<ROT>(cf, px, py, pz, sw.v[q][0], sw.v[q][1], sw.v[q][2], e);
        else eigenstrain<ROT>(cf, px, py, pz, e);
        cubic_stress<ROT>(cf, e, sg);
      }
#pragma unroll
      for (int v = 0; v < 6; v++) sgm[v][hy][hx] = sg[v];
    }
    stage_store<TY>(ring, sx, s, comb_x);
  };
  const T mI[3] = {(T)tb->m1[kInterior][0], (T)tb->m1[kInterior][1], (T)tb->m1[kInterior][2]};
  const T tI[3] = {(T)tb->gt1[kInterior][0], (T)tb->gt1[kInterior][1], (T)tb->gt1[kInterior][2]};
  auto xy_pass = [&](T A[3], T B[3]) {
#pragma unroll
    for (int c = 0; c < 3; c++) A[c] = B[c] = 0;
#pragma unroll 1
    for (int dy = -1; dy <= 1; dy++)
#pragma unroll
      for (int dx = -1; dx <= 1; dx++) {
        const int hx = lx + 1 + dx, hy = ly + 1 + dy;
        const T mm = mI[dx + 1] * mI[dy + 1], gm = tI[dx + 1] * mI[dy + 1], mg = mI[dx + 1] * tI[dy + 1];
        const T s0 = sgm[0][hy][hx], s1 = sgm[1][hy][hx], s2 = sgm[2][hy][hx];
        const T s3 = sgm[3][hy][hx], s4 = sgm[4][hy][hx], s5 = sgm[5][hy][hx];
        A[0] += gm * s0 + mg * s3;
        A[1] += gm * s3 + mg * s1;
        A[2] += gm * s5 + mg * s4;
        B[0] += mm * s5;
        B[1] += mm * s4;
        B[2] += mm * s2;
      }
  };
  auto zkind = [&](int t) { return t == 0 ? kLow : (t == d.nz - 1 ? kHigh : kInterior); };
  auto contrib = [&](int t, int dzo, const T A[3], const T B[3], T f[3], bool add) {
    const int zk = zkind(t);
    const T mz = (T)tb->m1[zk][dzo + 1], gz = (T)tb->gt1[zk][dzo + 1];
#pragma unroll
    for (int c = 0; c < 3; c++) f[c] = (add ? f[c] : (T)0) + mz * A[c] + gz * B[c];
  };
  T f0[3] = {0, 0, 0}, f1[3] = {0, 0, 0};  // z-sums of the body force of planes k and k + 1
  const int k0 = tc.k0;
  if (k0 > 0) {
    fetch(k0 - 1);
    stage(k0 - 1);
    __syncthreads();
    if (valid) {
      T A[3], B[3];
      xy_pass(A, B);
      contrib(k0, -1, A, B, f0, false);
    }
    __syncthreads();
  }
  fetch(k0);
  stage(k0);
  fetch(k0 + 1);
  __syncthreads();
  if (valid) {
    T A[3], B[3];
    xy_pass(A, B);
    contrib(k0, 0, A, B, f0, true);
    contrib(k0 + 1, -1, A, B, f1, false);
  }
  __syncthreads();
  const JacobiW<T, GEN> jw(tb);
  double v[3] = {0.0, 0.0, 0.0};
  for (int k = k0; k < tc.k1; k++) {
    stage(k + 1);
    if (k + 2 <= tc.k1) fetch(k + 2);
    __syncthreads();
    if (valid) {
      T A[3], B[3];
      xy_pass(A, B);
      if (k + 1 < d.nz) contrib(k, 1, A, B, f0, true);
      const int64_t n = col + pl * k;
      if (k == 0) {
#pragma unroll
        for (int c = 0; c < 3; c++) {
          x[c * N + n] = 0;
          r[c * N + n] = 0;
          p0[c * N + n] = 0;
          p1[c * N + n] = 0;
          if (dz) dz[c * N + n] = 0;
          if (fout) fout[c * N + n] = 0;
        }
      } else {
        const int zt = (k == d.nz - 1) ? 1 : 0;
        auto ld = [&](int ox, int oy, int oz, T u[3]) {
          const int sl = slot_of(k + oz);
#pragma unroll
          for (int c = 0; c < 3; c++) u[c] = ring[sl][c][ly + 1 + oy][lx + 1 + ox];
        };
        T Kx[3];
        fem_K_apply<T, GEN>(tb, zt, ld, Kx);
#pragma unroll
        for (int c = 0; c < 3; c++) {
          const T rr = f0[c] - Kx[c];
          const T z = rr * jw(zt, c);
          r[c * N + n] = (R)rr;
          if (dz) dz[c * N + n] = 0;
          if (fout) fout[c * N + n] = f0[c];
          v[0] += (double)f0[c] * f0[c];
          v[1] += (double)rr * z;
          v[2] += (double)rr * rr;
        }
      }
      // slide: plane k + 1 becomes the one being completed
#pragma unroll
      for (int c = 0; c < 3; c++) f0[c] = f1[c];
      if (k + 1 < d.nz) {
        contrib(k + 1, 0, A, B, f0, true);
        contrib(k + 2, -1, A, B, f1, false);
      }
    }
    __syncthreads();
  }
  block_partials<3, kThreads>(v, partials, tc.lid);
}

// Residual of a later refinement sweep, r = f - K x, from the body force f
// that the first sweep's setup stored (fem_setup_kernel with fout), so the
// eigenstress is not formed again.  Outputs as fem_setup_kernel: r, zeros
// in dz (and in x, r, p0, p1 on the clamped plane),
// and the partials (f.f, r.z, r.r) per tile.  x is staged in the three-plane
// LDS ring; K x is the same apply as in fem_setup_kernel, so the residual is
// bitwise the one the full setup would form.
template <typename T, typename R, bool GEN>
__global__ __launch_bounds__(kThreads, 4) void fem_resid_kernel(Dims d, TileMap tm, const FemTables* __restrict__ tb,
                                                             const T* __restrict__ f, T* __restrict__ x,
                                                             R* __restrict__ r, R* __restrict__ p0,
                                                             R* __restrict__ p1, R* __restrict__ dz,
                                                             double* partials) {
  constexpr int TY = kBY;
  using H = Halo<TY>;
  __shared__ T ring[3][3][TY + 2][kHX];
  const TileCoord tc = tile_coord(d, tm);
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int i = tc.i0 + lx, j = tc.j0 + ly;
  const bool valid = i < d.nx && j < d.ny;
  const int64_t N = d.N, pl = d.plane;
  const int64_t col = valid ? i + (int64_t)d.nx * j : 0;
  Stage<T, 3, H::NPT> sx;
  auto fetch_x = [&](int64_t m, int k, T* raw) {
    if (k == 0) return;  // the clamp
#pragma unroll
    for (int c = 0; c < 3; c++) raw[c] = x[c * N + m];
  };
  auto comb_x = [&](int, const T* raw, T* o) {
#pragma unroll
    for (int c = 0; c < 3; c++) o[c] = raw[c];
  };
  const int k0 = tc.k0;
  if (k0 > 0) {
    stage_fetch<TY>(sx, d, tc.i0, tc.j0, k0 - 1, fetch_x);
    stage_store<TY>(ring, sx, k0 - 1, comb_x);
  }
  stage_fetch<TY>(sx, d, tc.i0, tc.j0, k0, fetch_x);
  stage_store<TY>(ring, sx, k0, comb_x);
  stage_fetch<TY>(sx, d, tc.i0, tc.j0, k0 + 1, fetch_x);
  const JacobiW<T, GEN> jw(tb);
  double v[3] = {0.0, 0.0, 0.0};
  for (int k = k0; k < tc.k1; k++) {
    // the slot of plane k + 1 last held plane k - 2, read before the barrier
    // that ended the previous plane
    stage_store<TY>(ring, sx, k + 1, comb_x);
    if (k + 2 <= tc.k1) stage_fetch<TY>(sx, d, tc.i0, tc.j0, k + 2, fetch_x);
    __syncthreads();
    if (valid) {
      const int64_t n = col + pl * k;
      if (k == 0) {
#pragma unroll
        for (int c = 0; c < 3; c++) {
          x[c * N + n] = 0;
          r[c * N + n] = 0;
          p0[c * N + n] = 0;
          p1[c * N + n] = 0;
          dz[c * N + n] = 0;
        }
      } else {
        const int zt = (k == d.nz - 1) ? 1 : 0;
        auto ld = [&](int ox, int oy, int oz, T u[3]) {
          const int sl = slot_of(k + oz);
#pragma unroll
          for (int c = 0; c < 3; c++) u[c] = ring[sl][c][ly + 1 + oy][lx + 1 + ox];
        };
        T Kx[3];
        fem_K_apply<T, GEN>(tb, zt, ld, Kx);
#pragma unroll
        for (int c = 0; c < 3; c++) {
          const T fc = f[c * N + n];
          const T rr = fc - Kx[c];
          const T z = rr * jw(zt, c);
          r[c * N + n] = (R)rr;
          dz[c * N + n] = 0;
          v[0] += (double)fc * fc;
          v[1] += (double)rr * z;
          v[2] += (double)rr * rr;
        }
      }
    }
    __syncthreads();
  }
  block_partials<3, kThreads>(v, partials, tc.lid);
}

// Iteration kernel A: p_new = z + beta p_old on the tile and its halo (zero
// on the clamped plane), q = K p_new, x += alpha_prev p_old; partial p.q.
// p_old null: the first iteration, p_new = z and x untouched.
// At most 128 VGPRs: four waves per SIMD, so four 256-thread blocks per CU
// and the whole tile grid resident at once.
// unit_w: r holds the preconditioned residual z itself (multigrid), so the
// Jacobi weights are not applied.
template <typename T, bool GEN>
__global__ __launch_bounds__(kThreads, 4) void fem_cg_a_kernel(Dims d, TileMap tm, const FemTables* __restrict__ tb,
                                                            const T* __restrict__ r, const T* __restrict__ p_old,
                                                            T* __restrict__ p_new, T* __restrict__ x,
                                                            const CgScalars* sc, double* partials, int unit_w) {
  if (sc->done) return;
  constexpr int TY = kBY;
  __shared__ T ring[3][3][TY + 2][kHX];
  const T beta = (T)sc->beta, alpha = (T)sc->alpha;
  // the first iteration (p_old null): p = z, no deferred update of x (alpha
  // and beta are zero), so neither p_old nor x is read or written
  const bool first = p_old == nullptr;
  // Jacobi weights per component (equal for a cubic stiffness on the grid axes)
  const JacobiW<T, GEN> jw(tb);
  const TileCoord tc = tile_coord(d, tm);
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int i = tc.i0 + lx, j = tc.j0 + ly;
  const bool valid = i < d.nx && j < d.ny;
  const int64_t N = d.N;
  const int64_t col = valid ? i + (int64_t)d.nx * j : 0;
  auto fetch = [&](int64_t m, int k, T* raw) {
    if (k == 0) return;  // clamped plane: zero
#pragma unroll
    for (int c = 0; c < 3; c++) raw[c] = r[c * N + m];
    if (first) return;
#pragma unroll
    for (int c = 0; c < 3; c++) raw[3 + c] = p_old[c * N + m];
  };
  auto comb = [&](int k, const T* raw, T* out) {
    const bool top = k == d.nz - 1;
#pragma unroll
    for (int c = 0; c < 3; c++) out[c] = raw[c] * (unit_w ? (T)1 : jw(top, c)) + beta * raw[3 + c];
  };
  // centre values (p_old, x) of a plane
  auto centre = [&](int k, T* cv) {
#pragma unroll
    for (int c = 0; c < 6; c++) cv[c] = 0;
    if (!first && valid && k > 0 && k < tc.k1) {
      const int64_t n = col + d.plane * k;
#pragma unroll
      for (int c = 0; c < 3; c++) {
        cv[c] = p_old[c * N + n];
        cv[3 + c] = x[c * N + n];
      }
    }
  };
  Stage<T, 6, Halo<TY>::NPT> st;
  stage_fetch<TY>(st, d, tc.i0, tc.j0, tc.k0 - 1, fetch);
  stage_store<TY>(ring, st, tc.k0 - 1, comb);
  stage_fetch<TY>(st, d, tc.i0, tc.j0, tc.k0, fetch);
  stage_store<TY>(ring, st, tc.k0, comb);
  stage_fetch<TY>(st, d, tc.i0, tc.j0, tc.k0 + 1, fetch);
  T cv[6];
  centre(tc.k0, cv);
  double acc = 0.0;
  for (int k = tc.k0; k < tc.k1; k++) {
    stage_store<TY>(ring, st, k + 1, comb);
    if (k + 2 <= tc.k1) stage_fetch<TY>(st, d, tc.i0, tc.j0, k + 2, fetch);
    T nv[6];
    centre(k + 1, nv);
    __syncthreads();
    if (valid && k > 0) {
      const int zt = (k == d.nz - 1) ? 1 : 0;
      auto ld = [&](int dx, int dy, int dz, T u[3]) {
        const int s = slot_of(k + dz);
#pragma unroll
        for (int c = 0; c < 3; c++) u[c] = ring[s][c][ly + 1 + dy][lx + 1 + dx];
      };
      T q[3];
      fem_K_apply<T, GEN>(tb, zt, ld, q);
      const int64_t n = col + d.plane * k;
      const int s0 = slot_of(k);
#pragma unroll
      for (int c = 0; c < 3; c++) {
        const T pc = ring[s0][c][ly + 1][lx + 1];
        p_new[c * N + n] = pc;
        if (!first) x[c * N + n] = cv[3 + c] + alpha * cv[c];
        acc += (double)pc * q[c];
      }
    }
#pragma unroll
    for (int c = 0; c < 6; c++) cv[c] = nv[c];
    __syncthreads();
  }
  double v[1] = {acc};
  block_partials<1, kThreads>(v, partials, tc.lid);
}

// Iteration kernel B: r -= alpha K p (operator recomputed); partial (r.z, r.r).
template <typename T, bool GEN>
__global__ __launch_bounds__(kThreads, 4) void fem_cg_b_kernel(Dims d, TileMap tm, const FemTables* __restrict__ tb,
                                                            const T* __restrict__ p, T* __restrict__ r,
                                                            const CgScalars* sc, double* partials) {
  if (sc->done) return;
  constexpr int TY = kBY;
  __shared__ T ring[3][3][TY + 2][kHX];
  const T alpha = (T)sc->alpha;
  const JacobiW<T, GEN> jw(tb);
  const TileCoord tc = tile_coord(d, tm);
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int i = tc.i0 + lx, j = tc.j0 + ly;
  const bool valid = i < d.nx && j < d.ny;
  const int64_t N = d.N;
  const int64_t col = valid ? i + (int64_t)d.nx * j : 0;
  auto fetch = [&](int64_t m, int k, T* raw) {
    if (k == 0) return;
#pragma unroll
    for (int c = 0; c < 3; c++) raw[c] = p[c * N + m];
  };
  auto comb = [&](int, const T* raw, T* out) {
#pragma unroll
    for (int c = 0; c < 3; c++) out[c] = raw[c];
  };
  auto centre = [&](int k, T* cv) {
#pragma unroll
    for (int c = 0; c < 3; c++) cv[c] = 0;
    if (valid && k > 0 && k < tc.k1) {
      const int64_t n = col + d.plane * k;
#pragma unroll
      for (int c = 0; c < 3; c++) cv[c] = r[c * N + n];
    }
  };
  Stage<T, 3, Halo<TY>::NPT> st;
  stage_fetch<TY>(st, d, tc.i0, tc.j0, tc.k0 - 1, fetch);
  stage_store<TY>(ring, st, tc.k0 - 1, comb);
  stage_fetch<TY>(st, d, tc.i0, tc.j0, tc.k0, fetch);
  stage_store<TY>(ring, st, tc.k0, comb);
  stage_fetch<TY>(st, d, tc.i0, tc.j0, tc.k0 + 1, fetch);
  T cv[3];
  centre(tc.k0, cv);
  double a0 = 0.0, a1 = 0.0;
  for (int k = tc.k0; k < tc.k1; k++) {
    stage_store<TY>(ring, st, k + 1, comb);
    if (k + 2 <= tc.k1) stage_fetch<TY>(st, d, tc.i0, tc.j0, k + 2, fetch);
    T nv[3];
    centre(k + 1, nv);
    __syncthreads();
    if (valid && k > 0) {
      const int zt = (k == d.nz - 1) ? 1 : 0;
      auto ld = [&](int dx, int dy, int dz, T u[3]) {
        const int s = slot_of(k + dz);
#pragma unroll
        for (int c = 0; c < 3; c++) u[c] = ring[s][c][ly + 1 + dy][lx + 1 + dx];
      };
      T q[3];
      fem_K_apply<T, GEN>(tb, zt, ld, q);
      const int64_t n = col + d.plane * k;
#pragma unroll
      for (int c = 0; c < 3; c++) {
        const T rn = cv[c] - alpha * q[c];
        r[c * N + n] = rn;
        a0 += (double)rn * (rn * jw(zt, c));
        a1 += (double)rn * rn;
      }
    }
#pragma unroll
    for (int c = 0; c < 3; c++) cv[c] = nv[c];
    __syncthreads();
  }
  double v[2] = {a0, a1};
  block_partials<2, kThreads>(v, partials, tc.lid);
}

// ---------------------------------------------------------------------------
// Multigrid V-cycle of the FEM operator (preconditioner of the FEM CG)
// ---------------------------------------------------------------------------
// Level 0 is the FEM grid (operator from the FEM tables, tiled like the CG
// kernels); coarser levels hold Galerkin operators as per-plane 27-point
// block stencils.  Plane 0 of every level is the clamp: it is never written
// (the buffers hold zero there).

// Sum of v over the block, written by thread 0 to *dst.
template <int NT>
__device__ __forceinline__ void block_sum_to(double v, double* dst) {
  __shared__ double red[NT / 64];
  const int tid = tid_flat();
  const int lane = tid & 63, wv = tid >> 6;
  const double s = wave_sum(v);
  if (lane == 0) red[wv] = s;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int w = 0; w < NT / 64; w++) t += red[w];
    *dst = t;
  }
}

// The coarse correction at the nodes of a tile and its halo (kMgCorrect).
// With x and y halved, a fine node i has the coarse parents i >> 1 and
// (i + 1) >> 1 along each axis (one parent when i is even).  For each fine
// plane the footprint of the tile, CX x CY coarse columns starting at
// (i0 / 2 - 1, j0 / 2 - 1), is z-interpolated into an LDS table; halo point
// (hx, hy) then has its parents in table columns (hx + 1) >> 1, (hx >> 1) + 1
// and rows (hy + 1) >> 1, (hy >> 1) + 1 (i0 and j0 even).
template <int TY>
struct CoarseTile {
  static constexpr int CX = kBX / 2 + 2, CY = TY / 2 + 2, NP = CX * CY;
};
static_assert(CoarseTile<kBY>::NP <= kThreads, "one coarse column per thread");

template <typename T, int NC>
struct CoarseRegs {
  int64_t col;  // the coarse column this thread stages, -1 if none
  double w[2];  // z weights of the two parents of the plane being staged
  T v[2][NC];
};

__device__ __forceinline__ int pmod(int a, int n) { return ((a % n) + n) % n; }

template <int TY, typename T, int NC>
__device__ __forceinline__ void coarse_init(CoarseRegs<T, NC>& cr, const MgCoarse<T>& mc, int i0, int j0) {
  using C = CoarseTile<TY>;
  const int t = tid_flat();
  cr.col = -1;
  if (t < C::NP)
    cr.col = pmod(i0 / 2 - 1 + t % C::CX, mc.nx) + (int64_t)mc.nx * pmod(j0 / 2 - 1 + t / C::CX, mc.ny);
}

// Loads the coarse parents of stored fine plane k (weights zero outside the
// fine planes [0, fnz) and for fixed coarse planes).
template <typename T, int NC>
__device__ __forceinline__ void coarse_fetch(CoarseRegs<T, NC>& cr, const MgCoarse<T>& mc, int k, int fnz) {
  // the plane's parents and weights are uniform over the block (scalar
  // registers); only the loads depend on the thread's column
  const bool inside = k >= 0 && k < fnz;
  const MgZ z = mc.zmap[inside ? k + mc.zoff : mc.zoff];
  const int zi[2] = {z.lo, z.hi};
  const double zw[2] = {z.wlo, z.whi};
#pragma unroll
  for (int t = 0; t < 2; t++) {
    const bool live = inside && zw[t] != 0.0 && zi[t] != 0 && !(mc.top_fixed && zi[t] == mc.nz - 1);
    cr.w[t] = live ? zw[t] : 0.0;
#pragma unroll
    for (int c = 0; c < NC; c++) cr.v[t][c] = live && cr.col >= 0 ? mc.e[c * mc.N + cr.col + mc.plane * zi[t]] : (T)0;
  }
}

template <int TY, typename T, int NC>
__device__ __forceinline__ void coarse_store(double (&E)[2][NC][CoarseTile<TY>::CY][CoarseTile<TY>::CX],
                                             const CoarseRegs<T, NC>& cr, int k) {
  using C = CoarseTile<TY>;
  if (cr.col < 0) return;
  const int t = tid_flat();
#pragma unroll
  for (int c = 0; c < NC; c++)
    E[k & 1][c][t / C::CX][t % C::CX] = cr.w[0] * (double)cr.v[0][c] + cr.w[1] * (double)cr.v[1][c];
}

template <int TY, int NC>
__device__ __forceinline__ double coarse_interp(const double (&E)[2][NC][CoarseTile<TY>::CY][CoarseTile<TY>::CX],
                                                int k, int c, int hx, int hy) {
  const int a0 = (hx + 1) >> 1, a1 = (hx >> 1) + 1, b0 = (hy + 1) >> 1, b1 = (hy >> 1) + 1;
  const double(&e)[CoarseTile<TY>::CY][CoarseTile<TY>::CX] = E[k & 1][c];
  return 0.5 * (0.5 * (e[b0][a0] + e[b0][a1]) + 0.5 * (e[b1][a0] + e[b1][a1]));
}

// stage_store with the halo coordinates passed to comb(k, raw, out, hx, hy).
template <int TY, typename T, int NC, int RAW, int NPT, typename Comb>
__device__ __forceinline__ void stage_store_xy(T (&ring)[3][NC][TY + 2][kHX], const Stage<T, RAW, NPT>& st, int k,
                                               Comb comb) {
  using H = Halo<TY>;
  const int s = slot_of(k);
#pragma unroll
  for (int q = 0; q < NPT; q++) {
    const int t = tid_flat() + q * kThreads;
    if (t < H::HP) {
      const int hx = t % kHX, hy = t / kHX;
      T out[NC];
      comb(k, st.v[q], out, hx, hy);
#pragma unroll
      for (int c = 0; c < NC; c++) ring[s][c][hy][hx] = out[c];
    }
  }
}

// Fine level, kMgCorrect: out = x + omega D^-1 (b - K x) from
// x = omega D^-1 b + P e (e from mc), x formed while its planes are staged;
// with partials, the tile's sum of b . out goes to partials[lid * pstride +
// poff].  D^-1 of the fine level is the Jacobi weight of the FEM tables
// (interior or top row).  The stiffness is applied in pull form (each node
// reads its 27 neighbours from a three-plane LDS ring): the push form of
// mg_fine_kernel needs more registers than this kernel can spare.
template <typename T, bool GEN>
__global__ __launch_bounds__(kThreads, 4) void mg_correct_kernel(Dims d, TileMap tm, const FemTables* __restrict__ tb,
                                                              const double* __restrict__ dinv, double omega,
                                                              const T* __restrict__ b, T* __restrict__ out,
                                                              MgCoarse<T> mc, const CgScalars* sc, double* partials,
                                                              int pstride, int poff) {
  if (sc->done) return;
  constexpr int TY = kBY;
  __shared__ T ring[3][3][TY + 2][kHX];
  __shared__ double E[2][3][CoarseTile<TY>::CY][CoarseTile<TY>::CX];
  const TileCoord tc = tile_coord(d, tm);
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int i = tc.i0 + lx, j = tc.j0 + ly;
  const bool valid = i < d.nx && j < d.ny;
  const int64_t N = d.N;
  const int64_t col = valid ? i + (int64_t)d.nx * j : 0;
  auto fetch = [&](int64_t m, int k, T* raw) {
    if (k == 0) return;
#pragma unroll
    for (int c = 0; c < 3; c++) raw[c] = b[c * N + m];
  };
  // x = omega D^-1 b + P e on the planes with unknowns (1 .. nz-1)
  auto comb = [&](int k, const T* raw, T* o, int hx, int hy) {
    const bool live = k > 0 && k < d.nz;
#pragma unroll
    for (int c = 0; c < 3; c++)
      o[c] = live ? (T)(omega * dinv[3 * k + c] * (double)raw[c] + coarse_interp<TY, 3>(E, k, c, hx, hy)) : (T)0;
  };
  auto put = [&](const auto& stg, int k) { stage_store_xy<TY>(ring, stg, k, comb); };
  auto centre = [&](int k, T* cv) {
#pragma unroll
    for (int c = 0; c < 3; c++) cv[c] = 0;
    if (valid && k > 0 && k < tc.k1) {
      const int64_t n = col + d.plane * k;
#pragma unroll
      for (int c = 0; c < 3; c++) cv[c] = b[c * N + n];
    }
  };
  // the coarse tables of planes k0 - 1 and k0 precede their ring slots; the
  // one of k0 + 1 is written once nothing reads its buffer (that of k0 - 1)
  CoarseRegs<T, 3> cr;
  coarse_init<TY>(cr, mc, tc.i0, tc.j0);
  coarse_fetch(cr, mc, tc.k0 - 1, d.nz);
  coarse_store<TY>(E, cr, tc.k0 - 1);
  coarse_fetch(cr, mc, tc.k0, d.nz);
  coarse_store<TY>(E, cr, tc.k0);
  coarse_fetch(cr, mc, tc.k0 + 1, d.nz);
  __syncthreads();
  Stage<T, 3, Halo<TY>::NPT> st;
  stage_fetch<TY>(st, d, tc.i0, tc.j0, tc.k0 - 1, fetch);
  put(st, tc.k0 - 1);
  stage_fetch<TY>(st, d, tc.i0, tc.j0, tc.k0, fetch);
  put(st, tc.k0);
  __syncthreads();
  coarse_store<TY>(E, cr, tc.k0 + 1);
  __syncthreads();
  stage_fetch<TY>(st, d, tc.i0, tc.j0, tc.k0 + 1, fetch);
  T cv[3];
  centre(tc.k0, cv);
  double acc = 0.0;
  for (int k = tc.k0; k < tc.k1; k++) {
    put(st, k + 1);
    if (k + 2 <= tc.k1) {
      stage_fetch<TY>(st, d, tc.i0, tc.j0, k + 2, fetch);
      coarse_fetch(cr, mc, k + 2, d.nz);
    }
    T nv[3];
    centre(k + 1, nv);
    __syncthreads();
    if (valid && k > 0) {
      const int zt = (k == d.nz - 1) ? 1 : 0;
      auto ld = [&](int dx, int dy, int dz, T u[3]) {
        const int s = slot_of(k + dz);
#pragma unroll
        for (int c = 0; c < 3; c++) u[c] = ring[s][c][ly + 1 + dy][lx + 1 + dx];
      };
      T q[3];
      fem_K_apply<T, GEN>(tb, zt, ld, q);
      const int64_t n = col + d.plane * k;
      const int s0 = slot_of(k);
#pragma unroll
      for (int c = 0; c < 3; c++) {
        const T r = cv[c] - q[c];
        const T o = ring[s0][c][ly + 1][lx + 1] + (T)(omega * dinv[3 * k + c]) * r;
        out[c * N + n] = o;
        acc += (double)cv[c] * (double)o;
      }
    }
    // the table of plane k + 2 reuses the buffer of plane k, last read
    // before the barrier above
    if (k + 2 <= tc.k1) coarse_store<TY>(E, cr, k + 2);
#pragma unroll
    for (int c = 0; c < 3; c++) cv[c] = nv[c];
    __syncthreads();
  }
  if (partials) block_sum_to<kThreads>(acc, partials + (int64_t)tc.lid * pstride + poff);
}

// Stiffness apply in z-push form: the node values u(dx, dy) of source plane
// s (ld(dx, dy, u)) add their part of K u to the outputs of planes s - 1
// (acc[0], which sees plane s at dz = +1), s (acc[1], dz = 0) and s + 1
// (acc[2], dz = -1), each with the row kind of its own plane: Z0 and ZP are
// those of planes s and s + 1 (0 interior, 1 top, -1 no plane).  Plane s - 1
// is an interior row (a top row has no plane above it).  Each source value
// is read once per plane instead of once per output plane.
template <typename T, bool GEN, int Z0, int ZP, typename Load>
__device__ __forceinline__ void fem_K_push(const FemTables* __restrict__ tb, Load ld, T (&acc)[3][3]) {
#pragma unroll
  for (int dy = -1; dy <= 1; dy++)
#pragma unroll
    for (int dx = -1; dx <= 1; dx++) {
      T u[3];
      ld(dx, dy, u);
#pragma unroll
      for (int q = 0; q < 3; q++) {
        const int zt = q == 0 ? 0 : (q == 1 ? Z0 : ZP);
        const int dz = 1 - q;
        if (zt < 0 || (zt == 1 && dz > 0)) continue;
        const int off[3] = {dx, dy, dz};
        const int o = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
#pragma unroll
        for (int c = 0; c < 3; c++)
#pragma unroll
          for (int e = 0; e < 3; e++) {
            if (GEN) {
              acc[q][c] += (T)tb->K[zt][c][e][o] * u[e];
            } else {
              int sg = 1;
              const int cl = kc_class(zt, c, e, off, &sg);
              if (cl < 0) continue;
              const T k = (T)(zt ? tb->kc_top[cl] : tb->kc_int[cl]);
              acc[q][c] += (sg > 0 ? k : -k) * u[e];
            }
          }
      }
    }
}

// Fine level: out = b - K (omega D^-1 b) (kMgFirst) or out = x + omega D^-1
// (b - K x) (kMgSweep); with partials, the tile's sum of b . out goes to
// partials[lid * pstride + poff].  D^-1 of the fine level is the Jacobi
// weight of the FEM tables (interior or top row).  The z-march visits
// the source planes s = k0 - 1 .. k1 once each; plane s is staged in a
// three-slot LDS ring, pushed into the register accumulators of planes
// s - 1, s, s + 1 (fem_K_push), and plane s - 1 is then complete.  With
// three slots one barrier per plane suffices: the slot written while plane
// s is pushed last held plane s - 2.
template <typename T, bool GEN, int MODE>
__global__ __launch_bounds__(kThreads, 4) void mg_fine_kernel(Dims d, TileMap tm, const FemTables* __restrict__ tb,
                                                           const double* __restrict__ dinv, double omega,
                                                           const T* __restrict__ x, const T* __restrict__ b,
                                                           T* __restrict__ out, const CgScalars* sc, double* partials,
                                                           int pstride, int poff) {
  if (sc->done) return;
  constexpr int TY = kBY;
  constexpr bool FIRST = MODE == kMgFirst;
  constexpr bool UPDATE = MODE == kMgSweep;  // out = x + omega D^-1 r
  __shared__ T ring[3][3][TY + 2][kHX];
  const TileCoord tc = tile_coord(d, tm);
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int i = tc.i0 + lx, j = tc.j0 + ly;
  const bool valid = i < d.nx && j < d.ny;
  const int64_t N = d.N;
  const int64_t col = valid ? i + (int64_t)d.nx * j : 0;
  // plain loads: arithmetic on a loaded value would wait for the load here
  // and undo the prefetch; the first sweep's omega D^-1 is applied when the
  // plane is staged
  auto fetch = [&](int64_t m, int k, T* raw) {
    if (k == 0) return;
    const T* src = FIRST ? b : x;
#pragma unroll
    for (int c = 0; c < 3; c++) raw[c] = src[c * N + m];
  };
  auto comb = [&](int k, const T* raw, T* o) {
    const int zt = k == d.nz - 1 ? 1 : 0;
#pragma unroll
    for (int c = 0; c < 3; c++) o[c] = FIRST ? (T)(omega * tb->inv_diag[zt][c]) * raw[c] : raw[c];
  };
  auto centre = [&](int k, T* cv) {
#pragma unroll
    for (int c = 0; c < 3; c++) cv[c] = 0;
    if (valid && k > 0 && k < tc.k1) {
      const int64_t n = col + d.plane * k;
#pragma unroll
      for (int c = 0; c < 3; c++) cv[c] = b[c * N + n];
    }
  };
  Stage<T, 3, Halo<TY>::NPT> st;
  stage_fetch<TY>(st, d, tc.i0, tc.j0, tc.k0 - 1, fetch);
  stage_store<TY>(ring, st, tc.k0 - 1, comb);
  stage_fetch<TY>(st, d, tc.i0, tc.j0, tc.k0, fetch);
  T acc[3][3];
  T cvT[3], cvS[3], xT[3], xS[3];  // b and x at the centre of planes s - 1 (T) and s (S)
#pragma unroll
  for (int c = 0; c < 3; c++) {
    acc[0][c] = acc[1][c] = acc[2][c] = 0;
    cvT[c] = xT[c] = xS[c] = 0;
  }
  double dot = 0.0;
  for (int s = tc.k0 - 1; s <= tc.k1; s++) {
    if (s + 1 <= tc.k1) stage_store<TY>(ring, st, s + 1, comb);
    if (s + 2 <= tc.k1) stage_fetch<TY>(st, d, tc.i0, tc.j0, s + 2, fetch);
    centre(s, cvS);  // used once plane s is complete, an iteration later
    __syncthreads();
    const int sl = slot_of(s);
    auto ld = [&](int dx, int dy, T u[3]) {
#pragma unroll
      for (int c = 0; c < 3; c++) u[c] = ring[sl][c][ly + 1 + dy][lx + 1 + dx];
    };
    if (s > 0 && s < d.nz) {
      if (UPDATE) {
#pragma unroll
        for (int c = 0; c < 3; c++) xS[c] = ring[sl][c][ly + 1][lx + 1];
      }
      if (s < d.nz - 2) fem_K_push<T, GEN, 0, 0>(tb, ld, acc);
      else if (s == d.nz - 2) fem_K_push<T, GEN, 0, 1>(tb, ld, acc);
      else fem_K_push<T, GEN, 1, -1>(tb, ld, acc);
    }
    const int t = s - 1;  // complete: its last source plane was s
    if (valid && t >= 1 && t >= tc.k0 && t < tc.k1) {
      const int64_t n = col + d.plane * t;
#pragma unroll
      for (int c = 0; c < 3; c++) {
        const T r = cvT[c] - acc[0][c];
        const T o = UPDATE ? xT[c] + (T)(omega * dinv[3 * t + c]) * r : r;
        out[c * N + n] = o;
        dot += (double)cvT[c] * (double)o;
      }
    }
#pragma unroll
    for (int c = 0; c < 3; c++) {
      acc[0][c] = acc[1][c];
      acc[1][c] = acc[2][c];
      acc[2][c] = 0;
      cvT[c] = cvS[c];
      xT[c] = xS[c];
    }
  }
  if (partials) block_sum_to<kThreads>(dot, partials + (int64_t)tc.lid * pstride + poff);
}

// Coarse level (per-plane stencils tab[k][c][e][o], NC components): out =
// b - A x or out = x + omega D^-1 (b - A x).  Plane 0 and, with top_fixed,
// the top plane hold no unknowns (never written, zero).  One thread per node.
// With STAGE the block first copies its plane's stencil into LDS (one load
// per thread): the scalar loads of the NC x NC x 27 coefficients, more than
// the scalar registers hold, would otherwise form a chain of round trips
// that dominates the launch on the small levels.
template <typename T, int NC, bool STAGE>
__global__ __launch_bounds__(kThreads) void mg_level_kernel(Dims d, const double* __restrict__ tab,
                                                            const double* __restrict__ dinv, int mode, double omega,
                                                            const T* __restrict__ x, const T* __restrict__ b,
                                                            T* __restrict__ out, const CgScalars* sc, int top_fixed) {
  if (sc->done) return;
  const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y, k = blockIdx.z;
  const int ktop = d.nz - (top_fixed ? 1 : 0);
  if (k == 0 || k >= ktop) return;  // uniform over the block
  constexpr int NT = NC * NC * 27;
  __shared__ double ctab[STAGE ? NT : 1];
  const double* tk = tab + (size_t)k * NT;
  if constexpr (STAGE) {
    for (int t = tid_flat(); t < NT; t += kThreads) ctab[t] = tk[t];
    __syncthreads();
    tk = ctab;
  }
  if (i >= d.nx || j >= d.ny) return;
  const int64_t N = d.N;
  const int64_t n = i + (int64_t)d.nx * j + d.plane * k;
  // neighbour indices in 32 bits (coarse levels are small), per-component
  // base pointers uniform across the block
  const int pl = (int)d.plane;
  const int xi[3] = {wrap(i - 1, d.nx), i, wrap(i + 1, d.nx)};
  const int yo[3] = {wrap(j - 1, d.ny) * d.nx, j * d.nx, wrap(j + 1, d.ny) * d.nx};
  const T* xb[NC];
#pragma unroll
  for (int e = 0; e < NC; e++) xb[e] = x + e * N;
  double q[NC];
#pragma unroll
  for (int c = 0; c < NC; c++) q[c] = 0.0;
#pragma unroll
  for (int dz = -1; dz <= 1; dz++) {
    const int kk = k + dz;
    if (kk < 1 || kk >= ktop) continue;
    const int zo = kk * pl;
#pragma unroll
    for (int dy = -1; dy <= 1; dy++)
#pragma unroll
      for (int dx = -1; dx <= 1; dx++) {
        const int o = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
        const int m = xi[dx + 1] + yo[dy + 1] + zo;
        double u[NC];
#pragma unroll
        for (int e = 0; e < NC; e++) u[e] = (double)xb[e][m];
#pragma unroll
        for (int c = 0; c < NC; c++)
#pragma unroll
          for (int e = 0; e < NC; e++) q[c] += tk[(c * NC + e) * 27 + o] * u[e];
      }
  }
#pragma unroll
  for (int c = 0; c < NC; c++) {
    const double r = (double)b[c * N + n] - q[c];
    out[c * N + n] = (T)(mode == kMgResidual ? r : (double)x[c * N + n] + omega * dinv[NC * k + c] * r);
  }
}

// Levels with at least kMgMarchMinNodes nodes use mg_level_zm_kernel, FP64
// levels with at least kMgTileMinNodes mg_level_tile_kernel.
constexpr int64_t kMgTileMinNodes = 1 << 19;
constexpr int64_t kMgMarchMinNodes = 1 << 19;

// mg_level_kernel with the neighbourhood staged: the block's kBX x kBY
// columns of plane k and their one-node halo on planes k - 1, k and k + 1
// are loaded into LDS once (about 14 loads per node instead of 81), then each
// node applies its plane's stencil from LDS with the arithmetic, and the
// order of summation, of mg_level_kernel.
template <typename T, int NC>
__global__ __launch_bounds__(kThreads) void mg_level_tile_kernel(Dims d, const double* __restrict__ tab,
                                                                 const double* __restrict__ dinv, int mode,
                                                                 double omega, const T* __restrict__ x,
                                                                 const T* __restrict__ b, T* __restrict__ out,
                                                                 const CgScalars* sc, int top_fixed) {
  if (sc->done) return;
  const int k = blockIdx.z;
  const int ktop = d.nz - (top_fixed ? 1 : 0);
  if (k == 0 || k >= ktop) return;  // uniform over the block
  constexpr int NT = NC * NC * 27;
  constexpr int HX = kBX + 2, HY = kBY + 2, HP = HX * HY;
  __shared__ double ctab[NT];
  __shared__ T xs[3][NC][HY][HX];
  const double* tk = tab + (size_t)k * NT;
  for (int t = tid_flat(); t < NT; t += kThreads) ctab[t] = tk[t];
  const int i0 = blockIdx.x * kBX, j0 = blockIdx.y * kBY;
  const int64_t N = d.N;
  // planes k - 1 .. k + 1; zero outside the unknowns (plane 0, the fixed
  // top) and at halo positions no node of the tile reads
  for (int t = tid_flat(); t < 3 * HP; t += kThreads) {
    const int dz = t / HP, r = t - dz * HP, hy = r / HX, hx = r - hy * HX;
    const int kk = k - 1 + dz;
    const int gi = i0 + hx - 1, gj = j0 + hy - 1;
    T v[NC];
#pragma unroll
    for (int e = 0; e < NC; e++) v[e] = 0;
    if (kk >= 1 && kk < ktop && gi >= -1 && gi <= d.nx && gj >= -1 && gj <= d.ny) {
      const int64_t m = wrap(gi, d.nx) + (int64_t)d.nx * wrap(gj, d.ny) + d.plane * kk;
#pragma unroll
      for (int e = 0; e < NC; e++) v[e] = x[e * N + m];
    }
#pragma unroll
    for (int e = 0; e < NC; e++) xs[dz][e][hy][hx] = v[e];
  }
  __syncthreads();
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int i = i0 + lx, j = j0 + ly;
  if (i >= d.nx || j >= d.ny) return;
  const int64_t n = i + (int64_t)d.nx * j + d.plane * k;
  double q[NC];
#pragma unroll
  for (int c = 0; c < NC; c++) q[c] = 0.0;
#pragma unroll
  for (int dz = -1; dz <= 1; dz++) {
    const int kk = k + dz;
    if (kk < 1 || kk >= ktop) continue;
#pragma unroll
    for (int dy = -1; dy <= 1; dy++)
#pragma unroll
      for (int dx = -1; dx <= 1; dx++) {
        const int o = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
        double u[NC];
#pragma unroll
        for (int e = 0; e < NC; e++) u[e] = (double)xs[dz + 1][e][ly + 1 + dy][lx + 1 + dx];
#pragma unroll
        for (int c = 0; c < NC; c++)
#pragma unroll
          for (int e = 0; e < NC; e++) q[c] += ctab[(c * NC + e) * 27 + o] * u[e];
      }
  }
#pragma unroll
  for (int c = 0; c < NC; c++) {
    const double r = (double)b[c * N + n] - q[c];
    out[c * N + n] = (T)(mode == kMgResidual ? r : (double)x[c * N + n] + omega * dinv[NC * k + c] * r);
  }
}

// mg_level_kernel by 64 x 4 tiles marching up a z-chunk: each plane of x is
// fetched from memory once (with its one-node halo) into a three-plane LDS
// ring, software-pipelined like the solver-grid kernels (the loads of plane
// k + 2 are in flight while plane k is computed).  The plane's stencil is
// uniform over the block and read with scalar loads, so the LDS serves only
// the neighbour values (a table staged in LDS made the kernel LDS-bound: 27
// taps x NC^2 coefficient reads per node against 27 NC neighbour reads).
// Fixed planes are staged as zero and never written; the arithmetic and the
// order of summation are those of mg_level_kernel.
template <typename T, int NC>
__global__ __launch_bounds__(kThreads) void mg_level_zm_kernel(Dims d, TileMap tm, const double* __restrict__ tab,
                                                               const double* __restrict__ dinv, int mode,
                                                               double omega, const T* __restrict__ x,
                                                               const T* __restrict__ b, T* __restrict__ out,
                                                               const CgScalars* sc, int top_fixed) {
  if (sc->done) return;
  constexpr int TY = kBY;
  constexpr int NT = NC * NC * 27;
  __shared__ T ring[3][NC][TY + 2][kHX];
  const TileCoord tc = tile_coord(d, tm);
  const int ktop = d.nz - (top_fixed ? 1 : 0);
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int i = tc.i0 + lx, j = tc.j0 + ly;
  const bool valid = i < d.nx && j < d.ny;
  const int64_t N = d.N;
  const int64_t col = valid ? i + (int64_t)d.nx * j : 0;
  auto live = [&](int k) { return k >= 1 && k < ktop; };
  auto fetch = [&](int64_t m, int k, T* raw) {
    if (!live(k)) return;
#pragma unroll
    for (int e = 0; e < NC; e++) raw[e] = x[e * N + m];
  };
  auto comb = [&](int, const T* raw, T* o) {
#pragma unroll
    for (int e = 0; e < NC; e++) o[e] = raw[e];
  };
  auto centre = [&](int k, T* bv) {
#pragma unroll
    for (int c = 0; c < NC; c++) bv[c] = 0;
    if (valid && live(k)) {
      const int64_t n = col + d.plane * k;
#pragma unroll
      for (int c = 0; c < NC; c++) bv[c] = b[c * N + n];
    }
  };
  Stage<T, NC, Halo<TY>::NPT> st;
  stage_fetch<TY>(st, d, tc.i0, tc.j0, tc.k0 - 1, fetch);
  stage_store<TY>(ring, st, tc.k0 - 1, comb);
  stage_fetch<TY>(st, d, tc.i0, tc.j0, tc.k0, fetch);
  stage_store<TY>(ring, st, tc.k0, comb);
  stage_fetch<TY>(st, d, tc.i0, tc.j0, tc.k0 + 1, fetch);
  T bv[NC];
  centre(tc.k0, bv);
  for (int k = tc.k0; k < tc.k1; k++) {
    stage_store<TY>(ring, st, k + 1, comb);
    if (k + 2 <= tc.k1) stage_fetch<TY>(st, d, tc.i0, tc.j0, k + 2, fetch);
    T bn[NC];
    centre(k + 1, bn);
    __syncthreads();
    if (valid && live(k)) {
      const double* tk = tab + (size_t)k * NT;
      double q[NC];
#pragma unroll
      for (int c = 0; c < NC; c++) q[c] = 0.0;
#pragma unroll
      for (int dz = -1; dz <= 1; dz++) {
        if (!live(k + dz)) continue;
        const int s = slot_of(k + dz);
#pragma unroll
        for (int dy = -1; dy <= 1; dy++)
#pragma unroll
          for (int dx = -1; dx <= 1; dx++) {
            const int o = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
            double u[NC];
#pragma unroll
            for (int e = 0; e < NC; e++) u[e] = (double)ring[s][e][ly + 1 + dy][lx + 1 + dx];
#pragma unroll
            for (int c = 0; c < NC; c++)
#pragma unroll
              for (int e = 0; e < NC; e++) q[c] += tk[(c * NC + e) * 27 + o] * u[e];
          }
      }
      const int64_t n = col + d.plane * k;
      const int sk = slot_of(k);
#pragma unroll
      for (int c = 0; c < NC; c++) {
        const double r = (double)bv[c] - q[c];
        out[c * N + n] =
            (T)(mode == kMgResidual ? r : (double)ring[sk][c][ly + 1][lx + 1] + omega * dinv[NC * k + c] * r);
      }
    }
#pragma unroll
    for (int c = 0; c < NC; c++) bv[c] = bn[c];
    __syncthreads();
  }
}

// x = omega D^-1 b (the first sweep from zero); fixed planes get zero (their
// inverse diagonal is zero).
template <typename T, int NC>
__global__ __launch_bounds__(kThreads) void mg_scale_kernel(Dims d, const double* __restrict__ dinv, double omega,
                                                            const T* __restrict__ b, T* __restrict__ x,
                                                            const CgScalars* sc) {
  if (sc->done) return;
  const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y, k = blockIdx.z;
  if (i >= d.nx || j >= d.ny) return;
  const int64_t n = i + (int64_t)d.nx * j + d.plane * k;
#pragma unroll
  for (int c = 0; c < NC; c++) x[c * d.N + n] = (T)(omega * dinv[NC * k + c] * (double)b[c * d.N + n]);
}

// Parents of fine node i along a periodic axis: coarse node i/2 (even i) or
// the two coarse neighbours with weight 1/2 (odd i); identity when the axis
// is not coarsened.
__device__ __forceinline__ int mg_parents(int i, int nc, int coarsened, int idx[2], double w[2]) {
  if (!coarsened) {
    idx[0] = i, w[0] = 1.0;
    return 1;
  }
  if ((i & 1) == 0) {
    idx[0] = i >> 1, w[0] = 1.0;
    return 1;
  }
  idx[0] = (i - 1) >> 1, idx[1] = ((i + 1) >> 1) % nc, w[0] = w[1] = 0.5;
  return 2;
}

// Restriction (the transpose of the prolongation): coarse b = P^T r.  One
// thread per coarse node.  The z maps count the finer level's planes from its
// plane 0; its stored plane is that index minus zoff (the Poisson grid
// stores no ghost planes), and planes outside storage carry zero.  Fixed
// planes of the finer level (its plane 0 and, with ftop_fixed, its top
// plane) hold no unknowns and are never read: no kernel writes them, so
// they may hold anything (other precisions' data included).
template <typename T, int NC>
__global__ __launch_bounds__(kThreads) void mg_restrict_kernel(Dims df, Dims dc, int cx, int cy,
                                                               const MgZ* __restrict__ zmap,
                                                               const int* __restrict__ zfine, const T* __restrict__ rf,
                                                               T* __restrict__ bc, const CgScalars* sc, int zoff,
                                                               int fnz, int ftop_fixed, int ctop_fixed) {
  if (sc->done) return;
  const int I = blockIdx.x * kBX + threadIdx.x, J = blockIdx.y * kBY + threadIdx.y, K = blockIdx.z;
  if (I >= dc.nx || J >= dc.ny || K == 0 || (ctop_fixed && K == dc.nz - 1)) return;
  double acc[NC];
#pragma unroll
  for (int c = 0; c < NC; c++) acc[c] = 0.0;
  const int kf0 = zfine[K];
  for (int kf = kf0 - 1; kf <= kf0 + 1; kf++) {
    const int ks = kf - zoff;
    if (kf < 1 || kf >= fnz - (ftop_fixed ? 1 : 0) || ks < 0 || ks >= df.nz) continue;
    const MgZ z = zmap[kf];
    double wz = 0.0;
    if (z.lo == K) wz += z.wlo;
    if (z.hi == K && z.hi != z.lo) wz += z.whi;
    if (wz == 0.0) continue;
    for (int di = -1; di <= 1; di++) {
      if (!cx && di != 0) continue;
      const int fi = cx ? wrap(2 * I + di, df.nx) : I;
      const double wx = di == 0 ? 1.0 : 0.5;
      for (int dj = -1; dj <= 1; dj++) {
        if (!cy && dj != 0) continue;
        const int fj = cy ? wrap(2 * J + dj, df.ny) : J;
        const double w = wz * wx * (dj == 0 ? 1.0 : 0.5);
        const int64_t m = fi + (int64_t)df.nx * fj + df.plane * ks;
#pragma unroll
        for (int c = 0; c < NC; c++) acc[c] += w * (double)rf[c * df.N + m];
      }
    }
  }
  const int64_t nc = I + (int64_t)dc.nx * J + dc.plane * K;
#pragma unroll
  for (int c = 0; c < NC; c++) bc[c * dc.N + nc] = (T)acc[c];
}

// Prolongation and correction: xf += P xc, or, with bf, xf = omega D^-1 bf
// + P xc (the first sweep from zero, which the kMgFirst residual kernels
// never stored, plus the correction).  One thread per stored fine node
// (plane index + zoff in the z map); fixed planes are skipped.
template <typename T, int NC>
__global__ __launch_bounds__(kThreads) void mg_prolong_kernel(Dims df, Dims dc, int cx, int cy,
                                                              const MgZ* __restrict__ zmap, const T* __restrict__ xc,
                                                              T* __restrict__ xf, const CgScalars* sc, int zoff,
                                                              int ftop_fixed, int ctop_fixed,
                                                              const T* __restrict__ bf,
                                                              const double* __restrict__ dinv, double omega) {
  if (sc->done) return;
  const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y, k = blockIdx.z;
  const int kf = k + zoff;
  if (i >= df.nx || j >= df.ny || kf == 0 || (ftop_fixed && k == df.nz - 1)) return;
  int xi[2], yi[2];
  double xw[2], yw[2];
  const int nxp = mg_parents(i, dc.nx, cx, xi, xw), nyp = mg_parents(j, dc.ny, cy, yi, yw);
  const MgZ z = zmap[kf];
  const int zi[2] = {z.lo, z.hi};
  const double zw[2] = {z.wlo, z.whi};
  double acc[NC];
#pragma unroll
  for (int c = 0; c < NC; c++) acc[c] = 0.0;
  for (int a = 0; a < 2; a++) {
    if (zw[a] == 0.0 || zi[a] == 0 || (ctop_fixed && zi[a] == dc.nz - 1)) continue;
    for (int bq = 0; bq < nyp; bq++)
      for (int q = 0; q < nxp; q++) {
        const double w = zw[a] * yw[bq] * xw[q];
        const int64_t m = xi[q] + (int64_t)dc.nx * yi[bq] + dc.plane * zi[a];
#pragma unroll
        for (int c = 0; c < NC; c++) acc[c] += w * (double)xc[c * dc.N + m];
      }
  }
  const int64_t n = i + (int64_t)df.nx * j + df.plane * k;
#pragma unroll
  for (int c = 0; c < NC; c++) {
    const double base = bf ? omega * dinv[NC * k + c] * (double)bf[c * df.N + n] : (double)xf[c * df.N + n];
    xf[c * df.N + n] = (T)(base + acc[c]);
  }
}

// The transfers between a level and the next when both x and y are halved
// (the common case; the kernels above handle the others).
//
// Restriction by coarse columns: thread (I, J) owns KC coarse planes of one
// z-chunk and visits each contributing fine plane once, summing its 3 x 3
// in-plane footprint (weights 1/2, 1, 1/2 per axis) and pushing it into the
// planes the z map sends it to.  Large planes take KC = 4 (fewer re-reads of
// the fine planes shared by neighbouring coarse planes), small ones KC = 1
// (more threads).
template <typename T, int NC, int KC>
__global__ __launch_bounds__(kThreads) void mg_restrict2_kernel(Dims df, Dims dc, const MgZ* __restrict__ zmap,
                                                                const int* __restrict__ zfine,
                                                                const T* __restrict__ rf, T* __restrict__ bc,
                                                                const CgScalars* sc, int zoff, int fnz,
                                                                int ftop_fixed, int ctop_fixed) {
  if (sc->done) return;
  const int I = blockIdx.x * kBX + threadIdx.x, J = blockIdx.y * kBY + threadIdx.y;
  if (I >= dc.nx || J >= dc.ny) return;
  const int K0 = blockIdx.z * KC;
  const int Ktop = dc.nz - (ctop_fixed ? 1 : 0);  // coarse planes [1, Ktop) hold unknowns
  const int Ka = max(K0, 1), Kb = min(K0 + KC, Ktop);
  if (Ka >= Kb) return;
  double acc[KC][NC];
#pragma unroll
  for (int q = 0; q < KC; q++)
#pragma unroll
    for (int c = 0; c < NC; c++) acc[q][c] = 0.0;
  int fx[3], fy[3];
#pragma unroll
  for (int t = 0; t < 3; t++) {
    fx[t] = wrap(2 * I + t - 1, df.nx);
    fy[t] = wrap(2 * J + t - 1, df.ny);
  }
  const double w1[3] = {0.5, 1.0, 0.5};
  // the finer level's fixed planes are not read (see mg_restrict_kernel)
  const int kf0 = max(zfine[Ka] - 1, 1), kf1 = min(zfine[Kb - 1] + 1, fnz - 1 - (ftop_fixed ? 1 : 0));
  for (int kf = kf0; kf <= kf1; kf++) {
    const int ks = kf - zoff;
    if (ks < 0 || ks >= df.nz) continue;
    const MgZ z = zmap[kf];
    double s[NC];
#pragma unroll
    for (int c = 0; c < NC; c++) s[c] = 0.0;
#pragma unroll
    for (int b = 0; b < 3; b++)
#pragma unroll
      for (int a = 0; a < 3; a++) {
        const double w = w1[a] * w1[b];
        const int64_t m = fx[a] + (int64_t)df.nx * fy[b] + df.plane * ks;
#pragma unroll
        for (int c = 0; c < NC; c++) s[c] += w * (double)rf[c * df.N + m];
      }
#pragma unroll
    for (int q = 0; q < KC; q++) {
      const int K = K0 + q;
      double wz = 0.0;
      if (z.lo == K) wz += z.wlo;
      if (z.hi == K && z.hi != z.lo) wz += z.whi;
#pragma unroll
      for (int c = 0; c < NC; c++) acc[q][c] += wz * s[c];
    }
  }
#pragma unroll
  for (int q = 0; q < KC; q++) {
    const int K = K0 + q;
    if (K < Ka || K >= Kb) continue;
    const int64_t n = I + (int64_t)dc.nx * J + dc.plane * K;
#pragma unroll
    for (int c = 0; c < NC; c++) bc[c * dc.N + n] = (T)acc[q][c];
  }
}

// Prolongation by coarse footprints: thread (I, J) of fine plane k forms the
// z-interpolated coarse values at (I, J), (I+1, J), (I, J+1), (I+1, J+1) once
// and writes the four fine nodes (2I, 2J) .. (2I+1, 2J+1); the modes of
// mg_prolong_kernel.
template <typename T, int NC>
__global__ __launch_bounds__(kThreads) void mg_prolong2_kernel(Dims df, Dims dc, const MgZ* __restrict__ zmap,
                                                               const T* __restrict__ xc, T* __restrict__ xf,
                                                               const CgScalars* sc, int zoff, int ftop_fixed,
                                                               int ctop_fixed, const T* __restrict__ bf,
                                                               const double* __restrict__ dinv, double omega) {
  if (sc->done) return;
  const int I = blockIdx.x * kBX + threadIdx.x, J = blockIdx.y * kBY + threadIdx.y, k = blockIdx.z;
  const int kf = k + zoff;
  if (I >= dc.nx || J >= dc.ny || kf == 0 || (ftop_fixed && k == df.nz - 1)) return;
  const MgZ z = zmap[kf];
  const int zi[2] = {z.lo, z.hi};
  const double zw[2] = {z.wlo, z.whi};
  const int I1 = I + 1 == dc.nx ? 0 : I + 1, J1 = J + 1 == dc.ny ? 0 : J + 1;
  double e[2][2][NC];
#pragma unroll
  for (int b = 0; b < 2; b++)
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
      for (int c = 0; c < NC; c++) e[b][a][c] = 0.0;
  for (int t = 0; t < 2; t++) {
    if (zw[t] == 0.0 || zi[t] == 0 || (ctop_fixed && zi[t] == dc.nz - 1)) continue;
    const int64_t base = dc.plane * zi[t];
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
      for (int a = 0; a < 2; a++) {
        const int64_t m = (a ? I1 : I) + (int64_t)dc.nx * (b ? J1 : J) + base;
#pragma unroll
        for (int c = 0; c < NC; c++) e[b][a][c] += zw[t] * (double)xc[c * dc.N + m];
      }
  }
  // the fine pair (2I, 2I + 1) of a row is one 2-vector (fine nx is even)
  using T2 = typename Vec2<T>::type;
#pragma unroll
  for (int b = 0; b < 2; b++) {
    const int64_t n = 2 * I + (int64_t)df.nx * (2 * J + b) + df.plane * k;
#pragma unroll
    for (int c = 0; c < NC; c++) {
      // bilinear weights of the fine nodes (2I, 2J + b) and (2I + 1, 2J + b)
      const double v0 = b ? 0.5 * (e[0][0][c] + e[1][0][c]) : e[0][0][c];
      const double v1 = b ? 0.25 * (e[0][0][c] + e[0][1][c] + e[1][0][c] + e[1][1][c])
                          : 0.5 * (e[0][0][c] + e[0][1][c]);
      T2* dst = reinterpret_cast<T2*>(xf + c * df.N + n);
      double b0, b1;
      if (bf) {
        const T2 bv = *reinterpret_cast<const T2*>(bf + c * df.N + n);
        const double wgt = omega * dinv[NC * k + c];
        b0 = wgt * (double)bv.x;
        b1 = wgt * (double)bv.y;
      } else {
        const T2 xv = *dst;
        b0 = (double)xv.x;
        b1 = (double)xv.y;
      }
      T2 o;
      o.x = (T)(b0 + v0);
      o.y = (T)(b1 + v1);
      *dst = o;
    }
  }
}

// Coarsest level: x = M b over the unknowns (n / NC per component, planes 1
// upwards), M the dense inverse (row-major, n x n).  One block per row.
template <typename T, int NC>
__global__ __launch_bounds__(256) void mg_dense_kernel(Dims d, int n, const double* __restrict__ M,
                                                       const T* __restrict__ b, T* __restrict__ x,
                                                       const CgScalars* sc) {
  if (sc->done) return;
  const int row = blockIdx.x;
  const int64_t nu = n / NC;  // unknowns per component
  auto vec = [&](int64_t u) { return (u / nu) * d.N + d.plane + u % nu; };
  double s = 0.0;
  for (int t = threadIdx.x; t < n; t += 256) s += M[(int64_t)row * n + t] * (double)b[vec(t)];
  __shared__ double red[4];
  const double w = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
  __syncthreads();
  if (threadIdx.x == 0) x[vec(row)] = (T)(red[0] + red[1] + red[2] + red[3]);
}

// Poisson fine level (the potential grid, tiled like the CG kernels), the
// modes of the FEM fine level, with the operator of every stored plane
// counted (the electrode rows of the open top included); with
// emask the output is zeroed on the electrode nodes (the preconditioner of
// the reduced system), and with partials the tile's b . out goes to
// partials[lid * pstride + poff].
template <typename T, int MODE>
__global__ __launch_bounds__(kThreads) void mgp_fine_kernel(Dims d, TileMap tm, Coefs<T> cf,
                                                            const double* __restrict__ dinv, double omega,
                                                            const T* __restrict__ x, const T* __restrict__ b,
                                                            T* __restrict__ out, MgCoarse<T> mc,
                                                            const uint8_t* __restrict__ emask, const CgScalars* sc,
                                                            double* partials, int pstride, int poff) {
  if (sc->done) return;
  constexpr int TY = kBY;
  constexpr bool FIRST = MODE == kMgFirst, CORR = MODE == kMgCorrect;
  using C = CoarseTile<TY>;
  __shared__ T ring[3][1][TY + 2][kHX];
  __shared__ double E[2][1][CORR ? C::CY : 1][CORR ? C::CX : 1];
  const T c6 = cf.eps_over_h2;
  const TileCoord tc = tile_coord(d, tm);
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int i = tc.i0 + lx, j = tc.j0 + ly;
  const bool valid = i < d.nx && j < d.ny;
  const int64_t col = valid ? i + (int64_t)d.nx * j : 0;
  // plain loads (see mg_fine_kernel); the first sweep's omega D^-1 is applied
  // when the plane is staged (raw is zero outside the stored planes)
  auto fetch = [&](int64_t m, int, T* raw) { raw[0] = ((FIRST || CORR) ? b : x)[m]; };
  auto comb = [&](int k, const T* raw, T* o) {
    o[0] = FIRST && k >= 0 && k < d.nz ? (T)(omega * dinv[k]) * raw[0] : raw[0];
  };
  // kMgCorrect: x = omega D^-1 b + P e on the stored planes
  auto comb_corr = [&](int k, const T* raw, T* o, int hx, int hy) {
    if constexpr (CORR)
      o[0] = k >= 0 && k < d.nz ? (T)(omega * dinv[k] * (double)raw[0] + coarse_interp<TY, 1>(E, k, 0, hx, hy))
                                : (T)0;
    else
      o[0] = raw[0];
  };
  auto put = [&](const auto& stg, int k) {
    if constexpr (CORR) stage_store_xy<TY>(ring, stg, k, comb_corr);
    else stage_store<TY>(ring, stg, k, comb);
  };
  CoarseRegs<T, 1> cr;
  if constexpr (CORR) {
    coarse_init<TY>(cr, mc, tc.i0, tc.j0);
    coarse_fetch(cr, mc, tc.k0 - 1, d.nz);
    coarse_store<TY>(E, cr, tc.k0 - 1);
    coarse_fetch(cr, mc, tc.k0, d.nz);
    coarse_store<TY>(E, cr, tc.k0);
    coarse_fetch(cr, mc, tc.k0 + 1, d.nz);
    __syncthreads();
  }
  Stage<T, 1, Halo<TY>::NPT> st;
  stage_fetch<TY>(st, d, tc.i0, tc.j0, tc.k0 - 1, fetch);
  put(st, tc.k0 - 1);
  stage_fetch<TY>(st, d, tc.i0, tc.j0, tc.k0, fetch);
  put(st, tc.k0);
  if constexpr (CORR) {
    __syncthreads();
    coarse_store<TY>(E, cr, tc.k0 + 1);
    __syncthreads();
  }
  stage_fetch<TY>(st, d, tc.i0, tc.j0, tc.k0 + 1, fetch);
  T cb = valid ? b[col + d.plane * tc.k0] : (T)0;
  double acc = 0.0;
  for (int k = tc.k0; k < tc.k1; k++) {
    put(st, k + 1);
    if (k + 2 <= tc.k1) {
      stage_fetch<TY>(st, d, tc.i0, tc.j0, k + 2, fetch);
      if constexpr (CORR) coarse_fetch(cr, mc, k + 2, d.nz);
    }
    const T nb = (valid && k + 1 < tc.k1) ? b[col + d.plane * (k + 1)] : (T)0;
    __syncthreads();
    if (valid) {
      const int sm = slot_of(k - 1), s0 = slot_of(k), sp = slot_of(k + 1);
      const T pc = ring[s0][0][ly + 1][lx + 1];
      const T sxy = ring[s0][0][ly + 1][lx] + ring[s0][0][ly + 1][lx + 2] + ring[s0][0][ly][lx + 1] +
                    ring[s0][0][ly + 2][lx + 1];
      const T pdn = ring[sm][0][ly + 1][lx + 1], pup = ring[sp][0][ly + 1][lx + 1];
      T q;
      if (!cf.open) {
        q = c6 * (6 * pc - (sxy + pdn + pup));
      } else {
        const PlaneEps<T> e = plane_eps(d, cf, k);
        q = e.xy * (4 * pc - sxy) + e.up * (pc - pup) + e.dn * (pc - pdn);
      }
      const T r = cb - q;
      T o = (MODE == kMgSweep || CORR) ? pc + (T)(omega * dinv[k]) * r : r;
      if (emask != nullptr && k == d.nzf && emask[col] != 0) o = 0;
      out[col + d.plane * k] = o;
      acc += (double)cb * (double)o;
    }
    // the table of plane k + 2 reuses the buffer of plane k, last read
    // before the barrier above
    if constexpr (CORR)
      if (k + 2 <= tc.k1) coarse_store<TY>(E, cr, k + 2);
    cb = nb;
    __syncthreads();
  }
  if (partials) block_sum_to<kThreads>(acc, partials + (int64_t)tc.lid * pstride + poff);
}

// ---------------------------------------------------------------------------
// Force and time integration (Eq. 7, 19)
// ---------------------------------------------------------------------------
// At every node, with Pp = P + cdt V:
//   F = -L [ dfL/dP(Pp) - G Lap_h Pp - E - h^-3 s . deps0/dP(Pp) ]
//   E = -G_h phi (Dirichlet ghosts), s = C (int N_n eps(u) - int N_n eps0(Pp))
// then, by mode: write F; V = F; (V, P) <- ((V+F)/2, P + dt (V+F)/2);
// P <- P + dt F.  Reads (P, V) and writes (Pn, Vn), distinct buffers.
// Philox4x32-10 counter-based generator (Salmon et al., SC 2011): ten
// rounds of two 32 x 32 -> 64-bit products of counter words 0 and 2, whose
// high halves are mixed with words 1, 3 and the round key; the key moves by
// the two Weyl increments between rounds.
__device__ inline void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3, uint32_t k0,
                                     uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; r++) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Three standard normal variates of node n for one step: one Philox block,
// Box-Muller on words (0, 1) for x, y and on words (2, 3) for z.
__device__ inline void noise_variates(const NoiseSpec& ns, int64_t n, double xi[3]) {
  uint32_t w0 = (uint32_t)n, w1 = (uint32_t)((uint64_t)n >> 32), w2 = ns.step0, w3 = ns.step1;
  philox4x32_10(w0, w1, w2, w3, ns.key0, ns.key1);
  constexpr double kTwoM32 = 2.3283064365386962890625e-10;  // 2^-32
  constexpr double kTwoPi = 6.283185307179586476925286766559;
  const double r0 = sqrt(-2.0 * log(((double)w0 + 1.0) * kTwoM32));
  const double r1 = sqrt(-2.0 * log(((double)w2 + 1.0) * kTwoM32));
  double s0, c0;
  sincos(kTwoPi * ((double)w1 * kTwoM32), &s0, &c0);
  xi[0] = r0 * c0;
  xi[1] = r0 * s0;
  xi[2] = r1 * cos(kTwoPi * ((double)w3 * kTwoM32));
}

__global__ void noise_kernel(NoiseSpec ns, int64_t N, double* __restrict__ xi) {
  int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; n < N; n += stride) {
    double v[3];
    noise_variates(ns, n, v);
    xi[n] = v[0];
    xi[N + n] = v[1];
    xi[2 * N + n] = v[2];
  }
}

// The force is a tile kernel.  Its elastic term needs, at every node, the
// consistent-mass weighted strains w_v = int N_n (eps_v(u) - eps0_v(Pp)) over
// the 27 neighbours.  Those 3D stencils are products of 1D element
// integrals (mass m and int N_n N_m' = g; end rows in z), so they are applied
// in two passes.  Each source plane s is staged in LDS as (eps0(Pp), u) on
// the tile and its halo; every node of the tile reduces it in x and y, and
// pushes the result into the z-sums of the planes s - 1, s, s + 1 of its own
// column, held in registers; plane s - 1 is then complete.  With Voigt order
// (xx, yy, zz, xy, yz, xz) and in-plane rows m, g:
//   M_v = -(m x m) e_v + (g x m) u_x [xx] + (m x g) u_y [yy]
//         + (m x g) u_x + (g x m) u_y [xy] + (m x g) u_z [yz] + (g x m) u_z [xz]
//   Z_zz = (m x m) u_z, Z_yz = (m x m) u_y, Z_xz = (m x m) u_x
//   w_v(t) = sum_dz mz_t(dz) M_v(t + dz) + gz_t(dz) Z_v(t + dz)
// Pp is staged in a two-plane ring for the Laplacian.
constexpr int kEU = 9;  // staged per halo point: e_0..e_5, u_x, u_y, u_z

// At most 168 VGPRs: the 47.5 KB of LDS (FP64) allow three blocks per CU,
// so three waves per SIMD.  NOISE compiles the thermal-noise term.
template <typename T, bool ROT, bool NOISE>
__global__ __launch_bounds__(kThreads, 3) void force_kernel(
    Dims d, TileMap tm, Coefs<T> cf, const FemTables* __restrict__ tb, const T* __restrict__ P,
    const T* __restrict__ V, T cdt, const T* __restrict__ phi, const T* __restrict__ ghost_top,
    const T* __restrict__ u, int mode, NoiseSpec ns, T* __restrict__ Pn, T* __restrict__ Vn, T* __restrict__ Fout) {
  constexpr int TY = kBY;
  using H = Halo<TY>;
  __shared__ T eu[kEU][TY + 2][kHX];
  __shared__ T pc[2][3][TY + 2][kHX];
  const TileCoord tc = tile_coord(d, tm);
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int i = tc.i0 + lx, j = tc.j0 + ly;
  const bool valid = i < d.nx && j < d.ny;
  const int64_t N = d.N, pl = d.plane;
  const int64_t col = valid ? i + (int64_t)d.nx * j : 0;
  const bool hasV = V != nullptr;
  const bool elas = (cf.terms & kElas) != 0;
  // raw values of the next source plane: P, V, u of this thread's halo points
  Stage<T, 9, H::NPT> st;
  auto fetch = [&](int64_t m, int, T* raw) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
      raw[c] = P[c * N + m];
      raw[3 + c] = hasV ? V[c * N + m] : (T)0;
      raw[6 + c] = elas ? u[c * N + m] : (T)0;
    }
  };
  // stage the fetched plane s: Pp into the ring slot s & 1, (e, u) into eu
  auto stage = [&](int s) {
#pragma unroll
    for (int q = 0; q < H::NPT; q++) {
      const int t = tid_flat() + q * kThreads;
      if (t >= H::HP) continue;
      const int hx = t % kHX, hy = t / kHX;
      const T* raw = st.v[q];
      T pp[3];
#pragma unroll
      for (int c = 0; c < 3; c++) pp[c] = raw[c] + cdt * raw[3 + c];
#pragma unroll
      for (int c = 0; c < 3; c++) pc[s & 1][c][hy][hx] = pp[c];
      if (elas) {
        // points outside the grid were fetched as zeros: their e must be zero too
        const int gi = tc.i0 + hx - 1, gj = tc.j0 + hy - 1;
        const bool live = s >= 0 && s < d.nz && gi >= -1 && gi <= d.nx && gj >= -1 && gj <= d.ny;
        T e[6] = {0, 0, 0, 0, 0, 0};
        if (live) eigenstrain<ROT>(cf, pp[0], pp[1], pp[2], e);
#pragma unroll
        for (int v = 0; v < 6; v++) eu[v][hy][hx] = e[v];
#pragma unroll
        for (int c = 0; c < 3; c++) eu[6 + c][hy][hx] = raw[6 + c];
      }
    }
  };
  const T mI[3] = {(T)tb->m1[kInterior][0], (T)tb->m1[kInterior][1], (T)tb->m1[kInterior][2]};
  const T gI[3] = {(T)tb->g1[kInterior][0], (T)tb->g1[kInterior][1], (T)tb->g1[kInterior][2]};
  // in-plane pass of the staged plane at this node: M (6) and Z (zz, yz, xz)
  auto xy_pass = [&](T M[6], T Z[3]) {
#pragma unroll
    for (int v = 0; v < 6; v++) M[v] = 0;
    Z[0] = Z[1] = Z[2] = 0;
    // rows one at a time: unrolled, the 81 LDS loads of a node would all be
    // issued at once and hold ~160 registers
#pragma unroll 1
    for (int dy = -1; dy <= 1; dy++)
#pragma unroll
      for (int dx = -1; dx <= 1; dx++) {
        const int hx = lx + 1 + dx, hy = ly + 1 + dy;
        const T mm = mI[dx + 1] * mI[dy + 1], gm = gI[dx + 1] * mI[dy + 1], mg = mI[dx + 1] * gI[dy + 1];
#pragma unroll
        for (int v = 0; v < 6; v++) M[v] -= mm * eu[v][hy][hx];
        const T ux = eu[6][hy][hx], uy = eu[7][hy][hx], uz = eu[8][hy][hx];
        M[0] += gm * ux;
        M[1] += mg * uy;
        M[3] += mg * ux + gm * uy;
        M[4] += mg * uz;
        M[5] += gm * uz;
        Z[0] += mm * uz;
        Z[1] += mm * uy;
        Z[2] += mm * ux;
      }
  };
  auto zkind = [&](int t) { return t == 0 ? kLow : (t == d.nz - 1 ? kHigh : kInterior); };
  // w (target t) += (or =) the contribution of a source plane at z offset dz
  auto contrib = [&](int t, int dz, const T M[6], const T Z[3], T w[6], bool add) {
    const int zk = zkind(t);
    const T mz = (T)tb->m1[zk][dz + 1], gz = (T)tb->g1[zk][dz + 1];
    T c[6];
#pragma unroll
    for (int v = 0; v < 6; v++) c[v] = mz * M[v];
    c[2] += gz * Z[0];
    c[4] += gz * Z[1];
    c[5] += gz * Z[2];
#pragma unroll
    for (int v = 0; v < 6; v++) w[v] = add ? w[v] + c[v] : c[v];
  };
  T w0[6] = {0, 0, 0, 0, 0, 0}, w1[6] = {0, 0, 0, 0, 0, 0};  // z-sums of planes k and k + 1
  T pdn[3] = {0, 0, 0};                                        // Pp of the plane below, own column
  const int k0 = tc.k0;
  // phi of the own column at plane k - 1 (the bottom boundary value below
  // the grid), carried up the march from the plane's in-plane loads in a
  // per-thread LDS slot (no register is free across the elastic term)
  const bool elec = (cf.terms & kElec) != 0;
  __shared__ T phm[TY][kBX];
  if (valid && elec) phm[ly][lx] = k0 > 0 ? phi[col + pl * (k0 - 1)] : cf.phi_bottom;
  // prologue: sources k0 - 1 (if any) and k0
  if (k0 > 0) {
    stage_fetch<TY>(st, d, tc.i0, tc.j0, k0 - 1, fetch);
    stage(k0 - 1);
    __syncthreads();
    if (valid) {
#pragma unroll
      for (int c = 0; c < 3; c++) pdn[c] = pc[(k0 - 1) & 1][c][ly + 1][lx + 1];
      if (elas) {
        T M[6], Z[3];
        xy_pass(M, Z);
        contrib(k0, -1, M, Z, w0, false);
      }
    }
    __syncthreads();
  }
  stage_fetch<TY>(st, d, tc.i0, tc.j0, k0, fetch);
  stage(k0);
  stage_fetch<TY>(st, d, tc.i0, tc.j0, k0 + 1, fetch);
  __syncthreads();
  if (valid && elas) {
    T M[6], Z[3];
    xy_pass(M, Z);
    contrib(k0, 0, M, Z, w0, true);
    contrib(k0 + 1, -1, M, Z, w1, false);
  }
  __syncthreads();
  for (int k = k0; k < tc.k1; k++) {
    // source k + 1 (zeros above the grid) completes plane k
    stage(k + 1);
    if (k + 2 <= tc.k1) stage_fetch<TY>(st, d, tc.i0, tc.j0, k + 2, fetch);
    __syncthreads();
    if (valid) {
      const int64_t n = col + pl * k;
      const int s0 = k & 1, s1 = (k + 1) & 1;
      T p0[3];
#pragma unroll
      for (int c = 0; c < 3; c++) p0[c] = pc[s0][c][ly + 1][lx + 1];
      T F[3] = {0, 0, 0};
      if (elas) {
        T M[6], Z[3];
        xy_pass(M, Z);
        if (k + 1 < d.nz) contrib(k, 1, M, Z, w0, true);
        T sg[6], g[3];
        cubic_stress<ROT>(cf, w0, sg);
        stress_pull<ROT>(cf, p0, sg, g);
#pragma unroll
        for (int c = 0; c < 3; c++) F[c] -= cf.inv_h3 * g[c];
        // slide: plane k + 1 becomes the one being completed
#pragma unroll
        for (int v = 0; v < 6; v++) w0[v] = w1[v];
        if (k + 1 < d.nz) {
          contrib(k + 1, 0, M, Z, w0, true);
          contrib(k + 2, -1, M, Z, w1, false);
        }
      }
      if (cf.terms & kLandau) {
        T g[3];
        landau_gradient<ROT>(cf, p0, g);
#pragma unroll
        for (int c = 0; c < 3; c++) F[c] += g[c];
      }
      if (cf.terms & kGrad) {
#pragma unroll
        for (int c = 0; c < 3; c++) {
          T lap = pc[s0][c][ly + 1][lx] + pc[s0][c][ly + 1][lx + 2] + pc[s0][c][ly][lx + 1] +
                  pc[s0][c][ly + 2][lx + 1] - 4 * p0[c];
          if (k + 1 < d.nz) lap += pc[s1][c][ly + 1][lx + 1] - p0[c];
          if (k > 0) lap += pdn[c] - p0[c];
          F[c] -= cf.G * cf.inv_h2 * lap;
        }
      }
      if (elec) {
        const T zp = (k + 1 < d.nzp) ? phi[n + pl] : ghost_top[col];
        F[0] += (phi[nbr(d, i, j, k, 1, 0, 0)] - phi[nbr(d, i, j, k, -1, 0, 0)]) * cf.inv_2h;
        F[1] += (phi[nbr(d, i, j, k, 0, 1, 0)] - phi[nbr(d, i, j, k, 0, -1, 0)]) * cf.inv_2h;
        F[2] += (zp - phm[ly][lx]) * cf.inv_2h;
        phm[ly][lx] = phi[n];
      }
#pragma unroll
      for (int c = 0; c < 3; c++) F[c] *= -cf.L;
      if (NOISE && (mode == kPcStep || mode == kEulerStep)) {
        double xi[3];
        noise_variates(ns, n, xi);
#pragma unroll
        for (int c = 0; c < 3; c++) F[c] += (T)(ns.amp * xi[c]);
      }
      switch (mode) {
        case kForceOut:
#pragma unroll
          for (int c = 0; c < 3; c++) Fout[c * N + n] = F[c];
          break;
        case kPcInit:
#pragma unroll
          for (int c = 0; c < 3; c++) Vn[c * N + n] = F[c];
          break;
        case kPcStep:
          // FP64: P + dt V' = Pp + dt (V' - V) with Pp = P + dt V the staged
          // predictor (cdt = dt here), so P is not read again; FP32 reads P
          // again, as the extra rounding of Pp would show in the state
#pragma unroll
          for (int c = 0; c < 3; c++) {
            const T v = V[c * N + n];
            const T vn = (T)0.5 * (v + F[c]);
            Vn[c * N + n] = vn;
            if constexpr (sizeof(T) == sizeof(double)) Pn[c * N + n] = p0[c] + cf.dt * (vn - v);
            else Pn[c * N + n] = P[c * N + n] + cf.dt * vn;
          }
          break;
        default:  // kEulerStep: Pp = P (cdt = 0, no V)
#pragma unroll
          for (int c = 0; c < 3; c++) Pn[c * N + n] = p0[c] + cf.dt * F[c];
          break;
      }
#pragma unroll
      for (int c = 0; c < 3; c++) pdn[c] = p0[c];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Free energy (Eq. 1-6 on the grid), per-block partial sums
// ---------------------------------------------------------------------------
// Energies of the state P (storage S), evaluated in FP64:
//  bulk   h^3 fL(P_n)
//  grad   (G/2) h |P_m - P_n|^2 over the +x, +y, +z edges of n
//  elec   h^3 [ b_n phiP_n - phiP_n (A phiP)_n / 2 ] - h^3 P_n . E_app_n
//         with b = -D_h P, phiP = phi - phi_bc (phi solved at P with the
//         boundary values, phi_bc with P = 0); the first bracket is the
//         stationary value of the quadratic form, (h^3/2) rho^T A^-1 rho,
//         so its error is second order in the solve error
//  elas   u.K u / 2 - u.f + eps0^T C M eps0 / 2 at the solved u (again the
//         quadratic form, min over u of the elastic energy)
template <typename S>
__global__ __launch_bounds__(kThreads) void energy_kernel(Dims d, Coefs<double> cf, const FemTables* __restrict__ tb,
                                                          const S* __restrict__ P, const double* __restrict__ phi,
                                                          const double* __restrict__ phi_bc,
                                                          const double* __restrict__ ghost_top,
                                                          const double* __restrict__ u, double* partials) {
  const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y, k = blockIdx.z;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < d.nx && j < d.ny) {
    const int64_t N = d.N, pl = d.plane;
    const int64_t n = i + (int64_t)d.nx * j + pl * k;
    const double h3 = cf.h * cf.h * cf.h;
    auto Pc = [&](int c, int64_t m) -> double { return (double)P[c * N + m]; };
    const double p[3] = {Pc(0, n), Pc(1, n), Pc(2, n)};
    if (cf.terms & kLandau) v[0] = h3 * landau_density(cf, p);
    if (cf.terms & kGrad) {
      double s = 0.0;
      const int64_t ms[3] = {nbr(d, i, j, k, 1, 0, 0), nbr(d, i, j, k, 0, 1, 0), k + 1 < d.nz ? n + pl : -1};
#pragma unroll
      for (int e = 0; e < 3; e++) {
        if (ms[e] < 0) continue;
#pragma unroll
        for (int c = 0; c < 3; c++) {
          const double df = Pc(c, ms[e]) - p[c];
          s += df * df;
        }
      }
      v[1] = 0.5 * cf.G * cf.h * s;
    }
    if (cf.terms & kElec) {
      // applied part -h^3 P . E_app; the polarisation part is a sum over the
      // potential grid (elec_quad_kernel)
      const int64_t nxp = nbr(d, i, j, k, 1, 0, 0), nxm = nbr(d, i, j, k, -1, 0, 0);
      const int64_t nyp = nbr(d, i, j, k, 0, 1, 0), nym = nbr(d, i, j, k, 0, -1, 0);
      const double zp = k + 1 < d.nzp ? phi_bc[n + pl] : ghost_top[i + (int64_t)d.nx * j];
      const double zm = k > 0 ? phi_bc[n - pl] : cf.phi_bottom;
      const double E[3] = {-(phi_bc[nxp] - phi_bc[nxm]) * cf.inv_2h, -(phi_bc[nyp] - phi_bc[nym]) * cf.inv_2h,
                           -(zp - zm) * cf.inv_2h};
      v[2] = -h3 * (p[0] * E[0] + p[1] * E[1] + p[2] * E[2]);
    }
    if (cf.terms & kElas) {
      // eps0^T C (M eps0) / 2 on every row
      const int zt3 = (k == 0) ? kLow : ((k == d.nz - 1) ? kHigh : kInterior);
      const int dzmin = (k == 0) ? 0 : -1, dzmax = (k == d.nz - 1) ? 0 : 1;
      double me[6] = {0, 0, 0, 0, 0, 0};
      for (int dz = dzmin; dz <= dzmax; dz++)
        for (int dy = -1; dy <= 1; dy++)
          for (int dx = -1; dx <= 1; dx++) {
            const int o = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
            const int64_t m = nbr(d, i, j, k, dx, dy, dz);
            double e[6];
            eigenstrain(cf, Pc(0, m), Pc(1, m), Pc(2, m), e);
            for (int q = 0; q < 6; q++) me[q] += tb->Ms[zt3][o] * e[q];
          }
      double e0[6], cme[6];
      eigenstrain(cf, p[0], p[1], p[2], e0);
      cubic_stress(cf, me, cme);
      double el = 0.0;
      for (int q = 0; q < 6; q++) el += 0.5 * e0[q] * cme[q];
      if (k > 0) {
        const int zt = (k == d.nz - 1) ? 1 : 0;
        double f[3] = {0, 0, 0};
        for (int dz = -1; dz <= (zt ? 0 : 1); dz++)
          for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
              const int o = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
              const int64_t m = nbr(d, i, j, k, dx, dy, dz);
              double e[6], sg[6];
              eigenstrain(cf, Pc(0, m), Pc(1, m), Pc(2, m), e);
              cubic_stress(cf, e, sg);
              for (int c = 0; c < 3; c++)
                for (int q = 0; q < 6; q++) f[c] += tb->Bf[zt][c][q][o] * sg[q];
            }
        auto ld = [&](int dx, int dy, int dz, double uu[3]) {
          const int64_t m = nbr(d, i, j, k, dx, dy, dz);
          for (int c = 0; c < 3; c++) uu[c] = (k + dz == 0) ? 0.0 : u[c * N + m];
        };
        double Ku[3];
        fem_K_apply<double, true>(tb, zt, ld, Ku);
        for (int c = 0; c < 3; c++) el += 0.5 * u[c * N + n] * Ku[c] - u[c * N + n] * f[c];
      }
      v[3] = el;
    }
  }
  block_partials<4, kThreads>(v, partials, node_block_id());
}

// Polarisation part of the electrostatic energy, (h^3/2) f^T A f at the
// stationary point of -rho^T f - f^T A f / 2 (f = phi - phi_bc, the
// potential of P alone): per node of the potential grid h^3 (-rho f - f (A
// f) / 2), whose sum has an error second order in the solve error.
template <typename S>
__global__ __launch_bounds__(kThreads) void elec_quad_kernel(Dims d, Coefs<double> cf, const S* __restrict__ P,
                                                             const double* __restrict__ phi,
                                                             const double* __restrict__ phi_bc,
                                                             const uint8_t* __restrict__ emask, double* partials) {
  const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y, k = blockIdx.z;
  double v[1] = {0.0};
  auto is_el = [&](int kk, int64_t c) { return emask != nullptr && kk == d.nzf && emask[c] != 0; };
  if (i < d.nx && j < d.ny) {
    const int64_t Nf = d.Nf, pl = d.plane;
    const int64_t col = i + (int64_t)d.nx * j, n = col + pl * k;
    if (!is_el(k, col)) {
      const int64_t cxp = wrap(i + 1, d.nx) + (int64_t)d.nx * j, cxm = wrap(i - 1, d.nx) + (int64_t)d.nx * j;
      const int64_t cyp = i + (int64_t)d.nx * wrap(j + 1, d.ny), cym = i + (int64_t)d.nx * wrap(j - 1, d.ny);
      auto Pc = [&](int c, int64_t m) -> double { return (double)P[c * Nf + m]; };
      double rho = 0.0;
      if (k < d.nzf) rho += Pc(0, cxp + pl * k) - Pc(0, cxm + pl * k) + Pc(1, cyp + pl * k) - Pc(1, cym + pl * k);
      if (k + 1 < d.nzf) rho += Pc(2, n + pl);
      if (k > 0 && k - 1 < d.nzf) rho -= Pc(2, n - pl);
      rho *= cf.inv_2h;
      auto f = [&](int kk, int64_t c) -> double {
        const int64_t m = c + pl * kk;
        return is_el(kk, c) ? 0.0 : phi[m] - phi_bc[m];
      };
      const double f0 = f(k, col);
      const double sxy = f(k, cxp) + f(k, cxm) + f(k, cyp) + f(k, cym);
      const double fup = k + 1 < d.nz ? f(k + 1, col) : 0.0, fdn = k > 0 ? f(k - 1, col) : 0.0;
      const PlaneEps<double> e = plane_eps(d, cf, k);
      const double Af = e.xy * (4 * f0 - sxy) + e.up * (f0 - fup) + e.dn * (f0 - fdn);
      const double h3 = cf.h * cf.h * cf.h;
      v[0] = h3 * (-rho * f0 - 0.5 * f0 * Af);
    }
  }
  block_partials<1, kThreads>(v, partials, node_block_id());
}

// ---------------------------------------------------------------------------
// Linearised force and the adjoint step
// ---------------------------------------------------------------------------
// H w = (dF/dP)(X) w at the linearisation point X = P + cdt V, with u the
// displacement solved at X, psi the adjoint potential (A psi = -D_h w, zero
// boundary values) and du the adjoint displacement (K du = f(deps0),
// deps0 = (d eps0/dP)(X) w):
//   H w = -L [ Hess fL(X) w - G Lap_h w - E(psi) - h^-3 (ds . deps0/dP(X)
//              + s . d2eps0/dP2 w) ],  E(psi) = -G_h psi,
//   s = C (int N eps(u) - int N eps0(X)),  ds = C (int N eps(du) - int N deps0).
template <typename S>
__global__ __launch_bounds__(kThreads) void hvp_kernel(Dims d, Coefs<double> cf, const FemTables* __restrict__ tb,
                                                       const S* __restrict__ P, const S* __restrict__ V, double cdt,
                                                       const double* __restrict__ w, const double* __restrict__ u,
                                                       const double* __restrict__ psi, const double* __restrict__ du,
                                                       double* __restrict__ Hw) {
  const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y, k = blockIdx.z;
  if (i >= d.nx || j >= d.ny) return;
  const int64_t N = d.N, pl = d.plane;
  const int64_t n = i + (int64_t)d.nx * j + pl * k;
  auto X = [&](int64_t m, double out[3]) {
    for (int c = 0; c < 3; c++) out[c] = (double)P[c * N + m] + (V ? cdt * (double)V[c * N + m] : 0.0);
  };
  double x0[3], w0[3] = {w[n], w[N + n], w[2 * N + n]};
  X(n, x0);
  double acc[3] = {0, 0, 0};
  if (cf.terms & kLandau) {
    double hl[3];
    landau_hessian_apply(cf, x0, w0, hl);
    for (int c = 0; c < 3; c++) acc[c] += hl[c];
  }
  if (cf.terms & kGrad) {
    const int64_t ms[6] = {nbr(d, i, j, k, 1, 0, 0), nbr(d, i, j, k, -1, 0, 0), nbr(d, i, j, k, 0, 1, 0),
                           nbr(d, i, j, k, 0, -1, 0), k + 1 < d.nz ? n + pl : -1, k > 0 ? n - pl : -1};
    for (int c = 0; c < 3; c++) {
      double lap = 0.0;
      for (int t = 0; t < 6; t++)
        if (ms[t] >= 0) lap += w[c * N + ms[t]] - w0[c];
      acc[c] -= cf.G * cf.inv_h2 * lap;
    }
  }
  if (cf.terms & kElec) {
    const double zp = (k + 1 < d.nzp) ? psi[n + pl] : 0.0;
    const double zm = (k > 0) ? psi[n - pl] : 0.0;
    acc[0] += (psi[nbr(d, i, j, k, 1, 0, 0)] - psi[nbr(d, i, j, k, -1, 0, 0)]) * cf.inv_2h;
    acc[1] += (psi[nbr(d, i, j, k, 0, 1, 0)] - psi[nbr(d, i, j, k, 0, -1, 0)]) * cf.inv_2h;
    acc[2] += (zp - zm) * cf.inv_2h;
  }
  if (cf.terms & kElas) {
    const int zt = (k == 0) ? kLow : ((k == d.nz - 1) ? kHigh : kInterior);
    const int dzmin = (k == 0) ? 0 : -1, dzmax = (k == d.nz - 1) ? 0 : 1;
    double ws_[6] = {0, 0, 0, 0, 0, 0}, wd[6] = {0, 0, 0, 0, 0, 0};
    for (int dz = dzmin; dz <= dzmax; dz++)
      for (int dy = -1; dy <= 1; dy++)
        for (int dx = -1; dx <= 1; dx++) {
          const int o = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
          const int64_t m = nbr(d, i, j, k, dx, dy, dz);
          double a[3], e[6], de[6];
          X(m, a);
          eigenstrain(cf, a[0], a[1], a[2], e);
          eigenstrain_lin(cf, a[0], a[1], a[2], w[m], w[N + m], w[2 * N + m], de);
          const double ms = tb->Ms[zt][o];
          for (int q = 0; q < 6; q++) {
            double s1 = -ms * e[q], s2 = -ms * de[q];
            for (int c = 0; c < 3; c++) {
              s1 += tb->Su[zt][q][c][o] * u[c * N + m];
              s2 += tb->Su[zt][q][c][o] * du[c * N + m];
            }
            ws_[q] += s1;
            wd[q] += s2;
          }
        }
    double s[6], ds[6], g[3], hs[3];
    cubic_stress(cf, ws_, s);
    cubic_stress(cf, wd, ds);
    stress_pull(cf, x0, ds, g);
    stress_pull(cf, w0, s, hs);  // s . d2eps0/dP2 w (eps0 is quadratic in P)
    for (int c = 0; c < 3; c++) acc[c] -= cf.inv_h3 * (g[c] + hs[c]);
  }
  for (int c = 0; c < 3; c++) Hw[c * N + n] = -cf.L * acc[c];
}

// Adjoint bookkeeping (lam in state storage S, w and Hw in FP64):
//   kAdjPrepPc    w = (lamV + dt lamP) / 2
//   kAdjPrepEuler w = lamP
//   kAdjPrepInit  w = lamV
//   kAdjUpdPc     lamP += Hw, lamV = w + dt Hw
//   kAdjUpdEuler  lamP += dt Hw
//   kAdjUpdInit   lamP += Hw, lamV = 0
enum { kAdjPrepPc = 0, kAdjPrepEuler, kAdjPrepInit, kAdjUpdPc, kAdjUpdEuler, kAdjUpdInit };

template <typename S>
__global__ void adjoint_axpy_kernel(int mode, double dt, S* lamP, S* lamV, double* w, const double* Hw, int64_t n) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; t < n; t += stride) {
    switch (mode) {
      case kAdjPrepPc: w[t] = 0.5 * ((double)lamV[t] + dt * (double)lamP[t]); break;
      case kAdjPrepEuler: w[t] = (double)lamP[t]; break;
      case kAdjPrepInit: w[t] = (double)lamV[t]; break;
      case kAdjUpdPc:
        lamP[t] = (S)((double)lamP[t] + Hw[t]);
        lamV[t] = (S)(w[t] + dt * Hw[t]);
        break;
      case kAdjUpdEuler: lamP[t] = (S)((double)lamP[t] + dt * Hw[t]); break;
      default:
        lamP[t] = (S)((double)lamP[t] + Hw[t]);
        lamV[t] = (S)0;
        break;
    }
  }
}

// Partials of w . dF/dtheta:  electrode e (rectangle [x0,x1) x [y0,y1), unit
// voltage, basis potential phi_e): L w . E^(e), E^(e) = -G_h phi_e with the
// unit ghost values; a1 (phi_e null): -2 L w . X.
template <typename S>
__global__ __launch_bounds__(kThreads) void theta_dot_kernel(Dims d, Coefs<double> cf, const double* __restrict__ w,
                                                             const double* __restrict__ phi_e, int x0, int x1, int y0,
                                                             int y1, const S* __restrict__ P,
                                                             const S* __restrict__ V, double cdt, double* partials) {
  const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y, k = blockIdx.z;
  double v[1] = {0.0};
  if (i < d.nx && j < d.ny) {
    const int64_t N = d.N, pl = d.plane;
    const int64_t n = i + (int64_t)d.nx * j + pl * k;
    if (phi_e) {
      const double ghost = (i >= x0 && i < x1 && j >= y0 && j < y1) ? 1.0 : 0.0;
      const double zp = (k + 1 < d.nzp) ? phi_e[n + pl] : ghost;
      const double zm = (k > 0) ? phi_e[n - pl] : 0.0;
      const double E0 = -(phi_e[nbr(d, i, j, k, 1, 0, 0)] - phi_e[nbr(d, i, j, k, -1, 0, 0)]) * cf.inv_2h;
      const double E1 = -(phi_e[nbr(d, i, j, k, 0, 1, 0)] - phi_e[nbr(d, i, j, k, 0, -1, 0)]) * cf.inv_2h;
      const double E2 = -(zp - zm) * cf.inv_2h;
      v[0] = cf.L * (w[n] * E0 + w[N + n] * E1 + w[2 * N + n] * E2);
    } else {
      double s = 0.0;
      for (int c = 0; c < 3; c++)
        s += w[c * N + n] * ((double)P[c * N + n] + (V ? cdt * (double)V[c * N + n] : 0.0));
      v[0] = -2.0 * cf.L * s;
    }
  }
  block_partials<1, kThreads>(v, partials, node_block_id());
}

// ---------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------

namespace {
inline dim3 node_grid(const Dims& d) { return dim3((d.nx + kBX - 1) / kBX, (d.ny + kBY - 1) / kBY, d.nz); }
inline dim3 node_block() { return dim3(kBX, kBY, 1); }
inline int flat_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (int)(b > 65536 ? 65536 : (b < 1 ? 1 : b));
}
}  // namespace

int node_blocks(const Dims& d) {
  dim3 g = node_grid(d);
  return (int)(g.x * g.y * g.z);
}

// Tile map for tiles of 64 x ty nodes: the z-chunk length is chosen so that
// the grid has about `target` blocks (the number that stays resident on the
// chip at once), chunks of at least 4 planes.  PF_TILE_KZ overrides the
// chunk length (a tuning knob; results do not depend on it beyond rounding
// order).
TileMap make_tile_map(const Dims& d, int ty, int target) {
  TileMap t;
  t.ty = ty;
  t.ntx = (d.nx + kBX - 1) / kBX;
  t.nty = (d.ny + ty - 1) / ty;
  const int64_t cols = (int64_t)t.ntx * t.nty;
  int64_t kz = ((int64_t)d.nz * cols + target - 1) / target;
  if (kz < 4) kz = 4;
  if (const char* env = getenv("PF_TILE_KZ")) {
    const long v = strtol(env, nullptr, 10);
    if (v >= 1 && v <= 4096) kz = v;
  }
  if (kz > d.nz) kz = d.nz;
  t.kz = (int)kz;
  t.nkz = (d.nz + t.kz - 1) / t.kz;
  t.nblocks = (int)(cols * t.nkz);
  int gy = 4;
  if (const char* env = getenv("PF_TILE_GY")) {
    const long v = strtol(env, nullptr, 10);
    if (v >= 1 && v <= 64) gy = (int)v;
  }
  t.gy = gy < t.nty ? gy : t.nty;
  return t;
}

template <typename T>
hipError_t launch_fill(T* a, int64_t n, T v, hipStream_t s) {
  fill_kernel<T><<<flat_blocks(n), 256, 0, s>>>(a, n, v);
  return hipGetLastError();
}

template <typename T, typename U>
hipError_t launch_convert(const T* a, U* b, int64_t n, hipStream_t s) {
  convert_kernel<T, U><<<flat_blocks(n), 256, 0, s>>>(a, b, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cg_finish(T* x, const T* p, int64_t n, const CgScalars* sc, hipStream_t s) {
  cg_finish_kernel<T><<<flat_blocks(n), 256, 0, s>>>(x, p, n, sc);
  return hipGetLastError();
}

hipError_t launch_cg_reduce(const double* partials, int nblocks, int nv, CgScalars* sc, int mode, double tol,
                            int maxit, hipStream_t s, double tol2, double* out) {
  switch (nv) {
    case 1: cg_reduce_kernel<1><<<1, kRedThreads, 0, s>>>(partials, nblocks, sc, mode, tol, maxit, tol2, out); break;
    case 2: cg_reduce_kernel<2><<<1, kRedThreads, 0, s>>>(partials, nblocks, sc, mode, tol, maxit, tol2, out); break;
    case 3: cg_reduce_kernel<3><<<1, kRedThreads, 0, s>>>(partials, nblocks, sc, mode, tol, maxit, tol2, out); break;
    default: cg_reduce_kernel<4><<<1, kRedThreads, 0, s>>>(partials, nblocks, sc, mode, tol, maxit, tol2, out); break;
  }
  return hipGetLastError();
}

hipError_t launch_extrapolate(double* x, const ExtrapRing& ring, int64_t n, hipStream_t s) {
  const int nb = flat_blocks(n);
  switch (ring.m) {
    case 0: extrapolate_kernel<0><<<nb, 256, 0, s>>>(x, ring, n); break;
    case 1: extrapolate_kernel<1><<<nb, 256, 0, s>>>(x, ring, n); break;
    case 2: extrapolate_kernel<2><<<nb, 256, 0, s>>>(x, ring, n); break;
    case 3: extrapolate_kernel<3><<<nb, 256, 0, s>>>(x, ring, n); break;
    case 4: extrapolate_kernel<4><<<nb, 256, 0, s>>>(x, ring, n); break;
    case 5: extrapolate_kernel<5><<<nb, 256, 0, s>>>(x, ring, n); break;
    case 6: extrapolate_kernel<6><<<nb, 256, 0, s>>>(x, ring, n); break;
    case 7: extrapolate_kernel<7><<<nb, 256, 0, s>>>(x, ring, n); break;
    case 8: extrapolate_kernel<8><<<nb, 256, 0, s>>>(x, ring, n); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_extrap_score(const double* x, const ExtrapRing& ring, const ExtrapScore& sc, int64_t n,
                               hipStream_t s) {
  if (sc.mmax < 0 || sc.mmax > kMaxExtrap || sc.mmax >= ring.nh) return hipErrorInvalidValue;
  extrap_score_kernel<<<kScoreBlocks, 256, 0, s>>>(x, ring, sc, n);
  return hipGetLastError();
}

hipError_t launch_noise(const NoiseSpec& ns, int64_t N, double* xi, hipStream_t s) {
  noise_kernel<<<flat_blocks(N), 256, 0, s>>>(ns, N, xi);
  return hipGetLastError();
}

hipError_t launch_refine_update(double* x64, float* x32, const float* d, const float* p, const CgScalars* sc,
                                int64_t n, hipStream_t s) {
  refine_update_kernel<<<flat_blocks(n), 256, 0, s>>>(x64, x32, d, p, sc, n);
  return hipGetLastError();
}

template <typename T, typename S, typename R>
hipError_t launch_poisson_setup(const Dims& d, const TileMap& tm, const Coefs<T>& cf, const S* P, const S* V, T cdt,
                                int with_P, int with_bc, const T* ghost_top, T phi_bottom, const uint8_t* emask,
                                T* x, R* r, R* p, R* dz, double* partials, hipStream_t s) {
  poisson_setup_kernel<T, S, R><<<tm.nblocks, node_block(), 0, s>>>(d, tm, cf, P, V, cdt, with_P, with_bc, ghost_top,
                                                                    phi_bottom, emask, x, r, p, dz, partials);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_poisson_cg_a(const Dims& d, const TileMap& tm, const Coefs<T>& cf, const T* r, const T* p_old,
                               T* p_new, T* x, const CgScalars* sc, double* partials, int unit_w, hipStream_t s) {
  poisson_cg_a_kernel<T><<<tm.nblocks, node_block(), 0, s>>>(d, tm, cf, r, p_old, p_new, x, sc, partials, unit_w);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_poisson_cg_b(const Dims& d, const TileMap& tm, const Coefs<T>& cf, const T* p, T* r,
                               const uint8_t* emask, const CgScalars* sc, double* partials, hipStream_t s) {
  poisson_cg_b_kernel<T><<<tm.nblocks, node_block(), 0, s>>>(d, tm, cf, p, r, emask, sc, partials);
  return hipGetLastError();
}

template <typename T, typename S, typename R>
hipError_t launch_fem_setup(const Dims& d, const TileMap& tm, const Coefs<T>& cf, const FemTables* tb, bool gen,
                            const S* P, const S* V, T cdt, const T* W, T* x, R* r, R* p0, R* p1, R* dz,
                            T* fout, double* partials, hipStream_t s) {
#define PF_FEM_SETUP(GEN, ROT)                                                                               \
  fem_setup_kernel<T, S, R, GEN, ROT><<<tm.nblocks, node_block(), 0, s>>>(d, tm, cf, tb, P, V, cdt, W, x, r, p0, p1, \
                                                                          dz, fout, partials)
  if (gen) {
    if (cf.rotated) PF_FEM_SETUP(true, true);
    else PF_FEM_SETUP(true, false);
  } else {
    if (cf.rotated) PF_FEM_SETUP(false, true);
    else PF_FEM_SETUP(false, false);
  }
#undef PF_FEM_SETUP
  return hipGetLastError();
}

template <typename T, typename R>
hipError_t launch_fem_resid(const Dims& d, const TileMap& tm, const FemTables* tb, bool gen, const T* f, T* x, R* r,
                            R* p0, R* p1, R* dz, double* partials, hipStream_t s) {
  if (gen)
    fem_resid_kernel<T, R, true><<<tm.nblocks, node_block(), 0, s>>>(d, tm, tb, f, x, r, p0, p1, dz, partials);
  else
    fem_resid_kernel<T, R, false><<<tm.nblocks, node_block(), 0, s>>>(d, tm, tb, f, x, r, p0, p1, dz, partials);
  return hipGetLastError();
}

// gen: the stiffness has no cubic structure on the grid axes (rotated
// crystal), so no tap of the coupling blocks can be skipped.
template <typename T>
hipError_t launch_fem_cg_a(const Dims& d, const TileMap& tm, const FemTables* tb, bool gen, const T* r,
                           const T* p_old, T* p_new, T* x, const CgScalars* sc, double* partials, int unit_w,
                           hipStream_t s) {
  if (gen)
    fem_cg_a_kernel<T, true><<<tm.nblocks, node_block(), 0, s>>>(d, tm, tb, r, p_old, p_new, x, sc, partials, unit_w);
  else
    fem_cg_a_kernel<T, false><<<tm.nblocks, node_block(), 0, s>>>(d, tm, tb, r, p_old, p_new, x, sc, partials,
                                                                 unit_w);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fem_cg_b(const Dims& d, const TileMap& tm, const FemTables* tb, bool gen, const T* p, T* r,
                           const CgScalars* sc, double* partials, hipStream_t s) {
  if (gen) fem_cg_b_kernel<T, true><<<tm.nblocks, node_block(), 0, s>>>(d, tm, tb, p, r, sc, partials);
  else fem_cg_b_kernel<T, false><<<tm.nblocks, node_block(), 0, s>>>(d, tm, tb, p, r, sc, partials);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mg_fine(const Dims& d, const TileMap& tm, const FemTables* tb, bool gen, const double* dinv, int mode,
                          double omega, const T* x, const T* b, T* out, const MgCoarse<T>& mc, const CgScalars* sc,
                          double* partials, int pstride, int poff, hipStream_t s) {
  if (mode == kMgCorrect && (tm.ty % 2 != 0 || d.nx != 2 * mc.nx || d.ny != 2 * mc.ny)) return hipErrorInvalidValue;
#define PF_MG_FINE(GEN, MODE)                                                                                  \
  mg_fine_kernel<T, GEN, MODE><<<tm.nblocks, node_block(), 0, s>>>(d, tm, tb, dinv, omega, x, b, out, sc, partials, \
                                                                   pstride, poff)
#define PF_MG_CORRECT(GEN)                                                                                    \
  mg_correct_kernel<T, GEN><<<tm.nblocks, node_block(), 0, s>>>(d, tm, tb, dinv, omega, b, out, mc, sc, partials, \
                                                                pstride, poff)
#define PF_MG_FINE_MODES(GEN)                              \
  switch (mode) {                                          \
    case kMgSweep: PF_MG_FINE(GEN, kMgSweep); break;       \
    case kMgFirst: PF_MG_FINE(GEN, kMgFirst); break;       \
    case kMgCorrect: PF_MG_CORRECT(GEN); break;            \
    default: return hipErrorInvalidValue;                  \
  }
  if (gen) {
    PF_MG_FINE_MODES(true)
  } else {
    PF_MG_FINE_MODES(false)
  }
#undef PF_MG_FINE_MODES
#undef PF_MG_CORRECT
#undef PF_MG_FINE
  return hipGetLastError();
}

// The three-component stencils are staged in LDS (the Poisson stencil fits
// the scalar registers).
template <typename T>
hipError_t launch_mg_level(const Dims& d, int nc, const double* tab, const double* dinv, int mode, double omega,
                           const T* x, const T* b, T* out, const CgScalars* sc, int top_fixed, hipStream_t s) {
  // the largest levels march z with each plane staged once; mid-size FP64
  // levels stage a tile's neighbourhood per plane (more blocks in flight);
  // on small ones the node kernel's parallelism wins
  if (d.N >= kMgMarchMinNodes) {
    const TileMap tm = make_tile_map(d, kBY, 4096);
    if (nc == 3)
      mg_level_zm_kernel<T, 3><<<tm.nblocks, node_block(), 0, s>>>(d, tm, tab, dinv, mode, omega, x, b, out, sc,
                                                                  top_fixed);
    else
      mg_level_zm_kernel<T, 1><<<tm.nblocks, node_block(), 0, s>>>(d, tm, tab, dinv, mode, omega, x, b, out, sc,
                                                                  top_fixed);
    return hipGetLastError();
  }
  const bool tile = sizeof(T) == 8 && d.N >= kMgTileMinNodes;
  if (nc == 3) {
    if (tile)
      mg_level_tile_kernel<T, 3><<<node_grid(d), node_block(), 0, s>>>(d, tab, dinv, mode, omega, x, b, out, sc,
                                                                      top_fixed);
    else
      mg_level_kernel<T, 3, true><<<node_grid(d), node_block(), 0, s>>>(d, tab, dinv, mode, omega, x, b, out, sc,
                                                                       top_fixed);
  } else {
    if (tile)
      mg_level_tile_kernel<T, 1><<<node_grid(d), node_block(), 0, s>>>(d, tab, dinv, mode, omega, x, b, out, sc,
                                                                      top_fixed);
    else
      mg_level_kernel<T, 1, false><<<node_grid(d), node_block(), 0, s>>>(d, tab, dinv, mode, omega, x, b, out, sc,
                                                                        top_fixed);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mg_scale(const Dims& d, int nc, const double* dinv, double omega, const T* b, T* x,
                           const CgScalars* sc, hipStream_t s) {
  if (nc == 3) mg_scale_kernel<T, 3><<<node_grid(d), node_block(), 0, s>>>(d, dinv, omega, b, x, sc);
  else mg_scale_kernel<T, 1><<<node_grid(d), node_block(), 0, s>>>(d, dinv, omega, b, x, sc);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mg_restrict(const Dims& df, const Dims& dc, int nc, int cx, int cy, const MgZ* zmap,
                              const int* zfine, const T* rf, T* bc, const CgScalars* sc, int zoff, int fnz,
                              int ftop_fixed, int ctop_fixed, hipStream_t s) {
  if (cx && cy && df.nx == 2 * dc.nx && df.ny == 2 * dc.ny) {
    const bool wide = dc.plane >= 16384;
    const int kc = wide ? 4 : 1;
    const dim3 g((dc.nx + kBX - 1) / kBX, (dc.ny + kBY - 1) / kBY, (dc.nz + kc - 1) / kc);
#define PF_RESTRICT2(NC, KC) \
  mg_restrict2_kernel<T, NC, KC><<<g, node_block(), 0, s>>>(df, dc, zmap, zfine, rf, bc, sc, zoff, fnz, ftop_fixed, \
                                                            ctop_fixed)
    if (nc == 3) {
      if (wide) PF_RESTRICT2(3, 4);
      else PF_RESTRICT2(3, 1);
    } else {
      if (wide) PF_RESTRICT2(1, 4);
      else PF_RESTRICT2(1, 1);
    }
#undef PF_RESTRICT2
    return hipGetLastError();
  }
  if (nc == 3)
    mg_restrict_kernel<T, 3><<<node_grid(dc), node_block(), 0, s>>>(df, dc, cx, cy, zmap, zfine, rf, bc, sc, zoff,
                                                                     fnz, ftop_fixed, ctop_fixed);
  else
    mg_restrict_kernel<T, 1><<<node_grid(dc), node_block(), 0, s>>>(df, dc, cx, cy, zmap, zfine, rf, bc, sc, zoff,
                                                                     fnz, ftop_fixed, ctop_fixed);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mg_prolong(const Dims& df, const Dims& dc, int nc, int cx, int cy, const MgZ* zmap, const T* xc,
                             T* xf, const CgScalars* sc, int zoff, int ftop_fixed, int ctop_fixed, const T* bf,
                             const double* dinv, double omega, hipStream_t s) {
  if (cx && cy && df.nx == 2 * dc.nx && df.ny == 2 * dc.ny && dc.plane >= 16384) {
    const dim3 g((dc.nx + kBX - 1) / kBX, (dc.ny + kBY - 1) / kBY, df.nz);
    if (nc == 3)
      mg_prolong2_kernel<T, 3><<<g, node_block(), 0, s>>>(df, dc, zmap, xc, xf, sc, zoff, ftop_fixed, ctop_fixed, bf,
                                                          dinv, omega);
    else
      mg_prolong2_kernel<T, 1><<<g, node_block(), 0, s>>>(df, dc, zmap, xc, xf, sc, zoff, ftop_fixed, ctop_fixed, bf,
                                                          dinv, omega);
    return hipGetLastError();
  }
  if (nc == 3)
    mg_prolong_kernel<T, 3><<<node_grid(df), node_block(), 0, s>>>(df, dc, cx, cy, zmap, xc, xf, sc, zoff, ftop_fixed,
                                                                    ctop_fixed, bf, dinv, omega);
  else
    mg_prolong_kernel<T, 1><<<node_grid(df), node_block(), 0, s>>>(df, dc, cx, cy, zmap, xc, xf, sc, zoff, ftop_fixed,
                                                                    ctop_fixed, bf, dinv, omega);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mg_dense(const Dims& d, int nc, int n, const double* M, const T* b, T* x, const CgScalars* sc,
                           hipStream_t s) {
  if (nc == 3) mg_dense_kernel<T, 3><<<n, 256, 0, s>>>(d, n, M, b, x, sc);
  else mg_dense_kernel<T, 1><<<n, 256, 0, s>>>(d, n, M, b, x, sc);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mgp_fine(const Dims& d, const TileMap& tm, const Coefs<T>& cf, const double* dinv, int mode,
                           double omega, const T* x, const T* b, T* out, const MgCoarse<T>& mc,
                           const uint8_t* emask, const CgScalars* sc, double* partials, int pstride, int poff,
                           hipStream_t s) {
  if (mode == kMgCorrect && (tm.ty % 2 != 0 || d.nx != 2 * mc.nx || d.ny != 2 * mc.ny)) return hipErrorInvalidValue;
#define PF_MGP_FINE(MODE)                                                                                          \
  mgp_fine_kernel<T, MODE><<<tm.nblocks, node_block(), 0, s>>>(d, tm, cf, dinv, omega, x, b, out, mc, emask, sc, \
                                                               partials, pstride, poff)
  switch (mode) {
    case kMgSweep: PF_MGP_FINE(kMgSweep); break;
    case kMgFirst: PF_MGP_FINE(kMgFirst); break;
    case kMgCorrect: PF_MGP_FINE(kMgCorrect); break;
    default: return hipErrorInvalidValue;
  }
#undef PF_MGP_FINE
  return hipGetLastError();
}

template <typename T>
hipError_t launch_force(const Dims& d, const TileMap& tm, const Coefs<T>& cf, const FemTables* tb, const T* P,
                        const T* V, T cdt, const T* phi, const T* ghost_top, const T* u, int mode,
                        const NoiseSpec& ns, T* Pn, T* Vn, T* Fout, hipStream_t s) {
  const bool noise = ns.amp != 0.0;
#define PF_FORCE(ROT, NOISE)                                                                                  \
  force_kernel<T, ROT, NOISE><<<tm.nblocks, node_block(), 0, s>>>(d, tm, cf, tb, P, V, cdt, phi, ghost_top, u, \
                                                                  mode, ns, Pn, Vn, Fout)
  if (cf.rotated) {
    if (noise) PF_FORCE(true, true);
    else PF_FORCE(true, false);
  } else {
    if (noise) PF_FORCE(false, true);
    else PF_FORCE(false, false);
  }
#undef PF_FORCE
  return hipGetLastError();
}

template <typename S>
hipError_t launch_energy(const Dims& d, const Coefs<double>& cf, const FemTables* tb, const S* P, const double* phi,
                         const double* phi_bc, const double* ghost_top, const double* u, double* partials,
                         hipStream_t s) {
  energy_kernel<S><<<node_grid(d), node_block(), 0, s>>>(d, cf, tb, P, phi, phi_bc, ghost_top, u, partials);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_elec_quad(const Dims& dp, const Coefs<double>& cf, const S* P, const double* phi,
                            const double* phi_bc, const uint8_t* emask, double* partials, hipStream_t s) {
  elec_quad_kernel<S><<<node_grid(dp), node_block(), 0, s>>>(dp, cf, P, phi, phi_bc, emask, partials);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_hvp(const Dims& d, const Coefs<double>& cf, const FemTables* tb, const S* P, const S* V,
                      double cdt, const double* w, const double* u, const double* psi, const double* du, double* Hw,
                      hipStream_t s) {
  hvp_kernel<S><<<node_grid(d), node_block(), 0, s>>>(d, cf, tb, P, V, cdt, w, u, psi, du, Hw);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_adjoint_axpy(int mode, double dt, S* lamP, S* lamV, double* w, const double* Hw, int64_t n,
                               hipStream_t s) {
  adjoint_axpy_kernel<S><<<flat_blocks(n), 256, 0, s>>>(mode, dt, lamP, lamV, w, Hw, n);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_theta_dot(const Dims& d, const Coefs<double>& cf, const double* w, const double* phi_e, int x0,
                            int x1, int y0, int y1, const S* P, const S* V, double cdt, double* partials,
                            hipStream_t s) {
  theta_dot_kernel<S><<<node_grid(d), node_block(), 0, s>>>(d, cf, w, phi_e, x0, x1, y0, y1, P, V, cdt, partials);
  return hipGetLastError();
}

#define PF_INSTANTIATE_ADJ(S)                                                                                    \
  template hipError_t launch_elec_quad<S>(const Dims&, const Coefs<double>&, const S*, const double*,            \
                                          const double*, const uint8_t*, double*, hipStream_t);                  \
  template hipError_t launch_energy<S>(const Dims&, const Coefs<double>&, const FemTables*, const S*,            \
                                       const double*, const double*, const double*, const double*, double*,      \
                                       hipStream_t);                                                             \
  template hipError_t launch_hvp<S>(const Dims&, const Coefs<double>&, const FemTables*, const S*, const S*,     \
                                    double, const double*, const double*, const double*, const double*, double*, \
                                    hipStream_t);                                                                \
  template hipError_t launch_adjoint_axpy<S>(int, double, S*, S*, double*, const double*, int64_t, hipStream_t); \
  template hipError_t launch_theta_dot<S>(const Dims&, const Coefs<double>&, const double*, const double*, int,  \
                                          int, int, int, const S*, const S*, double, double*, hipStream_t);

PF_INSTANTIATE_ADJ(double)
PF_INSTANTIATE_ADJ(float)

#define PF_INSTANTIATE(T)                                                                                        \
  template hipError_t launch_fill<T>(T*, int64_t, T, hipStream_t);                                               \
  template hipError_t launch_cg_finish<T>(T*, const T*, int64_t, const CgScalars*, hipStream_t);                 \
  template hipError_t launch_poisson_cg_a<T>(const Dims&, const TileMap&, const Coefs<T>&, const T*, const T*,   \
                                             T*, T*, const CgScalars*, double*, int, hipStream_t);               \
  template hipError_t launch_poisson_cg_b<T>(const Dims&, const TileMap&, const Coefs<T>&, const T*, T*,         \
                                             const uint8_t*, const CgScalars*, double*, hipStream_t);            \
  template hipError_t launch_fem_cg_a<T>(const Dims&, const TileMap&, const FemTables*, bool, const T*, const T*, \
                                         T*, T*, const CgScalars*, double*, int, hipStream_t);                   \
  template hipError_t launch_fem_cg_b<T>(const Dims&, const TileMap&, const FemTables*, bool, const T*, T*,      \
                                         const CgScalars*, double*, hipStream_t);                                \
  template hipError_t launch_force<T>(const Dims&, const TileMap&, const Coefs<T>&, const FemTables*, const T*,  \
                                      const T*, T, const T*, const T*, const T*, int, const NoiseSpec&, T*, T*, T*, \
                                      hipStream_t);

PF_INSTANTIATE(double)
PF_INSTANTIATE(float)

#define PF_INSTANTIATE_MG(T)                                                                                     \
  template hipError_t launch_mg_fine<T>(const Dims&, const TileMap&, const FemTables*, bool, const double*, int,  \
                                        double, const T*, const T*, T*, const MgCoarse<T>&, const CgScalars*,     \
                                        double*, int, int, hipStream_t);                                          \
  template hipError_t launch_mg_level<T>(const Dims&, int, const double*, const double*, int, double, const T*,   \
                                         const T*, T*, const CgScalars*, int, hipStream_t);                       \
  template hipError_t launch_mg_scale<T>(const Dims&, int, const double*, double, const T*, T*, const CgScalars*, \
                                         hipStream_t);                                                            \
  template hipError_t launch_mg_restrict<T>(const Dims&, const Dims&, int, int, int, const MgZ*, const int*,      \
                                            const T*, T*, const CgScalars*, int, int, int, int, hipStream_t);     \
  template hipError_t launch_mg_prolong<T>(const Dims&, const Dims&, int, int, int, const MgZ*, const T*, T*,     \
                                           const CgScalars*, int, int, int, const T*, const double*, double,      \
                                           hipStream_t);                                                          \
  template hipError_t launch_mg_dense<T>(const Dims&, int, int, const double*, const T*, T*, const CgScalars*,    \
                                         hipStream_t);                                                            \
  template hipError_t launch_mgp_fine<T>(const Dims&, const TileMap&, const Coefs<T>&, const double*, int,        \
                                         double, const T*, const T*, T*, const MgCoarse<T>&, const uint8_t*,      \
                                         const CgScalars*, double*, int, int, hipStream_t);

PF_INSTANTIATE_MG(double)
PF_INSTANTIATE_MG(float)

#define PF_INSTANTIATE_SETUP(T, S, R)                                                                            \
  template hipError_t launch_poisson_setup<T, S, R>(const Dims&, const TileMap&, const Coefs<T>&, const S*,      \
                                                    const S*, T, int, int, const T*, T, const uint8_t*, T*, R*,  \
                                                    R*, R*, double*, hipStream_t);                               \
  template hipError_t launch_fem_setup<T, S, R>(const Dims&, const TileMap&, const Coefs<T>&, const FemTables*,   \
                                                bool, const S*, const S*, T, const T*, T*, R*, R*, R*, R*, T*,    \
                                                double*, hipStream_t);

PF_INSTANTIATE_SETUP(double, double, double)
PF_INSTANTIATE_SETUP(double, float, float)
PF_INSTANTIATE_SETUP(double, float, double)
PF_INSTANTIATE_SETUP(double, double, float)

template hipError_t launch_fem_resid<double, float>(const Dims&, const TileMap&, const FemTables*, bool,
                                                    const double*, double*, float*, float*, float*, float*, double*,
                                                    hipStream_t);
template hipError_t launch_convert<double, float>(const double*, float*, int64_t, hipStream_t);
template hipError_t launch_convert<float, double>(const float*, double*, int64_t, hipStream_t);

}  // namespace pf
