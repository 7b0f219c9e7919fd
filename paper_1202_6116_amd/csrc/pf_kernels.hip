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

namespace pf {

namespace {

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ __forceinline__ int tid_flat() { return threadIdx.x + threadIdx.y * blockDim.x; }

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
constexpr int kHX = kBX + 2, kHY = kBY + 2, kHP = kHX * kHY;

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

__device__ __forceinline__ TileCoord tile_coord(const Dims& d, const TileMap& tm) {
  const int lid = logical_block(tm.nblocks);
  TileCoord t;
  const int tx = lid % tm.ntx;
  const int ty = (lid / tm.ntx) % tm.nty;
  const int kc = lid / (tm.ntx * tm.nty);
  t.i0 = tx * kBX;
  t.j0 = ty * kBY;
  t.k0 = kc * tm.kz;
  t.k1 = min(d.nz, t.k0 + tm.kz);
  t.lid = lid;
  return t;
}

__device__ __forceinline__ int slot_of(int k) { return (k + 3) % 3; }

// Fills ring slot s with plane k of a tile (and its one-node halo) using
// f(n, k, out[NC]) for the values; points outside the grid in z, and tile
// points beyond the ragged edges, hold zero.
template <typename T, int NC, typename F>
__device__ __forceinline__ void load_plane(T (&ring)[3][NC][kHY][kHX], const Dims& d, int i0, int j0, int k, F f) {
  const int s = slot_of(k);
  for (int t = tid_flat(); t < kHP; t += kThreads) {
    const int hx = t % kHX, hy = t / kHX;
    int gi = i0 + hx - 1, gj = j0 + hy - 1;
    T val[NC];
#pragma unroll
    for (int c = 0; c < NC; c++) val[c] = 0;
    if (k >= 0 && k < d.nz && gi >= -1 && gi <= d.nx && gj >= -1 && gj <= d.ny) {
      gi = wrap(gi, d.nx);
      gj = wrap(gj, d.ny);
      f(gi + (int64_t)d.nx * gj + d.plane * k, k, val);
    }
#pragma unroll
    for (int c = 0; c < NC; c++) ring[s][c][hy][hx] = val[c];
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
enum { kRedSetup = 0, kRedAlpha = 1, kRedBeta = 2 };
constexpr int kRedThreads = 1024;

template <int NV>
__global__ __launch_bounds__(kRedThreads) void cg_reduce_kernel(const double* __restrict__ partials, int nblocks,
                                                                CgScalars* sc, int mode, double tol, int maxit) {
  if (mode != kRedSetup && sc->done) return;
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

// ---------------------------------------------------------------------------
// Poisson: A phi = -eps_b Lap_h phi (zero ghosts), b = -D_h P + ghost terms
// ---------------------------------------------------------------------------

// b from Pp = P + cdt V (V may be null) and the ghost planes; r = b - A x;
// p = r / diag; partial (b.b, r.z, r.r).  T: arithmetic and r, x, p;
// S: storage of P and V.
template <typename T, typename S>
__global__ __launch_bounds__(kThreads) void poisson_setup_kernel(
    Dims d, Coefs<T> cf, const S* __restrict__ P, const S* __restrict__ V, T cdt, int with_P, int with_bc,
    const T* __restrict__ ghost_top, T phi_bottom, const T* __restrict__ x, T* __restrict__ r, T* __restrict__ p,
    double* partials) {
  const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y, k = blockIdx.z;
  double v[3] = {0.0, 0.0, 0.0};
  if (i < d.nx && j < d.ny) {
    const int64_t N = d.N, pl = d.plane;
    const int64_t n = i + (int64_t)d.nx * j + pl * k;
    const int64_t nxp = wrap(i + 1, d.nx) + (int64_t)d.nx * j + pl * k;
    const int64_t nxm = wrap(i - 1, d.nx) + (int64_t)d.nx * j + pl * k;
    const int64_t nyp = i + (int64_t)d.nx * wrap(j + 1, d.ny) + pl * k;
    const int64_t nym = i + (int64_t)d.nx * wrap(j - 1, d.ny) + pl * k;
    const bool up = k + 1 < d.nz, dn = k > 0;
    auto pp = [&](int c, int64_t m) -> T { return (T)P[c * N + m] + (V ? cdt * (T)V[c * N + m] : (T)0); };
    T b = 0;
    if (with_P) {
      const T dx = pp(0, nxp) - pp(0, nxm);
      const T dy = pp(1, nyp) - pp(1, nym);
      const T zp = up ? pp(2, n + pl) : (T)0;
      const T zm = dn ? pp(2, n - pl) : (T)0;
      b = -(dx + dy + (zp - zm)) * cf.inv_2h;
    }
    if (with_bc) {
      if (k == 0) b += cf.eps_over_h2 * phi_bottom;
      if (k == d.nz - 1) b += cf.eps_over_h2 * ghost_top[i + (int64_t)d.nx * j];
    }
    T s = x[nxp] + x[nxm] + x[nyp] + x[nym];
    if (up) s += x[n + pl];
    if (dn) s += x[n - pl];
    const T Ax = cf.eps_over_h2 * (6 * x[n] - s);
    const T rr = b - Ax;
    const T z = rr * cf.inv_diag_poisson;
    r[n] = rr;
    p[n] = z;
    v[0] = (double)b * b;
    v[1] = (double)rr * z;
    v[2] = (double)rr * rr;
  }
  block_partials<3, kThreads>(v, partials, node_block_id());
}

// Iteration kernel A: p_new = z + beta p_old on the tile and its halo, q =
// A p_new, x += alpha_prev p_old (the deferred update of the previous
// iteration); partial p_new . q.
template <typename T>
__global__ __launch_bounds__(kThreads) void poisson_cg_a_kernel(Dims d, TileMap tm, Coefs<T> cf,
                                                                const T* __restrict__ r, const T* __restrict__ p_old,
                                                                T* __restrict__ p_new, T* __restrict__ x,
                                                                const CgScalars* sc, double* partials) {
  if (sc->done) return;
  __shared__ T ring[3][1][kHY][kHX];
  const T beta = (T)sc->beta, alpha = (T)sc->alpha, w = cf.inv_diag_poisson, c6 = cf.eps_over_h2;
  const TileCoord tc = tile_coord(d, tm);
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int i = tc.i0 + lx, j = tc.j0 + ly;
  const bool valid = i < d.nx && j < d.ny;
  auto f = [&](int64_t m, int, T* out) { out[0] = r[m] * w + beta * p_old[m]; };
  load_plane<T, 1>(ring, d, tc.i0, tc.j0, tc.k0 - 1, f);
  load_plane<T, 1>(ring, d, tc.i0, tc.j0, tc.k0, f);
  double acc = 0.0;
  for (int k = tc.k0; k < tc.k1; k++) {
    load_plane<T, 1>(ring, d, tc.i0, tc.j0, k + 1, f);
    __syncthreads();
    if (valid) {
      const int sm = slot_of(k - 1), s0 = slot_of(k), sp = slot_of(k + 1);
      const T pc = ring[s0][0][ly + 1][lx + 1];
      const T s = ring[s0][0][ly + 1][lx] + ring[s0][0][ly + 1][lx + 2] + ring[s0][0][ly][lx + 1] +
                  ring[s0][0][ly + 2][lx + 1] + ring[sm][0][ly + 1][lx + 1] + ring[sp][0][ly + 1][lx + 1];
      const T q = c6 * (6 * pc - s);
      const int64_t n = i + (int64_t)d.nx * j + d.plane * k;
      p_new[n] = pc;
      x[n] += alpha * p_old[n];
      acc += (double)pc * q;
    }
    __syncthreads();
  }
  double v[1] = {acc};
  block_partials<1, kThreads>(v, partials, tc.lid);
}

// Iteration kernel B: r -= alpha A p (operator recomputed); partial (r.z, r.r).
template <typename T>
__global__ __launch_bounds__(kThreads) void poisson_cg_b_kernel(Dims d, TileMap tm, Coefs<T> cf,
                                                                const T* __restrict__ p, T* __restrict__ r,
                                                                const CgScalars* sc, double* partials) {
  if (sc->done) return;
  __shared__ T ring[3][1][kHY][kHX];
  const T alpha = (T)sc->alpha, w = cf.inv_diag_poisson, c6 = cf.eps_over_h2;
  const TileCoord tc = tile_coord(d, tm);
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int i = tc.i0 + lx, j = tc.j0 + ly;
  const bool valid = i < d.nx && j < d.ny;
  auto f = [&](int64_t m, int, T* out) { out[0] = p[m]; };
  load_plane<T, 1>(ring, d, tc.i0, tc.j0, tc.k0 - 1, f);
  load_plane<T, 1>(ring, d, tc.i0, tc.j0, tc.k0, f);
  double a0 = 0.0, a1 = 0.0;
  for (int k = tc.k0; k < tc.k1; k++) {
    load_plane<T, 1>(ring, d, tc.i0, tc.j0, k + 1, f);
    __syncthreads();
    if (valid) {
      const int sm = slot_of(k - 1), s0 = slot_of(k), sp = slot_of(k + 1);
      const T pc = ring[s0][0][ly + 1][lx + 1];
      const T s = ring[s0][0][ly + 1][lx] + ring[s0][0][ly + 1][lx + 2] + ring[s0][0][ly][lx + 1] +
                  ring[s0][0][ly + 2][lx + 1] + ring[sm][0][ly + 1][lx + 1] + ring[sp][0][ly + 1][lx + 1];
      const T q = c6 * (6 * pc - s);
      const int64_t n = i + (int64_t)d.nx * j + d.plane * k;
      const T rn = r[n] - alpha * q;
      r[n] = rn;
      a0 += (double)rn * (rn * w);
      a1 += (double)rn * rn;
    }
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
// ld(dx, dy, dz, out[3]).  Interior rows skip the structurally zero taps of
// the coupling blocks (their 1D derivative factor vanishes at offset 0).
template <typename T, typename Load>
__device__ __forceinline__ void fem_K_apply(const FemTables* __restrict__ tb, int zt, Load ld, T out[3]) {
  out[0] = out[1] = out[2] = 0;
  if (zt == 0) {
#pragma unroll
    for (int dz = -1; dz <= 1; dz++)
#pragma unroll
      for (int dy = -1; dy <= 1; dy++)
#pragma unroll
        for (int dx = -1; dx <= 1; dx++) {
          const int o = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
          const int off[3] = {dx, dy, dz};
          T u[3];
          ld(dx, dy, dz, u);
#pragma unroll
          for (int c = 0; c < 3; c++)
#pragma unroll
            for (int e = 0; e < 3; e++) {
              if (c != e && (off[c] == 0 || off[e] == 0)) continue;
              out[c] += (T)tb->K[0][c][e][o] * u[e];
            }
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

template <typename T>
__device__ __forceinline__ void eigenstrain(const Coefs<T>& cf, T x, T y, T z, T e[6]) {
  const T x2 = x * x, y2 = y * y, z2 = z * z;
  e[0] = cf.Q11 * x2 + cf.Q12 * (y2 + z2);
  e[1] = cf.Q11 * y2 + cf.Q12 * (z2 + x2);
  e[2] = cf.Q11 * z2 + cf.Q12 * (x2 + y2);
  e[3] = 2 * cf.Q44 * x * y;
  e[4] = 2 * cf.Q44 * y * z;
  e[5] = 2 * cf.Q44 * z * x;
}

// sigma = C e for the cubic Voigt stiffness (engineering shear).
template <typename T>
__device__ __forceinline__ void cubic_stress(const Coefs<T>& cf, const T e[6], T s[6]) {
  s[0] = cf.C11 * e[0] + cf.C12 * (e[1] + e[2]);
  s[1] = cf.C11 * e[1] + cf.C12 * (e[2] + e[0]);
  s[2] = cf.C11 * e[2] + cf.C12 * (e[0] + e[1]);
  s[3] = cf.C44 * e[3];
  s[4] = cf.C44 * e[4];
  s[5] = cf.C44 * e[5];
}

}  // namespace

// f = body force of the eigenstrain of Pp = P + cdt V (Eq. 15); r = f - K x;
// p = r / diag.  The clamped plane k = 0 has x = r = p = 0 (both direction
// buffers).  Partial (f.f, r.z, r.r).
template <typename T, typename S>
__global__ __launch_bounds__(kThreads) void fem_setup_kernel(
    Dims d, Coefs<T> cf, const FemTables* __restrict__ tb, const S* __restrict__ P, const S* __restrict__ V, T cdt,
    T* __restrict__ x, T* __restrict__ r, T* __restrict__ p0, T* __restrict__ p1, double* partials) {
  const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y, k = blockIdx.z;
  double v[3] = {0.0, 0.0, 0.0};
  if (i < d.nx && j < d.ny) {
    const int64_t N = d.N;
    const int64_t n = i + (int64_t)d.nx * j + d.plane * k;
    if (k == 0) {
#pragma unroll
      for (int c = 0; c < 3; c++) {
        x[c * N + n] = 0;
        r[c * N + n] = 0;
        p0[c * N + n] = 0;
        p1[c * N + n] = 0;
      }
    } else {
      const int zt = (k == d.nz - 1) ? 1 : 0;
      const int dzmax = zt ? 0 : 1;
      T f[3] = {0, 0, 0};
      for (int dz = -1; dz <= dzmax; dz++)
#pragma unroll
        for (int dy = -1; dy <= 1; dy++)
#pragma unroll
          for (int dx = -1; dx <= 1; dx++) {
            const int o = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
            const int64_t m = nbr(d, i, j, k, dx, dy, dz);
            T px = (T)P[m], py = (T)P[N + m], pz = (T)P[2 * N + m];
            if (V) {
              px += cdt * (T)V[m];
              py += cdt * (T)V[N + m];
              pz += cdt * (T)V[2 * N + m];
            }
            T e[6], s[6];
            eigenstrain(cf, px, py, pz, e);
            cubic_stress(cf, e, s);
#pragma unroll
            for (int c = 0; c < 3; c++)
#pragma unroll
              for (int q = 0; q < 6; q++) f[c] += (T)tb->Bf[zt][c][q][o] * s[q];
          }
      auto ldx = [&](int dx, int dy, int dz, T u[3]) {
        const int64_t m = nbr(d, i, j, k, dx, dy, dz);
        if (k + dz == 0) {
          u[0] = u[1] = u[2] = 0;  // clamped column
        } else {
          u[0] = x[m];
          u[1] = x[N + m];
          u[2] = x[2 * N + m];
        }
      };
      T Kx[3];
      fem_K_apply<T>(tb, zt, ldx, Kx);
      const T wdiag = (T)tb->inv_diag[zt];
#pragma unroll
      for (int c = 0; c < 3; c++) {
        const T rr = f[c] - Kx[c];
        const T z = rr * wdiag;
        r[c * N + n] = rr;
        p0[c * N + n] = z;
        v[0] += (double)f[c] * f[c];
        v[1] += (double)rr * z;
        v[2] += (double)rr * rr;
      }
    }
  }
  block_partials<3, kThreads>(v, partials, node_block_id());
}

// Iteration kernel A: p_new = z + beta p_old on the tile and its halo (zero
// on the clamped plane), q = K p_new, x += alpha_prev p_old; partial p.q.
template <typename T>
__global__ __launch_bounds__(kThreads) void fem_cg_a_kernel(Dims d, TileMap tm, const FemTables* __restrict__ tb,
                                                            const T* __restrict__ r, const T* __restrict__ p_old,
                                                            T* __restrict__ p_new, T* __restrict__ x,
                                                            const CgScalars* sc, double* partials) {
  if (sc->done) return;
  __shared__ T ring[3][3][kHY][kHX];
  const T beta = (T)sc->beta, alpha = (T)sc->alpha;
  const T w_int = (T)tb->inv_diag[0], w_top = (T)tb->inv_diag[1];
  const TileCoord tc = tile_coord(d, tm);
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int i = tc.i0 + lx, j = tc.j0 + ly;
  const bool valid = i < d.nx && j < d.ny;
  const int64_t N = d.N;
  auto f = [&](int64_t m, int k, T* out) {
    if (k == 0) return;  // clamped plane: zero
    const T w = (k == d.nz - 1) ? w_top : w_int;
#pragma unroll
    for (int c = 0; c < 3; c++) out[c] = r[c * N + m] * w + beta * p_old[c * N + m];
  };
  load_plane<T, 3>(ring, d, tc.i0, tc.j0, tc.k0 - 1, f);
  load_plane<T, 3>(ring, d, tc.i0, tc.j0, tc.k0, f);
  double acc = 0.0;
  for (int k = tc.k0; k < tc.k1; k++) {
    load_plane<T, 3>(ring, d, tc.i0, tc.j0, k + 1, f);
    __syncthreads();
    if (valid && k > 0) {
      const int zt = (k == d.nz - 1) ? 1 : 0;
      auto ld = [&](int dx, int dy, int dz, T u[3]) {
        const int s = slot_of(k + dz);
#pragma unroll
        for (int c = 0; c < 3; c++) u[c] = ring[s][c][ly + 1 + dy][lx + 1 + dx];
      };
      T q[3];
      fem_K_apply<T>(tb, zt, ld, q);
      const int64_t n = i + (int64_t)d.nx * j + d.plane * k;
      const int s0 = slot_of(k);
#pragma unroll
      for (int c = 0; c < 3; c++) {
        const T pc = ring[s0][c][ly + 1][lx + 1];
        p_new[c * N + n] = pc;
        x[c * N + n] += alpha * p_old[c * N + n];
        acc += (double)pc * q[c];
      }
    }
    __syncthreads();
  }
  double v[1] = {acc};
  block_partials<1, kThreads>(v, partials, tc.lid);
}

// Iteration kernel B: r -= alpha K p (operator recomputed); partial (r.z, r.r).
template <typename T>
__global__ __launch_bounds__(kThreads) void fem_cg_b_kernel(Dims d, TileMap tm, const FemTables* __restrict__ tb,
                                                            const T* __restrict__ p, T* __restrict__ r,
                                                            const CgScalars* sc, double* partials) {
  if (sc->done) return;
  __shared__ T ring[3][3][kHY][kHX];
  const T alpha = (T)sc->alpha;
  const T w_int = (T)tb->inv_diag[0], w_top = (T)tb->inv_diag[1];
  const TileCoord tc = tile_coord(d, tm);
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int i = tc.i0 + lx, j = tc.j0 + ly;
  const bool valid = i < d.nx && j < d.ny;
  const int64_t N = d.N;
  auto f = [&](int64_t m, int k, T* out) {
    if (k == 0) return;
#pragma unroll
    for (int c = 0; c < 3; c++) out[c] = p[c * N + m];
  };
  load_plane<T, 3>(ring, d, tc.i0, tc.j0, tc.k0 - 1, f);
  load_plane<T, 3>(ring, d, tc.i0, tc.j0, tc.k0, f);
  double a0 = 0.0, a1 = 0.0;
  for (int k = tc.k0; k < tc.k1; k++) {
    load_plane<T, 3>(ring, d, tc.i0, tc.j0, k + 1, f);
    __syncthreads();
    if (valid && k > 0) {
      const int zt = (k == d.nz - 1) ? 1 : 0;
      auto ld = [&](int dx, int dy, int dz, T u[3]) {
        const int s = slot_of(k + dz);
#pragma unroll
        for (int c = 0; c < 3; c++) u[c] = ring[s][c][ly + 1 + dy][lx + 1 + dx];
      };
      T q[3];
      fem_K_apply<T>(tb, zt, ld, q);
      const T w = zt ? w_top : w_int;
      const int64_t n = i + (int64_t)d.nx * j + d.plane * k;
#pragma unroll
      for (int c = 0; c < 3; c++) {
        const T rn = r[c * N + n] - alpha * q[c];
        r[c * N + n] = rn;
        a0 += (double)rn * (rn * w);
        a1 += (double)rn * rn;
      }
    }
    __syncthreads();
  }
  double v[2] = {a0, a1};
  block_partials<2, kThreads>(v, partials, tc.lid);
}

// ---------------------------------------------------------------------------
// Force and time integration (Eq. 7, 19)
// ---------------------------------------------------------------------------
// At every node, with Pp = P + cdt V:
//   F = -L [ dfL/dP(Pp) - G Lap_h Pp - E - h^-3 s . deps0/dP(Pp) ]
//   E = -G_h phi (Dirichlet ghosts), s = C (int N_n eps(u) - int N_n eps0(Pp))
// then, by mode: write F; V = F; (V, P) <- ((V+F)/2, P + dt (V+F)/2);
// P <- P + dt F.  Reads (P, V) and writes (Pn, Vn), distinct buffers.
template <typename T>
__global__ __launch_bounds__(kThreads) void force_kernel(
    Dims d, Coefs<T> cf, const FemTables* __restrict__ tb, const T* __restrict__ P, const T* __restrict__ V, T cdt,
    const T* __restrict__ phi, const T* __restrict__ ghost_top, const T* __restrict__ u, int mode,
    T* __restrict__ Pn, T* __restrict__ Vn, T* __restrict__ Fout) {
  const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y, k = blockIdx.z;
  if (i >= d.nx || j >= d.ny) return;
  const int64_t N = d.N, pl = d.plane;
  const int64_t n = i + (int64_t)d.nx * j + pl * k;
  const bool hasV = V != nullptr;
  auto pp = [&](int64_t m, T out[3]) {
#pragma unroll
    for (int c = 0; c < 3; c++) out[c] = P[c * N + m] + (hasV ? cdt * V[c * N + m] : (T)0);
  };
  T p0[3];
  pp(n, p0);
  T F[3] = {0, 0, 0};
  if (cf.terms & kLandau) {
    const T x2 = p0[0] * p0[0], y2 = p0[1] * p0[1], z2 = p0[2] * p0[2];
    F[0] += 2 * cf.a1 * p0[0] + 4 * cf.a11 * x2 * p0[0] + 2 * cf.a12 * p0[0] * (y2 + z2);
    F[1] += 2 * cf.a1 * p0[1] + 4 * cf.a11 * y2 * p0[1] + 2 * cf.a12 * p0[1] * (z2 + x2);
    F[2] += 2 * cf.a1 * p0[2] + 4 * cf.a11 * z2 * p0[2] + 2 * cf.a12 * p0[2] * (x2 + y2);
  }
  if (cf.terms & kGrad) {
    T a[3], lap[3] = {0, 0, 0};
    const int64_t ms[4] = {nbr(d, i, j, k, 1, 0, 0), nbr(d, i, j, k, -1, 0, 0), nbr(d, i, j, k, 0, 1, 0),
                           nbr(d, i, j, k, 0, -1, 0)};
#pragma unroll
    for (int t = 0; t < 4; t++) {
      pp(ms[t], a);
#pragma unroll
      for (int c = 0; c < 3; c++) lap[c] += a[c] - p0[c];
    }
    if (k + 1 < d.nz) {
      pp(n + pl, a);
#pragma unroll
      for (int c = 0; c < 3; c++) lap[c] += a[c] - p0[c];
    }
    if (k > 0) {
      pp(n - pl, a);
#pragma unroll
      for (int c = 0; c < 3; c++) lap[c] += a[c] - p0[c];
    }
#pragma unroll
    for (int c = 0; c < 3; c++) F[c] -= cf.G * cf.inv_h2 * lap[c];
  }
  if (cf.terms & kElec) {
    const T zp = (k + 1 < d.nz) ? phi[n + pl] : ghost_top[i + (int64_t)d.nx * j];
    const T zm = (k > 0) ? phi[n - pl] : cf.phi_bottom;
    F[0] += (phi[nbr(d, i, j, k, 1, 0, 0)] - phi[nbr(d, i, j, k, -1, 0, 0)]) * cf.inv_2h;
    F[1] += (phi[nbr(d, i, j, k, 0, 1, 0)] - phi[nbr(d, i, j, k, 0, -1, 0)]) * cf.inv_2h;
    F[2] += (zp - zm) * cf.inv_2h;
  }
  if (cf.terms & kElas) {
    const int zt = (k == 0) ? kLow : ((k == d.nz - 1) ? kHigh : kInterior);
    const int dzmin = (k == 0) ? 0 : -1, dzmax = (k == d.nz - 1) ? 0 : 1;
    T w[6] = {0, 0, 0, 0, 0, 0};
    for (int dz = dzmin; dz <= dzmax; dz++)
#pragma unroll
      for (int dy = -1; dy <= 1; dy++)
#pragma unroll
        for (int dx = -1; dx <= 1; dx++) {
          const int o = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
          const int64_t m = nbr(d, i, j, k, dx, dy, dz);
          T a[3], e[6];
          pp(m, a);
          eigenstrain(cf, a[0], a[1], a[2], e);
          const T ms = (T)tb->Ms[zt][o];
          const T uu[3] = {u[m], u[N + m], u[2 * N + m]};
#pragma unroll
          for (int q = 0; q < 6; q++) {
            T acc = -ms * e[q];
#pragma unroll
            for (int c = 0; c < 3; c++) acc += (T)tb->Su[zt][q][c][o] * uu[c];
            w[q] += acc;
          }
        }
    T s[6];
    cubic_stress(cf, w, s);
    const T g0 = 2 * p0[0] * (cf.Q11 * s[0] + cf.Q12 * (s[1] + s[2])) + 2 * cf.Q44 * (p0[1] * s[3] + p0[2] * s[5]);
    const T g1 = 2 * p0[1] * (cf.Q11 * s[1] + cf.Q12 * (s[2] + s[0])) + 2 * cf.Q44 * (p0[0] * s[3] + p0[2] * s[4]);
    const T g2 = 2 * p0[2] * (cf.Q11 * s[2] + cf.Q12 * (s[0] + s[1])) + 2 * cf.Q44 * (p0[1] * s[4] + p0[0] * s[5]);
    F[0] -= cf.inv_h3 * g0;
    F[1] -= cf.inv_h3 * g1;
    F[2] -= cf.inv_h3 * g2;
  }
#pragma unroll
  for (int c = 0; c < 3; c++) F[c] *= -cf.L;
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
#pragma unroll
      for (int c = 0; c < 3; c++) {
        const T vn = (T)0.5 * (V[c * N + n] + F[c]);
        Vn[c * N + n] = vn;
        Pn[c * N + n] = P[c * N + n] + cf.dt * vn;
      }
      break;
    default:  // kEulerStep
#pragma unroll
      for (int c = 0; c < 3; c++) Pn[c * N + n] = P[c * N + n] + cf.dt * F[c];
      break;
  }
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

// z-chunk length: enough blocks to fill the chip (about 8 per CU), chunks
// of 4..32 planes.
TileMap make_tile_map(const Dims& d) {
  TileMap t;
  t.ntx = (d.nx + kBX - 1) / kBX;
  t.nty = (d.ny + kBY - 1) / kBY;
  const int64_t cols = (int64_t)t.ntx * t.nty;
  int64_t kz = (int64_t)d.nz * cols / 2048;
  kz = kz < 4 ? 4 : (kz > 32 ? 32 : kz);
  if (kz > d.nz) kz = d.nz;
  t.kz = (int)kz;
  t.nkz = (d.nz + t.kz - 1) / t.kz;
  t.nblocks = (int)(cols * t.nkz);
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
                            int maxit, hipStream_t s) {
  switch (nv) {
    case 1: cg_reduce_kernel<1><<<1, kRedThreads, 0, s>>>(partials, nblocks, sc, mode, tol, maxit); break;
    case 2: cg_reduce_kernel<2><<<1, kRedThreads, 0, s>>>(partials, nblocks, sc, mode, tol, maxit); break;
    default: cg_reduce_kernel<3><<<1, kRedThreads, 0, s>>>(partials, nblocks, sc, mode, tol, maxit); break;
  }
  return hipGetLastError();
}

template <typename T, typename S>
hipError_t launch_poisson_setup(const Dims& d, const Coefs<T>& cf, const S* P, const S* V, T cdt, int with_P,
                                int with_bc, const T* ghost_top, T phi_bottom, const T* x, T* r, T* p,
                                double* partials, hipStream_t s) {
  poisson_setup_kernel<T, S><<<node_grid(d), node_block(), 0, s>>>(d, cf, P, V, cdt, with_P, with_bc, ghost_top,
                                                                   phi_bottom, x, r, p, partials);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_poisson_cg_a(const Dims& d, const TileMap& tm, const Coefs<T>& cf, const T* r, const T* p_old,
                               T* p_new, T* x, const CgScalars* sc, double* partials, hipStream_t s) {
  poisson_cg_a_kernel<T><<<tm.nblocks, node_block(), 0, s>>>(d, tm, cf, r, p_old, p_new, x, sc, partials);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_poisson_cg_b(const Dims& d, const TileMap& tm, const Coefs<T>& cf, const T* p, T* r,
                               const CgScalars* sc, double* partials, hipStream_t s) {
  poisson_cg_b_kernel<T><<<tm.nblocks, node_block(), 0, s>>>(d, tm, cf, p, r, sc, partials);
  return hipGetLastError();
}

template <typename T, typename S>
hipError_t launch_fem_setup(const Dims& d, const Coefs<T>& cf, const FemTables* tb, const S* P, const S* V, T cdt,
                            T* x, T* r, T* p0, T* p1, double* partials, hipStream_t s) {
  fem_setup_kernel<T, S><<<node_grid(d), node_block(), 0, s>>>(d, cf, tb, P, V, cdt, x, r, p0, p1, partials);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fem_cg_a(const Dims& d, const TileMap& tm, const FemTables* tb, const T* r, const T* p_old,
                           T* p_new, T* x, const CgScalars* sc, double* partials, hipStream_t s) {
  fem_cg_a_kernel<T><<<tm.nblocks, node_block(), 0, s>>>(d, tm, tb, r, p_old, p_new, x, sc, partials);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fem_cg_b(const Dims& d, const TileMap& tm, const FemTables* tb, const T* p, T* r,
                           const CgScalars* sc, double* partials, hipStream_t s) {
  fem_cg_b_kernel<T><<<tm.nblocks, node_block(), 0, s>>>(d, tm, tb, p, r, sc, partials);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_force(const Dims& d, const Coefs<T>& cf, const FemTables* tb, const T* P, const T* V, T cdt,
                        const T* phi, const T* ghost_top, const T* u, int mode, T* Pn, T* Vn, T* Fout,
                        hipStream_t s) {
  force_kernel<T><<<node_grid(d), node_block(), 0, s>>>(d, cf, tb, P, V, cdt, phi, ghost_top, u, mode, Pn, Vn,
                                                        Fout);
  return hipGetLastError();
}

#define PF_INSTANTIATE(T)                                                                                        \
  template hipError_t launch_fill<T>(T*, int64_t, T, hipStream_t);                                               \
  template hipError_t launch_cg_finish<T>(T*, const T*, int64_t, const CgScalars*, hipStream_t);                 \
  template hipError_t launch_poisson_cg_a<T>(const Dims&, const TileMap&, const Coefs<T>&, const T*, const T*,   \
                                             T*, T*, const CgScalars*, double*, hipStream_t);                    \
  template hipError_t launch_poisson_cg_b<T>(const Dims&, const TileMap&, const Coefs<T>&, const T*, T*,         \
                                             const CgScalars*, double*, hipStream_t);                            \
  template hipError_t launch_fem_cg_a<T>(const Dims&, const TileMap&, const FemTables*, const T*, const T*, T*,  \
                                         T*, const CgScalars*, double*, hipStream_t);                            \
  template hipError_t launch_fem_cg_b<T>(const Dims&, const TileMap&, const FemTables*, const T*, T*,            \
                                         const CgScalars*, double*, hipStream_t);                                \
  template hipError_t launch_force<T>(const Dims&, const Coefs<T>&, const FemTables*, const T*, const T*, T,     \
                                      const T*, const T*, const T*, int, T*, T*, T*, hipStream_t);

PF_INSTANTIATE(double)
PF_INSTANTIATE(float)

#define PF_INSTANTIATE_SETUP(T, S)                                                                               \
  template hipError_t launch_poisson_setup<T, S>(const Dims&, const Coefs<T>&, const S*, const S*, T, int, int,  \
                                                 const T*, T, const T*, T*, T*, double*, hipStream_t);           \
  template hipError_t launch_fem_setup<T, S>(const Dims&, const Coefs<T>&, const FemTables*, const S*, const S*, \
                                             T, T*, T*, T*, T*, double*, hipStream_t);

PF_INSTANTIATE_SETUP(double, double)
PF_INSTANTIATE_SETUP(double, float)
PF_INSTANTIATE_SETUP(float, float)

template hipError_t launch_convert<double, float>(const double*, float*, int64_t, hipStream_t);
template hipError_t launch_convert<float, double>(const float*, double*, int64_t, hipStream_t);

}  // namespace pf
