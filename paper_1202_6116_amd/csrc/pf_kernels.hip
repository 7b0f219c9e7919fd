// HIP kernels of the TDGL step on gfx950: Poisson and FEM conjugate-gradient
// sweeps with fused reductions, the FEM body force, and the fused force +
// time-integration sweep.  One thread per grid node; blocks of 64 x 4 nodes
// in the x-y plane, one z-plane per block row of the grid.
//
// Numbering: node n = i + nx (j + ny k), fields are structure-of-arrays
// (component c of node n at c*N + n), periodic in x and y, k = 0 the clamped
// substrate side, k = nz-1 the free top (Sec. III.A-B of the paper).
#include "pf_internal.h"

#include <math.h>

namespace pf {

namespace {

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ __forceinline__ int tid_flat() { return threadIdx.x + threadIdx.y * blockDim.x; }

__device__ __forceinline__ int block_flat() {
  return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic block reduction of NV values into partials[bid*NV + t],
// then a ticket on `counter`.  Returns true (in every thread) in the block
// that finishes last; that block may then read all partials.
template <int NV>
__device__ bool reduce_to_partials(double (&v)[NV], double* partials, uint32_t* counter, int nblocks) {
  __shared__ double red[NV][kThreads / 64];
  __shared__ int is_last;
  const int tid = tid_flat();
  const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int t = 0; t < NV; t++) {
    double s = wave_sum(v[t]);
    if (lane == 0) red[t][wv] = s;
  }
  __syncthreads();
  if (tid == 0) {
    const int bid = block_flat();
#pragma unroll
    for (int t = 0; t < NV; t++) {
      double s = 0.0;
      for (int w = 0; w < kThreads / 64; w++) s += red[t][w];
      partials[(int64_t)bid * NV + t] = s;
    }
    __threadfence();
    const uint32_t ticket = atomicAdd(counter, 1u);
    is_last = (ticket == (uint32_t)(nblocks - 1));
  }
  __syncthreads();
  const bool last = is_last != 0;
  if (last) __threadfence();
  return last;
}

// In the last block: sum of all partials in a fixed order (thread t takes
// blocks t, t + 256, ...; then a fixed tree).  Result valid in thread 0.
template <int NV>
__device__ void sum_partials(const double* partials, int nblocks, double (&out)[NV]) {
  __shared__ double red[NV][kThreads / 64];
  const int tid = tid_flat();
  const int lane = tid & 63, wv = tid >> 6;
  double s[NV];
#pragma unroll
  for (int t = 0; t < NV; t++) s[t] = 0.0;
  for (int b = tid; b < nblocks; b += kThreads) {
#pragma unroll
    for (int t = 0; t < NV; t++) s[t] += __builtin_nontemporal_load(partials + (int64_t)b * NV + t);
  }
#pragma unroll
  for (int t = 0; t < NV; t++) {
    double w = wave_sum(s[t]);
    if (lane == 0) red[t][wv] = w;
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int t = 0; t < NV; t++) {
      double a = 0.0;
      for (int w = 0; w < kThreads / 64; w++) a += red[t][w];
      out[t] = a;
    }
  }
}

__device__ __forceinline__ bool finite(double x) { return isfinite(x); }

// Convergence test shared by the setup and update kernels:
// ||r|| <= tol ||b||.
__device__ __forceinline__ bool converged(double rnorm2, double bnorm2, double tol) {
  return sqrt(rnorm2) <= tol * sqrt(bnorm2);
}

}  // namespace

// ---------------------------------------------------------------------------
// Utility kernels
// ---------------------------------------------------------------------------

template <typename T>
__global__ void fill_kernel(T* a, int64_t n, T v) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; t < n; t += stride) a[t] = v;
}

template <typename T, typename U>
__global__ void convert_kernel(const T* a, U* b, int64_t n) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; t < n; t += stride) b[t] = (U)a[t];
}

// x += alpha * p (alpha read from the CG scalars); x = 0 for a zero rhs.
template <typename T>
__global__ void cg_finish_kernel(T* x, const T* p, int64_t n, const CgScalars* sc) {
  const T alpha = (T)sc->alpha;
  const bool zero = sc->zero_rhs != 0;
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; t < n; t += stride) x[t] = zero ? (T)0 : x[t] + alpha * p[t];
}

// ---------------------------------------------------------------------------
// Poisson: A phi = -eps_b Lap_h phi (zero ghosts), b = -D_h P + ghost terms
// ---------------------------------------------------------------------------

// b from the polarisation Pp = P + cdt V (V may be null) and the Dirichlet
// ghost planes; r = b - A x; p = r / diag; partial (b.b, r.z, r.r).
template <typename T>
__global__ __launch_bounds__(kThreads) void poisson_setup_kernel(
    Dims d, Coefs<T> cf, const T* __restrict__ P, const T* __restrict__ V, T cdt, int with_P, int with_bc,
    const T* __restrict__ ghost_top, T phi_bottom, const T* __restrict__ x, T* __restrict__ r, T* __restrict__ p,
    CgScalars* sc, double* partials, int nblocks, double tol, int maxit) {
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
    T b = 0;
    if (with_P) {
      T dx, dy, zp = 0, zm = 0;
      if (V) {
        dx = (P[nxp] + cdt * V[nxp]) - (P[nxm] + cdt * V[nxm]);
        dy = (P[N + nyp] + cdt * V[N + nyp]) - (P[N + nym] + cdt * V[N + nym]);
        if (up) zp = P[2 * N + n + pl] + cdt * V[2 * N + n + pl];
        if (dn) zm = P[2 * N + n - pl] + cdt * V[2 * N + n - pl];
      } else {
        dx = P[nxp] - P[nxm];
        dy = P[N + nyp] - P[N + nym];
        if (up) zp = P[2 * N + n + pl];
        if (dn) zm = P[2 * N + n - pl];
      }
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
  if (reduce_to_partials<3>(v, partials, &sc->counter, nblocks)) {
    double s[3];
    sum_partials<3>(partials, nblocks, s);
    if (tid_flat() == 0) {
      sc->bnorm2 = s[0];
      sc->rho = s[1];
      sc->rnorm2 = s[2];
      sc->alpha = 0.0;
      sc->beta = 0.0;
      sc->iter = 0;
      sc->tol = tol;
      sc->maxit = maxit;
      sc->zero_rhs = 0;
      if (!finite(s[0]) || !finite(s[1]) || !finite(s[2])) sc->done = kNonFinite;
      else if (s[0] == 0.0) { sc->done = kConverged; sc->zero_rhs = 1; sc->rnorm2 = 0.0; }
      else if (converged(s[2], s[0], tol)) sc->done = kConverged;
      else sc->done = maxit <= 0 ? kMaxIt : kRunning;
      sc->counter = 0;
    }
  }
}

// Direction update fused with the operator: p_new = z + beta p_old at every
// stencil point, q = A p_new, x += alpha_prev p_old (deferred update);
// partial (p_new . q) -> alpha = rho / (p.q).
template <typename T>
__global__ __launch_bounds__(kThreads) void poisson_cg_a_kernel(
    Dims d, Coefs<T> cf, const T* __restrict__ r, const T* __restrict__ p_old, T* __restrict__ p_new,
    T* __restrict__ x, CgScalars* sc, double* partials, int nblocks) {
  if (sc->done) return;
  const T beta = (T)sc->beta, alpha = (T)sc->alpha, w = cf.inv_diag_poisson;
  const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y, k = blockIdx.z;
  double v[1] = {0.0};
  if (i < d.nx && j < d.ny) {
    const int64_t pl = d.plane;
    const int64_t n = i + (int64_t)d.nx * j + pl * k;
    const int64_t nxp = wrap(i + 1, d.nx) + (int64_t)d.nx * j + pl * k;
    const int64_t nxm = wrap(i - 1, d.nx) + (int64_t)d.nx * j + pl * k;
    const int64_t nyp = i + (int64_t)d.nx * wrap(j + 1, d.ny) + pl * k;
    const int64_t nym = i + (int64_t)d.nx * wrap(j - 1, d.ny) + pl * k;
    auto pn = [&](int64_t m) { return r[m] * w + beta * p_old[m]; };
    const T po = p_old[n];
    const T pc = r[n] * w + beta * po;
    T s = pn(nxp) + pn(nxm) + pn(nyp) + pn(nym);
    if (k + 1 < d.nz) s += pn(n + pl);
    if (k > 0) s += pn(n - pl);
    const T q = cf.eps_over_h2 * (6 * pc - s);
    p_new[n] = pc;
    x[n] += alpha * po;
    v[0] = (double)pc * q;
  }
  if (reduce_to_partials<1>(v, partials, &sc->counter, nblocks)) {
    double s[1];
    sum_partials<1>(partials, nblocks, s);
    if (tid_flat() == 0) {
      if (!finite(s[0]) || !(s[0] > 0.0)) sc->done = kNonFinite;
      else sc->alpha = sc->rho / s[0];
      sc->counter = 0;
    }
  }
}

// Residual update with the operator recomputed: r -= alpha A p; partial
// (r.z, r.r) -> beta, convergence test.
template <typename T>
__global__ __launch_bounds__(kThreads) void poisson_cg_b_kernel(
    Dims d, Coefs<T> cf, const T* __restrict__ p, T* __restrict__ r, CgScalars* sc, double* partials, int nblocks) {
  if (sc->done) return;
  const T alpha = (T)sc->alpha;
  const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y, k = blockIdx.z;
  double v[2] = {0.0, 0.0};
  if (i < d.nx && j < d.ny) {
    const int64_t pl = d.plane;
    const int64_t n = i + (int64_t)d.nx * j + pl * k;
    const int64_t nxp = wrap(i + 1, d.nx) + (int64_t)d.nx * j + pl * k;
    const int64_t nxm = wrap(i - 1, d.nx) + (int64_t)d.nx * j + pl * k;
    const int64_t nyp = i + (int64_t)d.nx * wrap(j + 1, d.ny) + pl * k;
    const int64_t nym = i + (int64_t)d.nx * wrap(j - 1, d.ny) + pl * k;
    T s = p[nxp] + p[nxm] + p[nyp] + p[nym];
    if (k + 1 < d.nz) s += p[n + pl];
    if (k > 0) s += p[n - pl];
    const T q = cf.eps_over_h2 * (6 * p[n] - s);
    const T rn = r[n] - alpha * q;
    const T z = rn * cf.inv_diag_poisson;
    r[n] = rn;
    v[0] = (double)rn * z;
    v[1] = (double)rn * rn;
  }
  if (reduce_to_partials<2>(v, partials, &sc->counter, nblocks)) {
    double s[2];
    sum_partials<2>(partials, nblocks, s);
    if (tid_flat() == 0) {
      const int it = sc->iter + 1;
      sc->iter = it;
      sc->beta = s[0] / sc->rho;
      sc->rho = s[0];
      sc->rnorm2 = s[1];
      if (!finite(s[0]) || !finite(s[1])) sc->done = kNonFinite;
      else if (converged(s[1], sc->bnorm2, sc->tol)) sc->done = kConverged;
      else if (it >= sc->maxit) sc->done = kMaxIt;
      sc->counter = 0;
    }
  }
}

// ---------------------------------------------------------------------------
// FEM: 27-point block stencils from the trilinear hex element
// ---------------------------------------------------------------------------

namespace {

// K u at a row of type zt (0 interior, 1 top) for a neighbour loader
// ld(dx, dy, dz, out[3]).  Interior rows skip the structurally zero taps of
// the coupling blocks (the 1D derivative factor vanishes at offset 0).
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

template <typename T>
struct Node3 {
  int64_t n;        // linear index
  int i, j, k;
};

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
// p = r / diag.  Row k = 0 is clamped: x = r = p = 0 there (both direction
// buffers).  Partial (f.f, r.z, r.r).
template <typename T>
__global__ __launch_bounds__(kThreads) void fem_setup_kernel(
    Dims d, Coefs<T> cf, const FemTables* __restrict__ tb, const T* __restrict__ P, const T* __restrict__ V, T cdt,
    T* __restrict__ x, T* __restrict__ r, T* __restrict__ p0, T* __restrict__ p1, CgScalars* sc, double* partials,
    int nblocks, double tol, int maxit) {
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
            T px = P[m], py = P[N + m], pz = P[2 * N + m];
            if (V) {
              px += cdt * V[m];
              py += cdt * V[N + m];
              pz += cdt * V[2 * N + m];
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
  if (reduce_to_partials<3>(v, partials, &sc->counter, nblocks)) {
    double s[3];
    sum_partials<3>(partials, nblocks, s);
    if (tid_flat() == 0) {
      sc->bnorm2 = s[0];
      sc->rho = s[1];
      sc->rnorm2 = s[2];
      sc->alpha = 0.0;
      sc->beta = 0.0;
      sc->iter = 0;
      sc->tol = tol;
      sc->maxit = maxit;
      sc->zero_rhs = 0;
      if (!finite(s[0]) || !finite(s[1]) || !finite(s[2])) sc->done = kNonFinite;
      else if (s[0] == 0.0) { sc->done = kConverged; sc->zero_rhs = 1; sc->rnorm2 = 0.0; }
      else if (converged(s[2], s[0], tol)) sc->done = kConverged;
      else sc->done = maxit <= 0 ? kMaxIt : kRunning;
      sc->counter = 0;
    }
  }
}

// x after the setup kernel must be zero on k = 0 before it is read as a
// neighbour; the setup kernel's own reads of x skip that plane.

template <typename T>
__global__ __launch_bounds__(kThreads) void fem_cg_a_kernel(
    Dims d, Coefs<T> cf, const FemTables* __restrict__ tb, const T* __restrict__ r, const T* __restrict__ p_old,
    T* __restrict__ p_new, T* __restrict__ x, CgScalars* sc, double* partials, int nblocks) {
  if (sc->done) return;
  const T beta = (T)sc->beta, alpha = (T)sc->alpha;
  const T w_int = (T)tb->inv_diag[0], w_top = (T)tb->inv_diag[1];
  const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y, k = blockIdx.z;
  double v[1] = {0.0};
  if (i < d.nx && j < d.ny && k > 0) {
    const int64_t N = d.N;
    const int64_t n = i + (int64_t)d.nx * j + d.plane * k;
    const int zt = (k == d.nz - 1) ? 1 : 0;
    auto ld = [&](int dx, int dy, int dz, T u[3]) {
      const int kk = k + dz;
      const int64_t m = nbr(d, i, j, k, dx, dy, dz);
      const T w = (kk == d.nz - 1) ? w_top : w_int;
      if (kk == 0) {
        u[0] = u[1] = u[2] = 0;
      } else {
#pragma unroll
        for (int c = 0; c < 3; c++) u[c] = r[c * N + m] * w + beta * p_old[c * N + m];
      }
    };
    T q[3];
    fem_K_apply<T>(tb, zt, ld, q);
    const T w = zt ? w_top : w_int;
#pragma unroll
    for (int c = 0; c < 3; c++) {
      const T po = p_old[c * N + n];
      const T pc = r[c * N + n] * w + beta * po;
      p_new[c * N + n] = pc;
      x[c * N + n] += alpha * po;
      v[0] += (double)pc * q[c];
    }
  }
  if (reduce_to_partials<1>(v, partials, &sc->counter, nblocks)) {
    double s[1];
    sum_partials<1>(partials, nblocks, s);
    if (tid_flat() == 0) {
      if (!finite(s[0]) || !(s[0] > 0.0)) sc->done = kNonFinite;
      else sc->alpha = sc->rho / s[0];
      sc->counter = 0;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void fem_cg_b_kernel(
    Dims d, Coefs<T> cf, const FemTables* __restrict__ tb, const T* __restrict__ p, T* __restrict__ r, CgScalars* sc,
    double* partials, int nblocks) {
  if (sc->done) return;
  const T alpha = (T)sc->alpha;
  const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y, k = blockIdx.z;
  double v[2] = {0.0, 0.0};
  if (i < d.nx && j < d.ny && k > 0) {
    const int64_t N = d.N;
    const int64_t n = i + (int64_t)d.nx * j + d.plane * k;
    const int zt = (k == d.nz - 1) ? 1 : 0;
    auto ld = [&](int dx, int dy, int dz, T u[3]) {
      const int64_t m = nbr(d, i, j, k, dx, dy, dz);
#pragma unroll
      for (int c = 0; c < 3; c++) u[c] = p[c * N + m];
    };
    T q[3];
    fem_K_apply<T>(tb, zt, ld, q);
    const T w = (T)tb->inv_diag[zt];
#pragma unroll
    for (int c = 0; c < 3; c++) {
      const T rn = r[c * N + n] - alpha * q[c];
      const T z = rn * w;
      r[c * N + n] = rn;
      v[0] += (double)rn * z;
      v[1] += (double)rn * rn;
    }
  }
  if (reduce_to_partials<2>(v, partials, &sc->counter, nblocks)) {
    double s[2];
    sum_partials<2>(partials, nblocks, s);
    if (tid_flat() == 0) {
      const int it = sc->iter + 1;
      sc->iter = it;
      sc->beta = s[0] / sc->rho;
      sc->rho = s[0];
      sc->rnorm2 = s[1];
      if (!finite(s[0]) || !finite(s[1])) sc->done = kNonFinite;
      else if (converged(s[1], sc->bnorm2, sc->tol)) sc->done = kConverged;
      else if (it >= sc->maxit) sc->done = kMaxIt;
      sc->counter = 0;
    }
  }
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
  // Landau (Eq. 1)
  if (cf.terms & kLandau) {
    const T x2 = p0[0] * p0[0], y2 = p0[1] * p0[1], z2 = p0[2] * p0[2];
    F[0] += 2 * cf.a1 * p0[0] + 4 * cf.a11 * x2 * p0[0] + 2 * cf.a12 * p0[0] * (y2 + z2);
    F[1] += 2 * cf.a1 * p0[1] + 4 * cf.a11 * y2 * p0[1] + 2 * cf.a12 * p0[1] * (z2 + x2);
    F[2] += 2 * cf.a1 * p0[2] + 4 * cf.a11 * z2 * p0[2] + 2 * cf.a12 * p0[2] * (x2 + y2);
  }
  // gradient term: -G Lap_h Pp, zero-flux in z
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
  // electrostatic term: -E, E = -G_h phi with Dirichlet ghosts
  if (cf.terms & kElec) {
    const T zp = (k + 1 < d.nz) ? phi[n + pl] : ghost_top[i + (int64_t)d.nx * j];
    const T zm = (k > 0) ? phi[n - pl] : cf.phi_bottom;
    F[0] += (phi[nbr(d, i, j, k, 1, 0, 0)] - phi[nbr(d, i, j, k, -1, 0, 0)]) * cf.inv_2h;
    F[1] += (phi[nbr(d, i, j, k, 0, 1, 0)] - phi[nbr(d, i, j, k, 0, -1, 0)]) * cf.inv_2h;
    F[2] += (zp - zm) * cf.inv_2h;
  }
  // elastic term: -h^-3 s . deps0/dP
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
    // deps0/dP contracted with s
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

template <typename T>
hipError_t launch_poisson_setup(const Dims& d, const Coefs<T>& cf, const T* P, const T* V, T cdt, int with_P,
                                int with_bc, const T* ghost_top, T phi_bottom, const T* x, T* r, T* p,
                                CgScalars* sc, double* partials, double tol, int maxit, hipStream_t s) {
  poisson_setup_kernel<T><<<node_grid(d), node_block(), 0, s>>>(d, cf, P, V, cdt, with_P, with_bc, ghost_top,
                                                                phi_bottom, x, r, p, sc, partials, node_blocks(d),
                                                                tol, maxit);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_poisson_cg_a(const Dims& d, const Coefs<T>& cf, const T* r, const T* p_old, T* p_new, T* x,
                               CgScalars* sc, double* partials, hipStream_t s) {
  poisson_cg_a_kernel<T><<<node_grid(d), node_block(), 0, s>>>(d, cf, r, p_old, p_new, x, sc, partials,
                                                               node_blocks(d));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_poisson_cg_b(const Dims& d, const Coefs<T>& cf, const T* p, T* r, CgScalars* sc, double* partials,
                               hipStream_t s) {
  poisson_cg_b_kernel<T><<<node_grid(d), node_block(), 0, s>>>(d, cf, p, r, sc, partials, node_blocks(d));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fem_setup(const Dims& d, const Coefs<T>& cf, const FemTables* tb, const T* P, const T* V, T cdt,
                            T* x, T* r, T* p0, T* p1, CgScalars* sc, double* partials, double tol, int maxit,
                            hipStream_t s) {
  fem_setup_kernel<T><<<node_grid(d), node_block(), 0, s>>>(d, cf, tb, P, V, cdt, x, r, p0, p1, sc, partials,
                                                            node_blocks(d), tol, maxit);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fem_cg_a(const Dims& d, const Coefs<T>& cf, const FemTables* tb, const T* r, const T* p_old,
                           T* p_new, T* x, CgScalars* sc, double* partials, hipStream_t s) {
  fem_cg_a_kernel<T><<<node_grid(d), node_block(), 0, s>>>(d, cf, tb, r, p_old, p_new, x, sc, partials,
                                                           node_blocks(d));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fem_cg_b(const Dims& d, const Coefs<T>& cf, const FemTables* tb, const T* p, T* r, CgScalars* sc,
                           double* partials, hipStream_t s) {
  fem_cg_b_kernel<T><<<node_grid(d), node_block(), 0, s>>>(d, cf, tb, p, r, sc, partials, node_blocks(d));
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
  template hipError_t launch_poisson_setup<T>(const Dims&, const Coefs<T>&, const T*, const T*, T, int, int,     \
                                              const T*, T, const T*, T*, T*, CgScalars*, double*, double, int,   \
                                              hipStream_t);                                                      \
  template hipError_t launch_poisson_cg_a<T>(const Dims&, const Coefs<T>&, const T*, const T*, T*, T*,           \
                                             CgScalars*, double*, hipStream_t);                                  \
  template hipError_t launch_poisson_cg_b<T>(const Dims&, const Coefs<T>&, const T*, T*, CgScalars*, double*,    \
                                             hipStream_t);                                                       \
  template hipError_t launch_fem_setup<T>(const Dims&, const Coefs<T>&, const FemTables*, const T*, const T*, T, \
                                          T*, T*, T*, T*, CgScalars*, double*, double, int, hipStream_t);        \
  template hipError_t launch_fem_cg_a<T>(const Dims&, const Coefs<T>&, const FemTables*, const T*, const T*, T*, \
                                         T*, CgScalars*, double*, hipStream_t);                                  \
  template hipError_t launch_fem_cg_b<T>(const Dims&, const Coefs<T>&, const FemTables*, const T*, T*,           \
                                         CgScalars*, double*, hipStream_t);                                      \
  template hipError_t launch_force<T>(const Dims&, const Coefs<T>&, const FemTables*, const T*, const T*, T,     \
                                      const T*, const T*, const T*, int, T*, T*, T*, hipStream_t);

PF_INSTANTIATE(double)
PF_INSTANTIATE(float)
template hipError_t launch_convert<double, float>(const double*, float*, int64_t, hipStream_t);
template hipError_t launch_convert<float, double>(const float*, double*, int64_t, hipStream_t);

}  // namespace pf
