/*
 * pf_oracle.c -- plain FP64 CPU oracle for the time-domain ferroelectric
 * phase-field step of Ashraf & Salahuddin, "A Massively Parallel Time Domain
 * Phase Field Model for Multi-domain Ferroelectric Device Simulation"
 * (arXiv:1202.6116).
 *
 * TEST INFRASTRUCTURE.  This file is the independent reference that the GPU
 * library is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it.  It shares no code, header,
 * table or constant with the GPU library, and it is deliberately plain: every
 * operator is written out the way the paper (or the reading of it stated
 * next to the code) defines it, with no blocking, fusion or reordering.
 *
 * Equation numbers count the paper's displayed equations in order:
 * Eq. 1 bulk Landau energy, Eq. 2-3 gradient energy and its variation,
 * Eq. 4-5 electrostatic energy and field, Eq. 6 elastic energy, Eq. 7 TDGL,
 * Eq. 8-14 iso-parametric brick element (shape derivatives, node matrix,
 * Jacobian, physical derivatives, strain-displacement B, stiffness C,
 * element stiffness), Eq. 15 eigenstrain and body force, Eq. 16 K du = F,
 * Eq. 17-18 charge and Poisson, Eq. 19 predictor-corrector.
 *
 * Discrete conventions (readings of the paper, each listed in the design
 * notes):
 *   grid       node (i,j,k), n = i + nx*(j + ny*k), spacing h, periodic in
 *              x and y (Sec. III.B.4), k = 0 substrate side, k = nz-1 top.
 *              FD and FEM share the nodes (Sec. III.A, Fig. 1b).
 *   fields     structure of arrays: component c of node n at [c*N + n].
 *   Voigt      (xx, yy, zz, xy, yz, zx), engineering shear (rows of Eq. 12);
 *              the tensor eigenstrain Q44 Pi Pj becomes 2 Q44 Pi Pj.
 *   energy     F = F_bulk + F_grad + F_elec + F_elas, force F_n =
 *              -(L/h^3) dF/dP_n (Eq. 7 with a mobility L, no noise).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Parameters                                                                */
/* ------------------------------------------------------------------------ */

enum { OR_OK = 0, OR_EINVAL = -1, OR_ENOMEM = -2, OR_ENOCONV = -4, OR_ENONFINITE = -5 };
enum { OR_TERM_LANDAU = 1, OR_TERM_GRAD = 2, OR_TERM_ELEC = 4, OR_TERM_ELAS = 8 };
enum { OR_INT_PC = 0, OR_INT_EULER = 1 };
enum { OR_TOP_METAL = 0, OR_TOP_OPEN = 1 };

typedef struct {
    int32_t nx, ny, nz;
    double h;
    double a1, a11, a12;          /* Landau coefficients, Eq. 1 */
    double G;                     /* gradient coefficient G11, Eq. 2-3 */
    double L;                     /* mobility in Eq. 7 */
    double dt;                    /* time step, Eq. 19 */
    double eps_b;                 /* permittivity in Eq. 18 */
    double phi_bottom, phi_top;   /* Dirichlet values on the ghost planes */
    double C11, C12, C44;         /* cubic stiffness (Eq. 13 generalised) */
    double Q11, Q12, Q44;         /* electrostriction, Eq. 15 */
    int32_t n_el;                 /* electrodes on the top ghost plane */
    const int32_t *el_box;        /* n_el x {x0, x1, y0, y1}, half-open node ranges */
    const double *el_volts;       /* n_el voltages */
    int32_t integrator;           /* OR_INT_PC or OR_INT_EULER */
    int32_t maxit;                /* CG iteration cap */
    double tol_phi, tol_u;        /* relative residual tolerances */
    int32_t warm_start;           /* 0 cold, 1 previous solution, 2 extrapolated from earlier solutions */
    uint32_t terms;               /* OR_TERM_* mask */
    int32_t nonlocal_every;       /* recompute phi and u every k steps (<= 1: every step) */
    int32_t extrap_order;         /* warm_start 2: extrapolate from up to this many earlier solutions */
    double noise_sigma;           /* thermal noise amplitude (zeta of Eq. 7), 0: none */
    uint64_t noise_seed;          /* key of the noise generator */
    int32_t top_bc;               /* OR_TOP_METAL: Dirichlet ghost plane above the film;
                                     OR_TOP_OPEN: n_air air planes, zero normal field on top */
    int32_t n_air;                /* air planes of the potential grid (open top) */
    double eps_air;               /* permittivity of the air planes (open top) */
    double misfit[3];             /* substrate strain imposed on the film: xx, yy and engineering
                                     xy, grid frame (the clamp then holds an affine displacement) */
    double rot[9];                /* crystal-to-grid rotation R, row-major: v_grid = R v_crystal */
    /* derived by or_prepare from the crystal coefficients and R: */
    double Cg[36];                /* stiffness in the grid frame, Voigt 6x6 */
    double Qv[6][3][3];           /* eps0_v = P^T Qv[v] P (grid frame, engineering shear) */
} or_params;

typedef struct {
    int64_t iters_phi, iters_u;   /* CG iterations summed over the call */
    int32_t last_iters_phi, last_iters_u;
    double relres_phi, relres_u;  /* largest final relative residual in the call */
    int32_t nsolves_phi, nsolves_u;
} or_stats;

static inline int64_t nnodes(const or_params *p) { return (int64_t)p->nx * p->ny * p->nz; }

/* The potential grid: the film planes k < nz and, with the open top, n_air
 * air planes above them (Sec. III.C and IV: the open-circuit film carries
 * air layers with a Neumann condition on top). */
static inline int open_top(const or_params *p) { return p->top_bc == OR_TOP_OPEN; }
static inline int phi_planes(const or_params *p) { return p->nz + (open_top(p) ? p->n_air : 0); }
static inline int64_t nphi(const or_params *p) { return (int64_t)p->nx * p->ny * phi_planes(p); }

static inline int64_t node(const or_params *p, int i, int j, int k) {
    int nx = p->nx, ny = p->ny;
    if (i < 0 || i >= nx) i = ((i % nx) + nx) % nx;    /* periodic x */
    if (j < 0 || j >= ny) j = ((j % ny) + ny) % ny;    /* periodic y */
    return (int64_t)i + (int64_t)nx * ((int64_t)j + (int64_t)ny * k);
}

/* Deterministic FP64 dot product: fixed-size chunks summed in index order,
 * chunk sums added in chunk order, so the result does not depend on the
 * number of threads. */
#define OR_CHUNK 4096
static double dot(const double *a, const double *b, int64_t n) {
    int64_t nch = (n + OR_CHUNK - 1) / OR_CHUNK;
    double *part = (double *)malloc(sizeof(double) * (size_t)(nch > 0 ? nch : 1));
    #pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nch; c++) {
        int64_t lo = c * OR_CHUNK, hi = lo + OR_CHUNK < n ? lo + OR_CHUNK : n;
        double s = 0.0;
        for (int64_t t = lo; t < hi; t++) s += a[t] * b[t];
        part[c] = s;
    }
    double s = 0.0;
    for (int64_t c = 0; c < nch; c++) s += part[c];
    free(part);
    return s;
}

/* ------------------------------------------------------------------------ */
/* Crystal and grid frames                                                   */
/* ------------------------------------------------------------------------ */
/* The Landau coefficients, C and Q are given on the crystal axes; the grid
 * axes are R times them (Sec. II distinguishes crystal directions from grid
 * directions).  P is held on the grid axes: its crystal components are
 * R^T P.  Voigt order (xx, yy, zz, xy, yz, zx).                              */

static const int voigt_i[6] = {0, 1, 2, 0, 1, 2}, voigt_j[6] = {0, 1, 2, 1, 2, 0};

/* Cubic fourth-order tensors: T_iiii = d11, T_iijj = d12 (i != j),
 * T_ijij = T_ijji = d44 (i != j). */
static double cubic_tensor(double d11, double d12, double d44, int i, int j, int k, int l) {
    if (i == j && k == l) return i == k ? d11 : d12;
    if (i != j && ((i == k && j == l) || (i == l && j == k))) return d44;
    return 0.0;
}

/* T'_ijkl = R_ia R_jb R_kc R_ld T_abcd. */
static double rotated(const double R[9], double d11, double d12, double d44, int i, int j, int k, int l) {
    double s = 0;
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++)
            for (int c = 0; c < 3; c++)
                for (int d = 0; d < 3; d++) {
                    double t = cubic_tensor(d11, d12, d44, a, b, c, d);
                    if (t != 0) s += R[3 * i + a] * R[3 * j + b] * R[3 * k + c] * R[3 * l + d] * t;
                }
    return s;
}

/* Fills the grid-frame stiffness (Voigt, tensor stress against engineering
 * strain: C_vw = C'_{ij kl}) and the electrostriction forms: the tensor
 * eigenstrain is eps0_ij = Q'_ijkl P_k P_l with the crystal Q_iiii = Q11,
 * Q_iijj = Q12 and Q_ijij = Q_ijji = Q44/2 (so that eps0_ij = Q44 Pi Pj on
 * the crystal axes, Eq. 15); the engineering shear doubles it. */
void or_prepare(or_params *p) {
    for (int v = 0; v < 6; v++)
        for (int w = 0; w < 6; w++)
            p->Cg[6 * v + w] = rotated(p->rot, p->C11, p->C12, p->C44, voigt_i[v], voigt_j[v], voigt_i[w], voigt_j[w]);
    for (int v = 0; v < 6; v++) {
        double scale = v < 3 ? 1.0 : 2.0;
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                double qab = rotated(p->rot, p->Q11, p->Q12, 0.5 * p->Q44, voigt_i[v], voigt_j[v], a, b);
                double qba = rotated(p->rot, p->Q11, p->Q12, 0.5 * p->Q44, voigt_i[v], voigt_j[v], b, a);
                p->Qv[v][a][b] = scale * 0.5 * (qab + qba);
            }
    }
}

static void to_crystal(const or_params *p, const double P[3], double c[3]) {
    for (int a = 0; a < 3; a++) c[a] = p->rot[a] * P[0] + p->rot[3 + a] * P[1] + p->rot[6 + a] * P[2];
}

static void to_grid(const or_params *p, const double c[3], double P[3]) {
    for (int i = 0; i < 3; i++) P[i] = p->rot[3 * i] * c[0] + p->rot[3 * i + 1] * c[1] + p->rot[3 * i + 2] * c[2];
}

/* ------------------------------------------------------------------------ */
/* Landau energy (Eq. 1) and its derivatives                                 */
/* ------------------------------------------------------------------------ */
/* Eq. 1 on the crystal components p = R^T P.                                */

static double landau_energy_density(const or_params *p, double X, double Y, double Z) {
    double P[3] = {X, Y, Z}, c[3];
    to_crystal(p, P, c);
    double x2 = c[0] * c[0], y2 = c[1] * c[1], z2 = c[2] * c[2];
    return p->a1 * (x2 + y2 + z2) + p->a11 * (x2 * x2 + y2 * y2 + z2 * z2)
         + p->a12 * (x2 * y2 + y2 * z2 + z2 * x2);
}

/* Crystal frame: dF_bulk/dp_x = 2 a1 px + 4 a11 px^3 + 2 a12 px (py^2 + pz^2),
 * cyclic; the grid-frame gradient is R times it. */
static void landau_gradient(const or_params *p, double X, double Y, double Z, double g[3]) {
    double P[3] = {X, Y, Z}, c[3], gc[3];
    to_crystal(p, P, c);
    double x = c[0], y = c[1], z = c[2], x2 = x * x, y2 = y * y, z2 = z * z;
    gc[0] = 2 * p->a1 * x + 4 * p->a11 * x2 * x + 2 * p->a12 * x * (y2 + z2);
    gc[1] = 2 * p->a1 * y + 4 * p->a11 * y2 * y + 2 * p->a12 * y * (z2 + x2);
    gc[2] = 2 * p->a1 * z + 4 * p->a11 * z2 * z + 2 * p->a12 * z * (x2 + y2);
    to_grid(p, gc, g);
}

/* Second derivatives of Eq. 1: R Hc R^T with the crystal-frame Hessian Hc. */
static void landau_hessian(const or_params *p, double X, double Y, double Z, double H[3][3]) {
    double P[3] = {X, Y, Z}, c[3], Hc[3][3];
    to_crystal(p, P, c);
    double x = c[0], y = c[1], z = c[2], x2 = x * x, y2 = y * y, z2 = z * z;
    Hc[0][0] = 2 * p->a1 + 12 * p->a11 * x2 + 2 * p->a12 * (y2 + z2);
    Hc[1][1] = 2 * p->a1 + 12 * p->a11 * y2 + 2 * p->a12 * (z2 + x2);
    Hc[2][2] = 2 * p->a1 + 12 * p->a11 * z2 + 2 * p->a12 * (x2 + y2);
    Hc[0][1] = Hc[1][0] = 4 * p->a12 * x * y;
    Hc[1][2] = Hc[2][1] = 4 * p->a12 * y * z;
    Hc[0][2] = Hc[2][0] = 4 * p->a12 * x * z;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0;
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++) s += p->rot[3 * i + a] * Hc[a][b] * p->rot[3 * j + b];
            H[i][j] = s;
        }
}

/* ------------------------------------------------------------------------ */
/* Electrostriction (Eq. 15, first two lines)                                */
/* ------------------------------------------------------------------------ */

/* Voigt eigenstrain of one polarisation vector (grid frame, engineering
 * shear), eps0_v = P^T Qv[v] P. */
static void eigenstrain(const or_params *p, double x, double y, double z, double e[6]) {
    double P[3] = {x, y, z};
    for (int v = 0; v < 6; v++) {
        double s = 0;
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) s += p->Qv[v][a][b] * P[a] * P[b];
        e[v] = s;
    }
}

/* D[v][d] = d eps0_v / d P_d = 2 (Qv[v] P)_d. */
static void eigenstrain_jacobian(const or_params *p, double x, double y, double z, double D[6][3]) {
    double P[3] = {x, y, z};
    for (int v = 0; v < 6; v++)
        for (int d = 0; d < 3; d++) D[v][d] = 2 * (p->Qv[v][d][0] * P[0] + p->Qv[v][d][1] * P[1] + p->Qv[v][d][2] * P[2]);
}

/* Second derivative contracted with a stress and a direction:
 * out[d] = sum_v s_v * sum_e d^2 eps0_v / dP_d dP_e * lam_e = sum_v s_v 2 (Qv[v] lam)_d. */
static void eigenstrain_hessian_apply(const or_params *p, const double s[6], const double lam[3], double out[3]) {
    for (int d = 0; d < 3; d++) {
        double a = 0;
        for (int v = 0; v < 6; v++)
            a += s[v] * 2 * (p->Qv[v][d][0] * lam[0] + p->Qv[v][d][1] * lam[1] + p->Qv[v][d][2] * lam[2]);
        out[d] = a;
    }
}

/* ------------------------------------------------------------------------ */
/* Iso-parametric linear brick element (Eq. 8-14)                            */
/* ------------------------------------------------------------------------ */
/* Local node a = ai + 2 aj + 4 ak (ai, aj, ak in {0,1}) sits at natural
 * coordinates (2ai-1, 2aj-1, 2ak-1) and, in real space, at the corners
 * (+-h/2, +-h/2, +-h/2) of a cube of side h. Element dofs are node-major:
 * dof 3a + c is component c of local node a.                               */

static int corner_sign(int a, int axis) { return ((a >> axis) & 1) ? 1 : -1; }

/* Shape functions N_a(zeta, beta, eta) = (1 + zeta_a zeta)(1 + beta_a beta)(1 + eta_a eta)/8. */
static void shape_values(const double q[3], double N[8]) {
    for (int a = 0; a < 8; a++)
        N[a] = (1 + corner_sign(a, 0) * q[0]) * (1 + corner_sign(a, 1) * q[1]) * (1 + corner_sign(a, 2) * q[2]) / 8.0;
}

/* Eq. 8: dN_a / d(zeta, beta, eta), an 8x3 matrix. */
static void shape_natural_derivatives(const double q[3], double dN[8][3]) {
    for (int a = 0; a < 8; a++) {
        double s0 = corner_sign(a, 0), s1 = corner_sign(a, 1), s2 = corner_sign(a, 2);
        dN[a][0] = s0 * (1 + s1 * q[1]) * (1 + s2 * q[2]) / 8.0;
        dN[a][1] = s1 * (1 + s0 * q[0]) * (1 + s2 * q[2]) / 8.0;
        dN[a][2] = s2 * (1 + s0 * q[0]) * (1 + s1 * q[1]) / 8.0;
    }
}

/* Eq. 13 generalised to cubic symmetry (isotropic is C11 - C12 = 2 C44),
 * on the grid axes (or_prepare). */
static void stiffness_matrix(const or_params *p, double C[6][6]) {
    for (int r = 0; r < 6; r++)
        for (int c = 0; c < 6; c++) C[r][c] = p->Cg[6 * r + c];
}

/* For one quadrature point q: Eq. 9-12.  Returns |J| and fills B (6x24) and N. */
static double element_point(const or_params *p, const double q[3], double B[6][24], double N[8]) {
    double dN[8][3], R[8][3], J[3][3], Ji[3][3], dX[3][8];
    shape_natural_derivatives(q, dN);
    shape_values(q, N);
    for (int a = 0; a < 8; a++)                         /* Eq. 9: node coordinates */
        for (int c = 0; c < 3; c++) R[a][c] = corner_sign(a, c) * 0.5 * p->h;
    for (int r = 0; r < 3; r++)                         /* Eq. 10: J = (dN/dzeta)^T R */
        for (int c = 0; c < 3; c++) {
            double s = 0;
            for (int a = 0; a < 8; a++) s += dN[a][r] * R[a][c];
            J[r][c] = s;
        }
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
               - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
               + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    for (int r = 0; r < 3; r++)                         /* Eq. 11: dN/dX = J^-1 (dN/dzeta)^T */
        for (int a = 0; a < 8; a++) {
            double s = 0;
            for (int c = 0; c < 3; c++) s += Ji[r][c] * dN[a][c];
            dX[r][a] = s;
        }
    memset(B, 0, sizeof(double) * 6 * 24);              /* Eq. 12 */
    for (int a = 0; a < 8; a++) {
        double dx = dX[0][a], dy = dX[1][a], dz = dX[2][a];
        B[0][3 * a + 0] = dx;
        B[1][3 * a + 1] = dy;
        B[2][3 * a + 2] = dz;
        B[3][3 * a + 0] = dy; B[3][3 * a + 1] = dx;
        B[4][3 * a + 1] = dz; B[4][3 * a + 2] = dy;
        B[5][3 * a + 0] = dz; B[5][3 * a + 2] = dx;
    }
    return fabs(det);
}

/* The eight 2x2x2 Gauss points at +-1/sqrt(3), weight 1 (Eq. 14). */
static void gauss_point(int g, double q[3]) {
    double r = 1.0 / sqrt(3.0);
    q[0] = (g & 1) ? r : -r;
    q[1] = (g & 2) ? r : -r;
    q[2] = (g & 4) ? r : -r;
}

/* Eq. 14: Ke = sum_g |J| B_g^T C B_g. */
void or_element_stiffness(const or_params *p, double *Ke) {
    double C[6][6], B[6][24], N[8];
    stiffness_matrix(p, C);
    memset(Ke, 0, sizeof(double) * 576);
    for (int g = 0; g < 8; g++) {
        double q[3];
        gauss_point(g, q);
        double detJ = element_point(p, q, B, N);
        double CB[6][24];
        for (int r = 0; r < 6; r++)
            for (int c = 0; c < 24; c++) {
                double s = 0;
                for (int t = 0; t < 6; t++) s += C[r][t] * B[t][c];
                CB[r][c] = s;
            }
        for (int r = 0; r < 24; r++)
            for (int c = 0; c < 24; c++) {
                double s = 0;
                for (int t = 0; t < 6; t++) s += B[t][r] * CB[t][c];
                Ke[r * 24 + c] += detJ * s;
            }
    }
}

/* Eq. 15, third line: element body force f_e = sum_g |J| B_g^T C eps0_g with
 * the nodal eigenstrains interpolated to the Gauss points by the shape
 * functions (the eigenstrain is a nodal quantity, Sec. III.A). */
static void element_body_force(const or_params *p, const double e0[8][6], double f[24]) {
    double C[6][6], B[6][24], N[8];
    stiffness_matrix(p, C);
    memset(f, 0, sizeof(double) * 24);
    for (int g = 0; g < 8; g++) {
        double q[3];
        gauss_point(g, q);
        double detJ = element_point(p, q, B, N);
        double eg[6] = {0, 0, 0, 0, 0, 0}, sg[6];
        for (int b = 0; b < 8; b++)
            for (int v = 0; v < 6; v++) eg[v] += N[b] * e0[b][v];
        for (int r = 0; r < 6; r++) {
            double s = 0;
            for (int t = 0; t < 6; t++) s += C[r][t] * eg[t];
            sg[r] = s;
        }
        for (int c = 0; c < 24; c++) {
            double s = 0;
            for (int r = 0; r < 6; r++) s += B[r][c] * sg[r];
            f[c] += detJ * s;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Element topology                                                          */
/* ------------------------------------------------------------------------ */
/* Element (ci, cj, ck), 0 <= ck <= nz-2, joins the nodes (ci+bi, cj+bj,
 * ck+bk), wrapped in x and y.  A node (i,j,k) belongs to the elements with
 * corner (i-ai, j-aj, k-ak) that exist; it is their local node a.          */

static int64_t element_node(const or_params *p, int ci, int cj, int ck, int b) {
    return node(p, ci + (b & 1), cj + ((b >> 1) & 1), ck + ((b >> 2) & 1));
}

static int element_exists(const or_params *p, int ck) { return ck >= 0 && ck <= p->nz - 2; }

/* Nodal eigenstrain field (Voigt, e0[v*N + n]) of a polarisation field,
 * relative to the substrate strain. */
void or_nodal_eigenstrain(const or_params *p, const double *P, double *e0) {
    int64_t N = nnodes(p);
    /* The substrate holds the film at the in-plane strain eps_s: with the
     * affine displacement of that strain split off (the clamp then holds
     * u = 0), the elastic strain is B u - (eps0 - eps_s).                   */
    const double es[6] = {p->misfit[0], p->misfit[1], 0.0, p->misfit[2], 0.0, 0.0};
    #pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; n++) {
        double e[6];
        eigenstrain(p, P[n], P[N + n], P[2 * N + n], e);
        for (int v = 0; v < 6; v++) e0[v * N + n] = e[v] - es[v];
    }
}

/* Nodal eigenstrains of the 8 nodes of an element. */
static void element_eigenstrains(const or_params *p, const double *e0n, int ci, int cj, int ck, double e0[8][6]) {
    int64_t N = nnodes(p);
    for (int b = 0; b < 8; b++) {
        int64_t m = element_node(p, ci, cj, ck, b);
        for (int v = 0; v < 6; v++) e0[b][v] = e0n[v * N + m];
    }
}

/* ------------------------------------------------------------------------ */
/* FEM operator, node-wise (Sec. III.B.2 steps i-vi)                         */
/* ------------------------------------------------------------------------ */
/* Row of node n: gather, over the (up to) 8 elements holding n, the row of
 * Ke that belongs to n's local index, against the element's 8 nodes.  The
 * clamped substrate plane k = 0 is eliminated symmetrically: its rows are
 * identity rows and its columns are dropped (Sec. III.B.4).                */

void or_fem_apply(const or_params *p, const double *Ke, const double *u, double *Ku) {
    int64_t N = nnodes(p);
    #pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; n++) {
        int i = (int)(n % p->nx), j = (int)((n / p->nx) % p->ny), k = (int)(n / ((int64_t)p->nx * p->ny));
        double acc[3] = {0, 0, 0};
        if (k == 0) {
            for (int c = 0; c < 3; c++) Ku[c * N + n] = u[c * N + n];
            continue;
        }
        for (int a = 0; a < 8; a++) {
            int ci = i - (a & 1), cj = j - ((a >> 1) & 1), ck = k - ((a >> 2) & 1);
            if (!element_exists(p, ck)) continue;
            for (int b = 0; b < 8; b++) {
                if (ck + ((b >> 2) & 1) == 0) continue;       /* clamped column */
                int64_t m = element_node(p, ci, cj, ck, b);
                for (int c = 0; c < 3; c++)
                    for (int d = 0; d < 3; d++)
                        acc[c] += Ke[(3 * a + c) * 24 + 3 * b + d] * u[d * N + m];
            }
        }
        for (int c = 0; c < 3; c++) Ku[c * N + n] = acc[c];
    }
}

/* Dense K (3N x 3N, row index c*N + n) assembled node-wise: for every node,
 * its 8 elements are recomputed locally and the node's own rows gathered.  */
void or_fem_assemble_nodewise(const or_params *p, double *K) {
    int64_t N = nnodes(p), D = 3 * N;
    double Ke[576];
    or_element_stiffness(p, Ke);
    memset(K, 0, sizeof(double) * (size_t)(D * D));
    for (int64_t n = 0; n < N; n++) {                    /* step i */
        int i = (int)(n % p->nx), j = (int)((n / p->nx) % p->ny), k = (int)(n / ((int64_t)p->nx * p->ny));
        for (int a = 0; a < 8; a++) {                      /* step iii */
            int ci = i - (a & 1), cj = j - ((a >> 1) & 1), ck = k - ((a >> 2) & 1);
            if (!element_exists(p, ck)) continue;
            for (int b = 0; b < 8; b++) {                  /* steps iv-v */
                int64_t m = element_node(p, ci, cj, ck, b);   /* step ii: column node */
                for (int c = 0; c < 3; c++)                    /* step vi */
                    for (int d = 0; d < 3; d++)
                        K[(c * N + n) * D + d * N + m] += Ke[(3 * a + c) * 24 + 3 * b + d];
            }
        }
    }
    for (int64_t n = 0; n < N; n++) {                    /* clamp k = 0 symmetrically */
        if (n / ((int64_t)p->nx * p->ny) != 0) continue;
        for (int c = 0; c < 3; c++) {
            int64_t r = c * N + n;
            for (int64_t t = 0; t < D; t++) { K[r * D + t] = 0; K[t * D + r] = 0; }
            K[r * D + r] = 1;
        }
    }
}

/* Dense K assembled element by element (the scatter the paper started from). */
void or_fem_assemble_elementwise(const or_params *p, double *K) {
    int64_t N = nnodes(p), D = 3 * N;
    double Ke[576];
    or_element_stiffness(p, Ke);
    memset(K, 0, sizeof(double) * (size_t)(D * D));
    for (int ck = 0; ck <= p->nz - 2; ck++)
        for (int cj = 0; cj < p->ny; cj++)
            for (int ci = 0; ci < p->nx; ci++)
                for (int a = 0; a < 8; a++)
                    for (int b = 0; b < 8; b++) {
                        int64_t na = element_node(p, ci, cj, ck, a), nb = element_node(p, ci, cj, ck, b);
                        for (int c = 0; c < 3; c++)
                            for (int d = 0; d < 3; d++)
                                K[(c * N + na) * D + d * N + nb] += Ke[(3 * a + c) * 24 + 3 * b + d];
                    }
    for (int64_t n = 0; n < (int64_t)p->nx * p->ny; n++)
        for (int c = 0; c < 3; c++) {
            int64_t r = c * N + n;
            for (int64_t t = 0; t < D; t++) { K[r * D + t] = 0; K[t * D + r] = 0; }
            K[r * D + r] = 1;
        }
}

/* Jacobi diagonal of the clamped K, gathered node-wise like or_fem_apply. */
void or_fem_diagonal(const or_params *p, const double *Ke, double *diag) {
    int64_t N = nnodes(p);
    #pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; n++) {
        int k = (int)(n / ((int64_t)p->nx * p->ny));
        for (int c = 0; c < 3; c++) {
            double s = 0;
            if (k == 0) s = 1;
            else
                for (int a = 0; a < 8; a++)
                    if (element_exists(p, k - ((a >> 2) & 1))) s += Ke[(3 * a + c) * 24 + 3 * a + c];
            diag[c * N + n] = s;
        }
    }
}

/* Right-hand side of Eq. 16: nodal forces of Eq. 15 gathered node-wise over
 * the elements holding each node; zero on the clamped rows.                 */
void or_fem_rhs_e0(const or_params *p, const double *e0n, double *f) {
    int64_t N = nnodes(p);
    #pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; n++) {
        int i = (int)(n % p->nx), j = (int)((n / p->nx) % p->ny), k = (int)(n / ((int64_t)p->nx * p->ny));
        double acc[3] = {0, 0, 0};
        if (k > 0)
            for (int a = 0; a < 8; a++) {
                int ci = i - (a & 1), cj = j - ((a >> 1) & 1), ck = k - ((a >> 2) & 1);
                if (!element_exists(p, ck)) continue;
                double e0[8][6], fe[24];
                element_eigenstrains(p, e0n, ci, cj, ck, e0);
                element_body_force(p, e0, fe);
                for (int c = 0; c < 3; c++) acc[c] += fe[3 * a + c];
            }
        for (int c = 0; c < 3; c++) f[c * N + n] = acc[c];
    }
}

/* Stress returned to the nodes (how the total strain comes back to the FD
 * nodes, Sec. III.A): s_n = sum_{e holding n} sum_g |J| N_a(g) C (B_g u_e -
 * eps0_g), a Voigt 6-vector per node (s[v*N + n]).  s_n . d eps0/dP is
 * minus the derivative of the elastic energy with respect to P_n.        */
void or_stress_gather_e0(const or_params *p, const double *e0n, const double *u, double *s) {
    int64_t N = nnodes(p);
    double C[6][6];
    stiffness_matrix(p, C);
    #pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; n++) {
        int i = (int)(n % p->nx), j = (int)((n / p->nx) % p->ny), k = (int)(n / ((int64_t)p->nx * p->ny));
        double acc[6] = {0, 0, 0, 0, 0, 0};
        for (int a = 0; a < 8; a++) {
            int ci = i - (a & 1), cj = j - ((a >> 1) & 1), ck = k - ((a >> 2) & 1);
            if (!element_exists(p, ck)) continue;
            double e0[8][6], ue[24];
            element_eigenstrains(p, e0n, ci, cj, ck, e0);
            for (int b = 0; b < 8; b++) {
                int64_t m = element_node(p, ci, cj, ck, b);
                for (int d = 0; d < 3; d++) ue[3 * b + d] = u[d * N + m];
            }
            for (int g = 0; g < 8; g++) {
                double q[3], B[6][24], Nv[8], el[6];
                gauss_point(g, q);
                double detJ = element_point(p, q, B, Nv);
                for (int v = 0; v < 6; v++) {
                    double bu = 0, eg = 0;
                    for (int c = 0; c < 24; c++) bu += B[v][c] * ue[c];
                    for (int b = 0; b < 8; b++) eg += Nv[b] * e0[b][v];
                    el[v] = bu - eg;
                }
                for (int r = 0; r < 6; r++) {
                    double sg = 0;
                    for (int t = 0; t < 6; t++) sg += C[r][t] * el[t];
                    acc[r] += detJ * Nv[a] * sg;
                }
            }
        }
        for (int v = 0; v < 6; v++) s[v * N + n] = acc[v];
    }
}

/* Elastic energy (Eq. 6 read as 1/2 (eps - eps0)^T C (eps - eps0)) summed
 * over elements and Gauss points for a given displacement field.            */
double or_elastic_energy_e0(const or_params *p, const double *e0n, const double *u) {
    int64_t N = nnodes(p);
    int64_t ne = (int64_t)p->nx * p->ny * (p->nz - 1);
    double C[6][6];
    stiffness_matrix(p, C);
    double *pe = (double *)malloc(sizeof(double) * (size_t)(ne > 0 ? ne : 1));
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < ne; e++) {
        int ci = (int)(e % p->nx), cj = (int)((e / p->nx) % p->ny), ck = (int)(e / ((int64_t)p->nx * p->ny));
        double e0[8][6], ue[24], acc = 0;
        element_eigenstrains(p, e0n, ci, cj, ck, e0);
        for (int b = 0; b < 8; b++) {
            int64_t m = element_node(p, ci, cj, ck, b);
            for (int d = 0; d < 3; d++) ue[3 * b + d] = u[d * N + m];
        }
        for (int g = 0; g < 8; g++) {
            double q[3], B[6][24], Nv[8], el[6];
            gauss_point(g, q);
            double detJ = element_point(p, q, B, Nv);
            for (int v = 0; v < 6; v++) {
                double bu = 0, eg = 0;
                for (int c = 0; c < 24; c++) bu += B[v][c] * ue[c];
                for (int b = 0; b < 8; b++) eg += Nv[b] * e0[b][v];
                el[v] = bu - eg;
            }
            for (int r = 0; r < 6; r++) {
                double sg = 0;
                for (int t = 0; t < 6; t++) sg += C[r][t] * el[t];
                acc += 0.5 * detJ * el[r] * sg;
            }
        }
        pe[e] = acc;
    }
    double tot = 0;
    for (int64_t e = 0; e < ne; e++) tot += pe[e];
    free(pe);
    return tot;
}

/* The same three operators for the eigenstrain field of a polarisation. */
static double *nodal_eigenstrain_alloc(const or_params *p, const double *P) {
    double *e0n = (double *)malloc(sizeof(double) * (size_t)(6 * nnodes(p)));
    if (e0n) or_nodal_eigenstrain(p, P, e0n);
    return e0n;
}

int or_fem_rhs(const or_params *p, const double *P, double *f) {
    double *e0n = nodal_eigenstrain_alloc(p, P);
    if (!e0n) return OR_ENOMEM;
    or_fem_rhs_e0(p, e0n, f);
    free(e0n);
    return OR_OK;
}

int or_stress_gather(const or_params *p, const double *P, const double *u, double *s) {
    double *e0n = nodal_eigenstrain_alloc(p, P);
    if (!e0n) return OR_ENOMEM;
    or_stress_gather_e0(p, e0n, u, s);
    free(e0n);
    return OR_OK;
}

double or_elastic_energy(const or_params *p, const double *P, const double *u) {
    double *e0n = nodal_eigenstrain_alloc(p, P);
    if (!e0n) return NAN;
    double v = or_elastic_energy_e0(p, e0n, u);
    free(e0n);
    return v;
}

/* ------------------------------------------------------------------------ */
/* Finite differences: divergence, gradient, Laplacians (Eq. 3, 17-18)       */
/* ------------------------------------------------------------------------ */

/* Value of the top ghost plane k = nz at column (i, j): the voltage of the
 * electrode covering it, otherwise phi_top (Sec. III.C, Dirichlet).  With
 * the open top the plane k = nz is the first air plane and only its
 * electrode nodes are Dirichlet (value: the electrode voltage). */
double or_top_ghost(const or_params *p, int i, int j) {
    for (int e = 0; e < p->n_el; e++) {
        const int32_t *b = p->el_box + 4 * e;
        if (i >= b[0] && i < b[1] && j >= b[2] && j < b[3]) return p->el_volts[e];
    }
    return p->phi_top;
}

/* Node (i, j, k) of the potential grid is an electrode node of the open top. */
static int is_electrode(const or_params *p, int i, int j, int k) {
    if (!open_top(p) || k != p->nz) return 0;
    i = ((i % p->nx) + p->nx) % p->nx;
    j = ((j % p->ny) + p->ny) % p->ny;
    for (int e = 0; e < p->n_el; e++) {
        const int32_t *b = p->el_box + 4 * e;
        if (i >= b[0] && i < b[1] && j >= b[2] && j < b[3]) return 1;
    }
    return 0;
}

/* Permittivity of plane k of the potential grid: eps_b in the film, eps_air
 * above it. */
static double plane_eps(const or_params *p, int k) { return k < p->nz ? p->eps_b : p->eps_air; }

/* Permittivity of the z-face between planes k and k + 1: the harmonic mean
 * of the two (flux continuity across a layered dielectric); k = -1 is the
 * face to the bottom ghost plane; above the top plane it is the face to the
 * top ghost plane (metal) or none (open: zero normal field). */
static double face_eps(const or_params *p, int k) {
    int top = phi_planes(p) - 1;
    if (k < 0) return plane_eps(p, 0);
    if (k >= top) return open_top(p) ? 0.0 : plane_eps(p, top);
    double a = plane_eps(p, k), b = plane_eps(p, k + 1);
    return a == b ? a : 2 * a * b / (a + b);
}

/* rho = D_h P on the potential grid: central differences, P = 0 outside the
 * film (planes k = -1 and k >= nz). */
void or_divergence(const or_params *p, const double *P, double *rho) {
    int64_t N = nnodes(p), M = nphi(p);
    double h = p->h;
    #pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < M; n++) {
        int i = (int)(n % p->nx), j = (int)((n / p->nx) % p->ny), k = (int)(n / ((int64_t)p->nx * p->ny));
        double dx = 0, dy = 0, zp = 0, zm = 0;
        if (k < p->nz) {
            dx = P[node(p, i + 1, j, k)] - P[node(p, i - 1, j, k)];
            dy = P[N + node(p, i, j + 1, k)] - P[N + node(p, i, j - 1, k)];
        }
        if (k + 1 < p->nz) zp = P[2 * N + node(p, i, j, k + 1)];
        if (k - 1 >= 0 && k - 1 < p->nz) zm = P[2 * N + node(p, i, j, k - 1)];
        rho[n] = (dx + dy + zp - zm) / (2 * h);
    }
}

/* E = -G_h phi at the film nodes with central differences.  with_ghosts = 1
 * uses the Dirichlet ghost values (phi_bottom below; above the film the top
 * ghost plane, or with the open top the air plane k = nz of phi); 0 uses zero
 * ghosts. */
void or_efield(const or_params *p, const double *phi, int with_ghosts, double *E) {
    int64_t N = nnodes(p);
    double h = p->h;
    int planes = phi_planes(p);
    #pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; n++) {
        int i = (int)(n % p->nx), j = (int)((n / p->nx) % p->ny), k = (int)(n / ((int64_t)p->nx * p->ny));
        double zp = (k + 1 < planes) ? phi[node(p, i, j, k + 1)] : (with_ghosts ? or_top_ghost(p, i, j) : 0.0);
        double zm = (k - 1 >= 0) ? phi[node(p, i, j, k - 1)] : (with_ghosts ? p->phi_bottom : 0.0);
        E[n] = -(phi[node(p, i + 1, j, k)] - phi[node(p, i - 1, j, k)]) / (2 * h);
        E[N + n] = -(phi[node(p, i, j + 1, k)] - phi[node(p, i, j - 1, k)]) / (2 * h);
        E[2 * N + n] = -(zp - zm) / (2 * h);
    }
}

/* A phi = -div_h(eps grad_h phi) on the unknown nodes of the potential grid,
 * with zero values on the Dirichlet ghost planes and electrode nodes (their
 * values enter the right-hand side) and no flux through the open top; rows
 * of electrode nodes are zero.  eps is constant (eps_b) with the metal top,
 * so A = -eps_b Lap_h there. */
void or_poisson_apply(const or_params *p, const double *phi, double *out) {
    int64_t M = nphi(p);
    double ih2 = 1.0 / (p->h * p->h);
    int planes = phi_planes(p);
    #pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < M; n++) {
        int i = (int)(n % p->nx), j = (int)((n / p->nx) % p->ny), k = (int)(n / ((int64_t)p->nx * p->ny));
        if (is_electrode(p, i, j, k)) { out[n] = 0; continue; }
        double v = phi[n];
        double exy = plane_eps(p, k), eup = face_eps(p, k), edn = face_eps(p, k - 1);
        double sxy = 0;
        const int di[4] = {1, -1, 0, 0}, dj[4] = {0, 0, 1, -1};
        for (int t = 0; t < 4; t++)
            if (!is_electrode(p, i + di[t], j + dj[t], k)) sxy += phi[node(p, i + di[t], j + dj[t], k)];
        double up = (k + 1 < planes && !is_electrode(p, i, j, k + 1)) ? phi[node(p, i, j, k + 1)] : 0.0;
        double dn = (k - 1 >= 0 && !is_electrode(p, i, j, k - 1)) ? phi[node(p, i, j, k - 1)] : 0.0;
        out[n] = ih2 * (exy * (4 * v - sxy) + eup * (v - up) + edn * (v - dn));
    }
}

/* Right-hand side of A phi = -rho + (Dirichlet values times the coupling
 * eps_face / h^2): the bottom ghost plane (phi_bottom), the top ghost plane
 * (metal top) or the electrode nodes (open top).  with_P and with_bc select
 * the polarisation and boundary parts; zero on electrode nodes. */
void or_poisson_rhs(const or_params *p, const double *P, int with_P, int with_bc, double *b) {
    int64_t M = nphi(p);
    double ih2 = 1.0 / (p->h * p->h);
    if (with_P) or_divergence(p, P, b);
    else memset(b, 0, sizeof(double) * (size_t)M);
    #pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < M; n++) {
        int i = (int)(n % p->nx), j = (int)((n / p->nx) % p->ny), k = (int)(n / ((int64_t)p->nx * p->ny));
        if (is_electrode(p, i, j, k)) { b[n] = 0; continue; }
        double v = -b[n];
        if (with_bc) {
            if (k == 0) v += ih2 * face_eps(p, -1) * p->phi_bottom;
            if (!open_top(p) && k == p->nz - 1) v += ih2 * face_eps(p, k) * or_top_ghost(p, i, j);
            if (open_top(p)) {
                const int di[4] = {1, -1, 0, 0}, dj[4] = {0, 0, 1, -1};
                for (int t = 0; t < 4; t++) {
                    int ii = ((i + di[t]) % p->nx + p->nx) % p->nx, jj = ((j + dj[t]) % p->ny + p->ny) % p->ny;
                    if (is_electrode(p, ii, jj, k)) v += ih2 * plane_eps(p, k) * or_top_ghost(p, ii, jj);
                }
                if (is_electrode(p, i, j, k + 1)) v += ih2 * face_eps(p, k) * or_top_ghost(p, i, j);
                if (is_electrode(p, i, j, k - 1)) v += ih2 * face_eps(p, k - 1) * or_top_ghost(p, i, j);
            }
        }
        b[n] = v;
    }
}

/* 7-point Laplacian of each component with mirror (zero-flux) ghosts in z. */
void or_laplacian_neumann(const or_params *p, const double *P, double *out) {
    int64_t N = nnodes(p);
    double c = 1.0 / (p->h * p->h);
    #pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; n++) {
        int i = (int)(n % p->nx), j = (int)((n / p->nx) % p->ny), k = (int)(n / ((int64_t)p->nx * p->ny));
        for (int comp = 0; comp < 3; comp++) {
            const double *X = P + comp * N;
            double x0 = X[n];
            double s = (X[node(p, i + 1, j, k)] - x0) + (X[node(p, i - 1, j, k)] - x0)
                     + (X[node(p, i, j + 1, k)] - x0) + (X[node(p, i, j - 1, k)] - x0);
            if (k + 1 < p->nz) s += X[node(p, i, j, k + 1)] - x0;
            if (k - 1 >= 0) s += X[node(p, i, j, k - 1)] - x0;
            out[comp * N + n] = c * s;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Jacobi-preconditioned conjugate gradients                                  */
/* ------------------------------------------------------------------------ */
/* Stop when ||b - A x||_2 <= tol ||b||_2 (checked before every iteration,
 * on the recursively updated residual); b = 0 gives x = 0.                   */

typedef void (*apply_fn)(const or_params *, const void *, const double *, double *);

static int pcg(const or_params *p, apply_fn A, const void *actx, const double *diag, int64_t n,
               const double *b, double *x, double tol, int warm, int32_t *iters, double *relres) {
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *z = (double *)malloc(sizeof(double) * (size_t)n);
    double *d = (double *)malloc(sizeof(double) * (size_t)n);
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    if (!r || !z || !d || !q) { free(r); free(z); free(d); free(q); return OR_ENOMEM; }
    int status = OR_OK;
    double bnorm = sqrt(dot(b, b, n));
    *iters = 0;
    *relres = 0;
    if (!isfinite(bnorm)) { status = OR_ENONFINITE; goto done; }
    if (bnorm == 0.0) {
        memset(x, 0, sizeof(double) * (size_t)n);
        goto done;
    }
    if (!warm) memset(x, 0, sizeof(double) * (size_t)n);
    A(p, actx, x, q);
    #pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < n; t++) { r[t] = b[t] - q[t]; z[t] = r[t] / diag[t]; d[t] = z[t]; }
    double rz = dot(r, z, n);
    double rnorm = sqrt(dot(r, r, n));
    int k = 0;
    while (rnorm > tol * bnorm && k < p->maxit) {
        A(p, actx, d, q);
        double alpha = rz / dot(d, q, n);
        #pragma omp parallel for schedule(static)
        for (int64_t t = 0; t < n; t++) { x[t] += alpha * d[t]; r[t] -= alpha * q[t]; z[t] = r[t] / diag[t]; }
        double rz_new = dot(r, z, n);
        double beta = rz_new / rz;
        rz = rz_new;
        #pragma omp parallel for schedule(static)
        for (int64_t t = 0; t < n; t++) d[t] = z[t] + beta * d[t];
        rnorm = sqrt(dot(r, r, n));
        k++;
        if (!isfinite(rnorm)) { status = OR_ENONFINITE; break; }
    }
    *iters = k;
    *relres = rnorm / bnorm;
    if (status == OR_OK && !(rnorm <= tol * bnorm)) status = OR_ENOCONV;
done:
    free(r); free(z); free(d); free(q);
    return status;
}

static void poisson_apply_cb(const or_params *p, const void *ctx, const double *x, double *y) {
    (void)ctx;
    or_poisson_apply(p, x, y);
}

static void fem_apply_cb(const or_params *p, const void *ctx, const double *x, double *y) {
    or_fem_apply(p, (const double *)ctx, x, y);
}

/* Poisson solve (Eq. 17-18) for the polarisation P with the boundary values,
 * warm-started from phi when warm != 0.  Jacobi diagonal of A per plane,
 * (4 eps_k + eps_face_above + eps_face_below) / h^2.  The electrode nodes of
 * the open top are not unknowns: they receive their Dirichlet value (the
 * electrode voltage, or zero without the boundary part). */
int or_solve_poisson_parts(const or_params *p, const double *P, int with_P, int with_bc, double *phi,
                           double tol, int warm, int32_t *iters, double *relres) {
    int64_t M = nphi(p);
    double *b = (double *)malloc(sizeof(double) * (size_t)M);
    double *diag = (double *)malloc(sizeof(double) * (size_t)M);
    if (!b || !diag) { free(b); free(diag); return OR_ENOMEM; }
    or_poisson_rhs(p, P, with_P, with_bc, b);
    double ih2 = 1.0 / (p->h * p->h);
    for (int64_t n = 0; n < M; n++) {
        int k = (int)(n / ((int64_t)p->nx * p->ny));
        diag[n] = ih2 * (4 * plane_eps(p, k) + face_eps(p, k) + face_eps(p, k - 1));
    }
    int st = pcg(p, poisson_apply_cb, NULL, diag, M, b, phi, tol, warm, iters, relres);
    if (open_top(p))
        for (int j = 0; j < p->ny; j++)
            for (int i = 0; i < p->nx; i++)
                if (is_electrode(p, i, j, p->nz))
                    phi[node(p, i, j, p->nz)] = with_bc ? or_top_ghost(p, i, j) : 0.0;
    free(b); free(diag);
    return st;
}

int or_solve_phi(const or_params *p, const double *P, double *phi, int32_t *iters, double *relres) {
    return or_solve_poisson_parts(p, P, 1, 1, phi, p->tol_phi, p->warm_start, iters, relres);
}

/* Elastic equilibrium K u = f(P) (Eq. 16). */
int or_solve_u(const or_params *p, const double *P, double *u, int32_t *iters, double *relres) {
    int64_t N = nnodes(p);
    double Ke[576];
    or_element_stiffness(p, Ke);
    double *f = (double *)malloc(sizeof(double) * (size_t)(3 * N));
    double *diag = (double *)malloc(sizeof(double) * (size_t)(3 * N));
    if (!f || !diag) { free(f); free(diag); return OR_ENOMEM; }
    or_fem_rhs(p, P, f);
    or_fem_diagonal(p, Ke, diag);
    int st = pcg(p, fem_apply_cb, Ke, diag, 3 * N, f, u, p->tol_u, p->warm_start, iters, relres);
    free(f); free(diag);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Force (Eq. 7): F = -L [dfL/dP - G Lap P - E - h^-3 s . deps0/dP]          */
/* ------------------------------------------------------------------------ */

/* Thermodynamic force at P given the potential phi (full solution with the
 * Dirichlet ghosts) and displacement u solved at P.  Terms switched off in
 * p->terms contribute nothing; phi / u may then be NULL. */
int or_force(const or_params *p, const double *P, const double *phi, const double *u, double *F) {
    int64_t N = nnodes(p);
    if (((p->terms & OR_TERM_ELEC) && !phi) || ((p->terms & OR_TERM_ELAS) && !u)) return OR_EINVAL;
    double *lap = (double *)calloc((size_t)(3 * N), sizeof(double));
    double *E = (double *)calloc((size_t)(3 * N), sizeof(double));
    double *s = (double *)calloc((size_t)(6 * N), sizeof(double));
    if (!lap || !E || !s) { free(lap); free(E); free(s); return OR_ENOMEM; }
    if (p->terms & OR_TERM_GRAD) or_laplacian_neumann(p, P, lap);
    if (p->terms & OR_TERM_ELEC) or_efield(p, phi, 1, E);
    if (p->terms & OR_TERM_ELAS) or_stress_gather(p, P, u, s);
    double h3 = p->h * p->h * p->h;
    #pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; n++) {
        double x = P[n], y = P[N + n], z = P[2 * N + n];
        double g[3] = {0, 0, 0};
        if (p->terms & OR_TERM_LANDAU) landau_gradient(p, x, y, z, g);
        double el[3] = {0, 0, 0};
        if (p->terms & OR_TERM_ELAS) {
            double D[6][3];
            eigenstrain_jacobian(p, x, y, z, D);
            for (int d = 0; d < 3; d++)
                for (int v = 0; v < 6; v++) el[d] += s[v * N + n] * D[v][d];
        }
        for (int d = 0; d < 3; d++)
            F[d * N + n] = -p->L * (g[d] - p->G * lap[d * N + n] - E[d * N + n] - el[d] / h3);
    }
    free(lap); free(E); free(s);
    return OR_OK;
}

static void stats_add(or_stats *st, int which, int32_t it, double rr) {
    if (!st) return;
    if (which == 0) {
        st->iters_phi += it; st->last_iters_phi = it; st->nsolves_phi++;
        if (rr > st->relres_phi) st->relres_phi = rr;
    } else {
        st->iters_u += it; st->last_iters_u = it; st->nsolves_u++;
        if (rr > st->relres_u) st->relres_u = rr;
    }
}

/* Solves the non-local fields at P (warm-started from phi, u) and evaluates
 * the force.  refresh = 0 keeps phi and u as they are. */
static int force_with_solves(const or_params *p, const double *P, double *phi, double *u, double *F,
                             int refresh, or_stats *st) {
    int rc, worst = OR_OK;
    int32_t it;
    double rr;
    if (refresh && (p->terms & OR_TERM_ELEC)) {
        rc = or_solve_phi(p, P, phi, &it, &rr);
        stats_add(st, 0, it, rr);
        if (rc == OR_ENONFINITE || rc == OR_ENOMEM) return rc;
        if (rc != OR_OK) worst = rc;
    }
    if (refresh && (p->terms & OR_TERM_ELAS)) {
        rc = or_solve_u(p, P, u, &it, &rr);
        stats_add(st, 1, it, rr);
        if (rc == OR_ENONFINITE || rc == OR_ENOMEM) return rc;
        if (rc != OR_OK) worst = rc;
    }
    rc = or_force(p, P, phi, u, F);
    return rc != OR_OK ? rc : worst;
}

/* ------------------------------------------------------------------------ */
/* Thermal noise (the random force zeta of Eq. 7)                             */
/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC 2011): a 4 x 32-bit counter and a 2 x 32-bit key;
 * each of the ten rounds multiplies counter words 0 and 2 by two fixed
 * odd constants, keeps the 64-bit products' halves, and mixes the high
 * halves with words 1 and 3 and the round key; the key advances by two
 * Weyl constants between rounds.                                            */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    const uint64_t mul0 = 0xD2511F53u, mul1 = 0xCD9E8D57u;
    const uint32_t weyl0 = 0x9E3779B9u, weyl1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) { k0 += weyl0; k1 += weyl1; }
        uint64_t prod0 = mul0 * (uint64_t)c0, prod1 = mul1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The standard normal variates xi (3N, component-major like P) of a step:
 * node n draws one Philox block with counter (n low, n high, step low, step
 * high) and key (seed low, seed high); Box-Muller turns words 0, 1 into
 * xi_x, xi_y (cosine and sine branch) and words 2, 3 into xi_z (cosine), with
 * u = (w + 1) 2^-32 in (0, 1] for the radius and 2 pi w 2^-32 for the angle. */
void or_noise(const or_params *p, int64_t step, double *xi) {
    int64_t N = nnodes(p);
    const double two32 = 4294967296.0, two_pi = 6.283185307179586476925286766559;
    uint32_t key[2] = {(uint32_t)p->noise_seed, (uint32_t)(p->noise_seed >> 32)};
    #pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; n++) {
        uint32_t ctr[4] = {(uint32_t)n, (uint32_t)((uint64_t)n >> 32), (uint32_t)step,
                           (uint32_t)((uint64_t)step >> 32)};
        uint32_t w[4];
        or_philox4x32_10(ctr, key, w);
        double r0 = sqrt(-2.0 * log(((double)w[0] + 1.0) / two32));
        double a0 = two_pi * ((double)w[1] / two32);
        double r1 = sqrt(-2.0 * log(((double)w[2] + 1.0) / two32));
        double a1 = two_pi * ((double)w[3] / two32);
        xi[n] = r0 * cos(a0);
        xi[N + n] = r0 * sin(a0);
        xi[2 * N + n] = r1 * cos(a1);
    }
}

/* ------------------------------------------------------------------------ */
/* Time integration (Eq. 19)                                                  */
/* ------------------------------------------------------------------------ */
/* Predictor-corrector with the rate carried as state V ("velocity"):
 *   Pp = P + dt V;  V <- (V + F(Pp)) / 2;  P <- P + dt V.
 * Forward Euler: P <- P + dt F(P).  Each step does one force evaluation.
 * The initial rate is V0 = F(P0) (or_set_state).  With thermal noise the
 * force of step n is F + zeta_n, zeta_n = (sigma / sqrt(dt)) xi_n, so one
 * Euler step adds sigma sqrt(dt) xi_n (Euler-Maruyama); V0 has no noise.    */

int or_set_state(const or_params *p, const double *P, double *V, double *phi, double *u, or_stats *st) {
    if (p->integrator != OR_INT_PC) return OR_OK;
    return force_with_solves(p, P, phi, u, V, 1, st);
}

/* Initial guess for the next solve from the last solutions (warm_start 2):
 * with x the last solution and hist[0..m-1] the m solutions before it, newest
 * first, the guess is the value at the next step of the polynomial through
 * the m+1 equally spaced solutions,
 *   x_next = sum_{t=0..m} (-1)^t C(m+1, t+1) x_{n-t}
 * (m = 0: x; 1: 2x - x1; 2: 3x - 3x1 + x2; ...).  The history then shifts
 * (the oldest drops out, x becomes the newest). */
void or_extrapolate(double *x, double *hist, int64_t n, int m, int cap) {
    double c[16];
    for (int t = 0; t <= m; t++) {
        double b = 1;                 /* C(m+1, t+1) */
        for (int q = 0; q < t + 1; q++) b = b * (m + 1 - q) / (q + 1);
        c[t] = (t % 2 ? -1.0 : 1.0) * b;
    }
    for (int64_t e = 0; e < n; e++) {
        double g = c[0] * x[e];
        for (int t = 1; t <= m; t++) g += c[t] * hist[(int64_t)(t - 1) * n + e];
        for (int t = cap - 1; t > 0; t--) hist[(int64_t)t * n + e] = hist[(int64_t)(t - 1) * n + e];
        if (cap > 0) hist[e] = x[e];
        x[e] = g;
    }
}

/* step0 is the index of the first step (it decides, with nonlocal_every,
 * which steps refresh phi and u).  With warm_start 2 the solution history
 * starts empty at the call (phi and u passed in are the last solutions) and
 * the extrapolation order grows with it up to extrap_order. */
int or_step(const or_params *p, double *P, double *V, double *phi, double *u, int32_t nsteps, int64_t step0,
            or_stats *st) {
    int64_t N = nnodes(p), N3 = 3 * N;
    if (p->warm_start == 2 && (p->extrap_order < 0 || p->extrap_order > 15)) return OR_EINVAL;
    double *Pp = (double *)malloc(sizeof(double) * (size_t)N3);
    double *F = (double *)malloc(sizeof(double) * (size_t)N3);
    int64_t M = nphi(p);
    int cap = p->warm_start == 2 ? (p->extrap_order < 0 ? 0 : p->extrap_order) : 0;
    double *hist = cap > 0 ? (double *)calloc((size_t)((M + 3 * N) * cap), sizeof(double)) : NULL;
    double *xi = p->noise_sigma != 0 ? (double *)malloc(sizeof(double) * (size_t)N3) : NULL;
    if (!Pp || !F || (cap > 0 && !hist) || (p->noise_sigma != 0 && !xi)) {
        free(Pp); free(F); free(hist); free(xi);
        return OR_ENOMEM;
    }
    const double zeta_amp = p->noise_sigma / sqrt(p->dt);
    int nvalid = 0;
    int worst = OR_OK;
    for (int32_t s = 0; s < nsteps; s++) {
        int64_t step = step0 + s;
        int refresh = p->nonlocal_every <= 1 || (step % p->nonlocal_every) == 0;
        if (refresh && hist) {
            if (p->terms & OR_TERM_ELEC) or_extrapolate(phi, hist, M, nvalid, cap);
            if (p->terms & OR_TERM_ELAS) or_extrapolate(u, hist + (int64_t)cap * M, N3, nvalid, cap);
            if (nvalid < cap) nvalid++;
        }
        int rc;
        if (xi) or_noise(p, step, xi);
        if (p->integrator == OR_INT_PC) {
            for (int64_t t = 0; t < N3; t++) Pp[t] = P[t] + p->dt * V[t];
            rc = force_with_solves(p, Pp, phi, u, F, refresh, st);
            if (xi) for (int64_t t = 0; t < N3; t++) F[t] += zeta_amp * xi[t];
            for (int64_t t = 0; t < N3; t++) {
                V[t] = 0.5 * (V[t] + F[t]);
                P[t] = P[t] + p->dt * V[t];
            }
        } else {
            rc = force_with_solves(p, P, phi, u, F, refresh, st);
            if (xi) for (int64_t t = 0; t < N3; t++) F[t] += zeta_amp * xi[t];
            for (int64_t t = 0; t < N3; t++) P[t] = P[t] + p->dt * F[t];
        }
        if (rc == OR_ENONFINITE || rc == OR_ENOMEM) { worst = rc; break; }
        if (rc != OR_OK) worst = rc;
    }
    free(Pp); free(F); free(hist); free(xi);
    return worst;
}

/* ------------------------------------------------------------------------ */
/* Free energy (Eq. 1-6 on the grid)                                          */
/* ------------------------------------------------------------------------ */
/* out = {F_bulk, F_grad, F_elec, F_elas, total} at P:
 *  F_bulk = h^3 sum_n fL(P_n)
 *  F_grad = (G/2) h sum over nearest-neighbour edges |P_m - P_n|^2
 *           (edges wrap in x and y; none leave the film in z)
 *  F_elec = (h^3/2) sum P . G_h phi_P - h^3 sum P . E_app, phi_P the
 *           homogeneous solution for P and E_app = -G_h phi_bc the field of
 *           the boundary values with P = 0 (the linear-dielectric
 *           superposition of Sec. II)
 *  F_elas = elastic energy at the equilibrium displacement for P.
 * tol is the CG tolerance of the three solves.                               */
int or_energy(const or_params *p, const double *P, double tol, double out[5]) {
    int64_t N = nnodes(p);
    double h = p->h, h3 = h * h * h;
    for (int t = 0; t < 5; t++) out[t] = 0;
    double *work = (double *)calloc((size_t)N, sizeof(double));
    if (!work) return OR_ENOMEM;
    int64_t nc = (N + OR_CHUNK - 1) / OR_CHUNK;
    double *part = (double *)calloc((size_t)(nc > 0 ? nc : 1), sizeof(double));
    if (p->terms & OR_TERM_LANDAU) {
        #pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < nc; c++) {
            double s = 0;
            for (int64_t n = c * OR_CHUNK; n < N && n < (c + 1) * OR_CHUNK; n++)
                s += landau_energy_density(p, P[n], P[N + n], P[2 * N + n]);
            part[c] = s;
        }
        double s = 0;
        for (int64_t c = 0; c < nc; c++) s += part[c];
        out[0] = h3 * s;
    }
    if (p->terms & OR_TERM_GRAD) {
        #pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < nc; c++) {
            double s = 0;
            for (int64_t n = c * OR_CHUNK; n < N && n < (c + 1) * OR_CHUNK; n++) {
                int i = (int)(n % p->nx), j = (int)((n / p->nx) % p->ny), k = (int)(n / ((int64_t)p->nx * p->ny));
                int64_t nbr[3] = {node(p, i + 1, j, k), node(p, i, j + 1, k), k + 1 < p->nz ? node(p, i, j, k + 1) : -1};
                for (int e = 0; e < 3; e++) {
                    if (nbr[e] < 0) continue;
                    for (int comp = 0; comp < 3; comp++) {
                        double d = P[comp * N + nbr[e]] - P[comp * N + n];
                        s += d * d;
                    }
                }
            }
            part[c] = s;
        }
        double s = 0;
        for (int64_t c = 0; c < nc; c++) s += part[c];
        out[1] = 0.5 * p->G * h * s;
    }
    int status = OR_OK;
    int32_t it;
    double rr;
    if (p->terms & OR_TERM_ELEC) {
        double *phiP = (double *)calloc((size_t)nphi(p), sizeof(double));
        double *phib = (double *)calloc((size_t)nphi(p), sizeof(double));
        double *EP = (double *)calloc((size_t)(3 * N), sizeof(double));
        double *Eb = (double *)calloc((size_t)(3 * N), sizeof(double));
        int r1 = or_solve_poisson_parts(p, P, 1, 0, phiP, tol, 0, &it, &rr);
        int r2 = or_solve_poisson_parts(p, P, 0, 1, phib, tol, 0, &it, &rr);
        if (r1 != OR_OK) status = r1;
        if (r2 != OR_OK) status = r2;
        or_efield(p, phiP, 0, EP);
        or_efield(p, phib, 1, Eb);
        double s1 = 0, s2 = 0;
        for (int comp = 0; comp < 3; comp++) {
            s1 += dot(P + comp * N, EP + comp * N, N);
            s2 += dot(P + comp * N, Eb + comp * N, N);
        }
        /* G_h phi_P = -E_P */
        out[2] = -0.5 * h3 * s1 - h3 * s2;
        free(phiP); free(phib); free(EP); free(Eb);
    }
    if (p->terms & OR_TERM_ELAS) {
        double *u = (double *)calloc((size_t)(3 * N), sizeof(double));
        or_params q = *p;
        q.tol_u = tol;
        int r3 = or_solve_u(&q, P, u, &it, &rr);
        if (r3 != OR_OK) status = r3;
        out[3] = or_elastic_energy(p, P, u);
        free(u);
    }
    out[4] = out[0] + out[1] + out[2] + out[3];
    free(work); free(part);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Linearised force and discrete adjoint                                      */
/* ------------------------------------------------------------------------ */
/* The force is F = -(L/h^3) dF_h/dP, so its Jacobian H = dF/dP is symmetric.
 * H lam = -L [ Hess fL lam - G Lap lam - E(lam) - h^-3 (ds . deps0/dP
 *              + s . d2eps0/dP2 lam) ]
 * where E(lam) = -G_h psi with A psi = -D_h lam (zero boundary values),
 * deps0 = deps0/dP lam (nodal), K du = f(deps0) and ds = s(du, deps0).      */

/* Field of electrode e alone: P = 0, unit voltage on the strip of electrode
 * e, every other boundary value zero.  dF/dV_e = L E^(e). */
int or_electrode_field(const or_params *p, int e, double tol, double *E) {
    if (e < 0 || e >= p->n_el) return OR_EINVAL;
    double *volts = (double *)calloc((size_t)p->n_el, sizeof(double));
    double *phi = (double *)calloc((size_t)nphi(p), sizeof(double));
    if (!volts || !phi) { free(volts); free(phi); return OR_ENOMEM; }
    volts[e] = 1.0;
    or_params q = *p;
    q.phi_top = 0; q.phi_bottom = 0; q.el_volts = volts;
    int32_t it;
    double rr;
    int st = or_solve_poisson_parts(&q, NULL, 0, 1, phi, tol, 0, &it, &rr);
    or_efield(&q, phi, 1, E);
    free(volts); free(phi);
    return st;
}

/* out = H(P) lam; u is the displacement solved at P (may be NULL when the
 * elastic term is off).  tol is the tolerance of the two linearised solves. */
int or_hvp(const or_params *p, const double *P, const double *u, const double *lam, double tol, double *out) {
    int64_t N = nnodes(p);
    double h3 = p->h * p->h * p->h;
    int status = OR_OK;
    int32_t it;
    double rr;
    double *lap = (double *)calloc((size_t)(3 * N), sizeof(double));
    double *El = (double *)calloc((size_t)(3 * N), sizeof(double));
    double *el = (double *)calloc((size_t)(3 * N), sizeof(double));
    if (!lap || !El || !el) { free(lap); free(El); free(el); return OR_ENOMEM; }
    if (p->terms & OR_TERM_GRAD) or_laplacian_neumann(p, lam, lap);
    if (p->terms & OR_TERM_ELEC) {
        double *psi = (double *)calloc((size_t)nphi(p), sizeof(double));
        int rc = or_solve_poisson_parts(p, lam, 1, 0, psi, tol, 0, &it, &rr);
        if (rc != OR_OK) status = rc;
        or_efield(p, psi, 0, El);
        free(psi);
    }
    if (p->terms & OR_TERM_ELAS) {
        double *s = (double *)calloc((size_t)(6 * N), sizeof(double));
        double *de0 = (double *)calloc((size_t)(6 * N), sizeof(double));
        double *f = (double *)calloc((size_t)(3 * N), sizeof(double));
        double *du = (double *)calloc((size_t)(3 * N), sizeof(double));
        double *ds = (double *)calloc((size_t)(6 * N), sizeof(double));
        double *diag = (double *)calloc((size_t)(3 * N), sizeof(double));
        double Ke[576];
        or_element_stiffness(p, Ke);
        or_fem_diagonal(p, Ke, diag);
        or_stress_gather(p, P, u, s);
        for (int64_t n = 0; n < N; n++) {
            double D[6][3];
            eigenstrain_jacobian(p, P[n], P[N + n], P[2 * N + n], D);
            for (int v = 0; v < 6; v++)
                de0[v * N + n] = D[v][0] * lam[n] + D[v][1] * lam[N + n] + D[v][2] * lam[2 * N + n];
        }
        or_fem_rhs_e0(p, de0, f);
        int rc = pcg(p, fem_apply_cb, Ke, diag, 3 * N, f, du, tol, 0, &it, &rr);
        if (rc != OR_OK) status = rc;
        or_stress_gather_e0(p, de0, du, ds);
        for (int64_t n = 0; n < N; n++) {
            double D[6][3], sn[6], dsn[6], ln[3], hs[3];
            eigenstrain_jacobian(p, P[n], P[N + n], P[2 * N + n], D);
            for (int v = 0; v < 6; v++) { sn[v] = s[v * N + n]; dsn[v] = ds[v * N + n]; }
            for (int d = 0; d < 3; d++) ln[d] = lam[d * N + n];
            eigenstrain_hessian_apply(p, sn, ln, hs);
            for (int d = 0; d < 3; d++) {
                double a = hs[d];
                for (int v = 0; v < 6; v++) a += dsn[v] * D[v][d];
                el[d * N + n] = a;
            }
        }
        free(s); free(de0); free(f); free(du); free(ds); free(diag);
    }
    for (int64_t n = 0; n < N; n++) {
        double H[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        if (p->terms & OR_TERM_LANDAU) landau_hessian(p, P[n], P[N + n], P[2 * N + n], H);
        for (int d = 0; d < 3; d++) {
            double hl = H[d][0] * lam[n] + H[d][1] * lam[N + n] + H[d][2] * lam[2 * N + n];
            out[d * N + n] = -p->L * (hl - p->G * lap[d * N + n] - El[d * N + n] - el[d * N + n] / h3);
        }
    }
    free(lap); free(El); free(el);
    return status;
}

/* dtheta += w . dF/dtheta at P, theta = (V_1 .. V_nel, a1):
 * dF/dV_e = L E^(e) (Ebasis[e*3N ...]), dF/da1 = -2 L P. */
void or_dtheta_accumulate(const or_params *p, const double *P, const double *w, const double *Ebasis, double *dtheta) {
    int64_t N3 = 3 * nnodes(p);
    if (p->terms & OR_TERM_ELEC)
        for (int e = 0; e < p->n_el; e++) dtheta[e] += p->L * dot(w, Ebasis + e * N3, N3);
    if (p->terms & OR_TERM_LANDAU) dtheta[p->n_el] += -2 * p->L * dot(w, P, N3);
}

/* One reverse step.  In: state (P_n, V_n) before forward step n and the
 * adjoints (lamP, lamV) of the state after it; out: the adjoints of the
 * state before it.  Predictor-corrector (Eq. 19 with the carried rate):
 *   mu = lamV + dt lamP, w = mu/2, Pp = P_n + dt V_n,
 *   lamP <- lamP + H(Pp) w,  lamV <- w + dt H(Pp) w,  dtheta += w . dF/dtheta(Pp).
 * Euler: lamP <- lamP + dt H(P_n) lamP, dtheta += dt lamP . dF/dtheta(P_n).
 * The displacement at the linearisation point is solved here (cold, tol). */
int or_adjoint_step(const or_params *p, const double *Pn, const double *Vn, double *lamP, double *lamV,
                    const double *Ebasis, double tol, double *dtheta) {
    int64_t N3 = 3 * nnodes(p);
    double *X = (double *)malloc(sizeof(double) * (size_t)N3);
    double *w = (double *)malloc(sizeof(double) * (size_t)N3);
    double *Hw = (double *)malloc(sizeof(double) * (size_t)N3);
    double *u = (double *)calloc((size_t)N3, sizeof(double));
    if (!X || !w || !Hw || !u) { free(X); free(w); free(Hw); free(u); return OR_ENOMEM; }
    int status = OR_OK;
    int32_t it;
    double rr;
    or_params q = *p;
    q.tol_u = tol;
    q.warm_start = 0;
    if (p->integrator == OR_INT_PC) {
        for (int64_t t = 0; t < N3; t++) { X[t] = Pn[t] + p->dt * Vn[t]; w[t] = 0.5 * (lamV[t] + p->dt * lamP[t]); }
    } else {
        for (int64_t t = 0; t < N3; t++) { X[t] = Pn[t]; w[t] = lamP[t]; }
    }
    if (p->terms & OR_TERM_ELAS) {
        int rc = or_solve_u(&q, X, u, &it, &rr);
        if (rc != OR_OK) status = rc;
    }
    int rc = or_hvp(p, X, u, w, tol, Hw);
    if (rc != OR_OK) status = rc;
    if (p->integrator == OR_INT_PC) {
        or_dtheta_accumulate(p, X, w, Ebasis, dtheta);
        for (int64_t t = 0; t < N3; t++) { lamP[t] += Hw[t]; lamV[t] = w[t] + p->dt * Hw[t]; }
    } else {
        for (int64_t t = 0; t < N3; t++) w[t] *= p->dt;
        or_dtheta_accumulate(p, X, w, Ebasis, dtheta);
        for (int64_t t = 0; t < N3; t++) lamP[t] += p->dt * Hw[t];
    }
    free(X); free(w); free(Hw); free(u);
    return status;
}

/* Folds the initial rate V0 = F(P0) of the predictor-corrector into the
 * adjoints: lamP += H(P0) lamV, dtheta += lamV . dF/dtheta(P0), lamV = 0. */
int or_adjoint_initial_rate(const or_params *p, const double *P0, double *lamP, double *lamV,
                            const double *Ebasis, double tol, double *dtheta) {
    int64_t N3 = 3 * nnodes(p);
    if (p->integrator != OR_INT_PC) return OR_OK;
    double *Hw = (double *)malloc(sizeof(double) * (size_t)N3);
    double *u = (double *)calloc((size_t)N3, sizeof(double));
    if (!Hw || !u) { free(Hw); free(u); return OR_ENOMEM; }
    int status = OR_OK;
    int32_t it;
    double rr;
    or_params q = *p;
    q.tol_u = tol;
    q.warm_start = 0;
    if (p->terms & OR_TERM_ELAS) {
        int rc = or_solve_u(&q, P0, u, &it, &rr);
        if (rc != OR_OK) status = rc;
    }
    int rc = or_hvp(p, P0, u, lamV, tol, Hw);
    if (rc != OR_OK) status = rc;
    or_dtheta_accumulate(p, P0, lamV, Ebasis, dtheta);
    for (int64_t t = 0; t < N3; t++) { lamP[t] += Hw[t]; lamV[t] = 0; }
    free(Hw); free(u);
    return status;
}
