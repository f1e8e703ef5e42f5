/*
 * Plain FP64 CPU oracle of the Galilean-invariant preconditioned cascaded
 * central-moment D2Q9 lattice Boltzmann method (Hajabdollahi & Premnath,
 * arXiv:1806.10251).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is used by the tests, by the smoke
 * check and by the CPU-baseline leg of the benchmark.  The product path (the
 * HIP library) never links, loads or calls it, and it shares no code, header
 * or table with the product path.
 *
 * It is deliberately slow and literal: every time step runs its phases one
 * after another over the whole grid (stream, macroscopic fields, density
 * gradient, collision), in double precision on the full populations f (not
 * deviations), so that each phase can be checked against the paper by eye.
 *
 * Paper map (all equation numbers are the paper's):
 *   - lattice, raw moments ............ eq. 3, eq. 5, eq. 6
 *   - preconditioned raw equilibria ... eq. (eqmrawmoment), Sec. 3
 *   - source raw moments sigma' ....... the list after eq. (eqmrawmoment)
 *   - collide + stream ................ eqs. 2a, 2b; forcing transform below eq. 2
 *   - GI-corrected kernel ............. Sec. 5 (g3..g8), coefficients eqs. 45-47
 *   - local strain-rate estimator ..... eqs. 51-55 and the m^(1) definitions
 *   - uncorrected kernel (control) .... eq. 4
 *   - viscosity / gamma map ........... eq. 49 and Sec. 2 (nu = gamma/3 (1/w - 1/2))
 *   - boundaries ...................... Sec. 6 (half-way bounce-back, moving lid,
 *                                       parabolic inlet, convective outlet)
 *   - per-node body force ............. Sec. 6 (Hartmann, four-rolls mill)
 *   - strain rates by finite differences, raw-moment MRT form: the two
 *     alternatives Sec. 5 names (options strain_fd, mrt)
 *   - steady-state residual ........... not defined in the paper (it plots
 *     histories only): ||u^{n+1}-u^n||_2 / ||u^n||_2 over fluid nodes, a
 *     reading pinned against a decaying shear mode, not against the paper
 *
 * Readings taken where the paper is silent or inconsistent (each one is also
 * listed in the design notes of the repository):
 *   R1  collision basis K: the standard cascaded orthogonal basis (the paper
 *       defers K to its ref. [Hajabdollahi2017]); pinned by the prefactors
 *       w3/12, w4/4, w5/4 of Sec. 5 and the "-4 g6" relation of Sec. 5.
 *   R2  every kappa' in the Sec. 5 kernel is a raw moment of f = fbar + S/2.
 *   R3  eq. 55b: the printed sign of the c~1 term is wrong (Cramer's rule on
 *       eqs. 51-52 and the u = 0 limit); the solved form is used.
 *   R4  lambda^5 (eq. 47c,d): no factor rho, as eq. 28a with eq. 44c give.
 *   R5  the 2x2 strain system can become singular; guard: if D*D0 <= 0 or
 *       |D| < |D0|/4 (D0 = -2 a3 a4 rho^2), solve it with A = B = 0.
 *   R6  equilibrium used for initial states: the kernel's central-moment
 *       targets (raw fourth order follows the kernel, not the printed raw
 *       fourth-order equilibrium).
 *   R7  density-gradient neighbours: same time level; periodic sides wrap;
 *       a neighbour beyond a non-periodic side contributes the density of
 *       its mirror image across the half-way wall (the adjacent edge node:
 *       zero normal gradient); a solid neighbour contributes rho(x).
 *   R8  lid: momentum-augmented half-way bounce-back with rho_w = rho0; a
 *       link whose source lies outside the domain on both axes (a corner)
 *       is a stationary wall.  Inlet: the same moving-wall rule with the
 *       parabolic profile at the fluid node's y.
 *   R9  outlet: the convective equation d_t u + U_max d_x u = 0 is applied to
 *       the velocity of the last column, upwind in space and implicit in
 *       time, u*^{n+1} = (u*^n + U u^{n+1}(N-2)) / (1 + U); the outlet density
 *       is held at rho0 (zero gauge pressure); the three unknown incoming
 *       populations are set by non-equilibrium extrapolation from column N-2:
 *       f_a = f_a^eq(rho0, u*) + fbar_a(N-2) - f_a^eq(rho(N-2), u(N-2)).
 *       (Applying the convective equation to the populations themselves
 *       leaves the density level free: a uniform density drift then solves
 *       the discrete system and steady convergence stalls.)
 *   R17 finite-difference strain rates: the velocity of the post-stream
 *       state, the density-gradient stencil and the R7 neighbour rule.
 *   R18 raw-moment MRT: eq. 7 in the transformed variable with the printed
 *       raw equilibria of Sec. 3 (including the printed fourth order) and,
 *       with gi_correct, the second-order equilibria extended by D3, D4, D5.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PERIODIC 0
#define ORC_WALL 1
#define ORC_LID 2
#define ORC_INLET 3
#define ORC_OUTLET 4

#define SW 0 /* west  (x = 0)      */
#define SE 1 /* east  (x = nx)     */
#define SS 2 /* south (y = 0)      */
#define SN 3 /* north (y = ny)     */

/* D2Q9 velocities and weights (standard set; the paper lists the moment
 * basis, eq. 5, but not the velocity ordering). */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double WT[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

/* Columns 3..8 of the orthogonal collision basis K (reading R1). */
static const double KCOL[6][9] = {
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},  /* K3 = 3|e|^2 - 4        */
    {0, 1, -1, 1, -1, 0, 0, 0, 0},     /* K4 = ex^2 - ey^2        */
    {0, 0, 0, 0, 0, 1, -1, 1, -1},     /* K5 = ex ey              */
    {0, 0, 2, 0, -2, -1, -1, 1, 1},    /* K6 = -3 ex^2 ey + 2 ey  */
    {0, 2, 0, -2, 0, -1, 1, 1, -1},    /* K7 = -3 ex ey^2 + 2 ex  */
    {4, -2, -2, -2, -2, 1, 1, 1, 1},   /* K8 = 9ex^2ey^2-6|e|^2+4 */
};

typedef struct {
  double nu;      /* kinematic viscosity; w4 = w5 = 1/(3 nu/gamma + 1/2) */
  double omega3, omega6, omega7, omega8;
  double gamma;   /* preconditioning parameter */
  double u_lid;   /* lid speed (tangential; +x on S/N sides, +y on W/E) */
  double u_in_max;/* peak of the parabolic inlet profile (W side) */
  double rho0;    /* reference density */
  double fx, fy;  /* uniform body force */
  int32_t gi_correct;   /* 1: Sec. 5 kernel, 0: eq. 4 kernel */
  int32_t drho_stencil; /* 0: isotropic, 1: central difference */
  int32_t strain_fd;    /* 0: strain rates from the non-equilibrium moments
                           (eqs. 51-55); 1: finite differences of the velocity
                           at the same time level (the alternative named in
                           Sec. 5), with the density-gradient stencil */
  int32_t mrt;          /* 0: cascaded central-moment kernel (Sec. 5 / eq. 4);
                           1: non-orthogonal raw-moment MRT form (eq. 7 with
                           the raw equilibria of Sec. 3 and, when gi_correct,
                           the extended equilibria of the second-order moments) */
} orc_params;

typedef struct {
  int nx, ny;
  int side[4];
  orc_params p;
  double omega4, omega5;
  uint8_t *solid; /* [ny][nx] */
  double *f;      /* post-collision populations f~ [9][ny][nx] */
  double *fb;     /* post-stream populations fbar [9][ny][nx] */
  double *rho, *ux, *uy;    /* macroscopic fields of the last step */
  double *uxp, *uyp;        /* fields of the step before */
  double *drx, *dry;        /* density gradient */
  double *sxx, *syy;        /* strain rates by finite differences (strain_fd) */
  double *hist;   /* outlet history: [2][ny] velocity u* of the last column */
  double *hist_next;
  double *ffx, *ffy; /* per-node body force [ny][nx] (NULL: the uniform p.fx, p.fy) */
  double resid, mass;
  int64_t steps, guards;
} orc;

#define IDX(o, i, j) ((size_t)(j) * (o)->nx + (i))
#define FXN(o, k) ((o)->ffx ? (o)->ffx[k] : (o)->p.fx)
#define FYN(o, k) ((o)->ffy ? (o)->ffy[k] : (o)->p.fy)
#define FQ(o, arr, a, i, j) ((arr)[(size_t)(a) * (o)->nx * (o)->ny + IDX(o, i, j)])

/* ------------------------------------------------------------------ */
/* Raw moments and their inverse (eq. 3, eq. 5, eq. 6).                */
/* m = (k0, kx, ky, kxx, kyy, kxy, kxxy, kxyy, kxxyy) = sum f ex^m ey^n */
/* ------------------------------------------------------------------ */
void orc_raw_moments(const double f[9], double m[9]) {
  memset(m, 0, 9 * sizeof(double));
  for (int a = 0; a < 9; ++a) {
    double ex = EX[a], ey = EY[a];
    m[0] += f[a];
    m[1] += f[a] * ex;
    m[2] += f[a] * ey;
    m[3] += f[a] * ex * ex;
    m[4] += f[a] * ey * ey;
    m[5] += f[a] * ex * ey;
    m[6] += f[a] * ex * ex * ey;
    m[7] += f[a] * ex * ey * ey;
    m[8] += f[a] * ex * ex * ey * ey;
  }
}

/* Inverse of the raw-moment map on D2Q9 (solves eq. 6 for the populations). */
void orc_moments_to_pop(const double m[9], double f[9]) {
  double k0 = m[0], kx = m[1], ky = m[2], kxx = m[3], kyy = m[4], kxy = m[5];
  double kxxy = m[6], kxyy = m[7], kxxyy = m[8];
  f[0] = k0 - kxx - kyy + kxxyy;
  f[1] = 0.5 * (kx + kxx - kxyy - kxxyy);
  f[3] = 0.5 * (-kx + kxx + kxyy - kxxyy);
  f[2] = 0.5 * (ky + kyy - kxxy - kxxyy);
  f[4] = 0.5 * (-ky + kyy + kxxy - kxxyy);
  f[5] = 0.25 * (kxy + kxxy + kxyy + kxxyy);
  f[6] = 0.25 * (-kxy + kxxy - kxyy + kxxyy);
  f[7] = 0.25 * (kxy - kxxy - kxyy + kxxyy);
  f[8] = 0.25 * (-kxy - kxxy + kxyy + kxxyy);
}

/* Equilibrium populations at (rho, u) (reading R6): central-moment targets
 * of the Sec. 5 kernel, shifted to raw moments with the binomial theorem,
 * then mapped to populations.  For orders <= 3 these raw moments are the
 * printed preconditioned equilibria of Sec. 3. */
void orc_equilibrium(double rho, double ux, double uy, double gamma, double f[9]) {
  double g1 = 1.0 / gamma - 1.0;
  /* central moments about u */
  double cxx = rho / 3.0 + rho * ux * ux * g1;
  double cyy = rho / 3.0 + rho * uy * uy * g1;
  double cxy = rho * ux * uy * g1;
  double cxxy = rho * ux * ux * uy * g1 * (1.0 / gamma - 2.0);
  double cxyy = rho * ux * uy * uy * g1 * (1.0 / gamma - 2.0);
  double cxxyy = rho / 9.0;
  /* binomial shift: raw = sum over sub-moments; central kx = ky = 0 */
  double m[9];
  m[0] = rho;
  m[1] = rho * ux;
  m[2] = rho * uy;
  m[3] = cxx + rho * ux * ux;
  m[4] = cyy + rho * uy * uy;
  m[5] = cxy + rho * ux * uy;
  m[6] = cxxy + uy * cxx + 2.0 * ux * cxy + rho * ux * ux * uy;
  m[7] = cxyy + ux * cyy + 2.0 * uy * cxy + rho * ux * uy * uy;
  m[8] = cxxyy + 2.0 * ux * cxyy + 2.0 * uy * cxxy + ux * ux * cyy + uy * uy * cxx +
         4.0 * ux * uy * cxy + rho * ux * ux * uy * uy;
  orc_moments_to_pop(m, f);
}

/* Preconditioned source raw moments sigma' (Sec. 3, list after the raw
 * equilibria), uniform force F. */
static void source_moments(double fx, double fy, double ux, double uy, double gamma,
                           double s[9]) {
  double g2 = gamma * gamma;
  s[0] = 0.0;
  s[1] = fx / gamma;
  s[2] = fy / gamma;
  s[3] = 2.0 * fx * ux / g2;
  s[4] = 2.0 * fy * uy / g2;
  s[5] = (fx * uy + fy * ux) / g2;
  s[6] = fy * ux * ux + 2.0 * fx * ux * uy;
  s[7] = fx * uy * uy + 2.0 * fy * uy * ux;
  s[8] = 2.0 * (fx * ux * uy * uy + fy * uy * ux * ux);
}

/* ------------------------------------------------------------------ */
/* Local strain-rate estimator, eqs. 51-55 (readings R3, R5).          */
/* Returns 1 when the guard replaced the system.                      */
/* ------------------------------------------------------------------ */
int orc_strain(double rho, double ux, double uy, double m3, double m4, double drx,
               double dry, double omega3, double omega4, double gamma,
               double *dxux, double *dyuy) {
  double A = 4.0 / (gamma * gamma) - 1.0 / gamma;
  double B = 1.0 / (gamma * gamma) - 1.0 / gamma;
  double C = 1.0 / gamma - 1.0;
  double a3 = 2.0 / (3.0 * omega3), a4 = 2.0 / (3.0 * omega4);
  double ux2 = ux * ux, uy2 = uy * uy;
  /* eq. 54 */
  double er = C / 3.0 * (ux * drx + uy * dry);
  double ert = C / 3.0 * (ux * drx - uy * dry);
  /* eq. 53 with P, Q, P~, Q~ */
  double c1 = (a3 - 0.5 * (A * ux2 + B * uy2)) * rho;
  double c2 = (a3 - 0.5 * (A * uy2 + B * ux2)) * rho;
  double ct1 = (a4 - 0.5 * (A * ux2 - B * uy2)) * rho;
  double ct2 = (a4 - 0.5 * (A * uy2 - B * ux2)) * rho;
  double D = -c1 * ct2 - ct1 * c2;
  double D0 = -2.0 * a3 * a4 * rho * rho;
  int guarded = 0;
  if (D * D0 <= 0.0 || fabs(D) < 0.25 * fabs(D0)) {
    c1 = c2 = a3 * rho;
    ct1 = ct2 = a4 * rho;
    D = D0;
    guarded = 1;
  }
  /* eqs. 51, 52:  -c1 X - c2 Y = R3,  -c~1 X + c~2 Y = R4; Cramer's rule */
  double R3 = m3 - er, R4 = m4 - ert;
  *dxux = (ct2 * R3 + c2 * R4) / D;
  *dyuy = (ct1 * R3 - c1 * R4) / D;
  return guarded;
}

/* ------------------------------------------------------------------ */
/* One node's collision (eq. 2a with the Sec. 5 kernel, or eq. 4).     */
/* fbar: post-stream populations; drx, dry: density gradient.          */
/* diag (optional, 8 entries): rho, ux, uy, dxux, dyuy, guarded, m3, m4 */
/* ------------------------------------------------------------------ */
void orc_collide_ext(const double fbar[9], double drx, double dry, const double *strain,
                     const orc_params *p, double omega4, double omega5, double fout[9],
                     double diag[8]);

void orc_collide(const double fbar[9], double drx, double dry, const orc_params *p,
                 double omega4, double omega5, double fout[9], double diag[8]) {
  orc_collide_ext(fbar, drx, dry, NULL, p, omega4, omega5, fout, diag);
}

/* As orc_collide; strain (optional, 2 entries): d_x u_x and d_y u_y to use in
 * the corrections instead of the estimate of eqs. 51-55. */
void orc_collide_ext(const double fbar[9], double drx, double dry, const double *strain,
                     const orc_params *p, double omega4, double omega5, double fout[9],
                     double diag[8]) {
  double gamma = p->gamma;
  double mb[9];
  orc_raw_moments(fbar, mb);
  double rho = mb[0];
  /* rho u = sum e fbar + F/(2 gamma): the first moment of f = fbar + S/2 */
  double ux = (mb[1] + 0.5 * p->fx / gamma) / rho;
  double uy = (mb[2] + 0.5 * p->fy / gamma) / rho;
  double sg[9];
  source_moments(p->fx, p->fy, ux, uy, gamma, sg);
  /* reading R2: raw moments of f = fbar + S/2 */
  double Kxx = mb[3] + 0.5 * sg[3];
  double Kyy = mb[4] + 0.5 * sg[4];
  double Kxy = mb[5] + 0.5 * sg[5];
  double Kxxy = mb[6] + 0.5 * sg[6];
  double Kxyy = mb[7] + 0.5 * sg[7];
  double Kxxyy = mb[8] + 0.5 * sg[8];
  double ux2 = ux * ux, uy2 = uy * uy;
  /* second-order non-equilibrium moments (definitions after eq. 55) */
  double m3 = Kxx + Kyy - (2.0 / 3.0 * rho + rho * (ux2 + uy2) / gamma);
  double m4 = Kxx - Kyy - rho * (ux2 - uy2) / gamma;

  double w3 = p->omega3, w4 = omega4, w5 = omega5;
  double w6 = p->omega6, w7 = p->omega7, w8 = p->omega8;
  double D3 = 0.0, D4 = 0.0, D5 = 0.0, third;
  double dxux = 0.0, dyuy = 0.0;
  int guarded = 0;
  if (p->gi_correct) {
    double A = 4.0 / (gamma * gamma) - 1.0 / gamma;
    double B = 1.0 / (gamma * gamma) - 1.0 / gamma;
    double C = 1.0 / gamma - 1.0;
    double h3 = 1.0 / w3 - 0.5, h4 = 1.0 / w4 - 0.5, h5 = 1.0 / w5 - 0.5;
    if (strain) {
      dxux = strain[0];
      dyuy = strain[1];
    } else {
      guarded = orc_strain(rho, ux, uy, m3, m4, drx, dry, w3, w4, gamma, &dxux, &dyuy);
    }
    /* eq. 45: theta^3, lambda^3 */
    double th3x = -h3 * rho * (A * ux2 + B * uy2);
    double th3y = -h3 * rho * (A * uy2 + B * ux2);
    double la3x = -2.0 / 3.0 * h3 * C * ux;
    double la3y = -2.0 / 3.0 * h3 * C * uy;
    /* eq. 46: theta^4, lambda^4 */
    double th4x = -h4 * rho * (A * ux2 - B * uy2);
    double th4y = h4 * rho * (-A * uy2 + B * ux2);
    double la4x = -2.0 / 3.0 * h4 * C * ux;
    double la4y = -2.0 / 3.0 * h4 * C * uy;
    /* eq. 47 (reading R4: no rho in lambda^5) */
    double th5x = -h5 * rho * B * ux * uy;
    double th5y = -h5 * rho * B * ux * uy;
    double la5x = -1.0 / 3.0 * h5 * C * uy;
    double la5y = -1.0 / 3.0 * h5 * C * ux;
    /* extended equilibria, eq. 33 */
    D3 = th3x * dxux + th3y * dyuy + la3x * drx + la3y * dry;
    D4 = th4x * dxux - th4y * dyuy + la4x * drx - la4y * dry;
    D5 = th5x * dxux + th5y * dyuy + la5x * drx + la5y * dry;
    third = 3.0 / gamma - 1.0 / (gamma * gamma);
  } else {
    third = 2.0;
  }
  if (p->mrt) {
    /* raw-moment MRT (eq. 7): the raw moments m_b of f = fbar + S/2 in the
     * basis of eq. 5 relax with rate w_b towards the raw equilibria of Sec. 3
     * (second order extended by D3, D4, D5); f~ = fbar + T^-1 dm + S */
    double e3 = 2.0 / 3.0 * rho + rho * (ux2 + uy2) / gamma + D3;
    double e4 = rho * (ux2 - uy2) / gamma + D4;
    double e5 = rho * ux * uy / gamma + D5;
    double e6 = rho * uy / 3.0 + rho * ux2 * uy / (gamma * gamma);
    double e7 = rho * ux / 3.0 + rho * ux * uy2 / (gamma * gamma);
    double e8 = rho / 9.0 + rho * (ux2 + uy2) / 3.0 + rho * ux2 * uy2;
    double d3 = -w3 * (Kxx + Kyy - e3);
    double d4 = -w4 * (Kxx - Kyy - e4);
    double d5 = -w5 * (Kxy - e5);
    double d6 = -w6 * (Kxxy - e6);
    double d7 = -w7 * (Kxyy - e7);
    double d8 = -w8 * (Kxxyy - e8);
    double dk[9] = {0.0, 0.0, 0.0, 0.5 * (d3 + d4), 0.5 * (d3 - d4), d5, d6, d7, d8};
    double df[9], S[9];
    orc_moments_to_pop(dk, df);
    orc_moments_to_pop(sg, S);
    for (int a = 0; a < 9; ++a) fout[a] = fbar[a] + df[a] + S[a];
    if (diag) {
      diag[0] = rho; diag[1] = ux; diag[2] = uy; diag[3] = dxux; diag[4] = dyuy;
      diag[5] = guarded; diag[6] = m3; diag[7] = m4;
    }
    return;
  }
  /* cascaded kernel: Sec. 5 (gi_correct) or eq. 4 */
  double g3 = w3 / 12.0 * (-m3 + D3);
  double g4 = w4 / 4.0 * (-m4 + D4);
  double g5 = w5 / 4.0 * (rho * ux * uy / gamma - Kxy + D5);
  double g6 = w6 / 4.0 * (third * rho * ux2 * uy + Kxxy - 2.0 * ux * Kxy - uy * Kxx) -
              0.5 * uy * (3.0 * g3 + g4) - 2.0 * ux * g5;
  double g7 = w7 / 4.0 * (third * rho * ux * uy2 + Kxyy - 2.0 * uy * Kxy - ux * Kyy) -
              0.5 * ux * (3.0 * g3 - g4) - 2.0 * uy * g5;
  double g8 = w8 / 4.0 *
                  (rho / 9.0 + 3.0 * rho * ux2 * uy2 -
                   (Kxxyy - 2.0 * ux * Kxyy - 2.0 * uy * Kxxy + ux2 * Kyy + uy2 * Kxx +
                    4.0 * ux * uy * Kxy)) -
              2.0 * g3 - 0.5 * uy2 * (3.0 * g3 + g4) - 0.5 * ux2 * (3.0 * g3 - g4) -
              4.0 * ux * uy * g5 - 2.0 * uy * g6 - 2.0 * ux * g7;
  double g[6] = {g3, g4, g5, g6, g7, g8};
  double S[9];
  orc_moments_to_pop(sg, S);
  for (int a = 0; a < 9; ++a) {
    double v = fbar[a] + S[a];
    for (int b = 0; b < 6; ++b) v += KCOL[b][a] * g[b];
    fout[a] = v;
  }
  if (diag) {
    diag[0] = rho;
    diag[1] = ux;
    diag[2] = uy;
    diag[3] = dxux;
    diag[4] = dyuy;
    diag[5] = guarded;
    diag[6] = m3;
    diag[7] = m4;
  }
}

/* ------------------------------------------------------------------ */
/* Grid driver                                                         */
/* ------------------------------------------------------------------ */
static int is_solid(const orc *o, int i, int j) { return o->solid[IDX(o, i, j)] != 0; }

/* parabolic inlet profile at the fluid node's y = j + 1/2 (reading R8) */
static double inlet_u(const orc *o, int j) {
  double H = o->ny, y = j + 0.5;
  return 4.0 * o->p.u_in_max * y * (H - y) / (H * H);
}

/* Pull one population for fluid node (i, j) from the post-collision state,
 * eq. 2b with the boundary rules (reading R8).  *outlet is set when the link
 * comes through an OUTLET side (resolved afterwards by the caller). */
static double pull(const orc *o, int i, int j, int a, int *outlet) {
  int nx = o->nx, ny = o->ny;
  int si = i - EX[a], sj = j - EY[a];
  int xs = -1, ys = -1;
  if (si < 0) {
    if (o->side[SW] == ORC_PERIODIC) si += nx; else xs = SW;
  } else if (si >= nx) {
    if (o->side[SE] == ORC_PERIODIC) si -= nx; else xs = SE;
  }
  if (sj < 0) {
    if (o->side[SS] == ORC_PERIODIC) sj += ny; else ys = SS;
  } else if (sj >= ny) {
    if (o->side[SN] == ORC_PERIODIC) sj -= ny; else ys = SN;
  }
  if (outlet) *outlet = 0;
  double bb = FQ(o, o->f, OPP[a], i, j); /* half-way bounce-back */
  if (xs >= 0 && ys >= 0) return bb;     /* corner: stationary wall */
  if (xs >= 0 || ys >= 0) {
    int sd = xs >= 0 ? xs : ys;
    int kind = o->side[sd];
    double uwx = 0.0, uwy = 0.0;
    if (kind == ORC_WALL) return bb;
    if (kind == ORC_LID) {
      if (sd == SS || sd == SN) uwx = o->p.u_lid; else uwy = o->p.u_lid;
    } else if (kind == ORC_INLET) {
      uwx = inlet_u(o, j);
    } else { /* ORC_OUTLET */
      if (outlet) *outlet = 1;
      return 0.0;
    }
    /* momentum-augmented half-way bounce-back, rho_w = rho0 */
    return bb + 6.0 * WT[a] * o->p.rho0 * (EX[a] * uwx + EY[a] * uwy);
  }
  if (is_solid(o, si, sj)) return bb;
  return FQ(o, o->f, a, si, sj);
}

/* Outlet (reading R9) for fluid node (nx-1, j): fills the links that come
 * through the OUTLET side and records the new outlet velocity u*.  Reads only
 * the post-collision state f and the history, so the node order is free. */
static void outlet_links(orc *o, int j) {
  int nx = o->nx, ny = o->ny;
  double f2[9], m2[9], fe2[9], feo[9];
  for (int a = 0; a < 9; ++a) f2[a] = pull(o, nx - 2, j, a, NULL);
  orc_raw_moments(f2, m2);
  double r2 = m2[0];
  double u2 = (m2[1] + 0.5 * FXN(o, IDX(o, nx - 2, j)) / o->p.gamma) / r2;
  double v2 = (m2[2] + 0.5 * FYN(o, IDX(o, nx - 2, j)) / o->p.gamma) / r2;
  double U = o->p.u_in_max;
  double us = (o->hist[0 * ny + j] + U * u2) / (1.0 + U);
  double vs = (o->hist[1 * ny + j] + U * v2) / (1.0 + U);
  orc_equilibrium(r2, u2, v2, o->p.gamma, fe2);
  orc_equilibrium(o->p.rho0, us, vs, o->p.gamma, feo);
  for (int a = 0; a < 9; ++a) {
    int out = 0;
    (void)pull(o, nx - 1, j, a, &out);
    if (out) FQ(o, o->fb, a, nx - 1, j) = feo[a] + f2[a] - fe2[a];
  }
  o->hist_next[0 * ny + j] = us;
  o->hist_next[1 * ny + j] = vs;
}

/* Value of field q at the neighbour (i+di, j+dj) for a finite difference
 * (reading R7): periodic sides wrap; a neighbour beyond a non-periodic side
 * (whose wall lies half-way, at -1/2 or n - 1/2) takes the value of its
 * mirror image across that wall, the node on the lattice edge (zero normal
 * gradient at the wall); a solid neighbour takes the node's own value. */
static double nb_val(const orc *o, const double *q, int i, int j, int di, int dj) {
  int nx = o->nx, ny = o->ny;
  int ni = i + di, nj = j + dj;
  double own = q[IDX(o, i, j)];
  if (ni < 0 || ni >= nx) {
    if (o->side[ni < 0 ? SW : SE] != ORC_PERIODIC) ni = ni < 0 ? 0 : nx - 1;
    else ni = (ni + nx) % nx;
  }
  if (nj < 0 || nj >= ny) {
    if (o->side[nj < 0 ? SS : SN] != ORC_PERIODIC) nj = nj < 0 ? 0 : ny - 1;
    else nj = (nj + ny) % ny;
  }
  if (is_solid(o, ni, nj)) return own;
  return q[IDX(o, ni, nj)];
}

/* d/dx and d/dy of field q at (i, j): isotropic 3 sum_a w_a e_a q(x + e_a)
 * or central differences (drho_stencil). */
static void fd_grad(const orc *o, const double *q, int i, int j, double *gx, double *gy) {
  double x = 0.0, y = 0.0;
  if (o->p.drho_stencil == 0) {
    for (int a = 1; a < 9; ++a) {
      double v = nb_val(o, q, i, j, EX[a], EY[a]);
      x += 3.0 * WT[a] * EX[a] * v;
      y += 3.0 * WT[a] * EY[a] * v;
    }
  } else {
    x = 0.5 * (nb_val(o, q, i, j, 1, 0) - nb_val(o, q, i, j, -1, 0));
    y = 0.5 * (nb_val(o, q, i, j, 0, 1) - nb_val(o, q, i, j, 0, -1));
  }
  *gx = x;
  *gy = y;
}

/* Finite-difference gradient of a node field q [ny][nx] at every fluid node,
 * with the stencil of the parameters and the neighbour rule of reading R7
 * (the density-gradient step of Sec. 5 applies it to rho); solid nodes
 * receive 0.  Exposed so that the stencil and the neighbour rule can be
 * checked on their own. */
void orc_fd_gradient(const orc *o, const double *q, double *gx, double *gy) {
  for (int j = 0; j < o->ny; ++j)
    for (int i = 0; i < o->nx; ++i) {
      size_t k = IDX(o, i, j);
      if (o->solid[k]) {
        gx[k] = gy[k] = 0.0;
        continue;
      }
      fd_grad(o, q, i, j, &gx[k], &gy[k]);
    }
}

static int valid_sides(const int side[4]) {
  for (int s = 0; s < 4; ++s)
    if (side[s] < ORC_PERIODIC || side[s] > ORC_OUTLET) return 0;
  if ((side[SW] == ORC_PERIODIC) != (side[SE] == ORC_PERIODIC)) return 0;
  if ((side[SS] == ORC_PERIODIC) != (side[SN] == ORC_PERIODIC)) return 0;
  if (side[SE] == ORC_INLET || side[SS] == ORC_INLET || side[SN] == ORC_INLET) return 0;
  if (side[SW] == ORC_OUTLET || side[SS] == ORC_OUTLET || side[SN] == ORC_OUTLET) return 0;
  return 1;
}

double orc_omega_from_nu(double nu, double gamma) { return 1.0 / (3.0 * nu / gamma + 0.5); }

static void free_orc(orc *o) {
  free(o->ffx); free(o->ffy);
  free(o->solid); free(o->f); free(o->fb); free(o->rho); free(o->ux); free(o->uy);
  free(o->uxp); free(o->uyp); free(o->drx); free(o->dry); free(o->sxx); free(o->syy);
  free(o->hist); free(o->hist_next); free(o);
}

orc *orc_create(int nx, int ny, const int32_t side[4], const uint8_t *solid,
                const orc_params *p) {
  if (nx < 2 || ny < 2 || !p || !side) return NULL;
  int sd[4] = {side[0], side[1], side[2], side[3]};
  if (!valid_sides(sd)) return NULL;
  if (!(p->gamma > 0.0) || !(p->nu > 0.0) || !(p->rho0 > 0.0)) return NULL;
  double w4 = orc_omega_from_nu(p->nu, p->gamma);
  if (!(w4 > 0.0 && w4 < 2.0)) return NULL;
  orc *o = (orc *)calloc(1, sizeof(orc));
  if (!o) return NULL;
  o->nx = nx;
  o->ny = ny;
  memcpy(o->side, sd, sizeof sd);
  o->p = *p;
  o->omega4 = o->omega5 = w4;
  size_t n = (size_t)nx * ny;
  o->solid = (uint8_t *)calloc(n, 1);
  o->f = (double *)calloc(9 * n, sizeof(double));
  o->fb = (double *)calloc(9 * n, sizeof(double));
  o->rho = (double *)calloc(n, sizeof(double));
  o->ux = (double *)calloc(n, sizeof(double));
  o->uy = (double *)calloc(n, sizeof(double));
  o->uxp = (double *)calloc(n, sizeof(double));
  o->uyp = (double *)calloc(n, sizeof(double));
  o->drx = (double *)calloc(n, sizeof(double));
  o->dry = (double *)calloc(n, sizeof(double));
  o->sxx = (double *)calloc(n, sizeof(double));
  o->syy = (double *)calloc(n, sizeof(double));
  o->hist = (double *)calloc(2 * (size_t)ny, sizeof(double));
  o->hist_next = (double *)calloc(2 * (size_t)ny, sizeof(double));
  if (!o->solid || !o->f || !o->fb || !o->rho || !o->ux || !o->uy || !o->uxp ||
      !o->uyp || !o->drx || !o->dry || !o->sxx || !o->syy || !o->hist || !o->hist_next) {
    free_orc(o);
    return NULL;
  }
  if (solid) memcpy(o->solid, solid, n);
  {
    size_t fluid = 0;
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) fluid += !is_solid(o, i, j);
    if (fluid == 0) o->p.gamma = 0; /* no fluid node: invalid */
  }
  if (sd[SE] == ORC_OUTLET) {
    for (int j = 0; j < ny; ++j)
      if (is_solid(o, nx - 1, j) || is_solid(o, nx - 2, j)) {
        o->p.gamma = 0; /* mark invalid */
      }
  }
  {
    if (o->p.gamma == 0) {
      free_orc(o);
      return NULL;
    }
  }
  return o;
}

/* Per-node body force F(x, y) (copied; NULL, NULL returns to the uniform
 * force of the parameters).  Enters every place the uniform force does:
 * rho u = sum e fbar + F/(2 gamma) and the source moments of Sec. 2.
 * Returns 0, or -1 when only one component is given or memory runs out. */
int orc_set_force_field(orc *o, const double *fx, const double *fy) {
  if (!o || (!fx) != (!fy)) return -1;
  free(o->ffx);
  free(o->ffy);
  o->ffx = o->ffy = NULL;
  if (!fx) return 0;
  size_t n = (size_t)o->nx * o->ny;
  o->ffx = (double *)malloc(n * sizeof(double));
  o->ffy = (double *)malloc(n * sizeof(double));
  if (!o->ffx || !o->ffy) {
    free(o->ffx);
    free(o->ffy);
    o->ffx = o->ffy = NULL;
    return -1;
  }
  memcpy(o->ffx, fx, n * sizeof(double));
  memcpy(o->ffy, fy, n * sizeof(double));
  return 0;
}

void orc_destroy(orc *o) {
  if (o) free_orc(o);
}

/* Initial state: equilibrium at the given fields (NULL -> rho0, zero velocity).
 * Solid nodes hold the rest equilibrium and report zero fields. */
void orc_init_fields(orc *o, const double *rho, const double *ux, const double *uy) {
  int nx = o->nx, ny = o->ny;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      size_t k = IDX(o, i, j);
      double r = o->p.rho0, vx = 0.0, vy = 0.0;
      if (!o->solid[k]) {
        if (rho) r = rho[k];
        if (ux) vx = ux[k];
        if (uy) vy = uy[k];
      }
      double fe[9];
      orc_equilibrium(r, vx, vy, o->p.gamma, fe);
      for (int a = 0; a < 9; ++a) FQ(o, o->f, a, i, j) = fe[a];
      o->rho[k] = o->solid[k] ? 0.0 : r;
      o->ux[k] = o->solid[k] ? 0.0 : vx;
      o->uy[k] = o->solid[k] ? 0.0 : vy;
    }
  for (int j = 0; j < ny; ++j) {
    o->hist[0 * ny + j] = o->ux[IDX(o, nx - 1, j)];
    o->hist[1 * ny + j] = o->uy[IDX(o, nx - 1, j)];
  }
  o->steps = 0;
  o->resid = NAN;
  o->guards = 0;
}

static void one_step(orc *o) {
  int nx = o->nx, ny = o->ny;
  size_t n = (size_t)nx * ny;
  /* phase 1: stream (eq. 2b) with boundary links */
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      if (is_solid(o, i, j)) continue;
      int any_out = 0;
      for (int a = 0; a < 9; ++a) {
        int out = 0;
        double v = pull(o, i, j, a, &out);
        any_out |= out;
        FQ(o, o->fb, a, i, j) = v;
      }
      if (any_out) outlet_links(o, j);
    }
  if (o->side[SE] == ORC_OUTLET) {
    double *t = o->hist;
    o->hist = o->hist_next;
    o->hist_next = t;
  }
  /* phase 2: macroscopic fields of f = fbar + S/2 */
  memcpy(o->uxp, o->ux, n * sizeof(double));
  memcpy(o->uyp, o->uy, n * sizeof(double));
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      size_t k = IDX(o, i, j);
      if (o->solid[k]) continue;
      double r = 0.0, jx = 0.0, jy = 0.0;
      for (int a = 0; a < 9; ++a) {
        double v = FQ(o, o->fb, a, i, j);
        r += v;
        jx += EX[a] * v;
        jy += EY[a] * v;
      }
      o->rho[k] = r;
      o->ux[k] = (jx + 0.5 * FXN(o, k) / o->p.gamma) / r;
      o->uy[k] = (jy + 0.5 * FYN(o, k) / o->p.gamma) / r;
    }
  /* phase 3: density gradient at the same time level (reading R7) */
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      size_t k = IDX(o, i, j);
      if (o->solid[k]) continue;
      fd_grad(o, o->rho, i, j, &o->drx[k], &o->dry[k]);
      if (o->p.strain_fd) {
        double t;
        fd_grad(o, o->ux, i, j, &o->sxx[k], &t);
        fd_grad(o, o->uy, i, j, &t, &o->syy[k]);
      }
    }
  /* phase 4: collision (eq. 2a) */
  int64_t guards = 0;
#pragma omp parallel for schedule(static) reduction(+ : guards)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      size_t k = IDX(o, i, j);
      if (o->solid[k]) continue;
      double fb[9], fo[9], dg[8];
      for (int a = 0; a < 9; ++a) fb[a] = FQ(o, o->fb, a, i, j);
      orc_params pn = o->p;  /* the node's body force */
      pn.fx = FXN(o, k);
      pn.fy = FYN(o, k);
      double st[2] = {o->sxx[k], o->syy[k]};
      orc_collide_ext(fb, o->drx[k], o->dry[k], o->p.strain_fd ? st : NULL, &pn, o->omega4,
                      o->omega5, fo, dg);
      guards += dg[5] != 0.0;
      for (int a = 0; a < 9; ++a) FQ(o, o->f, a, i, j) = fo[a];
    }
  o->guards = guards;
  /* residual ||u^{n+1}-u^n||_2 / ||u^n||_2 and mass, summed in row order */
  double num = 0.0, den = 0.0, mass = 0.0;
  for (size_t k = 0; k < n; ++k) {
    if (o->solid[k]) continue;
    double dx = o->ux[k] - o->uxp[k], dy = o->uy[k] - o->uyp[k];
    num += dx * dx + dy * dy;
    den += o->uxp[k] * o->uxp[k] + o->uyp[k] * o->uyp[k];
    mass += o->rho[k];
  }
  o->resid = den > 0.0 ? sqrt(num / den) : (num > 0.0 ? INFINITY : 0.0);
  o->mass = mass;
  o->steps++;
}

/* Advance n steps.  Returns 0, or -4 when a field turned non-finite. */
int orc_step(orc *o, int64_t n) {
  for (int64_t s = 0; s < n; ++s) {
    one_step(o);
    if (!isfinite(o->mass) || isnan(o->resid)) return -4;
  }
  return 0;
}

/* Threads of the OpenMP loops of later steps (timing only; results do not
 * depend on it: the reductions are serial and in row order). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

double orc_residual(const orc *o) { return o->resid; }
double orc_mass(const orc *o) { return o->mass; }
int64_t orc_steps(const orc *o) { return o->steps; }
int64_t orc_guard_count(const orc *o) { return o->guards; }
double orc_omega4(const orc *o) { return o->omega4; }

void orc_fields(const orc *o, double *rho, double *ux, double *uy) {
  size_t n = (size_t)o->nx * o->ny;
  for (size_t k = 0; k < n; ++k) {
    if (rho) rho[k] = o->solid[k] ? 0.0 : o->rho[k];
    if (ux) ux[k] = o->solid[k] ? 0.0 : o->ux[k];
    if (uy) uy[k] = o->solid[k] ? 0.0 : o->uy[k];
  }
}

/* post-collision populations [9][ny][nx] */
void orc_get_f(const orc *o, double *f) {
  memcpy(f, o->f, 9 * (size_t)o->nx * o->ny * sizeof(double));
}
void orc_set_f(orc *o, const double *f) {
  memcpy(o->f, f, 9 * (size_t)o->nx * o->ny * sizeof(double));
}
