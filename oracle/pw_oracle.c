/*
 * Plain FP64 CPU oracle of the multipatch scalar-wave RK4 step of
 * "PatchworkWave" (Bowen et al., arXiv 2002.00088).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * leg of the benchmark may load this library.  It shares no source, header,
 * table or helper with the GPU library; every formula below is written out
 * again from the paper:
 *
 *   - covariant wave equation and its space/time split     (Sec. 2.2, Eqs. eom1-eom3)
 *   - Christoffel symbols from the metric                  (Sec. 2.2 and Appendix A)
 *   - one-form transformation law for Pi_mu                (Sec. 2.2)
 *   - classic RK4, two-part form u_{n+1/2}, u_{n+1}         (Sec. 2.3, Table rk4, Eqs. k1-k4)
 *   - Kreiss-Oliger dissipation, n = 5, eps = 0.005         (Sec. 2.3)
 *   - boundary hierarchy boundary -> periodic -> interpatch (Sec. 2.4, Fig. BC_order)
 *   - tensor-product Lagrange interpolation, 6 points/axis  (Sec. 2.4, Eq. Pijk)
 *   - global->local and local->global exchange via the
 *     background Cartesian frame, skip of uninterpolatable
 *     points                                               (Secs. 2.4.1, 2.4.2)
 *   - covered physical ghost cells of the global patch
 *     filled from the covering local patch                 (Sec. 2.4.2, last paragraph)
 *   - cover flags with a buffer of NG+1 live cells, flags
 *     frozen for the whole step                            (Sec. 2.4.2, Fig. cflag)
 *   - plane-wave exact solution, analytic outer BCs         (Sec. 3, Eq. wave_solution)
 *   - integrated relative error with the volume element    (Sec. 3.2)
 *   - Cartesian, spherical and cylindrical patch topologies,
 *     translating, circling and rotating patches            (Secs. 2.1, 3.2-3.4)
 *
 * Readings where the paper is silent or garbled (KO normalisation, mixed
 * derivative stencil, cell-centred grids, Chebyshev neighbourhoods for the
 * buffer, fallbacks for skipped points, wave speed v != 1) are listed in the
 * design notes of the repository and restated at the point of use.
 *
 * Parity pins: see the "not gpu" tests (polynomial exactness of every stencil,
 * the closed-form discrete Fourier-mode evolution, measured convergence order,
 * Lagrange exactness, closed-form spherical, cylindrical and spinning-patch
 * metrics, metrics against finite differences of the inverse map, transform
 * round trips, two-patch convergence order,
 * brute-force flag counts, energy and constraint behaviour; covered physical
 * ghosts against a brute-force cover test and exact polynomial interpolation,
 * several state vectors against one-vector worlds, the uncover fill against
 * polynomial fits through the stencil nodes).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NG 3           /* ghost width (Sec. 2.4.2: NG = 3) */
#define NF 5           /* phi, Pi_t, Pi_x, Pi_y, Pi_z */
#define MAXP 128
#define MAXSV 4
#define MAXG 32

enum { CART = 0, SPH = 1, CYL = 2 };
enum { STATIC = 0, LINEAR = 1, CIRCLE = 2 };
enum { FLAG_LIVE = 0, FLAG_EFFGHOST = 1, FLAG_DEACT = 2 };
enum { EX_NONE = 0, EX_PLANE = 1, EX_GAUSS = 2 };

/* ------------------------------------------------------------------------ */
/* Hyper-dual numbers a + b e1 + c e2 + d e1 e2 with e1^2 = e2^2 = 0.        */
/* Used to take first and mixed second derivatives of the coordinate maps.  */
/* ------------------------------------------------------------------------ */
typedef struct { double a, b, c, d; } hd;

static hd hd_const(double x) { hd r = {x, 0, 0, 0}; return r; }
static hd hd_add(hd x, hd y) { hd r = {x.a + y.a, x.b + y.b, x.c + y.c, x.d + y.d}; return r; }
static hd hd_scale(double s, hd x) { hd r = {s * x.a, s * x.b, s * x.c, s * x.d}; return r; }
static hd hd_mul(hd x, hd y) {
  hd r;
  r.a = x.a * y.a;
  r.b = x.a * y.b + x.b * y.a;
  r.c = x.a * y.c + x.c * y.a;
  r.d = x.a * y.d + x.b * y.c + x.c * y.b + x.d * y.a;
  return r;
}
/* f(x) for scalar f with derivative f1 and second derivative f2 at x.a */
static hd hd_fun(hd x, double f0, double f1, double f2) {
  hd r;
  r.a = f0;
  r.b = f1 * x.b;
  r.c = f1 * x.c;
  r.d = f1 * x.d + f2 * x.b * x.c;
  return r;
}
static hd hd_sin(hd x) { return hd_fun(x, sin(x.a), cos(x.a), -sin(x.a)); }
static hd hd_cos(hd x) { return hd_fun(x, cos(x.a), -sin(x.a), -cos(x.a)); }

/* ------------------------------------------------------------------------ */
/* Data structures                                                           */
/* ------------------------------------------------------------------------ */
typedef struct {
  int coord, is_global;
  int n[3], N[3];           /* interior cells, cells incl. ghosts (n + 2 NG) */
  double lo[3], hi[3], dx[3];
  int periodic[3];
  double R[3][3];           /* ZYZ Euler rotation at t = 0 */
  double spin[3];           /* angular velocity of a rotation about the centre (background frame) */
  int motion;
  double c0[3], vel[3], radius, speed, phase;
  unsigned sv_mask;
  double *u[MAXSV], *acc[MAXSV], *v[MAXSV], *k[MAXSV];
} or_patch;

typedef struct {
  int kind;
  double A, B, kap[3], psi;            /* plane wave */
  int ng;
  double amp[MAXG], xc[MAXG][3], w[MAXG]; /* Gaussian pulses */
} or_exact;

typedef struct {
  int np, nsv;
  double vs[MAXSV];         /* wave speed per state vector */
  int P[MAXSV];             /* interpolation points per axis per state vector */
  double eps;               /* KO strength */
  int buffer;               /* buffer width, NG + 1 in the paper */
  int form;                 /* 0: the paper's Pi_t equation (second derivatives of phi);
                               1: first-order form, Psi_i = Pi_i in place of d_i phi */
  int outer_bc;             /* global outer ghosts: 0 the exact solution (analytic BC);
                               1 evolved by the Sommerfeld radiative condition */
  int outer_ready;          /* Sommerfeld: the outer ghosts of u hold evolved values */
  or_patch p[MAXP];
  or_exact ex[MAXSV];
  double t;
  int flags_valid;
  uint8_t *flag;            /* global interior cells */
  int32_t *cover;           /* covering local patch or -1 */
  /* physical ghost cells of the global patch (outer ghosts whose periodic
   * wrap is not interior), and the local patch covering each one or -1 */
  int nghost;
  int32_t *ghost_ijk;       /* 3 per cell */
  int32_t *gcover;
  long long skip_local, skip_eff, skip_uncover, n_uncover;
  long long skip_outer, n_outer;
} or_world;

static long long pcells(const or_patch *p) { return (long long)p->N[0] * p->N[1] * p->N[2]; }
/* index of cell (i,j,k) (interior starts at 0, ghosts are negative / >= n) of field f */
static long long IX(const or_patch *p, int f, int i, int j, int k) {
  return (((long long)f * p->N[2] + (k + NG)) * p->N[1] + (j + NG)) * p->N[0] + (i + NG);
}
static long long GIX(const or_patch *g, int i, int j, int k) {
  return ((long long)k * g->n[1] + j) * g->n[0] + i;
}

/* numerical coordinate of the centre of cell i along axis a (cell-centred grid) */
static double xnum(const or_patch *p, int a, int i) { return p->lo[a] + (i + 0.5) * p->dx[a]; }

/* ------------------------------------------------------------------------ */
/* Coordinate maps X_B = c(t) + R . M(x') (Sec. 2.4.1: every patch knows its */
/* map from numerical to physical coordinates; all interpatch data travels  */
/* through the background Cartesian frame X_B).                             */
/* ------------------------------------------------------------------------ */
static void center_hd(const or_patch *p, hd t, hd c[3]) {
  for (int a = 0; a < 3; a++) c[a] = hd_const(p->c0[a]);
  if (p->motion == LINEAR) {
    for (int a = 0; a < 3; a++) c[a] = hd_add(c[a], hd_scale(p->vel[a], t));
  } else if (p->motion == CIRCLE) {
    double om = p->speed / p->radius;
    hd arg = hd_add(hd_scale(om, t), hd_const(p->phase));
    c[0] = hd_add(c[0], hd_scale(p->radius, hd_cos(arg)));
    c[1] = hd_add(c[1], hd_scale(p->radius, hd_sin(arg)));
  }
}

/* Orientation at time t: R(t) = Q(t) R(0), Q(t) the rotation by |w| t about the
 * axis w/|w| of the patch's angular velocity w (Rodrigues' formula,
 * Q = I + sin(th) K + (1 - cos(th)) K^2 with K the cross-product matrix of the
 * unit axis).  Without spin R(t) = R(0). */
static void orient_hd(const or_patch *p, hd t, hd Rt[3][3]) {
  const double wn = sqrt(p->spin[0] * p->spin[0] + p->spin[1] * p->spin[1] + p->spin[2] * p->spin[2]);
  if (wn == 0.0) {
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) Rt[a][b] = hd_const(p->R[a][b]);
    return;
  }
  const double k[3] = {p->spin[0] / wn, p->spin[1] / wn, p->spin[2] / wn};
  const double K[3][3] = {{0, -k[2], k[1]}, {k[2], 0, -k[0]}, {-k[1], k[0], 0}};
  double K2[3][3];
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) {
      K2[a][b] = 0.0;
      for (int m = 0; m < 3; m++) K2[a][b] += K[a][m] * K[m][b];
    }
  hd th = hd_scale(wn, t);
  hd sn = hd_sin(th), omc = hd_add(hd_const(1.0), hd_scale(-1.0, hd_cos(th)));
  hd Q[3][3];
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++)
      Q[a][b] = hd_add(hd_const(a == b ? 1.0 : 0.0), hd_add(hd_scale(K[a][b], sn), hd_scale(K2[a][b], omc)));
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) {
      hd s = hd_const(0.0);
      for (int m = 0; m < 3; m++) s = hd_add(s, hd_scale(p->R[m][b], Q[a][m]));
      Rt[a][b] = s;
    }
}

/* in = (t, x'1, x'2, x'3), out = (t, X, Y, Z) */
static void map_hd(const or_patch *p, const hd in[4], hd out[4]) {
  hd y[3];
  if (p->coord == CART) {
    y[0] = in[1]; y[1] = in[2]; y[2] = in[3];
  } else if (p->coord == CYL) {
    /* cylindrical x' = (r, phi, z): y = (r cos phi, r sin phi, z) */
    hd r = in[1], sp = hd_sin(in[2]), cp = hd_cos(in[2]);
    y[0] = hd_mul(r, cp);
    y[1] = hd_mul(r, sp);
    y[2] = in[3];
  } else {
    hd r = in[1], st = hd_sin(in[2]), ct = hd_cos(in[2]), sp = hd_sin(in[3]), cp = hd_cos(in[3]);
    y[0] = hd_mul(r, hd_mul(st, cp));
    y[1] = hd_mul(r, hd_mul(st, sp));
    y[2] = hd_mul(r, ct);
  }
  hd c[3], Rt[3][3];
  center_hd(p, in[0], c);
  orient_hd(p, in[0], Rt);
  out[0] = in[0];
  for (int a = 0; a < 3; a++) {
    hd s = c[a];
    for (int b = 0; b < 3; b++) s = hd_add(s, hd_mul(Rt[a][b], y[b]));
    out[1 + a] = s;
  }
}

static void map_fwd(const or_patch *p, double t, const double xp[3], double X[3]) {
  hd in[4] = {hd_const(t), hd_const(xp[0]), hd_const(xp[1]), hd_const(xp[2])}, out[4];
  map_hd(p, in, out);
  for (int a = 0; a < 3; a++) X[a] = out[1 + a].a;
}

static void center_val(const or_patch *p, double t, double c[3]) {
  hd c3[3];
  center_hd(p, hd_const(t), c3);
  for (int a = 0; a < 3; a++) c[a] = c3[a].a;
}

/* inverse map: background X -> numerical x' of patch p at time t */
static void map_inv(const or_patch *p, double t, const double X[3], double xp[3]) {
  double c[3], d[3], y[3];
  hd Rt[3][3];
  center_val(p, t, c);
  orient_hd(p, hd_const(t), Rt);
  for (int a = 0; a < 3; a++) d[a] = X[a] - c[a];
  for (int b = 0; b < 3; b++) y[b] = Rt[0][b].a * d[0] + Rt[1][b].a * d[1] + Rt[2][b].a * d[2];
  if (p->coord == CART) {
    for (int a = 0; a < 3; a++) xp[a] = y[a];
  } else if (p->coord == CYL) {
    xp[0] = sqrt(y[0] * y[0] + y[1] * y[1]);
    xp[1] = atan2(y[1], y[0]);
    xp[2] = y[2];
  } else {
    double r = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
    xp[0] = r;
    xp[1] = acos(y[2] / r);
    xp[2] = atan2(y[1], y[0]);
  }
}

/* E[alpha][mu] = d X^alpha / d x'^mu, 4x4 with index 0 = time */
static void jac4(const or_patch *p, double t, const double xp[3], double E[4][4]) {
  double x4[4] = {t, xp[0], xp[1], xp[2]};
  for (int mu = 0; mu < 4; mu++) {
    hd in[4], out[4];
    for (int k = 0; k < 4; k++) { in[k] = hd_const(x4[k]); in[k].b = (k == mu) ? 1.0 : 0.0; }
    map_hd(p, in, out);
    for (int al = 0; al < 4; al++) E[al][mu] = out[al].b;
  }
}

/* Gauss-Jordan inverse of a 4x4 matrix with partial pivoting */
static int inv4(const double A[4][4], double B[4][4]) {
  double M[4][8];
  for (int i = 0; i < 4; i++)
    for (int j = 0; j < 8; j++) M[i][j] = (j < 4) ? A[i][j] : (j - 4 == i ? 1.0 : 0.0);
  for (int c = 0; c < 4; c++) {
    int piv = c;
    for (int r = c + 1; r < 4; r++)
      if (fabs(M[r][c]) > fabs(M[piv][c])) piv = r;
    if (M[piv][c] == 0.0) return -1;
    if (piv != c)
      for (int j = 0; j < 8; j++) { double tmp = M[c][j]; M[c][j] = M[piv][j]; M[piv][j] = tmp; }
    double d = M[c][c];
    for (int j = 0; j < 8; j++) M[c][j] /= d;
    for (int r = 0; r < 4; r++) {
      if (r == c) continue;
      double f = M[r][c];
      if (f != 0.0)
        for (int j = 0; j < 8; j++) M[r][j] -= f * M[c][j];
    }
  }
  for (int i = 0; i < 4; i++)
    for (int j = 0; j < 4; j++) B[i][j] = M[i][j + 4];
  return 0;
}

/*
 * Inverse metric g^{mu nu} and the contraction C^lambda = g^{mu nu} Gamma^lambda_{mu nu}
 * of patch p at event (t, x').  The background is flat with
 * eta_{alpha beta} = diag(-v^2, 1, 1, 1) (the paper sets v = c = 1; a wave speed
 * v enters as d'Alembertian Lap - v^-2 d_t^2).  Following Sec. 2.2 and the
 * appendix: g_{mu nu} = E^a_mu E^b_nu eta_ab, g^{mu nu} its matrix inverse, and
 * Gamma^l_{mn} = 1/2 g^{ls} (d_m g_{sn} + d_n g_{ms} - d_s g_{mn}).
 * Metric derivatives come from exact second derivatives of the forward map.
 */
static void metric(const or_patch *p, double v, double t, const double xp[3],
                   double ginv[4][4], double C[4], double *sqrt_gamma) {
  double x4[4] = {t, xp[0], xp[1], xp[2]};
  double E[4][4], dE[4][4][4]; /* dE[rho][alpha][mu] = d^2 X^alpha / dx^rho dx^mu */
  for (int rho = 0; rho < 4; rho++)
    for (int mu = rho; mu < 4; mu++) {
      hd in[4], out[4];
      for (int k = 0; k < 4; k++) {
        in[k] = hd_const(x4[k]);
        in[k].b = (k == rho) ? 1.0 : 0.0;
        in[k].c = (k == mu) ? 1.0 : 0.0;
      }
      map_hd(p, in, out);
      for (int al = 0; al < 4; al++) {
        E[al][rho] = out[al].b;
        E[al][mu] = out[al].c;
        dE[rho][al][mu] = out[al].d;
        dE[mu][al][rho] = out[al].d;
      }
    }
  double eta[4] = {-v * v, 1.0, 1.0, 1.0};
  double g[4][4], dg[4][4][4];
  for (int m = 0; m < 4; m++)
    for (int n = 0; n < 4; n++) {
      double s = 0;
      for (int a = 0; a < 4; a++) s += E[a][m] * E[a][n] * eta[a];
      g[m][n] = s;
      for (int r = 0; r < 4; r++) {
        double q = 0;
        for (int a = 0; a < 4; a++) q += eta[a] * (dE[r][a][m] * E[a][n] + E[a][m] * dE[r][a][n]);
        dg[r][m][n] = q;
      }
    }
  inv4(g, ginv);
  for (int l = 0; l < 4; l++) {
    double s = 0;
    for (int m = 0; m < 4; m++)
      for (int n = 0; n < 4; n++) {
        double gam = 0;
        for (int q = 0; q < 4; q++) gam += 0.5 * ginv[l][q] * (dg[m][q][n] + dg[n][m][q] - dg[q][m][n]);
        s += ginv[m][n] * gam;
      }
    C[l] = s;
  }
  if (sqrt_gamma) {
    /* spatial volume element |det dX/dx'| */
    double (*J)[4] = E;
    double det = J[1][1] * (J[2][2] * J[3][3] - J[2][3] * J[3][2]) -
                 J[1][2] * (J[2][1] * J[3][3] - J[2][3] * J[3][1]) +
                 J[1][3] * (J[2][1] * J[3][2] - J[2][2] * J[3][1]);
    *sqrt_gamma = fabs(det);
  }
}

/* ------------------------------------------------------------------------ */
/* Exact solutions in the background frame: phi, d_t phi, grad phi          */
/* ------------------------------------------------------------------------ */

/* d^n/ds^n of g(s) = s exp(-s^2/w^2):  1/2 w^(1-n) (-1)^n H_{n+1}(s/w) e^{-(s/w)^2},
 * H the physicists' Hermite polynomials (derivatives of a Gaussian). */
static double gder(int n, double s, double w) {
  double u = s / w, hm = 1.0, h = 2.0 * u;
  for (int k = 1; k <= n; k++) { double hn = 2.0 * u * h - 2.0 * k * hm; hm = h; h = hn; }
  /* h = H_{n+1}(u) */
  double sg = (n % 2) ? -1.0 : 1.0;
  return 0.5 * pow(w, 1.0 - n) * sg * h * exp(-u * u);
}

/* Spherical pulse with phi(0,x) = exp(-|x-xc|^2/w^2), d_t phi(0,x) = 0:
 * rho*phi solves the 1-D wave equation, so with tau = v t
 *   phi = [g(tau+rho) - g(tau-rho)] / (2 rho).
 * Near rho = 0 the same expression is summed as its Taylor series in rho. */
static void gauss_pulse(double A, const double xc[3], double w, double v, double t,
                        const double X[3], double out[5]) {
  double d[3] = {X[0] - xc[0], X[1] - xc[1], X[2] - xc[2]};
  double rho = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  double tau = v * t, phi, dt, gradfac; /* grad phi = gradfac * d */
  if (rho < 0.05 * w) {
    double fk = 1.0;  /* (2k+1)! */
    double r2k = 1.0; /* rho^{2k} */
    double r2km2 = 0; /* rho^{2k-2} */
    phi = 0; dt = 0; gradfac = 0;
    for (int k = 0; k <= 5; k++) {
      if (k > 0) fk *= (2.0 * k) * (2.0 * k + 1.0);
      phi += gder(2 * k + 1, tau, w) * r2k / fk;
      dt += gder(2 * k + 2, tau, w) * r2k / fk;
      if (k >= 1) gradfac += gder(2 * k + 1, tau, w) * 2.0 * k * r2km2 / fk;
      r2km2 = (k == 0) ? 1.0 : r2km2 * rho * rho;
      r2k *= rho * rho;
    }
    dt *= v;
  } else {
    double gp = gder(0, tau + rho, w), gm = gder(0, tau - rho, w);
    double g1p = gder(1, tau + rho, w), g1m = gder(1, tau - rho, w);
    phi = (gp - gm) / (2.0 * rho);
    dt = v * (g1p - g1m) / (2.0 * rho);
    double drho = (g1p + g1m) / (2.0 * rho) - phi / rho;
    gradfac = drho / rho;
  }
  out[0] = A * phi;
  out[1] = A * dt;
  for (int a = 0; a < 3; a++) out[2 + a] = A * gradfac * d[a];
}

static void exact_bg(const or_exact *e, double v, double t, const double X[3], double out[5]) {
  for (int f = 0; f < 5; f++) out[f] = 0;
  if (e->kind == EX_PLANE) {
    /* phi = A sin(k.X - omega t + psi) + B, omega = v |k|   (Eq. wave_solution) */
    double kn = sqrt(e->kap[0] * e->kap[0] + e->kap[1] * e->kap[1] + e->kap[2] * e->kap[2]);
    double arg = e->kap[0] * X[0] + e->kap[1] * X[1] + e->kap[2] * X[2] - v * kn * t + e->psi;
    out[0] = e->A * sin(arg) + e->B;
    out[1] = -e->A * v * kn * cos(arg);
    for (int a = 0; a < 3; a++) out[2 + a] = e->A * e->kap[a] * cos(arg);
  } else if (e->kind == EX_GAUSS) {
    for (int g = 0; g < e->ng; g++) {
      double o[5];
      gauss_pulse(e->amp[g], e->xc[g], e->w[g], v, t, X, o);
      for (int f = 0; f < 5; f++) out[f] += o[f];
    }
  }
}

/* Exact state in the numerical frame of patch p: Pi_{mu'} = (dX^a/dx'^mu) Pi_a. */
static void exact_patch(const or_world *w, const or_patch *p, int sv, double t,
                        const double xp[3], double out[5]) {
  double X[3], bg[5], E[4][4];
  map_fwd(p, t, xp, X);
  exact_bg(&w->ex[sv], w->vs[sv], t, X, bg);
  jac4(p, t, xp, E);
  out[0] = bg[0];
  for (int mu = 0; mu < 4; mu++) {
    double s = 0;
    for (int a = 0; a < 4; a++) s += E[a][mu] * bg[1 + a];
    out[1 + mu] = s;
  }
}

/* ------------------------------------------------------------------------ */
/* Finite differences: textbook centred 4th-order weights, 6th undivided    */
/* difference for Kreiss-Oliger.                                             */
/* ------------------------------------------------------------------------ */
static const double W1[5] = {1.0 / 12, -8.0 / 12, 0.0, 8.0 / 12, -1.0 / 12};   /* d/dx  * dx   */
static const double W2[5] = {-1.0 / 12, 16.0 / 12, -30.0 / 12, 16.0 / 12, -1.0 / 12}; /* d2/dx2 * dx^2 */
static const double W6[7] = {1, -6, 15, -20, 15, -6, 1};                          /* Delta^6 */

static double at(const or_patch *p, const double *T, int f, int i, int j, int k, int d, int o) {
  int ii = i + (d == 0 ? o : 0), jj = j + (d == 1 ? o : 0), kk = k + (d == 2 ? o : 0);
  return T[IX(p, f, ii, jj, kk)];
}
static double D1(const or_patch *p, const double *T, int f, int i, int j, int k, int d) {
  double s = 0;
  for (int o = -2; o <= 2; o++) s += W1[o + 2] * at(p, T, f, i, j, k, d, o);
  return s / p->dx[d];
}
static double D2(const or_patch *p, const double *T, int f, int i, int j, int k, int d) {
  double s = 0;
  for (int o = -2; o <= 2; o++) s += W2[o + 2] * at(p, T, f, i, j, k, d, o);
  return s / (p->dx[d] * p->dx[d]);
}
/* mixed derivative as the composition of two first-derivative stencils */
static double D11(const or_patch *p, const double *T, int f, int i, int j, int k, int d, int e) {
  double s = 0;
  for (int o1 = -2; o1 <= 2; o1++)
    for (int o2 = -2; o2 <= 2; o2++) {
      int off[3] = {0, 0, 0};
      off[d] += o1;
      off[e] += o2;
      s += W1[o1 + 2] * W1[o2 + 2] * T[IX(p, f, i + off[0], j + off[1], k + off[2])];
    }
  return s / (p->dx[d] * p->dx[e]);
}
/* Kreiss-Oliger term with n = 5: (eps / 2^6) * sum_d Delta^6_d u / dx_d */
static double KO(const or_patch *p, const double *T, int f, int i, int j, int k, double eps) {
  double s = 0;
  for (int d = 0; d < 3; d++) {
    double q = 0;
    for (int o = -3; o <= 3; o++) q += W6[o + 3] * at(p, T, f, i, j, k, d, o);
    s += q / p->dx[d];
  }
  return eps / 64.0 * s;
}

/* RHS of Eqs. eom1-eom3 (S = 0) plus KO on every field at cell (i,j,k) */
static void rhs_cell(const or_world *w, const or_patch *p, int sv, const double *T, double t,
                     int i, int j, int k, double K[5]) {
  double xp[3] = {xnum(p, 0, i), xnum(p, 1, j), xnum(p, 2, k)};
  double gi[4][4], C[4];
  metric(p, w->vs[sv], t, xp, gi, C, NULL);
  double Pi = T[IX(p, 1, i, j, k)];
  double dphi[3], dpi[3], ddphi[3][3];
  for (int d = 0; d < 3; d++) {
    dphi[d] = D1(p, T, 0, i, j, k, d);
    dpi[d] = D1(p, T, 1, i, j, k, d);
  }
  for (int d = 0; d < 3; d++)
    for (int e = 0; e < 3; e++) ddphi[d][e] = (d == e) ? D2(p, T, 0, i, j, k, d) : D11(p, T, 0, i, j, k, d, e);
  if (w->form == 1) {
    /* first-order reduction: the evolved Psi_i = Pi_i stands for d_i phi, and
     * d_a Psi_b for d_a d_b phi (the wave operator as a divergence of Psi) */
    for (int d = 0; d < 3; d++) dphi[d] = T[IX(p, 2 + d, i, j, k)];
    for (int d = 0; d < 3; d++)
      for (int e = 0; e < 3; e++) ddphi[d][e] = D1(p, T, 2 + e, i, j, k, d);
  }
  double br = C[0] * Pi;
  for (int j2 = 0; j2 < 3; j2++) br += C[1 + j2] * dphi[j2];
  for (int j2 = 0; j2 < 3; j2++) br -= 2.0 * gi[0][1 + j2] * dpi[j2];
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) br -= gi[1 + a][1 + b] * ddphi[a][b];
  K[0] = Pi + KO(p, T, 0, i, j, k, w->eps);
  K[1] = br / gi[0][0] + KO(p, T, 1, i, j, k, w->eps);
  for (int d = 0; d < 3; d++) K[2 + d] = dpi[d] + KO(p, T, 2 + d, i, j, k, w->eps);
}

/* ------------------------------------------------------------------------ */
/* Lagrange interpolation (Sec. 2.4, Eq. Pijk)                              */
/* ------------------------------------------------------------------------ */
/* q is the fractional cell index (cell centre m sits at q = m).  The stencil of
 * P nodes starts at s = floor(q - (P-2)/2): for P = 6 that is i_c - 2 with i_c
 * the last node not beyond the point, as in the paper; for P = 5 it is centred
 * on the nearest node. */
static void lagrange(int P, double q, int *s, double wts[8]) {
  int s0 = (int)floor(q - 0.5 * (P - 2));
  *s = s0;
  for (int m = 0; m < P; m++) {
    double num = 1.0, den = 1.0;
    for (int l = 0; l < P; l++) {
      if (l == m) continue;
      num *= (q - (double)(s0 + l));
      den *= (double)(m - l);
    }
    wts[m] = num / den;
  }
}

static int wrapi(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }

static int is_interior(const or_patch *p, const int c[3]) {
  for (int a = 0; a < 3; a++)
    if (c[a] < 0 || c[a] >= p->n[a]) return 0;
  return 1;
}

/* Interpolate all fields of buffer T of donor d at background point X, time t.
 * Returns 1 if every stencil cell is a live interior cell, else 0 (skip). */
static int interp_donor(const or_world *w, int d, int sv, const double *T, double t,
                        const double X[3], double out[5], double xd[3]) {
  const or_patch *p = &w->p[d];
  int P = w->P[sv];
  double q[3], wt[3][8];
  int s[3];
  map_inv(p, t, X, xd);
  for (int a = 0; a < 3; a++) {
    q[a] = (xd[a] - p->lo[a]) / p->dx[a] - 0.5;
    if (!(q[a] == q[a])) return 0;
    if (q[a] < -1e6 || q[a] > 1e6 + p->n[a]) return 0;
    lagrange(P, q[a], &s[a], wt[a]);
    if (!p->periodic[a] && (s[a] < 0 || s[a] + P - 1 > p->n[a] - 1)) return 0;
  }
  if (p->is_global) {
    for (int c = 0; c < P; c++)
      for (int b = 0; b < P; b++)
        for (int a = 0; a < P; a++) {
          int ii = p->periodic[0] ? wrapi(s[0] + a, p->n[0]) : s[0] + a;
          int jj = p->periodic[1] ? wrapi(s[1] + b, p->n[1]) : s[1] + b;
          int kk = p->periodic[2] ? wrapi(s[2] + c, p->n[2]) : s[2] + c;
          uint8_t fl = w->flag[GIX(p, ii, jj, kk)];
          /* paper's buffer: live donors only; narrower buffer: effective
           * ghosts (already filled this stage) may serve as donors too */
          if (w->buffer >= NG + 1 ? fl != FLAG_LIVE : fl == FLAG_DEACT) return 0;
        }
  }
  for (int f = 0; f < NF; f++) {
    double sum = 0;
    for (int c = 0; c < P; c++)
      for (int b = 0; b < P; b++)
        for (int a = 0; a < P; a++) {
          int ii = p->periodic[0] ? wrapi(s[0] + a, p->n[0]) : s[0] + a;
          int jj = p->periodic[1] ? wrapi(s[1] + b, p->n[1]) : s[1] + b;
          int kk = p->periodic[2] ? wrapi(s[2] + c, p->n[2]) : s[2] + c;
          sum += wt[0][a] * wt[1][b] * wt[2][c] * T[IX(p, f, ii, jj, kk)];
        }
    out[f] = sum;
  }
  return 1;
}

/* Move an interpolated state from donor frame to receiver frame through the
 * background frame (Secs. 2.4.1-2.4.2): Pi^B_a = (dx_d^l/dX^a) Pi^d_l, then
 * Pi^r_mu = (dX^a/dx_r^mu) Pi^B_a.  dx_d/dX is the matrix inverse of dX/dx_d. */
static void transform(const or_patch *pd, const double xd[3], const or_patch *pr, const double xr[3],
                      double t, const double in[5], double out[5]) {
  double Ed[4][4], Ld[4][4], Er[4][4], B[4];
  jac4(pd, t, xd, Ed);
  inv4(Ed, Ld);
  jac4(pr, t, xr, Er);
  for (int a = 0; a < 4; a++) {
    double s = 0;
    for (int l = 0; l < 4; l++) s += Ld[l][a] * in[1 + l];
    B[a] = s;
  }
  out[0] = in[0];
  for (int mu = 0; mu < 4; mu++) {
    double s = 0;
    for (int a = 0; a < 4; a++) s += Er[a][mu] * B[a];
    out[1 + mu] = s;
  }
}

/* ------------------------------------------------------------------------ */
/* Cover flags (Sec. 2.4.2)                                                  */
/* ------------------------------------------------------------------------ */
static double bound_radius(const or_patch *p) {
  if (p->coord == SPH) return p->hi[0];
  if (p->coord == CYL) {
    double zm = fabs(p->lo[2]) > fabs(p->hi[2]) ? fabs(p->lo[2]) : fabs(p->hi[2]);
    return sqrt(p->hi[0] * p->hi[0] + zm * zm);
  }
  double m = 0;
  for (int c = 0; c < 8; c++) {
    double y0 = (c & 1) ? p->hi[0] : p->lo[0], y1 = (c & 2) ? p->hi[1] : p->lo[1], y2 = (c & 4) ? p->hi[2] : p->lo[2];
    double r = sqrt(y0 * y0 + y1 * y1 + y2 * y2);
    if (r > m) m = r;
  }
  return m;
}

/* is background point X inside the closed numerical box of local patch p at t? */
/* background position of global cell (i,j,k): the global patch is static and
 * unrotated at the origin, so a Cartesian global's numerical coordinates are X */
static void global_X(const or_patch *g, double t, int i, int j, int k, double X[3]) {
  double xp[3] = {xnum(g, 0, i), xnum(g, 1, j), xnum(g, 2, k)};
  if (g->coord == CART) {
    for (int a = 0; a < 3; a++) X[a] = xp[a];
  } else {
    map_fwd(g, t, xp, X);
  }
}

/* neighbour index along axis a of the global patch: wraps a periodic axis;
 * returns 0 if the index leaves a non-periodic axis */
static int gneighbour(const or_patch *g, int a, int i, int *out) {
  if (g->periodic[a]) { *out = wrapi(i, g->n[a]); return 1; }
  if (i < 0 || i >= g->n[a]) return 0;
  *out = i;
  return 1;
}

static int covers(const or_patch *p, double t, const double c[3], const double X[3]) {
  double d2 = 0, xp[3];
  for (int a = 0; a < 3; a++) d2 += (X[a] - c[a]) * (X[a] - c[a]);
  double R = bound_radius(p) * (1.0 + 1e-12) + 1e-12;
  if (d2 > R * R) return 0;
  map_inv(p, t, X, xp);
  for (int a = 0; a < 3; a++) {
    if (p->periodic[a]) continue;
    if (!(xp[a] >= p->lo[a] && xp[a] <= p->hi[a])) return 0;
  }
  return 1;
}

/* list of the physical ghost cells of the global patch: ghost cells whose
 * periodic wrap is not an interior cell (the outer boundary, not a periodic copy) */
static void list_physical_ghosts(or_world *w) {
  if (w->ghost_ijk) return;
  const or_patch *g = &w->p[0];
  long long cap = pcells(g), m = 0;
  w->ghost_ijk = (int32_t *)malloc(3 * cap * sizeof(int32_t));
  for (int k = -NG; k < g->n[2] + NG; k++)
    for (int j = -NG; j < g->n[1] + NG; j++)
      for (int i = -NG; i < g->n[0] + NG; i++) {
        int c[3] = {i, j, k}, cw[3];
        if (is_interior(g, c)) continue;
        for (int a = 0; a < 3; a++) cw[a] = g->periodic[a] ? wrapi(c[a], g->n[a]) : c[a];
        if (is_interior(g, cw)) continue;
        w->ghost_ijk[3 * m] = i;
        w->ghost_ijk[3 * m + 1] = j;
        w->ghost_ijk[3 * m + 2] = k;
        m++;
      }
  w->nghost = (int)m;
  w->gcover = (int32_t *)malloc((m > 0 ? m : 1) * sizeof(int32_t));
  for (long long q = 0; q < m; q++) w->gcover[q] = -1;
}

/* covered -> live if within `buffer` cells (Chebyshev) of an uncovered cell,
 * else effective ghost if within NG cells of a live cell, else deactivated.
 * Cells outside the global domain count as uncovered.  Also: the local patch
 * covering each physical ghost cell of the global patch (gcover, lower id
 * first), the targets of the covered-ghost fill (Sec. 2.4.2, last paragraph). */
static int compute_flags(or_world *w, double t, uint8_t *flag, int32_t *cover, int32_t *gcover) {
  const or_patch *g = &w->p[0];
  long long ncell = (long long)g->n[0] * g->n[1] * g->n[2];
  for (int q = 0; q < w->nghost; q++) gcover[q] = -1;
  for (int pi = 1; pi < w->np; pi++) {
    const or_patch *p = &w->p[pi];
    double cp[3];
    center_val(p, t, cp);
#pragma omp parallel for schedule(static)
    for (int q = 0; q < w->nghost; q++) {
      double X[3];
      global_X(g, t, w->ghost_ijk[3 * q], w->ghost_ijk[3 * q + 1], w->ghost_ijk[3 * q + 2], X);
      if (gcover[q] == -1 && covers(p, t, cp, X)) gcover[q] = pi;
    }
  }
  /* a cell covered by two local patches keeps the lower patch id; such
   * overlaps are allowed where the cell stays live (the buffers), and are an
   * error anywhere else */
  uint8_t *dbl = (uint8_t *)calloc(ncell, 1);
  for (long long c = 0; c < ncell; c++) cover[c] = -1;
  for (int pi = 1; pi < w->np; pi++) {
    const or_patch *p = &w->p[pi];
    double cp[3];
    center_val(p, t, cp);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < g->n[2]; k++)
      for (int j = 0; j < g->n[1]; j++)
        for (int i = 0; i < g->n[0]; i++) {
          double X[3];
          global_X(g, t, i, j, k, X);
          if (covers(p, t, cp, X)) {
            long long c = GIX(g, i, j, k);
            if (cover[c] != -1) dbl[c] = 1;
            else cover[c] = pi;
          }
        }
  }
  int B = w->buffer;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < g->n[2]; k++)
    for (int j = 0; j < g->n[1]; j++)
      for (int i = 0; i < g->n[0]; i++) {
        long long c = GIX(g, i, j, k);
        int live = (cover[c] == -1);
        for (int dk = -B; dk <= B && !live; dk++)
          for (int dj = -B; dj <= B && !live; dj++)
            for (int di = -B; di <= B && !live; di++) {
              int ii, jj, kk;
              if (!gneighbour(g, 0, i + di, &ii) || !gneighbour(g, 1, j + dj, &jj) || !gneighbour(g, 2, k + dk, &kk))
                live = 1;
              else if (cover[GIX(g, ii, jj, kk)] == -1)
                live = 1;
            }
        flag[c] = live ? FLAG_LIVE : FLAG_DEACT;
      }
  uint8_t *eff = (uint8_t *)calloc(ncell, 1);
#pragma omp parallel for schedule(static)
  for (int k = 0; k < g->n[2]; k++)
    for (int j = 0; j < g->n[1]; j++)
      for (int i = 0; i < g->n[0]; i++) {
        long long c = GIX(g, i, j, k);
        if (flag[c] == FLAG_LIVE) continue;
        int near = 0;
        for (int dk = -NG; dk <= NG && !near; dk++)
          for (int dj = -NG; dj <= NG && !near; dj++)
            for (int di = -NG; di <= NG && !near; di++) {
              int ii, jj, kk;
              if (!gneighbour(g, 0, i + di, &ii) || !gneighbour(g, 1, j + dj, &jj) || !gneighbour(g, 2, k + dk, &kk))
                continue;
              if (flag[GIX(g, ii, jj, kk)] == FLAG_LIVE) near = 1;
            }
        eff[c] = (uint8_t)near;
      }
  int overlap = 0;
  for (long long c = 0; c < ncell; c++) {
    if (eff[c]) flag[c] = FLAG_EFFGHOST;
    if (dbl[c] && flag[c] != FLAG_LIVE) overlap = 1;
  }
  free(eff);
  free(dbl);
  return overlap ? -5 : 0;
}

static int is_live(const or_world *w, const or_patch *p, int i, int j, int k) {
  if (!p->is_global || w->np == 1) return 1;
  return w->flag[GIX(p, i, j, k)] == FLAG_LIVE;
}

/* ------------------------------------------------------------------------ */
/* Ghost fill at time t (Sec. 2.4): boundary -> periodic -> interpatch       */
/* which = 0: the u buffers, which = 1: the stage buffers v                  */
/* ------------------------------------------------------------------------ */
static double *bufsel(or_patch *p, int sv, int which) { return which == 0 ? p->u[sv] : p->v[sv]; }


/* level 3a: global -> local, every non-periodic ghost cell of every local patch */
static void fill_g2l(or_world *w, int which, double t, long long *skips) {
  or_patch *g = &w->p[0];
  long long sk_l = 0;
  for (int pi = 1; pi < w->np; pi++) {
    or_patch *p = &w->p[pi];
    for (int sv = 0; sv < w->nsv; sv++) {
      if (!(p->sv_mask & (1u << sv)) || !(g->sv_mask & (1u << sv))) continue;
      double *T = bufsel(p, sv, which);
      const double *TG = bufsel(g, sv, which);
#pragma omp parallel for schedule(dynamic) reduction(+ : sk_l)
      for (int k = -NG; k < p->n[2] + NG; k++)
        for (int j = -NG; j < p->n[1] + NG; j++)
          for (int i = -NG; i < p->n[0] + NG; i++) {
            int c[3] = {i, j, k}, cw[3];
            if (is_interior(p, c)) continue;
            for (int a = 0; a < 3; a++) cw[a] = p->periodic[a] ? wrapi(c[a], p->n[a]) : c[a];
            if (is_interior(p, cw)) continue;
            double xr[3] = {xnum(p, 0, i), xnum(p, 1, j), xnum(p, 2, k)}, X[3], xd[3], ud[5], ur[5];
            map_fwd(p, t, xr, X);
            if (!interp_donor(w, 0, sv, TG, t, X, ud, xd)) { sk_l++; continue; }
            transform(g, xd, p, xr, t, ud, ur);
            for (int f = 0; f < NF; f++) T[IX(p, f, i, j, k)] = ur[f];
          }
    }
  }
  *skips += sk_l;
}

/* level 3b: local -> global, effective ghost cells of the global patch */
static void fill_l2g(or_world *w, int which, double t, long long *skips) {
  or_patch *g = &w->p[0];
  long long sk_e = 0;
  for (int sv = 0; sv < w->nsv; sv++) {
    if (!(g->sv_mask & (1u << sv))) continue;
    double *TG = bufsel(g, sv, which);
#pragma omp parallel for schedule(dynamic) reduction(+ : sk_e)
    for (int k = 0; k < g->n[2]; k++)
      for (int j = 0; j < g->n[1]; j++)
        for (int i = 0; i < g->n[0]; i++) {
          long long c = GIX(g, i, j, k);
          if (w->flag[c] != FLAG_EFFGHOST) continue;
          or_patch *p = &w->p[w->cover[c]];
          double xr[3] = {xnum(g, 0, i), xnum(g, 1, j), xnum(g, 2, k)}, X[3], xd[3], ud[5], ur[5];
          global_X(g, t, i, j, k, X);
          int ok = (p->sv_mask & (1u << sv)) && interp_donor(w, w->cover[c], sv, bufsel(p, sv, which), t, X, ud, xd);
          if (ok) {
            transform(p, xd, g, xr, t, ud, ur);
          } else {
            sk_e++;
            if (w->ex[sv].kind != EX_NONE) exact_patch(w, g, sv, t, xr, ur);
            else for (int f = 0; f < NF; f++) ur[f] = NAN;
          }
          for (int f = 0; f < NF; f++) TG[IX(g, f, i, j, k)] = ur[f];
        }
  }
  *skips += sk_e;
}

/* level 3c: local -> global, covered physical ghost cells of the global patch
 * (Sec. 2.4.2, last paragraph): an outer ghost cell of the global patch that
 * lies in a local patch takes the value interpolated from that patch; where
 * the stencil leaves the local interior the boundary value of levels 1-2
 * stays (skip).  The Sommerfeld variant evolves its outer ghosts instead. */
static void fill_outer_covered(or_world *w, int which, double t, long long *skips, long long *targets) {
  if (w->outer_bc != 0) return;
  or_patch *g = &w->p[0];
  long long sk = 0, nt = 0;
  for (int sv = 0; sv < w->nsv; sv++) {
    if (!(g->sv_mask & (1u << sv))) continue;
    double *TG = bufsel(g, sv, which);
#pragma omp parallel for schedule(dynamic) reduction(+ : sk, nt)
    for (int q = 0; q < w->nghost; q++) {
      int d = w->gcover[q];
      if (d < 0) continue;
      nt++;
      int i = w->ghost_ijk[3 * q], j = w->ghost_ijk[3 * q + 1], k = w->ghost_ijk[3 * q + 2];
      or_patch *p = &w->p[d];
      double xr[3] = {xnum(g, 0, i), xnum(g, 1, j), xnum(g, 2, k)}, X[3], xd[3], ud[5], ur[5];
      global_X(g, t, i, j, k, X);
      int ok = (p->sv_mask & (1u << sv)) && interp_donor(w, d, sv, bufsel(p, sv, which), t, X, ud, xd);
      if (!ok) { sk++; continue; }
      transform(p, xd, g, xr, t, ud, ur);
      for (int f = 0; f < NF; f++) TG[IX(g, f, i, j, k)] = ur[f];
    }
  }
  *skips += sk;
  *targets += nt;
}

static void fill_ghosts(or_world *w, int which, double t) {
  long long sk_l = 0, sk_e = 0;
  for (int pi = 0; pi < w->np; pi++) {
    or_patch *p = &w->p[pi];
    for (int sv = 0; sv < w->nsv; sv++) {
      if (!(p->sv_mask & (1u << sv))) continue;
      double *T = bufsel(p, sv, which);
      /* level 1 and 2: analytic outer boundary / nearest copy, then periodic copies */
#pragma omp parallel for schedule(dynamic)
      for (int k = -NG; k < p->n[2] + NG; k++)
        for (int j = -NG; j < p->n[1] + NG; j++)
          for (int i = -NG; i < p->n[0] + NG; i++) {
            int c[3] = {i, j, k};
            if (is_interior(p, c)) continue;
            int cw[3];
            for (int a = 0; a < 3; a++) cw[a] = p->periodic[a] ? wrapi(c[a], p->n[a]) : c[a];
            if (is_interior(p, cw)) {
              /* a periodic global patch with local patches copies after the
               * interpatch fill, so its copies carry the effective ghosts' values */
              if (p->is_global && w->np > 1) continue;
              for (int f = 0; f < NF; f++) T[IX(p, f, i, j, k)] = T[IX(p, f, cw[0], cw[1], cw[2])];
            } else if (p->is_global && w->outer_bc == 1) {
              continue; /* evolved by the radiative condition */
            } else if (w->ex[sv].kind != EX_NONE) {
              double xp[3] = {xnum(p, 0, i), xnum(p, 1, j), xnum(p, 2, k)}, e[5];
              exact_patch(w, p, sv, t, xp, e);
              for (int f = 0; f < NF; f++) T[IX(p, f, i, j, k)] = e[f];
            } else {
              int cc[3];
              for (int a = 0; a < 3; a++) cc[a] = cw[a] < 0 ? 0 : (cw[a] >= p->n[a] ? p->n[a] - 1 : cw[a]);
              for (int f = 0; f < NF; f++) T[IX(p, f, i, j, k)] = T[IX(p, f, cc[0], cc[1], cc[2])];
            }
          }
    }
  }
  if (w->np == 1) return;
  /* level 3: interpatch.  With the paper's buffer (NG + 1 live cells) neither
   * direction reads the other's output, and global -> local comes first.  With
   * a narrower buffer (the ablation of the original Patchwork flags) the
   * global -> local stencils may reach effective ghosts, which therefore are
   * filled first (interpolation of interpolated data). */
  if (w->buffer >= NG + 1) {
    fill_g2l(w, which, t, &sk_l);
    fill_l2g(w, which, t, &sk_e);
  } else {
    fill_l2g(w, which, t, &sk_e);
    fill_g2l(w, which, t, &sk_l);
  }
  fill_outer_covered(w, which, t, &w->skip_outer, &w->n_outer);
  /* periodic copies of the global patch (a spherical global's phi axis) */
  or_patch *g = &w->p[0];
  for (int sv = 0; sv < w->nsv; sv++) {
    if (!(g->sv_mask & (1u << sv))) continue;
    double *T = bufsel(g, sv, which);
    for (int k = -NG; k < g->n[2] + NG; k++)
      for (int j = -NG; j < g->n[1] + NG; j++)
        for (int i = -NG; i < g->n[0] + NG; i++) {
          int c[3] = {i, j, k}, cw[3];
          if (is_interior(g, c)) continue;
          for (int a = 0; a < 3; a++) cw[a] = g->periodic[a] ? wrapi(c[a], g->n[a]) : c[a];
          if (!is_interior(g, cw)) continue;
          for (int f = 0; f < NF; f++) T[IX(g, f, i, j, k)] = T[IX(g, f, cw[0], cw[1], cw[2])];
        }
  }
  w->skip_local += sk_l;
  w->skip_eff += sk_e;
}

/* ------------------------------------------------------------------------ */
/* Sommerfeld outer boundary (variant; the paper lays the exact solution into */
/* the outer ghosts).  Each outer ghost cell of the (non-periodic) global     */
/* patch is evolved with the radiative condition for waves leaving the       */
/* origin, d_t u = -v (X.grad u + u) / r, r = |X|, on every field (falloff    */
/* u ~ f(r - vt)/r, asymptotic value 0).  Derivatives: 4th-order centred      */
/* along axes where the cell is interior, 2nd-order one-sided (inward) along  */
/* axes where it is a ghost.                                                  */
/* ------------------------------------------------------------------------ */
static int is_outer_ghost(const or_patch *p, int i, int j, int k) {
  int c[3] = {i, j, k};
  return !is_interior(p, c);
}

static void radiative_rhs(const or_world *w, const or_patch *p, int sv, const double *T, int i, int j, int k,
                          double K[5]) {
  const int c[3] = {i, j, k};
  double X[3] = {xnum(p, 0, i), xnum(p, 1, j), xnum(p, 2, k)};
  double r = sqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
  double v = w->vs[sv];
  for (int f = 0; f < NF; f++) {
    double xgrad = 0.0;
    for (int a = 0; a < 3; a++) {
      int e[3] = {0, 0, 0};
      e[a] = 1;
#define UAT(s) T[IX(p, f, c[0] + (s) * e[0], c[1] + (s) * e[1], c[2] + (s) * e[2])]
      double d;
      if (c[a] < 0)
        d = (-3.0 * UAT(0) + 4.0 * UAT(1) - UAT(2)) / (2.0 * p->dx[a]);
      else if (c[a] >= p->n[a])
        d = (3.0 * UAT(0) - 4.0 * UAT(-1) + UAT(-2)) / (2.0 * p->dx[a]);
      else
        d = (UAT(-2) - 8.0 * UAT(-1) + 8.0 * UAT(1) - UAT(2)) / (12.0 * p->dx[a]);
#undef UAT
      xgrad += X[a] * d;
    }
    K[f] = -v * (xgrad + T[IX(p, f, i, j, k)]) / r;
  }
}

/* one-time fill of the outer ghosts of u before the first Sommerfeld step:
 * the exact solution if registered, else a copy of the nearest interior cell */
static void init_outer_ghosts(or_world *w, double t) {
  or_patch *p = &w->p[0];
  for (int sv = 0; sv < w->nsv; sv++) {
    if (!(p->sv_mask & (1u << sv))) continue;
    double *U = p->u[sv];
    for (int k = -NG; k < p->n[2] + NG; k++)
      for (int j = -NG; j < p->n[1] + NG; j++)
        for (int i = -NG; i < p->n[0] + NG; i++) {
          if (!is_outer_ghost(p, i, j, k)) continue;
          if (w->ex[sv].kind != EX_NONE) {
            double xp[3] = {xnum(p, 0, i), xnum(p, 1, j), xnum(p, 2, k)}, e[5];
            exact_patch(w, p, sv, t, xp, e);
            for (int f = 0; f < NF; f++) U[IX(p, f, i, j, k)] = e[f];
          } else {
            int cc[3] = {i, j, k};
            for (int a = 0; a < 3; a++) cc[a] = cc[a] < 0 ? 0 : (cc[a] >= p->n[a] ? p->n[a] - 1 : cc[a]);
            for (int f = 0; f < NF; f++) U[IX(p, f, i, j, k)] = U[IX(p, f, cc[0], cc[1], cc[2])];
          }
        }
  }
  w->outer_ready = 1;
}

/* ------------------------------------------------------------------------ */
/* RK4 step (Sec. 2.3)                                                       */
/* ------------------------------------------------------------------------ */
static void eval_rhs(or_world *w, int which, double t) {
  for (int pi = 0; pi < w->np; pi++) {
    or_patch *p = &w->p[pi];
    for (int sv = 0; sv < w->nsv; sv++) {
      if (!(p->sv_mask & (1u << sv))) continue;
      const double *T = bufsel(p, sv, which);
      double *K = p->k[sv];
#pragma omp parallel for schedule(dynamic)
      for (int k = 0; k < p->n[2]; k++)
        for (int j = 0; j < p->n[1]; j++)
          for (int i = 0; i < p->n[0]; i++) {
            if (!is_live(w, p, i, j, k)) continue;
            double Kc[5];
            rhs_cell(w, p, sv, T, t, i, j, k, Kc);
            for (int f = 0; f < NF; f++) K[IX(p, f, i, j, k)] = Kc[f];
          }
      if (p->is_global && w->outer_bc == 1) {
        for (int k = -NG; k < p->n[2] + NG; k++)
          for (int j = -NG; j < p->n[1] + NG; j++)
            for (int i = -NG; i < p->n[0] + NG; i++) {
              if (!is_outer_ghost(p, i, j, k)) continue;
              double Kc[5];
              radiative_rhs(w, p, sv, T, i, j, k, Kc);
              for (int f = 0; f < NF; f++) K[IX(p, f, i, j, k)] = Kc[f];
            }
      }
    }
  }
}

/* stage update on live cells:  acc = base_acc + bdt*K (bdt != 0), v = u + adt*K (adt != 0) */
static void stage_update(or_world *w, int first, double bdt, double adt, int last) {
  for (int pi = 0; pi < w->np; pi++) {
    or_patch *p = &w->p[pi];
    for (int sv = 0; sv < w->nsv; sv++) {
      if (!(p->sv_mask & (1u << sv))) continue;
      double *U = p->u[sv], *A = p->acc[sv], *V = p->v[sv], *K = p->k[sv];
#pragma omp parallel for schedule(static)
      for (int k = 0; k < p->n[2]; k++)
        for (int j = 0; j < p->n[1]; j++)
          for (int i = 0; i < p->n[0]; i++) {
            if (!is_live(w, p, i, j, k)) continue;
            for (int f = 0; f < NF; f++) {
              long long x = IX(p, f, i, j, k);
              if (last) {
                U[x] = A[x] + bdt * K[x];
              } else {
                A[x] = (first ? U[x] : A[x]) + bdt * K[x];
                V[x] = U[x] + adt * K[x];
              }
            }
          }
      if (p->is_global && w->outer_bc == 1) {
        for (int k = -NG; k < p->n[2] + NG; k++)
          for (int j = -NG; j < p->n[1] + NG; j++)
            for (int i = -NG; i < p->n[0] + NG; i++) {
              if (!is_outer_ghost(p, i, j, k)) continue;
              for (int f = 0; f < NF; f++) {
                long long x = IX(p, f, i, j, k);
                if (last) {
                  U[x] = A[x] + bdt * K[x];
                } else {
                  A[x] = (first ? U[x] : A[x]) + bdt * K[x];
                  V[x] = U[x] + adt * K[x];
                }
              }
            }
      }
    }
  }
}

static void poison_deactivated(or_world *w) {
  if (w->np == 1) return;
  or_patch *g = &w->p[0];
  for (int sv = 0; sv < w->nsv; sv++) {
    if (!(g->sv_mask & (1u << sv))) continue;
    for (int k = 0; k < g->n[2]; k++)
      for (int j = 0; j < g->n[1]; j++)
        for (int i = 0; i < g->n[0]; i++)
          if (w->flag[GIX(g, i, j, k)] == FLAG_DEACT)
            for (int f = 0; f < NF; f++) g->u[sv][IX(g, f, i, j, k)] = NAN;
  }
}

static int refresh_flags(or_world *w) {
  if (w->np == 1) { w->flags_valid = 1; return 0; }
  list_physical_ghosts(w);
  int rc = compute_flags(w, w->t, w->flag, w->cover, w->gcover);
  if (rc) return rc;
  poison_deactivated(w);
  w->flags_valid = 1;
  return 0;
}

/* cells live under the new flags that were not live during the step get
 * u_{n+1} interpolated from the covering local patch at t_{n+1}. */
static int end_of_step_flags(or_world *w) {
  if (w->np == 1) return 0;
  or_patch *g = &w->p[0];
  long long ncell = (long long)g->n[0] * g->n[1] * g->n[2];
  uint8_t *nf = (uint8_t *)malloc(ncell);
  int32_t *nc = (int32_t *)malloc(ncell * sizeof(int32_t));
  list_physical_ghosts(w);
  int32_t *ngc = (int32_t *)malloc((w->nghost > 0 ? w->nghost : 1) * sizeof(int32_t));
  int rc = compute_flags(w, w->t, nf, nc, ngc);
  if (rc) { free(nf); free(nc); free(ngc); return rc; }
  long long sk = 0, nu = 0;
  for (int sv = 0; sv < w->nsv; sv++) {
    if (!(g->sv_mask & (1u << sv))) continue;
#pragma omp parallel for schedule(dynamic) reduction(+ : sk, nu)
    for (int k = 0; k < g->n[2]; k++)
      for (int j = 0; j < g->n[1]; j++)
        for (int i = 0; i < g->n[0]; i++) {
          long long c = GIX(g, i, j, k);
          if (!(w->flag[c] != FLAG_LIVE && nf[c] == FLAG_LIVE)) continue;
          nu++;
          int d = nc[c] >= 0 ? nc[c] : w->cover[c];
          or_patch *p = &w->p[d];
          double xr[3] = {xnum(g, 0, i), xnum(g, 1, j), xnum(g, 2, k)}, X[3], xd[3], ud[5], ur[5];
          global_X(g, w->t, i, j, k, X);
          int ok = (p->sv_mask & (1u << sv)) && interp_donor(w, d, sv, p->u[sv], w->t, X, ud, xd);
          if (ok) {
            transform(p, xd, g, xr, w->t, ud, ur);
          } else {
            sk++;
            if (w->ex[sv].kind != EX_NONE) exact_patch(w, g, sv, w->t, xr, ur);
            else for (int f = 0; f < NF; f++) ur[f] = NAN;
          }
          for (int f = 0; f < NF; f++) g->u[sv][IX(g, f, i, j, k)] = ur[f];
        }
  }
  w->skip_uncover += sk;
  w->n_uncover += nu;
  memcpy(w->flag, nf, ncell);
  memcpy(w->cover, nc, ncell * sizeof(int32_t));
  memcpy(w->gcover, ngc, (w->nghost > 0 ? w->nghost : 1) * sizeof(int32_t));
  free(nf);
  free(nc);
  free(ngc);
  poison_deactivated(w);
  return 0;
}

/* ======================================================================== */
/* ctypes API                                                                */
/* ======================================================================== */
or_world *or_new(int nsv, const double *wave_speed, const int *interp_points, double ko_eps, int buffer) {
  if (nsv < 1 || nsv > MAXSV) return NULL;
  or_world *w = (or_world *)calloc(1, sizeof(or_world));
  w->nsv = nsv;
  for (int s = 0; s < nsv; s++) { w->vs[s] = wave_speed[s]; w->P[s] = interp_points[s]; }
  w->eps = ko_eps;
  w->buffer = buffer;
  return w;
}

/* form of the Pi_t equation: 0 the paper's (Eqs. eom1-eom3), 1 first-order */
int or_set_form(or_world *w, int form) {
  if (form != 0 && form != 1) return -1;
  w->form = form;
  return 0;
}

/* outer boundary of the global patch: 0 exact solution, 1 Sommerfeld (needs a
 * non-periodic global patch) */
int or_set_outer_bc(or_world *w, int bc) {
  if (bc != 0 && bc != 1) return -1;
  if (bc == 1 && w->np > 0)
    for (int a = 0; a < 3; a++)
      if (w->p[0].periodic[a]) return -1;
  w->outer_bc = bc;
  w->outer_ready = 0;
  return 0;
}

/* right-hand side at every outer ghost cell of the global patch from u
 * (Sommerfeld), into the full padded array dst (other cells untouched) */
int or_rhs_outer(or_world *w, int sv, double *dst) {
  if (w->np < 1) return -1;
  or_patch *p = &w->p[0];
  if (!p->u[sv]) return -1;
  for (int k = -NG; k < p->n[2] + NG; k++)
    for (int j = -NG; j < p->n[1] + NG; j++)
      for (int i = -NG; i < p->n[0] + NG; i++) {
        if (!is_outer_ghost(p, i, j, k)) continue;
        double Kc[5];
        radiative_rhs(w, p, sv, p->u[sv], i, j, k, Kc);
        for (int f = 0; f < NF; f++) dst[IX(p, f, i, j, k)] = Kc[f];
      }
  return 0;
}

void or_free(or_world *w) {
  if (!w) return;
  for (int pi = 0; pi < w->np; pi++)
    for (int s = 0; s < MAXSV; s++) {
      free(w->p[pi].u[s]); free(w->p[pi].acc[s]); free(w->p[pi].v[s]); free(w->p[pi].k[s]);
    }
  free(w->flag);
  free(w->cover);
  free(w->ghost_ijk);
  free(w->gcover);
  free(w);
}

/* ZYZ Euler rotation R = Rz(a) Ry(b) Rz(c) */
static void euler_zyz(const double e[3], double R[3][3]) {
  double ca = cos(e[0]), sa = sin(e[0]), cb = cos(e[1]), sb = sin(e[1]), cc = cos(e[2]), sc = sin(e[2]);
  double Z1[3][3] = {{ca, -sa, 0}, {sa, ca, 0}, {0, 0, 1}};
  double Y[3][3] = {{cb, 0, sb}, {0, 1, 0}, {-sb, 0, cb}};
  double Z2[3][3] = {{cc, -sc, 0}, {sc, cc, 0}, {0, 0, 1}};
  double T[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      T[i][j] = 0;
      for (int k = 0; k < 3; k++) T[i][j] += Y[i][k] * Z2[k][j];
    }
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      R[i][j] = 0;
      for (int k = 0; k < 3; k++) R[i][j] += Z1[i][k] * T[k][j];
    }
}

int or_add_patch(or_world *w, int coord, int is_global, const int *n, const double *lo, const double *hi,
                 const int *periodic, const double *euler, int motion, const double *c0, const double *vel,
                 double radius, double speed, double phase, unsigned sv_mask) {
  if (w->np >= MAXP) return -1;
  if ((w->np == 0) != (is_global != 0)) return -1;
  or_patch *p = &w->p[w->np];
  memset(p, 0, sizeof(*p));
  p->coord = coord;
  p->is_global = is_global;
  for (int a = 0; a < 3; a++) {
    p->n[a] = n[a];
    p->N[a] = n[a] + 2 * NG;
    p->lo[a] = lo[a];
    p->hi[a] = hi[a];
    p->dx[a] = (hi[a] - lo[a]) / n[a];
    p->periodic[a] = periodic[a];
    p->c0[a] = c0[a];
    p->vel[a] = vel[a];
  }
  euler_zyz(euler, p->R);
  p->motion = motion;
  p->radius = radius;
  p->speed = speed;
  p->phase = phase;
  p->sv_mask = sv_mask;
  long long m = pcells(p) * NF;
  for (int s = 0; s < w->nsv; s++) {
    if (!(sv_mask & (1u << s))) continue;
    p->u[s] = (double *)malloc(m * sizeof(double));
    p->acc[s] = (double *)malloc(m * sizeof(double));
    p->v[s] = (double *)malloc(m * sizeof(double));
    p->k[s] = (double *)malloc(m * sizeof(double));
    for (long long x = 0; x < m; x++) p->u[s][x] = p->acc[s][x] = p->v[s][x] = p->k[s][x] = NAN;
  }
  if (is_global) {
    long long nc = (long long)n[0] * n[1] * n[2];
    w->flag = (uint8_t *)malloc(nc);
    w->cover = (int32_t *)malloc(nc * sizeof(int32_t));
    memset(w->flag, FLAG_LIVE, nc);
    for (long long c = 0; c < nc; c++) w->cover[c] = -1;
  }
  w->flags_valid = 0;
  return w->np++;
}

int or_set_exact_plane(or_world *w, int sv, double A, double B, const double *kap, double psi) {
  or_exact *e = &w->ex[sv];
  memset(e, 0, sizeof(*e));
  e->kind = EX_PLANE;
  e->A = A; e->B = B; e->psi = psi;
  for (int a = 0; a < 3; a++) e->kap[a] = kap[a];
  return 0;
}

int or_set_exact_gauss(or_world *w, int sv, int ng, const double *amp, const double *xc, const double *wd) {
  if (ng > MAXG) return -1;
  or_exact *e = &w->ex[sv];
  memset(e, 0, sizeof(*e));
  e->kind = EX_GAUSS;
  e->ng = ng;
  for (int g = 0; g < ng; g++) {
    e->amp[g] = amp[g];
    e->w[g] = wd[g];
    for (int a = 0; a < 3; a++) e->xc[g][a] = xc[3 * g + a];
  }
  return 0;
}

/* interior arrays are [5][n2][n1][n0], n0 fastest */
int or_set_state(or_world *w, int pi, int sv, const double *src, double t0) {
  or_patch *p = &w->p[pi];
  if (!p->u[sv]) return -1;
  long long x = 0;
  for (int f = 0; f < NF; f++)
    for (int k = 0; k < p->n[2]; k++)
      for (int j = 0; j < p->n[1]; j++)
        for (int i = 0; i < p->n[0]; i++) p->u[sv][IX(p, f, i, j, k)] = src[x++];
  w->t = t0;
  w->flags_valid = 0;
  w->outer_ready = 0;
  return 0;
}

int or_get_state(or_world *w, int pi, int sv, double *dst) {
  or_patch *p = &w->p[pi];
  if (!p->u[sv]) return -1;
  long long x = 0;
  for (int f = 0; f < NF; f++)
    for (int k = 0; k < p->n[2]; k++)
      for (int j = 0; j < p->n[1]; j++)
        for (int i = 0; i < p->n[0]; i++) dst[x++] = p->u[sv][IX(p, f, i, j, k)];
  return 0;
}

/* whole array including ghost cells, [5][N2][N1][N0] */
int or_get_full(or_world *w, int pi, int sv, double *dst) {
  or_patch *p = &w->p[pi];
  if (!p->u[sv]) return -1;
  memcpy(dst, p->u[sv], pcells(p) * NF * sizeof(double));
  return 0;
}

int or_init_exact(or_world *w, double t0) {
  for (int pi = 0; pi < w->np; pi++) {
    or_patch *p = &w->p[pi];
    for (int sv = 0; sv < w->nsv; sv++) {
      if (!p->u[sv] || w->ex[sv].kind == EX_NONE) continue;
#pragma omp parallel for schedule(static)
      for (int k = 0; k < p->n[2]; k++)
        for (int j = 0; j < p->n[1]; j++)
          for (int i = 0; i < p->n[0]; i++) {
            double xp[3] = {xnum(p, 0, i), xnum(p, 1, j), xnum(p, 2, k)}, e[5];
            exact_patch(w, p, sv, t0, xp, e);
            for (int f = 0; f < NF; f++) p->u[sv][IX(p, f, i, j, k)] = e[f];
          }
    }
  }
  w->t = t0;
  w->flags_valid = 0;
  w->outer_ready = 0;
  return 0;
}

int or_prepare(or_world *w) { return refresh_flags(w); }

int or_get_flags(or_world *w, uint8_t *flag, int32_t *cover) {
  if (w->np < 1) return -1;
  const or_patch *g = &w->p[0];
  long long nc = (long long)g->n[0] * g->n[1] * g->n[2];
  if (!w->flags_valid) { int rc = refresh_flags(w); if (rc) return rc; }
  memcpy(flag, w->flag, nc);
  if (cover) memcpy(cover, w->cover, nc * sizeof(int32_t));
  return 0;
}

int or_exchange_ghosts(or_world *w, double t) {
  if (!w->flags_valid) { int rc = refresh_flags(w); if (rc) return rc; }
  fill_ghosts(w, 0, t);
  return 0;
}

int or_step(or_world *w, double dt, int nsteps) {
  for (int n = 0; n < nsteps; n++) {
    if (!w->flags_valid) { int rc = refresh_flags(w); if (rc) return rc; }
    double tn = w->t;
    if (w->outer_bc == 1 && !w->outer_ready) init_outer_ghosts(w, tn);
    /* K1 = f(t_n, u_n); u_{n+1/2} accumulates b1 K1 + b2 K2 + b3 K3 (Table rk4) */
    fill_ghosts(w, 0, tn);
    eval_rhs(w, 0, tn);
    stage_update(w, 1, dt / 6.0, dt / 2.0, 0);
    fill_ghosts(w, 1, tn + 0.5 * dt);
    eval_rhs(w, 1, tn + 0.5 * dt);
    stage_update(w, 0, dt / 3.0, dt / 2.0, 0);
    fill_ghosts(w, 1, tn + 0.5 * dt);
    eval_rhs(w, 1, tn + 0.5 * dt);
    stage_update(w, 0, dt / 3.0, dt, 0);
    /* K4 = f(t_n + dt, u_n + a43 dt K3); u_{n+1} = u_{n+1/2} + b4 dt K4 */
    fill_ghosts(w, 1, tn + dt);
    eval_rhs(w, 1, tn + dt);
    stage_update(w, 0, dt / 6.0, 0.0, 1);
    w->t = tn + dt;
    int rc = end_of_step_flags(w);
    if (rc) return rc;
  }
  return 0;
}

double or_time(const or_world *w) { return w->t; }

/* number of OpenMP threads of the oracle's loops (timing runs only) */
void or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int or_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* counters: skip_local, skip_eff, skip_uncover, n_uncover, skip_outer, n_outer */
void or_counters(const or_world *w, long long *out) {
  out[0] = w->skip_local; out[1] = w->skip_eff; out[2] = w->skip_uncover; out[3] = w->n_uncover;
  out[4] = w->skip_outer; out[5] = w->n_outer;
}

/* covering local patch (or -1) of every cell of the global patch's padded
 * array, [N2][N1][N0]: interior cells from the cover flags, physical ghost
 * cells from the covered-ghost list, periodic ghost copies -1 */
int or_cover_full(or_world *w, int32_t *dst) {
  if (w->np < 1) return -1;
  if (!w->flags_valid) { int rc = refresh_flags(w); if (rc) return rc; }
  const or_patch *g = &w->p[0];
  for (long long x = 0; x < pcells(g); x++) dst[x] = -1;
  for (int k = 0; k < g->n[2]; k++)
    for (int j = 0; j < g->n[1]; j++)
      for (int i = 0; i < g->n[0]; i++) dst[IX(g, 0, i, j, k)] = w->cover[GIX(g, i, j, k)];
  for (int q = 0; q < w->nghost; q++)
    dst[IX(g, 0, w->ghost_ijk[3 * q], w->ghost_ijk[3 * q + 1], w->ghost_ijk[3 * q + 2])] = w->gcover[q];
  return 0;
}

/*
 * Diagnostics over the live interior cells of patch pi, state vector sv.
 * out[0..4]   max |u_f|
 * out[5..9]   sum u_f^2
 * out[10..14] max |u_f - exact_f|       (0 when no exact solution)
 * out[15..19] sum (u_f - exact_f)^2
 * out[20]     integrated relative error of phi, sum |phi-phi_e|/|phi_e| sqrt(gamma) d^3x' (Sec. 3.2)
 * out[21]     number of live cells
 * out[22]     sum sqrt(gamma) d^3x' over live cells (covered volume)
 * out[23]     discrete energy 1/2 sum (Pi_t^2 - v^2 phi L phi) dx dy dz, L the sum of the
 *             4th-order second differences along the numerical axes
 * out[24..26] max |Pi_a - D_a phi|, a = 1..3 (the constraint Psi_a = d_a phi)
 *             out[23..26] over the live cells whose +-2 axis stencils reach live
 *             interior cells only (periodic axes wrap)
 */
/* live interior cell (i,j,k) + o e_a with a periodic axis wrapped; 0 if none */
static int star_cell(const or_world *w, const or_patch *p, int i, int j, int k, int a, int o, int c[3]) {
  c[0] = i; c[1] = j; c[2] = k;
  c[a] += o;
  if (p->periodic[a]) c[a] = wrapi(c[a], p->n[a]);
  if (c[a] < 0 || c[a] >= p->n[a]) return 0;
  return is_live(w, p, c[0], c[1], c[2]);
}

int or_diag(or_world *w, int pi, int sv, double *out) {
  or_patch *p = &w->p[pi];
  if (!p->u[sv]) return -1;
  if (!w->flags_valid) { int rc = refresh_flags(w); if (rc) return rc; }
  for (int x = 0; x < 27; x++) out[x] = 0;
  double cellvol = p->dx[0] * p->dx[1] * p->dx[2];
  for (int k = 0; k < p->n[2]; k++)
    for (int j = 0; j < p->n[1]; j++)
      for (int i = 0; i < p->n[0]; i++) {
        if (!is_live(w, p, i, j, k)) continue;
        double xp[3] = {xnum(p, 0, i), xnum(p, 1, j), xnum(p, 2, k)}, e[5] = {0, 0, 0, 0, 0};
        int has = w->ex[sv].kind != EX_NONE;
        if (has) exact_patch(w, p, sv, w->t, xp, e);
        for (int f = 0; f < NF; f++) {
          double val = p->u[sv][IX(p, f, i, j, k)];
          if (fabs(val) > out[f]) out[f] = fabs(val);
          out[5 + f] += val * val;
          if (has) {
            double d = val - e[f];
            if (fabs(d) > out[10 + f]) out[10 + f] = fabs(d);
            out[15 + f] += d * d;
          }
        }
        double gi[4][4], C[4], sg;
        metric(p, w->vs[sv], w->t, xp, gi, C, &sg);
        if (has) out[20] += fabs(p->u[sv][IX(p, 0, i, j, k)] - e[0]) / fabs(e[0]) * sg * cellvol;
        out[21] += 1;
        out[22] += sg * cellvol;
        /* energy density and constraint where the axis stencils stay on live cells */
        double ph[3][5];
        int ok = 1;
        for (int a = 0; a < 3 && ok; a++)
          for (int o = -2; o <= 2 && ok; o++) {
            int c[3];
            if (!star_cell(w, p, i, j, k, a, o, c)) ok = 0;
            else ph[a][o + 2] = p->u[sv][IX(p, 0, c[0], c[1], c[2])];
          }
        if (!ok) continue;
        double lap = 0;
        for (int a = 0; a < 3; a++) {
          lap += (-ph[a][0] + 16 * ph[a][1] - 30 * ph[a][2] + 16 * ph[a][3] - ph[a][4]) / (12 * p->dx[a] * p->dx[a]);
          double d1 = (ph[a][0] - 8 * ph[a][1] + 8 * ph[a][3] - ph[a][4]) / (12 * p->dx[a]);
          double c = fabs(p->u[sv][IX(p, 2 + a, i, j, k)] - d1);
          if (c > out[24 + a]) out[24 + a] = c;
        }
        double pit = p->u[sv][IX(p, 1, i, j, k)], phi = ph[0][2];
        out[23] += 0.5 * cellvol * (pit * pit - w->vs[sv] * w->vs[sv] * phi * lap);
      }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Unit entry points used by the pin tests                                  */
/* ------------------------------------------------------------------------ */
void or_metric_at(const or_world *w, int pi, int sv, double t, const double *xp, double *ginv16, double *C4,
                  double *sqrt_gamma) {
  double gi[4][4];
  metric(&w->p[pi], w->vs[sv], t, xp, gi, C4, sqrt_gamma);
  for (int a = 0; a < 4; a++)
    for (int b = 0; b < 4; b++) ginv16[4 * a + b] = gi[a][b];
}

void or_jac_at(const or_world *w, int pi, double t, const double *xp, double *E16) {
  double E[4][4];
  jac4(&w->p[pi], t, xp, E);
  for (int a = 0; a < 4; a++)
    for (int b = 0; b < 4; b++) E16[4 * a + b] = E[a][b];
}

void or_map_fwd(const or_world *w, int pi, double t, const double *xp, double *X) { map_fwd(&w->p[pi], t, xp, X); }
void or_map_inv(const or_world *w, int pi, double t, const double *X, double *xp) { map_inv(&w->p[pi], t, X, xp); }

/* Angular velocity (background frame) of a rotation of patch pi about its centre. */
int or_set_spin(or_world *w, int pi, const double *spin) {
  if (pi < 1 || pi >= w->np) return -1;
  for (int a = 0; a < 3; a++) w->p[pi].spin[a] = spin[a];
  w->flags_valid = 0;
  return 0;
}

void or_rotation(const or_world *w, int pi, double *R9) {
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) R9[3 * a + b] = w->p[pi].R[a][b];
}

void or_lagrange(int P, double q, int *s, double *wts) { lagrange(P, q, s, wts); }

/* transform a 5-state from donor frame (patch d at x'_d) to receiver frame (patch r at x'_r) */
void or_transform(const or_world *w, int d, const double *xd, int r, const double *xr, double t,
                  const double *in, double *out) {
  transform(&w->p[d], xd, &w->p[r], xr, t, in, out);
}

/* interpolate buffer u of donor d at background point X; returns validity */
int or_interp(or_world *w, int d, int sv, double t, const double *X, double *out, double *xd) {
  if (!w->flags_valid) { int rc = refresh_flags(w); if (rc) return rc; }
  return interp_donor(w, d, sv, w->p[d].u[sv], t, X, out, xd);
}

void or_exact_bg(const or_world *w, int sv, double t, const double *X, double *out) {
  exact_bg(&w->ex[sv], w->vs[sv], t, X, out);
}

void or_exact_patch(const or_world *w, int pi, int sv, double t, const double *xp, double *out) {
  exact_patch(w, &w->p[pi], sv, t, xp, out);
}

/* RHS at every live interior cell of patch pi from buffer u (ghosts as they are) at time t */
int or_rhs(or_world *w, int pi, int sv, double t, double *dst) {
  or_patch *p = &w->p[pi];
  if (!p->u[sv]) return -1;
  long long x = 0, per = (long long)p->n[0] * p->n[1] * p->n[2];
  for (int k = 0; k < p->n[2]; k++)
    for (int j = 0; j < p->n[1]; j++)
      for (int i = 0; i < p->n[0]; i++, x++) {
        double K[5];
        if (!is_live(w, p, i, j, k)) { for (int f = 0; f < NF; f++) dst[f * per + x] = NAN; continue; }
        rhs_cell(w, p, sv, p->u[sv], t, i, j, k, K);
        for (int f = 0; f < NF; f++) dst[f * per + x] = K[f];
      }
  return 0;
}

/* apply one stencil to field 0 of buffer u at interior cell (i,j,k):
 * op 0: D1 along d, 1: D2 along d, 2: D11 along (d,e), 3: Delta^6 along d (undivided) */
double or_stencil(or_world *w, int pi, int sv, int op, int d, int e, int i, int j, int k) {
  or_patch *p = &w->p[pi];
  const double *T = p->u[sv];
  if (op == 0) return D1(p, T, 0, i, j, k, d);
  if (op == 1) return D2(p, T, 0, i, j, k, d);
  if (op == 2) return D11(p, T, 0, i, j, k, d, e);
  double q = 0;
  for (int o = -3; o <= 3; o++) q += W6[o + 3] * at(p, T, 0, i, j, k, d, o);
  return q;
}

/* write the whole array including ghosts, [5][N2][N1][N0] */
int or_set_full(or_world *w, int pi, int sv, const double *src) {
  or_patch *p = &w->p[pi];
  if (!p->u[sv]) return -1;
  memcpy(p->u[sv], src, pcells(p) * NF * sizeof(double));
  return 0;
}
