// Internal device-side data structures and math of libpw (gfx950).
//
// Patch arrays are padded by NG = 3 ghost cells per side; each x-row is laid out
// [29 alignment pad][3 ghosts][n0 interior][3 ghosts][pad to a multiple of 32],
// so the first interior element of every row starts 128-byte aligned in FP32
// (256 in FP64): a tile row of 32 or 128 cells then writes whole cache lines.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define PW_NG 3
#define PW_OX 32         // row offset of interior cell i = 0
#define PW_MAXSV 4
#define PW_MAXPULSE 32
#define PW_NPTS 5    // interpolation widths P = 2 .. 6

namespace pw {

enum { CART = 0, SPH = 1, CYL = 2 };
enum { STATIC = 0, LINEAR = 1, CIRCLE = 2 };
enum { LIVE = 0, EFFGHOST = 1, DEACT = 2 };
enum { EX_NONE = 0, EX_PLANE = 1, EX_GAUSS = 2 };

struct PatchDev {
  int coord, is_global, motion;
  int n[3];
  int periodic[3];
  int pitch;            // elements per padded x-row
  int rows;             // n1 + 6
  int slabs;            // n2 + 6
  long long slab;       // pitch * rows
  long long fstride;    // elements per field (slab * slabs)
  double lo[3], hi[3], dx[3], idx[3];
  double R[9];          // row-major rotation, X = c + R y
  double c0[3], vel[3], radius, omega, phase;
  unsigned sv_mask;
  int bkt_base, bkt_n[3];  // donor buckets of 8 x 8 x 4 cells (local patches): first id, counts per axis
  double *u[PW_MAXSV];
  double *acc[PW_MAXSV];
  void *va[PW_MAXSV];
  void *vb[PW_MAXSV];
  float *us[PW_MAXSV];  // mixed precision: FP32 copy of u (stage-1 stencil input), else null
  // spherical patches: sin, cos of theta_j (j = -3 .. n1+2) and of phi_k
  // (k = -3 .. n2+2), laid out [sin th][cos th][sin ph][cos ph]; cylindrical
  // patches: sin, cos of phi_j (j = -3 .. n1+2), [sin ph][cos ph]; null otherwise
  const double *trig;
  double spin[3];  // angular velocity of a rotation about the centre (background frame)
};

// Pose of a patch at one stage time: centre, its first and second time
// derivatives, orientation R(t), the angular velocity w, and the components of
// c', c'' and w along the patch axes (b = R^T c', a = R^T c'', wp = R^T w).
struct PoseDev {
  double c[3], cd[3], cdd[3], b[3], a[3];
  double R[9], w[3], wp[3];
};

struct ExactDev {
  int kind;
  double amp, offset, kappa[3], phase, knorm;
  int n;
  double pa[PW_MAXPULSE], px[PW_MAXPULSE][3], pw[PW_MAXPULSE];
};

// Loads and stores through the global address space (the pointers held in the
// patch table are generic; these casts let the compiler emit global_load/store
// with a scalar base and a 32-bit offset instead of flat instructions).
template <typename T>
__device__ __forceinline__ T gld(const T *base, uint32_t off) {
  return ((const __attribute__((address_space(1))) T *)base)[off];
}
template <typename T>
__device__ __forceinline__ void gst(T *base, uint32_t off, T v) {
  ((__attribute__((address_space(1))) T *)base)[off] = v;
}

__host__ __device__ inline long long cell_index(const PatchDev &p, int i, int j, int k) {
  return (long long)(k + PW_NG) * p.slab + (long long)(j + PW_NG) * p.pitch + (i + PW_OX);
}

// ---------------------------------------------------------------------------
// Pose c(t) for the three motions (a patch map is X = c(t) + R M(x')).
// ---------------------------------------------------------------------------
__host__ __device__ inline void pose_at(const PatchDev &p, double t, PoseDev &o) {
  for (int a = 0; a < 3; a++) { o.c[a] = p.c0[a]; o.cd[a] = 0.0; o.cdd[a] = 0.0; }
  if (p.motion == LINEAR) {
    for (int a = 0; a < 3; a++) { o.c[a] = p.c0[a] + p.vel[a] * t; o.cd[a] = p.vel[a]; }
  } else if (p.motion == CIRCLE) {
    double arg = p.omega * t + p.phase;
    double s = sin(arg), c = cos(arg);
    o.c[0] += p.radius * c;
    o.c[1] += p.radius * s;
    o.cd[0] = -p.radius * p.omega * s;
    o.cd[1] = p.radius * p.omega * c;
    o.cdd[0] = -p.radius * p.omega * p.omega * c;
    o.cdd[1] = -p.radius * p.omega * p.omega * s;
  }
  // orientation: R(t) = Q R(0), Q the rotation by |w| t about w / |w|
  // (Rodrigues: Q = I + sin(th) K + (1 - cos(th)) K^2, K the cross-product matrix of the axis)
  const double wn = sqrt(p.spin[0] * p.spin[0] + p.spin[1] * p.spin[1] + p.spin[2] * p.spin[2]);
  for (int a = 0; a < 3; a++) o.w[a] = p.spin[a];
  if (wn == 0.0) {
    for (int m = 0; m < 9; m++) o.R[m] = p.R[m];
  } else {
    const double k[3] = {p.spin[0] / wn, p.spin[1] / wn, p.spin[2] / wn};
    const double K[9] = {0, -k[2], k[1], k[2], 0, -k[0], -k[1], k[0], 0};
    const double sn = sin(wn * t), omc = 1.0 - cos(wn * t);
    double Q[9];
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) {
        double k2 = 0.0;
        for (int m = 0; m < 3; m++) k2 += K[3 * a + m] * K[3 * m + b];
        Q[3 * a + b] = (a == b ? 1.0 : 0.0) + sn * K[3 * a + b] + omc * k2;
      }
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) {
        double s = 0.0;
        for (int m = 0; m < 3; m++) s += Q[3 * a + m] * p.R[3 * m + b];
        o.R[3 * a + b] = s;
      }
  }
  for (int i = 0; i < 3; i++) {
    o.b[i] = o.R[0 + i] * o.cd[0] + o.R[3 + i] * o.cd[1] + o.R[6 + i] * o.cd[2];
    o.a[i] = o.R[0 + i] * o.cdd[0] + o.R[3 + i] * o.cdd[1] + o.R[6 + i] * o.cdd[2];
    o.wp[i] = o.R[0 + i] * o.w[0] + o.R[3 + i] * o.w[1] + o.R[6 + i] * o.w[2];
  }
}

// Frame terms at the patch-frame point y (Eqs. eom1-eom3 in the moving frame):
// the shift beta = b + wp x y (minus the time derivative of y at fixed X) and
// acc = a - 2 wp x b - wp x (wp x y) (minus the second time derivative of y at
// fixed X).  Without spin these are b and a exactly.
__host__ __device__ inline void frame_terms(const PoseDev &ps, const double y[3], double beta[3], double acc[3]) {
  const double *w = ps.wp;
  const double wy[3] = {w[1] * y[2] - w[2] * y[1], w[2] * y[0] - w[0] * y[2], w[0] * y[1] - w[1] * y[0]};
  const double wb[3] = {w[1] * ps.b[2] - w[2] * ps.b[1], w[2] * ps.b[0] - w[0] * ps.b[2], w[0] * ps.b[1] - w[1] * ps.b[0]};
  const double wwy[3] = {w[1] * wy[2] - w[2] * wy[1], w[2] * wy[0] - w[0] * wy[2], w[0] * wy[1] - w[1] * wy[0]};
  for (int i = 0; i < 3; i++) {
    beta[i] = ps.b[i] + wy[i];
    acc[i] = ps.a[i] - 2.0 * wb[i] - wwy[i];
  }
}

// Velocity of the patch frame at patch-frame point y, in the background frame:
// V = c' + w x (R y).
__device__ inline void frame_velocity(const PoseDev &ps, const double y[3], double V[3]) {
  double Ry[3];
  for (int a = 0; a < 3; a++) Ry[a] = ps.R[3 * a] * y[0] + ps.R[3 * a + 1] * y[1] + ps.R[3 * a + 2] * y[2];
  V[0] = ps.cd[0] + (ps.w[1] * Ry[2] - ps.w[2] * Ry[1]);
  V[1] = ps.cd[1] + (ps.w[2] * Ry[0] - ps.w[0] * Ry[2]);
  V[2] = ps.cd[2] + (ps.w[0] * Ry[1] - ps.w[1] * Ry[0]);
}

// Cell centre along axis a, rounded as written (product, then sum; no fused
// multiply-add), so that decisions taken on it (the closed-box cover test, a
// centre exactly on a patch face) match a plain evaluation of the same formula.
__device__ inline double xnum(const PatchDev &p, int a, int i) {
#pragma clang fp contract(off)
  return p.lo[a] + (i + 0.5) * p.dx[a];
}

// Orthonormal frame of the numerical axes of a curvilinear patch at one point:
// e[a] = (dy/dx'^a) / h[a], h the scale factors, y the patch-frame Cartesian
// point.  Spherical x' = (r, theta, phi): e = (e_r, e_theta, e_phi),
// h = (1, r, r sin theta).  Cylindrical x' = (r, phi, z): e = (e_r, e_phi, e_z),
// h = (1, r, 1).
struct Basis {
  double e[3][3];
  double h[3];
};
__device__ inline void sph_frame(double r, double st, double ct, double sp, double cp, Basis &B) {
  B.e[0][0] = st * cp; B.e[0][1] = st * sp; B.e[0][2] = ct;
  B.e[1][0] = ct * cp; B.e[1][1] = ct * sp; B.e[1][2] = -st;
  B.e[2][0] = -sp;     B.e[2][1] = cp;      B.e[2][2] = 0.0;
  B.h[0] = 1.0; B.h[1] = r; B.h[2] = r * st;
}
__device__ inline void cyl_frame(double r, double sp, double cp, Basis &B) {
  B.e[0][0] = cp;  B.e[0][1] = sp; B.e[0][2] = 0.0;
  B.e[1][0] = -sp; B.e[1][1] = cp; B.e[1][2] = 0.0;
  B.e[2][0] = 0.0; B.e[2][1] = 0.0; B.e[2][2] = 1.0;
  B.h[0] = 1.0; B.h[1] = r; B.h[2] = 1.0;
}

// Angle tables of a curvilinear patch (filled with sincos of the grid angles,
// ghosts included).  Spherical: [sin th_j][cos th_j][sin ph_k][cos ph_k];
// cylindrical: [sin ph_j][cos ph_j].
__device__ inline void trig_axis(const PatchDev &p, int base, int len, int i, double &s, double &c) {
  s = p.trig[base + i + PW_NG];
  c = p.trig[base + len + i + PW_NG];
}

// Patch-frame point y and frame B at numerical x' (curvilinear patches).
__device__ inline void curv_point(const PatchDev &p, const double xp[3], Basis &B, double y[3]) {
  if (p.coord == SPH) {
    double st, ct, sp, cp;
    sincos(xp[1], &st, &ct);
    sincos(xp[2], &sp, &cp);
    sph_frame(xp[0], st, ct, sp, cp, B);
    for (int a = 0; a < 3; a++) y[a] = xp[0] * B.e[0][a];
  } else {
    double sp, cp;
    sincos(xp[1], &sp, &cp);
    cyl_frame(xp[0], sp, cp, B);
    y[0] = xp[0] * cp; y[1] = xp[0] * sp; y[2] = xp[2];
  }
}

// Forward map: numerical x' of patch p -> background X at pose ps.
__device__ inline void fwd_map(const PatchDev &p, const PoseDev &ps, const double xp[3], double X[3]) {
  double y[3];
  if (p.coord == CART) {
    y[0] = xp[0]; y[1] = xp[1]; y[2] = xp[2];
  } else {
    Basis B;
    curv_point(p, xp, B, y);
  }
  for (int a = 0; a < 3; a++) X[a] = ps.c[a] + ps.R[3 * a] * y[0] + ps.R[3 * a + 1] * y[1] + ps.R[3 * a + 2] * y[2];
}

// Inverse map: background X -> numerical x' of patch p at pose ps.
// Numerical coordinates of a curvilinear patch at patch-frame point y: (r,
// theta, phi) or (r, phi, z).  Not inlined: the inverse trigonometric
// functions stay out of the (register-bound) interpolation kernels that call
// it for a few of their points.
__device__ __noinline__ double3 curv_coords(int coord, double y0, double y1, double y2) {
  if (coord == SPH) {
    const double r = sqrt(y0 * y0 + y1 * y1 + y2 * y2);
    return make_double3(r, acos(y2 / r), atan2(y1, y0));
  }
  return make_double3(sqrt(y0 * y0 + y1 * y1), atan2(y1, y0), y2);
}

__device__ inline void inv_map(const PatchDev &p, const PoseDev &ps, const double X[3], double xp[3]) {
  double d[3] = {X[0] - ps.c[0], X[1] - ps.c[1], X[2] - ps.c[2]};
  double y[3];
  for (int b = 0; b < 3; b++) y[b] = ps.R[b] * d[0] + ps.R[3 + b] * d[1] + ps.R[6 + b] * d[2];
  if (p.coord == CART) {
    xp[0] = y[0]; xp[1] = y[1]; xp[2] = y[2];
  } else {
    const double3 v = curv_coords(p.coord, y[0], y[1], y[2]);
    xp[0] = v.x; xp[1] = v.y; xp[2] = v.z;
  }
}

// One-form from patch frame to background: given (Pi_t, Pi_i) in the numerical
// frame of p at patch-frame point y (frame B for curvilinear patches), return
// Pi_t^B and the background gradient G = d phi/dX: G = R gy with gy the
// gradient along the patch axes (sum_a Pi_a / h_a e_a on a curvilinear patch),
// and Pi_t^B = Pi_t - V.G with V the frame velocity at y.
__device__ inline void patch_to_bg_b(const PatchDev &p, const PoseDev &ps, const Basis &B, const double y[3],
                                     const double in[4], double &pit, double G[3]) {
  double gy[3];
  if (p.coord == CART) {
    gy[0] = in[1]; gy[1] = in[2]; gy[2] = in[3];
  } else {
    const double f0 = in[1] / B.h[0], f1 = in[2] / B.h[1], f2 = in[3] / B.h[2];
    for (int a = 0; a < 3; a++) gy[a] = f0 * B.e[0][a] + f1 * B.e[1][a] + f2 * B.e[2][a];
  }
  for (int a = 0; a < 3; a++) G[a] = ps.R[3 * a] * gy[0] + ps.R[3 * a + 1] * gy[1] + ps.R[3 * a + 2] * gy[2];
  double V[3];
  frame_velocity(ps, y, V);
  pit = in[0] - (V[0] * G[0] + V[1] * G[1] + V[2] * G[2]);
}
__device__ inline void patch_to_bg(const PatchDev &p, const PoseDev &ps, const double xp[3], const double in[4],
                                   double &pit, double G[3]) {
  Basis B;
  double y[3];
  if (p.coord == CART) {
    y[0] = xp[0]; y[1] = xp[1]; y[2] = xp[2];
  } else {
    curv_point(p, xp, B, y);
  }
  patch_to_bg_b(p, ps, B, y, in, pit, G);
}
// The same at the point of p that maps to background X (x' = its inverse map):
// the point y comes from the patch-frame Cartesian offset, and the angles'
// sines and cosines are ratios of y (no trigonometry).
__device__ inline void patch_to_bg_at(const PatchDev &p, const PoseDev &ps, const double X[3], const double xp[3],
                                      const double in[4], double &pit, double G[3]) {
  const double d[3] = {X[0] - ps.c[0], X[1] - ps.c[1], X[2] - ps.c[2]};
  double y[3];
  for (int b = 0; b < 3; b++) y[b] = ps.R[b] * d[0] + ps.R[3 + b] * d[1] + ps.R[6 + b] * d[2];
  double gy[3];
  if (p.coord == CART) {
    gy[0] = in[1]; gy[1] = in[2]; gy[2] = in[3];
  } else {
    const double rho = sqrt(y[0] * y[0] + y[1] * y[1]);
    double cp = 1.0, sp = 0.0;
    if (rho > 0.0) {
      cp = y[0] / rho;
      sp = y[1] / rho;
    }
    if (p.coord == SPH) {
      // gradient r-part + theta-part in the (rho, z) plane, phi-part along e_phi
      const double ir = 1.0 / xp[0], st = rho * ir, ct = y[2] * ir;
      const double ft = in[2] * ir, fp = rho > 0.0 ? in[3] / rho : 0.0;
      const double fh = in[1] * st + ft * ct;  // horizontal (e_rho) component
      gy[0] = fh * cp - fp * sp;
      gy[1] = fh * sp + fp * cp;
      gy[2] = in[1] * ct - ft * st;
    } else {
      const double fp = in[2] / xp[0];
      gy[0] = in[1] * cp - fp * sp;
      gy[1] = in[1] * sp + fp * cp;
      gy[2] = in[3];
    }
  }
  for (int a = 0; a < 3; a++) G[a] = ps.R[3 * a] * gy[0] + ps.R[3 * a + 1] * gy[1] + ps.R[3 * a + 2] * gy[2];
  double V[3];
  frame_velocity(ps, y, V);
  pit = in[0] - (V[0] * G[0] + V[1] * G[1] + V[2] * G[2]);
}

// Background one-form (Pi_t^B, G) -> numerical frame of p at point y:
// Pi_a = h_a e_a . gy on a curvilinear patch.
__device__ inline void bg_to_patch_b(const PatchDev &p, const PoseDev &ps, const Basis &B, const double y[3],
                                     double pit, const double G[3], double out[4]) {
  double gy[3];
  for (int b = 0; b < 3; b++) gy[b] = ps.R[b] * G[0] + ps.R[3 + b] * G[1] + ps.R[6 + b] * G[2];
  double V[3];
  frame_velocity(ps, y, V);
  out[0] = pit + V[0] * G[0] + V[1] * G[1] + V[2] * G[2];
  if (p.coord == CART) {
    out[1] = gy[0]; out[2] = gy[1]; out[3] = gy[2];
  } else {
    for (int a = 0; a < 3; a++) out[1 + a] = B.h[a] * (B.e[a][0] * gy[0] + B.e[a][1] * gy[1] + B.e[a][2] * gy[2]);
  }
}
__device__ inline void bg_to_patch(const PatchDev &p, const PoseDev &ps, const double xp[3], double pit,
                                   const double G[3], double out[4]) {
  Basis B;
  double y[3];
  if (p.coord == CART) {
    y[0] = xp[0]; y[1] = xp[1]; y[2] = xp[2];
  } else {
    curv_point(p, xp, B, y);
  }
  bg_to_patch_b(p, ps, B, y, pit, G, out);
}

// Grid point c (numerical indices, ghosts included) of p: its patch-frame
// point and frame (angle tables), its background position, and a background
// one-form carried to p there.
__device__ inline void grid_point(const PatchDev &p, const int c[3], Basis &B, double y[3]) {
  if (p.coord == CART) {
    for (int a = 0; a < 3; a++) y[a] = xnum(p, a, c[a]);
  } else if (p.coord == SPH) {
    const int t1 = p.n[1] + 2 * PW_NG, t2 = p.n[2] + 2 * PW_NG;
    double st, ct, sp, cp;
    trig_axis(p, 0, t1, c[1], st, ct);
    trig_axis(p, 2 * t1, t2, c[2], sp, cp);
    const double r = xnum(p, 0, c[0]);
    sph_frame(r, st, ct, sp, cp, B);
    for (int a = 0; a < 3; a++) y[a] = r * B.e[0][a];
  } else {
    const int t1 = p.n[1] + 2 * PW_NG;
    double sp, cp;
    trig_axis(p, 0, t1, c[1], sp, cp);
    const double r = xnum(p, 0, c[0]);
    cyl_frame(r, sp, cp, B);
    y[0] = r * cp; y[1] = r * sp; y[2] = xnum(p, 2, c[2]);
  }
}
__device__ inline void fwd_map_grid(const PatchDev &p, const PoseDev &ps, const int c[3], double X[3]) {
  double y[3];
  Basis B;
  grid_point(p, c, B, y);
  for (int a = 0; a < 3; a++) X[a] = ps.c[a] + ps.R[3 * a] * y[0] + ps.R[3 * a + 1] * y[1] + ps.R[3 * a + 2] * y[2];
}
__device__ inline void bg_to_patch_grid(const PatchDev &p, const PoseDev &ps, const int c[3], double pit,
                                        const double G[3], double out[4]) {
  Basis B;
  double y[3];
  grid_point(p, c, B, y);
  bg_to_patch_b(p, ps, B, y, pit, G, out);
}

// Background position of cell (i,j,k) of the global patch, which is static and
// unrotated at the origin: a Cartesian global's numerical coordinates are X,
// a spherical global maps through its angle tables.
__device__ inline void global_X(const PatchDev &g, const PoseDev &ps0, int i, int j, int k, double X[3]) {
  if (g.coord == CART) {
    X[0] = xnum(g, 0, i); X[1] = xnum(g, 1, j); X[2] = xnum(g, 2, k);
  } else {
    const int c[3] = {i, j, k};
    fwd_map_grid(g, ps0, c, X);
  }
}

// ---------------------------------------------------------------------------
// Exact solutions in the background frame: phi, d_t phi, grad phi.
// ---------------------------------------------------------------------------
// n-th derivative of g(s) = s exp(-s^2/w^2), via Hermite polynomials H_{n+1}:
// g^(n)(s) = (-1)^n / 2 * w^(1-n) * H_{n+1}(s/w) * exp(-(s/w)^2).
__device__ inline double gpulse_der(int n, double s, double w) {
  double u = s / w, hm = 1.0, h = 2.0 * u;
  for (int k = 1; k <= n; k++) {
    double hn = 2.0 * u * h - 2.0 * k * hm;
    hm = h;
    h = hn;
  }
  double wp = 1.0;
  for (int k = 1; k < n; k++) wp *= w;  // w^(n-1)
  double sg = (n & 1) ? -1.0 : 1.0;
  return 0.5 * sg * h * exp(-u * u) * (n == 0 ? w : 1.0 / wp);
}

// rho*phi obeys the 1-D wave equation; with tau = v t the pulse that starts at
// rest is phi = [g(tau + rho) - g(tau - rho)] / (2 rho), summed as its Taylor
// series in rho near the centre to avoid cancellation.
__device__ inline void pulse_eval(double A, const double xc[3], double w, double v, double t, const double X[3],
                                  double out[5]) {
  double d[3] = {X[0] - xc[0], X[1] - xc[1], X[2] - xc[2]};
  double rho = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  double tau = v * t, phi, pt, gf;
  if (rho < 0.05 * w) {
    double r2 = rho * rho, pw2 = 1.0, fact = 1.0;
    phi = 0.0; pt = 0.0; gf = 0.0;
    for (int k = 0; k <= 5; k++) {
      if (k > 0) fact *= (2.0 * k) * (2.0 * k + 1.0);
      double g1 = gpulse_der(2 * k + 1, tau, w);
      phi += g1 * pw2 / fact;
      pt += gpulse_der(2 * k + 2, tau, w) * pw2 / fact;
      if (k + 1 <= 5) {
        // gradient factor term k+1: 2(k+1) g^(2k+3) rho^(2k) / (2k+3)!
        double f3 = fact * (2.0 * k + 2.0) * (2.0 * k + 3.0);
        gf += gpulse_der(2 * k + 3, tau, w) * 2.0 * (k + 1) * pw2 / f3;
      }
      pw2 *= r2;
    }
    pt *= v;
  } else {
    // g(s) = s e^{-u^2} and g'(s) = (1 - 2 u^2) e^{-u^2} with u = s / w: one
    // exponential per sign, reciprocals instead of divisions
    const double iw = 1.0 / w, up = (tau + rho) * iw, um = (tau - rho) * iw;
    const double ep = exp(-up * up), em = exp(-um * um);
    const double gp = (tau + rho) * ep, gm = (tau - rho) * em;
    const double g1p = (1.0 - 2.0 * up * up) * ep, g1m = (1.0 - 2.0 * um * um) * em;
    const double irho = 1.0 / rho, i2r = 0.5 * irho;
    phi = (gp - gm) * i2r;
    pt = v * (g1p - g1m) * i2r;
    gf = ((g1p + g1m) * i2r - phi * irho) * irho;
  }
  out[0] = A * phi;
  out[1] = A * pt;
  for (int a = 0; a < 3; a++) out[2 + a] = A * gf * d[a];
}

__device__ inline void exact_bg(const ExactDev &e, double v, double t, const double X[3], double out[5]) {
  for (int f = 0; f < 5; f++) out[f] = 0.0;
  if (e.kind == EX_PLANE) {
    double arg = e.kappa[0] * X[0] + e.kappa[1] * X[1] + e.kappa[2] * X[2] - v * e.knorm * t + e.phase;
    double s, c;
    sincos(arg, &s, &c);
    out[0] = e.amp * s + e.offset;
    out[1] = -e.amp * v * e.knorm * c;
    for (int a = 0; a < 3; a++) out[2 + a] = e.amp * e.kappa[a] * c;
  } else if (e.kind == EX_GAUSS) {
    for (int g = 0; g < e.n; g++) {
      double o[5];
      pulse_eval(e.pa[g], e.px[g], e.pw[g], v, t, X, o);
      for (int f = 0; f < 5; f++) out[f] += o[f];
    }
  }
}

// Exact state in the numerical frame of patch p at x'.
__device__ inline void exact_patch(const ExactDev &e, double v, const PatchDev &p, const PoseDev &ps, double t,
                                   const double xp[3], double out[5]) {
  double X[3], bg[5];
  fwd_map(p, ps, xp, X);
  exact_bg(e, v, t, X, bg);
  double o4[4];
  bg_to_patch(p, ps, xp, bg[1], bg + 2, o4);
  out[0] = bg[0];
  for (int m = 0; m < 4; m++) out[1 + m] = o4[m];
}

// ---------------------------------------------------------------------------
// Lagrange weights (Eq. Pijk): stencil start s = floor(q - (P-2)/2), q the
// fractional cell index of the point.
// ---------------------------------------------------------------------------
__device__ inline int lagrange_w(int P, double q, double *w) {
  int s = (int)floor(q - 0.5 * (P - 2));
  double t = q - (double)s;  // position relative to the first node
  for (int m = 0; m < P; m++) {
    double num = 1.0, den = 1.0;
    for (int l = 0; l < P; l++) {
      if (l == m) continue;
      num *= (t - (double)l);
      den *= (double)(m - l);
    }
    w[m] = num / den;
  }
  return s;
}

// Compile-time-P Lagrange weights: the same nodes and start index as
// lagrange_w, with the constant denominators prod_{l != m} (m - l) folded.
template <int P>
__device__ inline double lagrange_den(int m) {
  double d = 1.0;
  for (int l = 0; l < P; l++)
    if (l != m) d *= (double)(m - l);
  return d;
}

template <int P>
__device__ inline int lagrange_wt(double q, double *w) {
  const int s = (int)floor(q - 0.5 * (P - 2));
  const double t = q - (double)s;
  double pre[P], suf[P];
  pre[0] = 1.0;
#pragma unroll
  for (int m = 1; m < P; m++) pre[m] = pre[m - 1] * (t - (double)(m - 1));
  suf[P - 1] = 1.0;
#pragma unroll
  for (int m = P - 2; m >= 0; m--) suf[m] = suf[m + 1] * (t - (double)(m + 1));
#pragma unroll
  for (int m = 0; m < P; m++) w[m] = pre[m] * suf[m] * (1.0 / lagrange_den<P>(m));
  return s;
}

// Weight of node m alone (used when a lane needs only a few of the weights).
template <int P>
__device__ inline double lagrange_one(double t, int m) {
  double num = 1.0;
#pragma unroll
  for (int l = 0; l < P; l++)
    if (l != m) num *= (t - (double)l);
  double den = 1.0;
#pragma unroll
  for (int l = 0; l < P; l++)
    if (l != m) den *= (double)(m - l);
  return num / den;
}

}  // namespace pw
