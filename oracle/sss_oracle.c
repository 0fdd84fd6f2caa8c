/*
 * sss_oracle.c -- plain FP64 CPU reference of the Student Splatting and
 * Scooping rasterizer hot path (3D Student Splatting and Scooping,
 * arXiv 2503.10148).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the HIP library.
 *
 * What it computes, in the order the paper states it:
 *   project   -- Sec. 3.2 eq. (t_2D) and SM Sec. "Forward Pass": each 3D
 *                Student's t (mean mu, Sigma = R S S^T R^T, dof nu) is mapped
 *                through the view transform and the local affine (EWA)
 *                approximation of the perspective map to a 2D Student's t
 *                with exponent -(nu+2)/2; nu is clamped to [1, 1e4]
 *                (SM "Implementation Details").
 *   bin       -- every visible component is listed in each 16x16 tile that
 *                its truncation rectangle touches; per tile the list is in
 *                ascending (depth key, component index) order.
 *   composite -- Sec. 3.4 eq. (SSS_color): signed front-to-back alpha
 *                compositing, alpha = o * T2D with o in [-1, 1].
 *   backward  -- SM Sec. "Backward Pass": the chain rule through alpha, T2D,
 *                h(x), the projected mean and covariance, down to mu, S, R,
 *                the SH colour, o and nu.  dT/dnu is the complete derivative
 *                (the printed one drops the term from the nu in the
 *                exponent).
 *   SGHMC     -- Sec. 3.4 eq. (sigmoidUpdate) / SM eq. (SGHMC) with the
 *                readings listed in the design notes; noise from
 *                Philox4x32-10 (Salmon et al., SC'11) and Box-Muller.
 *   Adam      -- Kingma & Ba (2015), used for the non-mean parameters.
 *
 * Conventions the paper does not fix (pixel centres at x+1/2, pinhole camera
 * in OpenCV axes, quaternion rotation, alpha cut-off 1/255 and clamp 0.99,
 * termination at T < 1e-4, truncation at the alpha level set, depth key as an
 * FP32 fma chain, real SH basis with the Condon-Shortley phase) are the
 * readings stated in the design notes.
 *
 * Layouts (all doubles unless noted, row-major):
 *   cam[20]  = viewmat (3x4 world->camera) [12], fx, fy, cx, cy, width, height,
 *              clamp_width, clamp_height (the image size whose half field of
 *              view bounds the EWA Jacobian; equal to width, height except
 *              for a window cut out of a larger image)
 *   opts[12] = alpha_min, alpha_max, t_min, z_near, nu_min, nu_max, lowpass,
 *              bg_r, bg_g, bg_b, family (0 Student's t, 1 Gaussian: the
 *              nu -> infinity limit exp(-h/2) of Sec. 3.2), trunc_mode (0: the
 *              rectangle bounds the alpha level set; 1: it bounds the smaller
 *              of that set and the ellipse holding the same probability mass
 *              as the Gaussian 3-sigma ellipse)
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_TILE 16

enum {
  PF_RECT_EDGE = 1,  /* a rectangle edge lies within 1e-9 of a tile border   */
  PF_DET = 2,        /* projected covariance nearly singular                  */
  PF_RGB_CLAMP = 4,  /* an SH colour channel within 1e-9 of the clamp at 0    */
  PF_TX_CLAMP = 8,   /* x/z or y/z within 1e-9 of the EWA frustum clamp       */
  PF_NU_CLAMP = 16,  /* unused: the clamp and its gradient gate compare the    */
                     /* FP32 input itself, identically on both sides           */
};
enum {
  XF_ALPHA_MIN = 1,  /* some |alpha| within 1e-5 (relative) of alpha_min      */
  XF_ALPHA_MAX = 2,  /* some |alpha| within 1e-5 (relative) of alpha_max      */
  XF_T_MIN = 4,      /* transmittance test within 1e-3 (relative) of t_min    */
  XF_COMPONENT = 8,  /* a component flagged by the projection contributed      */
};

/* ------------------------------------------------------------------------ */
/* Real spherical harmonics, degree <= 3.                                     */
/* Cartesian polynomial form of the textbook real SH with the Condon-Shortley */
/* phase; index k = l*l + l + m.  Each basis function is a short sum of       */
/* monomials c * x^a y^b z^c so that its gradient is mechanical.              */
/* ------------------------------------------------------------------------ */
typedef struct { double c; int a, b, e; } orc_mono;
typedef struct { int nterm; orc_mono t[3]; } orc_poly;

static orc_poly g_sh[16];
static int g_sh_ready = 0;

static void sh_init(void) {
  if (g_sh_ready) return;
  const double pi = 3.14159265358979323846;
  const double n0 = 0.5 * sqrt(1.0 / pi);
  const double n1 = sqrt(3.0 / (4.0 * pi));
  const double n2a = 0.5 * sqrt(15.0 / pi);
  const double n2b = 0.25 * sqrt(5.0 / pi);
  const double n2c = 0.25 * sqrt(15.0 / pi);
  const double n3a = 0.25 * sqrt(35.0 / (2.0 * pi));
  const double n3b = 0.5 * sqrt(105.0 / pi);
  const double n3c = 0.25 * sqrt(21.0 / (2.0 * pi));
  const double n3d = 0.25 * sqrt(7.0 / pi);
  const double n3e = 0.25 * sqrt(105.0 / pi);
  orc_poly p[16] = {
    /* l = 0 */
    {1, {{n0, 0, 0, 0}}},
    /* l = 1: m = -1, 0, 1 */
    {1, {{-n1, 0, 1, 0}}},
    {1, {{n1, 0, 0, 1}}},
    {1, {{-n1, 1, 0, 0}}},
    /* l = 2 */
    {1, {{n2a, 1, 1, 0}}},
    {1, {{-n2a, 0, 1, 1}}},
    {3, {{2.0 * n2b, 0, 0, 2}, {-n2b, 2, 0, 0}, {-n2b, 0, 2, 0}}},
    {1, {{-n2a, 1, 0, 1}}},
    {2, {{n2c, 2, 0, 0}, {-n2c, 0, 2, 0}}},
    /* l = 3 */
    {2, {{-3.0 * n3a, 2, 1, 0}, {n3a, 0, 3, 0}}},
    {1, {{n3b, 1, 1, 1}}},
    {3, {{-4.0 * n3c, 0, 1, 2}, {n3c, 2, 1, 0}, {n3c, 0, 3, 0}}},
    {3, {{2.0 * n3d, 0, 0, 3}, {-3.0 * n3d, 2, 0, 1}, {-3.0 * n3d, 0, 2, 1}}},
    {3, {{-4.0 * n3c, 1, 0, 2}, {n3c, 3, 0, 0}, {n3c, 1, 2, 0}}},
    {2, {{n3e, 2, 0, 1}, {-n3e, 0, 2, 1}}},
    {2, {{-n3a, 3, 0, 0}, {3.0 * n3a, 1, 2, 0}}},
  };
  memcpy(g_sh, p, sizeof(p));
  g_sh_ready = 1;
}

static double ipow(double x, int k) {
  double r = 1.0;
  for (int i = 0; i < k; ++i) r *= x;
  return r;
}

/* Y[k] and (optionally) dY[k][3] = gradient of the polynomial extension. */
void orc_sh_eval(int degree, const double* dir, double* Y, double* dY) {
  sh_init();
  const int K = (degree + 1) * (degree + 1);
  const double x = dir[0], y = dir[1], z = dir[2];
  for (int k = 0; k < K; ++k) {
    double v = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (int j = 0; j < g_sh[k].nterm; ++j) {
      const orc_mono m = g_sh[k].t[j];
      v += m.c * ipow(x, m.a) * ipow(y, m.b) * ipow(z, m.e);
      if (m.a > 0) gx += m.c * m.a * ipow(x, m.a - 1) * ipow(y, m.b) * ipow(z, m.e);
      if (m.b > 0) gy += m.c * m.b * ipow(x, m.a) * ipow(y, m.b - 1) * ipow(z, m.e);
      if (m.e > 0) gz += m.c * m.e * ipow(x, m.a) * ipow(y, m.b) * ipow(z, m.e - 1);
    }
    Y[k] = v;
    if (dY) { dY[3 * k + 0] = gx; dY[3 * k + 1] = gy; dY[3 * k + 2] = gz; }
  }
}

/* The same basis from its textbook definition: associated Legendre
 * functions (Condon-Shortley phase, standard three-term recurrence) times
 * cos(m phi) / sin(|m| phi) with the usual normalisation.  Used only to pin
 * the Cartesian table above. */
void orc_sh_eval_legendre(int degree, const double* dir, double* Y) {
  const double pi = 3.14159265358979323846;
  const double ct = dir[2];
  const double st = sqrt(fmax(0.0, 1.0 - ct * ct));
  const double phi = atan2(dir[1], dir[0]);
  double P[4][4];
  memset(P, 0, sizeof(P));
  for (int m = 0; m <= degree; ++m) {
    double pmm = 1.0;                       /* (-1)^m (2m-1)!! st^m */
    for (int i = 1; i <= m; ++i) pmm *= -(2.0 * i - 1.0) * st;
    P[m][m] = pmm;
    if (m + 1 <= degree) P[m + 1][m] = ct * (2.0 * m + 1.0) * pmm;
    for (int l = m + 2; l <= degree; ++l)
      P[l][m] = ((2.0 * l - 1.0) * ct * P[l - 1][m] - (l + m - 1.0) * P[l - 2][m]) / (double)(l - m);
  }
  for (int l = 0; l <= degree; ++l) {
    for (int m = -l; m <= l; ++m) {
      const int am = m < 0 ? -m : m;
      double fr = 1.0;                      /* (l-|m|)! / (l+|m|)! */
      for (int i = l - am + 1; i <= l + am; ++i) fr /= (double)i;
      const double K = sqrt((2.0 * l + 1.0) / (4.0 * pi) * fr);
      double v;
      if (m == 0) v = K * P[l][0];
      else if (m > 0) v = sqrt(2.0) * K * cos(m * phi) * P[l][m];
      else v = sqrt(2.0) * K * sin(am * phi) * P[l][am];
      Y[l * l + l + m] = v;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Geometry helpers                                                          */
/* ------------------------------------------------------------------------ */

/* Rotation matrix of a unit quaternion (w, x, y, z), row-major. */
static void quat_to_rot(const double* q, double* R) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z);       R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z);       R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y);       R[7] = 2.0 * (y * z + w * x);       R[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* dR[e][4]: partial derivative of R entry e w.r.t. (w, x, y, z). */
static void quat_to_rot_jac(const double* q, double dR[9][4]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  double J[9][4] = {
    {0.0, 0.0, -4.0 * y, -4.0 * z},
    {-2.0 * z, 2.0 * y, 2.0 * x, -2.0 * w},
    {2.0 * y, 2.0 * z, 2.0 * w, 2.0 * x},
    {2.0 * z, 2.0 * y, 2.0 * x, 2.0 * w},
    {0.0, -4.0 * x, 0.0, -4.0 * z},
    {-2.0 * x, -2.0 * w, 2.0 * z, 2.0 * y},
    {-2.0 * y, 2.0 * z, -2.0 * w, 2.0 * x},
    {2.0 * x, 2.0 * w, 2.0 * z, 2.0 * y},
    {0.0, -4.0 * x, -4.0 * y, 0.0},
  };
  memcpy(dR, J, sizeof(J));
}

static int near_integer(double v) {
  return fabs(v - nearbyint(v)) <= 1e-9 * fmax(1.0, fabs(v));
}

/* Depth key: the FP32 value of the camera-space depth, evaluated as a chain
 * of single-rounding fused multiply-adds so that every IEEE-754 machine
 * produces the same bits; positive floats order like their bit patterns. */
static uint32_t depth_key32(const double* cam, const double* mu, float* zf_out) {
  const float w20 = (float)cam[8], w21 = (float)cam[9], w22 = (float)cam[10], t2 = (float)cam[11];
  const float zf = fmaf(w20, (float)mu[0], fmaf(w21, (float)mu[1], fmaf(w22, (float)mu[2], t2)));
  uint32_t bits;
  memcpy(&bits, &zf, 4);
  *zf_out = zf;
  return bits;
}

/* Tile membership, by definition: a component is listed in tile (tx, ty)
 * when some point of the tile's box of pixel centres
 * [16 tx + 1/2, 16 tx + 31/2] x [16 ty + 1/2, 16 ty + 31/2] lies in its
 * ellipse {p : (p - m)^T Q (p - m) <= hr}, Q the conic (inverse 2D
 * covariance), i.e. when the minimum of the quadratic form over the box is
 * at most hr.  The minimum is 0 when the mean lies in the box; otherwise it
 * sits on the boundary, and along each edge the form is a one-dimensional
 * quadratic whose minimum is its vertex clamped to the edge.  hr = infinity
 * (no cut-off) lists every tile. */
static double box_min_h(const double* Q, double mx, double my, double bx0, double bx1, double by0, double by1) {
  const double a = Q[0], b = Q[1], c = Q[2];
  if (mx >= bx0 && mx <= bx1 && my >= by0 && my <= by1) return 0.0;
  double best = INFINITY;
  const double xs[2] = {bx0, bx1}, ys[2] = {by0, by1};
  for (int e = 0; e < 2; ++e) {
    /* vertical edge x = xs[e]: minimise over dy */
    const double dx = xs[e] - mx;
    const double dy = fmin(fmax(-b * dx / c, by0 - my), by1 - my);
    best = fmin(best, a * dx * dx + 2.0 * b * dx * dy + c * dy * dy);
  }
  for (int e = 0; e < 2; ++e) {
    /* horizontal edge y = ys[e]: minimise over dx */
    const double dy = ys[e] - my;
    const double dx = fmin(fmax(-b * dy / a, bx0 - mx), bx1 - mx);
    best = fmin(best, a * dx * dx + 2.0 * b * dx * dy + c * dy * dy);
  }
  return best;
}

/* Whether tile (tx, ty) is listed; sets *edge when the box minimum lies
 * within 1e-9 (relative) of hr, where the FP32/FP64 rounding of another
 * formulation of the same test could decide the other way. */
static int tile_listed(const double* Q, double mx, double my, double hr, int tx, int ty, int* edge) {
  if (isinf(hr)) return 1;
  const double hmin = box_min_h(Q, mx, my, ORC_TILE * tx + 0.5, ORC_TILE * tx + 15.5, ORC_TILE * ty + 0.5,
                                ORC_TILE * ty + 15.5);
  if (fabs(hmin - hr) <= 1e-9 * hr) *edge = 1;
  return hmin <= hr;
}

int orc_tiles_x(const double* cam) { return ((int)cam[16] + ORC_TILE - 1) / ORC_TILE; }
int orc_tiles_y(const double* cam) { return ((int)cam[17] + ORC_TILE - 1) / ORC_TILE; }

/* ------------------------------------------------------------------------ */
/* Projection (forward)                                                      */
/* ------------------------------------------------------------------------ */
void orc_project(int n, int sh_degree, const double* means, const double* scales,
                 const double* quats, const double* nu, const double* opac,
                 const double* sh, const double* cam, const double* opts,
                 int32_t* valid, double* mean2d, double* cov2d, double* conic,
                 double* rgb, double* nu_c, double* hstar, double* hrect, int32_t* rect,
                 uint32_t* key, int32_t* touched, int32_t* pflags) {
  sh_init();
  const int K = (sh_degree + 1) * (sh_degree + 1);
  const double* Wm = cam;  /* 3x4 */
  const double fx = cam[12], fy = cam[13], cx = cam[14], cy = cam[15];
  const int W = (int)cam[16], H = (int)cam[17];
  const int tx_n = orc_tiles_x(cam), ty_n = orc_tiles_y(cam);
  const double alpha_min = opts[0], z_near = opts[3], nu_min = opts[4], nu_max = opts[5];
  const double lowpass = opts[6];
  const double limx = 1.3 * (cam[18] / (2.0 * fx)), limy = 1.3 * (cam[19] / (2.0 * fy));
  /* camera centre: -R^T t */
  double campos[3];
  for (int a = 0; a < 3; ++a)
    campos[a] = -(Wm[0 * 4 + a] * Wm[3] + Wm[1 * 4 + a] * Wm[7] + Wm[2 * 4 + a] * Wm[11]);

#pragma omp parallel for schedule(static)
  for (int i = 0; i < n; ++i) {
    const double* mu = means + 3 * i;
    valid[i] = 0; touched[i] = 0; pflags[i] = 0;
    mean2d[2 * i] = mean2d[2 * i + 1] = 0.0;
    for (int a = 0; a < 3; ++a) { cov2d[3 * i + a] = 0.0; conic[3 * i + a] = 0.0; rgb[3 * i + a] = 0.0; }
    nu_c[i] = 0.0; hstar[i] = 0.0;
    for (int a = 0; a < 4; ++a) rect[4 * i + a] = 0;

    float zf;
    key[i] = depth_key32(cam, mu, &zf);
    if (!(zf > (float)z_near)) continue;                 /* near plane */
    const double o = opac[i];
    if (!(fabs(o) >= alpha_min)) continue;               /* can never pass the cut-off */

    /* camera-space position */
    const double X = Wm[0] * mu[0] + Wm[1] * mu[1] + Wm[2] * mu[2] + Wm[3];
    const double Y = Wm[4] * mu[0] + Wm[5] * mu[1] + Wm[6] * mu[2] + Wm[7];
    const double Z = Wm[8] * mu[0] + Wm[9] * mu[1] + Wm[10] * mu[2] + Wm[11];

    /* Sigma = R diag(s^2) R^T */
    const double* q = quats + 4 * i;
    const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (!(qn > 0.0)) continue;
    const double qu[4] = {q[0] / qn, q[1] / qn, q[2] / qn, q[3] / qn};
    double Rq[9];
    quat_to_rot(qu, Rq);
    const double* s = scales + 3 * i;
    double Sig[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) acc += Rq[3 * r + k] * s[k] * s[k] * Rq[3 * c + k];
        Sig[3 * r + c] = acc;
      }

    /* local affine approximation of the perspective map (EWA) */
    const double xz = X / Z, yz = Y / Z;
    const double txz = fmin(fmax(xz, -limx), limx);
    const double tyz = fmin(fmax(yz, -limy), limy);
    if (fabs(fabs(xz) - limx) <= 1e-9 * limx || fabs(fabs(yz) - limy) <= 1e-9 * limy) pflags[i] |= PF_TX_CLAMP;
    double J[6] = {fx / Z, 0.0, -fx * txz / Z, 0.0, fy / Z, -fy * tyz / Z};
    double M[6];                                         /* M = J * Rview */
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 3; ++c)
        M[3 * r + c] = J[3 * r + 0] * Wm[0 * 4 + c] + J[3 * r + 1] * Wm[1 * 4 + c] + J[3 * r + 2] * Wm[2 * 4 + c];
    double S2[4];                                        /* M Sigma M^T */
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c) {
        double acc = 0.0;
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) acc += M[3 * r + a] * Sig[3 * a + b] * M[3 * c + b];
        S2[2 * r + c] = acc;
      }
    const double A = S2[0] + lowpass, B = S2[1], D = S2[3] + lowpass;
    const double det = A * D - B * B;
    if (!(det > 0.0)) continue;
    if (det <= 1e-9 * A * D) pflags[i] |= PF_DET;

    const double mx = fx * xz + cx, my = fy * yz + cy;
    const double nuc = fmin(fmax(nu[i], nu_min), nu_max);

    /* truncation: the alpha level set |o| T2D(h) = alpha_min, i.e.
       h* = nu ((|o|/alpha_min)^(2/(nu+2)) - 1); outside it |alpha| < alpha_min */
    int x0, x1, y0, y1;
    double hs, hr;
    if (alpha_min > 0.0) {
      hs = opts[10] == 1.0 ? 2.0 * log(fabs(o) / alpha_min) : nuc * expm1(2.0 / (nuc + 2.0) * log(fabs(o) / alpha_min));
      /* coverage rule (Sec. 3.2 truncation by a critical value): h of a 2D t
         variable has P(h <= q) = 1 - (1 + q/nu)^(-nu/2); the Gaussian 3-sigma
         ellipse holds 1 - exp(-9/2), reached at q = nu (exp(9/nu) - 1)
         (q = 9 for the Gaussian).  Beyond h* nothing is drawn anyway, so the
         rectangle uses the smaller of the two. */
      hr = hs;
      if (opts[11] == 1.0) {
        const double q = opts[10] == 1.0 ? 9.0 : nuc * expm1(9.0 / nuc);
        if (q < hr) hr = q;
      }
      const double ex = sqrt(hr * A), ey = sqrt(hr * D);
      const double lx = (mx - ex) / ORC_TILE, hx = (mx + ex) / ORC_TILE;
      const double ly = (my - ey) / ORC_TILE, hy = (my + ey) / ORC_TILE;
      if (hx < 0.0 || lx >= tx_n || hy < 0.0 || ly >= ty_n) continue;   /* off-screen */
      if (near_integer(lx) || near_integer(hx) || near_integer(ly) || near_integer(hy)) pflags[i] |= PF_RECT_EDGE;
      x0 = (int)fmax(0.0, floor(lx)); x1 = (int)fmin((double)(tx_n - 1), floor(hx));
      y0 = (int)fmax(0.0, floor(ly)); y1 = (int)fmin((double)(ty_n - 1), floor(hy));
    } else {
      hs = hr = INFINITY;
      x0 = 0; x1 = tx_n - 1; y0 = 0; y1 = ty_n - 1;
    }
    /* tiles: those of the rectangle whose pixel-centre box meets the ellipse */
    int count = 0, edge = 0;
    const double Qc[3] = {D / det, -B / det, A / det};
    for (int ty = y0; ty <= y1; ++ty)
      for (int tx = x0; tx <= x1; ++tx) count += tile_listed(Qc, mx, my, hr, tx, ty, &edge);
    if (edge) pflags[i] |= PF_RECT_EDGE;
    if (count == 0) continue;

    /* colour: SH at the viewing direction, offset by 1/2, clamped at 0 */
    double v[3] = {mu[0] - campos[0], mu[1] - campos[1], mu[2] - campos[2]};
    const double vn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    const double dir[3] = {v[0] / vn, v[1] / vn, v[2] / vn};
    double Yb[16];
    orc_sh_eval(sh_degree, dir, Yb, NULL);
    for (int c = 0; c < 3; ++c) {
      double acc = 0.0;
      for (int k = 0; k < K; ++k) acc += Yb[k] * sh[(size_t)i * K * 3 + 3 * k + c];
      acc += 0.5;
      if (fabs(acc) <= 1e-9) pflags[i] |= PF_RGB_CLAMP;
      rgb[3 * i + c] = acc > 0.0 ? acc : 0.0;
    }

    valid[i] = 1;
    mean2d[2 * i] = mx; mean2d[2 * i + 1] = my;
    cov2d[3 * i] = A; cov2d[3 * i + 1] = B; cov2d[3 * i + 2] = D;
    conic[3 * i] = Qc[0]; conic[3 * i + 1] = Qc[1]; conic[3 * i + 2] = Qc[2];
    nu_c[i] = nuc;
    hstar[i] = hs;
    hrect[i] = hr;
    rect[4 * i] = x0; rect[4 * i + 1] = y0; rect[4 * i + 2] = x1; rect[4 * i + 3] = y1;
    touched[i] = count;
  }
}

/* ------------------------------------------------------------------------ */
/* Binning: per-tile lists in ascending (depth key, index) order             */
/* ------------------------------------------------------------------------ */
typedef struct { int64_t tile; uint32_t key; int32_t idx; } orc_pair;

static int pair_cmp(const void* pa, const void* pb) {
  const orc_pair* a = (const orc_pair*)pa;
  const orc_pair* b = (const orc_pair*)pb;
  if (a->tile != b->tile) return a->tile < b->tile ? -1 : 1;
  if (a->key != b->key) return a->key < b->key ? -1 : 1;
  if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;
  return 0;
}

/* rect[4*i] = x0,y0,x1,y1 (inclusive tile range); touched[i] == 0 means not
 * listed.  With geometry (mean2d, conic, hrect non-NULL) a tile of the
 * rectangle is listed when its pixel-centre box meets the ellipse
 * (tile_listed), else the whole rectangle is listed.  Writes
 * tile_start[n_tiles+1] and tile_list[] (component indices).  Returns the
 * number of pairs, or -(needed) when it exceeds list_cap. */
int64_t orc_bin(int n, const int32_t* touched, const int32_t* rect, const uint32_t* key,
                const double* mean2d, const double* conic, const double* hrect,
                int tiles_x, int tiles_y, int32_t* tile_start, int32_t* tile_list, int64_t list_cap) {
  int64_t m = 0;
  for (int i = 0; i < n; ++i) m += touched[i] > 0 ? touched[i] : 0;
  if (m > list_cap) return -m;
  orc_pair* pairs = (orc_pair*)malloc(sizeof(orc_pair) * (size_t)(m > 0 ? m : 1));
  int64_t p = 0;
  for (int i = 0; i < n; ++i) {
    if (touched[i] <= 0) continue;
    for (int ty = rect[4 * i + 1]; ty <= rect[4 * i + 3]; ++ty) {
      for (int tx = rect[4 * i]; tx <= rect[4 * i + 2]; ++tx) {
        int edge = 0;
        if (mean2d && !tile_listed(conic + 3 * i, mean2d[2 * i], mean2d[2 * i + 1], hrect[i], tx, ty, &edge)) continue;
        if (p == m) { free(pairs); return -(m + 1); }   /* touched does not match the tiles */
        pairs[p].tile = (int64_t)ty * tiles_x + tx;
        pairs[p].key = key[i];
        pairs[p].idx = i;
        ++p;
      }
    }
  }
  if (p != m) { free(pairs); return -(m + 1); }
  qsort(pairs, (size_t)m, sizeof(orc_pair), pair_cmp);
  const int64_t nt = (int64_t)tiles_x * tiles_y;
  int64_t cur = 0;
  for (int64_t t = 0; t <= nt; ++t) {
    while (cur < m && pairs[cur].tile < t) ++cur;
    tile_start[t] = (int32_t)cur;
  }
  for (int64_t j = 0; j < m; ++j) tile_list[j] = pairs[j].idx;
  free(pairs);
  return m;
}

/* ------------------------------------------------------------------------ */
/* Compositing                                                                */
/* ------------------------------------------------------------------------ */

/* 2D Student's t, eq. (t_2D): (1 + h/nu)^(-(nu+2)/2). */
static double t2d(double h, double nu) { return exp(-0.5 * (nu + 2.0) * log1p(h / nu)); }

typedef struct {
  int32_t idx;
  double alpha, T, t2, h, dx, dy;
  int clamped;
} orc_hit;

/* Composite one pixel over an ordered list.  Fills hits[] (may be NULL) with
 * the composited entries, returns how many.  *ncon = list position after the
 * last composited entry; *xf = explanation flags. */
static int composite_pixel(double px, double py, const int32_t* list, int64_t len,
                           const double* mean2d, const double* conic, const double* rgb,
                           const double* opac, const double* nu_c, const int32_t* pflags,
                           const double* opts, double* out3, double* tfin, int32_t* ncon,
                           int32_t* xf, orc_hit* hits, int max_hits) {
  const double amin = opts[0], amax = opts[1], tmin = opts[2];
  double T = 1.0, C[3] = {0.0, 0.0, 0.0};
  int nh = 0, flags = 0;
  int32_t last = 0;
  for (int64_t k = 0; k < len; ++k) {
    const int32_t i = list[k];
    const double dx = px - mean2d[2 * i], dy = py - mean2d[2 * i + 1];
    const double a = conic[3 * i], b = conic[3 * i + 1], c = conic[3 * i + 2];
    const double h = a * dx * dx + 2.0 * b * dx * dy + c * dy * dy;
    const double tt = opts[10] == 1.0 ? exp(-0.5 * h) : t2d(h, nu_c[i]);
    double alpha = opac[i] * tt;
    if (fabs(fabs(alpha) - amin) <= 1e-5 * amin) flags |= XF_ALPHA_MIN;
    if (fabs(alpha) < amin) continue;
    if (pflags[i]) flags |= XF_COMPONENT;
    if (fabs(fabs(alpha) - amax) <= 1e-5 * amax) flags |= XF_ALPHA_MAX;
    int clamped = 0;
    if (alpha > amax) { alpha = amax; clamped = 1; }
    if (alpha < -amax) { alpha = -amax; clamped = 1; }
    const double Tn = T * (1.0 - alpha);
    if (fabs(Tn - tmin) <= 1e-3 * tmin) flags |= XF_T_MIN;
    if (Tn < tmin) break;
    for (int ch = 0; ch < 3; ++ch) C[ch] += rgb[3 * i + ch] * alpha * T;
    if (hits && nh < max_hits) {
      hits[nh].idx = i; hits[nh].alpha = alpha; hits[nh].T = T; hits[nh].t2 = tt;
      hits[nh].h = h; hits[nh].dx = dx; hits[nh].dy = dy; hits[nh].clamped = clamped;
    }
    ++nh;
    T = Tn;
    last = (int32_t)(k + 1);
  }
  for (int ch = 0; ch < 3; ++ch) out3[ch] = C[ch] + T * opts[7 + ch];
  *tfin = T;
  *ncon = last;
  *xf = flags;
  return nh;
}

/* Tiled forward: pixel (x, y) composites the list of its tile. */
void orc_render_tiled(const double* mean2d, const double* conic, const double* rgb,
                      const double* opac, const double* nu_c, const int32_t* pflags,
                      int W, int H, const int32_t* tile_start, const int32_t* tile_list,
                      const double* opts, double* image, double* tfinal, int32_t* ncontrib,
                      int32_t* xflags) {
  const int tx_n = (W + ORC_TILE - 1) / ORC_TILE;
#pragma omp parallel for schedule(dynamic, 4)
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      const int64_t t = (int64_t)(y / ORC_TILE) * tx_n + x / ORC_TILE;
      const int64_t p = (int64_t)y * W + x;
      composite_pixel(x + 0.5, y + 0.5, tile_list + tile_start[t], tile_start[t + 1] - tile_start[t],
                      mean2d, conic, rgb, opac, nu_c, pflags, opts, image + 3 * p, tfinal + p,
                      ncontrib + p, xflags + p, NULL, 0);
    }
}

static const uint32_t* g_sort_key;
static int idx_key_cmp(const void* pa, const void* pb) {
  const int32_t a = *(const int32_t*)pa, b = *(const int32_t*)pb;
  if (g_sort_key[a] != g_sort_key[b]) return g_sort_key[a] < g_sort_key[b] ? -1 : 1;
  return a < b ? -1 : (a > b ? 1 : 0);
}

/* Brute-force forward: every pixel walks every visible component in
 * ascending (depth key, index) order, with no tiles and no rectangles. */
void orc_render_brute(int n, const int32_t* valid, const uint32_t* key, const double* mean2d,
                      const double* conic, const double* rgb, const double* opac,
                      const double* nu_c, const int32_t* pflags, int W, int H,
                      const double* opts, double* image, double* tfinal, int32_t* ncontrib,
                      int32_t* xflags) {
  int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int m = 0;
  for (int i = 0; i < n; ++i)
    if (valid[i]) order[m++] = i;
  g_sort_key = key;
  qsort(order, (size_t)m, sizeof(int32_t), idx_key_cmp);
#pragma omp parallel for schedule(dynamic, 4)
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      const int64_t p = (int64_t)y * W + x;
      int32_t nc;
      composite_pixel(x + 0.5, y + 0.5, order, m, mean2d, conic, rgb, opac, nu_c, pflags, opts,
                      image + 3 * p, tfinal + p, &nc, xflags + p, NULL, 0);
      ncontrib[p] = nc;  /* position in the global order, not a tile list */
    }
  free(order);
}

/* ------------------------------------------------------------------------ */
/* Backward through the compositing (per pixel, back to front)               */
/* ------------------------------------------------------------------------ */
/* With S_{n+1} = bg and S_j = c_j a_j + (1 - a_j) S_{j+1}, the output is
 * C = sum_{j<=k} c_j a_j T_j + T_{k+1} S_{k+1}, hence
 * dC/da_j = T_j (c_j - S_{j+1}).  dC/dc_j = a_j T_j.  Then a = o T2D unless
 * clamped, and T2D(h, nu) with h = d^T Q d, d = pixel - mean2d. */
void orc_render_backward(int n, const double* mean2d, const double* conic, const double* rgb,
                         const double* opac, const double* nu_c, const int32_t* pflags,
                         int W, int H, const int32_t* tile_start, const int32_t* tile_list,
                         const double* opts, const double* dl_dimg, double* g_mean2d,
                         double* g_conic, double* g_rgb, double* g_opac, double* g_nu) {
  const int tx_n = (W + ORC_TILE - 1) / ORC_TILE;
  /* Pixel rows are shared among the threads; each thread adds its pixels'
   * terms into its own ten sums per component (mean2d 2, conic 3, rgb 3,
   * opacity, nu), and the partial sums are added into the outputs in thread
   * order afterwards. */
  const int nt = omp_get_max_threads();
  double* part = (double*)calloc((size_t)nt * (size_t)n * 10, sizeof(double));
#pragma omp parallel num_threads(nt)
  {
    double* acc = part + (size_t)omp_get_thread_num() * (size_t)n * 10;
    int cap = 1024;
    orc_hit* hits = (orc_hit*)malloc(sizeof(orc_hit) * cap);
#pragma omp for schedule(dynamic, 1)
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) {
        const int64_t t = (int64_t)(y / ORC_TILE) * tx_n + x / ORC_TILE;
        const int64_t p = (int64_t)y * W + x;
        const int64_t len = tile_start[t + 1] - tile_start[t];
        if (len > cap) { cap = (int)len; hits = (orc_hit*)realloc(hits, sizeof(orc_hit) * cap); }
        double out[3], tf;
        int32_t nc, xf;
        const int nh = composite_pixel(x + 0.5, y + 0.5, tile_list + tile_start[t], len, mean2d, conic,
                                       rgb, opac, nu_c, pflags, opts, out, &tf, &nc, &xf, hits, cap);
        const double* g = dl_dimg + 3 * p;
        double S[3] = {opts[7], opts[8], opts[9]};
        for (int j = nh - 1; j >= 0; --j) {
          const orc_hit* e = &hits[j];
          const int32_t i = e->idx;
          const double* c = rgb + 3 * i;
          double* a10 = acc + (size_t)i * 10;
          double dalpha = 0.0;
          for (int ch = 0; ch < 3; ++ch) {
            dalpha += g[ch] * e->T * (c[ch] - S[ch]);
            a10[5 + ch] += g[ch] * e->alpha * e->T;
          }
          for (int ch = 0; ch < 3; ++ch) S[ch] = c[ch] * e->alpha + (1.0 - e->alpha) * S[ch];
          if (e->clamped) continue;
          a10[8] += dalpha * e->t2;
          const double dt2 = dalpha * opac[i];
          const double nu = nu_c[i], h = e->h;
          /* dT2D/dh = -(nu+2)/(2 nu) (1 + h/nu)^(-(nu+4)/2); Gaussian: -T/2 */
          const double dt_dh = opts[10] == 1.0 ? -0.5 * e->t2 : -e->t2 * (nu + 2.0) / (2.0 * (nu + h));
          /* dT2D/dnu, both the base and the exponent depend on nu; Gaussian: 0 */
          const double dt_dnu = opts[10] == 1.0 ? 0.0
                                                : e->t2 * 0.5 * ((nu + 2.0) * h / (nu * (nu + h)) - log1p(h / nu));
          const double dh = dt2 * dt_dh;
          const double a = conic[3 * i], b = conic[3 * i + 1], cc = conic[3 * i + 2];
          a10[0] += dh * (-2.0) * (a * e->dx + b * e->dy);
          a10[1] += dh * (-2.0) * (b * e->dx + cc * e->dy);
          a10[2] += dh * e->dx * e->dx;
          a10[3] += dh * 2.0 * e->dx * e->dy;
          a10[4] += dh * e->dy * e->dy;
          a10[9] += dt2 * dt_dnu;
        }
      }
    free(hits);
  }
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n; ++i)
    for (int th = 0; th < nt; ++th) {
      const double* a10 = part + ((size_t)th * (size_t)n + (size_t)i) * 10;
      g_mean2d[2 * i] += a10[0];
      g_mean2d[2 * i + 1] += a10[1];
      for (int k = 0; k < 3; ++k) g_conic[3 * i + k] += a10[2 + k];
      for (int k = 0; k < 3; ++k) g_rgb[3 * i + k] += a10[5 + k];
      g_opac[i] += a10[8];
      g_nu[i] += a10[9];
    }
  free(part);
}

/* Thread count of the OpenMP loops (the CPU baseline times 1 and all). */
void orc_set_threads(int k) { omp_set_num_threads(k > 0 ? k : 1); }
int orc_max_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------ */
/* Backward through the projection (per component)                           */
/* ------------------------------------------------------------------------ */
void orc_project_backward(int n, int sh_degree, const double* means, const double* scales,
                          const double* quats, const double* nu, const double* opac,
                          const double* sh, const double* cam, const double* opts,
                          const int32_t* valid, const double* g_mean2d, const double* g_conic,
                          const double* g_rgb, const double* g_opac, const double* g_nu,
                          double* d_means, double* d_scales, double* d_quats, double* d_nu,
                          double* d_opac, double* d_sh) {
  sh_init();
  const int K = (sh_degree + 1) * (sh_degree + 1);
  const double* Wm = cam;
  const double fx = cam[12], fy = cam[13];
  const double nu_min = opts[4], nu_max = opts[5], lowpass = opts[6];
  const double limx = 1.3 * (cam[18] / (2.0 * fx)), limy = 1.3 * (cam[19] / (2.0 * fy));
  double campos[3];
  for (int a = 0; a < 3; ++a)
    campos[a] = -(Wm[0 * 4 + a] * Wm[3] + Wm[1 * 4 + a] * Wm[7] + Wm[2 * 4 + a] * Wm[11]);

#pragma omp parallel for schedule(static)
  for (int i = 0; i < n; ++i) {
    if (!valid[i]) continue;
    const double* mu = means + 3 * i;
    const double* s = scales + 3 * i;
    const double* q = quats + 4 * i;

    /* opacity and nu enter the compositing directly */
    d_opac[i] += g_opac[i];
    if (nu[i] >= nu_min && nu[i] <= nu_max) d_nu[i] += g_nu[i];

    /* ---- recompute the forward intermediates ---- */
    const double X = Wm[0] * mu[0] + Wm[1] * mu[1] + Wm[2] * mu[2] + Wm[3];
    const double Y = Wm[4] * mu[0] + Wm[5] * mu[1] + Wm[6] * mu[2] + Wm[7];
    const double Z = Wm[8] * mu[0] + Wm[9] * mu[1] + Wm[10] * mu[2] + Wm[11];
    const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double qu[4] = {q[0] / qn, q[1] / qn, q[2] / qn, q[3] / qn};
    double Rq[9];
    quat_to_rot(qu, Rq);
    double Sig[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) acc += Rq[3 * r + k] * s[k] * s[k] * Rq[3 * c + k];
        Sig[3 * r + c] = acc;
      }
    const double xz = X / Z, yz = Y / Z;
    const int cx_clamped = xz < -limx || xz > limx;
    const int cy_clamped = yz < -limy || yz > limy;
    const double txz = fmin(fmax(xz, -limx), limx);
    const double tyz = fmin(fmax(yz, -limy), limy);
    const double J[6] = {fx / Z, 0.0, -fx * txz / Z, 0.0, fy / Z, -fy * tyz / Z};
    double M[6];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 3; ++c)
        M[3 * r + c] = J[3 * r + 0] * Wm[0 * 4 + c] + J[3 * r + 1] * Wm[1 * 4 + c] + J[3 * r + 2] * Wm[2 * 4 + c];
    double S2[4];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c) {
        double acc = 0.0;
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) acc += M[3 * r + a] * Sig[3 * a + b] * M[3 * c + b];
        S2[2 * r + c] = acc;
      }
    const double A = S2[0] + lowpass, B = S2[1], D = S2[3] + lowpass;
    const double det = A * D - B * B;

    /* ---- conic (a, b, c) = (D, -B, A) / det  ->  (A, B, D) ---- */
    const double ga = g_conic[3 * i], gb = g_conic[3 * i + 1], gc = g_conic[3 * i + 2];
    const double d2 = det * det;
    /* partials of det: dA = D, dB = -2B, dD = A */
    const double gA = ga * (-D * D / d2) + gb * (B * D / d2) + gc * (1.0 / det - A * D / d2);
    const double gD = ga * (1.0 / det - D * A / d2) + gb * (B * A / d2) + gc * (-A * A / d2);
    const double gB = ga * (2.0 * B * D / d2) + gb * (-1.0 / det - 2.0 * B * B / d2) + gc * (2.0 * A * B / d2);
    /* Sigma2 = M Sigma M^T; symmetric upstream G with the off-diagonal shared */
    const double G[4] = {gA, 0.5 * gB, 0.5 * gB, gD};
    double gSig[9];                                      /* M^T G M */
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double acc = 0.0;
        for (int r = 0; r < 2; ++r)
          for (int c = 0; c < 2; ++c) acc += M[3 * r + a] * G[2 * r + c] * M[3 * c + b];
        gSig[3 * a + b] = acc;
      }
    double gM[6];                                        /* 2 G M Sigma */
    for (int r = 0; r < 2; ++r)
      for (int b = 0; b < 3; ++b) {
        double acc = 0.0;
        for (int c = 0; c < 2; ++c)
          for (int a = 0; a < 3; ++a) acc += G[2 * r + c] * M[3 * c + a] * Sig[3 * a + b];
        gM[3 * r + b] = 2.0 * acc;
      }
    double gJ[6];                                        /* gM Rview^T */
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 3; ++c)
        gJ[3 * r + c] = gM[3 * r + 0] * Wm[c * 4 + 0] + gM[3 * r + 1] * Wm[c * 4 + 1] + gM[3 * r + 2] * Wm[c * 4 + 2];

    /* ---- camera-space position gradient ---- */
    double gX = 0.0, gY = 0.0, gZ = 0.0;
    /* mean2d = (fx X/Z + cx, fy Y/Z + cy) */
    gX += g_mean2d[2 * i] * fx / Z;
    gY += g_mean2d[2 * i + 1] * fy / Z;
    gZ += -g_mean2d[2 * i] * fx * X / (Z * Z) - g_mean2d[2 * i + 1] * fy * Y / (Z * Z);
    /* J00 = fx/Z, J11 = fy/Z */
    gZ += gJ[0] * (-fx / (Z * Z)) + gJ[4] * (-fy / (Z * Z));
    /* J02 = -fx * clamp(X/Z) / Z */
    if (cx_clamped) gZ += gJ[2] * fx * txz / (Z * Z);
    else { gX += gJ[2] * (-fx / (Z * Z)); gZ += gJ[2] * 2.0 * fx * X / (Z * Z * Z); }
    if (cy_clamped) gZ += gJ[5] * fy * tyz / (Z * Z);
    else { gY += gJ[5] * (-fy / (Z * Z)); gZ += gJ[5] * 2.0 * fy * Y / (Z * Z * Z); }
    /* t_c = Rview mu + t */
    for (int a = 0; a < 3; ++a) d_means[3 * i + a] += Wm[0 * 4 + a] * gX + Wm[1 * 4 + a] * gY + Wm[2 * 4 + a] * gZ;

    /* ---- Sigma = Rq diag(s^2) Rq^T ---- */
    double RtGR[9];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double acc = 0.0;
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c) acc += Rq[3 * r + a] * gSig[3 * r + c] * Rq[3 * c + b];
        RtGR[3 * a + b] = acc;
      }
    for (int k = 0; k < 3; ++k) d_scales[3 * i + k] += 2.0 * s[k] * RtGR[4 * k];
    double gR[9];                                        /* 2 gSig Rq diag(s^2) */
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) {
        double acc = 0.0;
        for (int c = 0; c < 3; ++c) acc += gSig[3 * r + c] * Rq[3 * c + k];
        gR[3 * r + k] = 2.0 * acc * s[k] * s[k];
      }
    double dR[9][4];
    quat_to_rot_jac(qu, dR);
    double gqu[4] = {0.0, 0.0, 0.0, 0.0};
    for (int e = 0; e < 9; ++e)
      for (int a = 0; a < 4; ++a) gqu[a] += gR[e] * dR[e][a];
    const double dotq = gqu[0] * qu[0] + gqu[1] * qu[1] + gqu[2] * qu[2] + gqu[3] * qu[3];
    for (int a = 0; a < 4; ++a) d_quats[4 * i + a] += (gqu[a] - qu[a] * dotq) / qn;

    /* ---- colour ---- */
    double v[3] = {mu[0] - campos[0], mu[1] - campos[1], mu[2] - campos[2]};
    const double vn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    const double dir[3] = {v[0] / vn, v[1] / vn, v[2] / vn};
    double Yb[16], dY[48];
    orc_sh_eval(sh_degree, dir, Yb, dY);
    double gdir[3] = {0.0, 0.0, 0.0};
    for (int c = 0; c < 3; ++c) {
      double raw = 0.5;
      for (int k = 0; k < K; ++k) raw += Yb[k] * sh[(size_t)i * K * 3 + 3 * k + c];
      if (!(raw > 0.0)) continue;
      const double gcol = g_rgb[3 * i + c];
      for (int k = 0; k < K; ++k) {
        d_sh[(size_t)i * K * 3 + 3 * k + c] += gcol * Yb[k];
        for (int a = 0; a < 3; ++a) gdir[a] += gcol * sh[(size_t)i * K * 3 + 3 * k + c] * dY[3 * k + a];
      }
    }
    const double dd = gdir[0] * dir[0] + gdir[1] * dir[1] + gdir[2] * dir[2];
    for (int a = 0; a < 3; ++a) d_means[3 * i + a] += (gdir[a] - dir[a] * dd) / vn;
  }
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)                          */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    if (r < 9) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Three standard normals for component i at a given step: counter
 * (i, step_lo, step_hi, 0), key (seed_lo, seed_hi); uniforms
 * u = ((x >> 9) + 1/2) 2^-23 in (0, 1); Box-Muller on (u0, u1) and (u2, u3). */
void orc_normals3(uint64_t i, uint64_t seed, uint64_t step, double* z) {
  const uint32_t ctr[4] = {(uint32_t)i, (uint32_t)step, (uint32_t)(step >> 32), (uint32_t)(i >> 32)};
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t x[4];
  orc_philox4x32_10(ctr, key, x);
  double u[4];
  for (int a = 0; a < 4; ++a) u[a] = ((double)(x[a] >> 9) + 0.5) * (1.0 / 8388608.0);
  const double two_pi = 6.28318530717958647692;
  const double r0 = sqrt(-2.0 * log(u[0])), r1 = sqrt(-2.0 * log(u[2]));
  z[0] = r0 * cos(two_pi * u[1]);
  z[1] = r0 * sin(two_pi * u[1]);
  z[2] = r1 * cos(two_pi * u[3]);
}

/* ------------------------------------------------------------------------ */
/* SGHMC on the means                                                          */
/* ------------------------------------------------------------------------ */
/* Per component, with eps = lr, C = friction, switch s = sigmoid(k((1-|o|)-t))
 * (on for |o| <= 1 - t) and n ~ N(0, 2 eps C) per axis:
 *   F   = s eps (1 - eps C) r               (0 during burn-in)
 *   mu <- mu - eps^2 G + F + s eps n        (burn-in: s eps Sigma n)
 *   r  <- (1 - eps C) r - eps G + n
 * With s = 1 this is mu_{t+1} = mu_t + eps r_{t+1}, the SM's expansion. */
void orc_sghmc_step(int n, double* means, double* mom, const double* grad, const double* opac,
                    const double* scales, const double* quats, double lr, double friction,
                    double k, double t, int burn_in, int noise_on, uint64_t seed, uint64_t step) {
  for (int i = 0; i < n; ++i) {
    const double sw = 1.0 / (1.0 + exp(-k * ((1.0 - fabs(opac[i])) - t)));
    double z[3] = {0.0, 0.0, 0.0};
    if (noise_on) orc_normals3((uint64_t)i, seed, step, z);
    const double sd = sqrt(2.0 * lr * friction);
    double nz[3] = {sd * z[0], sd * z[1], sd * z[2]};
    double kick[3] = {nz[0], nz[1], nz[2]};
    if (burn_in) {
      const double* q = quats + 4 * i;
      const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
      const double qu[4] = {q[0] / qn, q[1] / qn, q[2] / qn, q[3] / qn};
      double Rq[9];
      quat_to_rot(qu, Rq);
      const double* s = scales + 3 * i;
      for (int r = 0; r < 3; ++r) {
        double acc = 0.0;
        for (int c = 0; c < 3; ++c) {
          double sig = 0.0;
          for (int m = 0; m < 3; ++m) sig += Rq[3 * r + m] * s[m] * s[m] * Rq[3 * c + m];
          acc += sig * nz[c];
        }
        kick[r] = acc;
      }
    }
    for (int a = 0; a < 3; ++a) {
      const double r = mom[3 * i + a], G = grad[3 * i + a];
      const double F = burn_in ? 0.0 : sw * lr * (1.0 - lr * friction) * r;
      means[3 * i + a] = means[3 * i + a] - lr * lr * G + F + sw * lr * kick[a];
      mom[3 * i + a] = (1.0 - lr * friction) * r - lr * G + nz[a];
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Adam (Kingma & Ba) with an optional box [lo, hi]                            */
/* ------------------------------------------------------------------------ */
void orc_adam_step(int64_t count, double* param, const double* grad, double* m, double* v,
                   double lr, double b1, double b2, double eps, int64_t t, double lo, double hi) {
  const double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
  for (int64_t j = 0; j < count; ++j) {
    m[j] = b1 * m[j] + (1.0 - b1) * grad[j];
    v[j] = b2 * v[j] + (1.0 - b2) * grad[j] * grad[j];
    const double mh = m[j] / c1, vh = v[j] / c2;
    double p = param[j] - lr * mh / (sqrt(vh) + eps);
    if (p < lo) p = lo;
    if (p > hi) p = hi;
    param[j] = p;
  }
}

/* ------------------------------------------------------------------------ */
/* Recycling (Sec. 3.4 eq. relocation, SM "Component Recycling")              */
/* ------------------------------------------------------------------------ */
/* ln beta(x, y) through ln Gamma (SM eq. beta4). */
double orc_lnbeta(double x, double y) { return lgamma(x) + lgamma(y) - lgamma(x + y); }

/* N components placed at one old component's mean reproduce, in the 1D
 * integral of the composited opacity, the old component: the new opacity
 * from (1 - o_new)^N = 1 - |o_old| and the covariance scale factor
 *   Sigma_new / Sigma_old = o_old^2 (nu_old / nu_new) (beta(1/2, (nu_old+2)/2) / K)^2
 *   K = sum_{i=1..N} sum_{k=0..i-1} C(i-1, k) (-1)^k o_new^(k+1) beta(1/2, ((k+1)(nu_new+3)-1)/2).
 * The sign of the new opacity is the sign of o_old. */
void orc_relocate(double o_old, double nu_old, double nu_new, int N, double* o_new, double* factor) {
  const double a = fabs(o_old);
  const double on = 1.0 - pow(1.0 - a, 1.0 / (double)N);
  double K = 0.0;
  for (int i = 1; i <= N; ++i) {
    double binom = 1.0;                                /* C(i-1, k) */
    for (int k = 0; k <= i - 1; ++k) {
      const double term = binom * ((k % 2) ? -1.0 : 1.0) * pow(on, (double)(k + 1)) *
                          exp(orc_lnbeta(0.5, ((k + 1) * (nu_new + 3.0) - 1.0) / 2.0));
      K += term;
      binom = binom * (double)(i - 1 - k) / (double)(k + 1);
    }
  }
  const double b_old = exp(orc_lnbeta(0.5, (nu_old + 2.0) / 2.0));
  *o_new = o_old < 0.0 ? -on : on;
  *factor = a * a * (nu_old / nu_new) * (b_old / K) * (b_old / K);
}

/* One recycling step over a whole scene (Sec. 3.4 "Adding and Recycling
 * Components"; SM "Component Recycling"), the oracle of sss_relocate:
 *  1. dead = |o| <= dead_opacity, taken in index order, at most
 *     floor(n * max_fraction) of them;
 *  2. targets from a multinomial over the live components with integer
 *     weights w_i = floor(|o_i| 2^24) (exact, so the draw is reproducible
 *     bit for bit): draw j uses Philox4x32-10 with key (seed lo, seed hi) and
 *     counter (j lo, step lo, step hi, 2^31 | j hi); r = (x1 << 32) | x0 and the
 *     drawn weight position is floor(r * W / 2^64), W = sum of weights; the
 *     target is the component whose weight interval contains it;
 *  3. a target drawn m times ends with N = m + 1 components at its mean: the
 *     moved ones copy its mean, rotation, nu and SH, all N get the opacity and
 *     covariance factor of orc_relocate (nu_new = nu_old, scales multiplied
 *     by sqrt(factor)), and the moved ones' optimiser state is reset.
 * Writes target[j] for the moved components (dead[j] -> target[j]); returns
 * the number moved.  state/state_width: per-component rows zeroed for moved
 * components (momentum, Adam moments). */
int64_t orc_relocate_step(int64_t n, int sh_degree, double* means, double* scales, double* quats, double* nu,
                          double* opac, double* sh, double dead_opacity, double max_fraction, uint64_t seed,
                          uint64_t step, int n_state, double** state, const int* state_width,
                          int64_t* dead_out, int64_t* target_out) {
  const int K3 = 3 * (sh_degree + 1) * (sh_degree + 1);
  const int64_t cap = (int64_t)floor((double)n * max_fraction);
  int64_t nd = 0;
  for (int64_t i = 0; i < n && nd < cap; ++i)
    if (fabs((float)opac[i]) <= (float)dead_opacity) dead_out[nd++] = i;
  uint64_t* excl = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n + 1));
  uint64_t W = 0;
  for (int64_t i = 0; i < n; ++i) {
    excl[i] = W;
    const float a = fabsf((float)opac[i]);
    if (!(a <= (float)dead_opacity)) W += (uint64_t)floorf(a * 16777216.0f);
  }
  excl[n] = W;
  if (W == 0 || nd == 0) { free(excl); return 0; }
  int32_t* m = (int32_t*)calloc((size_t)n, sizeof(int32_t));
  for (int64_t j = 0; j < nd; ++j) {
    const uint32_t ctr[4] = {(uint32_t)j, (uint32_t)step, (uint32_t)(step >> 32), 0x80000000u | (uint32_t)(j >> 32)};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    const uint64_t r = ((uint64_t)x[1] << 32) | x[0];
    const uint64_t pos = (uint64_t)(((unsigned __int128)r * W) >> 64);
    int64_t lo = 0, hi = n;                       /* last t with excl[t] <= pos */
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) / 2;
      if (excl[mid] <= pos) lo = mid; else hi = mid;
    }
    target_out[j] = lo;
    m[lo] += 1;
  }
  /* moved components copy the (old) target, with the new opacity and scale */
  for (int64_t j = 0; j < nd; ++j) {
    const int64_t d = dead_out[j], t = target_out[j];
    const double nut = fmin(fmax(nu[t], 1.0), 1e4);
    double on, f;
    orc_relocate(opac[t], nut, nut, m[t] + 1, &on, &f);
    for (int a = 0; a < 3; ++a) { means[3 * d + a] = means[3 * t + a]; scales[3 * d + a] = scales[3 * t + a] * sqrt(f); }
    for (int a = 0; a < 4; ++a) quats[4 * d + a] = quats[4 * t + a];
    nu[d] = nu[t];
    opac[d] = on;
    for (int a = 0; a < K3; ++a) sh[(size_t)d * K3 + a] = sh[(size_t)t * K3 + a];
    for (int s = 0; s < n_state; ++s)
      for (int a = 0; a < state_width[s]; ++a) state[s][(size_t)d * state_width[s] + a] = 0.0;
  }
  for (int64_t t = 0; t < n; ++t) {
    if (!m[t]) continue;
    const double nut = fmin(fmax(nu[t], 1.0), 1e4);
    double on, f;
    orc_relocate(opac[t], nut, nut, m[t] + 1, &on, &f);
    opac[t] = on;
    for (int a = 0; a < 3; ++a) scales[3 * t + a] *= sqrt(f);
  }
  free(m);
  free(excl);
  return nd;
}
