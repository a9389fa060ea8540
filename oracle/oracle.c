/*
 * oracle.c -- plain, slow FP64 CPU reference solver ("the oracle") for the 3D
 * Newtonian adiabatic finite-volume hydro update of AthenaK (Stone et al.
 * 2024, arXiv:2409.16053).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or
 * call this file. Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it. It shares no source with the GPU path.
 *
 * What it computes, in the paper's order (Sec. 3, "reconstruct, solve, and
 * advance"):
 *   ghost-zone fill (Sec. 2, boundary conditions)
 *   -> conserved to primitive, W = [rho, v, u_g], p = (gamma-1) u_g (Sec. 3.1, Eq. 4)
 *   -> reconstruction on primitives, PLM, PPM4, PPMX or WENO-Z (Sec. 3)
 *   -> HLLC Riemann fluxes in x, y and z (Sec. 3; Toro's textbook, Ch. 10)
 *   -> flux divergence and a low-storage SSP-RK stage (Sec. 3, method of lines;
 *      RK1, RK2, RK3 or the ten-stage fourth-order RK4)
 *   -> optionally, first-order flux correction with LLF fluxes (Sec. 3, FOFC)
 *   -> CFL time step, Eq. 3: CFL times the minimum over all cells and all
 *      dimensions of dx_d / lambda_max,d.
 * It works on the whole mesh with no MeshBlock decomposition: splitting the
 * mesh into blocks changes no per-cell arithmetic. The or_smr_* functions at
 * the end take a mesh with a statically refined box of blocks (two levels,
 * Sec. 2); there each leaf block is ghost-filled and updated on its own.
 *
 * Readings where the paper is silent (each is listed with its reason in the
 * design notes): PLM uses the van Leer harmonic-mean limiter; PPM4 is
 * Colella & Woodward (1984) Eqs. 1.6-1.10 without steepening or flattening;
 * WENO-Z uses the Jiang-Shu smoothness indicators with the squared WENO-Z
 * weights of Borges et al. (2008); PPMX uses the extremum-preserving limiters
 * of Colella & Sekora (2008); LLF is Rusanov's flux; FOFC replaces the fluxes
 * on all faces of a cell whose stage result has rho or p <= 0;
 * the reconstructed energy variable is u_g; HLLC is Toro-Spruce-Speares with
 * PVRS pressure-based wave speeds; RK2 is SSPRK(2,2) and RK3 SSPRK(3,3) of
 * Shu & Osher, both in two-register low-storage form;
 * lambda_d = |v_d| + c_s; floors act on W only and never change U; outflow is
 * a zero-gradient copy of U.
 *
 * Plain loops, FP64, compiled with -ffp-contract=off. Optional OpenMP over
 * k-planes: every cell's arithmetic is independent of the thread count and
 * the time-step minimum is exact, so results do not depend on it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_PERIODIC = 0, OR_OUTFLOW = 1 };
enum { OR_PLM = 0, OR_PPM4 = 1, OR_WENOZ = 2, OR_PPMX = 3 };
enum { OR_OK = 0, OR_ERR_ARG = 1, OR_ERR_NOMEM = 2, OR_ERR_STATE = 4 };

/* Problem description passed from Python (ctypes mirror in oracle/__init__.py). */
typedef struct {
  int32_t n[3];      /* interior cells nx, ny, nz                      */
  int32_t bc[3][2];  /* per axis (lower, upper): OR_PERIODIC/OR_OUTFLOW */
  int32_t recon;     /* OR_PLM (2 ghosts), OR_PPM4/WENOZ/PPMX (3)      */
  int32_t fofc;      /* 1: first-order flux correction in every stage  */
  int32_t rk;        /* stages of the SSP-RK integrator: 1, 2 or 3     */
  double dx[3];      /* cell widths                                    */
  double gamma;      /* ratio of specific heats, > 1                   */
  double cfl;        /* Courant number                                 */
  double rho_floor;  /* density floor applied to W                     */
  double p_floor;    /* pressure floor applied to W                    */
} or_params;

/* A stored array with ghosts: [5][nz+2g][ny+2g][nx+2g]. */
typedef struct {
  int n[3];
  int g;
  int s[3];      /* stored extent per axis */
  size_t sv;     /* stride of one variable */
} grid;

static void grid_init(grid* G, const or_params* p, int g) {
  for (int d = 0; d < 3; ++d) { G->n[d] = p->n[d]; G->s[d] = p->n[d] + 2 * g; }
  G->g = g;
  G->sv = (size_t)G->s[0] * G->s[1] * G->s[2];
}

/* index of variable v at cell (i,j,k); i,j,k in [-g, n+g) */
static size_t at(const grid* G, int v, int i, int j, int k) {
  return (size_t)v * G->sv +
         ((size_t)(k + G->g) * G->s[1] + (size_t)(j + G->g)) * G->s[0] + (size_t)(i + G->g);
}

int or_nghost(int recon) { return recon == OR_PLM ? 2 : 3; }

void or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int or_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------
 * Ghost zones (Sec. 2, boundary conditions are applied through ghost cells).
 * Periodic: the cell one period away. Outflow: the nearest interior cell
 * (zero gradient). The x faces are filled first over the interior (j,k),
 * then y over all i, then z over all (i,j), so edge and corner ghosts end up
 * filled too, although the dimension-by-dimension stencil never reads them.
 * ---------------------------------------------------------------------- */
static int src_index(int c, int n, int bclo, int bchi) {
  if (c < 0) return bclo == OR_PERIODIC ? ((c % n) + n) % n : 0;
  if (c >= n) return bchi == OR_PERIODIC ? c % n : n - 1;
  return c;
}

static void fill_ghosts(const or_params* p, const grid* G, double* U) {
  const int g = G->g, nx = G->n[0], ny = G->n[1], nz = G->n[2];
  for (int v = 0; v < 5; ++v) {
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = -g; i < nx + g; ++i) {
          if (i >= 0 && i < nx) continue;
          int si = src_index(i, nx, p->bc[0][0], p->bc[0][1]);
          U[at(G, v, i, j, k)] = U[at(G, v, si, j, k)];
        }
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
      for (int j = -g; j < ny + g; ++j) {
        if (j >= 0 && j < ny) continue;
        int sj = src_index(j, ny, p->bc[1][0], p->bc[1][1]);
        for (int i = -g; i < nx + g; ++i) U[at(G, v, i, j, k)] = U[at(G, v, i, sj, k)];
      }
#pragma omp parallel for schedule(static)
    for (int k = -g; k < nz + g; ++k) {
      if (k >= 0 && k < nz) continue;
      int sk = src_index(k, nz, p->bc[2][0], p->bc[2][1]);
      for (int j = -g; j < ny + g; ++j)
        for (int i = -g; i < nx + g; ++i) U[at(G, v, i, j, k)] = U[at(G, v, i, j, sk)];
    }
  }
}

/* ------------------------------------------------------------------------
 * Conserved -> primitive (Sec. 3.1, Eq. 4): rho; v = M / rho;
 * u_g = E - |M|^2 / (2 rho). Floors act on W only: rho below rho_floor is
 * raised to it (and used for v and u_g), u_g below p_floor/(gamma-1) is raised
 * to it. Returns 1 if a floor fired. *bad is set when U is non-finite or
 * rho <= 0 (an unrecoverable state).
 * ---------------------------------------------------------------------- */
int or_c2p(const or_params* p, const double u[5], double w[5], int* bad) {
  int hit = 0;
  double rho = u[0];
  if (bad) {
    int b = 0;
    for (int q = 0; q < 5; ++q) b |= !isfinite(u[q]);
    b |= !(rho > 0.0);
    *bad = b;
  }
  if (rho < p->rho_floor) { rho = p->rho_floor; hit = 1; }
  double ke2 = u[1] * u[1] + u[2] * u[2] + u[3] * u[3];
  double ug = u[4] - 0.5 * ke2 / rho;
  double ufloor = p->p_floor / (p->gamma - 1.0);
  if (ug < ufloor) { ug = ufloor; hit = 1; }
  w[0] = rho;
  w[1] = u[1] / rho;
  w[2] = u[2] / rho;
  w[3] = u[3] / rho;
  w[4] = ug;
  return hit;
}

/* ------------------------------------------------------------------------
 * Reconstruction (Sec. 3: always on primitive variables).
 * ---------------------------------------------------------------------- */

/* PLM: van Leer harmonic-mean limited slope of a cell from its neighbours;
 * the cell's left and right face values are w0 -/+ slope/2. */
void or_plm_cell(double wm, double w0, double wp, double* left, double* right) {
  double dl = w0 - wm, dr = wp - w0;
  double prod = dl * dr;
  double slope = prod > 0.0 ? 2.0 * prod / (dl + dr) : 0.0;
  *left = w0 - 0.5 * slope;
  *right = w0 + 0.5 * slope;
}

/* PPM4 monotonised central slope (Colella & Woodward 1984, Eq. 1.8). */
static double cw_slope(double wm, double w0, double wp) {
  double dl = w0 - wm, dr = wp - w0;
  if (!(dl * dr > 0.0)) return 0.0;
  double da = 0.5 * (wp - wm);
  double m = fabs(da);
  if (2.0 * fabs(dl) < m) m = 2.0 * fabs(dl);
  if (2.0 * fabs(dr) < m) m = 2.0 * fabs(dr);
  return copysign(m, da);
}

/* PPM4 interface value between cells c and c+1 (CW84 Eq. 1.6, uniform mesh). */
static double cw_interface(double wc, double wc1, double sc, double sc1) {
  return wc + 0.5 * (wc1 - wc) - (sc1 - sc) / 6.0;
}

/* PPM4 face values of cell c from w[0..4] = cells c-2..c+2: interface values
 * on both sides, then the monotonicity constraints of CW84 Eq. 1.10. */
void or_ppm4_cell(const double w[5], double* left, double* right) {
  double s_m = cw_slope(w[0], w[1], w[2]);
  double s_0 = cw_slope(w[1], w[2], w[3]);
  double s_p = cw_slope(w[2], w[3], w[4]);
  double aL = cw_interface(w[1], w[2], s_m, s_0);
  double aR = cw_interface(w[2], w[3], s_0, s_p);
  double a = w[2];
  if ((aR - a) * (a - aL) <= 0.0) {
    aL = a;
    aR = a;
  } else {
    double d = aR - aL;
    double m6 = d * (a - 0.5 * (aL + aR));
    double d26 = d * d / 6.0;
    if (m6 > d26) aL = 3.0 * a - 2.0 * aR;
    else if (-d26 > m6) aR = 3.0 * a - 2.0 * aL;
  }
  *left = aL;
  *right = aR;
}

/* ------------------------------------------------------------------------
 * WENO-Z (Sec. 3 names the improved WENO-Z of Acker et al. 2016 and defers
 * its details). Fifth-order weighted combination of the three third-order
 * candidate values of the face, with the Jiang-Shu smoothness indicators
 * beta_k, the global indicator tau5 = |beta_0 - beta_2| and the WENO-Z
 * weights alpha_k = d_k (1 + (tau5 / (beta_k + eps))^2), linear weights
 * d = (1/10, 6/10, 3/10) (Borges et al. 2008). The ratio is capped at 1e15,
 * which keeps the weights finite in single precision and changes them only
 * where one candidate already has weight 1 to within 1e-30.
 * ---------------------------------------------------------------------- */
#define OR_WENO_EPS 1e-36
#define OR_WENO_CAP 1e15

/* value at the right face of the middle cell of w[0..4] (cells c-2..c+2) */
static double weno_right(const double w[5]) {
  const double b0 = 13.0 / 12.0 * (w[0] - 2.0 * w[1] + w[2]) * (w[0] - 2.0 * w[1] + w[2]) +
                    0.25 * (w[0] - 4.0 * w[1] + 3.0 * w[2]) * (w[0] - 4.0 * w[1] + 3.0 * w[2]);
  const double b1 = 13.0 / 12.0 * (w[1] - 2.0 * w[2] + w[3]) * (w[1] - 2.0 * w[2] + w[3]) +
                    0.25 * (w[1] - w[3]) * (w[1] - w[3]);
  const double b2 = 13.0 / 12.0 * (w[2] - 2.0 * w[3] + w[4]) * (w[2] - 2.0 * w[3] + w[4]) +
                    0.25 * (3.0 * w[2] - 4.0 * w[3] + w[4]) * (3.0 * w[2] - 4.0 * w[3] + w[4]);
  const double beta[3] = {b0, b1, b2};
  const double d[3] = {0.1, 0.6, 0.3};
  /* candidates minus the cell value: (2 w0 - 7 w1 + 11 w2)/6, (-w1 + 5 w2 + 2 w3)/6
   * and (2 w2 + 5 w3 - w4)/6, written in differences so that a constant
   * state is reproduced exactly */
  const double dq[3] = {(2.0 * (w[0] - w[1]) - 5.0 * (w[1] - w[2])) / 6.0,
                        (2.0 * (w[3] - w[2]) - (w[1] - w[2])) / 6.0,
                        (4.0 * (w[3] - w[2]) - (w[4] - w[3])) / 6.0};
  const double tau = fabs(b0 - b2);
  double num = 0.0, den = 0.0;
  for (int k = 0; k < 3; ++k) {
    double r = tau / (beta[k] + OR_WENO_EPS);
    if (r > OR_WENO_CAP) r = OR_WENO_CAP;
    const double a = d[k] * (1.0 + r * r);
    num += a * dq[k];
    den += a;
  }
  return w[2] + num / den;
}

/* WENO-Z face values of cell c from w[0..4] = cells c-2..c+2; the left face
 * is the right-face formula applied to the mirrored stencil. */
void or_wenoz_cell(const double w[5], double* left, double* right) {
  const double m[5] = {w[4], w[3], w[2], w[1], w[0]};
  *right = weno_right(w);
  *left = weno_right(m);
}

/* ------------------------------------------------------------------------
 * PPMX: PPM with the extremum-preserving limiters of Colella & Sekora (2008)
 * as used by McCorquodale & Colella (Sec. 3 names them, without formulas).
 * A limited second difference keeps the sign of all its arguments and the
 * smallest magnitude among them, the neighbouring second differences
 * weighted by C = 1.25; it is 0 if the signs differ.
 *  1. Fourth-order interface value between b and c (neighbours a, d):
 *     7/12 (b + c) - 1/12 (a + d), evaluated in differences.
 *  2. If that value f lies outside [b, c], it is replaced by
 *     (b + c)/2 - D/6, D the limited second difference of 3 (b - 2f + c),
 *     with neighbours a - 2b + c and b - 2c + d.
 *  3. Cell w_i with edges aL, aR, dm = w_i - aL, dp = aR - w_i. At an
 *     extremum (dm dp <= 0, or the cell average itself is a local extremum)
 *     the parabola's curvature 6 (aL + aR - 2 w_i) is limited against the
 *     centred and the two one-sided second differences of the cell averages,
 *     and both edge offsets are scaled by limited / unlimited curvature (0 if
 *     the curvature is 0). Elsewhere the usual PPM overshoot test applies:
 *     an edge offset larger than twice the other is cut to twice it.
 * ---------------------------------------------------------------------- */
#define OR_PPMX_C 1.25

static double lim2(int n, const double* x) {
  /* x[0] is the second difference to limit; x[1..n-1] its neighbours */
  int pos = 1, neg = 1;
  for (int q = 0; q < n; ++q) {
    pos &= x[q] > 0.0;
    neg &= x[q] < 0.0;
  }
  if (!pos && !neg) return 0.0;
  double m = fabs(x[0]);
  for (int q = 1; q < n; ++q)
    if (OR_PPMX_C * fabs(x[q]) < m) m = OR_PPMX_C * fabs(x[q]);
  return pos ? m : -m;
}

/* limited interface value between b and c, neighbours a and d; the
 * fourth-order value 7/12 (b + c) - 1/12 (a + d) is written as
 * (b + c)/2 - ((a - b) + (d - c))/12 so that a constant state is reproduced
 * exactly (otherwise rounding puts f just outside [b, b] and the limiter's
 * branch is decided by rounding) */
static double ppmx_interface(double a, double b, double c, double d) {
  double f = 0.5 * (b + c) - ((a - b) + (d - c)) / 12.0;
  if ((f - b) * (c - f) < 0.0) {
    const double x[3] = {3.0 * (b - 2.0 * f + c), a - 2.0 * b + c, b - 2.0 * c + d};
    f = 0.5 * (b + c) - lim2(3, x) / 6.0;
  }
  return f;
}

/* PPMX face values of cell c from w[0..4] = cells c-2..c+2 */
void or_ppmx_cell(const double w[5], double* left, double* right) {
  double aL = ppmx_interface(w[0], w[1], w[2], w[3]);
  double aR = ppmx_interface(w[1], w[2], w[3], w[4]);
  const double a = w[2];
  const double dm = a - aL, dp = aR - a;
  if (dm * dp <= 0.0 || (w[3] - a) * (a - w[1]) <= 0.0) {
    const double d2 = 6.0 * (aL + aR - 2.0 * a);
    const double x[4] = {d2, w[1] - 2.0 * a + w[3], w[0] - 2.0 * w[1] + a, a - 2.0 * w[3] + w[4]};
    const double ratio = d2 != 0.0 ? lim2(4, x) / d2 : 0.0;
    aL = a - ratio * dm;
    aR = a + ratio * dp;
  } else {
    if (fabs(dp) >= 2.0 * fabs(dm)) aR = a + 2.0 * dm;
    if (fabs(dm) >= 2.0 * fabs(dp)) aL = a - 2.0 * dp;
  }
  *left = aL;
  *right = aR;
}

/* ------------------------------------------------------------------------
 * HLLC Riemann solver (Sec. 3 names HLLC; the Toro-Spruce-Speares solver of
 * Toro's textbook Ch. 10 with PVRS pressure-based wave-speed estimates).
 * States are primitive [rho, u_n, u_t1, u_t2, p]; the flux is
 * [mass, normal momentum, t1 momentum, t2 momentum, energy].
 * ---------------------------------------------------------------------- */
void or_hllc(double gamma, const double wl[5], const double wr[5], double f[5]) {
  const double rl = wl[0], ul = wl[1], vl = wl[2], zl = wl[3], pl = wl[4];
  const double rr = wr[0], ur = wr[1], vr = wr[2], zr = wr[3], pr = wr[4];
  const double gm1 = gamma - 1.0;
  const double el = pl / gm1 + 0.5 * rl * (ul * ul + vl * vl + zl * zl);
  const double er = pr / gm1 + 0.5 * rr * (ur * ur + vr * vr + zr * zr);
  const double al = sqrt(gamma * pl / rl), ar = sqrt(gamma * pr / rr);

  /* PVRS estimate of the star pressure, clipped at zero */
  double ppv = 0.5 * (pl + pr) - 0.5 * (ur - ul) * (0.5 * (rl + rr)) * (0.5 * (al + ar));
  double ps = ppv > 0.0 ? ppv : 0.0;
  double ql = ps <= pl ? 1.0 : sqrt(1.0 + (gamma + 1.0) / (2.0 * gamma) * (ps / pl - 1.0));
  double qr = ps <= pr ? 1.0 : sqrt(1.0 + (gamma + 1.0) / (2.0 * gamma) * (ps / pr - 1.0));
  double sl = ul - al * ql, sr = ur + ar * qr;
  double sstar = (pr - pl + rl * ul * (sl - ul) - rr * ur * (sr - ur)) /
                 (rl * (sl - ul) - rr * (sr - ur));

  double fl[5] = {rl * ul, rl * ul * ul + pl, rl * ul * vl, rl * ul * zl, ul * (el + pl)};
  double fr[5] = {rr * ur, rr * ur * ur + pr, rr * ur * vr, rr * ur * zr, ur * (er + pr)};

  /* selection and tie-breaks: S_L >= 0 -> F_L; S* >= 0 -> F*_L;
   * S_R > 0 -> F*_R; otherwise F_R */
  if (sl >= 0.0) {
    memcpy(f, fl, sizeof fl);
    return;
  }
  if (!(sstar >= 0.0) && !(sr > 0.0)) {
    memcpy(f, fr, sizeof fr);
    return;
  }
  /* star state on the side of the contact that holds the face */
  const int left = sstar >= 0.0;
  const double rk = left ? rl : rr, uk = left ? ul : ur, vk = left ? vl : vr;
  const double zk = left ? zl : zr, pk = left ? pl : pr, ek = left ? el : er;
  const double sk = left ? sl : sr;
  const double* fk = left ? fl : fr;
  double fac = rk * (sk - uk) / (sk - sstar);
  double us[5];
  us[0] = fac;
  us[1] = fac * sstar;
  us[2] = fac * vk;
  us[3] = fac * zk;
  us[4] = fac * (ek / rk + (sstar - uk) * (sstar + pk / (rk * (sk - uk))));
  double uk5[5] = {rk, rk * uk, rk * vk, rk * zk, ek};
  for (int q = 0; q < 5; ++q) f[q] = fk[q] + sk * (us[q] - uk5[q]);
}

/* ------------------------------------------------------------------------
 * Local Lax-Friedrichs (Rusanov) flux (Sec. 3 names LLF; Toro's textbook):
 * the mean of the two physical fluxes minus half the largest local signal
 * speed a = max(|u_L| + c_L, |u_R| + c_R) times the jump in U. Same state and
 * flux ordering as or_hllc.
 * ---------------------------------------------------------------------- */
void or_llf(double gamma, const double wl[5], const double wr[5], double f[5]) {
  const double gm1 = gamma - 1.0;
  double ul[5], ur[5], fl[5], fr[5];
  const double* w[2] = {wl, wr};
  double* uu[2] = {ul, ur};
  double* ff[2] = {fl, fr};
  double a = 0.0;
  for (int s = 0; s < 2; ++s) {
    const double r = w[s][0], un = w[s][1], v1 = w[s][2], v2 = w[s][3], pr = w[s][4];
    const double e = pr / gm1 + 0.5 * r * (un * un + v1 * v1 + v2 * v2);
    uu[s][0] = r;
    uu[s][1] = r * un;
    uu[s][2] = r * v1;
    uu[s][3] = r * v2;
    uu[s][4] = e;
    ff[s][0] = r * un;
    ff[s][1] = r * un * un + pr;
    ff[s][2] = r * un * v1;
    ff[s][3] = r * un * v2;
    ff[s][4] = un * (e + pr);
    const double sp = fabs(un) + sqrt(gamma * pr / r);
    if (sp > a) a = sp;
  }
  for (int q = 0; q < 5; ++q) f[q] = 0.5 * (fl[q] + fr[q]) - 0.5 * a * (ur[q] - ul[q]);
}

/* ------------------------------------------------------------------------
 * One stage's flux divergence L(U) on interior cells (method of lines).
 * ---------------------------------------------------------------------- */
typedef struct {
  grid G;          /* ghosted state / primitive arrays */
  double* U;       /* ghosted conserved state          */
  double* W;       /* ghosted primitives (rho, v, u_g) */
  double* F[3];    /* face fluxes per direction        */
  double* L;       /* divergence, interior [5][nz][ny][nx] */
  size_t fsv[3];   /* flux variable strides            */
} work;

static size_t ncell(const or_params* p) { return (size_t)p->n[0] * p->n[1] * p->n[2]; }

static size_t lin(const or_params* p, int i, int j, int k) {
  return ((size_t)k * p->n[1] + j) * p->n[0] + i;
}

static int work_alloc(work* w, const or_params* p) {
  memset(w, 0, sizeof *w);
  grid_init(&w->G, p, or_nghost(p->recon));
  size_t st = 5 * w->G.sv;
  w->U = malloc(st * sizeof(double));
  w->W = malloc(st * sizeof(double));
  w->L = malloc(5 * ncell(p) * sizeof(double));
  for (int d = 0; d < 3; ++d) {
    size_t nf = (size_t)(p->n[0] + (d == 0)) * (p->n[1] + (d == 1)) * (p->n[2] + (d == 2));
    w->fsv[d] = nf;
    w->F[d] = malloc(5 * nf * sizeof(double));
  }
  if (!w->U || !w->W || !w->L || !w->F[0] || !w->F[1] || !w->F[2]) return OR_ERR_NOMEM;
  return OR_OK;
}

static void work_free(work* w) {
  free(w->U); free(w->W); free(w->L);
  for (int d = 0; d < 3; ++d) free(w->F[d]);
}

/* Face states along direction d for the face between cells c-1 and c at
 * transverse position (i,j,k) with the normal index replaced by c. */
static void face_states(const or_params* p, const work* w, int d, int i, int j, int k,
                        double wl[5], double wr[5]) {
  const grid* G = &w->G;
  const int di = d == 0, dj = d == 1, dk = d == 2;
  for (int v = 0; v < 5; ++v) {
    double s[6];
    if (p->recon == OR_PLM) {
      for (int o = -2; o <= 1; ++o) s[o + 2] = w->W[at(G, v, i + o * di, j + o * dj, k + o * dk)];
      double l0, r0, l1, r1;
      or_plm_cell(s[0], s[1], s[2], &l0, &r0); /* cell c-1 */
      or_plm_cell(s[1], s[2], s[3], &l1, &r1); /* cell c   */
      wl[v] = r0;
      wr[v] = l1;
    } else {
      for (int o = -3; o <= 2; ++o) s[o + 3] = w->W[at(G, v, i + o * di, j + o * dj, k + o * dk)];
      double l0, r0, l1, r1;
      if (p->recon == OR_PPM4) {
        or_ppm4_cell(&s[0], &l0, &r0); /* cell c-1: cells c-3..c+1 */
        or_ppm4_cell(&s[1], &l1, &r1); /* cell c:   cells c-2..c+2 */
      } else if (p->recon == OR_PPMX) {
        or_ppmx_cell(&s[0], &l0, &r0);
        or_ppmx_cell(&s[1], &l1, &r1);
      } else {
        or_wenoz_cell(&s[0], &l0, &r0);
        or_wenoz_cell(&s[1], &l1, &r1);
      }
      wl[v] = r0;
      wr[v] = l1;
    }
  }
}

/* Riemann flux at one face along d: rotate so the normal velocity comes
 * first, form p = (gamma-1) u_g, solve (HLLC, or LLF when llf != 0), rotate
 * back into (Mx, My, Mz). */
static void face_flux(const or_params* p, int d, const double wl[5], const double wr[5],
                      double out[5], int llf) {
  const int n = 1 + d, t1 = 1 + (d + 1) % 3, t2 = 1 + (d + 2) % 3;
  double ql[5] = {wl[0], wl[n], wl[t1], wl[t2], (p->gamma - 1.0) * wl[4]};
  double qr[5] = {wr[0], wr[n], wr[t1], wr[t2], (p->gamma - 1.0) * wr[4]};
  double f[5];
  if (llf) or_llf(p->gamma, ql, qr, f);
  else or_hllc(p->gamma, ql, qr, f);
  out[0] = f[0];
  out[n] = f[1];
  out[t1] = f[2];
  out[t2] = f[3];
  out[4] = f[4];
}

static void flux_divergence(const or_params* p, work* w);
static long long prims_and_fluxes(const or_params* p, work* w, int* bad);

/* L(U) for the interior state Uin[5][nz][ny][nx]. Returns floor hits on
 * interior cells; sets *bad if any interior cell is unrecoverable. */
static long long divergence(const or_params* p, work* w, const double* Uin, int* bad) {
  const grid* G = &w->G;
  const int nx = p->n[0], ny = p->n[1], nz = p->n[2];
  const size_t nc = ncell(p);

  /* copy the interior into the ghosted array, then fill the ghosts */
  for (int v = 0; v < 5; ++v) {
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) w->U[at(G, v, i, j, k)] = Uin[v * nc + lin(p, i, j, k)];
  }
  fill_ghosts(p, G, w->U);
  const long long hits = prims_and_fluxes(p, w, bad);
  flux_divergence(p, w);
  return hits;
}

/* Primitives on every stored cell of the ghosted w->U, then the face fluxes
 * in x, y and z into w->F. Returns floor hits on interior cells; sets *bad
 * if any interior cell is unrecoverable. */
static long long prims_and_fluxes(const or_params* p, work* w, int* bad) {
  const grid* G = &w->G;
  const int nx = p->n[0], ny = p->n[1], nz = p->n[2], g = G->g;
  long long hits = 0;
  int anybad = 0;

  /* primitives on every stored cell */
#pragma omp parallel for schedule(static) reduction(+ : hits) reduction(| : anybad)
  for (int k = -g; k < nz + g; ++k)
    for (int j = -g; j < ny + g; ++j)
      for (int i = -g; i < nx + g; ++i) {
        double u[5], q[5];
        int b = 0;
        for (int v = 0; v < 5; ++v) u[v] = w->U[at(G, v, i, j, k)];
        int h = or_c2p(p, u, q, &b);
        for (int v = 0; v < 5; ++v) w->W[at(G, v, i, j, k)] = q[v];
        int interior = i >= 0 && i < nx && j >= 0 && j < ny && k >= 0 && k < nz;
        if (interior) {
          hits += h;
          anybad |= b;
        }
      }

  /* fluxes in x, y, z */
  for (int d = 0; d < 3; ++d) {
    const int fx = nx + (d == 0), fy = ny + (d == 1), fz = nz + (d == 2);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < fz; ++k)
      for (int j = 0; j < fy; ++j)
        for (int i = 0; i < fx; ++i) {
          double wl[5], wr[5], f[5];
          face_states(p, w, d, i, j, k, wl, wr);
          face_flux(p, d, wl, wr, f, 0);
          for (int v = 0; v < 5; ++v) w->F[d][(size_t)v * w->fsv[d] + ((size_t)k * fy + j) * fx + i] = f[v];
        }
  }
  if (bad) *bad = anybad;
  return hits;
}

/* L = -(Fx+ - Fx-)/dx - (Fy+ - Fy-)/dy - (Fz+ - Fz-)/dz, summed x, y, z,
 * from the face fluxes held in w->F. */
static void flux_divergence(const or_params* p, work* w) {
  const int nx = p->n[0], ny = p->n[1], nz = p->n[2];
  const size_t nc = ncell(p);
  for (int v = 0; v < 5; ++v) {
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          const double* Fx = w->F[0] + (size_t)v * w->fsv[0];
          const double* Fy = w->F[1] + (size_t)v * w->fsv[1];
          const double* Fz = w->F[2] + (size_t)v * w->fsv[2];
          size_t xm = ((size_t)k * ny + j) * (nx + 1) + i;
          size_t ym = ((size_t)k * (ny + 1) + j) * nx + i;
          size_t zm = ((size_t)k * ny + j) * nx + i;
          double l = -(Fx[xm + 1] - Fx[xm]) / p->dx[0];
          l -= (Fy[ym + nx] - Fy[ym]) / p->dx[1];
          l -= (Fz[zm + (size_t)nx * ny] - Fz[zm]) / p->dx[2];
          w->L[v * nc + lin(p, i, j, k)] = l;
        }
  }
}

/* ------------------------------------------------------------------------
 * CFL time step (Sec. 3, Eq. 3): CFL * min over interior cells and
 * dimensions of dx_d / (|v_d| + c_s), c_s = sqrt(gamma p / rho).
 * ---------------------------------------------------------------------- */
double or_new_dt(const or_params* p, const double* U) {
  const size_t nc = ncell(p);
  double m = INFINITY;
#pragma omp parallel for schedule(static) reduction(min : m)
  for (size_t c = 0; c < nc; ++c) {
    double u[5], q[5];
    for (int v = 0; v < 5; ++v) u[v] = U[v * nc + c];
    or_c2p(p, u, q, NULL);
    double pr = (p->gamma - 1.0) * q[4];
    double cs = sqrt(p->gamma * pr / q[0]);
    for (int d = 0; d < 3; ++d) {
      double r = p->dx[d] / (fabs(q[1 + d]) + cs);
      if (r < m) m = r;
    }
  }
  return p->cfl * m;
}

/* ------------------------------------------------------------------------
 * The stage update, then first-order flux correction (FOFC, Sec. 3): if the
 * updated density or pressure of an interior cell is not positive, the fluxes
 * on all faces of that cell are replaced by LLF fluxes of the first-order
 * (piecewise-constant) states -- the primitives of the two cells sharing the
 * face -- and the stage update is recomputed with the corrected fluxes.
 * A stage forms Uout = a U0 + b Ust + c h L(Ust) from the step-start state
 * U0 and the previous stage's state Ust (coefficients in rk_stage below).
 * Returns the number of corrected cells.
 * ---------------------------------------------------------------------- */
typedef struct {
  double a, b, c;
} rk_coef;

/* Stage coefficients of the two-register low-storage SSP-RK integrators
 * (Sec. 3 cites Ketcheson 2010 for the family):
 *   RK1 forward Euler:            (0, 1, 1)
 *   RK2 SSPRK(2,2):               (0, 1, 1), (1/2, 1/2, 1/2)
 *   RK3 SSPRK(3,3) (Shu & Osher): (0, 1, 1), (3/4, 1/4, 1/4), (1/3, 2/3, 2/3)
 * (RK4 is SSPRK(10,4), in or_advance.) */
static rk_coef rk_stage(int rk, int stage) {
  rk_coef k = {0.0, 1.0, 1.0};
  if (stage == 1) return k;
  if (rk == 2) {
    k.a = 0.5; k.b = 0.5; k.c = 0.5;
  } else if (stage == 2) {
    k.a = 0.75; k.b = 0.25; k.c = 0.25;
  } else {
    k.a = 1.0 / 3.0; k.b = 2.0 / 3.0; k.c = 2.0 / 3.0;
  }
  return k;
}

/* SSPRK(10,4) of Ketcheson (2008) in its two-register low-storage form:
 * nine stages q1 <- q1 + h/6 L(q1); after the fifth, q2 <- q2/25 + 9 q1/25
 * and q1 <- 15 q2 - 5 q1; the tenth u <- q2 + 3/5 q1 + h/10 L(q1). */
static const rk_coef RK4_STAGE = {0.0, 1.0, 1.0 / 6.0};
static const rk_coef RK4_LAST = {1.0, 3.0 / 5.0, 1.0 / 10.0};

static void rk4_mix(double* Q2, double* q1, size_t nt) {
  for (size_t c = 0; c < nt; ++c) {
    Q2[c] = Q2[c] / 25.0 + 9.0 / 25.0 * q1[c];
    q1[c] = 15.0 * Q2[c] - 5.0 * q1[c];
  }
}

static void stage_formula(const or_params* p, const work* w, rk_coef k, const double* U0,
                          const double* Ust, double h, double* Uout) {
  const size_t nt = 5 * ncell(p);
  if (k.a == 0.0) {  /* Ust + c h L */
#pragma omp parallel for schedule(static)
    for (size_t c = 0; c < nt; ++c) Uout[c] = Ust[c] + k.c * h * w->L[c];
  } else {
#pragma omp parallel for schedule(static)
    for (size_t c = 0; c < nt; ++c) Uout[c] = k.a * U0[c] + k.b * Ust[c] + k.c * h * w->L[c];
  }
}

static long long stage_apply(const or_params* p, work* w, rk_coef k, const double* U0,
                             const double* Ust, double h, double* Uout) {
  stage_formula(p, w, k, U0, Ust, h, Uout);
  if (!p->fofc) return 0;
  const int nx = p->n[0], ny = p->n[1], nz = p->n[2];
  const size_t nc = ncell(p);
  long long flagged = 0;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const size_t c = lin(p, i, j, k);
        const double r = Uout[c], mx = Uout[nc + c], my = Uout[2 * nc + c];
        const double mz = Uout[3 * nc + c], e = Uout[4 * nc + c];
        const double pr = (p->gamma - 1.0) * (e - 0.5 * (mx * mx + my * my + mz * mz) / r);
        if (r > 0.0 && pr > 0.0) continue;
        ++flagged;
        /* replace the six face fluxes of this cell */
        for (int d = 0; d < 3; ++d) {
          const int di = d == 0, dj = d == 1, dk = d == 2;
          const int fx = nx + di, fy = ny + dj;
          for (int side = 0; side < 2; ++side) {
            /* face between cells (c-1, c) for side 0 and (c, c+1) for side 1 */
            const int li = i - di * (1 - side), lj = j - dj * (1 - side), lk = k - dk * (1 - side);
            double wl[5], wr[5], f[5];
            for (int v = 0; v < 5; ++v) {
              wl[v] = w->W[at(&w->G, v, li, lj, lk)];
              wr[v] = w->W[at(&w->G, v, li + di, lj + dj, lk + dk)];
            }
            face_flux(p, d, wl, wr, f, 1);
            const int fi = i + di * side, fj = j + dj * side, fk = k + dk * side;
            for (int v = 0; v < 5; ++v)
              w->F[d][(size_t)v * w->fsv[d] + ((size_t)fk * fy + fj) * fx + fi] = f[v];
            /* on a periodic axis the faces 0 and n are one face stored twice */
            const int fn = d == 0 ? fi : (d == 1 ? fj : fk);
            if (p->bc[d][0] == OR_PERIODIC && (fn == 0 || fn == p->n[d])) {
              const int tw = fn == 0 ? p->n[d] : 0;
              const int ti = d == 0 ? tw : fi, tj = d == 1 ? tw : fj, tk = d == 2 ? tw : fk;
              for (int v = 0; v < 5; ++v)
                w->F[d][(size_t)v * w->fsv[d] + ((size_t)tk * fy + tj) * fx + ti] = f[v];
            }
          }
        }
      }
  if (flagged) {
    flux_divergence(p, w);
    stage_formula(p, w, k, U0, Ust, h, Uout);
  }
  return flagged;
}

/* ------------------------------------------------------------------------
 * Advance U[5][nz][ny][nx] by nsteps SSP-RK steps (Sec. 3, method of lines,
 * low-storage SSP-RK of the Ketcheson 2010 family; p->rk stages). With RK2:
 *   U1      = Un + dt L(Un)
 *   U(n+1)  = Un/2 + U1/2 + dt L(U1)/2
 * with RK3:
 *   U1      = Un + dt L(Un)
 *   U2      = 3/4 Un + 1/4 U1 + 1/4 dt L(U1)
 *   U(n+1)  = 1/3 Un + 2/3 U2 + 2/3 dt L(U2)
 * and with RK4 the ten-stage SSPRK(10,4) spelled out below.
 * (each stage followed by FOFC when enabled), then dt for the next step from
 * U(n+1). *dt carries the step size in and the next one out; *t,
 * *floor_hits and *fofc_cells accumulate (either counter may be NULL).
 * Returns OR_ERR_STATE when an interior cell held a non-finite value or
 * rho <= 0 (the step still runs).
 * ---------------------------------------------------------------------- */
int or_advance(const or_params* p, double* U, int nsteps, double* t, double* dt,
               long long* floor_hits, long long* fofc_cells) {
  if (!p || !U || !t || !dt || nsteps < 0) return OR_ERR_ARG;
  for (int d = 0; d < 3; ++d) {
    if (p->n[d] < 1) return OR_ERR_ARG;
    if ((p->bc[d][0] == OR_PERIODIC) != (p->bc[d][1] == OR_PERIODIC)) return OR_ERR_ARG;
  }
  if (p->rk < 1 || p->rk > 4 || p->recon < OR_PLM || p->recon > OR_PPMX) return OR_ERR_ARG;
  work w;
  if (work_alloc(&w, p) != OR_OK) { work_free(&w); return OR_ERR_NOMEM; }
  const size_t nt = 5 * ncell(p);
  double* U1 = malloc(nt * sizeof(double));
  double* U2 = malloc(nt * sizeof(double));
  double* Q2 = p->rk == 4 ? malloc(nt * sizeof(double)) : NULL;
  if (!U1 || !U2 || (p->rk == 4 && !Q2)) {
    free(U1); free(U2); free(Q2); work_free(&w);
    return OR_ERR_NOMEM;
  }
  int status = OR_OK;
  long long hits = 0, fofc = 0;
  for (int s = 0; s < nsteps; ++s) {
    const double h = *dt;
    const double* st = U;  /* state the stage differentiates */
    if (p->rk == 4) {
      /* SSPRK(10,4) (RK4_STAGE, RK4_LAST, rk4_mix); q1 alternates between U1
       * and U2 so that no stage overwrites its own input. */
      memcpy(Q2, U, nt * sizeof(double));
      for (int stage = 1; stage <= 10; ++stage) {
        int bad = 0;
        hits += divergence(p, &w, st, &bad);
        if (bad) status = OR_ERR_STATE;
        double* out = (stage & 1) ? U1 : U2;
        fofc += stage_apply(p, &w, stage < 10 ? RK4_STAGE : RK4_LAST, Q2, st, h, out);
        st = out;
        if (stage == 5) rk4_mix(Q2, out, nt);
      }
    } else {
      for (int stage = 1; stage <= p->rk; ++stage) {
        int bad = 0;
        hits += divergence(p, &w, st, &bad);
        if (bad) status = OR_ERR_STATE;
        double* out = (stage & 1) ? U1 : U2;  /* never the stage's own input */
        fofc += stage_apply(p, &w, rk_stage(p->rk, stage), U, st, h, out);
        st = out;
      }
    }
    memcpy(U, st, nt * sizeof(double));
    *t += h;
    *dt = or_new_dt(p, U);
  }
  if (floor_hits) *floor_hits += hits;
  if (fofc_cells) *fofc_cells += fofc;
  free(U1);
  free(U2);
  free(Q2);
  work_free(&w);
  return status;
}

/* L(U) alone, for tests: Uin interior [5][nz][ny][nx] -> L same layout. */
int or_divergence(const or_params* p, const double* Uin, double* Lout, long long* floor_hits) {
  work w;
  if (work_alloc(&w, p) != OR_OK) { work_free(&w); return OR_ERR_NOMEM; }
  int bad = 0;
  long long h = divergence(p, &w, Uin, &bad);
  memcpy(Lout, w.L, 5 * ncell(p) * sizeof(double));
  if (floor_hits) *floor_hits = h;
  work_free(&w);
  return bad ? OR_ERR_STATE : OR_OK;
}

/* Ghost fill alone, for tests: Uin interior -> Uout ghosted [5][nz+2g][ny+2g][nx+2g]. */
int or_fill_ghosts(const or_params* p, const double* Uin, double* Uout) {
  grid G;
  grid_init(&G, p, or_nghost(p->recon));
  const size_t nc = ncell(p);
  for (int v = 0; v < 5; ++v)
    for (int k = 0; k < p->n[2]; ++k)
      for (int j = 0; j < p->n[1]; ++j)
        for (int i = 0; i < p->n[0]; ++i) Uout[at(&G, v, i, j, k)] = Uin[v * nc + lin(p, i, j, k)];
  fill_ghosts(p, &G, Uout);
  return OR_OK;
}

/* ------------------------------------------------------------------------
 * Static mesh refinement (Sec. 2: the mesh is a tree of MeshBlocks that all
 * hold the same number of cells; blocks that share a face differ by at most
 * one level; ghost zones across a level change are filled by restriction or
 * prolongation, and the flux through a face shared with finer blocks is
 * replaced by the finer blocks' fluxes so that the update stays
 * conservative).
 *
 * The mesh: root blocks of block[] cells tile the root grid p->n. The root
 * blocks inside any of the boxes [lo, hi) (root-block units per axis) are
 * refined once into 8 children of block[] cells at half the cell width
 * (level 1); with two levels, face neighbours differ by at most one level
 * whatever the boxes, so any union of boxes is a valid mesh. Leaves
 * are ordered root by root, x fastest; a refined root contributes its
 * children with the child's x offset fastest, then y, then z. The state is
 * U[leaf][5][bz][by][bx], x fastest.
 *
 * The ghost cells of a leaf at level L hold the mesh's representation at
 * level L, evaluated at the ghost cell's global index (indices outside the
 * domain first follow the boundary condition at that level: periodic wrap,
 * outflow clamp to the nearest interior cell):
 *   level 0 at coarse cell I: the coarse leaf's cell when its root is not
 *     refined; otherwise the mean of the 8 fine cells covering I, summed in
 *     pairs along x, then y, then z, times 1/8 (restriction);
 *   level 1 at fine cell i: the fine leaf's cell when its root is refined;
 *     otherwise C + (sgn_x s_x + sgn_y s_y + sgn_z s_z)/4, with C the level-0
 *     value at I = floor(i/2), s_d the minmod of the two level-0 differences
 *     next to I along d (neighbours again by the boundary condition), and
 *     sgn_d = +1 for the upper child (i odd), -1 for the lower (prolongation,
 *     linear and limited; it conserves: the 8 children average to C).
 * A coarse face shared with 4 fine faces takes the mean of their 4 fluxes,
 * summed in pairs along the lower transverse axis first.
 * ---------------------------------------------------------------------- */
#define OR_MAX_BOXES 8

typedef struct {
  int32_t block[3];                  /* cells per block, even and >= 2 * ghosts per axis */
  int32_t nbox;                      /* refined boxes, 0..OR_MAX_BOXES (0: none)          */
  int32_t box[OR_MAX_BOXES][2][3];   /* box b refines the root blocks with               */
                                     /* box[b][0][d] <= root index < box[b][1][d]        */
} or_smr;

typedef struct {
  or_params p;   /* the root grid */
  int b[3];      /* cells per block */
  int nr[3];     /* root blocks per axis */
  int nroot;
  int* rref;     /* per root block: 1 if refined */
  int* rleaf;    /* per root block: its leaf, or its first child */
  int nleaf;
  int* lev;      /* per leaf: level 0 or 1 */
  int* loc;      /* per leaf: 3 block coordinates at its level */
  size_t vs, bs; /* doubles per variable and per leaf */
} smr_mesh;

static void smr_free(smr_mesh* m) {
  free(m->rref); free(m->rleaf); free(m->lev); free(m->loc);
}

static int smr_init(smr_mesh* m, const or_params* p, const or_smr* s) {
  memset(m, 0, sizeof *m);
  m->p = *p;
  const int g = or_nghost(p->recon);
  if (s->nbox < 0 || s->nbox > OR_MAX_BOXES) return OR_ERR_ARG;
  for (int d = 0; d < 3; ++d) {
    m->b[d] = s->block[d];
    if (m->b[d] < 2 * g || (m->b[d] & 1) || p->n[d] % m->b[d]) return OR_ERR_ARG;
    if ((p->bc[d][0] == OR_PERIODIC) != (p->bc[d][1] == OR_PERIODIC)) return OR_ERR_ARG;
    m->nr[d] = p->n[d] / m->b[d];
    for (int b = 0; b < s->nbox; ++b)
      if (s->box[b][0][d] < 0 || s->box[b][1][d] > m->nr[d] || s->box[b][0][d] >= s->box[b][1][d])
        return OR_ERR_ARG;
  }
  m->nroot = m->nr[0] * m->nr[1] * m->nr[2];
  m->rref = calloc((size_t)m->nroot, sizeof(int));
  m->rleaf = calloc((size_t)m->nroot, sizeof(int));
  if (!m->rref || !m->rleaf) return OR_ERR_NOMEM;
  int nleaf = 0;
  for (int rz = 0; rz < m->nr[2]; ++rz)
    for (int ry = 0; ry < m->nr[1]; ++ry)
      for (int rx = 0; rx < m->nr[0]; ++rx) {
        const int r = rx + m->nr[0] * (ry + m->nr[1] * rz);
        int in = 0;
        for (int b = 0; b < s->nbox; ++b)
          in |= rx >= s->box[b][0][0] && rx < s->box[b][1][0] && ry >= s->box[b][0][1] &&
                ry < s->box[b][1][1] && rz >= s->box[b][0][2] && rz < s->box[b][1][2];
        m->rref[r] = in;
        m->rleaf[r] = nleaf;
        nleaf += in ? 8 : 1;
      }
  m->nleaf = nleaf;
  m->lev = malloc((size_t)nleaf * sizeof(int));
  m->loc = malloc((size_t)nleaf * 3 * sizeof(int));
  if (!m->lev || !m->loc) return OR_ERR_NOMEM;
  for (int rz = 0; rz < m->nr[2]; ++rz)
    for (int ry = 0; ry < m->nr[1]; ++ry)
      for (int rx = 0; rx < m->nr[0]; ++rx) {
        const int r = rx + m->nr[0] * (ry + m->nr[1] * rz);
        const int q0 = m->rleaf[r];
        if (!m->rref[r]) {
          m->lev[q0] = 0;
          m->loc[3 * q0] = rx; m->loc[3 * q0 + 1] = ry; m->loc[3 * q0 + 2] = rz;
          continue;
        }
        for (int c = 0; c < 8; ++c) {
          const int q = q0 + c;
          m->lev[q] = 1;
          m->loc[3 * q] = 2 * rx + (c & 1);
          m->loc[3 * q + 1] = 2 * ry + ((c >> 1) & 1);
          m->loc[3 * q + 2] = 2 * rz + ((c >> 2) & 1);
        }
      }
  m->vs = (size_t)m->b[0] * m->b[1] * m->b[2];
  m->bs = 5 * m->vs;
  return OR_OK;
}

static size_t smr_cell(const smr_mesh* m, int i, int j, int k) {
  return ((size_t)k * m->b[1] + j) * m->b[0] + i;
}

/* Fine cell (i,j,k) (level-1 global indices, inside a refined root). */
static double smr_fine(const smr_mesh* m, const double* U, int v, int i, int j, int k) {
  const int lx = i / m->b[0], ly = j / m->b[1], lz = k / m->b[2];
  const int r = lx / 2 + m->nr[0] * (ly / 2 + m->nr[1] * (lz / 2));
  const int q = m->rleaf[r] + (lx & 1) + 2 * (ly & 1) + 4 * (lz & 1);
  return U[(size_t)q * m->bs + (size_t)v * m->vs +
           smr_cell(m, i - lx * m->b[0], j - ly * m->b[1], k - lz * m->b[2])];
}

/* Level-0 representation at coarse cell (I,J,K), inside the domain. */
static double smr_rep0(const smr_mesh* m, const double* U, int v, int I, int J, int K) {
  const int rx = I / m->b[0], ry = J / m->b[1], rz = K / m->b[2];
  const int r = rx + m->nr[0] * (ry + m->nr[1] * rz);
  if (!m->rref[r])
    return U[(size_t)m->rleaf[r] * m->bs + (size_t)v * m->vs +
             smr_cell(m, I - rx * m->b[0], J - ry * m->b[1], K - rz * m->b[2])];
  double f[8];
  for (int c = 0; c < 8; ++c)
    f[c] = smr_fine(m, U, v, 2 * I + (c & 1), 2 * J + ((c >> 1) & 1), 2 * K + ((c >> 2) & 1));
  return (((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7]))) * 0.125;
}

static double smr_minmod(double a, double b) {
  if (!(a * b > 0.0)) return 0.0;
  return fabs(a) < fabs(b) ? a : b;
}

/* Level-1 representation at fine cell (i,j,k), inside the domain. */
static double smr_rep1(const smr_mesh* m, const double* U, int v, int i, int j, int k) {
  const int r = i / (2 * m->b[0]) + m->nr[0] * (j / (2 * m->b[1]) + m->nr[1] * (k / (2 * m->b[2])));
  if (m->rref[r]) return smr_fine(m, U, v, i, j, k);
  const int c[3] = {i / 2, j / 2, k / 2};
  const int f[3] = {i, j, k};
  const double C = smr_rep0(m, U, v, c[0], c[1], c[2]);
  double t[3];
  for (int d = 0; d < 3; ++d) {
    int lo[3] = {c[0], c[1], c[2]}, hi[3] = {c[0], c[1], c[2]};
    lo[d] = src_index(c[d] - 1, m->p.n[d], m->p.bc[d][0], m->p.bc[d][1]);
    hi[d] = src_index(c[d] + 1, m->p.n[d], m->p.bc[d][0], m->p.bc[d][1]);
    const double dl = C - smr_rep0(m, U, v, lo[0], lo[1], lo[2]);
    const double dr = smr_rep0(m, U, v, hi[0], hi[1], hi[2]) - C;
    const double sd = smr_minmod(dl, dr);
    t[d] = (f[d] & 1) ? sd : -sd;
  }
  return C + 0.25 * ((t[0] + t[1]) + t[2]);
}

/* Ghosted copy of leaf q: interior, then the face ghosts (ng deep, interior
 * transverse extent) from the level representation; edges and corners, which
 * the dimension-by-dimension stencil never reads, are set to 0. */
static void smr_fill_leaf(const smr_mesh* m, const double* U, int q, const grid* G, double* Ug) {
  const int L = m->lev[q], g = G->g;
  const int base[3] = {m->loc[3 * q] * m->b[0], m->loc[3 * q + 1] * m->b[1], m->loc[3 * q + 2] * m->b[2]};
  const int N[3] = {m->p.n[0] << L, m->p.n[1] << L, m->p.n[2] << L};
  memset(Ug, 0, 5 * G->sv * sizeof(double));
  for (int v = 0; v < 5; ++v)
    for (int k = -g; k < m->b[2] + g; ++k)
      for (int j = -g; j < m->b[1] + g; ++j)
        for (int i = -g; i < m->b[0] + g; ++i) {
          const int l[3] = {i, j, k};
          int out = 0, dd = -1;
          for (int d = 0; d < 3; ++d)
            if (l[d] < 0 || l[d] >= m->b[d]) { ++out; dd = d; }
          if (out == 0) {
            Ug[at(G, v, i, j, k)] = U[(size_t)q * m->bs + (size_t)v * m->vs + smr_cell(m, i, j, k)];
            continue;
          }
          if (out > 1) continue;
          int gi[3] = {base[0] + i, base[1] + j, base[2] + k};
          gi[dd] = src_index(gi[dd], N[dd], m->p.bc[dd][0], m->p.bc[dd][1]);
          Ug[at(G, v, i, j, k)] = L == 0 ? smr_rep0(m, U, v, gi[0], gi[1], gi[2])
                                         : smr_rep1(m, U, v, gi[0], gi[1], gi[2]);
        }
}

static or_params smr_leaf_params(const smr_mesh* m, int q) {
  or_params pl = m->p;
  for (int d = 0; d < 3; ++d) {
    pl.n[d] = m->b[d];
    pl.dx[d] = m->lev[q] ? 0.5 * m->p.dx[d] : m->p.dx[d];
  }
  return pl;
}

/* Flux of face (i,j,k) along d of leaf q's flux array (face indices). */
static double* smr_face(const smr_mesh* m, work* w, int d, int v, int i, int j, int k) {
  const int fx = m->b[0] + (d == 0), fy = m->b[1] + (d == 1);
  return &w->F[d][(size_t)v * w->fsv[d] + ((size_t)k * fy + j) * fx + i];
}

/* Replace the coarse fluxes on faces shared with refined roots by the mean
 * of the 4 fine fluxes (the fine leaves' own, already in their work). */
static void smr_correct_fluxes(const smr_mesh* m, work* w) {
  for (int q = 0; q < m->nleaf; ++q) {
    if (m->lev[q] != 0) continue;
    const int rc[3] = {m->loc[3 * q], m->loc[3 * q + 1], m->loc[3 * q + 2]};
    for (int d = 0; d < 3; ++d) {
      const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
      for (int side = 0; side < 2; ++side) {
        int rn[3] = {rc[0], rc[1], rc[2]};
        rn[d] += side ? 1 : -1;
        if (rn[d] < 0 || rn[d] >= m->nr[d]) {
          if (m->p.bc[d][0] != OR_PERIODIC) continue;
          rn[d] = (rn[d] + m->nr[d]) % m->nr[d];
        }
        if (!m->rref[rn[0] + m->nr[0] * (rn[1] + m->nr[1] * rn[2])]) continue;
        /* fine cell just across the face, along d (level-1 global index) */
        const int N1 = 2 * m->p.n[d];
        const int fd = ((side ? 2 * (rc[d] + 1) * m->b[d] : 2 * rc[d] * m->b[d] - 1) + N1) % N1;
        for (int b2 = 0; b2 < m->b[t2]; ++b2)
          for (int b1 = 0; b1 < m->b[t1]; ++b1) {
            int cf[3];
            cf[d] = side ? m->b[d] : 0;
            cf[t1] = b1;
            cf[t2] = b2;
            for (int v = 0; v < 5; ++v) {
              double f[4];
              for (int e = 0; e < 4; ++e) {
                int gf[3];
                gf[d] = fd;
                gf[t1] = 2 * (rc[t1] * m->b[t1] + b1) + (e & 1);
                gf[t2] = 2 * (rc[t2] * m->b[t2] + b2) + (e >> 1);
                const int lx = gf[0] / m->b[0], ly = gf[1] / m->b[1], lz = gf[2] / m->b[2];
                const int r = lx / 2 + m->nr[0] * (ly / 2 + m->nr[1] * (lz / 2));
                const int qf = m->rleaf[r] + (lx & 1) + 2 * (ly & 1) + 4 * (lz & 1);
                int lf[3] = {gf[0] - lx * m->b[0], gf[1] - ly * m->b[1], gf[2] - lz * m->b[2]};
                lf[d] = side ? 0 : m->b[d];  /* the fine leaf's face on the coarse side */
                f[e] = *smr_face(m, &w[qf], d, v, lf[0], lf[1], lf[2]);
              }
              *smr_face(m, &w[q], d, v, cf[0], cf[1], cf[2]) = ((f[0] + f[1]) + (f[2] + f[3])) * 0.25;
            }
          }
      }
    }
  }
}

/* L for every leaf of the leaf-major state S: ghost fill, fluxes, flux
 * correction (when `correct`; else each leaf keeps its own fluxes on every
 * face), divergence (into w[q].L). */
static long long smr_divergence(const smr_mesh* m, work* w, const double* S, int correct, int* bad) {
  long long hits = 0;
  int anybad = 0;
  for (int q = 0; q < m->nleaf; ++q) {
    const or_params pl = smr_leaf_params(m, q);
    smr_fill_leaf(m, S, q, &w[q].G, w[q].U);
    int b = 0;
    hits += prims_and_fluxes(&pl, &w[q], &b);
    anybad |= b;
  }
  if (correct) smr_correct_fluxes(m, w);
  for (int q = 0; q < m->nleaf; ++q) {
    const or_params pl = smr_leaf_params(m, q);
    flux_divergence(&pl, &w[q]);
  }
  if (bad) *bad = anybad;
  return hits;
}

static void smr_stage(const smr_mesh* m, work* w, rk_coef k, const double* U0, const double* Ust,
                      double h, double* Uout) {
  for (int q = 0; q < m->nleaf; ++q) {
    const or_params pl = smr_leaf_params(m, q);
    const size_t o = (size_t)q * m->bs;
    stage_formula(&pl, &w[q], k, U0 + o, Ust + o, h, Uout + o);
  }
}

/* The leaf at the same level across face (d, side) of leaf q, or -1 when the
 * region across is on the other level or beyond an outflow boundary. */
static int smr_same_level(const smr_mesh* m, int q, int d, int side) {
  const int L = m->lev[q];
  int l[3] = {m->loc[3 * q], m->loc[3 * q + 1], m->loc[3 * q + 2]};
  const int nl = m->nr[d] << L;
  l[d] += side ? 1 : -1;
  if (l[d] < 0 || l[d] >= nl) {
    if (m->p.bc[d][0] != OR_PERIODIC) return -1;
    l[d] = (l[d] + nl) % nl;
  }
  const int r = (l[0] >> L) + m->nr[0] * ((l[1] >> L) + m->nr[1] * (l[2] >> L));
  if (m->rref[r] != L) return -1;
  return L == 0 ? m->rleaf[r] : m->rleaf[r] + (l[0] & 1) + 2 * (l[1] & 1) + 4 * (l[2] & 1);
}

/* FOFC on the leaves of one level: the provisional update of every leaf of
 * the level from its fluxes as they stand (into Uout), then every face of a
 * cell whose provisional density or pressure is not positive takes the LLF
 * flux of the first-order states at the leaf's level (the cell and, across
 * the face, the neighbour cell or the ghost value there); a face shared with a
 * same-level neighbour leaf is replaced in both leaves. Returns the flagged
 * cells. */
static long long smr_fofc_level(const smr_mesh* m, work* w, rk_coef k, const double* U0,
                                const double* Ust, double h, double* Uout, int level) {
  for (int q = 0; q < m->nleaf; ++q) {
    if (m->lev[q] != level) continue;
    const or_params pl = smr_leaf_params(m, q);
    const size_t o = (size_t)q * m->bs;
    flux_divergence(&pl, &w[q]);
    stage_formula(&pl, &w[q], k, U0 + o, Ust + o, h, Uout + o);
  }
  long long flagged = 0;
  for (int q = 0; q < m->nleaf; ++q) {
    if (m->lev[q] != level) continue;
    const or_params pl = smr_leaf_params(m, q);
    const double* Uq = Uout + (size_t)q * m->bs;
    for (int kk = 0; kk < m->b[2]; ++kk)
      for (int j = 0; j < m->b[1]; ++j)
        for (int i = 0; i < m->b[0]; ++i) {
          const size_t c = smr_cell(m, i, j, kk);
          const double r = Uq[c], mx = Uq[m->vs + c], my = Uq[2 * m->vs + c];
          const double mz = Uq[3 * m->vs + c], e = Uq[4 * m->vs + c];
          const double pr = (m->p.gamma - 1.0) * (e - 0.5 * (mx * mx + my * my + mz * mz) / r);
          if (r > 0.0 && pr > 0.0) continue;
          ++flagged;
          for (int d = 0; d < 3; ++d) {
            const int di = d == 0, dj = d == 1, dk = d == 2;
            for (int side = 0; side < 2; ++side) {
              const int li = i + di * (side - 1), lj = j + dj * (side - 1), lk = kk + dk * (side - 1);
              double wl[5], wr[5], f[5];
              for (int v = 0; v < 5; ++v) {
                wl[v] = w[q].W[at(&w[q].G, v, li, lj, lk)];
                wr[v] = w[q].W[at(&w[q].G, v, li + di, lj + dj, lk + dk)];
              }
              face_flux(&pl, d, wl, wr, f, 1);
              int fc[3] = {i + di * side, j + dj * side, kk + dk * side};
              for (int v = 0; v < 5; ++v) *smr_face(m, &w[q], d, v, fc[0], fc[1], fc[2]) = f[v];
              if (fc[d] == 0 || fc[d] == m->b[d]) {
                const int qn = smr_same_level(m, q, d, fc[d] == m->b[d]);
                if (qn >= 0) {
                  fc[d] = fc[d] == 0 ? m->b[d] : 0;
                  for (int v = 0; v < 5; ++v) *smr_face(m, &w[qn], d, v, fc[0], fc[1], fc[2]) = f[v];
                }
              }
            }
          }
        }
  }
  return flagged;
}

/* First-order flux correction on a refined mesh (Sec. 3 FOFC with the
 * level-boundary flux correction of Sec. 2), finest level first; w holds
 * every leaf's own fluxes. FOFC on the fine leaves; the coarse faces next to
 * finer leaves take the mean of the 4 fine fluxes as they stand after it;
 * FOFC on the coarse leaves, whose provisional update thus already has the
 * fine side's fluxes on level faces; the level faces once more take the fine
 * mean (the fine side's fluxes rule there, also for a corrected coarse cell);
 * the stage from the final fluxes into Uout. Returns the flagged cells. */
static long long smr_fofc(const smr_mesh* m, work* w, rk_coef k, const double* U0, const double* Ust,
                          double h, double* Uout) {
  long long flagged = smr_fofc_level(m, w, k, U0, Ust, h, Uout, 1);
  smr_correct_fluxes(m, w);
  flagged += smr_fofc_level(m, w, k, U0, Ust, h, Uout, 0);
  smr_correct_fluxes(m, w);
  for (int q = 0; q < m->nleaf; ++q) {
    const or_params pl = smr_leaf_params(m, q);
    flux_divergence(&pl, &w[q]);
  }
  smr_stage(m, w, k, U0, Ust, h, Uout);
  return flagged;
}

/* On any return, smr_close(m, *w) releases what was allocated. */
static int smr_open(smr_mesh* m, work** w, const or_params* p, const or_smr* s) {
  *w = NULL;
  memset(m, 0, sizeof *m);
  if (!p || !s) return OR_ERR_ARG;
  if (p->recon < OR_PLM || p->recon > OR_PPMX || p->rk < 1 || p->rk > 4) return OR_ERR_ARG;
  int st = smr_init(m, p, s);
  if (st != OR_OK) return st;
  *w = calloc((size_t)m->nleaf, sizeof(work));
  if (!*w) return OR_ERR_NOMEM;
  for (int q = 0; q < m->nleaf; ++q) {
    const or_params pl = smr_leaf_params(m, q);
    if (work_alloc(&(*w)[q], &pl) != OR_OK) return OR_ERR_NOMEM;
  }
  return OR_OK;
}

static void smr_close(smr_mesh* m, work* w) {
  if (w)
    for (int q = 0; q < m->nleaf; ++q) work_free(&w[q]);  /* calloc'd: unset pointers are NULL */
  free(w);
  smr_free(m);
}

/* Number of leaves, and (when out != NULL) per leaf: level, x, y, z block
 * coordinates at that level. Negative status on a bad configuration. */
int or_smr_leaves(const or_params* p, const or_smr* s, int32_t* out) {
  smr_mesh m;
  int st = smr_init(&m, p, s);
  if (st != OR_OK) { smr_free(&m); return -st; }
  if (out)
    for (int q = 0; q < m.nleaf; ++q) {
      out[4 * q] = m.lev[q];
      for (int d = 0; d < 3; ++d) out[4 * q + 1 + d] = m.loc[3 * q + d];
    }
  const int n = m.nleaf;
  smr_free(&m);
  return n;
}

/* CFL time step over all leaves, each at its own cell width. */
double or_smr_new_dt(const or_params* p, const or_smr* s, const double* U) {
  smr_mesh m;
  if (smr_init(&m, p, s) != OR_OK) { smr_free(&m); return NAN; }
  double dt = INFINITY;
  for (int q = 0; q < m.nleaf; ++q) {
    const or_params pl = smr_leaf_params(&m, q);
    const double d = or_new_dt(&pl, U + (size_t)q * m.bs);
    if (d < dt) dt = d;
  }
  smr_free(&m);
  return dt;
}

/* Advance the leaf-major state by nsteps SSP-RK steps (the stage sequence of
 * or_advance; every stage's L comes from smr_divergence, with p->fofc
 * without the level correction, which smr_fofc then applies). *fofc_cells
 * (may be NULL) accumulates the flagged cells. */
int or_smr_advance(const or_params* p, const or_smr* s, double* U, int nsteps, double* t,
                   double* dt, long long* floor_hits, long long* fofc_cells) {
  if (!U || !t || !dt || nsteps < 0) return OR_ERR_ARG;
  smr_mesh m;
  work* w;
  int st = smr_open(&m, &w, p, s);
  if (st != OR_OK) { smr_close(&m, w); return st; }
  const size_t nt = (size_t)m.nleaf * m.bs;
  double* U1 = malloc(nt * sizeof(double));
  double* U2 = malloc(nt * sizeof(double));
  double* Q2 = p->rk == 4 ? malloc(nt * sizeof(double)) : NULL;
  if (!U1 || !U2 || (p->rk == 4 && !Q2)) {
    free(U1); free(U2); free(Q2); smr_close(&m, w);
    return OR_ERR_NOMEM;
  }
  int status = OR_OK;
  long long hits = 0, fofc = 0;
  for (int n = 0; n < nsteps; ++n) {
    const double h = *dt;
    const double* S = U;
    const int nst = p->rk == 4 ? 10 : p->rk;
    if (p->rk == 4) memcpy(Q2, U, nt * sizeof(double));
    for (int stage = 1; stage <= nst; ++stage) {
      int bad = 0;
      hits += smr_divergence(&m, w, S, !p->fofc, &bad);
      if (bad) status = OR_ERR_STATE;
      double* out = (stage & 1) ? U1 : U2;
      const rk_coef kc = p->rk == 4 ? (stage < 10 ? RK4_STAGE : RK4_LAST) : rk_stage(p->rk, stage);
      const double* U0 = p->rk == 4 ? Q2 : U;
      if (p->fofc)
        fofc += smr_fofc(&m, w, kc, U0, S, h, out);
      else
        smr_stage(&m, w, kc, U0, S, h, out);
      if (p->rk == 4 && stage == 5) rk4_mix(Q2, out, nt);
      S = out;
    }
    memcpy(U, S, nt * sizeof(double));
    *t += h;
    *dt = or_smr_new_dt(p, s, U);
  }
  if (floor_hits) *floor_hits += hits;
  if (fofc_cells) *fofc_cells += fofc;
  free(U1); free(U2); free(Q2);
  smr_close(&m, w);
  return status;
}

/* Tests: ghosted leaves [leaf][5][bz+2g][by+2g][bx+2g] (face ghosts from the
 * level representation, edges and corners 0) and L per leaf after the flux
 * correction ([leaf][5][bz][by][bx]). */
int or_smr_fill_ghosts(const or_params* p, const or_smr* s, const double* U, double* Gout) {
  smr_mesh m;
  work* w;
  int st = smr_open(&m, &w, p, s);
  if (st != OR_OK) { smr_close(&m, w); return st; }
  const size_t gs = 5 * w[0].G.sv;
  for (int q = 0; q < m.nleaf; ++q) smr_fill_leaf(&m, U, q, &w[q].G, Gout + (size_t)q * gs);
  smr_close(&m, w);
  return OR_OK;
}

int or_smr_divergence(const or_params* p, const or_smr* s, const double* U, double* Lout,
                      long long* floor_hits) {
  smr_mesh m;
  work* w;
  int st = smr_open(&m, &w, p, s);
  if (st != OR_OK) { smr_close(&m, w); return st; }
  int bad = 0;
  const long long h = smr_divergence(&m, w, U, 1, &bad);
  for (int q = 0; q < m.nleaf; ++q) memcpy(Lout + (size_t)q * m.bs, w[q].L, m.bs * sizeof(double));
  if (floor_hits) *floor_hits = h;
  smr_close(&m, w);
  return bad ? OR_ERR_STATE : OR_OK;
}
