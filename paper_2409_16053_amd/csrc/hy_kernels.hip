// hy_kernels.hip -- gfx950 kernels of the 3D Newtonian adiabatic hydro update.
//
// One fused kernel per RK stage performs the whole reconstruct-solve-advance
// sequence of Stone et al. 2024 (arXiv:2409.16053), Sec. 3: ghost zones,
// cons-to-prim (Sec. 3.1, Eq. 4), PLM, PPM4, PPMX or WENO-Z reconstruction
// on primitives, HLLC fluxes in x, y and z, the flux divergence and the
// low-storage SSP-RK stage update; the last stage also reduces the CFL time
// step of Sec. 3, Eq. 3.
//
// Work decomposition. A workgroup owns an x-y tile (TX x TY columns) of one
// MeshBlock and marches along z through a chunk of planes. Each owned column
// keeps its z stencil (primitives, slopes or PPM edge values, and the lower
// z-face flux) in registers, so z neighbours cost no memory traffic. For the
// current plane the primitives of the tile and of its x/y ghost zones sit in
// LDS; all x- and y-faces of the plane are spread evenly over the threads,
// each computing both one-sided reconstructions and the HLLC flux of its face
// and leaving it in LDS for the divergence. Global memory is only touched by
// x-contiguous rows: one new plane of U per step of the march, the ghost rows
// of the tile, and the output row.
//
// Ghost zones are not stored: a tile's ghost cells are read straight from
// the neighbouring MeshBlock's interior (same level, same device), or from the
// nearest interior cell at an outflow boundary, which is exactly what the
// paper's ghost-zone copy would have put there (Sec. 2, "Boundary conditions").
//
// Precision. T = double or float is the type of reconstruction and the
// Riemann solve. Cons-to-prim, the flux divergence, the RK update and the time
// step are always FP64. The library is built with -ffp-contract=on: a * b + c
// within one source expression becomes an FMA, decided per expression when it
// is compiled, so every instantiation still performs identical per-cell
// arithmetic; the Newton steps of the reciprocals are written as FMAs.
#include <algorithm>

#include "hy_internal.h"

namespace hy {

constexpr unsigned long long kInfBits = 0x7FF0000000000000ull;

// ---------------------------------------------------------------- helpers
// Reciprocal and square root. FP64: the hardware reciprocal estimate refined
// by two Newton-Raphson steps (error squared each step) to full double
// precision; callers only form x * rcp(y) where y != 0 on every selected
// branch. FP32 (mixed path, reconstruction and Riemann solve only): the
// native 1-ulp instructions.
__device__ __forceinline__ double rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Reciprocal for limiter and weight arithmetic, where a few ulps do not
// matter: FP64 takes one Newton-Raphson step (the estimate's ~3e-8 relative
// error squared, i.e. within ~8 ulp); FP32 the native instruction.
__device__ __forceinline__ double rcp_lim(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float rcp_lim(float x) { return __builtin_amdgcn_rcpf(x); }

// Square root. FP64: the hardware reciprocal-square-root estimate, one
// Goldschmidt step (g ~ sqrt(x), h ~ 1/(2 sqrt(x)); the error is squared) and
// a final Newton correction of g (squared again), which lands within an ulp;
// x == 0 gives 0. Arguments here are sound-speed-like quantities >= 0. FP32:
// the native instruction.
__device__ __forceinline__ double rsqrt_(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, x);
  g = fma(d, h, g);
  return x == 0.0 ? 0.0 : g;
}
__device__ __forceinline__ float rsqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }

// XCD-aware remap: the dispatcher hands workgroup w to XCD w % 8. Give each
// XCD a contiguous run of logical tiles so that tiles sharing ghost rows share
// an L2.
__device__ __forceinline__ int xcd_remap(int w, int G) {
  const int q = G >> 3, r = G & 7;
  const int x = w & 7, s = w >> 3;
  return x * q + (x < r ? x : r) + s;
}

// ---------------------------------------------------------- reconstruction
// PLM: half the van Leer harmonic-mean slope of a cell from its neighbours,
// dl dr / (dl + dr) when dl dr > 0 (faces are w0 -/+ this; halving the
// slope 2 dl dr / (dl + dr) is exact, so nothing else changes).
template <typename T>
__device__ __forceinline__ T plm_half_slope(T wm, T w0, T wp) {
  const T dl = w0 - wm, dr = wp - w0;
  const T prod = dl * dr;
  const T s = prod * rcp_lim(dl + dr);
  return prod > T(0) ? s : T(0);
}

// PPM4 (Colella & Woodward 1984): monotonised central slope, Eq. 1.8.
template <typename T>
__device__ __forceinline__ T ppm_dm(T wm, T w0, T wp) {
  const T dl = w0 - wm, dr = wp - w0;
  const T da = T(0.5) * (wp - wm);
  T m = fabs(da);
  m = fmin(m, T(2) * fabs(dl));
  m = fmin(m, T(2) * fabs(dr));
  return dl * dr > T(0) ? copysign(m, da) : T(0);
}

// PPM4 interface value between cells c and c+1, Eq. 1.6 on a uniform mesh.
template <typename T>
__device__ __forceinline__ T ppm_iface(T wc, T wc1, T dmc, T dmc1) {
  return (wc + T(0.5) * (wc1 - wc)) - (dmc1 - dmc) * T(1.0 / 6.0);
}

// PPM4 monotonicity constraints, Eq. 1.10: edge values (aL, aR) of a cell
// with average a.
template <typename T>
__device__ __forceinline__ void ppm_mono(T a, T& aL, T& aR) {
  const bool ext = (aR - a) * (a - aL) <= T(0);
  const T d = aR - aL;
  const T m6 = d * (a - T(0.5) * (aL + aR));
  const T d26 = (d * d) * T(1.0 / 6.0);
  const bool over_l = m6 > d26;
  const bool over_r = !over_l && (-d26 > m6);
  const T nL = over_l ? T(3) * a - T(2) * aR : aL;
  const T nR = over_r ? T(3) * a - T(2) * aL : aR;
  aL = ext ? a : nL;
  aR = ext ? a : nR;
}

// WENO-Z (Sec. 3; Borges et al. 2008 weights on the Jiang-Shu smoothness
// indicators). From the cells (w0..w4) = c-2..c+2: the three third-order
// candidate values of the right face of cell c, written as differences from
// w2 (times 6) so that a constant state is reproduced exactly, weighted by
// alpha_k = d_k (1 + r_k^2), r_k = min(tau5 / (beta_k + eps), 1e15),
// tau5 = |beta_0 - beta_2|, d = (1, 6, 3)/10. The cap keeps the weights finite
// in FP32 and changes them only where one candidate already has weight 1 to
// within 1e-30.
template <typename T>
struct WenoInd {
  T b0, b1, b2;
};

template <typename T>
__device__ __forceinline__ WenoInd<T> weno_ind(T w0, T w1, T w2, T w3, T w4) {
  const T e0 = w0 - T(2) * w1 + w2, f0 = w0 - T(4) * w1 + T(3) * w2;
  const T e1 = w1 - T(2) * w2 + w3, f1 = w1 - w3;
  const T e2 = w2 - T(2) * w3 + w4, f2 = T(3) * w2 - T(4) * w3 + w4;
  const T c13 = T(13.0 / 12.0);
  return WenoInd<T>{c13 * e0 * e0 + T(0.25) * f0 * f0, c13 * e1 * e1 + T(0.25) * f1 * f1,
                    c13 * e2 * e2 + T(0.25) * f2 * f2};
}

// Weighted sum of the candidates (given as 6 x difference from wc) with the
// indicators ordered as the candidates.
template <typename T>
__device__ __forceinline__ T weno_mix(T wc, T q0, T q1, T q2, T b0, T b1, T b2) {
  const T eps = T(1e-36), cap = T(1e15);
  const T tau = fabs(b0 - b2);
  const T r0 = fmin(tau * rcp_lim(b0 + eps), cap);
  const T r1 = fmin(tau * rcp_lim(b1 + eps), cap);
  const T r2 = fmin(tau * rcp_lim(b2 + eps), cap);
  const T a0 = T(0.1) * (T(1) + r0 * r0);
  const T a1 = T(0.6) * (T(1) + r1 * r1);
  const T a2 = T(0.3) * (T(1) + r2 * r2);
  // normalise the weights first: a_k can reach 1e30, which must not meet a
  // large candidate in FP32
  const T id = rcp_lim((a0 + a1) + a2);
  const T mix = ((a0 * id) * q0 + (a1 * id) * q1) + (a2 * id) * q2;
  return wc + mix * T(1.0 / 6.0);
}

// Right face value of the middle cell of (w0..w4).
template <typename T>
__device__ __forceinline__ T weno_right(T w0, T w1, T w2, T w3, T w4) {
  const WenoInd<T> b = weno_ind(w0, w1, w2, w3, w4);
  const T q0 = T(2) * (w0 - w1) - T(5) * (w1 - w2);
  const T q1 = T(2) * (w3 - w2) - (w1 - w2);
  const T q2 = T(4) * (w3 - w2) - (w4 - w3);
  return weno_mix(w2, q0, q1, q2, b.b0, b.b1, b.b2);
}

// Both face values of the middle cell, sharing the indicators: the left face
// is the right-face formula on the mirrored stencil, whose indicators are
// (beta_2, beta_1, beta_0).
template <typename T>
__device__ __forceinline__ void weno_cell(T w0, T w1, T w2, T w3, T w4, T& left, T& right) {
  const WenoInd<T> b = weno_ind(w0, w1, w2, w3, w4);
  right = weno_mix(w2, T(2) * (w0 - w1) - T(5) * (w1 - w2), T(2) * (w3 - w2) - (w1 - w2),
                   T(4) * (w3 - w2) - (w4 - w3), b.b0, b.b1, b.b2);
  left = weno_mix(w2, T(2) * (w4 - w3) - T(5) * (w3 - w2), T(2) * (w1 - w2) - (w3 - w2),
                  T(4) * (w1 - w2) - (w0 - w1), b.b2, b.b1, b.b0);
}

// PPMX (Sec. 3; the extremum-preserving limiters of Colella & Sekora 2008 as
// used by McCorquodale & Colella). A limited second difference keeps the
// common sign of its arguments and the smallest magnitude among the first
// and 1.25 x the others, or is 0 when the signs differ.
template <typename T>
__device__ __forceinline__ T ppmx_lim3(T d, T l, T r) {
  const bool pos = d > T(0) && l > T(0) && r > T(0);
  const bool neg = d < T(0) && l < T(0) && r < T(0);
  const T m = fmin(fabs(d), fmin(T(1.25) * fabs(l), T(1.25) * fabs(r)));
  return pos ? m : (neg ? -m : T(0));
}

template <typename T>
__device__ __forceinline__ T ppmx_lim4(T d, T c, T l, T r) {
  const bool pos = d > T(0) && c > T(0) && l > T(0) && r > T(0);
  const bool neg = d < T(0) && c < T(0) && l < T(0) && r < T(0);
  const T m = fmin(fmin(fabs(d), T(1.25) * fabs(c)), fmin(T(1.25) * fabs(l), T(1.25) * fabs(r)));
  return pos ? m : (neg ? -m : T(0));
}

// Fourth-order interface value between b and c (neighbours a, d),
// 7/12 (b + c) - 1/12 (a + d) written in differences so that a constant state
// is reproduced exactly; a value outside [b, c] is replaced by
// (b + c)/2 - D/6, D the limited 3 (b - 2f + c).
template <typename T>
__device__ __forceinline__ T ppmx_iface(T a, T b, T c, T d) {
  const T f = T(0.5) * (b + c) - ((a - b) + (d - c)) / T(12);
  const T g = T(0.5) * (b + c) - ppmx_lim3(T(3) * (b - T(2) * f + c), a - T(2) * b + c, b - T(2) * c + d) / T(6);
  return (f - b) * (c - f) < T(0) ? g : f;
}

// Edges (aL, aR) of the cell w2 of (w0..w4) from its interface values: at an
// extremum both edge offsets are scaled by limited / unlimited curvature,
// elsewhere an offset larger than twice the other is cut to twice it.
template <typename T>
__device__ __forceinline__ void ppmx_cell(T w0, T w1, T w2, T w3, T w4, T& aL, T& aR) {
  const T dm = w2 - aL, dp = aR - w2;
  const bool ext = dm * dp <= T(0) || (w3 - w2) * (w2 - w1) <= T(0);
  const T d2 = T(6) * (aL + aR - T(2) * w2);
  const T lim = ppmx_lim4(d2, w1 - T(2) * w2 + w3, w0 - T(2) * w1 + w2, w2 - T(2) * w3 + w4);
  // a true division: d2 can be tiny (a curvature of velocity noise), where
  // a reciprocal of a subnormal would overflow
  const T ratio = d2 != T(0) ? lim / d2 : T(0);
  const T eL = w2 - ratio * dm, eR = w2 + ratio * dp;
  const T mR = fabs(dp) >= T(2) * fabs(dm) ? w2 + T(2) * dm : aR;
  const T mL = fabs(dm) >= T(2) * fabs(dp) ? w2 - T(2) * dp : aL;
  aL = ext ? eL : mL;
  aR = ext ? eR : mR;
}

// --------------------------------------------------------------- HLLC
// Toro-Spruce-Speares HLLC with pressure-based (PVRS) wave speeds (Toro's
// textbook, Ch. 10). States are [rho, u_n, u_t1, u_t2, u_g]; p = (gamma-1) u_g.
// Flux out: [mass, normal momentum, t1 momentum, t2 momentum, energy].
// Selection: S_L >= 0 -> F_L; S* >= 0 -> F*_L; S_R > 0 -> F*_R; else F_R.
template <typename T>
struct Gas {
  T gamma, gm1, cq;  // cq = (gamma + 1) / (2 gamma)
};

// The q factor of the pressure-based speeds is folded into one root:
// a_K q_K = sqrt(gamma/rho_K * max(p_K, p_K + cq (p* - p_K))), which equals
// a_K when p* <= p_K. The star state uses one reciprocal r = 1/(S_K - S*):
// fac = m_K r and p_K/m_K * fac = p_K r, with m_K = rho_K (S_K - u_K).
template <typename T>
__device__ __forceinline__ void hllc(const Gas<T>& g, T rl, T ul, T vl, T wl, T ugl, T rr,
                                     T ur, T vr, T wr, T ugr, T f[5]) {
  const T pl = g.gm1 * ugl, pr = g.gm1 * ugr;
  const T el = ugl + T(0.5) * rl * ((ul * ul + vl * vl) + wl * wl);
  const T er = ugr + T(0.5) * rr * ((ur * ur + vr * vr) + wr * wr);
  const T il = rcp(rl), ir = rcp(rr);
  const T gil = g.gamma * il, gir = g.gamma * ir;
  const T al = rsqrt_(gil * pl), ar = rsqrt_(gir * pr);

  const T ppv = T(0.5) * (pl + pr) - T(0.5) * (ur - ul) * (T(0.5) * (rl + rr)) * (T(0.5) * (al + ar));
  const T ps = fmax(ppv, T(0));
  const T sl = ul - rsqrt_(gil * fmax(pl, pl + g.cq * (ps - pl)));
  const T sr = ur + rsqrt_(gir * fmax(pr, pr + g.cq * (ps - pr)));
  const T ml = rl * (sl - ul), mr = rr * (sr - ur);
  const T sst = ((pr - pl) + ml * ul - mr * ur) * rcp(ml - mr);

  const bool c1 = sl >= T(0), c2 = sst >= T(0), c3 = sr > T(0);
  const bool useL = c1 || c2;                 // side K of the selected flux
  const bool direct = c1 || (!c2 && !c3);     // F_K itself, no star state

  const T rk = useL ? rl : rr, uk = useL ? ul : ur, vk = useL ? vl : vr;
  const T wk = useL ? wl : wr, pk = useL ? pl : pr, ek = useL ? el : er;
  const T sk = useL ? sl : sr, mk = useL ? ml : mr, ik = useL ? il : ir;

  const T mu = rk * uk;
  const T fk0 = mu, fk1 = mu * uk + pk, fk2 = mu * vk, fk3 = mu * wk, fk4 = uk * (ek + pk);

  const T rs = rcp(sk - sst);
  const T fac = mk * rs;
  const T us0 = fac, us1 = fac * sst, us2 = fac * vk, us3 = fac * wk;
  const T us4 = fac * (ek * ik + (sst - uk) * sst) + (sst - uk) * pk * rs;
  f[0] = direct ? fk0 : fk0 + sk * (us0 - rk);
  f[1] = direct ? fk1 : fk1 + sk * (us1 - mu);
  f[2] = direct ? fk2 : fk2 + sk * (us2 - rk * vk);
  f[3] = direct ? fk3 : fk3 + sk * (us3 - rk * wk);
  f[4] = direct ? fk4 : fk4 + sk * (us4 - ek);
}

// Local Lax-Friedrichs flux, same state and flux ordering as hllc(): the mean
// of the physical fluxes minus half the largest signal speed
// max(|u_L| + c_L, |u_R| + c_R) times the jump in the conserved state.
template <typename T>
__device__ __forceinline__ void llf(const Gas<T>& g, T rl, T ul, T vl, T wl, T ugl, T rr, T ur,
                                    T vr, T wr, T ugr, T f[5]) {
  const T pl = g.gm1 * ugl, pr = g.gm1 * ugr;
  const T el = ugl + T(0.5) * rl * ((ul * ul + vl * vl) + wl * wl);
  const T er = ugr + T(0.5) * rr * ((ur * ur + vr * vr) + wr * wr);
  const T a = fmax(fabs(ul) + rsqrt_(g.gamma * pl * rcp(rl)), fabs(ur) + rsqrt_(g.gamma * pr * rcp(rr)));
  const T ml = rl * ul, mr = rr * ur;
  f[0] = T(0.5) * (ml + mr) - T(0.5) * a * (rr - rl);
  f[1] = T(0.5) * ((ml * ul + pl) + (mr * ur + pr)) - T(0.5) * a * (mr - ml);
  f[2] = T(0.5) * (ml * vl + mr * vr) - T(0.5) * a * (rr * vr - rl * vl);
  f[3] = T(0.5) * (ml * wl + mr * wr) - T(0.5) * a * (rr * wr - rl * wl);
  f[4] = T(0.5) * (ul * (el + pl) + ur * (er + pr)) - T(0.5) * a * (er - el);
}

// --------------------------------------------------------- cons -> prim
// Sec. 3.1, Eq. 4: rho, v = M/rho, u_g = E - |M|^2/(2 rho). Floors act on the
// primitives only. `hit` counts a floor firing, `bad` a non-finite state or
// rho <= 0. Always FP64 (the kinetic-energy cancellation needs it).
struct Floors {
  double rho, ug;
};

__device__ __forceinline__ void c2p(const Floors& fl, const double u[5], double w[5], int& hit,
                                    int& bad) {
  bool b = !(u[0] > 0.0);
#pragma unroll
  for (int q = 0; q < 5; ++q) b = b || !isfinite(u[q]);
  bad |= b ? 1 : 0;
  double rho = u[0];
  const bool fr = rho < fl.rho;
  rho = fr ? fl.rho : rho;
  const double irho = rcp(rho);
  const double ke2 = (u[1] * u[1] + u[2] * u[2]) + u[3] * u[3];
  double ug = u[4] - (0.5 * ke2) * irho;
  const bool fu = ug < fl.ug;
  ug = fu ? fl.ug : ug;
  hit += (fr || fu) ? 1 : 0;
  w[0] = rho;
  w[1] = u[1] * irho;
  w[2] = u[2] * irho;
  w[3] = u[3] * irho;
  w[4] = ug;
}

// dx_d / (|v_d| + c_s) minimised over d for one cell (Sec. 3, Eq. 3).
__device__ __forceinline__ double cell_dt(const Floors& fl, double gamma, double gm1,
                                          const double dx[3], const double u[5]) {
  double w[5];
  int h = 0, b = 0;
  c2p(fl, u, w, h, b);
  const double cs = rsqrt_(gamma * (gm1 * w[4]) * rcp(w[0]));
  double m = dx[0] * rcp(fabs(w[1]) + cs);
  m = fmin(m, dx[1] * rcp(fabs(w[2]) + cs));
  m = fmin(m, dx[2] * rcp(fabs(w[3]) + cs));
  return m;
}

// Cell widths of block m (half the root widths on level 1).
__device__ __forceinline__ void block_dx(const DevProblem& P, int64_t m, double dx[3]) {
  const double s = (P.binfo && P.binfo[m * kLeafInts] != 0) ? 0.5 : 1.0;
  dx[0] = P.dx[0] * s;
  dx[1] = P.dx[1] * s;
  dx[2] = P.dx[2] * s;
}

// ------------------------------------------------------- block geometry
struct Geo {
  int bx, by, bz;
  int m;       // this tile's block
  int nb[6];   // neighbour block per face (-x,+x,-y,+y,-z,+z); -1 = outflow
  int lev;     // refinement level (0 without refinement)
  int nleaf;   // blocks below this index are leaves; above, ghost slabs
  int64_t bstride, vstride;
  int64_t sbase[6];  // per face with a ghost slab across: offset of that slab's
                     // packed cells (variable 0) in a register
};

// UNIFORM: m is the same in every lane of the wave (the stage kernel's tile
// block), which lets the leaf table's entries live in scalar registers. SMR:
// the mesh may be refined (false only in stage kernels launched for uniform
// meshes alone).
template <bool UNIFORM = false, bool SMR = true>
__device__ __forceinline__ void geo_init(Geo& g, const DevProblem& P, int m) {
  g.bx = P.bx;
  g.by = P.by;
  g.bz = P.bz;
  g.m = m;
  g.bstride = P.bstride;
  g.vstride = P.vstride;
  g.lev = 0;
  g.nleaf = P.nblocks;
  if (SMR && P.binfo) {  // refined mesh: the leaf table (a slab stands in for a level change)
    const int32_t* b = P.binfo + (int64_t)m * kLeafInts;
    g.lev = UNIFORM ? __builtin_amdgcn_readfirstlane(b[0]) : b[0];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      g.nb[f] = UNIFORM ? __builtin_amdgcn_readfirstlane(b[1 + f]) : b[1 + f];
      // slabs are packed 2^slab_k2 to a block after the leaves (DevProblem::slab_cells)
      const int vb = g.nb[f] - P.nblocks;
      g.sbase[f] = (int64_t)(P.nblocks + (vb >> P.slab_k2)) * P.bstride +
                   (int64_t)(vb & ((1 << P.slab_k2) - 1)) * P.slab_cells;
    }
    return;
  }
  const int nbx = P.nbx, nby = P.nby, nbz = P.nbz;
  const int mx = m % nbx, t = m / nbx, my = t % nby, mz = t / nby;
  const int sxy = nbx * nby;
  g.nb[0] = mx > 0 ? m - 1 : (P.periodic[0] ? m + (nbx - 1) : -1);
  g.nb[1] = mx < nbx - 1 ? m + 1 : (P.periodic[0] ? m - (nbx - 1) : -1);
  g.nb[2] = my > 0 ? m - nbx : (P.periodic[1] ? m + (nby - 1) * nbx : -1);
  g.nb[3] = my < nby - 1 ? m + nbx : (P.periodic[1] ? m - (nby - 1) * nbx : -1);
  g.nb[4] = mz > 0 ? m - sxy : (P.periodic[2] ? m + (nbz - 1) * sxy : -1);
  g.nb[5] = mz < nbz - 1 ? m + sxy : (P.periodic[2] ? m - (nbz - 1) * sxy : -1);
}

// Offset (in doubles, variable 0) of cell (i,j,k) given in this block's local
// coordinates, of which at most one may lie outside the block by <= its size:
// the ghost-zone rule of periodic / neighbour copies and outflow clamping.
// Across a level change the neighbour is a ghost slab (mb_out >= nleaf),
// whose layers next to the face are packed (DevProblem::slab_cells): then
// mb_out * bstride + the value returned is the cell's offset. SMR = false: a
// uniform mesh, no slabs.
template <bool SMR = true>
__device__ __forceinline__ int64_t ghost_local(const Geo& g, int i, int j, int k, int& mb_out) {
  int mb = g.m, f = 0;
  if (i < 0) {
    if (g.nb[0] >= 0) { mb = g.nb[0]; i += g.bx; f = 0; } else { i = 0; }
  } else if (i >= g.bx) {
    if (g.nb[1] >= 0) { mb = g.nb[1]; i -= g.bx; f = 1; } else { i = g.bx - 1; }
  }
  if (j < 0) {
    if (g.nb[2] >= 0) { mb = g.nb[2]; j += g.by; f = 2; } else { j = 0; }
  } else if (j >= g.by) {
    if (g.nb[3] >= 0) { mb = g.nb[3]; j -= g.by; f = 3; } else { j = g.by - 1; }
  }
  if (k < 0) {
    if (g.nb[4] >= 0) { mb = g.nb[4]; k += g.bz; f = 4; } else { k = 0; }
  } else if (k >= g.bz) {
    if (g.nb[5] >= 0) { mb = g.nb[5]; k -= g.bz; f = 5; } else { k = g.bz - 1; }
  }
  if (SMR && mb >= g.nleaf) {  // the ghost slab of this block's face f
    const int d = f >> 1;
    const int c = d == 0 ? i : (d == 1 ? j : k);
    const int n = d == 0 ? g.bx : (d == 1 ? g.by : g.bz);
    const int layer = (f & 1) ? c : n - 1 - c;  // 0 next to the face
    const int a1 = d == 0 ? j : i, a2 = d == 2 ? j : k;
    const int n1 = d == 0 ? g.by : g.bx, n2 = d == 2 ? g.by : g.bz;
    mb_out = mb;  // mb * bstride + the value returned is the slab cell's offset
    return g.sbase[f] - (int64_t)mb * g.bstride + ((int64_t)layer * n2 + a2) * n1 + a1;
  }
  mb_out = mb;
  return ((int64_t)k * g.by + j) * g.bx + i;
}

template <bool SMR = true>
__device__ __forceinline__ int64_t ghost_off(const Geo& g, int i, int j, int k) {
  int mb;
  const int64_t l = ghost_local<SMR>(g, i, j, k, mb);
  return (int64_t)mb * g.bstride + l;
}

// ghost_off for a cell of this block's column (i, j) at a plane k outside the
// block (below or above it by <= bz): only the z faces are crossed, so the
// whole choice is wave-uniform when k is.
template <bool SMR = true>
__device__ __forceinline__ int64_t ghost_off_z(const Geo& g, int i, int j, int k) {
  const bool up = k >= g.bz;
  const int nb = up ? g.nb[5] : g.nb[4];
  if (nb < 0) return (int64_t)g.m * g.bstride + ((int64_t)(up ? g.bz - 1 : 0) * g.by + j) * g.bx + i;
  const int kk = up ? k - g.bz : k + g.bz;
  if (SMR && nb >= g.nleaf) {  // the ghost slab of this block's z face
    const int layer = up ? kk : g.bz - 1 - kk;
    return (up ? g.sbase[5] : g.sbase[4]) + ((int64_t)layer * g.by + j) * g.bx + i;
  }
  return (int64_t)nb * g.bstride + ((int64_t)kk * g.by + j) * g.bx + i;
}

// ghost_off for a cell of plane k (inside the block) of which i or j (not
// both) may lie outside the block by <= its size.
template <bool SMR = true>
__device__ __forceinline__ int64_t ghost_off_xy(const Geo& g, int i, int j, int k) {
  int mb = g.m, f = -1;
  if (i < 0) {
    if (g.nb[0] >= 0) { mb = g.nb[0]; i += g.bx; f = 0; } else { i = 0; }
  } else if (i >= g.bx) {
    if (g.nb[1] >= 0) { mb = g.nb[1]; i -= g.bx; f = 1; } else { i = g.bx - 1; }
  }
  if (j < 0) {
    if (g.nb[2] >= 0) { mb = g.nb[2]; j += g.by; f = 2; } else { j = 0; }
  } else if (j >= g.by) {
    if (g.nb[3] >= 0) { mb = g.nb[3]; j -= g.by; f = 3; } else { j = g.by - 1; }
  }
  if (SMR && mb >= g.nleaf) {  // the ghost slab of this block's x or y face f
    const bool x = f < 2;
    const int c = x ? i : j, n = x ? g.bx : g.by;
    const int layer = (f & 1) ? c : n - 1 - c;
    const int a1 = x ? j : i, n1 = x ? g.by : g.bx;
    return g.sbase[f] + ((int64_t)layer * g.bz + k) * n1 + a1;
  }
  return (int64_t)mb * g.bstride + ((int64_t)k * g.by + j) * g.bx + i;
}

__device__ __forceinline__ void load5(const double* __restrict__ base, int64_t off, int64_t vs,
                                      double u[5]) {
#pragma unroll
  for (int q = 0; q < 5; ++q) u[q] = __builtin_nontemporal_load(base + off + q * vs);
}

__device__ __forceinline__ void load5c(const double* __restrict__ base, int64_t off, int64_t vs,
                                       double u[5]) {
#pragma unroll
  for (int q = 0; q < 5; ++q) u[q] = base[off + q * vs];
}

// --------------------------------------------------------- z-march queues
// Per-column register state of the z sweep. PLM: the face k+1/2 needs cells
// k-1..k+2; PPM4: cells k-2..k+3.
template <int RECON, typename T>
struct ZQueue;

template <typename T>
struct ZQueue<0, T> {       // PLM
  T w0[5], w1[5];           // primitives at k and k+1
  T s0[5];                  // half the limited slope at k
  double fm[5];             // z-flux through the face k-1/2
};

template <typename T>
struct ZQueue<1, T> {       // PPM4
  T w0[5], w1[5], w2[5];    // primitives at k, k+1, k+2
  T dm1[5];                 // limited slope at k+1
  T a1[5];                  // interface value at k+1/2
  T ar0[5];                 // monotonised right edge of cell k
  double fm[5];
};

template <typename T>
struct ZQueue<2, T> {       // WENO-Z
  T wm[5], w0[5], w1[5], w2[5];  // primitives at k-1, k, k+1, k+2
  T ar0[5];                 // right face value of cell k
  double fm[5];
};

template <typename T>
struct ZQueue<3, T> {       // PPMX
  T wm[5], w0[5], w1[5], w2[5];  // primitives at k-1, k, k+1, k+2
  T a1[5];                  // limited interface value at k+1/2
  T ar0[5];                 // right edge of cell k
  double fm[5];
};

template <typename T>
__device__ __forceinline__ void zflux(const Gas<T>& g, const T wl[5], const T wr[5], double f[5]) {
  // z-normal: (n, t1, t2) = (vz, vx, vy)
  T h[5];
  hllc(g, wl[0], wl[3], wl[1], wl[2], wl[4], wr[0], wr[3], wr[1], wr[2], wr[4], h);
  f[0] = (double)h[0];
  f[3] = (double)h[1];
  f[1] = (double)h[2];
  f[2] = (double)h[3];
  f[4] = (double)h[4];
}

// ------------------------------------------------------------ one face
// Flux through the face between LDS cells (base - STR) and base along
// direction DIR (0 = x, 1 = y), in conserved-variable order. PLM reads two
// cells on each side, PPM4, PPMX and WENO-Z three.
template <int RECON, int DIR, typename T, int STR, int PLANE>
__device__ __forceinline__ void face_flux(const Gas<T>& gas, const T* __restrict__ sW, int base,
                                          T out[5]) {
  T wl[5], wr[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const T* s = sW + v * PLANE + base;
    if constexpr (RECON == 0) {
      const T c0 = s[-2 * STR], c1 = s[-STR], c2 = s[0], c3 = s[STR];
      wl[v] = c1 + plm_half_slope(c0, c1, c2);
      wr[v] = c2 - plm_half_slope(c1, c2, c3);
    } else if constexpr (RECON == 2) {
      const T c0 = s[-3 * STR], c1 = s[-2 * STR], c2 = s[-STR];
      const T c3 = s[0], c4 = s[STR], c5 = s[2 * STR];
      wl[v] = weno_right(c0, c1, c2, c3, c4);  // right face of cell c2
      wr[v] = weno_right(c5, c4, c3, c2, c1);  // left face of cell c3 (mirrored)
    } else if constexpr (RECON == 3) {
      const T c0 = s[-3 * STR], c1 = s[-2 * STR], c2 = s[-STR];
      const T c3 = s[0], c4 = s[STR], c5 = s[2 * STR];
      const T im = ppmx_iface(c0, c1, c2, c3), i0 = ppmx_iface(c1, c2, c3, c4);
      const T ip = ppmx_iface(c2, c3, c4, c5);
      T l2 = im, r2 = i0, l3 = i0, r3 = ip;
      ppmx_cell(c0, c1, c2, c3, c4, l2, r2);
      ppmx_cell(c1, c2, c3, c4, c5, l3, r3);
      wl[v] = r2;
      wr[v] = l3;
    } else {
      const T c0 = s[-3 * STR], c1 = s[-2 * STR], c2 = s[-STR];
      const T c3 = s[0], c4 = s[STR], c5 = s[2 * STR];
      const T d1 = ppm_dm(c0, c1, c2), d2 = ppm_dm(c1, c2, c3);
      const T d3 = ppm_dm(c2, c3, c4), d4 = ppm_dm(c3, c4, c5);
      const T am = ppm_iface(c1, c2, d1, d2);
      const T a0 = ppm_iface(c2, c3, d2, d3);
      const T ap = ppm_iface(c3, c4, d3, d4);
      T l1 = am, r1 = a0;
      ppm_mono(c2, l1, r1);
      T l2 = a0, r2 = ap;
      ppm_mono(c3, l2, r2);
      wl[v] = r1;
      wr[v] = l2;
    }
  }
  T f[5];
  if constexpr (DIR == 0) {  // (n, t1, t2) = (vx, vy, vz)
    hllc(gas, wl[0], wl[1], wl[2], wl[3], wl[4], wr[0], wr[1], wr[2], wr[3], wr[4], f);
    out[0] = f[0]; out[1] = f[1]; out[2] = f[2]; out[3] = f[3]; out[4] = f[4];
  } else {                   // (n, t1, t2) = (vy, vz, vx)
    hllc(gas, wl[0], wl[2], wl[3], wl[1], wl[4], wr[0], wr[2], wr[3], wr[1], wr[4], f);
    out[0] = f[0]; out[2] = f[1]; out[3] = f[2]; out[1] = f[3]; out[4] = f[4];
  }
}

// A level-0 leaf with a ghost slab on some face (finer leaves across): the
// flux correction changes its cells on those faces after each stage.
__device__ __forceinline__ bool smr_cf_leaf(const Geo& g, int nblocks) {
  return g.lev == 0 && (g.nb[0] >= nblocks || g.nb[1] >= nblocks || g.nb[2] >= nblocks ||
                        g.nb[3] >= nblocks || g.nb[4] >= nblocks || g.nb[5] >= nblocks);
}

// Bit 2 d + side set when that face of cell (i,j,k) of a level-0 leaf is a
// level face: the cell lies on the block face and finer leaves are across
// (a ghost slab stands in for them).
__device__ __forceinline__ int level_faces(const Geo& g, int nblocks, int i, int j, int k) {
  int b = 0;
  if (i == 0 && g.nb[0] >= nblocks) b |= 1;
  if (i == g.bx - 1 && g.nb[1] >= nblocks) b |= 2;
  if (j == 0 && g.nb[2] >= nblocks) b |= 4;
  if (j == g.by - 1 && g.nb[3] >= nblocks) b |= 8;
  if (k == 0 && g.nb[4] >= nblocks) b |= 16;
  if (k == g.bz - 1 && g.nb[5] >= nblocks) b |= 32;
  return b;
}

// FOFC flag of the cell (i,j,k) in block-local coordinates (ghost rule of
// ghost_local); a cell across a level change (in a ghost slab) counts as not
// flagged: FOFC replaces fluxes within one level only.
__device__ __forceinline__ bool flag_at(const DevProblem& P, const Geo& g, int i, int j, int k) {
  int mb;
  const int64_t l = ghost_local(g, i, j, k, mb);
  return mb < P.nblocks && P.flags[(int64_t)mb * g.vstride + l] != 0;
}

// -------------------------------------------------------------- the stage
// A pointer that is the same in every lane, moved to scalar registers. The
// compiler does not prove the stage's register pointers uniform (they come
// from a table indexed by the batch entry) and otherwise keeps them in vector
// registers, which costs registers, spills in the larger variants and a
// looser load schedule.
template <typename P>
__device__ __forceinline__ P* uniform_ptr(P* p) {
  const unsigned long long v = (unsigned long long)p;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return (P*)(((unsigned long long)hi << 32) | lo);
}

// STAGE 1 (stages without a step-start term, never a step's last):
// dst = src + c dt L(src). STAGE 2 (the others): dst = a U + b src +
// c dt L(src). Registers and weights come from rk_stage_of (RK2:
// V = U + dt L(U), then U = U/2 + V/2 + dt L(V)/2; RK3 and RK4 in its
// table). The last stage of a problem also reduces the minimum of
// dx_d/lambda_d over its new state for the next time step.
template <int RECON, typename T, int TX, int TY, int WPE, int STAGE, bool SMR>
__global__ void __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(WPE)))
k_stage(const StageArgs a) {
  constexpr int NG = RECON == 0 ? 2 : 3;
  constexpr int NT = TX * TY;
  constexpr int SX = TX + 2 * NG;
  constexpr int SY = TY + 2 * NG;
  constexpr int PLANE = SX * SY;
  constexpr int NXF = (TX + 1) * TY;
  constexpr int NYF = TX * (TY + 1);
  constexpr int NF = NXF + NYF;
  constexpr int NXFP = (NXF + kWave - 1) / kWave * kWave;
  constexpr int NFP = NXFP + NYF;
  constexpr int NHX = 2 * NG * TY;
  constexpr int NH = NHX + 2 * NG * TX;
  constexpr int NWAVE = NT / kWave;
  static_assert(NT % kWave == 0, "tile must be whole wavefronts");

  __shared__ T sW[5 * PLANE];
  __shared__ T sF[5 * NF];
  __shared__ unsigned long long sRed[NWAVE];

  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;

  for (int L = xcd_remap(blockIdx.x, gridDim.x); L < a.ntiles; L += gridDim.x) {
    // ---- locate problem, block and tile (uniform across the workgroup)
    int q = 0;
    while (q + 1 < a.nprob && a.e[q + 1].tile0 <= L) ++q;
    const BatchEntry E = a.e[q];
    const DevProblem& P = *E.p;
    const int loc = L - E.tile0;
    const int per_blk = E.ntx * E.nty * E.ntz;
    const int m = loc / per_blk;
    int r = loc - m * per_blk;
    const int tzi = r / (E.ntx * E.nty);
    r -= tzi * (E.ntx * E.nty);
    const int tyi = r / E.ntx;
    const int txi = r - tyi * E.ntx;

    Geo geo;
    geo_init<true, SMR>(geo, P, m);
    const int i0 = txi * TX, j0 = tyi * TY, k0 = tzi * E.kc;
    const int nxv = min(TX, geo.bx - i0), nyv = min(TY, geo.by - j0);
    const int kend = min(k0 + E.kc, geo.bz);
    const bool own = tx < nxv && ty < nyv;
    const int gi = i0 + tx, gj = j0 + ty;  // owned column, block-local

    const RkStage& rs = P.rk[E.stage - 1];
    const double* __restrict__ Sin = uniform_ptr(rs.src);
    double* __restrict__ Out = uniform_ptr(rs.dst);
    const double* __restrict__ U0 = uniform_ptr((const double*)P.U);
    const double ca = rs.a, cb = rs.b, cc = rs.c;
    const bool last = STAGE == 2 && E.stage == P.nstages;  // uniform over the workgroup
    const int64_t vs = geo.vstride;

    const double gamma = P.gamma, gm1 = gamma - 1.0;
    const Gas<T> gas{T(gamma), T(gm1), T((gamma + 1.0) / (2.0 * gamma))};
    const Floors fl{P.rho_floor, P.p_floor / gm1};
    const double dt = P.cfl * __longlong_as_double((long long)P.dtmin[E.parity]);
    // a level-1 block has half the root widths: scaling by a power of two
    // commutes with rounding (and with the minimum of the time step), so the
    // root widths are used and the results scaled once
    const double isc = SMR && geo.lev ? 2.0 : 1.0, dsc = SMR && geo.lev ? 0.5 : 1.0;
    // the tiles of a coarse leaf next to finer ones leave the time step to
    // k_smr_dt, which runs after the flux correction has changed the leaf
    const bool last_dt = last && !(SMR && P.binfo && smr_cf_leaf(geo, P.nblocks));
    const double idx = (1.0 / P.dx[0]) * isc, idy = (1.0 / P.dx[1]) * isc, idz = (1.0 / P.dx[2]) * isc;
    const bool count = (E.flags & 1) != 0;

    // the slot this step reduces into; a one-stage step has no earlier
    // launch to clear it, so the copy that ends its previous step does
    if (E.stage == 1 && P.nstages > 1 && loc == 0 && tid == 0) P.dtmin[E.parity ^ 1] = kInfBits;
    const bool fofc = P.fofc && count;
    if (fofc && loc == 0 && tid == 0) {  // fold the counter of two stages ago
      *P.fofc_total = *P.fofc_total + P.fofc_cnt[(E.seq + 1) & 1];
      P.fofc_cnt[(E.seq + 1) & 1] = 0ull;
    }

    int hits = 0, bad = 0;
    double mydt = __longlong_as_double((long long)kInfBits);

    // column offset of the owned cell in plane k (valid for 0 <= k < bz)
    const int64_t col0 = (int64_t)m * geo.bstride + (int64_t)gj * geo.bx + gi;
    const int64_t pstride = (int64_t)geo.by * geo.bx;

    auto col_load = [&](int k, double u[5]) {
      const int64_t off = (k >= 0 && k < geo.bz) ? col0 + k * pstride : ghost_off_z<SMR>(geo, gi, gj, k);
      load5c(Sin, off, vs, u);
    };
    auto to_prim = [&](const double u[5], T w[5], int k) {
      double wd[5];
      int h = 0, b = 0;
      c2p(fl, u, wd, h, b);
      if (k >= k0 && k < kend) {  // interior cell of this tile: count once
        hits += h;
        bad |= b;
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) w[v] = (T)wd[v];
    };

    ZQueue<RECON, T> zq;
    if (own) {
      if constexpr (RECON == 0) {
        double u[5];
        T wa[5], wb[5], wc[5], wd[5];
        col_load(k0 - 2, u); to_prim(u, wa, k0 - 2);
        col_load(k0 - 1, u); to_prim(u, wb, k0 - 1);
        col_load(k0, u); to_prim(u, wc, k0);
        col_load(k0 + 1, u); to_prim(u, wd, k0 + 1);
        T wl[5], wr[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          const T sb = plm_half_slope(wa[v], wb[v], wc[v]);
          const T sc = plm_half_slope(wb[v], wc[v], wd[v]);
          wl[v] = wb[v] + sb;
          wr[v] = wc[v] - sc;
          zq.w0[v] = wc[v];
          zq.w1[v] = wd[v];
          zq.s0[v] = sc;
        }
        zflux(gas, wl, wr, zq.fm);
      } else if constexpr (RECON == 3) {
        double u[5];
        T c[6][5];
#pragma unroll
        for (int o = 0; o < 6; ++o) {
          col_load(k0 - 3 + o, u);
          to_prim(u, c[o], k0 - 3 + o);
        }
        T wl[5], wr[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          const T im = ppmx_iface(c[0][v], c[1][v], c[2][v], c[3][v]);  // k0-3/2
          const T i0 = ppmx_iface(c[1][v], c[2][v], c[3][v], c[4][v]);  // k0-1/2
          const T ip = ppmx_iface(c[2][v], c[3][v], c[4][v], c[5][v]);  // k0+1/2
          T l2 = im, r2 = i0, l3 = i0, r3 = ip;
          ppmx_cell(c[0][v], c[1][v], c[2][v], c[3][v], c[4][v], l2, r2);  // cell k0-1
          ppmx_cell(c[1][v], c[2][v], c[3][v], c[4][v], c[5][v], l3, r3);  // cell k0
          wl[v] = r2;
          wr[v] = l3;
          zq.ar0[v] = r3;
          zq.a1[v] = ip;
          zq.wm[v] = c[2][v];
          zq.w0[v] = c[3][v];
          zq.w1[v] = c[4][v];
          zq.w2[v] = c[5][v];
        }
        zflux(gas, wl, wr, zq.fm);
      } else if constexpr (RECON == 2) {
        double u[5];
        T c[6][5];
#pragma unroll
        for (int o = 0; o < 6; ++o) {
          col_load(k0 - 3 + o, u);
          to_prim(u, c[o], k0 - 3 + o);
        }
        T wl[5], wr[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          wl[v] = weno_right(c[0][v], c[1][v], c[2][v], c[3][v], c[4][v]);  // cell k0-1
          T lk;
          weno_cell(c[1][v], c[2][v], c[3][v], c[4][v], c[5][v], lk, zq.ar0[v]);  // cell k0
          wr[v] = lk;
          zq.wm[v] = c[2][v];
          zq.w0[v] = c[3][v];
          zq.w1[v] = c[4][v];
          zq.w2[v] = c[5][v];
        }
        zflux(gas, wl, wr, zq.fm);
      } else {
        double u[5];
        T c[6][5];
#pragma unroll
        for (int o = 0; o < 6; ++o) {
          col_load(k0 - 3 + o, u);
          to_prim(u, c[o], k0 - 3 + o);
        }
        T wl[5], wr[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          // slopes at k0-2 .. k0+1 (cells c[1..4])
          const T d1 = ppm_dm(c[0][v], c[1][v], c[2][v]);
          const T d2 = ppm_dm(c[1][v], c[2][v], c[3][v]);
          const T d3 = ppm_dm(c[2][v], c[3][v], c[4][v]);
          const T d4 = ppm_dm(c[3][v], c[4][v], c[5][v]);
          const T am = ppm_iface(c[1][v], c[2][v], d1, d2);  // k0-3/2
          const T a0 = ppm_iface(c[2][v], c[3][v], d2, d3);  // k0-1/2
          const T ap = ppm_iface(c[3][v], c[4][v], d3, d4);  // k0+1/2
          T l1 = am, r1 = a0;                                 // cell k0-1
          ppm_mono(c[2][v], l1, r1);
          T l2 = a0, r2 = ap;                                 // cell k0
          ppm_mono(c[3][v], l2, r2);
          wl[v] = r1;
          wr[v] = l2;
          zq.w0[v] = c[3][v];
          zq.w1[v] = c[4][v];
          zq.w2[v] = c[5][v];
          zq.dm1[v] = d4;
          zq.a1[v] = ap;
          zq.ar0[v] = r2;
        }
        zflux(gas, wl, wr, zq.fm);
      }
    }

    for (int k = k0; k < kend; ++k) {
      // ---- primitives of plane k into LDS: owned cells from the queue,
      //      ghost cells of the tile from neighbours / boundary conditions
      if (own) {
#pragma unroll
        for (int v = 0; v < 5; ++v) sW[v * PLANE + (ty + NG) * SX + (tx + NG)] = zq.w0[v];
      }
      for (int h = tid; h < NH; h += NT) {
        int li, lj;
        bool ok;
        if (h < NHX) {
          const int side = h / (NG * TY);
          const int rem = h - side * (NG * TY);
          lj = rem / NG;
          const int g = rem - lj * NG;
          li = side ? nxv + g : g - NG;
          ok = lj < nyv;
        } else {
          const int hh = h - NHX;
          const int side = hh / (NG * TX);
          const int rem = hh - side * (NG * TX);
          const int g = rem / TX;
          li = rem - g * TX;
          lj = side ? nyv + g : g - NG;
          ok = li < nxv;
        }
        if (ok) {
          double u[5], wd[5];
          load5c(Sin, ghost_off_xy<SMR>(geo, i0 + li, j0 + lj, k), vs, u);
          int hh = 0, bb = 0;
          c2p(fl, u, wd, hh, bb);
#pragma unroll
          for (int v = 0; v < 5; ++v) sW[v * PLANE + (lj + NG) * SX + (li + NG)] = (T)wd[v];
        }
      }
      __syncthreads();

      // ---- x- and y-faces of plane k, spread over all threads. The x-face
      //      items are padded to whole wavefronts so that every wavefront
      //      runs a single direction.
      for (int w = tid; w < NFP; w += NT) {
        if (w < NXFP) {
          const int fj = w / (TX + 1);
          const int fi = w - fj * (TX + 1);
          if (w < NXF && fi <= nxv && fj < nyv) {
            T f[5];
            face_flux<RECON, 0, T, 1, PLANE>(gas, sW, (fj + NG) * SX + (fi + NG), f);
#pragma unroll
            for (int v = 0; v < 5; ++v) sF[v * NF + w] = f[v];
          }
        } else {
          const int ww = w - NXFP;
          const int fj = ww / TX;
          const int fi = ww - fj * TX;
          if (fi < nxv && fj <= nyv) {
            T f[5];
            face_flux<RECON, 1, T, SX, PLANE>(gas, sW, (fj + NG) * SX + (fi + NG), f);
#pragma unroll
            for (int v = 0; v < 5; ++v) sF[v * NF + NXF + ww] = f[v];
          }
        }
      }

      // ---- z-face k+1/2 of the owned column (registers only)
      double fz[5];
      if (own) {
        double un[5];
        col_load(k + (RECON == 0 ? 2 : 3), un);
        if constexpr (RECON == 0) {
          T w2[5];
          to_prim(un, w2, k + 2);
          T wl[5], wr[5], s1[5];
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            s1[v] = plm_half_slope(zq.w0[v], zq.w1[v], w2[v]);
            wl[v] = zq.w0[v] + zq.s0[v];
            wr[v] = zq.w1[v] - s1[v];
          }
          zflux(gas, wl, wr, fz);
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            zq.w0[v] = zq.w1[v];
            zq.w1[v] = w2[v];
            zq.s0[v] = s1[v];
          }
        } else if constexpr (RECON == 3) {
          T w3[5];
          to_prim(un, w3, k + 3);
          T wl[5], wr[5], r1[5], a2[5];
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            a2[v] = ppmx_iface(zq.w0[v], zq.w1[v], zq.w2[v], w3[v]);  // k+3/2
            T l1 = zq.a1[v];
            r1[v] = a2[v];
            ppmx_cell(zq.wm[v], zq.w0[v], zq.w1[v], zq.w2[v], w3[v], l1, r1[v]);  // cell k+1
            wl[v] = zq.ar0[v];
            wr[v] = l1;
          }
          zflux(gas, wl, wr, fz);
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            zq.wm[v] = zq.w0[v];
            zq.w0[v] = zq.w1[v];
            zq.w1[v] = zq.w2[v];
            zq.w2[v] = w3[v];
            zq.a1[v] = a2[v];
            zq.ar0[v] = r1[v];
          }
        } else if constexpr (RECON == 2) {
          T w3[5];
          to_prim(un, w3, k + 3);
          T wl[5], wr[5], r1[5];
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            T l1;
            weno_cell(zq.wm[v], zq.w0[v], zq.w1[v], zq.w2[v], w3[v], l1, r1[v]);  // cell k+1
            wl[v] = zq.ar0[v];
            wr[v] = l1;
          }
          zflux(gas, wl, wr, fz);
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            zq.wm[v] = zq.w0[v];
            zq.w0[v] = zq.w1[v];
            zq.w1[v] = zq.w2[v];
            zq.w2[v] = w3[v];
            zq.ar0[v] = r1[v];
          }
        } else {
          T w3[5];
          to_prim(un, w3, k + 3);
          T wl[5], wr[5], d2[5], a2[5], r1[5];
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            d2[v] = ppm_dm(zq.w1[v], zq.w2[v], w3[v]);                 // slope at k+2
            a2[v] = ppm_iface(zq.w1[v], zq.w2[v], zq.dm1[v], d2[v]);    // k+3/2
            T l1 = zq.a1[v];
            r1[v] = a2[v];
            ppm_mono(zq.w1[v], l1, r1[v]);                              // cell k+1
            wl[v] = zq.ar0[v];
            wr[v] = l1;
          }
          zflux(gas, wl, wr, fz);
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            zq.w0[v] = zq.w1[v];
            zq.w1[v] = zq.w2[v];
            zq.w2[v] = w3[v];
            zq.dm1[v] = d2[v];
            zq.a1[v] = a2[v];
            zq.ar0[v] = r1[v];
          }
        }
      }
      __syncthreads();

      // ---- divergence and RK stage update of the owned cell
      if (own) {
        const int64_t off = col0 + k * pstride;
        const int wx = ty * (TX + 1) + tx;
        const int wy = NXF + ty * TX + tx;
        double uc[5], un0[5];
        load5c(Sin, off, vs, uc);
        if (STAGE == 2) load5(U0, off, vs, un0);
        double unew[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          const double fxm = (double)sF[v * NF + wx], fxp = (double)sF[v * NF + wx + 1];
          const double fym = (double)sF[v * NF + wy], fyp = (double)sF[v * NF + wy + TX];
          double l = -(fxp - fxm) * idx;
          l -= (fyp - fym) * idy;
          l -= (fz[v] - zq.fm[v]) * idz;
          if (STAGE == 1) {
            unew[v] = uc[v] + (cc * dt) * l;
          } else {
            unew[v] = (ca * un0[v] + cb * uc[v]) + (cc * dt) * l;
          }
          zq.fm[v] = fz[v];
        }
        bool flag = false;
        if (fofc) {  // first-order flux correction: flag a non-positive result
          // (every counted stage rewrites every flag, so no flag outlives
          // the stage that set it)
          const double ke2 = (unew[1] * unew[1] + unew[2] * unew[2]) + unew[3] * unew[3];
          const double pn = gm1 * (unew[4] - (0.5 * ke2) * rcp(unew[0]));
          flag = !(unew[0] > 0.0) || !(pn > 0.0);
          P.flags[(int64_t)m * geo.vstride + k * pstride + (int64_t)gj * geo.bx + gi] = flag ? 1 : 0;
          if (flag) atomicAdd(P.fofc_cnt + (E.seq & 1), 1ull);
        }
        // a flagged cell is recomputed from scratch by k_fofc_fix; skipping
        // its store keeps the step-start state in place for the last stage,
        // which updates U in place
        if (!flag) {
#pragma unroll
          for (int v = 0; v < 5; ++v) __builtin_nontemporal_store(unew[v], Out + off + v * vs);
        }
        if (last_dt) mydt = fmin(mydt, dsc * cell_dt(fl, gamma, gm1, P.dx, unew));
      }
    }

    // ---- per-tile reductions: floors, bad-state flag, time step
    if (count) {
      if (hits) atomicAdd(P.floor_hits, (unsigned long long)hits);
      if (bad) atomicOr(P.err, 1u);
    }
    if (last_dt) {
      unsigned long long b = (unsigned long long)__double_as_longlong(mydt);
#pragma unroll
      for (int s = kWave / 2; s > 0; s >>= 1) {
        const unsigned long long o = __shfl_xor(b, s, kWave);
        b = o < b ? o : b;
      }
      if ((tid & (kWave - 1)) == 0) sRed[tid / kWave] = b;
      __syncthreads();
      if (tid == 0) {
        unsigned long long mn = sRed[0];
        for (int wv = 1; wv < NWAVE; ++wv) mn = sRed[wv] < mn ? sRed[wv] : mn;
        atomicMin(P.dtmin + (E.parity ^ 1), mn);
      }
    }
    if (last && loc == 0 && tid == 0) *P.time = *P.time + dt;
    __syncthreads();  // LDS reuse by the next tile of this workgroup
  }
}

// ----------------------------------------------- first-order flux correction
// Primitive of the cell at block-local (i,j,k) (at most one coordinate outside
// the block), rounded to T exactly as the stage kernel rounds it.
template <typename T>
__device__ __forceinline__ void prim_at(const Geo& geo, const Floors& fl,
                                        const double* __restrict__ S, int i, int j, int k, T w[5]) {
  double u[5], wd[5];
  int h = 0, b = 0;
  load5c(S, ghost_off(geo, i, j, k), geo.vstride, u);
  c2p(fl, u, wd, h, b);
#pragma unroll
  for (int v = 0; v < 5; ++v) w[v] = (T)wd[v];
}

// The stage kernel's high-order flux and the first-order LLF flux through the
// face between the cells (i,j,k) - e_d and (i,j,k), in conserved order.
template <int RECON, typename T>
__device__ void face_pair(const Geo& geo, const Floors& fl, const Gas<T>& gas,
                          const double* __restrict__ S, int d, int i, int j, int k, T fho[5],
                          T flf[5]) {
  constexpr int NG = RECON == 0 ? 2 : 3;
  T c[2 * NG][5];
  const int di = d == 0, dj = d == 1, dk = d == 2;
#pragma unroll
  for (int o = 0; o < 2 * NG; ++o)
    prim_at(geo, fl, S, i + (o - NG) * di, j + (o - NG) * dj, k + (o - NG) * dk, c[o]);
  T wl[5], wr[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    if constexpr (RECON == 0) {
      wl[v] = c[1][v] + plm_half_slope(c[0][v], c[1][v], c[2][v]);
      wr[v] = c[2][v] - plm_half_slope(c[1][v], c[2][v], c[3][v]);
    } else if constexpr (RECON == 2) {
      wl[v] = weno_right(c[0][v], c[1][v], c[2][v], c[3][v], c[4][v]);
      wr[v] = weno_right(c[5][v], c[4][v], c[3][v], c[2][v], c[1][v]);
    } else if constexpr (RECON == 3) {
      const T im = ppmx_iface(c[0][v], c[1][v], c[2][v], c[3][v]);
      const T i0 = ppmx_iface(c[1][v], c[2][v], c[3][v], c[4][v]);
      const T ip = ppmx_iface(c[2][v], c[3][v], c[4][v], c[5][v]);
      T l2 = im, r2 = i0, l3 = i0, r3 = ip;
      ppmx_cell(c[0][v], c[1][v], c[2][v], c[3][v], c[4][v], l2, r2);
      ppmx_cell(c[1][v], c[2][v], c[3][v], c[4][v], c[5][v], l3, r3);
      wl[v] = r2;
      wr[v] = l3;
    } else {
      const T d1 = ppm_dm(c[0][v], c[1][v], c[2][v]), d2 = ppm_dm(c[1][v], c[2][v], c[3][v]);
      const T d3 = ppm_dm(c[2][v], c[3][v], c[4][v]), d4 = ppm_dm(c[3][v], c[4][v], c[5][v]);
      const T am = ppm_iface(c[1][v], c[2][v], d1, d2);
      const T a0 = ppm_iface(c[2][v], c[3][v], d2, d3);
      const T ap = ppm_iface(c[3][v], c[4][v], d3, d4);
      T l1 = am, r1 = a0;
      ppm_mono(c[2][v], l1, r1);
      T l2 = a0, r2 = ap;
      ppm_mono(c[3][v], l2, r2);
      wl[v] = r1;
      wr[v] = l2;
    }
  }
  const T* a = c[NG - 1];
  const T* b = c[NG];
  // normal and tangential velocity slots per direction: x (1,2,3), y (2,3,1), z (3,1,2)
  const int n = 1 + d, t1 = 1 + (d + 1) % 3, t2 = 1 + (d + 2) % 3;
  T f[5], g[5];
  hllc(gas, wl[0], wl[n], wl[t1], wl[t2], wl[4], wr[0], wr[n], wr[t1], wr[t2], wr[4], f);
  llf(gas, a[0], a[n], a[t1], a[t2], a[4], b[0], b[n], b[t1], b[t2], b[4], g);
  fho[0] = f[0]; fho[n] = f[1]; fho[t1] = f[2]; fho[t2] = f[3]; fho[4] = f[4];
  flf[0] = g[0]; flf[n] = g[1]; flf[t1] = g[2]; flf[t2] = g[3]; flf[4] = g[4];
}

// The LLF flux of the first-order states through the same face.
template <typename T>
__device__ void face_llf(const Geo& geo, const Floors& fl, const Gas<T>& gas,
                         const double* __restrict__ S, int d, int i, int j, int k, T out[5]) {
  const int di = d == 0, dj = d == 1, dk = d == 2;
  T a[5], b[5];
  prim_at(geo, fl, S, i - di, j - dj, k - dk, a);
  prim_at(geo, fl, S, i, j, k, b);
  const int n = 1 + d, t1 = 1 + (d + 1) % 3, t2 = 1 + (d + 2) % 3;
  T g[5];
  llf(gas, a[0], a[n], a[t1], a[t2], a[4], b[0], b[n], b[t1], b[t2], b[4], g);
  out[0] = g[0]; out[n] = g[1]; out[t1] = g[2]; out[t2] = g[3]; out[4] = g[4];
}

// One of the 4 fine fluxes (e: child offset along t1 + 2 x along t2) through
// face (d, side) of level-0 leaf q at the face cell (a1, a2) along the
// tangential axes t1 < t2, formed by the fine leaf across exactly as its
// stage kernel forms it; with `use_flags`, the LLF flux instead when the fine
// cell next to the face is flagged (FOFC on the fine level).
template <int RECON, typename T>
__device__ void fine_face(const DevProblem& P, const Floors& fl, const Gas<T>& gas,
                          const double* __restrict__ S, int q, int d, int side, int a1, int a2,
                          int e, bool use_flags, double out[5]) {
  const int bd[3] = {P.bx, P.by, P.bz};
  const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
  const int32_t* bq = P.binfo + (int64_t)q * kLeafInts;
  const int n1 = 2 * P.nroot[d] * bd[d];
  int g3[3], lf[3];
  g3[d] = side ? 2 * (bq[7 + d] + 1) * bd[d] : 2 * bq[7 + d] * bd[d] - 1;
  g3[d] = (g3[d] + n1) % n1;
  g3[t1] = 2 * (bq[7 + t1] * bd[t1] + a1) + (e & 1);
  g3[t2] = 2 * (bq[7 + t2] * bd[t2] + a2) + (e >> 1);
  const int lx = g3[0] / bd[0], ly = g3[1] / bd[1], lz = g3[2] / bd[2];
  const int r = (lx >> 1) + P.nroot[0] * ((ly >> 1) + P.nroot[1] * (lz >> 1));
  const int qf = P.rinfo[2 * r + 1] + (lx & 1) + 2 * (ly & 1) + 4 * (lz & 1);
  lf[0] = g3[0] - lx * bd[0];
  lf[1] = g3[1] - ly * bd[1];
  lf[2] = g3[2] - lz * bd[2];
  // face_pair's cell index is the face's upper cell: the fine leaf's first
  // cell when the coarse face is an upper one, one past its last otherwise
  const int inner = side ? 0 : bd[d] - 1;
  lf[d] = side ? 0 : bd[d];
  Geo g;
  geo_init(g, P, qf);
  T fho[5], flf[5];
  face_pair<RECON, T>(g, fl, gas, S, d, lf[0], lf[1], lf[2], fho, flf);
  bool llf_here = false;
  if (use_flags) {
    int c3[3] = {lf[0], lf[1], lf[2]};
    c3[d] = inner;
    llf_here = P.flags[(int64_t)qf * P.vstride + ((int64_t)c3[2] * P.by + c3[1]) * P.bx + c3[0]] != 0;
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) out[v] = llf_here ? (double)flf[v] : (double)fho[v];
}

// Mean of the 4 fine fluxes through that face, summed in pairs.
template <int RECON, typename T>
__device__ void fine_face_mean(const DevProblem& P, const Floors& fl, const Gas<T>& gas,
                               const double* __restrict__ S, int q, int d, int side, int a1, int a2,
                               bool use_flags, double out[5]) {
  double f[4][5];
#pragma unroll 1
  for (int e = 0; e < 4; ++e) fine_face<RECON, T>(P, fl, gas, S, q, d, side, a1, a2, e, use_flags, f[e]);
#pragma unroll
  for (int v = 0; v < 5; ++v) out[v] = ((f[0][v] + f[1][v]) + (f[2][v] + f[3][v])) * 0.25;
}

// Before a correction pass: per unit of kFixPlanes planes of a leaf, whether
// any of its cells is flagged, and whether one on each of its four side faces
// is (so that k_fofc_fix can pass over the units with no flagged cell in them
// or next to them). Exits at once when nothing was flagged.
__global__ void __launch_bounds__(256) k_fofc_mark(const FixArgs a) {
  const FixEntry E = a.e[blockIdx.y];
  const DevProblem& P = *E.p;
  if (P.fofc_cnt[E.seq & 1] == 0ull) return;
  const int units = (P.bz + kFixPlanes - 1) / kFixPlanes;
  const int64_t plane = (int64_t)P.bx * P.by;
  __shared__ int acc;
  for (int w = blockIdx.x; w < P.nblocks * units; w += gridDim.x) {
    const int m = w / units, k0 = (w - m * units) * kFixPlanes;
    const int k1 = min(k0 + kFixPlanes, P.bz);
    const uint8_t* f = P.flags + (int64_t)m * P.vstride + k0 * plane;
    if (threadIdx.x == 0) acc = 0;
    __syncthreads();
    int bits = 0;
    for (int64_t r = threadIdx.x; r < (k1 - k0) * plane; r += blockDim.x) {
      if (!f[r]) continue;
      const int rem = (int)(r % plane), j = rem / P.bx, i = rem - j * P.bx;
      bits |= 1 | (i == 0 ? 2 : 0) | (i == P.bx - 1 ? 4 : 0) | (j == 0 ? 8 : 0) | (j == P.by - 1 ? 16 : 0);
    }
    if (bits) atomicOr(&acc, bits);
    __syncthreads();
    if (threadIdx.x == 0) P.fixmask[w] = (uint8_t)acc;
    __syncthreads();  // acc is reset for the next unit
  }
}

// Replace, for every cell flagged in this stage, the fluxes on all its faces by
// LLF fluxes of the first-order states. A flagged cell (whose store the stage
// kernel skipped) is recomputed from scratch with LLF fluxes on all six
// faces, so a non-finite high-order flux never enters it; an unflagged cell
// with flagged face neighbours adds c_s dt (F_LLF - F_HO) / dx of those faces
// to its stage result (c_s is the stage's weight of dt L; every F_HO it saw
// was finite, or its result would have been flagged). Exits at once when
// nothing was flagged. A problem's last stage also resets the time-step slot
// for k_fofc_dt.
template <int RECON, typename T>
__global__ void __launch_bounds__(256) k_fofc_fix(const FixArgs a) {
  const FixEntry E = a.e[blockIdx.y];
  const DevProblem& P = *E.p;
  if (P.fofc_cnt[E.seq & 1] == 0ull) return;
  const RkStage& rs = P.rk[E.stage - 1];
  if (E.last && blockIdx.x == 0 && threadIdx.x == 0) P.dtmin[E.parity ^ 1] = kInfBits;
  const double* __restrict__ S = rs.src;
  double* Out = rs.dst;  // is P.U itself in a problem's last stage (not for RK1)
  const double gamma = P.gamma, gm1 = gamma - 1.0;
  const Gas<T> gas{T(gamma), T(gm1), T((gamma + 1.0) / (2.0 * gamma))};
  const Floors fl{P.rho_floor, P.p_floor / gm1};
  const double dt = P.cfl * __longlong_as_double((long long)P.dtmin[E.parity]);
  const double cst = rs.c * dt;
  const int slabs = (P.bz + kFixPlanes - 1) / kFixPlanes;
  for (int w = blockIdx.x; w < P.nblocks * slabs; w += gridDim.x) {
    const int m = w / slabs, sl = w - m * slabs, k0 = sl * kFixPlanes;
    Geo geo;
    geo_init(geo, P, m);
    {  // a unit with no flagged cell in it or next to it changes nothing
      bool need = (P.fixmask[w] & 1) || (sl > 0 && (P.fixmask[w - 1] & 1)) ||
                  (sl + 1 < slabs && (P.fixmask[w + 1] & 1));
      // x and y neighbours (same planes): a flagged cell on their face towards this unit
      for (int f = 0; f < 4; ++f)
        need = need || (geo.nb[f] >= 0 && geo.nb[f] < P.nblocks &&
                        (P.fixmask[geo.nb[f] * slabs + sl] & (2 << (f ^ 1))));
      if (sl == 0 && geo.nb[4] >= 0 && geo.nb[4] < P.nblocks)
        need = need || (P.fixmask[geo.nb[4] * slabs + slabs - 1] & 1);
      if (sl + 1 == slabs && geo.nb[5] >= 0 && geo.nb[5] < P.nblocks) need = need || (P.fixmask[geo.nb[5] * slabs] & 1);
      if (!need) continue;
    }
    const double isc = geo.lev ? 2.0 : 1.0;  // a level-1 leaf has half the root widths
    const double id[3] = {(1.0 / P.dx[0]) * isc, (1.0 / P.dx[1]) * isc, (1.0 / P.dx[2]) * isc};
    const bool coarse_cf = P.binfo && smr_cf_leaf(geo, P.nblocks);
    const int k1 = min(k0 + kFixPlanes, geo.bz);
    const int64_t plane = (int64_t)geo.bx * geo.by;
    for (int64_t r = (int64_t)k0 * plane + threadIdx.x; r < (int64_t)k1 * plane; r += blockDim.x) {
      const int k = (int)(r / plane);
      const int rem = (int)(r - k * plane);
      const int j = rem / geo.bx, i = rem - j * geo.bx;
      const bool me = P.flags[(int64_t)m * geo.vstride + r] != 0;
      bool nb[6];
      nb[0] = flag_at(P, geo, i - 1, j, k);
      nb[1] = flag_at(P, geo, i + 1, j, k);
      nb[2] = flag_at(P, geo, i, j - 1, k);
      nb[3] = flag_at(P, geo, i, j + 1, k);
      nb[4] = flag_at(P, geo, i, j, k - 1);
      nb[5] = flag_at(P, geo, i, j, k + 1);
      if (!(me || nb[0] || nb[1] || nb[2] || nb[3] || nb[4] || nb[5])) continue;
      const int64_t off = (int64_t)m * geo.bstride + r;
      if (me) {
        // the stage formula with first-order LLF fluxes on every face,
        // divergence summed in x, y, z order as in the stage kernel; on a
        // level face of a level-0 cell the fine side's fluxes (after FOFC on
        // the fine level) stay
        const int lvf = coarse_cf ? level_faces(geo, P.nblocks, i, j, k) : 0;
        const int c3[3] = {i, j, k};
        double l[5];
        for (int d = 0; d < 3; ++d) {
          double fs[2][5];
          for (int s2 = 0; s2 < 2; ++s2) {
            if ((lvf >> (2 * d + s2)) & 1) {
              fine_face_mean<RECON, T>(P, fl, gas, S, m, d, s2, c3[d == 0 ? 1 : 0], c3[d == 2 ? 1 : 2], true,
                                       fs[s2]);
            } else {
              T g[5];
              face_llf<T>(geo, fl, gas, S, d, i + s2 * (d == 0), j + s2 * (d == 1), k + s2 * (d == 2), g);
#pragma unroll
              for (int v = 0; v < 5; ++v) fs[s2][v] = (double)g[v];
            }
          }
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            const double df = (fs[1][v] - fs[0][v]) * id[d];
            l[v] = d == 0 ? -df : l[v] - df;
          }
        }
        double us[5], unew[5];
        load5(S, off, geo.vstride, us);
        if (rs.a == 0.0) {
#pragma unroll
          for (int v = 0; v < 5; ++v) unew[v] = us[v] + (rs.c * dt) * l[v];
        } else {
          double u0[5];
#pragma unroll
          for (int v = 0; v < 5; ++v) u0[v] = P.U[off + v * geo.vstride];
#pragma unroll
          for (int v = 0; v < 5; ++v) unew[v] = (rs.a * u0[v] + rs.b * us[v]) + (rs.c * dt) * l[v];
        }
#pragma unroll
        for (int v = 0; v < 5; ++v) Out[off + v * geo.vstride] = unew[v];
        continue;
      }
      double dL[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
      for (int d = 0; d < 3; ++d) {
        for (int s = 0; s < 2; ++s) {
          if (!nb[2 * d + s]) continue;
          T fho[5], flf[5];
          face_pair<RECON, T>(geo, fl, gas, S, d, i + s * (d == 0), j + s * (d == 1), k + s * (d == 2),
                              fho, flf);
          // L = -(F_upper - F_lower)/dx: a lower face enters with +, an upper with -
          const double sg = s ? -id[d] : id[d];
#pragma unroll
          for (int v = 0; v < 5; ++v) dL[v] += sg * ((double)flf[v] - (double)fho[v]);
        }
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) Out[off + v * geo.vstride] += cst * dL[v];
    }
  }
}

// After a corrected last stage: the time step from the corrected state.
__global__ void __launch_bounds__(256) k_fofc_dt(const FixArgs a) {
  const FixEntry E = a.e[blockIdx.y];
  const DevProblem& P = *E.p;
  if (!E.last || P.fofc_cnt[E.seq & 1] == 0ull) return;
  const double gamma = P.gamma, gm1 = gamma - 1.0;
  const Floors fl{P.rho_floor, P.p_floor / gm1};
  const int64_t ncell = (int64_t)P.nblocks * P.vstride;
  const double* __restrict__ Un = P.rk[P.nstages - 1].dst;  // the new state
  double mydt = __longlong_as_double((long long)kInfBits);
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncell;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = c / P.vstride, rr = c - m * P.vstride;
    if (P.binfo) {  // a level-0 leaf next to finer ones: k_smr_dt, after the flux correction
      Geo g;
      geo_init(g, P, (int)m);
      if (smr_cf_leaf(g, P.nblocks)) continue;
    }
    double u[5], dxb[3];
    load5c(Un, m * P.bstride + rr, P.vstride, u);
    block_dx(P, m, dxb);
    mydt = fmin(mydt, cell_dt(fl, gamma, gm1, dxb, u));
  }
  unsigned long long b = (unsigned long long)__double_as_longlong(mydt);
  for (int s = kWave / 2; s > 0; s >>= 1) {
    const unsigned long long o = __shfl_xor(b, s, kWave);
    b = o < b ? o : b;
  }
  __shared__ unsigned long long red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = b;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long mn = red[0];
    for (int w = 1; w < 4; ++w) mn = red[w] < mn ? red[w] : mn;
    atomicMin(P.dtmin + (E.parity ^ 1), mn);
  }
}

// Pointwise step between RK stages (rk_combine_after): op 1 copies V to U
// (RK1), op 2 is the SSPRK(10,4) mix after stage 5, U <- U/25 + 9 V/25, then
// V <- 15 U - 5 V, element by element. Op 1 ends a one-stage step: it also
// clears the time-step slot this step read, which the next step reduces into.
__global__ void __launch_bounds__(256) k_combine(const FixArgs a, int op) {
  const FixEntry E = a.e[blockIdx.y];
  const DevProblem& P = *E.p;
  if (op == 1 && blockIdx.x == 0 && threadIdx.x == 0) P.dtmin[E.parity] = kInfBits;
  const int64_t n = (int64_t)P.nblocks * P.bstride;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = P.V[i];
    if (op == 1) {
      P.U[i] = v;
    } else {
      const double u = P.U[i] / 25.0 + 9.0 / 25.0 * v;
      P.U[i] = u;
      P.V[i] = 15.0 * u - 5.0 * v;
    }
  }
}

// ------------------------------------------------------ static refinement
// A refined mesh's ghost slabs hold the state's representation at the slab
// owner's level, at the ghost cell's global index (periodic wrap at that
// level; an outflow face has no slab):
//  level 0, coarse cell I: the coarse leaf's cell, or in a refined root the
//    mean of its 8 fine cells, summed in pairs along x, then y, then z;
//  level 1, fine cell i: the fine leaf's cell, or in an unrefined root the
//    coarse value at floor(i/2) plus, per axis, a quarter of the minmod of the
//    two level-0 differences next to it, signed towards the fine cell.
__device__ __forceinline__ int wrap_or_clamp(int c, int n, int periodic) {
  if (c < 0) return periodic ? c + n : 0;
  if (c >= n) return periodic ? c - n : n - 1;
  return c;
}

// All 5 variables of level-1 cell (i,j,k) inside a refined root.
__device__ void smr_fine5(const DevProblem& P, const double* S, int i, int j, int k, double u[5]) {
  const int lx = i / P.bx, ly = j / P.by, lz = k / P.bz;
  const int r = (lx >> 1) + P.nroot[0] * ((ly >> 1) + P.nroot[1] * (lz >> 1));
  const int q = P.rinfo[2 * r + 1] + (lx & 1) + 2 * (ly & 1) + 4 * (lz & 1);
  load5c(S, (int64_t)q * P.bstride + ((int64_t)(k - lz * P.bz) * P.by + (j - ly * P.by)) * P.bx + (i - lx * P.bx),
         P.vstride, u);
}

__device__ void smr_level0(const DevProblem& P, const double* S, int I, int J, int K, double u[5]) {
  const int rx = I / P.bx, ry = J / P.by, rz = K / P.bz;
  const int r = rx + P.nroot[0] * (ry + P.nroot[1] * rz);
  if (!P.rinfo[2 * r]) {
    load5c(S, (int64_t)P.rinfo[2 * r + 1] * P.bstride +
               ((int64_t)(K - rz * P.bz) * P.by + (J - ry * P.by)) * P.bx + (I - rx * P.bx),
           P.vstride, u);
    return;
  }
  double f[8][5];
#pragma unroll
  for (int c = 0; c < 8; ++c) smr_fine5(P, S, 2 * I + (c & 1), 2 * J + ((c >> 1) & 1), 2 * K + (c >> 2), f[c]);
#pragma unroll
  for (int v = 0; v < 5; ++v)
    u[v] = (((f[0][v] + f[1][v]) + (f[2][v] + f[3][v])) + ((f[4][v] + f[5][v]) + (f[6][v] + f[7][v]))) * 0.125;
}

__device__ __forceinline__ double minmod2(double a, double b) {
  if (!(a * b > 0.0)) return 0.0;
  return fabs(a) < fabs(b) ? a : b;
}

constexpr int kGhostCC = 32;  // coarse cells per k_smr_ghost prolongation pass (256 threads)

// Fill every ghost slab of one problem (grid row = slab) from the stage's
// source register, all 5 variables per cell. The slabs are packed after the
// leaves in the same register (DevProblem::slab_cells): layer l along the
// face normal (0 next to the face), then the tangential axes, which is where
// ghost_local and its variants look for them.
__global__ void __launch_bounds__(256) k_smr_ghost(const DevProblem* __restrict__ Pp, int stage, int ng) {
  const DevProblem& P = *Pp;
  double* S = const_cast<double*>(P.rk[stage - 1].src);
  const int vb = blockIdx.y;
  const int own = P.vinfo[2 * vb], f = P.vinfo[2 * vb + 1];
  const int d = f >> 1, side = f & 1;
  const int32_t* b = P.binfo + (int64_t)own * kLeafInts;
  const int lev = b[0];
  const int bd[3] = {P.bx, P.by, P.bz};
  const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
  const int nl = (P.nroot[d] * bd[d]) << lev;
  double* slab = S + (int64_t)(P.nblocks + (vb >> P.slab_k2)) * P.bstride +
                 (int64_t)(vb & ((1 << P.slab_k2) - 1)) * P.slab_cells;
  auto ghost_d = [&](int l) {  // global index along d of ghost layer l, at the slab's level
    return wrap_or_clamp(side ? b[7 + d] * bd[d] + bd[d] + l : b[7 + d] * bd[d] - 1 - l, nl, P.periodic[d]);
  };
  if (lev == 0) {  // coarse slab next to a refined root: restriction, one thread per ghost cell
    const int area = bd[t1] * bd[t2];
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < ng * area; c += gridDim.x * blockDim.x) {
      const int l = c / area, rem = c - l * area;
      const int a2 = rem / bd[t1], a1 = rem - a2 * bd[t1];
      int g3[3];
      g3[t1] = b[7 + t1] * bd[t1] + a1;
      g3[t2] = b[7 + t2] * bd[t2] + a2;
      g3[d] = ghost_d(l);
      double u[5];
      smr_level0(P, S, g3[0], g3[1], g3[2], u);
      double* o = slab + ((int64_t)l * bd[t2] + a2) * bd[t1] + a1;  // packed: layer, then t2, t1
#pragma unroll
      for (int v = 0; v < 5; ++v) o[v * P.vstride] = u[v];
    }
    return;
  }
  // fine slab next to an unrefined root: prolongation. Per pass, kGhostCC
  // coarse cells under the slab: 7 threads per coarse cell fetch its level-0
  // value and its 6 neighbours' into LDS, then 8 threads per coarse cell form
  // its children that lie in the slab (each child with the arithmetic of R30).
  __shared__ double sv[kGhostCC][7][5];
  const int h1 = bd[t1] / 2, h2 = bd[t2] / 2;
  const int ncc = ((ng + 1) / 2) * h1 * h2;
  const int n0[3] = {P.nroot[0] * P.bx, P.nroot[1] * P.by, P.nroot[2] * P.bz};
  auto coarse_of = [&](int cidx, int c3[3], int& L, int& c1, int& c2) {
    L = cidx / (h1 * h2);
    const int rem = cidx - L * (h1 * h2);
    c2 = rem / h1;
    c1 = rem - c2 * h1;
    c3[t1] = (b[7 + t1] * bd[t1] >> 1) + c1;
    c3[t2] = (b[7 + t2] * bd[t2] >> 1) + c2;
    c3[d] = ghost_d(2 * L) >> 1;
  };
  for (int base = blockIdx.x * kGhostCC; base < ncc; base += gridDim.x * kGhostCC) {
    {
      const int cs = threadIdx.x / 7, kk = threadIdx.x - 7 * cs;  // kk 0: the cell; 1 + 2a + up: neighbours
      if (cs < kGhostCC && base + cs < ncc) {
        int c3[3], L, c1, c2;
        coarse_of(base + cs, c3, L, c1, c2);
        if (kk > 0) {
          const int a = (kk - 1) >> 1, up = (kk - 1) & 1;
          c3[a] = wrap_or_clamp(c3[a] + (up ? 1 : -1), n0[a], P.periodic[a]);
        }
        double u[5];
        smr_level0(P, S, c3[0], c3[1], c3[2], u);
#pragma unroll
        for (int v = 0; v < 5; ++v) sv[cs][kk][v] = u[v];
      }
    }
    __syncthreads();
    {
      const int cs = threadIdx.x >> 3, e = threadIdx.x & 7;
      if (cs < kGhostCC && base + cs < ncc) {
        int c3[3], L, c1, c2;
        coarse_of(base + cs, c3, L, c1, c2);
        const int l = 2 * L + (e & 1);
        if (l < ng) {
          int odd[3];
          odd[d] = ghost_d(l) & 1;
          odd[t1] = (e >> 1) & 1;  // leaf bases are even: the local parity is the global one
          odd[t2] = e >> 2;
          double* o = slab + ((int64_t)l * bd[t2] + (2 * c2 + odd[t2])) * bd[t1] + (2 * c1 + odd[t1]);
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            const double C = sv[cs][0][v];
            double t[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              const double sl = minmod2(C - sv[cs][1 + 2 * a][v], sv[cs][2 + 2 * a][v] - C);
              t[a] = odd[a] ? sl : -sl;
            }
            o[v * P.vstride] = C + 0.25 * ((t[0] + t[1]) + t[2]);
          }
        }
      }
    }
    __syncthreads();  // sv is reused by the next pass
  }
}

// The level-0 cells on level faces (next to finer leaves). Cell c of grid
// row e (coarse face (q, f) next to finer leaves) is the face cell (a1, a2)
// along the tangential axes; a cell on several level faces belongs to the row
// of its lowest face index (returns false in the other rows), so each is
// handled once, all its level faces together.
__device__ __forceinline__ bool cf_cell(const DevProblem& P, const Geo& geo, int f, int c, int cc[3]) {
  const int d = f >> 1, side = f & 1;
  const int bd[3] = {P.bx, P.by, P.bz};
  const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
  cc[t2] = c / bd[t1];
  cc[t1] = c - cc[t2] * bd[t1];
  cc[d] = side ? bd[d] - 1 : 0;
  return (level_faces(geo, P.nblocks, cc[0], cc[1], cc[2]) & ((1 << f) - 1)) == 0;
}

constexpr int kSmrCells = 51;  // face cells per k_smr_flux workgroup pass (5 threads each)

// Flux correction (Sec. 2: the flux through a coarse face shared with finer
// blocks is the finer blocks' flux): each level-0 cell on level faces adds,
// for each of them in x, y, z order, c dt (F_coarse - mean F_fine) / dx on an
// upper face, the opposite on a lower one, both fluxes recomputed from the
// stage's source exactly as the stage kernel formed them. A cell belongs to
// one grid row (cf_cell), so no cell is updated twice at once.
template <int RECON, typename T>
__global__ void __launch_bounds__(256) k_smr_flux(const DevProblem* __restrict__ Pp, int stage, int parity) {
  const DevProblem& P = *Pp;
  const int e = blockIdx.y;
  const int q = P.cfinfo[2 * e], f = P.cfinfo[2 * e + 1];
  const int d = f >> 1;
  const RkStage& rs = P.rk[stage - 1];
  const double* __restrict__ S = rs.src;
  double* Out = rs.dst;
  const double gamma = P.gamma, gm1 = gamma - 1.0;
  const Gas<T> gas{T(gamma), T(gm1), T((gamma + 1.0) / (2.0 * gamma))};
  const Floors fl{P.rho_floor, P.p_floor / gm1};
  const double cst = rs.c * (P.cfl * __longlong_as_double((long long)P.dtmin[parity]));
  const int bd[3] = {P.bx, P.by, P.bz};
  Geo geo;
  geo_init(geo, P, q);
  // five threads per face cell: h = 0 the coarse flux, h = 1..4 the fine
  // ones (more threads in flight than one thread doing all five)
  __shared__ double sFl[kSmrCells][5][5];
  const int cs = threadIdx.x / 5, h = threadIdx.x - 5 * cs;
  const int area = (d == 0 ? P.by : P.bx) * (d == 2 ? P.by : P.bz);
  for (int base = blockIdx.x * kSmrCells; base < area; base += gridDim.x * kSmrCells) {
    const int c = base + cs;
    int cc[3] = {0, 0, 0};
    const bool mine = cs < kSmrCells && c < area && cf_cell(P, geo, f, c, cc);
    const int lvf = mine ? level_faces(geo, P.nblocks, cc[0], cc[1], cc[2]) : 0;
    for (int d2 = 0; d2 < 3; ++d2) {  // the same number of barriers in every thread
      const int s2 = (lvf >> (2 * d2 + 1)) & 1;
      const bool act = ((lvf >> (2 * d2)) & 3) != 0;  // a level face along d2 (one side at most)
      const int u1 = d2 == 0 ? 1 : 0, u2 = d2 == 2 ? 1 : 2;
      if (act) {
        double fo[5];
        if (h == 0) {
          int lf[3] = {cc[0], cc[1], cc[2]};
          lf[d2] = s2 ? bd[d2] : 0;  // face_pair's cell index: the face's upper cell
          T fho[5], unused[5];
          face_pair<RECON, T>(geo, fl, gas, S, d2, lf[0], lf[1], lf[2], fho, unused);
#pragma unroll
          for (int v = 0; v < 5; ++v) fo[v] = (double)fho[v];
        } else {
          fine_face<RECON, T>(P, fl, gas, S, q, d2, s2, cc[u1], cc[u2], h - 1, false, fo);
        }
#pragma unroll
        for (int v = 0; v < 5; ++v) sFl[cs][h][v] = fo[v];
      }
      __syncthreads();
      if (act && h == 0) {
        const double idc = 1.0 / P.dx[d2];  // the coarse leaf is on level 0
        const int64_t off = (int64_t)q * P.bstride + ((int64_t)cc[2] * P.by + cc[1]) * P.bx + cc[0];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          const double fc = sFl[cs][0][v];
          const double mean = ((sFl[cs][1][v] + sFl[cs][2][v]) + (sFl[cs][3][v] + sFl[cs][4][v])) * 0.25;
          const double dl = s2 ? (fc - mean) * idc : (mean - fc) * idc;
          Out[off + v * P.vstride] += cst * dl;
        }
      }
      __syncthreads();  // sFl is reused by the next direction / group
    }
  }
}

// Before a stage that updates U in place: keep the step-start values of the
// level-0 level-face cells (the stage kernel may overwrite them before
// k_smr_cell has decided whether FOFC recomputes them from scratch).
__global__ void __launch_bounds__(256) k_smr_save(const DevProblem* __restrict__ Pp) {
  const DevProblem& P = *Pp;
  const int e = blockIdx.y;
  const int q = P.cfinfo[2 * e], f = P.cfinfo[2 * e + 1];
  const int d = f >> 1;
  const int area = (d == 0 ? P.by : P.bx) * (d == 2 ? P.by : P.bz);
  Geo geo;
  geo_init(geo, P, q);
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < area; c += gridDim.x * blockDim.x) {
    int cc[3];
    if (!cf_cell(P, geo, f, c, cc)) continue;
    const int64_t off = (int64_t)q * P.bstride + ((int64_t)cc[2] * P.by + cc[1]) * P.bx + cc[0];
    double* sv = P.cfsave + ((int64_t)e * P.cfarea + c) * 5;
#pragma unroll
    for (int v = 0; v < 5; ++v) sv[v] = P.U[off + v * P.vstride];
  }
}

// The stage update of those cells computed whole from the stage's source:
// on a level face the mean of the 4 fine fluxes as FOFC on the fine level
// left them (each the LLF flux when the fine cell behind it is flagged), on
// every other face the cell's own high-order flux. The stage kernel tested
// them with their own coarse fluxes; this test replaces that one (flag and
// counter adjusted). A result that is positive is stored; a flagged cell is
// left to k_fofc_fix, with its step-start value put back into U when the
// stage updates U in place (the stage kernel may have stored over it).
template <int RECON, typename T>
__global__ void __launch_bounds__(256) k_smr_cell(const DevProblem* __restrict__ Pp, int stage, int parity,
                                                  unsigned seq) {
  const DevProblem& P = *Pp;
  const int e = blockIdx.y;
  const int q = P.cfinfo[2 * e], f = P.cfinfo[2 * e + 1];
  const int d = f >> 1;
  const RkStage& rs = P.rk[stage - 1];
  const double* __restrict__ S = rs.src;
  double* Out = rs.dst;
  const bool inplace = Out == P.U;
  const double gamma = P.gamma, gm1 = gamma - 1.0;
  const Gas<T> gas{T(gamma), T(gm1), T((gamma + 1.0) / (2.0 * gamma))};
  const Floors fl{P.rho_floor, P.p_floor / gm1};
  const double dt = P.cfl * __longlong_as_double((long long)P.dtmin[parity]);
  const double id[3] = {1.0 / P.dx[0], 1.0 / P.dx[1], 1.0 / P.dx[2]};  // level-0 widths
  const int area = (d == 0 ? P.by : P.bx) * (d == 2 ? P.by : P.bz);
  Geo geo;
  geo_init(geo, P, q);
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < area; c += gridDim.x * blockDim.x) {
    int cc[3];
    if (!cf_cell(P, geo, f, c, cc)) continue;
    const int lvf = level_faces(geo, P.nblocks, cc[0], cc[1], cc[2]);
    double l[5];
    for (int d2 = 0; d2 < 3; ++d2) {
      const int u1 = d2 == 0 ? 1 : 0, u2 = d2 == 2 ? 1 : 2;
      double fs[2][5];
      for (int s2 = 0; s2 < 2; ++s2) {
        if ((lvf >> (2 * d2 + s2)) & 1) {
          fine_face_mean<RECON, T>(P, fl, gas, S, q, d2, s2, cc[u1], cc[u2], true, fs[s2]);
        } else {
          T fho[5], unused[5];
          face_pair<RECON, T>(geo, fl, gas, S, d2, cc[0] + s2 * (d2 == 0), cc[1] + s2 * (d2 == 1),
                              cc[2] + s2 * (d2 == 2), fho, unused);
#pragma unroll
          for (int v = 0; v < 5; ++v) fs[s2][v] = (double)fho[v];
        }
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const double df = (fs[1][v] - fs[0][v]) * id[d2];
        l[v] = d2 == 0 ? -df : l[v] - df;
      }
    }
    const int64_t r = ((int64_t)cc[2] * P.by + cc[1]) * P.bx + cc[0];
    const int64_t off = (int64_t)q * P.bstride + r;
    const double* sv = P.cfsave + ((int64_t)e * P.cfarea + c) * 5;
    double us[5], u0[5], unew[5];
    load5c(S, off, P.vstride, us);
#pragma unroll
    for (int v = 0; v < 5; ++v) u0[v] = inplace ? sv[v] : P.U[off + v * P.vstride];
    if (rs.a == 0.0) {
#pragma unroll
      for (int v = 0; v < 5; ++v) unew[v] = us[v] + (rs.c * dt) * l[v];
    } else {
#pragma unroll
      for (int v = 0; v < 5; ++v) unew[v] = (rs.a * u0[v] + rs.b * us[v]) + (rs.c * dt) * l[v];
    }
    const double ke2 = (unew[1] * unew[1] + unew[2] * unew[2]) + unew[3] * unew[3];
    const double pn = gm1 * (unew[4] - (0.5 * ke2) * rcp(unew[0]));
    const bool flag = !(unew[0] > 0.0) || !(pn > 0.0);
    const bool was = P.flags[(int64_t)q * P.vstride + r] != 0;
    P.flags[(int64_t)q * P.vstride + r] = flag ? 1 : 0;
    if (flag != was) atomicAdd(P.fofc_cnt + (seq & 1), flag ? 1ull : ~0ull);  // +1 or -1
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      if (!flag)
        Out[off + v * P.vstride] = unew[v];
      else if (inplace)
        Out[off + v * P.vstride] = u0[v];
    }
  }
}

// Time step of the corrected new state over the level-0 leaves next to finer
// ones (the stage kernel left them out), into dtmin[slot]. One grid row per
// leaf; the rows of other leaves return at once.
__global__ void __launch_bounds__(256) k_smr_dt(const DevProblem* __restrict__ Pp, int slot) {
  const DevProblem& P = *Pp;
  const int m = blockIdx.y;
  Geo g;
  geo_init(g, P, m);
  if (!smr_cf_leaf(g, P.nblocks)) return;  // the whole workgroup
  const double gamma = P.gamma, gm1 = gamma - 1.0;
  const Floors fl{P.rho_floor, P.p_floor / gm1};
  const double* __restrict__ Un = P.rk[P.nstages - 1].dst;
  double mydt = __longlong_as_double((long long)kInfBits);
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < P.vstride;
       c += (int64_t)gridDim.x * blockDim.x) {
    double u[5];
    load5c(Un, (int64_t)m * P.bstride + c, P.vstride, u);
    mydt = fmin(mydt, cell_dt(fl, gamma, gm1, P.dx, u));  // level-0 widths
  }
  unsigned long long b = (unsigned long long)__double_as_longlong(mydt);
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const unsigned long long x = __shfl_xor(b, o, kWave);
    b = x < b ? x : b;
  }
  __shared__ unsigned long long red[256 / kWave];
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = b;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long mn = red[0];
    for (int w = 1; w < 256 / kWave; ++w) mn = red[w] < mn ? red[w] : mn;
    atomicMin(P.dtmin + slot, mn);
  }
}

// ------------------------------------------------------------ small kernels
// Time step of a stored state into dtmin[slot] (after k_reset_dt).
__global__ void __launch_bounds__(256) k_dt(const DevProblem* __restrict__ Pp, int slot, int flags) {
  const DevProblem& P = *Pp;
  const int64_t ncell = (int64_t)P.nblocks * P.vstride;
  const double gamma = P.gamma, gm1 = gamma - 1.0;
  const Floors fl{P.rho_floor, P.p_floor / gm1};
  double mydt = __longlong_as_double((long long)kInfBits);
  int bad = 0;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncell;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = c / P.vstride, rr = c - m * P.vstride;
    double u[5], dxb[3];
    load5c(P.U, m * P.bstride + rr, P.vstride, u);
    double w[5];
    int h = 0;
    c2p(fl, u, w, h, bad);
    block_dx(P, m, dxb);
    mydt = fmin(mydt, cell_dt(fl, gamma, gm1, dxb, u));
  }
  if ((flags & 1) && bad) atomicOr(P.err, 1u);
  unsigned long long b = (unsigned long long)__double_as_longlong(mydt);
  for (int s = kWave / 2; s > 0; s >>= 1) {
    const unsigned long long o = __shfl_xor(b, s, kWave);
    b = o < b ? o : b;
  }
  __shared__ unsigned long long red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = b;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long mn = red[0];
    for (int w = 1; w < 4; ++w) mn = red[w] < mn ? red[w] : mn;
    atomicMin(P.dtmin + slot, mn);
  }
}

// Header fields set from the device (no memset nodes: safe under capture).
// clear bit 0: error flag; bit 1: floor counter and time.
__global__ void k_reset(const DevProblem* __restrict__ Pp, int slot, int clear) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const DevProblem& P = *Pp;
    P.dtmin[slot] = kInfBits;
    if (clear & 1) *P.err = 0u;
    if (clear & 2) {
      *P.floor_hits = 0ull;
      *P.time = 0.0;
    }
  }
}

// Global [5][nz][ny][nx] <-> MeshBlockPack [m][5][bz][by][bx].
__global__ void __launch_bounds__(256) k_scatter(const DevProblem* __restrict__ Pp,
                                                 const double* __restrict__ src,
                                                 double* __restrict__ dst, int to_blocks) {
  const DevProblem& P = *Pp;
  const int64_t nx = (int64_t)P.bx * P.nbx, ny = (int64_t)P.by * P.nby;
  const int64_t nz = (int64_t)P.bz * P.nbz;
  const int64_t n = 5 * nx * ny * nz;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n;
       g += (int64_t)gridDim.x * blockDim.x) {
    int64_t t = g;
    const int64_t i = t % nx; t /= nx;
    const int64_t j = t % ny; t /= ny;
    const int64_t k = t % nz;
    const int64_t v = t / nz;
    const int64_t m = (i / P.bx) + P.nbx * ((j / P.by) + P.nby * (k / P.bz));
    const int64_t b = m * P.bstride + v * P.vstride +
                      ((k % P.bz) * P.by + (j % P.by)) * P.bx + (i % P.bx);
    if (to_blocks) dst[b] = src[g];
    else dst[g] = src[b];
  }
}

// Write a problem header (descriptor and counters) passed by value into the
// workspace: the allocation-free entry point sets up its scratch workspace
// with kernels only (no host-to-device copy).
__global__ void __launch_bounds__(256) k_put_header(const HeaderBytes h, unsigned char* __restrict__ dst) {
  for (int i = threadIdx.x; i < kHeaderBytes; i += blockDim.x) dst[i] = h.b[i];
}

// Time, next time step and error flag of a problem into out[0..2] (device).
__global__ void k_result(const DevProblem* __restrict__ Pp, int slot, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const DevProblem& P = *Pp;
    out[0] = *P.time;
    out[1] = P.cfl * __longlong_as_double((long long)P.dtmin[slot]);
    out[2] = *P.err ? 1.0 : 0.0;
  }
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Plain streaming copy (16 bytes per lane per iteration).
__global__ void __launch_bounds__(256) k_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                              int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// ------------------------------------------------------ dispatch tables
// Compiled tile shapes (TX x TY threads); TX*TY must be a multiple of 64.
// Compiled tile shapes: TX x TY threads (a multiple of 64) and the occupancy
// the register allocator targets (waves per SIMD; more waves hide latency
// better but may force spills).
#define HY_K(R, T, TX, TY, W, S) \
  {(const void*)&k_stage<R, T, TX, TY, W, S, false>, (const void*)&k_stage<R, T, TX, TY, W, S, true>}
#define HY_RECON_SET(R, TX, TY, W)                                                    \
  {{HY_K(R, double, TX, TY, W, 1), HY_K(R, double, TX, TY, W, 2)},                    \
   {HY_K(R, float, TX, TY, W, 1), HY_K(R, float, TX, TY, W, 2)}}
#define HY_STAGE_SET(TX, TY, W)                                                       \
  {TX, TY, W,                                                                         \
   {HY_RECON_SET(0, TX, TY, W), HY_RECON_SET(1, TX, TY, W), HY_RECON_SET(2, TX, TY, W),     \
    HY_RECON_SET(3, TX, TY, W)}}

struct StageVariant {
  int tx, ty, wpe;
  const void* fn[4][2][2][2];  // [recon][precision][kind: first, later stage][refined mesh]
};

static const StageVariant kStageVariants[] = {
    HY_STAGE_SET(64, 8, 2), HY_STAGE_SET(64, 8, 4), HY_STAGE_SET(32, 8, 2), HY_STAGE_SET(32, 8, 3),
    HY_STAGE_SET(32, 8, 4), HY_STAGE_SET(16, 16, 4), HY_STAGE_SET(64, 4, 3), HY_STAGE_SET(32, 16, 2),
};

int num_stage_variants() { return (int)(sizeof(kStageVariants) / sizeof(kStageVariants[0])); }

void stage_variant_shape(int v, int* tx, int* ty) {
  *tx = kStageVariants[v].tx;
  *ty = kStageVariants[v].ty;
}

int stage_variant_waves(int v) { return kStageVariants[v].wpe; }

// kind 1: the first RK stage; kind 2: any later stage.
const void* stage_kernel(int v, int recon, int prec, int kind, int smr) {
  return kStageVariants[v].fn[recon][prec][kind - 1][smr ? 1 : 0];
}

hipError_t launch_stage(int v, int recon, int prec, int kind, int smr, const StageArgs& a, int grid,
                        hipStream_t s) {
  const StageVariant& sv = kStageVariants[v];
  void* args[] = {(void*)&a};
  return hipLaunchKernel(sv.fn[recon][prec][kind - 1][smr ? 1 : 0], dim3(grid), dim3(sv.tx * sv.ty), args,
                         0, s);
}

hipError_t launch_fofc(int recon, int prec, const FixArgs& a, int grid_x, hipStream_t s) {
  static const void* fix[4][2] = {
      {(const void*)&k_fofc_fix<0, double>, (const void*)&k_fofc_fix<0, float>},
      {(const void*)&k_fofc_fix<1, double>, (const void*)&k_fofc_fix<1, float>},
      {(const void*)&k_fofc_fix<2, double>, (const void*)&k_fofc_fix<2, float>},
      {(const void*)&k_fofc_fix<3, double>, (const void*)&k_fofc_fix<3, float>}};
  void* args[] = {(void*)&a};
  hipError_t e = hipLaunchKernel((const void*)&k_fofc_mark, dim3(grid_x, a.nprob), dim3(256), args, 0, s);
  if (e != hipSuccess) return e;
  e = hipLaunchKernel(fix[recon][prec], dim3(grid_x, a.nprob), dim3(256), args, 0, s);
  if (e != hipSuccess || !a.any_last) return e;
  return hipLaunchKernel((const void*)&k_fofc_dt, dim3(grid_x, a.nprob), dim3(256), args, 0, s);
}

int fofc_grid(int nblocks, int bz) { return nblocks * ((bz + kFixPlanes - 1) / kFixPlanes); }

hipError_t launch_combine(const FixArgs& a, int op, int grid_x, hipStream_t s) {
  hipLaunchKernelGGL(k_combine, dim3(grid_x, a.nprob), dim3(256), 0, s, a, op);
  return hipGetLastError();
}

hipError_t launch_reset(const DevProblem* p, int slot, int clear, hipStream_t s) {
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, p, slot, clear);
  return hipGetLastError();
}

hipError_t launch_dt(const DevProblem* p, int64_t ncell, int slot, int flags, hipStream_t s) {
  int64_t g = (ncell + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_dt, dim3((unsigned)g), dim3(256), 0, s, p, slot, flags);
  return hipGetLastError();
}

hipError_t launch_scatter(const DevProblem* p, const double* src, double* dst, int64_t n,
                          int to_blocks, hipStream_t s) {
  int64_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_scatter, dim3((unsigned)g), dim3(256), 0, s, p, src, dst, to_blocks);
  return hipGetLastError();
}

hipError_t launch_put_header(const HeaderBytes& h, void* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_put_header, dim3(1), dim3(256), 0, s, h, (unsigned char*)dst);
  return hipGetLastError();
}

hipError_t launch_result(const DevProblem* p, int slot, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_result, dim3(1), dim3(64), 0, s, p, slot, out);
  return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const int64_t n = (int64_t)(bytes / 16);
  int64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)g), dim3(256), 0, s, (const u32x4*)src, (u32x4*)dst, n);
  return hipGetLastError();
}


hipError_t launch_smr_ghost(const DevProblem* p, int stage, int ng, int nvirt, const int32_t block[3],
                            hipStream_t s) {
  const int area = std::max(block[1] * block[2], std::max(block[0] * block[2], block[0] * block[1]));
  const int gx = std::max(1, std::min((ng * area + 255) / 256, 1024));
  hipLaunchKernelGGL(k_smr_ghost, dim3(gx, nvirt), dim3(256), 0, s, p, stage, ng);
  return hipGetLastError();
}

hipError_t launch_smr_dt(const DevProblem* p, int nleaf, const int32_t block[3], int slot,
                         hipStream_t s) {
  const int cells = block[0] * block[1] * block[2];
  const int gx = std::max(1, std::min((cells + 255) / 256, 64));
  hipLaunchKernelGGL(k_smr_dt, dim3(gx, nleaf), dim3(256), 0, s, p, slot);
  return hipGetLastError();
}

hipError_t launch_smr_save(const DevProblem* p, int ncf, const int32_t block[3], hipStream_t s) {
  const int area = std::max(block[1] * block[2], std::max(block[0] * block[2], block[0] * block[1]));
  const int gx = std::max(1, std::min((area + 255) / 256, 1024));
  hipLaunchKernelGGL(k_smr_save, dim3(gx, ncf), dim3(256), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_smr_cell(int recon, int prec, const DevProblem* p, int stage, int parity, unsigned seq,
                           int ncf, const int32_t block[3], hipStream_t s) {
  using K = void (*)(const DevProblem*, int, int, unsigned);
  static const K tab[4][2] = {{k_smr_cell<0, double>, k_smr_cell<0, float>},
                              {k_smr_cell<1, double>, k_smr_cell<1, float>},
                              {k_smr_cell<2, double>, k_smr_cell<2, float>},
                              {k_smr_cell<3, double>, k_smr_cell<3, float>}};
  if (recon < 0 || recon > 3 || prec < 0 || prec > 1) return hipErrorInvalidValue;
  const int area = std::max(block[1] * block[2], std::max(block[0] * block[2], block[0] * block[1]));
  const int gx = std::max(1, std::min((area + 255) / 256, 1024));
  hipLaunchKernelGGL(tab[recon][prec], dim3(gx, ncf), dim3(256), 0, s, p, stage, parity, seq);
  return hipGetLastError();
}

hipError_t launch_smr_flux(int recon, int prec, const DevProblem* p, int stage, int parity, int ncf,
                           const int32_t block[3], hipStream_t s) {
  using K = void (*)(const DevProblem*, int, int);
  static const K tab[4][2] = {{k_smr_flux<0, double>, k_smr_flux<0, float>},
                              {k_smr_flux<1, double>, k_smr_flux<1, float>},
                              {k_smr_flux<2, double>, k_smr_flux<2, float>},
                              {k_smr_flux<3, double>, k_smr_flux<3, float>}};
  if (recon < 0 || recon > 3 || prec < 0 || prec > 1) return hipErrorInvalidValue;
  const int area = std::max(block[1] * block[2], std::max(block[0] * block[2], block[0] * block[1]));
  const int gx = std::max(1, std::min((area + kSmrCells - 1) / kSmrCells, 1024));
  hipLaunchKernelGGL(tab[recon][prec], dim3(gx, ncf), dim3(256), 0, s, p, stage, parity);
  return hipGetLastError();
}


}  // namespace hy
