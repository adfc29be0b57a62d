// TEST INFRASTRUCTURE — the CPU oracle. Only the test suite, the smoke check and the
// CPU-baseline leg of the benchmark may load or run anything under oracle/. It shares no code
// with the HIP path and is deliberately plain: one node or one interface at a time, in the
// order and notation of the paper (Zhao & Zhang, "Well-balanced fifth-order finite difference
// Hermite WENO scheme for the shallow water equations", 2022).
//
// Where the paper is silent the oracle takes these readings (each is listed with its reason in
// the design notes of the repository):
//   * Lax-Friedrichs alpha is global per direction and per right-hand-side evaluation:
//     alpha_x = max |u|+c, alpha_y = max |v|+c over the nodes of the state being differentiated.
//   * The interface characteristic matrices use the arithmetic mean of (eta, m, w, b) of the
//     two nodes adjacent to the interface.
//   * The limiter's characteristic matrices use the node state U_i, x-Jacobian for V and
//     y-Jacobian for Q.
//   * The right-hand side of each Runge-Kutta stage takes the unmodified stage derivatives;
//     the limited derivatives enter only as the Runge-Kutta base (eq. (2.11) read literally).
//   * The 2D semi-discrete source terms carry a minus sign (the printed plus signs in the 2D
//     scheme contradict the PDE (3.4) and the 1D scheme (2.8)).
//   * dt = CFL / (alpha_x/dx + alpha_y/dy) from the state at the start of the step.
//   * Nodes sit at cell centres x_i = x0 + (i+1/2) dx; boundaries are periodic or reflective
//     (mirror about the wall face with the parity of each field).
#pragma once
#include <algorithm>
#include <cstddef>
#include <vector>

#include "scalar.hpp"

namespace orc {

enum { BC_PERIODIC = 0, BC_REFLECTIVE = 1 };
enum { FL_FIXED_DT = 1, FL_FIXED_ALPHA = 2, FL_NO_LIMITER = 4, FL_LIMIT_BEFORE_RHS = 8 };
enum { OK = 0, E_INVAL = -1, E_DRY = -4, E_NONFINITE = -5 };

template <class T> struct Params {
  int dim = 2, nx = 0, ny = 1;
  T dx = T(1), dy = T(1), g = T(9.812), cfl = T(0.6), eps = T(1e-6);
  int bcx = BC_PERIODIC, bcy = BC_PERIODIC, flags = 0;
  T fixed_dt = T(0);
  T ax_fixed[3] = {T(0), T(0), T(0)}, ay_fixed[3] = {T(0), T(0), T(0)};
};

// ---------------------------------------------------------------- padded node planes
// A plane of node values with G ghost nodes on each side (in y only for 2D).
template <class T> struct Plane {
  int nx = 0, ny = 0, gx = 0, gy = 0, sx = 0;
  std::vector<T> a;
  void init(int nx_, int ny_, int g, bool two_d) {
    nx = nx_; ny = ny_; gx = g; gy = two_d ? g : 0; sx = nx + 2 * gx;
    a.assign((size_t)sx * (size_t)(ny + 2 * gy), T(0));
  }
  T& operator()(int i, int j) { return a[(size_t)(j + gy) * sx + (size_t)(i + gx)]; }
  const T& operator()(int i, int j) const { return a[(size_t)(j + gy) * sx + (size_t)(i + gx)]; }
};

template <class T> inline T flip(int parity, const T& v) { return parity > 0 ? v : -v; }
template <class T> inline T pm(bool plus, const T& v) { return plus ? v : -v; }

// Fill the ghost nodes. Periodic: wrap. Reflective: ghost -1-k mirrors node k about the wall
// face, multiplied by the field's parity (+1 even, -1 odd) across that wall. Corners are never
// read by the cross-shaped stencils; they are poisoned so that any accidental read shows.
template <class T>
void fill_ghosts(Plane<T>& f, int bcx, int bcy, int par_x, int par_y) {
  const int nx = f.nx, ny = f.ny;
  for (int j = 0; j < ny; ++j)
    for (int k = 1; k <= f.gx; ++k) {
      if (bcx == BC_PERIODIC) {
        f(-k, j) = f(nx - k, j);
        f(nx - 1 + k, j) = f(k - 1, j);
      } else {
        f(-k, j) = flip(par_x, f(k - 1, j));
        f(nx - 1 + k, j) = flip(par_x, f(nx - k, j));
      }
    }
  if (f.gy == 0) return;
  for (int i = 0; i < nx; ++i)
    for (int k = 1; k <= f.gy; ++k) {
      if (bcy == BC_PERIODIC) {
        f(i, -k) = f(i, ny - k);
        f(i, ny - 1 + k) = f(i, k - 1);
      } else {
        f(i, -k) = flip(par_y, f(i, k - 1));
        f(i, ny - 1 + k) = flip(par_y, f(i, ny - k));
      }
    }
  for (int j = 1; j <= f.gy; ++j)
    for (int k = 1; k <= f.gx; ++k) {
      f(-k, -j) = poison<T>(); f(nx - 1 + k, -j) = poison<T>();
      f(-k, ny - 1 + j) = poison<T>(); f(nx - 1 + k, ny - 1 + j) = poison<T>();
    }
}

// ---------------------------------------------------------------- scalar HWENO building blocks
// All in the "+" orientation of Sec. 2.1: stencil values at x_{i-1}, x_i, x_{i+1} (index 0,1,2),
// f = flux values, p = derivative-flux values, evaluated at the interface x_{i+1/2}. The "-"
// orientation is the mirror image about x_{i+1/2}: reverse the stencil (i+2, i+1, i) and negate
// every derivative; a reconstructed value keeps its sign, a reconstructed derivative flips it.

// Values of the three cubic Hermite candidates q1, q2, q3 at x_{i+1/2} (Sec. 2.1).
template <class T> void hw_candidates(const T f[3], const T p[3], T dx, T q[3]) {
  static const T half = T(1) / T(2), sixth = T(1) / T(6), twelfth = T(1) / T(12);
  q[0] = half * (f[0] + f[1]) + sixth * dx * (p[0] + T(5) * p[1]);
  q[1] = half * (f[1] + f[2]) + sixth * dx * (p[1] - p[2]);
  q[2] = twelfth * (f[0] + T(10) * f[1] + f[2]) + half * dx * p[1];
}

// Smoothness indicators beta_1..beta_3 of the three candidates (Sec. 2.1).
template <class T> void hw_beta(const T f[3], const T p[3], T dx, T be[3]) {
  static const T c133 = T(13) / T(3), c78120 = T(781) / T(20), c1312 = T(13) / T(12),
                 c78180 = T(781) / T(80);
  const T a = sq(dx * p[1]);
  be[0] = a + c133 * sq(T(3) * (f[0] - f[1]) + dx * (p[0] + T(2) * p[1])) +
          c78120 * sq(T(2) * (f[0] - f[1]) + dx * (p[0] + p[1]));
  be[1] = a + c133 * sq(T(3) * (f[1] - f[2]) + dx * (p[2] + T(2) * p[1])) +
          c78120 * sq(T(2) * (f[1] - f[2]) + dx * (p[2] + p[1]));
  be[2] = a + c1312 * sq(f[0] - T(2) * f[1] + f[2]) + c78180 * sq(f[0] - f[2] + T(2) * dx * p[1]);
}

// Nonlinear weights omega_l = w~_l / sum w~, w~_l = gamma_l / (beta_l + eps)^2 (eq. (2.7)).
template <class T> void hw_weights(const T be[3], const T lin[3], T eps, T w[3]) {
  T wt[3];
  for (int l = 0; l < 3; ++l) wt[l] = lin[l] / sq(be[l] + eps);
  const T s = wt[0] + wt[1] + wt[2];
  for (int l = 0; l < 3; ++l) w[l] = wt[l] / s;
}

template <class T> const T* hw_gamma() {
  static const T g[3] = {T(3) / T(10), T(3) / T(10), T(4) / T(10)};
  return g;
}

// Nonlinear HWENO value at x_{i+1/2} (eq. (2.5)); also returns the weights used.
template <class T> T hweno_value(const T f[3], const T p[3], T dx, T eps, T w[3]) {
  T q[3], be[3];
  hw_candidates(f, p, dx, q);
  hw_beta(f, p, dx, be);
  hw_weights(be, hw_gamma<T>(), eps, w);
  return w[0] * q[0] + w[1] * q[1] + w[2] * q[2];
}

// The same candidates combined with weights computed elsewhere (the source split of Step 2
// reuses the flux's nonlinear weights).
template <class T> T hweno_with_weights(const T w[3], const T f[3], const T p[3], T dx) {
  T q[3];
  hw_candidates(f, p, dx, q);
  return w[0] * q[0] + w[1] * q[1] + w[2] * q[2];
}

// Derivative of the quintic Hermite polynomial Q at x_{i+1/2} (eq. (2.6)).
template <class T> T hermite_dQ(const T f[3], const T p[3], T dx) {
  static const T quarter = T(1) / T(4), twelfth = T(1) / T(12);
  return quarter * (f[0] - T(8) * f[1] + T(7) * f[2]) / dx + twelfth * (p[0] - T(2) * p[1] - T(5) * p[2]);
}

// Four-point central flux of the mixed derivative terms (eq. (3.7)).
template <class T> T central4(T a, T b, T c, T d) {
  static const T k1 = T(1) / T(12), k7 = T(7) / T(12);
  return k7 * (b + c) - k1 * (a + d);
}

// HWENO limiter of one characteristic component at x_i (Sec. 2.2): mu at x_{i-1}, x_i, x_{i+1}
// and the derivatives nu at x_{i-1}, x_{i+1}; linear weights (1/4, 1/4, 1/2).
template <class T> T hweno_limit(T mm, T m0, T mp, T nm, T np, T dx, T eps) {
  static const T c133 = T(13) / T(3), quarter = T(1) / T(4), c1312 = T(13) / T(12), half = T(1) / T(2);
  static const T lin[3] = {T(1) / T(4), T(1) / T(4), T(1) / T(2)};
  T dp[3], be[3], w[3];
  dp[0] = T(2) * (m0 - mm) / dx - nm;
  dp[1] = T(2) * (mp - m0) / dx - np;
  dp[2] = half * (mp - mm) / dx;
  be[0] = sq(T(2) * m0 - T(2) * mm - nm * dx) + c133 * sq(m0 - mm - nm * dx);
  be[1] = sq(T(2) * mp - T(2) * m0 - np * dx) + c133 * sq(mp - m0 - np * dx);
  be[2] = quarter * sq(mp - mm) + c1312 * sq(mm - T(2) * m0 + mp);
  hw_weights(be, lin, eps, w);
  return w[0] * dp[0] + w[1] * dp[1] + w[2] * dp[2];
}

// ---------------------------------------------------------------- model: fluxes and Jacobians
// 1D pre-balanced flux (eq. (2.2)): U = (eta, m), h = eta - b.
template <class T> void flux_1d(const T U[2], T b, T g, T F[2]) {
  static const T half = T(1) / T(2);
  F[0] = U[1];
  F[1] = U[1] * U[1] / (U[0] - b) + half * g * (U[0] * U[0] - T(2) * U[0] * b);
}
// Phi = dF/dU V + dF/db B (eq. (2.3)).
template <class T> void dflux_1d(const T U[2], T b, const T V[2], T B, T g, T P[2]) {
  const T h = U[0] - b, u = U[1] / h;
  P[0] = V[1];
  P[1] = (g * h - u * u) * V[0] + T(2) * u * V[1] + (u * u - g * U[0]) * B;
}

// 2D fluxes (eq. (3.3)): U = (eta, m, w).
template <class T> void flux_x(const T U[3], T b, T g, T F[3]) {
  static const T half = T(1) / T(2);
  const T h = U[0] - b;
  F[0] = U[1];
  F[1] = U[1] * U[1] / h + half * g * (U[0] * U[0] - T(2) * U[0] * b);
  F[2] = U[1] * U[2] / h;
}
template <class T> void flux_y(const T U[3], T b, T g, T F[3]) {
  static const T half = T(1) / T(2);
  const T h = U[0] - b;
  F[0] = U[2];
  F[1] = U[1] * U[2] / h;
  F[2] = U[2] * U[2] / h + half * g * (U[0] * U[0] - T(2) * U[0] * b);
}
// Jacobians dF/dU (3x3) and dF/db (3) of F1 and F2.
template <class T> void jac_x(const T U[3], T b, T g, T J[3][3], T Jb[3]) {
  const T h = U[0] - b, u = U[1] / h, v = U[2] / h;
  J[0][0] = T(0);         J[0][1] = T(1);     J[0][2] = T(0);
  J[1][0] = g * h - u * u; J[1][1] = T(2) * u; J[1][2] = T(0);
  J[2][0] = -(u * v);     J[2][1] = v;        J[2][2] = u;
  Jb[0] = T(0); Jb[1] = u * u - g * U[0]; Jb[2] = u * v;
}
template <class T> void jac_y(const T U[3], T b, T g, T J[3][3], T Jb[3]) {
  const T h = U[0] - b, u = U[1] / h, v = U[2] / h;
  J[0][0] = T(0);         J[0][1] = T(0); J[0][2] = T(1);
  J[1][0] = -(u * v);     J[1][1] = v;    J[1][2] = u;
  J[2][0] = g * h - v * v; J[2][1] = T(0); J[2][2] = T(2) * v;
  Jb[0] = T(0); Jb[1] = u * v; Jb[2] = v * v - g * U[0];
}
// Derivative fluxes (Sec. 3): dF/dU D + dF/db B, e.g. Phi1 = jac_x (V, B1), Psi1 = jac_x (Q, B2),
// Phi2 = jac_y (V, B1), Psi2 = jac_y (Q, B2).
template <class T> void jmul(const T J[3][3], const T Jb[3], const T D[3], T B, T P[3]) {
  for (int c = 0; c < 3; ++c) P[c] = J[c][0] * D[0] + J[c][1] * D[1] + J[c][2] * D[2] + Jb[c] * B;
}

// ---------------------------------------------------------------- characteristic matrices
// Rows of L are left eigenvectors, columns of R right eigenvectors of the flux Jacobian, at the
// state (eta, m[, w]) over bottom b; c = sqrt(g h).
template <class T> void eig_1d(T eta, T m, T b, T g, T L[2][2], T R[2][2]) {
  const T h = eta - b, u = m / h, c = sqrt_(g * h), i2c = T(1) / (T(2) * c);
  R[0][0] = T(1);  R[0][1] = T(1);
  R[1][0] = u - c; R[1][1] = u + c;
  L[0][0] = (u + c) * i2c;    L[0][1] = -i2c;
  L[1][0] = -((u - c) * i2c); L[1][1] = i2c;
}
template <class T> void eig_x(T eta, T m, T w, T b, T g, T L[3][3], T R[3][3]) {
  const T h = eta - b, u = m / h, v = w / h, c = sqrt_(g * h), i2c = T(1) / (T(2) * c);
  // columns (1, u-c, v), (0, 0, 1), (1, u+c, v)
  R[0][0] = T(1);  R[0][1] = T(0); R[0][2] = T(1);
  R[1][0] = u - c; R[1][1] = T(0); R[1][2] = u + c;
  R[2][0] = v;     R[2][1] = T(1); R[2][2] = v;
  L[0][0] = (u + c) * i2c;    L[0][1] = -i2c; L[0][2] = T(0);
  L[1][0] = -v;               L[1][1] = T(0); L[1][2] = T(1);
  L[2][0] = -((u - c) * i2c); L[2][1] = i2c;  L[2][2] = T(0);
}
template <class T> void eig_y(T eta, T m, T w, T b, T g, T L[3][3], T R[3][3]) {
  const T h = eta - b, u = m / h, v = w / h, c = sqrt_(g * h), i2c = T(1) / (T(2) * c);
  // columns (1, u, v-c), (0, 1, 0), (1, u, v+c)
  R[0][0] = T(1);  R[0][1] = T(0); R[0][2] = T(1);
  R[1][0] = u;     R[1][1] = T(1); R[1][2] = u;
  R[2][0] = v - c; R[2][1] = T(0); R[2][2] = v + c;
  L[0][0] = (v + c) * i2c;    L[0][1] = T(0); L[0][2] = -i2c;
  L[1][0] = -u;               L[1][1] = T(1); L[1][2] = T(0);
  L[2][0] = -((v - c) * i2c); L[2][1] = T(0); L[2][2] = i2c;
}

template <class T, int N> T dotn(const T a[N], const T b[N]) {
  T s = a[0] * b[0];
  for (int k = 1; k < N; ++k) s += a[k] * b[k];
  return s;
}

// ---------------------------------------------------------------- one interface x_{i+1/2}
// Inputs are the four nodes i-1, i, i+1, i+2 (index 0..3). N = 2 (1D) or 3 (2D); `slot` is the
// component that carries the bottom in the source-split vector (b~ = (0,b[,0]) along x,
// b- = (0,0,b) along y). Outputs:
//   Fh  : nonlinear HWENO flux F^ = F^+ + F^-, characteristic-wise (Step 1)
//   bh  : the bottom vector reconstructed with the same projection and weights (Step 2)
//   Dh  : linear Hermite flux of the derivative equation along this direction (Step 1)
//   Bh  : slot component of the bottom-derivative vector, same linear reconstruction (Step 2)
//   Mh  : four-point central flux of the mixed derivative flux (2D only, eq. (3.7))
//   BMh : four-point central flux of the mixed bottom derivative (2D only)
template <class T, int N> struct Iface {
  T Fh[N], bh[N], Dh[N], Bh, Mh[N], BMh;
};

template <class T, int N>
Iface<T, N> interface_flux(const T L[N][N], const T R[N][N], int slot, T alpha, T dx, T eps,
                           const T U[4][N], const T D[4][N], const T F[4][N], const T P[4][N],
                           const T b[4], const T Bn[4], const T M[4][N], const T Bt[4]) {
  static const T half = T(1) / T(2);
  Iface<T, N> o;
  for (int c = 0; c < N; ++c) { o.Fh[c] = T(0); o.bh[c] = T(0); o.Dh[c] = T(0); o.Mh[c] = T(0); }
  o.Bh = T(0); o.BMh = T(0);
  T wF[2][N], wb[2][N];
  for (int sd = 0; sd < 2; ++sd) {
    const bool plus = (sd == 0);
    const int st[3] = {plus ? 0 : 3, plus ? 1 : 2, plus ? 2 : 1};  // upwind stencil order
    // Lax-Friedrichs split (eq. (2.4)) and the source split b~^± = b~/2, B~^± = B~/2.
    T Fs[3][N], Ps[3][N], bs[3], Bs[3];
    for (int n = 0; n < 3; ++n) {
      const int k = st[n];
      for (int c = 0; c < N; ++c) {
        Fs[n][c] = half * (F[k][c] + pm(plus, alpha * U[k][c]));
        Ps[n][c] = half * (P[k][c] + pm(plus, alpha * D[k][c]));
      }
      bs[n] = half * b[k];
      Bs[n] = half * Bn[k];
    }
    // Characteristic-wise nonlinear reconstruction of F^±; the bottom vector reuses the weights.
    for (int ch = 0; ch < N; ++ch) {
      T f[3], p[3], fb[3], pb[3], w[3];
      for (int n = 0; n < 3; ++n) {
        f[n] = dotn<T, N>(L[ch], Fs[n]);
        p[n] = pm(plus, dotn<T, N>(L[ch], Ps[n]));
        fb[n] = L[ch][slot] * bs[n];
        pb[n] = pm(plus, L[ch][slot] * Bs[n]);
      }
      wF[sd][ch] = hweno_value(f, p, dx, eps, w);
      wb[sd][ch] = hweno_with_weights(w, fb, pb, dx);
    }
    // Linear Hermite derivative fluxes, component by component.
    for (int c = 0; c < N; ++c) {
      T f[3], p[3];
      for (int n = 0; n < 3; ++n) { f[n] = Fs[n][c]; p[n] = pm(plus, Ps[n][c]); }
      o.Dh[c] += pm(plus, hermite_dQ(f, p, dx));
    }
    {
      T p[3];
      for (int n = 0; n < 3; ++n) p[n] = pm(plus, Bs[n]);
      o.Bh += pm(plus, hermite_dQ(bs, p, dx));
    }
  }
  for (int c = 0; c < N; ++c) {
    T sF[N], sb[N];
    for (int ch = 0; ch < N; ++ch) { sF[ch] = wF[0][ch] + wF[1][ch]; sb[ch] = wb[0][ch] + wb[1][ch]; }
    o.Fh[c] = dotn<T, N>(R[c], sF);
    o.bh[c] = dotn<T, N>(R[c], sb);
  }
  if (M) {
    for (int c = 0; c < N; ++c) o.Mh[c] = central4(M[0][c], M[1][c], M[2][c], M[3][c]);
    o.BMh = central4(Bt[0], Bt[1], Bt[2], Bt[3]);
  }
  return o;
}

}  // namespace orc
