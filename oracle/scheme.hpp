// TEST INFRASTRUCTURE — the CPU oracle's semi-discrete scheme and time stepping (1D and 2D).
// Only the test suite, the smoke check and the CPU-baseline leg of the benchmark may use it.
//
// State layout (flat, interior nodes only, x fastest):
//   1D: U = (eta, m),    D = (H, M)                       — 2 + 2 planes of nx
//   2D: U = (eta, m, w), D = (H1, M1, W1, H2, M2, W2)     — 3 + 6 planes of nx*ny
// The bottom b and its derivatives (B = b_x [, b_y]) are static.
#pragma once
#include <cmath>
#include <cstring>
#include <vector>

#include "hweno_oracle.hpp"

#ifdef _OPENMP
#include <omp.h>
#endif

namespace orc {

#define ORC_PARALLEL_FOR _Pragma("omp parallel for schedule(static) if(parallel_ok<T>::value)")

// SSP-RK3 with modified derivatives (eq. (2.11)). U: equilibrium variables, D: their
// derivatives (flattened). f(k, U, D, RU, RD) evaluates the right-hand side of stage k,
// lim(U, D, Dmod) the limited derivatives. Read literally, the right-hand side takes the
// unmodified stage derivatives and the limited ones are the Runge-Kutta base; with lim_first the
// right-hand side takes the limited ones instead.
template <class T, class Rhs, class Lim>
void ssprk3(T* U, T* D, size_t NU, size_t ND, T dt, Rhs f, Lim lim, bool lim_first) {
  // The convex combinations are written over a common denominator, (3a + b)/4 and (a + 2b)/3:
  // the same arithmetic as 3/4 a + 1/4 b and 1/3 a + 2/3 b, but a constant state stays exactly
  // constant, and the lake-at-rest round-off then matches the magnitudes printed in Tables 1-3.
  std::vector<T> Dn(ND), U1(NU), D1(ND), U2(NU), D2(ND), RU(NU), RD(ND), Dm(ND);
  // stage 1: U1 = U^n + dt R(U^n, V^n),  D1 = D^{n,mod} + dt R_x(U^n, V^n)
  lim(U, D, Dn.data());
  f(0, U, lim_first ? Dn.data() : D, RU.data(), RD.data());
  for (size_t q = 0; q < NU; ++q) U1[q] = U[q] + dt * RU[q];
  for (size_t q = 0; q < ND; ++q) D1[q] = Dn[q] + dt * RD[q];
  // stage 2: U2 = 3/4 U^n + 1/4 (U1 + dt R(S1)),  D2 = 3/4 D^{n,mod} + 1/4 (D1^mod + dt R_x(S1))
  lim(U1.data(), D1.data(), Dm.data());
  f(1, U1.data(), lim_first ? Dm.data() : D1.data(), RU.data(), RD.data());
  for (size_t q = 0; q < NU; ++q) U2[q] = (T(3) * U[q] + (U1[q] + dt * RU[q])) / T(4);
  for (size_t q = 0; q < ND; ++q) D2[q] = (T(3) * Dn[q] + (Dm[q] + dt * RD[q])) / T(4);
  // stage 3: U^{n+1} = 1/3 U^n + 2/3 (U2 + dt R(S2)),  D^{n+1} = 1/3 D^{n,mod} + 2/3 (D2^mod + dt R_x(S2))
  lim(U2.data(), D2.data(), Dm.data());
  f(2, U2.data(), lim_first ? Dm.data() : D2.data(), RU.data(), RD.data());
  for (size_t q = 0; q < NU; ++q) U[q] = (U[q] + T(2) * (U2[q] + dt * RU[q])) / T(3);
  for (size_t q = 0; q < ND; ++q) D[q] = (Dn[q] + T(2) * (Dm[q] + dt * RD[q])) / T(3);
}

template <class T> struct Scheme {
  Params<T> P;
  int nu = 0, nd = 0;   // number of U planes and D planes
  size_t n = 0;         // nodes per plane
  Plane<T> b, B1, B2;
  int err = OK;

  bool two_d() const { return P.dim == 2; }

  void setup(const Params<T>& p, const T* bb, const T* bx, const T* by) {
    P = p;
    n = (size_t)P.nx * (size_t)(two_d() ? P.ny : 1);
    nu = two_d() ? 3 : 2;
    nd = two_d() ? 6 : 2;
    const int ny = two_d() ? P.ny : 1;
    b.init(P.nx, ny, 2, two_d()); B1.init(P.nx, ny, 2, two_d()); B2.init(P.nx, ny, 2, two_d());
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < P.nx; ++i) {
        const size_t q = (size_t)j * P.nx + i;
        b(i, j) = bb[q];
        B1(i, j) = bx[q];
        B2(i, j) = two_d() ? by[q] : T(0);
      }
    // parities across an x-wall / y-wall: b even, b_x odd across x, b_y odd across y
    fill_ghosts(b, P.bcx, P.bcy, +1, +1);
    fill_ghosts(B1, P.bcx, P.bcy, -1, +1);
    fill_ghosts(B2, P.bcx, P.bcy, +1, -1);
  }

  // Load interior planes into padded planes and fill their ghosts.
  void load(const T* U, const T* D, std::vector<Plane<T>>& Up, std::vector<Plane<T>>& Dp) const {
    static const int ux1[2] = {+1, -1}, dx1[2] = {-1, +1};
    static const int ux2[3] = {+1, -1, +1}, uy2[3] = {+1, +1, -1};
    static const int dx2[6] = {-1, +1, -1, +1, -1, +1}, dy2[6] = {+1, +1, -1, -1, -1, +1};
    const int ny = two_d() ? P.ny : 1;
    Up.resize(nu); Dp.resize(nd);
    for (int f = 0; f < nu + nd; ++f) {
      Plane<T>& pl = f < nu ? Up[f] : Dp[f - nu];
      const T* src = f < nu ? U + (size_t)f * n : D + (size_t)(f - nu) * n;
      pl.init(P.nx, ny, 2, two_d());
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < P.nx; ++i) pl(i, j) = src[(size_t)j * P.nx + i];
      int px, py = +1;
      if (two_d()) { px = f < nu ? ux2[f] : dx2[f - nu]; py = f < nu ? uy2[f] : dy2[f - nu]; }
      else px = f < nu ? ux1[f] : dx1[f - nu];
      fill_ghosts(pl, P.bcx, P.bcy, px, py);
    }
  }

  // Lax-Friedrichs speeds of a state: max |u|+c and max |v|+c over the nodes (reading A-1).
  void alpha(const T* U, T& ax, T& ay) {
    ax = T(0); ay = T(0);
    for (size_t q = 0; q < n; ++q) {
      const int j = (int)(q / P.nx), i = (int)(q % P.nx);
      const T h = U[q] - b(i, j);
      const double hd = to_double(h);
      if (!std::isfinite(to_double(U[q])) || !std::isfinite(to_double(U[n + q])) ||
          (two_d() && !std::isfinite(to_double(U[2 * n + q])))) { err = E_NONFINITE; continue; }
      if (!(hd > 0)) { err = E_DRY; continue; }
      const T c = sqrt_(P.g * h);
      ax = max_(ax, abs_(U[n + q] / h) + c);
      if (two_d()) ay = max_(ay, abs_(U[2 * n + q] / h) + c);
    }
  }

  // ------------------------------------------------------------ right-hand side, 1D (eq. (2.8))
  void rhs_1d(const T* U, const T* D, T ax, T* RU, T* RD) const {
    std::vector<Plane<T>> Up, Dp;
    load(U, D, Up, Dp);
    const int nx = P.nx;
    const T g = P.g, idx = T(1) / P.dx;
    std::vector<T> Un((size_t)4 * (nx + 4)), Vn(Un.size()), Fn(Un.size()), Pn(Un.size()),
        bn(nx + 4), Bn(nx + 4);
    for (int i = -2; i <= nx + 1; ++i) {
      const int s = i + 2;
      T u[2] = {Up[0](i, 0), Up[1](i, 0)}, v[2] = {Dp[0](i, 0), Dp[1](i, 0)}, F[2], Ph[2];
      flux_1d(u, b(i, 0), g, F);
      dflux_1d(u, b(i, 0), v, B1(i, 0), g, Ph);
      for (int c = 0; c < 2; ++c) { Un[2 * s + c] = u[c]; Vn[2 * s + c] = v[c]; Fn[2 * s + c] = F[c]; Pn[2 * s + c] = Ph[c]; }
      bn[s] = b(i, 0); Bn[s] = B1(i, 0);
    }
    std::vector<Iface<T, 2>> fx(nx + 1);
    for (int i = -1; i <= nx - 1; ++i) {  // interface i+1/2 uses nodes i-1..i+2
      T u4[4][2], v4[4][2], f4[4][2], p4[4][2], b4[4], B4[4];
      for (int k = 0; k < 4; ++k) {
        const int s = i - 1 + k + 2;
        for (int c = 0; c < 2; ++c) { u4[k][c] = Un[2 * s + c]; v4[k][c] = Vn[2 * s + c]; f4[k][c] = Fn[2 * s + c]; p4[k][c] = Pn[2 * s + c]; }
        b4[k] = bn[s]; B4[k] = Bn[s];
      }
      T L[2][2], R[2][2];
      static const T half = T(1) / T(2);
      eig_1d(half * (u4[1][0] + u4[2][0]), half * (u4[1][1] + u4[2][1]), half * (b4[1] + b4[2]), g, L, R);
      fx[i + 1] = interface_flux<T, 2>(L, R, 1, ax, P.dx, P.eps, u4, v4, f4, p4, b4, B4, nullptr, nullptr);
    }
    for (int i = 0; i < nx; ++i) {
      const Iface<T, 2>& r = fx[i + 1];
      const Iface<T, 2>& l = fx[i];
      const T eta = Up[0](i, 0), H = Dp[0](i, 0);
      for (int c = 0; c < 2; ++c) {
        const T db = r.bh[c] - l.bh[c];
        RU[(size_t)c * nx + i] = -((r.Fh[c] - l.Fh[c]) + g * eta * db) * idx;
        T dv = (r.Dh[c] - l.Dh[c]) + g * H * db;
        if (c == 1) dv += g * eta * (r.Bh - l.Bh);
        RD[(size_t)c * nx + i] = -dv * idx;
      }
    }
  }

  // ------------------------------------------------------------ right-hand side, 2D (eq. (3.8))
  void rhs_2d(const T* U, const T* D, T ax, T ay, T* RU, T* RD) const {
    std::vector<Plane<T>> Up, Dp;
    load(U, D, Up, Dp);
    const int nx = P.nx, ny = P.ny;
    const T g = P.g, idx = T(1) / P.dx, idy = T(1) / P.dy;
    static const T half = T(1) / T(2);

    // x-sweep: (F1, Phi1) by Step 1, (b~, B~1) by Step 2, mixed Psi1 and B~2 by eq. (3.7).
    ORC_PARALLEL_FOR
    for (int j = 0; j < ny; ++j) {
      const int m = nx + 4;
      std::vector<T> Un(3 * m), Vn(3 * m), Fn(3 * m), Pn(3 * m), Mn(3 * m), bn(m), Bn(m), Bt(m);
      for (int i = -2; i <= nx + 1; ++i) {
        const int s = i + 2;
        T u[3], v[3], q[3], J[3][3], Jb[3];
        for (int c = 0; c < 3; ++c) { u[c] = Up[c](i, j); v[c] = Dp[c](i, j); q[c] = Dp[3 + c](i, j); }
        flux_x(u, b(i, j), g, &Fn[3 * s]);
        jac_x(u, b(i, j), g, J, Jb);
        jmul(J, Jb, v, B1(i, j), &Pn[3 * s]);  // Phi1
        jmul(J, Jb, q, B2(i, j), &Mn[3 * s]);  // Psi1 (mixed)
        for (int c = 0; c < 3; ++c) { Un[3 * s + c] = u[c]; Vn[3 * s + c] = v[c]; }
        bn[s] = b(i, j); Bn[s] = B1(i, j); Bt[s] = B2(i, j);
      }
      std::vector<Iface<T, 3>> fx(nx + 1);
      for (int i = -1; i <= nx - 1; ++i) {
        T u4[4][3], v4[4][3], f4[4][3], p4[4][3], m4[4][3], b4[4], Bn4[4], Bt4[4];
        for (int k = 0; k < 4; ++k) {
          const int s = i - 1 + k + 2;
          for (int c = 0; c < 3; ++c) {
            u4[k][c] = Un[3 * s + c]; v4[k][c] = Vn[3 * s + c]; f4[k][c] = Fn[3 * s + c];
            p4[k][c] = Pn[3 * s + c]; m4[k][c] = Mn[3 * s + c];
          }
          b4[k] = bn[s]; Bn4[k] = Bn[s]; Bt4[k] = Bt[s];
        }
        T L[3][3], R[3][3];
        eig_x(half * (u4[1][0] + u4[2][0]), half * (u4[1][1] + u4[2][1]), half * (u4[1][2] + u4[2][2]),
              half * (b4[1] + b4[2]), g, L, R);
        fx[i + 1] = interface_flux<T, 3>(L, R, 1, ax, P.dx, P.eps, u4, v4, f4, p4, b4, Bn4, m4, Bt4);
      }
      for (int i = 0; i < nx; ++i) {
        const Iface<T, 3>& r = fx[i + 1];
        const Iface<T, 3>& l = fx[i];
        const size_t q = (size_t)j * nx + i;
        const T eta = Up[0](i, j), H1 = Dp[0](i, j), H2 = Dp[3](i, j);
        for (int c = 0; c < 3; ++c) {
          const T db = r.bh[c] - l.bh[c];
          RU[c * n + q] = -((r.Fh[c] - l.Fh[c]) + g * eta * db) * idx;
          T dv = (r.Dh[c] - l.Dh[c]) + g * H1 * db;
          T dq = (r.Mh[c] - l.Mh[c]) + g * H2 * db;
          if (c == 1) { dv += g * eta * (r.Bh - l.Bh); dq += g * eta * (r.BMh - l.BMh); }
          RD[c * n + q] = -dv * idx;
          RD[(3 + c) * n + q] = -dq * idx;
        }
      }
    }

    // y-sweep: (F2, Psi2) by Step 1, (b-, B-2) by Step 2, mixed Phi2 and B-1 by eq. (3.7).
    ORC_PARALLEL_FOR
    for (int i = 0; i < nx; ++i) {
      const int m = ny + 4;
      std::vector<T> Un(3 * m), Qn(3 * m), Fn(3 * m), Pn(3 * m), Mn(3 * m), bn(m), Bn(m), Bt(m);
      for (int j = -2; j <= ny + 1; ++j) {
        const int s = j + 2;
        T u[3], v[3], q[3], J[3][3], Jb[3];
        for (int c = 0; c < 3; ++c) { u[c] = Up[c](i, j); v[c] = Dp[c](i, j); q[c] = Dp[3 + c](i, j); }
        flux_y(u, b(i, j), g, &Fn[3 * s]);
        jac_y(u, b(i, j), g, J, Jb);
        jmul(J, Jb, q, B2(i, j), &Pn[3 * s]);  // Psi2
        jmul(J, Jb, v, B1(i, j), &Mn[3 * s]);  // Phi2 (mixed)
        for (int c = 0; c < 3; ++c) { Un[3 * s + c] = u[c]; Qn[3 * s + c] = q[c]; }
        bn[s] = b(i, j); Bn[s] = B2(i, j); Bt[s] = B1(i, j);
      }
      std::vector<Iface<T, 3>> fy(ny + 1);
      for (int j = -1; j <= ny - 1; ++j) {
        T u4[4][3], q4[4][3], f4[4][3], p4[4][3], m4[4][3], b4[4], Bn4[4], Bt4[4];
        for (int k = 0; k < 4; ++k) {
          const int s = j - 1 + k + 2;
          for (int c = 0; c < 3; ++c) {
            u4[k][c] = Un[3 * s + c]; q4[k][c] = Qn[3 * s + c]; f4[k][c] = Fn[3 * s + c];
            p4[k][c] = Pn[3 * s + c]; m4[k][c] = Mn[3 * s + c];
          }
          b4[k] = bn[s]; Bn4[k] = Bn[s]; Bt4[k] = Bt[s];
        }
        T L[3][3], R[3][3];
        eig_y(half * (u4[1][0] + u4[2][0]), half * (u4[1][1] + u4[2][1]), half * (u4[1][2] + u4[2][2]),
              half * (b4[1] + b4[2]), g, L, R);
        fy[j + 1] = interface_flux<T, 3>(L, R, 2, ay, P.dy, P.eps, u4, q4, f4, p4, b4, Bn4, m4, Bt4);
      }
      for (int j = 0; j < ny; ++j) {
        const Iface<T, 3>& r = fy[j + 1];
        const Iface<T, 3>& l = fy[j];
        const size_t q = (size_t)j * nx + i;
        const T eta = Up[0](i, j), H1 = Dp[0](i, j), H2 = Dp[3](i, j);
        for (int c = 0; c < 3; ++c) {
          const T db = r.bh[c] - l.bh[c];
          RU[c * n + q] -= ((r.Fh[c] - l.Fh[c]) + g * eta * db) * idy;
          T dq = (r.Dh[c] - l.Dh[c]) + g * H2 * db;
          T dv = (r.Mh[c] - l.Mh[c]) + g * H1 * db;
          if (c == 2) { dq += g * eta * (r.Bh - l.Bh); dv += g * eta * (r.BMh - l.BMh); }
          RD[(3 + c) * n + q] -= dq * idy;
          RD[c * n + q] -= dv * idy;
        }
      }
    }
  }

  void rhs(const T* U, const T* D, T ax, T ay, T* RU, T* RD) const {
    if (two_d()) rhs_2d(U, D, ax, ay, RU, RD);
    else rhs_1d(U, D, ax, RU, RD);
  }

  // ------------------------------------------------------------ HWENO limiter (Sec. 2.2, 3)
  void limit(const T* U, const T* D, T* Dm) const {
    std::vector<Plane<T>> Up, Dp;
    load(U, D, Up, Dp);
    const int nx = P.nx, ny = two_d() ? P.ny : 1;
    ORC_PARALLEL_FOR
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const size_t q = (size_t)j * nx + i;
        if (!two_d()) {
          T L[2][2], R[2][2], nm[2];
          eig_1d(Up[0](i, j), Up[1](i, j), b(i, j), P.g, L, R);
          for (int ch = 0; ch < 2; ++ch) {
            T mu[3], nu[2];
            for (int l = -1; l <= 1; ++l) { T u[2] = {Up[0](i + l, j), Up[1](i + l, j)}; mu[l + 1] = dotn<T, 2>(L[ch], u); }
            for (int s = 0; s < 2; ++s) { const int l = s ? 1 : -1; T v[2] = {Dp[0](i + l, j), Dp[1](i + l, j)}; nu[s] = dotn<T, 2>(L[ch], v); }
            nm[ch] = hweno_limit(mu[0], mu[1], mu[2], nu[0], nu[1], P.dx, P.eps);
          }
          for (int c = 0; c < 2; ++c) Dm[c * n + q] = dotn<T, 2>(R[c], nm);
          continue;
        }
        for (int dir = 0; dir < 2; ++dir) {  // V with x-neighbours, Q with y-neighbours
          T L[3][3], R[3][3], nm[3];
          if (dir == 0) eig_x(Up[0](i, j), Up[1](i, j), Up[2](i, j), b(i, j), P.g, L, R);
          else eig_y(Up[0](i, j), Up[1](i, j), Up[2](i, j), b(i, j), P.g, L, R);
          const int di = dir == 0 ? 1 : 0, dj = dir == 0 ? 0 : 1;
          const T h = dir == 0 ? P.dx : P.dy;
          for (int ch = 0; ch < 3; ++ch) {
            T mu[3], nu[2];
            for (int l = -1; l <= 1; ++l) {
              T u[3] = {Up[0](i + l * di, j + l * dj), Up[1](i + l * di, j + l * dj), Up[2](i + l * di, j + l * dj)};
              mu[l + 1] = dotn<T, 3>(L[ch], u);
            }
            for (int s = 0; s < 2; ++s) {
              const int l = s ? 1 : -1;
              T v[3];
              for (int c = 0; c < 3; ++c) v[c] = Dp[3 * dir + c](i + l * di, j + l * dj);
              nu[s] = dotn<T, 3>(L[ch], v);
            }
            nm[ch] = hweno_limit(mu[0], mu[1], mu[2], nu[0], nu[1], h, P.eps);
          }
          for (int c = 0; c < 3; ++c) Dm[(3 * dir + c) * n + q] = dotn<T, 3>(R[c], nm);
        }
      }
  }

  // ------------------------------------------------------------ one SSP-RK3 step (eq. (2.11))
  // S = (U, D) in place. Returns the dt used.
  T step(T* S, T dt_in) {
    T* U = S;
    T* D = S + (size_t)nu * n;
    const bool fixed_alpha = (P.flags & FL_FIXED_ALPHA) != 0;
    const bool no_lim = (P.flags & FL_NO_LIMITER) != 0;
    T ax, ay;
    alpha(U, ax, ay);
    if (err) return T(0);
    T dt = dt_in;
    if (!(to_double(dt) > 0)) dt = two_d() ? P.cfl / (ax / P.dx + ay / P.dy) : P.cfl / (ax / P.dx);
    const size_t ND = (size_t)nd * n;
    auto lim = [&](const T* u, const T* d, T* out) {
      if (no_lim) std::memcpy((void*)out, (const void*)d, ND * sizeof(T));
      else limit(u, d, out);
    };
    auto f = [&](int k, const T* u, const T* d, T* ru, T* rd) {
      T a, c;
      if (fixed_alpha) { a = P.ax_fixed[k]; c = P.ay_fixed[k]; }
      else if (k == 0) { a = ax; c = ay; }
      else alpha(u, a, c);
      if (err) return;
      rhs(u, d, a, c, ru, rd);
    };
    ssprk3(U, D, (size_t)nu * n, ND, dt, f, lim, (P.flags & FL_LIMIT_BEFORE_RHS) != 0);
    return err ? T(0) : dt;
  }

  // Advance nsteps steps, or until t_end when t_end > 0 (the last step is clipped to t_end).
  int run(T* S, int nsteps, double t_end, double* t_out, int* steps_out) {
    T t = T(0);
    int k = 0;
    for (; nsteps <= 0 || k < nsteps; ++k) {
      if (t_end > 0 && !(to_double(t) < t_end)) break;
      T dt = (P.flags & FL_FIXED_DT) ? P.fixed_dt : T(0);
      if (t_end > 0) {
        T ax, ay;
        if (!(to_double(dt) > 0)) {
          alpha(S, ax, ay);
          if (err) break;
          dt = two_d() ? P.cfl / (ax / P.dx + ay / P.dy) : P.cfl / (ax / P.dx);
        }
        if (to_double(t + dt) > t_end) dt = T(t_end) - t;
      }
      const T used = step(S, dt);
      if (err) break;
      t = t + used;
    }
    if (t_out) *t_out = to_double(t);
    if (steps_out) *steps_out = k;
    return err;
  }
};

}  // namespace orc
