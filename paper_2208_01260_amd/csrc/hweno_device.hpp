// Device arithmetic of the well-balanced fifth-order finite-difference HWENO scheme for the
// shallow water equations (Zhao & Zhang, arXiv 2208.01260), FP64, for gfx950.
//
// Everything here works in the frame of one sweep direction: a vector (eta, m_n, m_t) holds
// the surface, the momentum normal to the interfaces of the sweep and the tangential one. The
// y-sweep is then the x-sweep applied to (eta, w, m) with the roles of the x- and
// y-derivatives exchanged, so one device routine serves both directions.
#pragma once
#include <hip/hip_runtime.h>

namespace swe {

// Slots of a raw node record (paper variables, 2D order; 1D uses eta, m, H1=H, M1=M, b, B1=B).
enum { S_ETA = 0, S_M, S_W, S_H1, S_M1, S_W1, S_H2, S_M2, S_W2, S_B, S_BX, S_BY, NREC };

// Constants of the reconstructions (Sec. 2.1 and 2.2).
constexpr double K16 = 1.0 / 6.0, K112 = 1.0 / 12.0, K133 = 13.0 / 3.0, K1312 = 13.0 / 12.0;
constexpr double K78120 = 781.0 / 20.0, K78180 = 781.0 / 80.0;

// Reciprocal for operands in the normal range: hardware estimate refined by two Newton steps
// (error below one unit in the last place; the inputs here are depths, wave speeds and sums of
// squared smoothness indicators, never zero, denormal or infinite).
__device__ __forceinline__ double rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// One node seen from a sweep: U, its derivative along the sweep D, the normal flux F, its
// derivative along the sweep P (Phi_1 for x, Psi_2 for y) and across it Q (the mixed term:
// Psi_1 for x, Phi_2 for y), the bottom and its two derivatives.
struct NodeF {
  double e, mn, mt;
  double d0, d1, d2;
  double f0, f1, f2;
  double p0, p1, p2;
  double q0, q1, q2;
  double b, bn, bt;
};

// Fluxes of eq. (3.3) and their total derivatives dF/dU D + dF/db B (eq. (3.5)).
template <int DIR>
__device__ __forceinline__ void node_frame(const double* __restrict__ r, double g, NodeF& o) {
  const double e = r[S_ETA], b = r[S_B];
  const double mn = DIR == 0 ? r[S_M] : r[S_W];
  const double mt = DIR == 0 ? r[S_W] : r[S_M];
  const double dn0 = DIR == 0 ? r[S_H1] : r[S_H2];
  const double dn1 = DIR == 0 ? r[S_M1] : r[S_W2];
  const double dn2 = DIR == 0 ? r[S_W1] : r[S_M2];
  const double dt0 = DIR == 0 ? r[S_H2] : r[S_H1];
  const double dt1 = DIR == 0 ? r[S_M2] : r[S_W1];
  const double dt2 = DIR == 0 ? r[S_W2] : r[S_M1];
  const double bn = DIR == 0 ? r[S_BX] : r[S_BY];
  const double bt = DIR == 0 ? r[S_BY] : r[S_BX];
  const double h = e - b, ih = rcp(h);
  const double un = mn * ih, ut = mt * ih;
  const double j10 = g * h - un * un, j11 = 2.0 * un, j20 = -(un * ut);
  const double jb1 = un * un - g * e, jb2 = un * ut;
  o.e = e; o.mn = mn; o.mt = mt;
  o.d0 = dn0; o.d1 = dn1; o.d2 = dn2;
  o.f0 = mn;
  o.f1 = mn * un + g * e * (0.5 * e - b);
  o.f2 = mn * ut;
  o.p0 = dn1;
  o.p1 = j10 * dn0 + j11 * dn1 + jb1 * bn;
  o.p2 = j20 * dn0 + ut * dn1 + un * dn2 + jb2 * bn;
  o.q0 = dt1;
  o.q1 = j10 * dt0 + j11 * dt1 + jb1 * bt;
  o.q2 = j20 * dt0 + ut * dt1 + un * dt2 + jb2 * bt;
  o.b = b; o.bn = bn; o.bt = bt;
}

struct W3 { double w1, w2, w3; };

// Upwind HWENO value at x_{i+1/2} from the stencil (i-1, i, i+1): f are split flux values,
// s = dx * (split derivative-flux values). Smoothness indicators and candidate values of
// Sec. 2.1; the weights gamma_l / (beta_l + eps)^2, normalised, are formed with one division as
// gamma_1 e2 e3 : gamma_2 e1 e3 : gamma_3 e1 e2 with e_l = (beta_l + eps)^2.
__device__ __forceinline__ double hweno_side(double f0, double f1, double f2, double s0, double s1, double s2,
                                             double eps, W3& w) {
  const double d01 = f0 - f1, d12 = f1 - f2;
  const double t = s1 * s1;
  const double a1 = 3.0 * d01 + s0 + 2.0 * s1, c1 = 2.0 * d01 + s0 + s1;
  const double a2 = 3.0 * d12 + s2 + 2.0 * s1, c2 = 2.0 * d12 + s2 + s1;
  const double a3 = (f0 + f2) - 2.0 * f1, c3 = (f0 - f2) + 2.0 * s1;
  const double be1 = t + K133 * (a1 * a1) + K78120 * (c1 * c1);
  const double be2 = t + K133 * (a2 * a2) + K78120 * (c2 * c2);
  const double be3 = t + K1312 * (a3 * a3) + K78180 * (c3 * c3);
  const double e1 = (be1 + eps) * (be1 + eps);
  const double e2 = (be2 + eps) * (be2 + eps);
  const double e3 = (be3 + eps) * (be3 + eps);
  const double u1 = 0.3 * (e2 * e3), u2 = 0.3 * (e1 * e3), u3 = 0.4 * (e1 * e2);
  const double is = rcp((u1 + u2) + u3);
  w.w1 = u1 * is; w.w2 = u2 * is; w.w3 = u3 * is;
  const double q1 = 0.5 * (f0 + f1) + K16 * (s0 + 5.0 * s1);
  const double q2 = 0.5 * (f1 + f2) + K16 * (s1 - s2);
  const double q3 = K112 * ((f0 + f2) + 10.0 * f1) + 0.5 * s1;
  return w.w1 * q1 + w.w2 * q2 + w.w3 * q3;
}

// The three candidate values combined with given weights (the source split of Step 2).
__device__ __forceinline__ double hweno_with(double f0, double f1, double f2, double s0, double s1, double s2,
                                             const W3& w) {
  const double q1 = 0.5 * (f0 + f1) + K16 * (s0 + 5.0 * s1);
  const double q2 = 0.5 * (f1 + f2) + K16 * (s1 - s2);
  const double q3 = K112 * ((f0 + f2) + 10.0 * f1) + 0.5 * s1;
  return w.w1 * q1 + w.w2 * q2 + w.w3 * q3;
}

// Interface quantities at x_{i+1/2}, frame order (eta, n, t).
struct IfO {
  double F0, F1, F2;  // nonlinear flux F^ = F^+ + F^-
  double B0, B1, B2;  // bottom vector reconstructed with the flux's projection and weights
  double P0, P1, P2;  // linear Hermite flux of the derivative equation along the sweep
  double PB;          // its bottom-derivative counterpart (n component)
  double M0, M1, M2;  // four-point central flux of the mixed derivative flux
  double MB;          // four-point central flux of the mixed bottom derivative (n component)
};

// Interface x_{i+1/2} of a sweep. fetch(k, X) provides the fluxes of node i-1+k (k = 0..3),
// either computed from a raw record or read from where another lane left them; nodes are
// fetched and projected one at a time so that only one node's quantities are live.
// alpha = Lax-Friedrichs speed of this direction.
template <class Fetch>
__device__ __forceinline__ void interface_flux(Fetch fetch, double alpha, double dx, double eps, double g, IfO& o) {
  NodeF XB, XC;
  fetch(1, XB);
  fetch(2, XC);
  // characteristic matrices at the arithmetic mean of the two adjacent nodes
  const double em = 0.5 * (XB.e + XC.e), mnm = 0.5 * (XB.mn + XC.mn), mtm = 0.5 * (XB.mt + XC.mt);
  const double bm = 0.5 * (XB.b + XC.b);
  const double h = em - bm, ih = rcp(h);
  const double un = mnm * ih, ut = mtm * ih;
  const double cs = sqrt(g * h), i2c = 0.5 * rcp(cs);
  const double l1a = (un + cs) * i2c, l3a = (cs - un) * i2c;
  // rows: l1 = (l1a, -i2c, 0), l2 = (-ut, 0, 1), l3 = (l3a, i2c, 0)
  const double ha = 0.5 * alpha, hdx = 0.5 * dx, hadx = ha * dx;

  // projected, split values: f^± = (L F ± alpha L U)/2, s^± = dx (L P ± alpha L D)/2
  double fpA[3], spA[3], fpB[3], spB[3], fmB[3], smB[3], fpC[3], spC[3], fmC[3], smC[3], fmD[3], smD[3];
  double bA, bB, bC, bD, sbA, sbB, sbC, sbD;  // bottom and dx * its derivative along the sweep
  double q1s[4], q7s[4];                      // partial sums of the mixed four-point flux
#define SWE_PROJ(X, FP, SP, FM, SM, PLUS, MINUS)                                                  \
  {                                                                                               \
    const double lf[3] = {l1a * X.f0 - i2c * X.f1, X.f2 - ut * X.f0, l3a * X.f0 + i2c * X.f1}; \
    const double lu[3] = {l1a * X.e - i2c * X.mn, X.mt - ut * X.e, l3a * X.e + i2c * X.mn};    \
    const double lp[3] = {l1a * X.p0 - i2c * X.p1, X.p2 - ut * X.p0, l3a * X.p0 + i2c * X.p1}; \
    const double ld[3] = {l1a * X.d0 - i2c * X.d1, X.d2 - ut * X.d0, l3a * X.d0 + i2c * X.d1}; \
    _Pragma("unroll") for (int k = 0; k < 3; ++k) {                                               \
      if (PLUS) { FP[k] = 0.5 * lf[k] + ha * lu[k]; SP[k] = hdx * lp[k] + hadx * ld[k]; }         \
      if (MINUS) { FM[k] = 0.5 * lf[k] - ha * lu[k]; SM[k] = hdx * lp[k] - hadx * ld[k]; }        \
    }                                                                                             \
  }
  double dummy[3];
  SWE_PROJ(XB, fpB, spB, fmB, smB, true, true)
  bB = XB.b; sbB = dx * XB.bn;
  q7s[0] = XB.q0; q7s[1] = XB.q1; q7s[2] = XB.q2; q7s[3] = XB.bt;
  SWE_PROJ(XC, fpC, spC, fmC, smC, true, true)
  bC = XC.b; sbC = dx * XC.bn;
  q7s[0] += XC.q0; q7s[1] += XC.q1; q7s[2] += XC.q2; q7s[3] += XC.bt;
  {
    NodeF X;
    fetch(0, X);
    SWE_PROJ(X, fpA, spA, dummy, dummy, true, false)
    bA = X.b; sbA = dx * X.bn;
    q1s[0] = X.q0; q1s[1] = X.q1; q1s[2] = X.q2; q1s[3] = X.bt;
  }
  {
    NodeF X;
    fetch(3, X);
    SWE_PROJ(X, dummy, dummy, fmD, smD, false, true)
    bD = X.b; sbD = dx * X.bn;
    q1s[0] += X.q0; q1s[1] += X.q1; q1s[2] += X.q2; q1s[3] += X.bt;
  }
#undef SWE_PROJ

  // nonlinear reconstruction per characteristic field and side; the bottom reuses the weights
  const double i4dx = 0.25 / dx, i12dx = K112 / dx;
  double s[3], t[3], Z1 = 0.0, Z3 = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    W3 wp, wm;
    const double vp = hweno_side(fpA[k], fpB[k], fpC[k], spA[k], spB[k], spC[k], eps, wp);
    const double vm = hweno_side(fmD[k], fmC[k], fmB[k], -smD[k], -smC[k], -smB[k], eps, wm);
    s[k] = vp + vm;
    if (k != 1) {  // the middle characteristic row annihilates (0, b, 0)
      const double z = hweno_with(bA, bB, bC, sbA, sbB, sbC, wp) + hweno_with(bD, bC, bB, -sbD, -sbC, -sbB, wm);
      if (k == 0) Z1 = z; else Z3 = z;
    }
    // linear Hermite derivative Q'^+(f^+, s^+/dx) + Q'^-(f^-, s^-/dx) of this characteristic field
    t[k] = ((fpA[k] - fmD[k]) + 8.0 * (fmC[k] - fpB[k]) + 7.0 * (fpC[k] - fmB[k])) * i4dx +
           ((spA[k] + smD[k]) - 2.0 * (spB[k] + smC[k]) - 5.0 * (spC[k] + smB[k])) * i12dx;
  }
  // back to the conservative frame: R columns (1, un-c, ut), (0, 0, 1), (1, un+c, ut)
  const double umc = un - cs, upc = un + cs;
  o.F0 = s[0] + s[2];
  o.F1 = umc * s[0] + upc * s[2];
  o.F2 = ut * (s[0] + s[2]) + s[1];
  // char. projections of b~^± = (0, b/2, 0): -i2c b / 2 (row 1), +i2c b / 2 (row 3)
  const double sb1 = -0.5 * i2c * Z1, sb3 = 0.5 * i2c * Z3;
  o.B0 = sb1 + sb3;
  o.B1 = umc * sb1 + upc * sb3;
  o.B2 = ut * (sb1 + sb3);
  // the linear derivative-equation flux: componentwise Q' is R (char.-wise Q') since L is fixed
  o.P0 = t[0] + t[2];
  o.P1 = umc * t[0] + upc * t[2];
  o.P2 = ut * (t[0] + t[2]) + t[1];
  // bottom derivative, n component: Q'^+(b/2, B/2) + Q'^-(b/2, B/2)
  o.PB = 0.5 * (((bA - bD) + 15.0 * (bC - bB)) * i4dx + ((sbA + sbD) - 7.0 * (sbB + sbC)) * i12dx);
  // four-point central flux of the mixed terms (eq. (3.7))
  o.M0 = K112 * (7.0 * q7s[0] - q1s[0]);
  o.M1 = K112 * (7.0 * q7s[1] - q1s[1]);
  o.M2 = K112 * (7.0 * q7s[2] - q1s[2]);
  o.MB = K112 * (7.0 * q7s[3] - q1s[3]);
}

// HWENO limiter of one characteristic component (Sec. 2.2): mu at x_{i-1}, x_i, x_{i+1}, nu at
// x_{i-1}, x_{i+1}; linear weights (1/4, 1/4, 1/2).
__device__ __forceinline__ double limit_char(double mm, double m0, double mp, double nm, double np, double dx,
                                             double idx, double eps) {
  const double a1 = 2.0 * (m0 - mm) - nm * dx;       // dx * p1'(x_i)
  const double a2 = 2.0 * (mp - m0) - np * dx;       // dx * p2'(x_i)
  const double a3 = 0.5 * (mp - mm);                 // dx * p3'(x_i)
  const double c1 = (m0 - mm) - nm * dx, c2 = (mp - m0) - np * dx, c3 = (mm + mp) - 2.0 * m0;
  const double be1 = a1 * a1 + K133 * (c1 * c1);
  const double be2 = a2 * a2 + K133 * (c2 * c2);
  const double be3 = a3 * a3 + K1312 * (c3 * c3);
  const double e1 = (be1 + eps) * (be1 + eps), e2 = (be2 + eps) * (be2 + eps), e3 = (be3 + eps) * (be3 + eps);
  const double u1 = 0.25 * (e2 * e3), u2 = 0.25 * (e1 * e3), u3 = 0.5 * (e1 * e2);
  const double is = rcp((u1 + u2) + u3);
  return ((u1 * a1 + u2 * a2) + u3 * a3) * is * idx;
}

// Limited derivative at a node in the frame of one direction: own state (e, mn, mt, b);
// neighbour surface/momenta at -1 and +1; neighbour derivatives along this direction at -1, +1.
__device__ __forceinline__ void limit_frame(double e0, double mn0, double mt0, double b0, double em, double mnm,
                                            double mtm, double ep, double mnp, double mtp, double dm0, double dm1,
                                            double dm2, double dp0, double dp1, double dp2, double dx, double idx,
                                            double eps, double g, double out[3]) {
  const double h = e0 - b0, ih = rcp(h);
  const double un = mn0 * ih, ut = mt0 * ih;
  const double cs = sqrt(g * h), i2c = 0.5 * rcp(cs);
  const double l1a = (un + cs) * i2c, l3a = (cs - un) * i2c;
  const double v1 = limit_char(l1a * em - i2c * mnm, l1a * e0 - i2c * mn0, l1a * ep - i2c * mnp,
                               l1a * dm0 - i2c * dm1, l1a * dp0 - i2c * dp1, dx, idx, eps);
  const double v2 = limit_char(mtm - ut * em, mt0 - ut * e0, mtp - ut * ep, dm2 - ut * dm0, dp2 - ut * dp0, dx, idx, eps);
  const double v3 = limit_char(l3a * em + i2c * mnm, l3a * e0 + i2c * mn0, l3a * ep + i2c * mnp,
                               l3a * dm0 + i2c * dm1, l3a * dp0 + i2c * dp1, dx, idx, eps);
  out[0] = v1 + v3;
  out[1] = (un - cs) * v1 + (un + cs) * v3;
  out[2] = ut * (v1 + v3) + v2;
}

}  // namespace swe
