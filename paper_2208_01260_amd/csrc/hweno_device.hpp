// Device arithmetic of the well-balanced fifth-order finite-difference HWENO scheme for the
// shallow water equations (Zhao & Zhang, arXiv 2208.01260) for gfx950, templated on the
// arithmetic type (double; float for the single-precision variant).
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
// Square roots of the smoothness indicators' coefficients, folded into the differences:
// 13/3, 781/20, 13/12, 781/80.
constexpr double RA = 2.0816659994661326, RC = 6.248999919987197;
constexpr double RB = 1.0408329997330663, RD = 3.1244999599935985;

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
// Single precision: the hardware estimate and one Newton step.
__device__ __forceinline__ float rcp(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  const float e = fmaf(-x, r, 1.0f);
  return fmaf(r, e, r);
}

// Square root of a positive normal argument (g h): the hardware reciprocal square root estimate
// refined by one Goldschmidt step and two residual corrections (equal to the IEEE square root on
// 4M random arguments over 2^-60 .. 2^60). A non-positive argument gives NaN.
__device__ __forceinline__ double sqrt_pos(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double s = x * y, h = 0.5 * y;
  const double r = fma(-s, h, 0.5);
  s = fma(s, r, s);
  h = fma(h, r, h);
  s = fma(fma(-s, s, x), h, s);
  return fma(fma(-s, s, x), h, s);
}
__device__ __forceinline__ float sqrt_pos(float x) { return sqrtf(x); }

// One node seen from a sweep: U, its derivative along the sweep D, the normal flux F, its
// derivative along the sweep P (Phi_1 for x, Psi_2 for y) and across it Q (the mixed term:
// Psi_1 for x, Phi_2 for y), the bottom and its two derivatives.
template <class T>
struct NodeF {
  T e, mn, mt;
  T d0, d1, d2;
  T f0, f1, f2;
  T p0, p1, p2;
  T q0, q1, q2;
  T b, bn, bt;
};

// Fluxes of eq. (3.3) and their total derivatives dF/dU D + dF/db B (eq. (3.5)).
template <int DIR, class T>
__device__ __forceinline__ void node_frame(const T* __restrict__ r, T g, NodeF<T>& o) {
  const T e = r[S_ETA], b = r[S_B];
  const T mn = DIR == 0 ? r[S_M] : r[S_W];
  const T mt = DIR == 0 ? r[S_W] : r[S_M];
  const T dn0 = DIR == 0 ? r[S_H1] : r[S_H2];
  const T dn1 = DIR == 0 ? r[S_M1] : r[S_W2];
  const T dn2 = DIR == 0 ? r[S_W1] : r[S_M2];
  const T dt0 = DIR == 0 ? r[S_H2] : r[S_H1];
  const T dt1 = DIR == 0 ? r[S_M2] : r[S_W1];
  const T dt2 = DIR == 0 ? r[S_W2] : r[S_M1];
  const T bn = DIR == 0 ? r[S_BX] : r[S_BY];
  const T bt = DIR == 0 ? r[S_BY] : r[S_BX];
  const T h = e - b, ih = rcp(h);
  const T un = mn * ih, ut = mt * ih;
  const T j10 = g * h - un * un, j11 = T(2.0) * un, j20 = -(un * ut);
  const T jb1 = un * un - g * e, jb2 = un * ut;
  o.e = e; o.mn = mn; o.mt = mt;
  o.d0 = dn0; o.d1 = dn1; o.d2 = dn2;
  o.f0 = mn;
  o.f1 = mn * un + g * e * (T(0.5) * e - b);
  o.f2 = mn * ut;
  o.p0 = dn1;
  o.p1 = j10 * dn0 + j11 * dn1 + jb1 * bn;
  o.p2 = j20 * dn0 + ut * dn1 + un * dn2 + jb2 * bn;
  o.q0 = dt1;
  o.q1 = j10 * dt0 + j11 * dt1 + jb1 * bt;
  o.q2 = j20 * dt0 + ut * dt1 + un * dt2 + jb2 * bt;
  o.b = b; o.bn = bn; o.bt = bt;
}

// Weights of one side up to a common factor (u_l) and their sum.
template <class T>
struct W3 { T u1, u2, u3, su; };

// Upwind HWENO value at x_{i+1/2} from the stencil (i-1, i, i+1): f are split flux values,
// s = dx * (split derivative-flux values); candidate values and smoothness indicators of
// Sec. 2.1. The value is returned as f1 + N / (2 su): each doubled candidate 2 q_l is written as
// 2 f1 + r_l with the deviations
//   r1 = (f0 - f1) + (s0 + 5 s1) / 3,  r2 = (f2 - f1) + (s1 - s2) / 3,  r3 = (f0 - 2 f1 + f2) / 6 + s1,
// so N = sum_l u_l r_l. Each indicator is s1^2 + (k_a a)^2 + (k_c c)^2 with the square roots k of
// its coefficients folded into the differences a, c (eps is added once to the shared s1^2); the
// first differences are taken from the deviations, 3 d01 + s0 + 2 s1 = 3 (r1 - s1) and
// 3 d12 + s2 + 2 s1 = 3 (s1 - r2). The weights gamma_l / (beta_l + eps)^2 are kept unnormalised as
// gamma_1 e2 e3 : gamma_2 e1 e3 : gamma_3 e1 e2 (e_l = (beta_l + eps)^2, scaled by 10/3). Returns N;
// w receives the weights and their sum su.
template <class T>
__device__ __forceinline__ T hweno_side(T f0, T f1, T f2, T s0, T s1, T s2, T eps, W3<T>& w) {
  const T d01 = f0 - f1, d12 = f1 - f2, dd = d01 - d12;
  const T r1 = fma(T(1.0 / 3.0), fma(T(5.0), s1, s0), d01);
  const T r2 = fma(T(1.0 / 3.0), s1 - s2, -d12);
  const T r3 = fma(T(1.0 / 6.0), dd, s1);
  const T te = fma(s1, s1, eps);
  const T ma = T(3.0 * RA) * s1, rc = T(RC) * s1;
  const T a1 = fma(T(3.0 * RA), r1, -ma);                   // RA (3 d01 + s0 + 2 s1)
  const T c1 = fma(T(2.0 * RC), d01, fma(T(RC), s0, rc));  // RC (2 d01 + s0 + s1)
  const T a2 = fma(T(-3.0 * RA), r2, ma);                   // RA (3 d12 + s2 + 2 s1)
  const T c2 = fma(T(2.0 * RC), d12, fma(T(RC), s2, rc));  // RC (2 d12 + s2 + s1)
  const T a3 = T(RB) * dd;                                  // RB (f0 - 2 f1 + f2)
  const T c3 = fma(T(RD), d01 + d12, T(2.0 * RD) * s1);     // RD (f0 - f2 + 2 s1)
  const T g1 = fma(a1, a1, fma(c1, c1, te));
  const T g2 = fma(a2, a2, fma(c2, c2, te));
  const T g3 = fma(a3, a3, fma(c3, c3, te));
  const T e1 = g1 * g1, e2 = g2 * g2, e3 = g3 * g3;
  w.u1 = e2 * e3;
  w.u2 = e1 * e3;
  w.u3 = T(4.0 / 3.0) * (e1 * e2);
  w.su = (w.u1 + w.u2) + w.u3;
  return fma(w.u3, r3, fma(w.u2, r2, w.u1 * r1));
}

// The deviations of the three candidates combined with given weights (the source split of
// Step 2): returns N for the value f1 + N / (2 su).
template <class T>
__device__ __forceinline__ T hweno_with(T f0, T f1, T f2, T s0, T s1, T s2, const W3<T>& w) {
  const T d01 = f0 - f1, d12 = f1 - f2;
  const T r1 = fma(T(1.0 / 3.0), fma(T(5.0), s1, s0), d01);
  const T r2 = fma(T(1.0 / 3.0), s1 - s2, -d12);
  const T r3 = fma(T(1.0 / 6.0), d01 - d12, s1);
  return fma(w.u3, r3, fma(w.u2, r2, w.u1 * r1));
}

// Sum of the two sides' values at one interface, (fa + Na / (2 sa)) + (fb + Nb / (2 sb)). In
// double precision both share one reciprocal of 2 sa sb (the sums lie between 3 eps^4 and about
// 1e150 for any physical state, so the product stays normal); in single precision, where the
// product of two sums near 3 eps^4 would underflow, each side has its own.
template <class T>
struct Pair {
  T q, sa, sb;  // q = 1 / (2 sa sb) (double) or the pair (1 / (2 sa), 1 / (2 sb)) (float)
  __device__ __forceinline__ Pair(T sa_, T sb_) : sa(sa_), sb(sb_) {
    if constexpr (sizeof(T) == 8) {
      const T p = sa * sb;
      q = rcp(p + p);
    } else {
      q = rcp(sa + sa);
      sb = rcp(sb + sb);
    }
  }
  __device__ __forceinline__ T sum(T fa, T na, T fb, T nb) const {
    if constexpr (sizeof(T) == 8) return fma(fma(na, sb, nb * sa), q, fa + fb);
    else return fma(na, q, fa) + fma(nb, sb, fb);
  }
};

// Interface quantities at x_{i+1/2}, frame order (eta, n, t).
template <class T>
struct IfO {
  T F0, F1, F2;  // nonlinear flux F^ = F^+ + F^-
  T B0, B1, B2;  // bottom vector reconstructed with the flux's projection and weights
  T P0, P1, P2;  // linear Hermite flux of the derivative equation along the sweep
  T PB;          // its bottom-derivative counterpart (n component)
  T M0, M1, M2;  // four-point central flux of the mixed derivative flux
  T MB;          // four-point central flux of the mixed bottom derivative (n component)
};

// Interface x_{i+1/2} of a sweep. fetch(k, X) provides the fluxes of node i-1+k (k = 0..3),
// either computed from a raw record or read from where another lane left them; nodes are
// fetched and projected one at a time so that only one node's quantities are live.
// alpha = Lax-Friedrichs speed of this direction.
template <class T, class Fetch>
__device__ __forceinline__ void interface_flux(Fetch fetch, T alpha, T dx, T eps, T g, IfO<T>& o) {
  NodeF<T> XB, XC;
  fetch(1, XB);
  fetch(2, XC);
  // characteristic matrices at the arithmetic mean of the two adjacent nodes
  const T em = T(0.5) * (XB.e + XC.e), mnm = T(0.5) * (XB.mn + XC.mn), mtm = T(0.5) * (XB.mt + XC.mt);
  const T bm = T(0.5) * (XB.b + XC.b);
  const T h = em - bm, ih = rcp(h);
  const T un = mnm * ih, ut = mtm * ih;
  const T cs = sqrt_pos(g * h), i2c = T(0.5) * rcp(cs);
  const T l1a = (un + cs) * i2c, l3a = (cs - un) * i2c;
  // rows: l1 = (l1a, -i2c, 0), l2 = (-ut, 0, 1), l3 = (l3a, i2c, 0)
  // projected, split values f^± = L (F ± alpha U) / 2, s^± = dx L (P ± alpha D) / 2, formed from
  // the split sums with the rows of L scaled by 1/2 (f) and dx/2 (s)
  const T hl1 = T(0.5) * l1a, hl3 = T(0.5) * l3a, hi2 = T(0.5) * i2c, hut = T(0.5) * ut;
  const T hdx = T(0.5) * dx;
  const T sl1 = hdx * l1a, sl3 = hdx * l3a, si2 = hdx * i2c, sut = hdx * ut;

  T fpA[3], spA[3], fpB[3], spB[3], fmB[3], smB[3], fpC[3], spC[3], fmC[3], smC[3], fmD[3], smD[3];
  T bA, bB, bC, bD, sbA, sbB, sbC, sbD;  // bottom and dx * its derivative along the sweep
  T q1s[4], q7s[4];                      // partial sums of the mixed four-point flux
#define SWE_PROJ(L1, L3, I2, UT, SG, V0, V1, V2, Y)   \
  {                                                    \
    const T p_ = I2 * (V1);                            \
    Y[0] = fma(L1, V0, -p_);                           \
    Y[1] = fma(-(UT), V0, SG * (V2));                  \
    Y[2] = fma(L3, V0, p_);                            \
  }
#define SWE_SPLIT(X, SGN, FY, SY)                                                        \
  {                                                                                      \
    const T a_ = SGN * alpha;                                                            \
    const T g0 = fma(a_, X.e, X.f0), g1 = fma(a_, X.mn, X.f1), g2 = fma(a_, X.mt, X.f2); \
    SWE_PROJ(hl1, hl3, hi2, hut, T(0.5), g0, g1, g2, FY)                                 \
    const T h0 = fma(a_, X.d0, X.p0), h1 = fma(a_, X.d1, X.p1), h2 = fma(a_, X.d2, X.p2); \
    SWE_PROJ(sl1, sl3, si2, sut, hdx, h0, h1, h2, SY)                                    \
  }
  SWE_SPLIT(XB, T(1.0), fpB, spB)
  SWE_SPLIT(XB, T(-1.0), fmB, smB)
  bB = XB.b; sbB = dx * XB.bn;
  q7s[0] = XB.q0; q7s[1] = XB.q1; q7s[2] = XB.q2; q7s[3] = XB.bt;
  SWE_SPLIT(XC, T(1.0), fpC, spC)
  SWE_SPLIT(XC, T(-1.0), fmC, smC)
  bC = XC.b; sbC = dx * XC.bn;
  q7s[0] += XC.q0; q7s[1] += XC.q1; q7s[2] += XC.q2; q7s[3] += XC.bt;
  {
    NodeF<T> X;
    fetch(0, X);
    SWE_SPLIT(X, T(1.0), fpA, spA)
    bA = X.b; sbA = dx * X.bn;
    q1s[0] = X.q0; q1s[1] = X.q1; q1s[2] = X.q2; q1s[3] = X.bt;
  }
  {
    NodeF<T> X;
    fetch(3, X);
    SWE_SPLIT(X, T(-1.0), fmD, smD)
    bD = X.b; sbD = dx * X.bn;
    q1s[0] += X.q0; q1s[1] += X.q1; q1s[2] += X.q2; q1s[3] += X.bt;
  }
#undef SWE_SPLIT
#undef SWE_PROJ

  // nonlinear reconstruction per characteristic field and side; the bottom reuses the weights
  const T i4dx = T(0.25) / dx, i12dx = T(K112) / dx;
  T s[3], t[3], Z1 = T(0.0), Z3 = T(0.0);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    W3<T> wp, wm;
    const T np = hweno_side(fpA[k], fpB[k], fpC[k], spA[k], spB[k], spC[k], eps, wp);
    const T nm = hweno_side(fmD[k], fmC[k], fmB[k], -smD[k], -smC[k], -smB[k], eps, wm);
    const Pair<T> pr(wp.su, wm.su);
    s[k] = pr.sum(fpB[k], np, fmC[k], nm);
    if (k != 1) {  // the middle characteristic row annihilates (0, b, 0)
      const T z = pr.sum(bB, hweno_with(bA, bB, bC, sbA, sbB, sbC, wp), bC,
                         hweno_with(bD, bC, bB, -sbD, -sbC, -sbB, wm));
      if (k == 0) Z1 = z; else Z3 = z;
    }
    // linear Hermite derivative Q'^+(f^+, s^+/dx) + Q'^-(f^-, s^-/dx) of this characteristic field
    t[k] = ((fpA[k] - fmD[k]) + T(8.0) * (fmC[k] - fpB[k]) + T(7.0) * (fpC[k] - fmB[k])) * i4dx +
           ((spA[k] + smD[k]) - T(2.0) * (spB[k] + smC[k]) - T(5.0) * (spC[k] + smB[k])) * i12dx;
  }
  // back to the conservative frame: R columns (1, un-c, ut), (0, 0, 1), (1, un+c, ut)
  const T umc = un - cs, upc = un + cs;
  o.F0 = s[0] + s[2];
  o.F1 = umc * s[0] + upc * s[2];
  o.F2 = ut * (s[0] + s[2]) + s[1];
  // char. projections of b~^± = (0, b/2, 0): -i2c b / 2 (row 1), +i2c b / 2 (row 3)
  const T sb1 = -T(0.5) * i2c * Z1, sb3 = T(0.5) * i2c * Z3;
  o.B0 = sb1 + sb3;
  o.B1 = umc * sb1 + upc * sb3;
  o.B2 = ut * (sb1 + sb3);
  // the linear derivative-equation flux: componentwise Q' is R (char.-wise Q') since L is fixed
  o.P0 = t[0] + t[2];
  o.P1 = umc * t[0] + upc * t[2];
  o.P2 = ut * (t[0] + t[2]) + t[1];
  // bottom derivative, n component: Q'^+(b/2, B/2) + Q'^-(b/2, B/2)
  o.PB = T(0.5) * (((bA - bD) + T(15.0) * (bC - bB)) * i4dx + ((sbA + sbD) - T(7.0) * (sbB + sbC)) * i12dx);
  // four-point central flux of the mixed terms (eq. (3.7))
  o.M0 = T(K112) * (T(7.0) * q7s[0] - q1s[0]);
  o.M1 = T(K112) * (T(7.0) * q7s[1] - q1s[1]);
  o.M2 = T(K112) * (T(7.0) * q7s[2] - q1s[2]);
  o.MB = T(K112) * (T(7.0) * q7s[3] - q1s[3]);
}

// HWENO limiter of one characteristic component (Sec. 2.2): mu at x_{i-1}, x_i, x_{i+1}, nu at
// x_{i-1}, x_{i+1}; linear weights (1/4, 1/4, 1/2). The limited derivative is n / s / dx with the
// weights kept unnormalised (common factor 4 / (e1 e2 e3)); the first differences of the three
// candidates are shared with their second ones (a_l = c_l + d for the two one-sided ones).
template <class T>
struct LimNS { T n, s; };
template <class T>
__device__ __forceinline__ LimNS<T> limit_char_ns(T mm, T m0, T mp, T nm, T np, T dx, T eps) {
  const T dl = m0 - mm, dr = mp - m0;
  const T c1 = fma(-nm, dx, dl), c2 = fma(-np, dx, dr), c3 = dr - dl;
  const T a1 = c1 + dl;                  // dx * p1'(x_i) = 2 (m0 - mm) - dx nm
  const T a2 = c2 + dr;                  // dx * p2'(x_i) = 2 (mp - m0) - dx np
  const T a3 = T(0.5) * (dl + dr);       // dx * p3'(x_i)
  const T g1 = fma(a1, a1, fma(T(K133) * c1, c1, eps));
  const T g2 = fma(a2, a2, fma(T(K133) * c2, c2, eps));
  const T g3 = fma(a3, a3, fma(T(K1312) * c3, c3, eps));
  const T e1 = g1 * g1, e2 = g2 * g2, e3 = g3 * g3;
  const T u1 = e2 * e3, u2 = e1 * e3, u3 = T(2.0) * (e1 * e2);
  return {fma(u3, a3, fma(u2, a2, u1 * a1)), (u1 + u2) + u3};
}
template <class T>
__device__ __forceinline__ T limit_char(T mm, T m0, T mp, T nm, T np, T dx, T idx, T eps) {
  const LimNS<T> r = limit_char_ns(mm, m0, mp, nm, np, dx, eps);
  return r.n * rcp(r.s) * idx;
}

// Limited derivative at a node in the frame of one direction: own state (e, mn, mt, b);
// neighbour surface/momenta at -1 and +1; neighbour derivatives along this direction at -1, +1.
// In double precision the three components share one reciprocal of the product of their weight
// sums (each between 4 eps^4 and about 1e100 for any physical state, so the product stays
// normal for eps >= 1e-20); in single precision each has its own.
template <class T>
__device__ __forceinline__ void limit_frame(T e0, T mn0, T mt0, T b0, T em, T mnm,
                                            T mtm, T ep, T mnp, T mtp, T dm0, T dm1,
                                            T dm2, T dp0, T dp1, T dp2, T dx, T idx,
                                            T eps, T g, T out[3]) {
  const T h = e0 - b0, ih = rcp(h);
  const T un = mn0 * ih, ut = mt0 * ih;
  const T cs = sqrt_pos(g * h), i2c = T(0.5) * rcp(cs);
  const T l1a = (un + cs) * i2c, l3a = (cs - un) * i2c;
  const LimNS<T> c1 = limit_char_ns(l1a * em - i2c * mnm, l1a * e0 - i2c * mn0, l1a * ep - i2c * mnp,
                                    l1a * dm0 - i2c * dm1, l1a * dp0 - i2c * dp1, dx, eps);
  const LimNS<T> c2 = limit_char_ns(mtm - ut * em, mt0 - ut * e0, mtp - ut * ep, dm2 - ut * dm0, dp2 - ut * dp0, dx, eps);
  const LimNS<T> c3 = limit_char_ns(l3a * em + i2c * mnm, l3a * e0 + i2c * mn0, l3a * ep + i2c * mnp,
                                    l3a * dm0 + i2c * dm1, l3a * dp0 + i2c * dp1, dx, eps);
  T v1, v2, v3;
  if constexpr (sizeof(T) == 8) {
    const T s13 = c1.s * c3.s;
    const T r = rcp(s13 * c2.s) * idx;
    v1 = (c1.n * (c2.s * c3.s)) * r;
    v2 = (c2.n * s13) * r;
    v3 = (c3.n * (c1.s * c2.s)) * r;
  } else {
    v1 = c1.n * rcp(c1.s) * idx;
    v2 = c2.n * rcp(c2.s) * idx;
    v3 = c3.n * rcp(c3.s) * idx;
  }
  out[0] = v1 + v3;
  out[1] = (un - cs) * v1 + (un + cs) * v3;
  out[2] = ut * (v1 + v3) + v2;
}

}  // namespace swe
