// Reverse mode (vector-Jacobian products) of the device arithmetic in hweno_device.hpp, FP64.
//
// Every routine here recomputes the forward quantities it needs from the same inputs as its
// forward counterpart and then runs the chain rule backwards through the same formulas: the
// Lax-Friedrichs split, characteristic projection at the interface mean state, the nonlinear
// HWENO weights and candidates (Sec. 2.1), the source split that reuses the weights (Step 2),
// the linear Hermite derivative fluxes (eq. (2.6)), the four-point mixed terms (eq. (3.7)), the
// node fluxes and their total derivatives (eqs. (3.3), (3.5)) and the limiter (Sec. 2.2). The
// Lax-Friedrichs speed alpha is a constant here (the adjoint is taken with alpha frozen).
#pragma once
#include "hweno_device.hpp"

namespace swe {

// Adjoints of the fields of a NodeF (same names).
struct NodeB {
  double e, mn, mt;
  double d0, d1, d2;
  double f0, f1, f2;
  double p0, p1, p2;
  double q0, q1, q2;
  double b, bn, bt;
};

__device__ __forceinline__ void nodeb_zero(NodeB& x) {
  x.e = x.mn = x.mt = x.d0 = x.d1 = x.d2 = x.f0 = x.f1 = x.f2 = 0.0;
  x.p0 = x.p1 = x.p2 = x.q0 = x.q1 = x.q2 = x.b = x.bn = x.bt = 0.0;
}

// Reverse of hweno_side: v = sum_l w_l q_l with the weights of the smoothness indicators.
// vb = adjoint of v; wb = extra adjoints of the three weights (from the bottom reconstruction
// that reuses them). Adds the adjoints of f0..f2, s0..s2.
__device__ __forceinline__ void hweno_side_vjp(double f0, double f1, double f2, double s0, double s1, double s2,
                                               double eps, double vb, const double wb_extra[3], double& f0b,
                                               double& f1b, double& f2b, double& s0b, double& s1b, double& s2b) {
  // forward
  const double d01 = f0 - f1, d12 = f1 - f2;
  const double a1 = 3.0 * d01 + s0 + 2.0 * s1, c1 = 2.0 * d01 + s0 + s1;
  const double a2 = 3.0 * d12 + s2 + 2.0 * s1, c2 = 2.0 * d12 + s2 + s1;
  const double a3 = (f0 + f2) - 2.0 * f1, c3 = (f0 - f2) + 2.0 * s1;
  const double t = s1 * s1;
  const double be1 = t + K133 * (a1 * a1) + K78120 * (c1 * c1);
  const double be2 = t + K133 * (a2 * a2) + K78120 * (c2 * c2);
  const double be3 = t + K1312 * (a3 * a3) + K78180 * (c3 * c3);
  const double g1 = be1 + eps, g2 = be2 + eps, g3 = be3 + eps;
  const double e1 = g1 * g1, e2 = g2 * g2, e3 = g3 * g3;
  const double u1 = 0.3 * (e2 * e3), u2 = 0.3 * (e1 * e3), u3 = 0.4 * (e1 * e2);
  const double is = rcp((u1 + u2) + u3);
  const double w1 = u1 * is, w2 = u2 * is, w3 = u3 * is;
  const double q1 = 0.5 * (f0 + f1) + K16 * (s0 + 5.0 * s1);
  const double q2 = 0.5 * (f1 + f2) + K16 * (s1 - s2);
  const double q3 = K112 * ((f0 + f2) + 10.0 * f1) + 0.5 * s1;
  // v = w . q
  const double q1b = w1 * vb, q2b = w2 * vb, q3b = w3 * vb;
  const double w1b = q1 * vb + wb_extra[0], w2b = q2 * vb + wb_extra[1], w3b = q3 * vb + wb_extra[2];
  // w_l = u_l / U
  const double dotw = w1b * w1 + w2b * w2 + w3b * w3;
  const double u1b = (w1b - dotw) * is, u2b = (w2b - dotw) * is, u3b = (w3b - dotw) * is;
  const double e1b = 0.3 * e3 * u2b + 0.4 * e2 * u3b;
  const double e2b = 0.3 * e3 * u1b + 0.4 * e1 * u3b;
  const double e3b = 0.3 * e2 * u1b + 0.3 * e1 * u2b;
  const double be1b = 2.0 * g1 * e1b, be2b = 2.0 * g2 * e2b, be3b = 2.0 * g3 * e3b;
  const double tb = be1b + be2b + be3b;
  const double a1b = 2.0 * K133 * a1 * be1b, c1b = 2.0 * K78120 * c1 * be1b;
  const double a2b = 2.0 * K133 * a2 * be2b, c2b = 2.0 * K78120 * c2 * be2b;
  const double a3b = 2.0 * K1312 * a3 * be3b, c3b = 2.0 * K78180 * c3 * be3b;
  const double d01b = 3.0 * a1b + 2.0 * c1b, d12b = 3.0 * a2b + 2.0 * c2b;
  f0b += a3b + c3b + d01b + 0.5 * q1b + K112 * q3b;
  f1b += -2.0 * a3b - d01b + d12b + 0.5 * q1b + 0.5 * q2b + 10.0 * K112 * q3b;
  f2b += a3b - c3b - d12b + 0.5 * q2b + K112 * q3b;
  s0b += a1b + c1b + K16 * q1b;
  s1b += 2.0 * s1 * tb + 2.0 * a1b + c1b + 2.0 * a2b + c2b + 2.0 * c3b + 5.0 * K16 * q1b + K16 * q2b + 0.5 * q3b;
  s2b += a2b + c2b - K16 * q2b;
}

// Forward HWENO value of one side with its normalised weights w (the formulas of Sec. 2.1 as
// the reverse below differentiates them).
__device__ __forceinline__ double side_value(double f0, double f1, double f2, double s0, double s1, double s2,
                                             double eps, double w[3]) {
  const double d01 = f0 - f1, d12 = f1 - f2;
  const double a1 = 3.0 * d01 + s0 + 2.0 * s1, c1 = 2.0 * d01 + s0 + s1;
  const double a2 = 3.0 * d12 + s2 + 2.0 * s1, c2 = 2.0 * d12 + s2 + s1;
  const double a3 = (f0 + f2) - 2.0 * f1, c3 = (f0 - f2) + 2.0 * s1;
  const double t = s1 * s1;
  const double g1 = t + K133 * (a1 * a1) + K78120 * (c1 * c1) + eps;
  const double g2 = t + K133 * (a2 * a2) + K78120 * (c2 * c2) + eps;
  const double g3 = t + K1312 * (a3 * a3) + K78180 * (c3 * c3) + eps;
  const double e1 = g1 * g1, e2 = g2 * g2, e3 = g3 * g3;
  const double u1 = 0.3 * (e2 * e3), u2 = 0.3 * (e1 * e3), u3 = 0.4 * (e1 * e2);
  const double is = rcp((u1 + u2) + u3);
  w[0] = u1 * is; w[1] = u2 * is; w[2] = u3 * is;
  const double q1 = 0.5 * (f0 + f1) + K16 * (s0 + 5.0 * s1);
  const double q2 = 0.5 * (f1 + f2) + K16 * (s1 - s2);
  const double q3 = K112 * ((f0 + f2) + 10.0 * f1) + 0.5 * s1;
  return w[0] * q1 + w[1] * q2 + w[2] * q3;
}

// Candidates combined with given normalised weights (the source split of Step 2).
__device__ __forceinline__ double with_value(double f0, double f1, double f2, double s0, double s1, double s2,
                                             const double w[3]) {
  const double q1 = 0.5 * (f0 + f1) + K16 * (s0 + 5.0 * s1);
  const double q2 = 0.5 * (f1 + f2) + K16 * (s1 - s2);
  const double q3 = K112 * ((f0 + f2) + 10.0 * f1) + 0.5 * s1;
  return w[0] * q1 + w[1] * q2 + w[2] * q3;
}

// Reverse of hweno_with: z = sum_l w_l q_l(f, s) with given weights. Adds the adjoints of the
// values, derivatives and weights.
__device__ __forceinline__ void hweno_with_vjp(double f0, double f1, double f2, double s0, double s1, double s2,
                                               const double w[3], double zb, double& f0b, double& f1b, double& f2b,
                                               double& s0b, double& s1b, double& s2b, double wb[3]) {
  const double q1 = 0.5 * (f0 + f1) + K16 * (s0 + 5.0 * s1);
  const double q2 = 0.5 * (f1 + f2) + K16 * (s1 - s2);
  const double q3 = K112 * ((f0 + f2) + 10.0 * f1) + 0.5 * s1;
  wb[0] += q1 * zb; wb[1] += q2 * zb; wb[2] += q3 * zb;
  const double q1b = w[0] * zb, q2b = w[1] * zb, q3b = w[2] * zb;
  f0b += 0.5 * q1b + K112 * q3b;
  f1b += 0.5 * q1b + 0.5 * q2b + 10.0 * K112 * q3b;
  f2b += 0.5 * q2b + K112 * q3b;
  s0b += K16 * q1b;
  s1b += 5.0 * K16 * q1b + K16 * q2b + 0.5 * q3b;
  s2b -= K16 * q2b;
}

// Reverse of one projected triple: y = (l1a v0 - i2c v1, v2 - ut v0, l3a v0 + i2c v1).
__device__ __forceinline__ void proj_vjp(double l1a, double l3a, double i2c, double ut, double v0, double v1,
                                         const double yb[3], double& v0b, double& v1b, double& v2b, double& l1ab,
                                         double& l3ab, double& i2cb, double& utb) {
  v0b += l1a * yb[0] - ut * yb[1] + l3a * yb[2];
  v1b += i2c * (yb[2] - yb[0]);
  v2b += yb[1];
  l1ab += v0 * yb[0];
  l3ab += v0 * yb[2];
  i2cb += v1 * (yb[2] - yb[0]);
  utb -= v0 * yb[1];
}

// Row f of the characteristic matrix L applied to a triple: rows (l1a, -i2c, 0), (-ut, 0, 1),
// (l3a, i2c, 0); proj_vjp is its reverse over the three rows.
__device__ __forceinline__ double proj_row(int f, double l1a, double l3a, double i2c, double ut, double v0, double v1,
                                           double v2) {
  return f == 0 ? l1a * v0 - i2c * v1 : (f == 1 ? v2 - ut * v0 : l3a * v0 + i2c * v1);
}

// Reverse of node_frame<DIR>: adds the adjoint of the raw record r (slots of hweno_device.hpp)
// given the adjoints of the NodeF fields.
template <int DIR>
__device__ __forceinline__ void node_frame_vjp(const double* __restrict__ r, double g, const NodeB& X,
                                               double rb[NREC]) {
  const int sMN = DIR == 0 ? S_M : S_W, sMT = DIR == 0 ? S_W : S_M;
  const int sDN0 = DIR == 0 ? S_H1 : S_H2, sDN1 = DIR == 0 ? S_M1 : S_W2, sDN2 = DIR == 0 ? S_W1 : S_M2;
  const int sDT0 = DIR == 0 ? S_H2 : S_H1, sDT1 = DIR == 0 ? S_M2 : S_W1, sDT2 = DIR == 0 ? S_W2 : S_M1;
  const int sBN = DIR == 0 ? S_BX : S_BY, sBT = DIR == 0 ? S_BY : S_BX;
  const double e = r[S_ETA], b = r[S_B], mn = r[sMN], mt = r[sMT];
  const double dn0 = r[sDN0], dn1 = r[sDN1], dn2 = r[sDN2];
  const double dt0 = r[sDT0], dt1 = r[sDT1], dt2 = r[sDT2];
  const double bn = r[sBN], bt = r[sBT];
  const double h = e - b, ih = rcp(h);
  const double un = mn * ih, ut = mt * ih;
  const double j10 = g * h - un * un, j11 = 2.0 * un, j20 = -(un * ut);
  const double jb1 = un * un - g * e, jb2 = un * ut;
  // pass-through fields
  double eb = X.e, mnb = X.mn, mtb = X.mt, bb = X.b, bnb = X.bn, btb = X.bt;
  double dn0b = X.d0, dn1b = X.d1, dn2b = X.d2, dt0b = 0.0, dt1b = 0.0, dt2b = 0.0;
  double unb = 0.0, utb = 0.0, hb = 0.0;
  // f = (mn, mn un + g e (e/2 - b), mn ut)
  mnb += X.f0 + un * X.f1 + ut * X.f2;
  unb += mn * X.f1;
  utb += mn * X.f2;
  eb += g * h * X.f1;
  bb -= g * e * X.f1;
  // p = (dn1, j10 dn0 + j11 dn1 + jb1 bn, j20 dn0 + ut dn1 + un dn2 + jb2 bn), q likewise with dt, bt
  dn1b += X.p0 + j11 * X.p1 + ut * X.p2;
  dn0b += j10 * X.p1 + j20 * X.p2;
  dn2b += un * X.p2;
  bnb += jb1 * X.p1 + jb2 * X.p2;
  dt1b += X.q0 + j11 * X.q1 + ut * X.q2;
  dt0b += j10 * X.q1 + j20 * X.q2;
  dt2b += un * X.q2;
  btb += jb1 * X.q1 + jb2 * X.q2;
  const double j10b = dn0 * X.p1 + dt0 * X.q1;
  const double j11b = dn1 * X.p1 + dt1 * X.q1;
  const double jb1b = bn * X.p1 + bt * X.q1;
  const double j20b = dn0 * X.p2 + dt0 * X.q2;
  const double jb2b = bn * X.p2 + bt * X.q2;
  utb += dn1 * X.p2 + dt1 * X.q2;
  unb += dn2 * X.p2 + dt2 * X.q2;
  hb += g * j10b;
  unb += -2.0 * un * j10b + 2.0 * j11b - ut * j20b + 2.0 * un * jb1b + ut * jb2b;
  utb += -un * j20b + un * jb2b;
  eb -= g * jb1b;
  mnb += ih * unb;
  mtb += ih * utb;
  const double ihb = mn * unb + mt * utb;
  hb -= ih * ih * ihb;
  eb += hb;
  bb -= hb;
  rb[S_ETA] += eb; rb[sMN] += mnb; rb[sMT] += mtb;
  rb[sDN0] += dn0b; rb[sDN1] += dn1b; rb[sDN2] += dn2b;
  rb[sDT0] += dt0b; rb[sDT1] += dt1b; rb[sDT2] += dt2b;
  rb[S_B] += bb; rb[sBN] += bnb; rb[sBT] += btb;
}

// Reverse of limit_char: adds the adjoints of mm, m0, mp, nm, np given that of the result.
__device__ __forceinline__ void limit_char_vjp(double mm, double m0, double mp, double nm, double np, double dx,
                                               double idx, double eps, double ob, double& mmb, double& m0b,
                                               double& mpb, double& nmb, double& npb) {
  const double a1 = 2.0 * (m0 - mm) - nm * dx;
  const double a2 = 2.0 * (mp - m0) - np * dx;
  const double a3 = 0.5 * (mp - mm);
  const double c1 = (m0 - mm) - nm * dx, c2 = (mp - m0) - np * dx, c3 = (mm + mp) - 2.0 * m0;
  const double be1 = a1 * a1 + K133 * (c1 * c1);
  const double be2 = a2 * a2 + K133 * (c2 * c2);
  const double be3 = a3 * a3 + K1312 * (c3 * c3);
  const double g1 = be1 + eps, g2 = be2 + eps, g3 = be3 + eps;
  const double e1 = g1 * g1, e2 = g2 * g2, e3 = g3 * g3;
  const double u1 = 0.25 * (e2 * e3), u2 = 0.25 * (e1 * e3), u3 = 0.5 * (e1 * e2);
  const double is = rcp((u1 + u2) + u3);
  const double w1 = u1 * is, w2 = u2 * is, w3 = u3 * is;
  const double Ab = ob * idx;
  double a1b = w1 * Ab, a2b = w2 * Ab, a3b = w3 * Ab;
  const double w1b = a1 * Ab, w2b = a2 * Ab, w3b = a3 * Ab;
  const double dotw = w1b * w1 + w2b * w2 + w3b * w3;
  const double u1b = (w1b - dotw) * is, u2b = (w2b - dotw) * is, u3b = (w3b - dotw) * is;
  const double e1b = 0.25 * e3 * u2b + 0.5 * e2 * u3b;
  const double e2b = 0.25 * e3 * u1b + 0.5 * e1 * u3b;
  const double e3b = 0.25 * e2 * u1b + 0.25 * e1 * u2b;
  const double be1b = 2.0 * g1 * e1b, be2b = 2.0 * g2 * e2b, be3b = 2.0 * g3 * e3b;
  a1b += 2.0 * a1 * be1b;
  a2b += 2.0 * a2 * be2b;
  a3b += 2.0 * a3 * be3b;
  const double c1b = 2.0 * K133 * c1 * be1b, c2b = 2.0 * K133 * c2 * be2b, c3b = 2.0 * K1312 * c3 * be3b;
  m0b += 2.0 * a1b - 2.0 * a2b + c1b - c2b - 2.0 * c3b;
  mmb += -2.0 * a1b - 0.5 * a3b - c1b + c3b;
  mpb += 2.0 * a2b + 0.5 * a3b + c2b + c3b;
  nmb -= dx * (a1b + c1b);
  npb -= dx * (a2b + c2b);
}

// Reverse of limit_frame (same argument order): ob = adjoints of out[0..3]; the adjoints of
// the inputs are added to the arrays: own (e0, mn0, mt0, b0), minus neighbour
// (em, mnm, mtm, dm0, dm1, dm2), plus neighbour (ep, mnp, mtp, dp0, dp1, dp2).
__device__ __forceinline__ void limit_frame_vjp(double e0, double mn0, double mt0, double b0, double em, double mnm,
                                                double mtm, double ep, double mnp, double mtp, double dm0,
                                                double dm1, double dm2, double dp0, double dp1, double dp2, double dx,
                                                double idx, double eps, double g, const double ob[3], double own[4],
                                                double mb[6], double pb[6]) {
  const double h = e0 - b0, ih = rcp(h);
  const double un = mn0 * ih, ut = mt0 * ih;
  const double cs = sqrt(g * h), i2c = 0.5 * rcp(cs);
  const double l1a = (un + cs) * i2c, l3a = (cs - un) * i2c;
  // the three characteristic inputs (mm, m0, mp, nm, np) of each limited component
  const double x1[5] = {l1a * em - i2c * mnm, l1a * e0 - i2c * mn0, l1a * ep - i2c * mnp, l1a * dm0 - i2c * dm1,
                        l1a * dp0 - i2c * dp1};
  const double x2[5] = {mtm - ut * em, mt0 - ut * e0, mtp - ut * ep, dm2 - ut * dm0, dp2 - ut * dp0};
  const double x3[5] = {l3a * em + i2c * mnm, l3a * e0 + i2c * mn0, l3a * ep + i2c * mnp, l3a * dm0 + i2c * dm1,
                        l3a * dp0 + i2c * dp1};
  const double v1 = limit_char(x1[0], x1[1], x1[2], x1[3], x1[4], dx, idx, eps);
  const double v3 = limit_char(x3[0], x3[1], x3[2], x3[3], x3[4], dx, idx, eps);
  // out = (v1 + v3, (un - cs) v1 + (un + cs) v3, ut (v1 + v3) + v2)
  const double v1b = ob[0] + (un - cs) * ob[1] + ut * ob[2];
  const double v3b = ob[0] + (un + cs) * ob[1] + ut * ob[2];
  const double v2b = ob[2];
  double unb = (v1 + v3) * ob[1], csb = (v3 - v1) * ob[1], utb = (v1 + v3) * ob[2];
  double x1b[5] = {0, 0, 0, 0, 0}, x2b[5] = {0, 0, 0, 0, 0}, x3b[5] = {0, 0, 0, 0, 0};
  limit_char_vjp(x1[0], x1[1], x1[2], x1[3], x1[4], dx, idx, eps, v1b, x1b[0], x1b[1], x1b[2], x1b[3], x1b[4]);
  limit_char_vjp(x2[0], x2[1], x2[2], x2[3], x2[4], dx, idx, eps, v2b, x2b[0], x2b[1], x2b[2], x2b[3], x2b[4]);
  limit_char_vjp(x3[0], x3[1], x3[2], x3[3], x3[4], dx, idx, eps, v3b, x3b[0], x3b[1], x3b[2], x3b[3], x3b[4]);
  // x1 = l1a a - i2c c, x2 = t - ut a, x3 = l3a a + i2c c for (a, c, t) = (e, mn, mt) or (d0, d1, d2)
  const double av[5] = {em, e0, ep, dm0, dp0};
  const double cv[5] = {mnm, mn0, mnp, dm1, dp1};
  double ab[5], cb[5], tb[5];
  double l1ab = 0.0, l3ab = 0.0, i2cb = 0.0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    ab[k] = l1a * x1b[k] - ut * x2b[k] + l3a * x3b[k];
    cb[k] = i2c * (x3b[k] - x1b[k]);
    tb[k] = x2b[k];
    l1ab += av[k] * x1b[k];
    l3ab += av[k] * x3b[k];
    i2cb += cv[k] * (x3b[k] - x1b[k]);
    utb -= av[k] * x2b[k];
  }
  unb += i2c * (l1ab - l3ab);
  csb += i2c * (l1ab + l3ab);
  i2cb += (un + cs) * l1ab + (cs - un) * l3ab;
  csb += -2.0 * i2c * i2c * i2cb;
  double hb = g * i2c * csb;
  const double ihb = mn0 * unb + mt0 * utb;
  hb -= ih * ih * ihb;
  own[0] += ab[1] + hb;          // e0
  own[1] += cb[1] + ih * unb;    // mn0
  own[2] += tb[1] + ih * utb;    // mt0
  own[3] -= hb;                  // b0
  mb[0] += ab[0]; mb[1] += cb[0]; mb[2] += tb[0]; mb[3] += ab[3]; mb[4] += cb[3]; mb[5] += tb[3];
  pb[0] += ab[2]; pb[1] += cb[2]; pb[2] += tb[2]; pb[3] += ab[4]; pb[4] += cb[4]; pb[5] += tb[4];
}

}  // namespace swe
