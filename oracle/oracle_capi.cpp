// TEST INFRASTRUCTURE — C entry points of the CPU oracle (liboracle.so). Only the test suite, the
// smoke check and the CPU-baseline leg of the benchmark may load this library.
//
// Arrays are host double arrays, planes [field][ny][nx] with x fastest:
//   1D state: eta, m, H, M            (4 planes of nx)
//   2D state: eta, m, w, H1, M1, W1, H2, M2, W2   (9 planes of nx*ny)
// b, bx (= b_x) and by (= b_y, 2D only) are single planes. Return codes: 0 ok, -1 invalid
// argument, -4 dry node (h <= 0), -5 non-finite value.
#include <cmath>
#include <cstring>
#include <vector>

#include "scheme.hpp"

using namespace orc;

extern "C" {

typedef struct {
  int dim, nx, ny;
  double x0, x1, y0, y1;
  double g, cfl, eps;
  int bc_x, bc_y, flags;
  double fixed_dt;
  double alpha_x[3], alpha_y[3];
} orc_params;

}  // extern "C"

namespace {

bool valid(const orc_params* p) {
  if (!p) return false;
  if (p->dim != 1 && p->dim != 2) return false;
  if (p->nx < 4) return false;
  if (p->dim == 2 && p->ny < 4) return false;
  if (p->dim == 1 && p->ny != 1) return false;
  if (!(p->x1 > p->x0)) return false;
  if (p->dim == 2 && !(p->y1 > p->y0)) return false;
  if (!(p->g > 0) || !(p->eps > 0) || !(p->cfl > 0)) return false;
  if (p->bc_x < 0 || p->bc_x > 1 || p->bc_y < 0 || p->bc_y > 1) return false;
  return true;
}

template <class T> Params<T> convert(const orc_params* p) {
  Params<T> q;
  q.dim = p->dim; q.nx = p->nx; q.ny = p->dim == 2 ? p->ny : 1;
  q.dx = (T(p->x1) - T(p->x0)) / T(p->nx);
  q.dy = p->dim == 2 ? (T(p->y1) - T(p->y0)) / T(p->ny) : T(1);
  q.g = T(p->g); q.cfl = T(p->cfl); q.eps = T(p->eps);
  q.bcx = p->bc_x; q.bcy = p->bc_y; q.flags = p->flags;
  q.fixed_dt = T(p->fixed_dt);
  for (int k = 0; k < 3; ++k) { q.ax_fixed[k] = T(p->alpha_x[k]); q.ay_fixed[k] = T(p->alpha_y[k]); }
  return q;
}

size_t nodes(const orc_params* p) { return (size_t)p->nx * (size_t)(p->dim == 2 ? p->ny : 1); }
int nfields(const orc_params* p) { return p->dim == 2 ? 9 : 4; }

template <class T> std::vector<T> to_t(const double* x, size_t n) {
  std::vector<T> v(n);
  for (size_t i = 0; i < n; ++i) v[i] = T(x[i]);
  return v;
}

template <class T> int make(const orc_params* p, const double* b, const double* bx, const double* by, Scheme<T>& s) {
  if (!valid(p) || !b || !bx || (p->dim == 2 && !by)) return E_INVAL;
  const size_t n = nodes(p);
  std::vector<T> bb = to_t<T>(b, n), bbx = to_t<T>(bx, n), bby = p->dim == 2 ? to_t<T>(by, n) : std::vector<T>(n, T(0));
  s.setup(convert<T>(p), bb.data(), bbx.data(), bby.data());
  return OK;
}

// Run in precision T and return (final - initial) state computed in T (so that a quadruple
// round-off difference survives the conversion to double).
template <class T>
int run_delta(const orc_params* p, const double* state, const double* b, const double* bx, const double* by,
              int nsteps, double t_end, double* delta, double* t_out, int* steps_out) {
  Scheme<T> s;
  int e = make(p, b, bx, by, s);
  if (e) return e;
  const size_t N = (size_t)nfields(p) * nodes(p);
  std::vector<T> S0 = to_t<T>(state, N), S = S0;
  e = s.run(S.data(), nsteps, t_end, t_out, steps_out);
  for (size_t q = 0; q < N; ++q) delta[q] = to_double(S[q] - S0[q]);
  return e;
}

}  // namespace

extern "C" {

void orc_set_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : 1);
#else
  (void)n;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int orc_alpha(const orc_params* p, const double* state, const double* b, const double* bx, const double* by,
              double* ax, double* ay) {
  Scheme<double> s;
  int e = make(p, b, bx, by, s);
  if (e) return e;
  double a = 0, c = 0;
  s.alpha(state, a, c);
  *ax = a; *ay = c;
  return s.err;
}

// Right-hand side of the semi-discrete scheme; alpha_x < 0 means "compute from the state".
int orc_rhs(const orc_params* p, const double* state, const double* b, const double* bx, const double* by,
            double alpha_x, double alpha_y, double* rhs) {
  Scheme<double> s;
  int e = make(p, b, bx, by, s);
  if (e) return e;
  const size_t n = nodes(p);
  if (alpha_x < 0) {
    s.alpha(state, alpha_x, alpha_y);
    if (s.err) return s.err;
  }
  s.rhs(state, state + (size_t)s.nu * n, alpha_x, alpha_y, rhs, rhs + (size_t)s.nu * n);
  return OK;
}

// The limited derivatives Lim(S): 2 planes (1D) or 6 planes (2D).
int orc_limit(const orc_params* p, const double* state, const double* b, const double* bx, const double* by,
              double* dmod) {
  Scheme<double> s;
  int e = make(p, b, bx, by, s);
  if (e) return e;
  s.limit(state, state + (size_t)s.nu * nodes(p), dmod);
  return OK;
}

int orc_step(const orc_params* p, double* state, const double* b, const double* bx, const double* by,
             double dt, double* dt_used) {
  Scheme<double> s;
  int e = make(p, b, bx, by, s);
  if (e) return e;
  if ((p->flags & FL_FIXED_DT) && !(dt > 0)) dt = p->fixed_dt;
  const double used = s.step(state, dt);
  if (dt_used) *dt_used = used;
  return s.err;
}

int orc_run(const orc_params* p, double* state, const double* b, const double* bx, const double* by,
            int nsteps, double t_end, double* t_out, int* steps_out) {
  Scheme<double> s;
  int e = make(p, b, bx, by, s);
  if (e) return e;
  return s.run(state, nsteps, t_end, t_out, steps_out);
}

// The scheme run in single precision (Scheme<float>), inputs rounded to float, results widened
// to double: the right-hand side (alpha_x < 0: alpha from the rounded state, in float) and a
// run of the state in place.
int orc_rhs_f32(const orc_params* p, const double* state, const double* b, const double* bx, const double* by,
                double alpha_x, double alpha_y, double* rhs) {
  Scheme<float> s;
  int e = make(p, b, bx, by, s);
  if (e) return e;
  const size_t n = nodes(p), N = (size_t)nfields(p) * n;
  std::vector<float> S = to_t<float>(state, N), R(N);
  float ax = float(alpha_x), ay = float(alpha_y);
  if (alpha_x < 0) {
    s.alpha(S.data(), ax, ay);
    if (s.err) return s.err;
  }
  s.rhs(S.data(), S.data() + (size_t)s.nu * n, ax, ay, R.data(), R.data() + (size_t)s.nu * n);
  for (size_t q = 0; q < N; ++q) rhs[q] = double(R[q]);
  return OK;
}

int orc_run_f32(const orc_params* p, double* state, const double* b, const double* bx, const double* by,
                int nsteps, double t_end, double* t_out, int* steps_out) {
  Scheme<float> s;
  int e = make(p, b, bx, by, s);
  if (e) return e;
  const size_t N = (size_t)nfields(p) * nodes(p);
  std::vector<float> S = to_t<float>(state, N);
  e = s.run(S.data(), nsteps, t_end, t_out, steps_out);
  for (size_t q = 0; q < N; ++q) state[q] = double(S[q]);
  return e;
}

int orc_run_delta_f32(const orc_params* p, const double* state, const double* b, const double* bx, const double* by,
                      int nsteps, double t_end, double* delta, double* t_out, int* steps_out) {
  return run_delta<float>(p, state, b, bx, by, nsteps, t_end, delta, t_out, steps_out);
}
int orc_run_delta_f64(const orc_params* p, const double* state, const double* b, const double* bx, const double* by,
                      int nsteps, double t_end, double* delta, double* t_out, int* steps_out) {
  return run_delta<double>(p, state, b, bx, by, nsteps, t_end, delta, t_out, steps_out);
}
int orc_run_delta_f128(const orc_params* p, const double* state, const double* b, const double* bx, const double* by,
                       int nsteps, double t_end, double* delta, double* t_out, int* steps_out) {
  return run_delta<__float128>(p, state, b, bx, by, nsteps, t_end, delta, t_out, steps_out);
}

// Forward-mode tangents (Dual<double>) of the limiter and of a run: the value and the
// directional derivative along (dstate, db, dbx, dby). A run is differentiable when alpha and
// dt are fixed (flags FIXED_ALPHA | FIXED_DT); otherwise the max in alpha is differentiated
// along its active branch.
int orc_limit_jvp(const orc_params* p, const double* state, const double* dstate, const double* b, const double* bx,
                  const double* by, const double* db, const double* dbx, const double* dby, double* dmod,
                  double* ddmod) {
  if (!valid(p) || !state || !dstate || !b || !bx || !db || !dbx) return E_INVAL;
  if (p->dim == 2 && (!by || !dby)) return E_INVAL;
  using D = Dual<double>;
  const size_t n = nodes(p), N = (size_t)nfields(p) * n;
  std::vector<D> bb(n), bbx(n), bby(n), S(N);
  for (size_t q = 0; q < n; ++q) {
    bb[q] = D(b[q], db[q]); bbx[q] = D(bx[q], dbx[q]);
    bby[q] = p->dim == 2 ? D(by[q], dby[q]) : D(0.0, 0.0);
  }
  for (size_t q = 0; q < N; ++q) S[q] = D(state[q], dstate[q]);
  Scheme<D> s;
  s.setup(convert<D>(p), bb.data(), bbx.data(), bby.data());
  const size_t ND = (size_t)s.nd * n;
  std::vector<D> M(ND);
  s.limit(S.data(), S.data() + (size_t)s.nu * n, M.data());
  for (size_t q = 0; q < ND; ++q) { dmod[q] = M[q].v; ddmod[q] = M[q].d; }
  return OK;
}

int orc_run_jvp(const orc_params* p, const double* state, const double* dstate, const double* b, const double* bx,
                const double* by, const double* db, const double* dbx, const double* dby, int nsteps,
                double* out, double* dout) {
  if (!valid(p) || !state || !dstate || !b || !bx || !db || !dbx || nsteps < 1) return E_INVAL;
  if (p->dim == 2 && (!by || !dby)) return E_INVAL;
  using D = Dual<double>;
  const size_t n = nodes(p), N = (size_t)nfields(p) * n;
  std::vector<D> bb(n), bbx(n), bby(n), S(N);
  for (size_t q = 0; q < n; ++q) {
    bb[q] = D(b[q], db[q]); bbx[q] = D(bx[q], dbx[q]);
    bby[q] = p->dim == 2 ? D(by[q], dby[q]) : D(0.0, 0.0);
  }
  for (size_t q = 0; q < N; ++q) S[q] = D(state[q], dstate[q]);
  Scheme<D> s;
  s.setup(convert<D>(p), bb.data(), bbx.data(), bby.data());
  int k = 0;
  const int e = s.run(S.data(), nsteps, 0.0, nullptr, &k);
  for (size_t q = 0; q < N; ++q) { out[q] = S[q].v; dout[q] = S[q].d; }
  return e;
}

// Count the arithmetic of one right-hand side (alpha given): counts = {add/sub, mul, div, sqrt, cmp}.
int orc_count_rhs(const orc_params* p, const double* state, const double* b, const double* bx, const double* by,
                  double alpha_x, double alpha_y, long long* counts) {
  Scheme<Counted> s;
  int e = make(p, b, bx, by, s);
  if (e) return e;
  const size_t n = nodes(p), N = (size_t)nfields(p) * n;
  std::vector<Counted> S = to_t<Counted>(state, N), R(N);
  Counted::reset();
  s.rhs(S.data(), S.data() + (size_t)s.nu * n, Counted(alpha_x), Counted(alpha_y), R.data(), R.data() + (size_t)s.nu * n);
  counts[0] = Counted::n_add; counts[1] = Counted::n_mul; counts[2] = Counted::n_div;
  counts[3] = Counted::n_sqrt; counts[4] = Counted::n_cmp;
  return OK;
}

// Tangent (Jacobian-vector product) of the right-hand side with alpha frozen:
// drhs = dR/dS dstate + dR/db db + dR/dbx dbx + dR/dby dby.
int orc_rhs_jvp(const orc_params* p, const double* state, const double* dstate, const double* b, const double* bx,
                const double* by, const double* db, const double* dbx, const double* dby, double alpha_x,
                double alpha_y, double* rhs, double* drhs) {
  if (!valid(p) || !state || !dstate || !b || !bx || !db || !dbx) return E_INVAL;
  if (p->dim == 2 && (!by || !dby)) return E_INVAL;
  using D = Dual<double>;
  const size_t n = nodes(p), N = (size_t)nfields(p) * n;
  std::vector<D> bb(n), bbx(n), bby(n), S(N), R(N);
  for (size_t q = 0; q < n; ++q) {
    bb[q] = D(b[q], db[q]); bbx[q] = D(bx[q], dbx[q]);
    bby[q] = p->dim == 2 ? D(by[q], dby[q]) : D(0.0, 0.0);
  }
  for (size_t q = 0; q < N; ++q) S[q] = D(state[q], dstate[q]);
  Scheme<D> s;
  s.setup(convert<D>(p), bb.data(), bbx.data(), bby.data());
  s.rhs(S.data(), S.data() + (size_t)s.nu * n, D(alpha_x), D(alpha_y), R.data(), R.data() + (size_t)s.nu * n);
  for (size_t q = 0; q < N; ++q) { rhs[q] = R[q].v; drhs[q] = R[q].d; }
  return OK;
}

// ---------------------------------------------------------------- building blocks (pins)
void orc_hw_candidates(const double* f, const double* p, double dx, double* q) { hw_candidates(f, p, dx, q); }
void orc_hw_beta(const double* f, const double* p, double dx, double* be) { hw_beta(f, p, dx, be); }
void orc_hw_weights(const double* be, double eps, double* w) { hw_weights(be, hw_gamma<double>(), eps, w); }
double orc_hweno_value(const double* f, const double* p, double dx, double eps, double* w) {
  return hweno_value(f, p, dx, eps, w);
}
double orc_hermite_dQ(const double* f, const double* p, double dx) { return hermite_dQ(f, p, dx); }
double orc_central4(double a, double b, double c, double d) { return central4(a, b, c, d); }
double orc_hweno_limit(double mm, double m0, double mp, double nm, double np, double dx, double eps) {
  return hweno_limit(mm, m0, mp, nm, np, dx, eps);
}

// dir: 0 = x (F1, Jacobian of F1, x-eigenvectors), 1 = y (F2, ...). 1D variants take 2-vectors.
void orc_flux2d(int dir, const double* U, double b, double g, double* F) {
  if (dir == 0) flux_x(U, b, g, F); else flux_y(U, b, g, F);
}
void orc_dflux2d(int dir, const double* U, double b, const double* Dv, double B, double g, double* P) {
  double J[3][3], Jb[3];
  if (dir == 0) jac_x(U, b, g, J, Jb); else jac_y(U, b, g, J, Jb);
  jmul(J, Jb, Dv, B, P);
}
// Forward-mode derivative of the flux itself: dF = d/ds F(U + s dU, b + s db) at s = 0.
void orc_flux2d_tangent(int dir, const double* U, double b, const double* dU, double db, double g, double* dF) {
  using D = Dual<double>;
  D u[3] = {D(U[0], dU[0]), D(U[1], dU[1]), D(U[2], dU[2])}, F[3];
  if (dir == 0) flux_x(u, D(b, db), D(g), F); else flux_y(u, D(b, db), D(g), F);
  for (int c = 0; c < 3; ++c) dF[c] = F[c].d;
}
void orc_eig2d(int dir, double eta, double m, double w, double b, double g, double* L, double* R) {
  double l[3][3], r[3][3];
  if (dir == 0) eig_x(eta, m, w, b, g, l, r); else eig_y(eta, m, w, b, g, l, r);
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) { L[3 * i + j] = l[i][j]; R[3 * i + j] = r[i][j]; }
}
void orc_flux1d(const double* U, double b, double g, double* F) { flux_1d(U, b, g, F); }
void orc_dflux1d(const double* U, double b, const double* V, double B, double g, double* P) { dflux_1d(U, b, V, B, g, P); }
void orc_flux1d_tangent(const double* U, double b, const double* dU, double db, double g, double* dF) {
  using D = Dual<double>;
  D u[2] = {D(U[0], dU[0]), D(U[1], dU[1])}, F[2];
  flux_1d(u, D(b, db), D(g), F);
  dF[0] = F[0].d; dF[1] = F[1].d;
}
void orc_eig1d(double eta, double m, double b, double g, double* L, double* R) {
  double l[2][2], r[2][2];
  eig_1d(eta, m, b, g, l, r);
  for (int i = 0; i < 2; ++i) for (int j = 0; j < 2; ++j) { L[2 * i + j] = l[i][j]; R[2 * i + j] = r[i][j]; }
}

}  // extern "C"

extern "C" {
// The Runge-Kutta driver on a scalar model: R(U, D) = (lam U, lam D), Lim(U, D) = mu D.
void orc_ssprk3_linear(double lam, double mu, double dt, int lim_first, double* U, double* D) {
  auto f = [&](int, const double* u, const double* d, double* ru, double* rd) { ru[0] = lam * u[0]; rd[0] = lam * d[0]; };
  auto lim = [&](const double*, const double* d, double* out) { out[0] = mu * d[0]; };
  ssprk3(U, D, 1, 1, dt, f, lim, lim_first != 0);
}
}

extern "C" {
// Count the arithmetic of one limiter evaluation Lim(S): counts = {add/sub, mul, div, sqrt, cmp}.
int orc_count_limit(const orc_params* p, const double* state, const double* b, const double* bx, const double* by,
                    long long* counts) {
  Scheme<Counted> s;
  int e = make(p, b, bx, by, s);
  if (e) return e;
  const size_t n = nodes(p), N = (size_t)nfields(p) * n;
  std::vector<Counted> S = to_t<Counted>(state, N), Dm((size_t)s.nd * n);
  Counted::reset();
  s.limit(S.data(), S.data() + (size_t)s.nu * n, Dm.data());
  counts[0] = Counted::n_add; counts[1] = Counted::n_mul; counts[2] = Counted::n_div;
  counts[3] = Counted::n_sqrt; counts[4] = Counted::n_cmp;
  return OK;
}
}
