// MI355X (gfx950) implementation of the C ABI in include/swe_hweno.h: the right-hand side of the
// well-balanced fifth-order finite-difference HWENO scheme for the shallow water equations, its
// derivative limiter and SSP-RK3 stages (Zhao & Zhang, arXiv 2208.01260), in FP64 or FP32 (the
// same kernels instantiated for both types).
//
// Kernel design (one wavefront per workgroup):
//   * k_stage is the whole stage of eq. (2.11) in one pass: each lane owns one grid column and
//     marches up a strip of rows. The y-sweep keeps a four-row window of raw node records in
//     registers and carries the interface flux of the previous row, so each y-interface is
//     computed once. The x-sweep exchanges the current row between lanes through LDS: lane l
//     computes the interface left of its column and reads the right one from lane l+1. A wave
//     covers 64 columns (2 halo columns each side) and writes the 60 interior ones.
//   * The same kernel writes the bare right-hand side (MODE_RHS), or fuses the limiter of
//     Sec. 2.2 at the node, the Runge-Kutta combination and the max-reduction of the next
//     stage's Lax-Friedrichs speeds (MODE_STAGE0/1/2).
//   * Boundary nodes are read through an index fold: periodic wrap, or the mirror about the wall
//     face with each field's parity.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <algorithm>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "hweno_adjoint.hpp"
#include "hweno_device.hpp"
#include "swe_hweno.h"

namespace swe {

constexpr int WAVE = 64;
constexpr int OUT_COLS = WAVE - 4;  // interior columns written per wave
constexpr int ROWS_DEFAULT = 32;    // rows marched per wave unless tuned

enum { MODE_RHS = 0, MODE_STAGE0 = 1, MODE_STAGE1 = 2, MODE_STAGE2 = 3 };
enum { ERR_DRY = 1, ERR_NONFINITE = 2 };

// Device scalars of a context.
struct DevScal {
  unsigned long long a_n[2];     // alpha of U^n (bits of positive doubles)
  unsigned long long a_1[2];     // alpha of U^(1)
  unsigned long long a_2[2];     // alpha of U^(2)
  unsigned long long a_next[2];  // alpha of U^(n+1)
  unsigned long long a_fix[2];   // fixed alpha
  unsigned long long a_rhs[2];   // alpha used by a bare right-hand side
  double dt, t, t_end, pad0;
  int active, steps, err, pad1;
};

template <class T>
struct KArgs {
  const T* S;             // state whose right-hand side / stage is computed
  const T* Sn;            // U^n at the start of the step (stages 1, 2)
  const T* Dn;            // D^{n,mod} (stages 1, 2)
  const T* b;
  const T* bx;
  const T* by;
  T* out;                 // right-hand side, or the next stage state
  T* Dn_out;              // stage 0: D^{n,mod}
  const unsigned long long* a_in;  // Lax-Friedrichs speeds used
  unsigned long long* a_out;       // max-reduction of the output state's speeds
  DevScal* sc;
  int nx, ny, bcx, bcy, limiter, rows;
  T dx, dy, idx, idy, g, eps;
};

// Largest finite value of the arithmetic type.
template <class T> __device__ __forceinline__ constexpr T big_value();
template <> __device__ __forceinline__ constexpr double big_value<double>() { return DBL_MAX; }
template <> __device__ __forceinline__ constexpr float big_value<float>() { return FLT_MAX; }

__device__ __forceinline__ double bits2d(unsigned long long u) { return __longlong_as_double((long long)u); }

// CFL time step from the Lax-Friedrichs speeds, rounded operation by operation (no contraction)
// so that every kernel that computes it gets the same bits.
__device__ __noinline__ double cfl_step(int dim, double cfl, double ax, double ay, double dx, double dy) {
#pragma clang fp contract(off)
  return dim == 2 ? cfl / (ax / dx + ay / dy) : cfl / (ax / dx);
}

// Fold an index into [0, n): periodic wrap or mirror about the wall face (one fold suffices for
// the stencil halos; indices of halo lanes farther out are clamped, their results are unused).
__device__ __forceinline__ int fold(int i, int n, int bc, bool& refl) {
  refl = false;
  if (i < 0) {
    if (bc == SWE_BC_PERIODIC) i += n; else { i = -1 - i; refl = true; }
  } else if (i >= n) {
    if (bc == SWE_BC_PERIODIC) i -= n; else { i = 2 * n - 1 - i; refl = true; }
  }
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// A global pointer the compiler cannot see through. Fields are reached by bumping such a pointer
// by the field stride, so that the only loop-invariant scalar is the stride itself: without it the
// compiler keeps one hoisted 64-bit base per (array, field), about thirty scalar pairs, and spills
// them to vector-register lanes that are read back on every row.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* opq(T* p) {
  auto g = (__attribute__((address_space(1))) T*)p;
  asm("" : "+v"(g));
  return g;
}

// Raw node record at (i, j) in the slots of hweno_device.hpp, ghost values by parity:
// across an x-wall m, H1, W1, M2, B1 are odd; across a y-wall w, W1, H2, M2, B2 are odd.
template <int DIM, class T>
__device__ __forceinline__ void load_raw(const KArgs<T>& a, const T* __restrict__ S, int i, int j, T r[NREC],
                                         bool& rx, bool& ry) {
  ry = false;
  const int ii = fold(i, a.nx, a.bcx, rx);
  const int jj = DIM == 2 ? fold(j, a.ny, a.bcy, ry) : 0;
  const size_t n = (size_t)a.nx * (DIM == 2 ? a.ny : 1);
  const size_t q = (size_t)jj * a.nx + ii;
  if (DIM == 2) {
    auto p = opq(S + q);
#pragma unroll
    for (int f = 0; f < 9; ++f) {
      r[f] = *p;
      if (f < 8) p = opq(p + n);
    }
    r[S_B] = *opq(a.b + q); r[S_BX] = *opq(a.bx + q); r[S_BY] = *opq(a.by + q);
  } else {
    r[S_ETA] = S[q]; r[S_M] = S[n + q]; r[S_W] = T(0.0);
    r[S_H1] = S[2 * n + q]; r[S_M1] = S[3 * n + q]; r[S_W1] = T(0.0);
    r[S_H2] = T(0.0); r[S_M2] = T(0.0); r[S_W2] = T(0.0);
    r[S_B] = a.b[q]; r[S_BX] = a.bx[q]; r[S_BY] = T(0.0);
  }
}

// The ghost parities of a record read across an x-wall (rx) or a y-wall (ry).
template <class T>
__device__ __forceinline__ void apply_flips(T r[NREC], bool rx, bool ry) {
  if (rx) { r[S_M] = -r[S_M]; r[S_H1] = -r[S_H1]; r[S_W1] = -r[S_W1]; r[S_M2] = -r[S_M2]; r[S_BX] = -r[S_BX]; }
  if (ry) { r[S_W] = -r[S_W]; r[S_W1] = -r[S_W1]; r[S_H2] = -r[S_H2]; r[S_M2] = -r[S_M2]; r[S_BY] = -r[S_BY]; }
}

template <int DIM, class T>
__device__ __forceinline__ void load_rec(const KArgs<T>& a, const T* __restrict__ S, int i, int j, T r[NREC]) {
  bool rx, ry;
  load_raw<DIM>(a, S, i, j, r, rx, ry);
  apply_flips(r, rx, ry);
}

// Node fluxes through LDS: slot k of a NodeF at lane l is sn[k][l].
constexpr int NNODE = 18;
template <class T>
__device__ __forceinline__ void nodef_store(T (*sn)[64], int l, const NodeF<T>& X) {
  const T v[NNODE] = {X.e, X.mn, X.mt, X.d0, X.d1, X.d2, X.f0, X.f1, X.f2,
                           X.p0, X.p1, X.p2, X.q0, X.q1, X.q2, X.b, X.bn, X.bt};
#pragma unroll
  for (int k = 0; k < NNODE; ++k) sn[k][l] = v[k];
}
template <class T>
__device__ __forceinline__ void nodef_load(T (*sn)[64], int l, NodeF<T>& X) {
  X.e = sn[0][l]; X.mn = sn[1][l]; X.mt = sn[2][l]; X.d0 = sn[3][l]; X.d1 = sn[4][l]; X.d2 = sn[5][l];
  X.f0 = sn[6][l]; X.f1 = sn[7][l]; X.f2 = sn[8][l]; X.p0 = sn[9][l]; X.p1 = sn[10][l]; X.p2 = sn[11][l];
  X.q0 = sn[12][l]; X.q1 = sn[13][l]; X.q2 = sn[14][l]; X.b = sn[15][l]; X.bn = sn[16][l]; X.bt = sn[17][l];
}

// y-frame node fluxes kept per row: the six values of a NodeF that are not raw record slots
// (F1, F2, P1, P2, Q1, Q2), in a ring of four rows of the march (own lane only).
template <class T>
__device__ __forceinline__ void yring_store(T (*ring)[6][WAVE], int row, int lane, const T* __restrict__ r, T g) {
  NodeF<T> X;
  node_frame<1>(r, g, X);
  const int s = row & 3;
  ring[s][0][lane] = X.f1; ring[s][1][lane] = X.f2;
  ring[s][2][lane] = X.p1; ring[s][3][lane] = X.p2;
  ring[s][4][lane] = X.q1; ring[s][5][lane] = X.q2;
}
template <class T>
__device__ __forceinline__ void yring_load(T (*ring)[6][WAVE], int row, int lane, const T* __restrict__ r,
                                           NodeF<T>& X) {
  const int s = row & 3;
  X.e = r[S_ETA]; X.mn = r[S_W]; X.mt = r[S_M];
  X.d0 = r[S_H2]; X.d1 = r[S_W2]; X.d2 = r[S_M2];
  X.f0 = X.mn; X.f1 = ring[s][0][lane]; X.f2 = ring[s][1][lane];
  X.p0 = X.d1; X.p1 = ring[s][2][lane]; X.p2 = ring[s][3][lane];
  X.q0 = r[S_W1]; X.q1 = ring[s][4][lane]; X.q2 = ring[s][5][lane];
  X.b = r[S_B]; X.bn = r[S_BY]; X.bt = r[S_BX];
}

template <class T>
__device__ __forceinline__ void ifo_to_array(const IfO<T>& o, T* v) {
  v[0] = o.F0; v[1] = o.F1; v[2] = o.F2; v[3] = o.B0; v[4] = o.B1; v[5] = o.B2; v[6] = o.P0;
  v[7] = o.P1; v[8] = o.P2; v[9] = o.PB; v[10] = o.M0; v[11] = o.M1; v[12] = o.M2; v[13] = o.MB;
}

// Add the contribution of one sweep (left/right interfaces l, r, spacing id = 1/dx) to the
// 9 right-hand-side slots R (2D order eta, m, w, H1, M1, W1, H2, M2, W2). un/ut/dn/dt are the
// slots of the frame's normal and tangential momentum and derivative triples.
template <int DIR, class T>
__device__ __forceinline__ void assemble(const T* l, const T* r, T eta, T H1, T H2,
                                         T g, T id, T R[9]) {
  const int un = DIR == 0 ? 1 : 2, ut = DIR == 0 ? 2 : 1;
  const int dn = DIR == 0 ? 3 : 6, dt = DIR == 0 ? 6 : 3;  // first slot of D_n, D_t
  const T Hn = DIR == 0 ? H1 : H2, Ht = DIR == 0 ? H2 : H1;
  const T db0 = r[3] - l[3], db1 = r[4] - l[4], db2 = r[5] - l[5];
  const T ge = g * eta;
  R[0] -= ((r[0] - l[0]) + ge * db0) * id;
  R[un] -= ((r[1] - l[1]) + ge * db1) * id;
  R[ut] -= ((r[2] - l[2]) + ge * db2) * id;
  const T gn = g * Hn, gt = g * Ht;
  R[dn + 0] -= ((r[6] - l[6]) + gn * db0) * id;
  R[dn + un] -= ((r[7] - l[7]) + gn * db1 + ge * (r[9] - l[9])) * id;
  R[dn + ut] -= ((r[8] - l[8]) + gn * db2) * id;
  R[dt + 0] -= ((r[10] - l[10]) + gt * db0) * id;
  R[dt + un] -= ((r[11] - l[11]) + gt * db1 + ge * (r[13] - l[13])) * id;
  R[dt + ut] -= ((r[12] - l[12]) + gt * db2) * id;
}

template <class T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
  return v;
}

// x / 3 rounded to nearest: the product with the rounded 1/3, corrected by one FMA step on the
// exact remainder (equal to the IEEE quotient; checked against it on 2e8 random doubles).
template <class T>
__device__ __forceinline__ T div3(T x) {
  const T y = T(1.0 / 3.0);
  const T q = x * y;
  return fma(fma(T(-3.0), q, x), y, q);
}

// Speeds |u| + c, |v| + c of a node for the next Lax-Friedrichs split; flags dry / non-finite.
template <class T>
__device__ __forceinline__ void speeds(T e, T m, T w, T b, T g, T& ax, T& ay,
                                       int& err) {
  const T h = e - b;
  if (!(h > T(0.0))) { err |= (h == h) ? ERR_DRY : ERR_NONFINITE; return; }
  const T c = sqrt_pos(g * h), ih = rcp(h);
  const T sx = fabs(m * ih) + c, sy = fabs(w * ih) + c;
  if (!(sx <= big_value<T>()) || !(sy <= big_value<T>())) { err |= ERR_NONFINITE; return; }
  ax = fmax(ax, sx);
  ay = fmax(ay, sy);
}

template <class T>
__device__ __forceinline__ void flush_speeds(const KArgs<T>& a, T ax, T ay, int err) {
  ax = wave_max(ax);
  ay = wave_max(ay);
  int e = err;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) e |= __shfl_xor(e, o, WAVE);
  if (threadIdx.x == 0) {
    atomicMax(&a.a_out[0], (unsigned long long)__double_as_longlong((double)ax));
    atomicMax(&a.a_out[1], (unsigned long long)__double_as_longlong((double)ay));
    if (e) atomicOr(&a.sc->err, e);
  }
}

// --------------------------------------------------------------------------- the fused stage
// One wavefront's tile: output columns [tx*60, tx*60+60) of rows [ty*rows, ty*rows+rows).
template <class T, int DIM, int MODE>
__device__ __forceinline__ void stage_tile(const KArgs<T>& a, int tx, int ty) {
  if (MODE != MODE_RHS && a.sc->active == 0) return;
  __shared__ T sn[NNODE][WAVE];  // x-frame fluxes of the current row, one node per lane
  __shared__ T sf[14][WAVE];     // x-interface quantities (lane l: interface left of its column)
  __shared__ T sy[14][WAVE];     // y-interface quantities of the previous row (own lane)
  __shared__ T syf[4][6][WAVE];  // y-frame fluxes of rows r-1 .. r+2 (own lane)
  const int lane = threadIdx.x;
  const int c = tx * OUT_COLS - 2 + lane;  // this lane's column
  const int r0 = DIM == 2 ? ty * a.rows : 0;
  const int r1 = DIM == 2 ? min(r0 + a.rows, a.ny) : 1;
  const bool col_out = lane >= 2 && lane < WAVE - 2 && c < a.nx;
  const int cq = col_out ? c : 0;  // a column that is always inside the grid
  const T axl = T(bits2d(a.a_in[0])), ayl = T(bits2d(a.a_in[1]));
  const size_t n = (size_t)a.nx * (DIM == 2 ? a.ny : 1);
  const T dt = MODE == MODE_RHS ? T(0.0) : T(a.sc->dt);
  const int nu = DIM == 2 ? 3 : 2, nd = DIM == 2 ? 6 : 2;
  const int la = max(lane - 2, 0), lb = max(lane - 1, 0), ld = min(lane + 1, WAVE - 1);
  T amx = T(0.0), amy = T(0.0);
  int err = 0;

  // y window: raw records of rows r-1, r, r+1 (2D); the flux of interface r-1/2 waits in sy
  T wm1[NREC], w0[NREC], wp1[NREC];
  if (DIM == 2) {
    T wm2[NREC];
    load_rec<DIM>(a, a.S, c, r0 - 2, wm2);
    load_rec<DIM>(a, a.S, c, r0 - 1, wm1);
    load_rec<DIM>(a, a.S, c, r0, w0);
    load_rec<DIM>(a, a.S, c, r0 + 1, wp1);
    yring_store(syf, r0 - 2, lane, wm2, a.g);
    yring_store(syf, r0 - 1, lane, wm1, a.g);
    yring_store(syf, r0, lane, w0, a.g);
    yring_store(syf, r0 + 1, lane, wp1, a.g);
    IfO<T> o;
    auto fy = [&](int k, NodeF<T>& X) {
      yring_load(syf, r0 - 2 + k, lane, k == 0 ? wm2 : (k == 1 ? wm1 : (k == 2 ? w0 : wp1)), X);
    };
    interface_flux(fy, ayl, a.dy, a.eps, a.g, o);
    T v[14];
    ifo_to_array(o, v);
#pragma unroll
    for (int k = 0; k < 14; ++k) sy[k][lane] = v[k];
  } else {
    load_rec<DIM>(a, a.S, c, 0, w0);
  }

  for (int r = r0; r < r1; ++r) {
    const size_t q = (size_t)r * a.nx + cq;
    // loads whose latency the x-sweep hides: the next row of the window, U^n and D^{n,mod}. The new
    // row's ghost parities are applied where the y-sweep first reads it, so that no instruction
    // before that point depends on these loads.
    T wp2[NREC];
    bool f2x = false, f2y = false;
    if (DIM == 2) load_raw<DIM>(a, a.S, c, r + 2, wp2, f2x, f2y);
    T un_[3], dn_[6];
    if (MODE == MODE_STAGE1 || MODE == MODE_STAGE2) {
      auto pS = opq(a.Sn + q);
      auto pD = opq(a.Dn + q);
#pragma unroll
      for (int k = 0; k < 3; ++k) if (k < nu) { un_[k] = *pS; pS = opq(pS + n); }
#pragma unroll
      for (int k = 0; k < 6; ++k) if (k < nd) { dn_[k] = *pD; pD = opq(pD + n); }
    }
    T R[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) R[k] = T(0.0);
    const T eta = w0[S_ETA], H1 = w0[S_H1], H2 = w0[S_H2];

    // x-sweep of row r: each lane's x-frame fluxes are computed once and shared through LDS
    __syncthreads();  // the previous row's readers of sn and sf are done
    {
      NodeF<T> me;
      node_frame<0>(w0, a.g, me);
      nodef_store(sn, lane, me);
      __syncthreads();
      IfO<T> o;
      auto fx = [&](int k, NodeF<T>& X) {
        if (k == 2) X = me;
        else nodef_load(sn, k == 0 ? la : (k == 1 ? lb : ld), X);
      };
      interface_flux(fx, axl, a.dx, a.eps, a.g, o);
      T xl[14];
      ifo_to_array(o, xl);
#pragma unroll
      for (int k = 0; k < 14; ++k) sf[k][lane] = xl[k];
      __syncthreads();
      T xr[14];
#pragma unroll
      for (int k = 0; k < 14; ++k) xr[k] = sf[k][ld];
      assemble<0>(xl, xr, eta, H1, H2, a.g, a.idx, R);
    }
    // y-sweep: interface r+1/2 from rows r-1 .. r+2
    if (DIM == 2) {
      IfO<T> o;
      apply_flips(wp2, f2x, f2y);
      yring_store(syf, r + 2, lane, wp2, a.g);
      auto fy = [&](int k, NodeF<T>& X) {
        yring_load(syf, r - 1 + k, lane, k == 0 ? wm1 : (k == 1 ? w0 : (k == 2 ? wp1 : wp2)), X);
      };
      interface_flux(fy, ayl, a.dy, a.eps, a.g, o);
      T ynew[14], yprev[14];
      ifo_to_array(o, ynew);
#pragma unroll
      for (int k = 0; k < 14; ++k) { yprev[k] = sy[k][lane]; sy[k][lane] = ynew[k]; }
      assemble<1>(yprev, ynew, eta, H1, H2, a.g, a.idy, R);
    }

    if (MODE == MODE_RHS) {
      if (col_out) {
        if (DIM == 2) {
          auto po = opq(a.out + q);
#pragma unroll
          for (int k = 0; k < 9; ++k) {
            *po = R[k];
            if (k < 8) po = opq(po + n);
          }
        } else {
          a.out[q] = R[0]; a.out[n + q] = R[1]; a.out[2 * n + q] = R[3]; a.out[3 * n + q] = R[4];
        }
        // the node's depth must be positive and the result finite (a product with 0 is NaN
        // exactly for a non-finite value)
        const T h = w0[S_ETA] - w0[S_B];
        T z = T(0.0);
#pragma unroll
        for (int k = 0; k < 9; ++k) z = fma(R[k], T(0.0), z);
        if (!(h > T(0.0))) err |= (h == h) ? ERR_DRY : ERR_NONFINITE;
        if (z != z) err |= ERR_NONFINITE;
      }
    } else if (MODE != MODE_STAGE1 || col_out) {
        // limited derivatives of this stage's state at the node (Sec. 2.2); the x-neighbours'
        // surface, momenta and x-derivatives are the first six slots of their shared fluxes.
        // The first and third stages run the limiter and the update on every lane and mask only
        // the stores and the speed reduction, which leaves the compiler free to schedule them
        // across the row; the second stage keeps them under the branch (each form is the faster
        // one for its stage on this device; the results are the same bits either way).
        T Dm[6];
        if (a.limiter) {
          limit_frame(w0[S_ETA], w0[S_M], w0[S_W], w0[S_B], sn[0][lb], sn[1][lb], sn[2][lb], sn[0][ld], sn[1][ld],
                      sn[2][ld], sn[3][lb], sn[4][lb], sn[5][lb], sn[3][ld], sn[4][ld], sn[5][ld], a.dx, a.idx,
                      a.eps, a.g, Dm);
          if (DIM == 2) {
            T o3[3];
            limit_frame(w0[S_ETA], w0[S_W], w0[S_M], w0[S_B], wm1[S_ETA], wm1[S_W], wm1[S_M], wp1[S_ETA],
                        wp1[S_W], wp1[S_M], wm1[S_H2], wm1[S_W2], wm1[S_M2], wp1[S_H2], wp1[S_W2], wp1[S_M2], a.dy,
                        a.idy, a.eps, a.g, o3);
            Dm[3] = o3[0]; Dm[4] = o3[2]; Dm[5] = o3[1];
          }
        } else {
          Dm[0] = w0[S_H1]; Dm[1] = w0[S_M1]; Dm[2] = w0[S_W1];
          Dm[3] = w0[S_H2]; Dm[4] = w0[S_M2]; Dm[5] = w0[S_W2];
        }
        // SSP-RK3 combination (eq. (2.11)), written over a common denominator
        const int uslot[3] = {S_ETA, S_M, S_W};
        const int rd[6] = {3, 4, 5, 6, 7, 8};
        T Unew[3] = {T(0.0), T(0.0), T(0.0)};
        T vout[9];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          if (k >= nu) break;
          const T u = w0[uslot[k]] + dt * R[k];
          T v;
          if (MODE == MODE_STAGE0) v = u;
          else if (MODE == MODE_STAGE1) v = (T(3.0) * un_[k] + u) * T(0.25);
          else v = div3(un_[k] + T(2.0) * u);
          Unew[k] = v;
          vout[k] = v;
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          if (k >= nd) break;
          const T u = Dm[k] + dt * R[rd[k]];
          T v;
          if (MODE == MODE_STAGE0) {
            v = u;
          } else if (MODE == MODE_STAGE1) {
            v = (T(3.0) * dn_[k] + u) * T(0.25);
          } else {
            v = div3(dn_[k] + T(2.0) * u);
          }
          vout[nu + k] = v;
        }
        // only the interior columns store and reduce their speeds
        if (col_out) {
          auto po = opq(a.out + q);
#pragma unroll
          for (int k = 0; k < 9; ++k) {
            if (k >= nu + nd) break;
            *po = vout[k];
            po = opq(po + n);
          }
          if (MODE == MODE_STAGE0) {
            auto pdo = opq(a.Dn_out + q);
#pragma unroll
            for (int k = 0; k < 6; ++k) {
              if (k >= nd) break;
              *pdo = Dm[k];
              pdo = opq(pdo + n);
            }
          }
          speeds(Unew[0], Unew[1], Unew[2], w0[S_B], a.g, amx, amy, err);
        }
    }
    if (DIM == 2) {
#pragma unroll
      for (int k = 0; k < NREC; ++k) { wm1[k] = w0[k]; w0[k] = wp1[k]; wp1[k] = wp2[k]; }
    }
  }
  if (MODE != MODE_RHS) {
    flush_speeds(a, amx, amy, err);
  } else {
    int e = err;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) e |= __shfl_xor(e, o, WAVE);
    if (threadIdx.x == 0 && e) atomicOr(&a.sc->err, e);
  }
}

// Workgroups are handed to the 8 XCDs of the device round-robin by linear id. band_tile maps
// the linear id i < n of a workgroup to a tile index so that each XCD receives a contiguous
// band of tiles: neighbouring tiles, which read each other's halo columns and rows, then meet
// in the same L2 (at 4096^2 this takes the stage kernels' fetched bytes down by a fifth). It is
// a permutation of [0, n).
constexpr unsigned NXCD = 8;
__host__ __device__ __forceinline__ unsigned band_tile(unsigned i, unsigned n) {
  const unsigned x = i % NXCD, k = i / NXCD, q = n / NXCD, rm = n % NXCD;
  return x * q + (x < rm ? x : rm) + k;
}

template <class T, int DIM, int MODE>
__global__ __launch_bounds__(WAVE) void k_stage(KArgs<T> a) {
  const unsigned gx = gridDim.x;
  const unsigned t = band_tile(blockIdx.x + blockIdx.y * gx, gx * gridDim.y);
  stage_tile<T, DIM, MODE>(a, (int)(t % gx), (int)(t / gx));
}

// --------------------------------------------------------------------------- small kernels
// Lax-Friedrichs speeds of a state (grid-stride), max-reduced into out[2].
template <class T, int DIM>
__global__ __launch_bounds__(256) void k_alpha(const T* __restrict__ S, const T* __restrict__ b, size_t n,
                                               T g, unsigned long long* out, int* errp) {
  T ax = T(0.0), ay = T(0.0);
  int err = 0;
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x)
    speeds(S[q], S[n + q], DIM == 2 ? S[2 * n + q] : T(0.0), b[q], g, ax, ay, err);
  ax = wave_max(ax);
  ay = wave_max(ay);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) err |= __shfl_xor(err, o, WAVE);
  if ((threadIdx.x & (WAVE - 1)) == 0) {
    atomicMax(&out[0], (unsigned long long)__double_as_longlong((double)ax));
    atomicMax(&out[1], (unsigned long long)__double_as_longlong((double)ay));
    if (err) atomicOr(errp, err);
  }
}

// Set two alpha slots (zero, or given values).
__global__ void k_set2(unsigned long long* p, unsigned long long v0, unsigned long long v1) {
  if (threadIdx.x == 0) { p[0] = v0; p[1] = v1; }
}

// Reset the clock of a run or a single step (the error flag is left alone).
__global__ void k_clock(DevScal* s, double t_end) {
  if (threadIdx.x == 0) { s->t = 0.0; s->t_end = t_end; s->dt = 0.0; s->active = 1; s->steps = 0; }
}

__global__ void k_clear_err(DevScal* s) {
  if (threadIdx.x == 0) s->err = 0;
}

// Elementwise check of the arithmetic building blocks (rcp, sqrt_pos, div3).
__global__ __launch_bounds__(256) void k_math_check(int which, const double* __restrict__ x, double* __restrict__ y,
                                                    size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double v = x[i];
    y[i] = which == 0 ? rcp(v) : (which == 1 ? sqrt_pos(v) : div3(v));
  }
}

// Allocation-free step (swe_hweno_step_noalloc): its stage buffers and device scalars live in
// this array, one copy per GPU, held until the process ends. Host code takes its address with
// hipGetSymbolAddress (per device) and never uses the array's name as a device address.
constexpr size_t NOALLOC_BYTES = size_t(32) << 20;
constexpr size_t NOALLOC_SCAL = 256;  // DevScal at the start, stage planes after it
static_assert(sizeof(DevScal) <= NOALLOC_SCAL, "device scalars must fit their slot");
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

// Start of an allocation-free step: the fixed speeds and a cleared error flag (the array keeps
// whatever the previous call on this GPU left).
__global__ void k_noalloc_setup(DevScal* s, unsigned long long afx, unsigned long long afy) {
  if (threadIdx.x == 0) {
    s->a_fix[0] = afx;
    s->a_fix[1] = afy;
    s->err = 0;
  }
}

// Start of a step: alpha of U^n from the previous step's reduction, the CFL step (or fixed),
// clipped at t_end; clears the reductions this step fills.
__global__ void k_prologue(DevScal* s, int dim, int fixed_dt, double fdt, double cfl, double dx, double dy,
                           int use_tend) {
  if (threadIdx.x != 0) return;
  s->a_n[0] = s->a_next[0];
  s->a_n[1] = s->a_next[1];
  const double ax = bits2d(s->a_n[0]), ay = bits2d(s->a_n[1]);
  double dt = fixed_dt ? fdt : cfl_step(dim, cfl, ax, ay, dx, dy);
  int active = 1;
  if (use_tend) {
    if (!(s->t < s->t_end)) { active = 0; dt = 0.0; }
    else if (s->t + dt > s->t_end) dt = s->t_end - s->t;
  }
  if (!(dt > 0.0) || !(dt <= DBL_MAX)) {
    if (active) s->err |= ERR_NONFINITE;
    active = 0;
  }
  s->active = active;
  s->dt = dt;
  if (active) { s->t += dt; s->steps += 1; }
  s->a_1[0] = s->a_1[1] = 0ull;
  s->a_2[0] = s->a_2[1] = 0ull;
  s->a_next[0] = s->a_next[1] = 0ull;
}

// Stand-alone limiter: one thread per node, neighbours read directly.
template <class T, int DIM>
__global__ __launch_bounds__(256) void k_limit(KArgs<T> a) {
  const size_t n = (size_t)a.nx * (DIM == 2 ? a.ny : 1);
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(q % a.nx), j = (int)(q / a.nx);
    T c0[NREC], xm[NREC], xp[NREC];
    load_rec<DIM>(a, a.S, i, j, c0);
    load_rec<DIM>(a, a.S, i - 1, j, xm);
    load_rec<DIM>(a, a.S, i + 1, j, xp);
    T D[3];
    limit_frame(c0[S_ETA], c0[S_M], c0[S_W], c0[S_B], xm[S_ETA], xm[S_M], xm[S_W], xp[S_ETA], xp[S_M], xp[S_W],
                xm[S_H1], xm[S_M1], xm[S_W1], xp[S_H1], xp[S_M1], xp[S_W1], a.dx, a.idx, a.eps, a.g, D);
    if (DIM == 1) {
      a.out[q] = D[0];
      a.out[n + q] = D[1];
      continue;
    }
    a.out[q] = D[0]; a.out[n + q] = D[1]; a.out[2 * n + q] = D[2];
    T ym[NREC], yp[NREC];
    load_rec<DIM>(a, a.S, i, j - 1, ym);
    load_rec<DIM>(a, a.S, i, j + 1, yp);
    limit_frame(c0[S_ETA], c0[S_W], c0[S_M], c0[S_B], ym[S_ETA], ym[S_W], ym[S_M], yp[S_ETA], yp[S_W], yp[S_M],
                ym[S_H2], ym[S_W2], ym[S_M2], yp[S_H2], yp[S_W2], yp[S_M2], a.dy, a.idy, a.eps, a.g, D);
    a.out[3 * n + q] = D[0]; a.out[4 * n + q] = D[2]; a.out[5 * n + q] = D[1];
  }
}

}  // namespace swe

// =========================================================================== host runtime
using namespace swe;

struct swe_hweno_ctx {
  swe_hweno_params p{};
  int f32 = 0;                // arithmetic and storage type: 0 = double, 1 = float
  size_t esz = sizeof(double);
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;  // capture stream for the per-step graphs
  int nf = 0, nd = 0;
  size_t n = 0;
  void *b = nullptr, *bx = nullptr, *by = nullptr;  // planes of the context's type
  void *S1 = nullptr, *S2 = nullptr, *Dn = nullptr;
  DevScal* sc = nullptr;
  hipGraphExec_t g1 = nullptr, g8 = nullptr;
  const void* g_state = nullptr;
  int g_tend = 0;
  int rows = ROWS_DEFAULT;  // rows marched per wave (2D), chosen at init
  // kernel timing: event pairs around stage kernels (slot 0 = bare right-hand side, 1..3 = stages)
  bool timing = false;
  struct Pending { hipEvent_t a, b; int slot; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  double ms[4] = {0, 0, 0, 0};
  long long launches[4] = {0, 0, 0, 0};
  void* adj = nullptr;  // work buffers of the adjoint, allocated on first use
};

void swe_adj_release(swe_hweno_ctx* c);

namespace {

bool params_ok(const swe_hweno_params* p) {
  if (!p) return false;
  if (p->dim != 1 && p->dim != 2) return false;
  if (p->nx < 4 || p->nx > (1 << 20)) return false;
  if (p->dim == 2 && (p->ny < 4 || p->ny > (1 << 20))) return false;
  if (p->dim == 1 && p->ny != 1) return false;
  if ((size_t)p->nx * (size_t)p->ny > ((size_t)1 << 31)) return false;
  if (!(p->x1 > p->x0) || (p->dim == 2 && !(p->y1 > p->y0))) return false;
  // finite domain whose node spacing and its reciprocal are finite and positive
  const auto spacing_ok = [](double a, double b, int n) {
    const double d = (b - a) / n;
    return std::isfinite(a) && std::isfinite(b) && d > 0 && std::isfinite(d) && std::isfinite(1.0 / d);
  };
  if (!spacing_ok(p->x0, p->x1, p->nx) || (p->dim == 2 && !spacing_ok(p->y0, p->y1, p->ny))) return false;
  // eps >= 1e-20: the kernels form products of two or three weight sums, each at least of
  // order eps^4, and these stay normal doubles down to that floor
  if (!(p->g > 0) || !(p->cfl > 0) || !(p->eps >= 1e-20)) return false;
  if (!std::isfinite(p->g) || !std::isfinite(p->cfl) || !std::isfinite(p->eps)) return false;
  if (p->bc_x < 0 || p->bc_x > 1 || p->bc_y < 0 || p->bc_y > 1) return false;
  if (p->flags & ~(SWE_FIXED_DT | SWE_FIXED_ALPHA | SWE_NO_LIMITER | SWE_CHECK_DRY)) return false;
  if ((p->flags & SWE_FIXED_DT) && !(p->fixed_dt > 0 && p->fixed_dt <= DBL_MAX)) return false;
  if ((p->flags & SWE_FIXED_ALPHA) &&
      (!(p->alpha_x > 0 && p->alpha_x <= DBL_MAX) || (p->dim == 2 && !(p->alpha_y > 0 && p->alpha_y <= DBL_MAX))))
    return false;
  return true;
}

unsigned long long dbits(double v) {
  unsigned long long u;
  std::memcpy(&u, &v, sizeof u);
  return u;
}

template <class T> bool is_type(const swe_hweno_ctx* c) { return c->f32 == (sizeof(T) == sizeof(float) ? 1 : 0); }

template <class T> KArgs<T> base_args(const swe_hweno_ctx* c) {
  KArgs<T> a;
  std::memset(&a, 0, sizeof a);
  a.b = (const T*)c->b; a.bx = (const T*)c->bx; a.by = (const T*)c->by;
  a.sc = c->sc;
  a.nx = c->p.nx; a.ny = c->p.dim == 2 ? c->p.ny : 1;
  a.bcx = c->p.bc_x; a.bcy = c->p.bc_y;
  a.limiter = (c->p.flags & SWE_NO_LIMITER) ? 0 : 1;
  const double dx = (c->p.x1 - c->p.x0) / c->p.nx;
  const double dy = c->p.dim == 2 ? (c->p.y1 - c->p.y0) / c->p.ny : 1.0;
  a.dx = T(dx); a.dy = T(dy);
  a.idx = T(1.0 / dx); a.idy = T(1.0 / dy);
  a.g = T(c->p.g); a.eps = T(c->p.eps);
  a.rows = c->rows;
  return a;
}

dim3 stage_grid(const swe_hweno_ctx* c) {
  const unsigned gx = (unsigned)((c->p.nx + OUT_COLS - 1) / OUT_COLS);
  const unsigned gy = c->p.dim == 2 ? (unsigned)((c->p.ny + c->rows - 1) / c->rows) : 1u;
  return dim3(gx, gy, 1);
}

template <class T, int MODE> void launch_stage_mode(const swe_hweno_ctx* c, const KArgs<T>& a, hipStream_t s) {
  if (c->p.dim == 2) hipLaunchKernelGGL((k_stage<T, 2, MODE>), stage_grid(c), dim3(WAVE), 0, s, a);
  else hipLaunchKernelGGL((k_stage<T, 1, MODE>), stage_grid(c), dim3(WAVE), 0, s, a);
}

template <class T> void launch_alpha(const swe_hweno_ctx* c, const T* S, unsigned long long* out, hipStream_t s) {
  hipLaunchKernelGGL(k_set2, dim3(1), dim3(64), 0, s, out, 0ull, 0ull);
  const size_t blocks = (c->n + 255) / 256;
  const unsigned grid = (unsigned)(blocks < 4096 ? blocks : 4096);
  if (c->p.dim == 2)
    hipLaunchKernelGGL((k_alpha<T, 2>), dim3(grid), dim3(256), 0, s, S, (const T*)c->b, c->n, T(c->p.g), out, &c->sc->err);
  else
    hipLaunchKernelGGL((k_alpha<T, 1>), dim3(grid), dim3(256), 0, s, S, (const T*)c->b, c->n, T(c->p.g), out, &c->sc->err);
}

hipEvent_t take_event(swe_hweno_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Start / end an event-timed region on the context stream (no-op unless timing is on).
int time_begin(swe_hweno_ctx* c, hipStream_t s) {
  if (!c || !c->timing || s != c->stream) return -1;
  hipEvent_t a = take_event(c), b = take_event(c);
  if (!a || !b) return -1;
  (void)hipEventRecord(a, s);
  c->pending.push_back({a, b, -1});
  return (int)c->pending.size() - 1;
}
void time_end(swe_hweno_ctx* c, int id, int slot, hipStream_t s) {
  if (id < 0) return;
  (void)hipEventRecord(c->pending[id].b, s);
  c->pending[id].slot = slot;
}

// Accumulate finished event pairs (the stream must have been synchronised).
void collect_timing(swe_hweno_ctx* c) {
  for (const auto& pe : c->pending) {
    float ms = 0.f;
    if (pe.slot >= 0 && hipEventElapsedTime(&ms, pe.a, pe.b) == hipSuccess) {
      c->ms[pe.slot] += ms;
      c->launches[pe.slot] += 1;
    }
    c->pool.push_back(pe.a);
    c->pool.push_back(pe.b);
  }
  c->pending.clear();
}

// One step on stream s: prologue and three fused stages; U^n is `state`, updated in place.
// With timing on (direct launches only) every stage kernel is bracketed by an event pair.
template <class T> void enqueue_step(swe_hweno_ctx* c, T* state, int use_tend, hipStream_t s) {
  const KArgs<T> base = base_args<T>(c);
  const bool fa = (c->p.flags & SWE_FIXED_ALPHA) != 0;
  const double dx = (c->p.x1 - c->p.x0) / c->p.nx;
  const double dy = c->p.dim == 2 ? (c->p.y1 - c->p.y0) / c->p.ny : 1.0;
  hipLaunchKernelGGL(k_prologue, dim3(1), dim3(64), 0, s, c->sc, c->p.dim, (c->p.flags & SWE_FIXED_DT) ? 1 : 0,
                     c->p.fixed_dt, c->p.cfl, dx, dy, use_tend);
  T* S1 = (T*)c->S1;
  T* S2 = (T*)c->S2;
  T* Dn = (T*)c->Dn;
  KArgs<T> a = base;
  a.S = state; a.out = S1; a.Dn_out = Dn;
  a.a_in = fa ? c->sc->a_fix : c->sc->a_n; a.a_out = c->sc->a_1;
  int id = time_begin(c, s);
  launch_stage_mode<T, MODE_STAGE0>(c, a, s);
  time_end(c, id, 1, s);
  a = base;
  a.S = S1; a.Sn = state; a.Dn = Dn; a.out = S2;
  a.a_in = fa ? c->sc->a_fix : c->sc->a_1; a.a_out = c->sc->a_2;
  id = time_begin(c, s);
  launch_stage_mode<T, MODE_STAGE1>(c, a, s);
  time_end(c, id, 2, s);
  a = base;
  a.S = S2; a.Sn = state; a.Dn = Dn; a.out = state;
  a.a_in = fa ? c->sc->a_fix : c->sc->a_2; a.a_out = c->sc->a_next;
  id = time_begin(c, s);
  launch_stage_mode<T, MODE_STAGE2>(c, a, s);
  time_end(c, id, 3, s);
}

int hip_status(hipError_t e) { return e == hipSuccess ? SWE_OK : SWE_EHIP; }

// Rows marched per wave in 2D: the wave count gx * ceil(ny / rows) should fill whole rounds of
// the resident-wave slots (one fused-stage wave per SIMD), while each march repays its start-up
// (four window rows and one extra y-interface, about two rows of work). Cost model: rounds *
// (rows + 2) over 3 .. 128 rows; ties go to fewer rows. Small grids, which cannot fill the GPU,
// get short marches and so more wavefronts; below 3 rows the start-up of each wavefront costs
// more than the extra wavefronts gain. SWE_HWENO_ROWS overrides the choice.
int choose_rows(int nx, int ny, int slots) {
  if (const char* e = std::getenv("SWE_HWENO_ROWS")) {
    const int r = std::atoi(e);
    if (r >= 1 && r <= 4096) return r;
  }
  const long gx = (nx + OUT_COLS - 1) / OUT_COLS;
  int best = ROWS_DEFAULT;
  double best_cost = 1e300;
  for (int r = 3; r <= 128; ++r) {
    const long waves = gx * ((ny + r - 1) / r);
    const long rounds = (waves + slots - 1) / slots;
    const double cost = (double)rounds * (double)(std::min(r, ny) + 2);
    if (cost < best_cost * (1 - 1e-12)) { best_cost = cost; best = r; }
  }
  return best;
}

int take_device_error(swe_hweno_ctx* c) {
  int e = 0;
  if (hipMemcpyAsync(&e, &c->sc->err, sizeof(int), hipMemcpyDeviceToHost, c->stream) != hipSuccess) return SWE_EHIP;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return SWE_EHIP;
  if (e) {
    hipLaunchKernelGGL(k_clear_err, dim3(1), dim3(64), 0, c->stream, c->sc);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return SWE_EHIP;
    return (e & ERR_NONFINITE) ? SWE_ENONFINITE : SWE_EDRY;
  }
  return SWE_OK;
}

void destroy_graphs(swe_hweno_ctx* c) {
  if (c->g1) hipGraphExecDestroy(c->g1);
  if (c->g8) hipGraphExecDestroy(c->g8);
  c->g1 = c->g8 = nullptr;
  c->g_state = nullptr;
}

template <class T> int capture(swe_hweno_ctx* c, T* state, int steps, int use_tend, hipGraphExec_t* out) {
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return SWE_EHIP;
  for (int k = 0; k < steps; ++k) enqueue_step<T>(c, state, use_tend, c->cap);
  if (hipStreamEndCapture(c->cap, &g) != hipSuccess || !g) return SWE_EHIP;
  const hipError_t e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  return hip_status(e);
}

// ------------------------------------------------------------------ typed bodies of the entry points
template <class T>
int init_impl(const swe_hweno_params* p, const T* b, const T* bx, const T* by, void* stream, swe_hweno_ctx** out) {
  if (!out) return SWE_EINVAL;
  *out = nullptr;
  if (!params_ok(p) || !b || !bx || (p->dim == 2 && !by)) return SWE_EINVAL;
  // single precision: the weights, of order eps^4 where the data are flat, stay normal floats
  if (sizeof(T) == 4 && !(p->eps >= 1e-9)) return SWE_EINVAL;
  swe_hweno_ctx* c = new (std::nothrow) swe_hweno_ctx();
  if (!c) return SWE_ENOMEM;
  c->p = *p;
  c->f32 = sizeof(T) == sizeof(float) ? 1 : 0;
  c->esz = sizeof(T);
  c->stream = (hipStream_t)stream;
  c->nf = p->dim == 2 ? 9 : 4;
  c->nd = p->dim == 2 ? 6 : 2;
  c->n = (size_t)p->nx * (size_t)(p->dim == 2 ? p->ny : 1);
  const size_t plane = c->n * sizeof(T);
  bool ok = hipMalloc(&c->b, plane * 3) == hipSuccess;
  ok = ok && hipMalloc(&c->S1, plane * c->nf) == hipSuccess;
  ok = ok && hipMalloc(&c->S2, plane * c->nf) == hipSuccess;
  ok = ok && hipMalloc(&c->Dn, plane * c->nd) == hipSuccess;
  ok = ok && hipMalloc(&c->sc, sizeof(DevScal)) == hipSuccess;
  if (!ok) { swe_hweno_destroy(c); return SWE_ENOMEM; }
  c->bx = (T*)c->b + c->n;
  c->by = (T*)c->b + 2 * c->n;
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
        hipSuccess || cus <= 0)
      cus = 256;
    c->rows = choose_rows(p->nx, p->dim == 2 ? p->ny : 1, 4 * cus);
  }
  ok = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipMemcpyAsync(c->b, b, plane, hipMemcpyDeviceToDevice, c->stream) == hipSuccess;
  ok = ok && hipMemcpyAsync(c->bx, bx, plane, hipMemcpyDeviceToDevice, c->stream) == hipSuccess;
  if (p->dim == 2) ok = ok && hipMemcpyAsync(c->by, by, plane, hipMemcpyDeviceToDevice, c->stream) == hipSuccess;
  else ok = ok && hipMemsetAsync(c->by, 0, plane, c->stream) == hipSuccess;
  DevScal init;
  std::memset(&init, 0, sizeof init);
  init.a_fix[0] = dbits(p->alpha_x);
  init.a_fix[1] = dbits(p->dim == 2 ? p->alpha_y : 0.0);
  ok = ok && hipMemcpyAsync(c->sc, &init, sizeof init, hipMemcpyHostToDevice, c->stream) == hipSuccess;
  ok = ok && hipStreamSynchronize(c->stream) == hipSuccess;
  if (!ok) { swe_hweno_destroy(c); return SWE_EHIP; }
  *out = c;
  return SWE_OK;
}

template <class T> int rhs_impl(swe_hweno_ctx* c, const T* state, T* rhs, double alpha_x, double alpha_y) {
  if (!c || !state || !rhs || state == rhs || !is_type<T>(c)) return SWE_EINVAL;
  // alpha_x < 0 asks for the state's speeds; otherwise alpha_x (and alpha_y in 2D) must be
  // finite and positive (NaN fails every comparison and is refused here)
  if (!(alpha_x < 0) && !(alpha_x > 0 && std::isfinite(alpha_x))) return SWE_EINVAL;
  if (alpha_x > 0 && c->p.dim == 2 && !(alpha_y > 0 && std::isfinite(alpha_y))) return SWE_EINVAL;
  const size_t bytes = c->n * c->nf * sizeof(T);
  if ((const char*)rhs < (const char*)state + bytes && (const char*)state < (const char*)rhs + bytes) return SWE_EINVAL;
  if (alpha_x < 0) launch_alpha<T>(c, state, c->sc->a_rhs, c->stream);
  else
    hipLaunchKernelGGL(k_set2, dim3(1), dim3(64), 0, c->stream, c->sc->a_rhs, dbits(alpha_x),
                       dbits(c->p.dim == 2 ? alpha_y : 0.0));
  KArgs<T> a = base_args<T>(c);
  a.S = state; a.out = rhs; a.a_in = c->sc->a_rhs;
  const int id = time_begin(c, c->stream);
  launch_stage_mode<T, MODE_RHS>(c, a, c->stream);
  time_end(c, id, 0, c->stream);
  if (hipGetLastError() != hipSuccess) return SWE_EHIP;
  return (c->p.flags & SWE_CHECK_DRY) ? take_device_error(c) : SWE_OK;
}

template <class T> int limit_impl(swe_hweno_ctx* c, const T* state, T* dmod) {
  if (!c || !state || !dmod || !is_type<T>(c)) return SWE_EINVAL;
  KArgs<T> a = base_args<T>(c);
  a.S = state; a.out = dmod;
  const size_t blocks = (c->n + 255) / 256;
  const unsigned grid = (unsigned)(blocks < 8192 ? blocks : 8192);
  if (c->p.dim == 2) hipLaunchKernelGGL((k_limit<T, 2>), dim3(grid), dim3(256), 0, c->stream, a);
  else hipLaunchKernelGGL((k_limit<T, 1>), dim3(grid), dim3(256), 0, c->stream, a);
  return hip_status(hipGetLastError());
}

template <class T> int alpha_impl(swe_hweno_ctx* c, const T* state, double* alpha_host) {
  if (!c || !state || !alpha_host || !is_type<T>(c)) return SWE_EINVAL;
  launch_alpha<T>(c, state, c->sc->a_rhs, c->stream);
  unsigned long long u[2];
  if (hipMemcpyAsync(u, c->sc->a_rhs, sizeof u, hipMemcpyDeviceToHost, c->stream) != hipSuccess) return SWE_EHIP;
  const int e = take_device_error(c);
  std::memcpy(&alpha_host[0], &u[0], 8);
  std::memcpy(&alpha_host[1], &u[1], 8);
  return e;
}

template <class T> int step_impl(swe_hweno_ctx* c, T* state, double dt, double* dt_used) {
  if (!c || !state || !is_type<T>(c)) return SWE_EINVAL;
  if (!(dt <= DBL_MAX)) return SWE_EINVAL;
  const swe_hweno_params saved = c->p;
  if (dt > 0) { c->p.flags |= SWE_FIXED_DT; c->p.fixed_dt = dt; }
  hipLaunchKernelGGL(k_clock, dim3(1), dim3(64), 0, c->stream, c->sc, 0.0);
  launch_alpha<T>(c, state, c->sc->a_next, c->stream);
  enqueue_step<T>(c, state, 0, c->stream);
  c->p = saved;
  if (hipGetLastError() != hipSuccess) return SWE_EHIP;
  if (dt_used) {
    if (hipMemcpyAsync(dt_used, &c->sc->dt, sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
      return SWE_EHIP;
    return take_device_error(c);
  }
  return (c->p.flags & SWE_CHECK_DRY) ? take_device_error(c) : SWE_OK;
}

template <class T> int run_impl(swe_hweno_ctx* c, T* state, int nsteps, double t_end, double* t_out, int* steps_out) {
  if (!c || !state || !is_type<T>(c)) return SWE_EINVAL;
  if (!(t_end <= DBL_MAX) || (nsteps <= 0 && !(t_end > 0))) return SWE_EINVAL;
  const int use_tend = t_end > 0 ? 1 : 0;
  if (!c->timing && (c->g_state != state || c->g_tend != use_tend)) {
    destroy_graphs(c);
    int e = capture<T>(c, state, 1, use_tend, &c->g1);
    if (!e) e = capture<T>(c, state, 8, use_tend, &c->g8);
    if (e) { destroy_graphs(c); return e; }
    c->g_state = state;
    c->g_tend = use_tend;
  }
  // t = 0, t_end, steps = 0 and alpha of the initial state
  hipLaunchKernelGGL(k_clock, dim3(1), dim3(64), 0, c->stream, c->sc, t_end);
  launch_alpha<T>(c, state, c->sc->a_next, c->stream);
  if (hipGetLastError() != hipSuccess) return SWE_EHIP;
  int done = 0;
  const int chunk = 64;
  for (;;) {
    int todo = nsteps > 0 ? nsteps - done : chunk;
    if (todo <= 0) break;
    if (use_tend && todo > chunk) todo = chunk;
    int k = 0;
    if (c->timing) {
      for (; k < todo; ++k) enqueue_step<T>(c, state, use_tend, c->stream);
      if (hipGetLastError() != hipSuccess) return SWE_EHIP;
    }
    for (; k + 8 <= todo; k += 8)
      if (hipGraphLaunch(c->g8, c->stream) != hipSuccess) return SWE_EHIP;
    for (; k < todo; ++k)
      if (hipGraphLaunch(c->g1, c->stream) != hipSuccess) return SWE_EHIP;
    done += todo;
    if (use_tend) {
      int active = 0;
      if (hipMemcpyAsync(&active, &c->sc->active, sizeof(int), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        return SWE_EHIP;
      if (hipStreamSynchronize(c->stream) != hipSuccess) return SWE_EHIP;
      if (!active) break;
    }
  }
  double t = 0;
  int steps = 0;
  if (hipMemcpyAsync(&t, &c->sc->t, sizeof t, hipMemcpyDeviceToHost, c->stream) != hipSuccess) return SWE_EHIP;
  if (hipMemcpyAsync(&steps, &c->sc->steps, sizeof steps, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
    return SWE_EHIP;
  const int e = take_device_error(c);
  if (c->timing) collect_timing(c);
  if (t_out) *t_out = t;
  if (steps_out) *steps_out = steps;
  return e;
}

// Device address of `scratch` on the current device, looked up once per device.
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_addr;

int scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return SWE_EHIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it == g_scratch_addr.end()) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return SWE_EHIP;
    it = g_scratch_addr.emplace(dev, ptr).first;
  }
  *out = it->second;
  return SWE_OK;
}

// Bytes of scratch an allocation-free step needs: device scalars, then S1, S2 (nf planes each)
// and D^{n,mod} (nd planes).
size_t noalloc_bytes(const swe_hweno_params* p) {
  const size_t n = (size_t)p->nx * (size_t)(p->dim == 2 ? p->ny : 1);
  const size_t planes = p->dim == 2 ? 2 * 9 + 6 : 2 * 4 + 2;
  return NOALLOC_SCAL + planes * n * sizeof(double);
}

int step_noalloc_impl(const swe_hweno_params* p, double* state, const double* b, const double* bx,
                      const double* by, double dt, void* stream, double* dt_used) {
  if (!params_ok(p) || !state || !b || !bx || (p->dim == 2 && !by)) return SWE_EINVAL;
  if (!(dt <= DBL_MAX)) return SWE_EINVAL;
  if (noalloc_bytes(p) > NOALLOC_BYTES) return SWE_EINVAL;
  void* base = nullptr;
  if (const int e = scratch_address(&base)) return e;
  // a context on the host stack that points into the scratch array and at the caller's bottom
  swe_hweno_ctx c;
  c.p = *p;
  c.stream = (hipStream_t)stream;
  c.nf = p->dim == 2 ? 9 : 4;
  c.nd = p->dim == 2 ? 6 : 2;
  c.n = (size_t)p->nx * (size_t)(p->dim == 2 ? p->ny : 1);
  c.b = (void*)b;
  c.bx = (void*)bx;
  c.by = (void*)by;
  c.sc = (DevScal*)base;
  double* planes = (double*)((char*)base + NOALLOC_SCAL);
  c.S1 = planes;
  c.S2 = planes + (size_t)c.nf * c.n;
  c.Dn = planes + (size_t)2 * c.nf * c.n;
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
        hipSuccess || cus <= 0)
      cus = 256;
    c.rows = choose_rows(p->nx, p->dim == 2 ? p->ny : 1, 4 * cus);
  }
  if (dt > 0) { c.p.flags |= SWE_FIXED_DT; c.p.fixed_dt = dt; }
  hipLaunchKernelGGL(k_noalloc_setup, dim3(1), dim3(64), 0, c.stream, c.sc, dbits(p->alpha_x),
                     dbits(p->dim == 2 ? p->alpha_y : 0.0));
  hipLaunchKernelGGL(k_clock, dim3(1), dim3(64), 0, c.stream, c.sc, 0.0);
  launch_alpha<double>(&c, state, c.sc->a_next, c.stream);
  enqueue_step<double>(&c, state, 0, c.stream);
  if (hipGetLastError() != hipSuccess) return SWE_EHIP;
  if (dt_used) {
    if (hipMemcpyAsync(dt_used, &c.sc->dt, sizeof(double), hipMemcpyDeviceToHost, c.stream) != hipSuccess)
      return SWE_EHIP;
    return take_device_error(&c);
  }
  return SWE_OK;
}

}  // namespace

extern "C" {

int swe_hweno_abi_version(void) { return SWE_HWENO_ABI_VERSION; }

int swe_hweno_tile(int* cols_per_wave, int* rows_per_wave) {
  if (!cols_per_wave || !rows_per_wave) return SWE_EINVAL;
  *cols_per_wave = OUT_COLS;
  *rows_per_wave = ROWS_DEFAULT;
  return SWE_OK;
}

int swe_hweno_ctx_tile(const swe_hweno_ctx* c, int* cols_per_wave, int* rows_per_wave) {
  if (!c || !cols_per_wave || !rows_per_wave) return SWE_EINVAL;
  *cols_per_wave = OUT_COLS;
  *rows_per_wave = c->rows;
  return SWE_OK;
}

const char* swe_hweno_strerror(int code) {
  switch (code) {
    case SWE_OK: return "ok";
    case SWE_EINVAL: return "invalid argument";
    case SWE_ENOMEM: return "device allocation failed";
    case SWE_EHIP: return "HIP runtime error";
    case SWE_EDRY: return "dry node (h <= 0)";
    case SWE_ENONFINITE: return "non-finite value";
    default: return "unknown error";
  }
}

int swe_hweno_init(const swe_hweno_params* p, const double* b, const double* bx, const double* by, void* stream,
                   swe_hweno_ctx** out) {
  return init_impl<double>(p, b, bx, by, stream, out);
}
int swe_hweno_init_f32(const swe_hweno_params* p, const float* b, const float* bx, const float* by, void* stream,
                       swe_hweno_ctx** out) {
  return init_impl<float>(p, b, bx, by, stream, out);
}

void swe_hweno_destroy(swe_hweno_ctx* c) {
  if (!c) return;
  if (c->stream || c->b) (void)hipStreamSynchronize(c->stream);
  destroy_graphs(c);
  collect_timing(c);
  for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  if (c->b) (void)hipFree(c->b);
  if (c->S1) (void)hipFree(c->S1);
  if (c->S2) (void)hipFree(c->S2);
  if (c->Dn) (void)hipFree(c->Dn);
  if (c->sc) (void)hipFree(c->sc);
  swe_adj_release(c);
  delete c;
}

int swe_hweno_rhs(swe_hweno_ctx* c, const double* state, double* rhs, double alpha_x, double alpha_y) {
  return rhs_impl<double>(c, state, rhs, alpha_x, alpha_y);
}
int swe_hweno_rhs_f32(swe_hweno_ctx* c, const float* state, float* rhs, double alpha_x, double alpha_y) {
  return rhs_impl<float>(c, state, rhs, alpha_x, alpha_y);
}

int swe_hweno_limit(swe_hweno_ctx* c, const double* state, double* dmod) { return limit_impl<double>(c, state, dmod); }
int swe_hweno_limit_f32(swe_hweno_ctx* c, const float* state, float* dmod) { return limit_impl<float>(c, state, dmod); }

int swe_hweno_alpha(swe_hweno_ctx* c, const double* state, double* alpha_host) {
  return alpha_impl<double>(c, state, alpha_host);
}
int swe_hweno_alpha_f32(swe_hweno_ctx* c, const float* state, double* alpha_host) {
  return alpha_impl<float>(c, state, alpha_host);
}

int swe_hweno_step(swe_hweno_ctx* c, double* state, double dt, double* dt_used) {
  return step_impl<double>(c, state, dt, dt_used);
}
int swe_hweno_step_f32(swe_hweno_ctx* c, float* state, double dt, double* dt_used) {
  return step_impl<float>(c, state, dt, dt_used);
}

int swe_hweno_run(swe_hweno_ctx* c, double* state, int nsteps, double t_end, double* t_out, int* steps_out) {
  return run_impl<double>(c, state, nsteps, t_end, t_out, steps_out);
}
int swe_hweno_run_f32(swe_hweno_ctx* c, float* state, int nsteps, double t_end, double* t_out, int* steps_out) {
  return run_impl<float>(c, state, nsteps, t_end, t_out, steps_out);
}

int swe_hweno_set_timing(swe_hweno_ctx* c, int on) {
  if (!c) return SWE_EINVAL;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return SWE_EHIP;
  collect_timing(c);
  c->timing = on != 0;
  for (int k = 0; k < 4; ++k) { c->ms[k] = 0; c->launches[k] = 0; }
  return SWE_OK;
}

int swe_hweno_get_timing(swe_hweno_ctx* c, double* ms, long long* launches) {
  if (!c || !ms || !launches) return SWE_EINVAL;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return SWE_EHIP;
  collect_timing(c);
  for (int k = 0; k < 4; ++k) { ms[k] = c->ms[k]; launches[k] = c->launches[k]; }
  return SWE_OK;
}

int swe_hweno_step_noalloc(const swe_hweno_params* params, double* state, const double* b, const double* bx,
                           const double* by, double dt, void* stream, double* dt_used) {
  return step_noalloc_impl(params, state, b, bx, by, dt, stream, dt_used);
}

unsigned long swe_hweno_noalloc_capacity(void) { return (unsigned long)NOALLOC_BYTES; }

int swe_hweno_math_check(int which, const double* x, double* y, unsigned long n, void* stream) {
  if (which < 0 || which > 2 || !x || !y || n == 0) return SWE_EINVAL;
  const size_t blocks = (n + 255) / 256;
  const unsigned grid = (unsigned)(blocks < 8192 ? blocks : 8192);
  hipLaunchKernelGGL(k_math_check, dim3(grid), dim3(256), 0, (hipStream_t)stream, which, x, y, (size_t)n);
  if (hipGetLastError() != hipSuccess) return SWE_EHIP;
  return hip_status(hipStreamSynchronize((hipStream_t)stream));
}

#ifndef SWE_HWENO_SOURCE_HASH
#define SWE_HWENO_SOURCE_HASH "unstamped"
#endif
const char* swe_hweno_source_hash(void) { return SWE_HWENO_SOURCE_HASH; }

int swe_hweno_sync(swe_hweno_ctx* c) {
  if (!c) return SWE_EINVAL;
  return take_device_error(c);
}

}  // extern "C"

#include "swe_hweno_batch.inc"
#include "swe_hweno_adjoint.inc"
