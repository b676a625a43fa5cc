// Broken-line fit of one track and its adjoint (paper section 3.4).
//
// One thread per track, everything in registers: N (the number of hits) is a
// template parameter so that every per-hit array is unrolled.  The fit is
// formulated relative to the first hit:
//   * pre-fit: the circle through hits 0, N/2 and N-1, written as its
//     curvature kp and its unit tangent (tx, ty) at hit 0, computed from the
//     two chords without ever forming the centre (which runs off to infinity
//     for stiff tracks);
//   * every hit in the frame (tangent, normal) at hit 0: arc length
//     s = atan2(kp xt, 1 - kp xn) / kp and left offset
//     u = A / (1 + sqrt(1 - kp A)), A = 2 xn - kp (xt^2 + xn^2), both free of
//     cancellation as kp -> 0;
//   * the S-Z fit solves for the deviation w_k from the pre-fit line
//     z = z_0 + t s, so the unknowns are small numbers;
//   * both broken-line systems are banded (bandwidth 2, plus the curvature
//     border in the transverse one) and factorised by a band Cholesky;
//   * the perigee conversion is done in double.
// Positions relative to hit 0 and their frame coordinates are formed in
// double whatever the fit precision S, because that is where single precision
// would lose the sagitta to cancellation.
//
// The adjoint recomputes the forward pass and sweeps it backwards.  The two
// linear solves are differentiated with the usual identity for a minimum of a
// quadratic: with lambda = M^-1 xbar, every parameter theta of the system
// receives d/dtheta of sum_i w_i (gchi2 e_i^2 + e_i (a_i . lambda)) at fixed
// solution x, where e_i = m_i - a_i . x are the residuals (measurements and
// kinks) of chi^2 = sum_i w_i e_i^2.
#pragma once

#include <cmath>
#include <cstdint>

#ifdef __HIPCC__
#define PT_HD __host__ __device__
#else
#define PT_HD
#endif

namespace pt {
namespace fit {

PT_HD inline float m_sqrt(float x) { return sqrtf(x); }
PT_HD inline double m_sqrt(double x) { return sqrt(x); }
PT_HD inline float m_atan2(float y, float x) { return atan2f(y, x); }
PT_HD inline double m_atan2(double y, double x) { return atan2(y, x); }
PT_HD inline float m_log(float x) { return logf(x); }
PT_HD inline double m_log(double x) { return log(x); }
PT_HD inline float m_abs(float x) { return fabsf(x); }
PT_HD inline double m_abs(double x) { return fabs(x); }
PT_HD inline bool m_finite(double x) { return __builtin_isfinite(x); }

struct Consts {
  double K;         // p_T = K / |kappa|
  double x0;        // material per crossing (X/X0)
  double ha, hb;    // Highland constants
  double VT;        // transverse measurement variance
  double VZb;       // barrel longitudinal variance
  double VRd;       // disk radial variance
  double pcap;      // momentum cap
  double thr;       // conditioning threshold for the double-precision refit
};

enum { ST_OK = 0, ST_BAD_ORDER = 1, ST_F64 = 2, ST_FAILED = 4 };

// SPD band system: unknowns 0..NB-1 couple within bandwidth 2; with BORDER an
// extra unknown NB couples with all.  Matrix given by its lower band.
template <int NB, bool BORDER, class T>
struct Band {
  static constexpr int M = NB + (BORDER ? 1 : 0);
  T d[M];      // diagonal of the Cholesky factor L
  T e1[NB];    // L[i+1][i]
  T e2[NB];    // L[i+2][i]
  T bd[NB];    // L[NB][i]
  bool ok;

  // diag[i] = A[i][i], off1[i] = A[i+1][i], off2[i] = A[i+2][i], brow[i] = A[NB][i]
  PT_HD void factor(const T* diag, const T* off1, const T* off2, const T* brow, T bdiag) {
    ok = true;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      T s = diag[i];
      if (i >= 1) s -= e1[i - 1] * e1[i - 1];
      if (i >= 2) s -= e2[i - 2] * e2[i - 2];
      if (!(s > T(0))) ok = false;
      d[i] = m_sqrt(s);
      const T inv = T(1) / d[i];
      if (i + 1 < NB) {
        T v = off1[i];
        if (i >= 1) v -= e2[i - 1] * e1[i - 1];
        e1[i] = v * inv;
      } else {
        e1[i] = T(0);
      }
      e2[i] = (i + 2 < NB) ? off2[i] * inv : T(0);
      if constexpr (BORDER) {
        T v = brow[i];
        if (i >= 1) v -= bd[i - 1] * e1[i - 1];
        if (i >= 2) v -= bd[i - 2] * e2[i - 2];
        bd[i] = v * inv;
      } else {
        bd[i] = T(0);
      }
    }
    if constexpr (BORDER) {
      T s = bdiag;
#pragma unroll
      for (int i = 0; i < NB; ++i) s -= bd[i] * bd[i];
      if (!(s > T(0))) ok = false;
      d[M - 1] = m_sqrt(s);
    }
  }

  // x <- A^-1 x
  PT_HD void solve(T* x) const {
    T y[M];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      T v = x[i];
      if (i >= 1) v -= e1[i - 1] * y[i - 1];
      if (i >= 2) v -= e2[i - 2] * y[i - 2];
      y[i] = v / d[i];
    }
    if constexpr (BORDER) {
      T v = x[NB];
#pragma unroll
      for (int i = 0; i < NB; ++i) v -= bd[i] * y[i];
      y[NB] = v / d[NB];
      x[NB] = y[NB] / d[NB];
    }
#pragma unroll
    for (int i = NB - 1; i >= 0; --i) {
      T v = y[i];
      if (i + 1 < NB) v -= e1[i] * x[i + 1];
      if (i + 2 < NB) v -= e2[i] * x[i + 2];
      if constexpr (BORDER) v -= bd[i] * x[NB];
      x[i] = v / d[i];
    }
  }
};

template <int N, class S>
struct State {
  // inputs: hit 0 absolute, others relative to it (double)
  double P0x, P0y, P0z;
  double rx[N], ry[N], rz[N];
  bool barrel[N];
  // pre-fit circle, in double in both precisions: it is the linearisation
  // point of the fit, and an error in it leaks into the fitted curvature of
  // tracks far from it
  double ax, ay, bx, by, cr, la, lb, ld, kp, ux, uy, sb, cb, tx, ty;
  // per hit
  S xt[N], xn[N], s[N], A[N], sq[N], u[N], m[N], wZm[N];
  double sd[N];  // arc lengths in double (the S-Z residuals and the spacings need them)
  S D[N - 1];
  // slope and momentum
  S t, sec2, pT, p;
  bool capped;
  // scattering at inner hits j = 1..N-2 (index j)
  S path[N], Xm[N], lg[N], th2[N], wT[N], wZ[N];
  // solves
  Band<N, true, S> circ;
  Band<N, false, S> line;
  S xc[N + 1];  // fitted offsets u_0..u_{N-1} and curvature correction
  S wl[N];      // fitted deviations from the pre-fit line
  S eu[N], ez[N];      // measurement residuals at the optimum
  S beta[N], gam[N];   // kinks at the inner hits (index j = 1..N-2)
  S chi2;
  S cond;       // conditioning estimate of the transverse system
  // perigee (double)
  double kappa, Qx, Qy, dk, du0, ca, sa, cpsi, spsi, U, sqU, d0, hx, hy, phi0, hn, cph, sph, at, an;
  double Ys, Xs, ds, cot, z0;
  int status;
};

template <int N, class S>
PT_HD inline void forward(const Consts& C, State<N, S>& f) {
  constexpr int b = N / 2;
  f.status = ST_OK;
  // ---- pre-fit circle through hits 0, b, N-1
  f.ax = f.rx[b];
  f.ay = f.ry[b];
  f.bx = f.rx[N - 1];
  f.by = f.ry[N - 1];
  f.cr = f.ax * f.by - f.ay * f.bx;
  f.la = m_sqrt(f.ax * f.ax + f.ay * f.ay);
  f.lb = m_sqrt(f.bx * f.bx + f.by * f.by);
  const double dx = f.bx - f.ax, dy = f.by - f.ay;
  f.ld = m_sqrt(dx * dx + dy * dy);
  f.kp = 2.0 * f.cr / (f.la * f.lb * f.ld);
  f.ux = f.bx / f.lb;
  f.uy = f.by / f.lb;
  f.sb = f.kp * f.lb * 0.5;
  const double c2 = 1.0 - f.sb * f.sb;
  f.cb = m_sqrt(c2 > 0.0 ? c2 : 0.0);
  f.tx = f.ux * f.cb + f.uy * f.sb;
  f.ty = -f.ux * f.sb + f.uy * f.cb;
  // ---- hits in the frame (tangent, normal) at hit 0
  const double tx = double(f.tx), ty = double(f.ty);
  f.xt[0] = f.xn[0] = f.s[0] = f.A[0] = f.u[0] = f.m[0] = S(0);
  f.sd[0] = 0.0;
  f.sq[0] = S(1);
#pragma unroll
  for (int k = 1; k < N; ++k) {
    const double xtd = tx * f.rx[k] + ty * f.ry[k];
    const double xnd = -ty * f.rx[k] + tx * f.ry[k];
    const S xt = S(xtd), xn = S(xnd);
    f.xt[k] = xt;
    f.xn[k] = xn;
    f.sd[k] = (f.kp != S(0)) ? atan2(double(f.kp) * xtd, 1.0 - double(f.kp) * xnd) / double(f.kp) : xtd;
    f.s[k] = S(f.sd[k]);
    // A is a small difference of two terms of the size of the sagitta: double
    f.A[k] = S(2.0 * xnd - double(f.kp) * (xtd * xtd + xnd * xnd));
    const S q = S(1) - f.kp * f.A[k];
    f.sq[k] = m_sqrt(q > S(0) ? q : S(0));
    f.u[k] = f.A[k] / (S(1) + f.sq[k]);
  }
#pragma unroll
  for (int k = 0; k + 1 < N; ++k) {
    f.D[k] = S(f.sd[k + 1] - f.sd[k]);
    if (!(f.D[k] > S(0))) f.status = ST_BAD_ORDER;
  }
  if (f.status != ST_OK) return;
  // ---- slope and momentum
  f.t = S(f.rz[N - 1]) / f.s[N - 1];
  f.sec2 = S(1) + f.t * f.t;
  if (f.kp != S(0)) {
    f.pT = S(C.K) / m_abs(f.kp);
    const S pp = f.pT * m_sqrt(f.sec2);
    f.capped = !(pp < S(C.pcap));
    f.p = f.capped ? S(C.pcap) : pp;
  } else {
    f.pT = S(0);
    f.capped = true;
    f.p = S(C.pcap);
  }
  // ---- multiple scattering at the inner hits
  const S sqs = m_sqrt(f.sec2);
  const S th0 = S(C.ha) / f.p;
#pragma unroll
  for (int j = 1; j + 1 < N; ++j) {
    f.path[j] = f.barrel[j] ? sqs : sqs / m_abs(f.t);
    f.Xm[j] = S(C.x0) * f.path[j];
    f.lg[j] = S(1) + S(C.hb) * m_log(f.Xm[j]);
    f.th2[j] = th0 * th0 * f.Xm[j] * f.lg[j] * f.lg[j];
    f.wT[j] = S(1) / (f.th2[j] * f.sec2);
    f.wZ[j] = S(1) / (f.th2[j] * f.sec2 * f.sec2);
  }
  // ---- longitudinal measurements relative to the pre-fit line
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const S VZ = f.barrel[k] ? S(C.VZb) : S(C.VRd) * f.t * f.t;
    f.wZm[k] = S(1) / VZ;
    if (k > 0) f.m[k] = S(f.rz[k] - double(f.t) * f.sd[k]);
  }
  // ---- transverse broken line: unknowns u_0..u_{N-1}, dk
  const S wm = S(1) / S(C.VT);
  S diag[N], off1[N], off2[N], brow[N], bdiag = S(0);
  S ldiag[N], loff1[N], loff2[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    diag[k] = wm;
    off1[k] = off2[k] = brow[k] = S(0);
    ldiag[k] = f.wZm[k];
    loff1[k] = loff2[k] = S(0);
  }
  f.cond = S(0);
#pragma unroll
  for (int j = 1; j + 1 < N; ++j) {
    const S cm = S(1) / f.D[j - 1], cp = S(1) / f.D[j];
    const S c0 = -(cm + cp);
    const S ck = -(f.D[j - 1] + f.D[j]) * S(0.5);
    const S w = f.wT[j];
    diag[j - 1] += w * cm * cm;
    diag[j] += w * c0 * c0;
    diag[j + 1] += w * cp * cp;
    off1[j - 1] += w * c0 * cm;
    off1[j] += w * cp * c0;
    off2[j - 1] += w * cp * cm;
    brow[j - 1] += w * ck * cm;
    brow[j] += w * ck * c0;
    brow[j + 1] += w * ck * cp;
    bdiag += w * ck * ck;
    const S e = w * (cm + cp) * (cm + cp) * S(C.VT);
    if (e > f.cond) f.cond = e;
    const S v = f.wZ[j];
    ldiag[j - 1] += v * cm * cm;
    ldiag[j] += v * c0 * c0;
    ldiag[j + 1] += v * cp * cp;
    loff1[j - 1] += v * c0 * cm;
    loff1[j] += v * cp * c0;
    loff2[j - 1] += v * cp * cm;
  }
  f.circ.factor(diag, off1, off2, brow, bdiag);
  f.line.factor(ldiag, loff1, loff2, nullptr, S(0));
  if (!f.circ.ok || !f.line.ok) {
    f.status = ST_FAILED;
    return;
  }
#pragma unroll
  for (int k = 0; k < N; ++k) {
    f.xc[k] = f.u[k] * wm;
    f.wl[k] = f.m[k] * f.wZm[k];
  }
  f.xc[N] = S(0);
  f.circ.solve(f.xc);
  f.line.solve(f.wl);
  if constexpr (sizeof(S) < sizeof(double)) {
    // One step of iterative refinement: the residual of the normal equations
    // is formed in double, applying the matrix from its definition (weights
    // times kinks of the current solution, coefficients from the double arc
    // lengths), and corrected with the single-precision Cholesky factor.  The
    // float solve alone is limited by the rounding of the assembled matrix,
    // which shows on badly fitting combinations whose curvature correction
    // nearly cancels the pre-fit curvature.
    double rcd[N + 1], rld[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      rcd[i] = double(f.u[i]) * double(wm) - double(wm) * double(f.xc[i]);
      rld[i] = double(f.m[i]) * double(f.wZm[i]) - double(f.wZm[i]) * double(f.wl[i]);
    }
    rcd[N] = 0.0;
#pragma unroll
    for (int j = 1; j + 1 < N; ++j) {
      const double dm = f.sd[j] - f.sd[j - 1], dp = f.sd[j + 1] - f.sd[j];
      const double cm = 1.0 / dm, cp = 1.0 / dp, c0 = -(cm + cp), ck = -(dm + dp) * 0.5;
      const double bt = cm * double(f.xc[j - 1]) + c0 * double(f.xc[j]) + cp * double(f.xc[j + 1]) +
                        ck * double(f.xc[N]);
      const double gm = cm * double(f.wl[j - 1]) + c0 * double(f.wl[j]) + cp * double(f.wl[j + 1]);
      const double wb = double(f.wT[j]) * bt, wg = double(f.wZ[j]) * gm;
      rcd[j - 1] -= wb * cm;
      rcd[j] -= wb * c0;
      rcd[j + 1] -= wb * cp;
      rcd[N] -= wb * ck;
      rld[j - 1] -= wg * cm;
      rld[j] -= wg * c0;
      rld[j + 1] -= wg * cp;
    }
    S rc[N + 1], rl[N];
#pragma unroll
    for (int i = 0; i <= N; ++i) rc[i] = S(rcd[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) rl[i] = S(rld[i]);
    f.circ.solve(rc);
    f.line.solve(rl);
#pragma unroll
    for (int i = 0; i <= N; ++i) f.xc[i] = S(double(f.xc[i]) + double(rc[i]));
#pragma unroll
    for (int i = 0; i < N; ++i) f.wl[i] = S(double(f.wl[i]) + double(rl[i]));
  }
  // ---- residuals and chi^2 at the optimum.  The kinks are formed from the
  // solution; the measurement residuals come from the normal equations,
  // e_k = V_k (B^T W kinks)_k, which holds at the optimum and, unlike
  // u_k - x_k, does not cancel when the scattering weights are small and the
  // fit follows the measurements closely.
#pragma unroll
  for (int k = 0; k < N; ++k) {
    f.eu[k] = S(0);
    f.ez[k] = S(0);
    f.beta[k] = S(0);
    f.gam[k] = S(0);
  }
#pragma unroll
  for (int j = 1; j + 1 < N; ++j) {
    const S cm = S(1) / f.D[j - 1], cp = S(1) / f.D[j];
    const S c0 = -(cm + cp);
    const S ck = -(f.D[j - 1] + f.D[j]) * S(0.5);
    f.beta[j] = cm * f.xc[j - 1] + c0 * f.xc[j] + cp * f.xc[j + 1] + ck * f.xc[N];
    f.gam[j] = cm * f.wl[j - 1] + c0 * f.wl[j] + cp * f.wl[j + 1];
    const S wb = f.wT[j] * f.beta[j];
    const S wg = f.wZ[j] * f.gam[j];
    f.eu[j - 1] += wb * cm;
    f.eu[j] += wb * c0;
    f.eu[j + 1] += wb * cp;
    f.ez[j - 1] += wg * cm;
    f.ez[j] += wg * c0;
    f.ez[j + 1] += wg * cp;
  }
  S chi = S(0);
#pragma unroll
  for (int k = 0; k < N; ++k) {
    f.eu[k] *= S(C.VT);
    f.ez[k] /= f.wZm[k];
    chi += f.eu[k] * f.eu[k] * wm + f.ez[k] * f.ez[k] * f.wZm[k];
  }
#pragma unroll
  for (int j = 1; j + 1 < N; ++j) chi += f.wT[j] * f.beta[j] * f.beta[j] + f.wZ[j] * f.gam[j] * f.gam[j];
  f.chi2 = chi;
  // ---- perigee parameters (double), with the pre-fit tangent renormalised
  const double tn = sqrt(tx * tx + ty * ty);
  const double ex = tx / tn, ey = ty / tn;
  const double D0 = double(f.D[0]);
  const double u0 = double(f.xc[0]), u1 = double(f.xc[1]);
  f.dk = double(f.xc[N]);
  f.kappa = double(f.kp) + f.dk;
  f.Qx = f.P0x - u0 * ey;
  f.Qy = f.P0y + u0 * ex;
  f.du0 = (u1 - u0) / D0 - f.dk * D0 * 0.5;
  f.ca = 1.0 / sqrt(1.0 + f.du0 * f.du0);
  f.sa = f.du0 * f.ca;
  f.cpsi = ex * f.ca - ey * f.sa;
  f.spsi = ey * f.ca + ex * f.sa;
  f.U = f.kappa * (f.Qx * f.Qx + f.Qy * f.Qy) + 2.0 * (-f.Qx * f.spsi + f.Qy * f.cpsi);
  f.sqU = sqrt(1.0 + f.kappa * f.U);
  f.d0 = f.U / (1.0 + f.sqU);
  f.hx = f.cpsi + f.kappa * f.Qy;
  f.hy = f.spsi - f.kappa * f.Qx;
  f.phi0 = atan2(f.hy, f.hx);
  f.hn = sqrt(f.hx * f.hx + f.hy * f.hy);
  f.cph = f.hx / f.hn;
  f.sph = f.hy / f.hn;
  f.at = f.Qx * f.cph + f.Qy * f.sph;
  f.an = -f.Qx * f.sph + f.Qy * f.cph;
  if (f.kappa != 0.0) {
    f.Ys = f.kappa * f.at;
    f.Xs = 1.0 + f.kappa * (f.d0 - f.an);
    f.ds = atan2(f.Ys, f.Xs) / f.kappa;
  } else {
    f.Ys = 0.0;
    f.Xs = 1.0;
    f.ds = f.at;
  }
  f.cot = double(f.t) + (double(f.wl[1]) - double(f.wl[0])) / D0;
  f.z0 = f.P0z + double(f.wl[0]) - f.cot * f.ds;
  if (!m_finite(f.kappa) || !m_finite(f.phi0) || !m_finite(f.d0) || !m_finite(f.z0) ||
      !m_finite(f.cot) || !m_finite(double(f.chi2)))
    f.status = ST_FAILED;
}

// Reverse sweep of the perigee conversion alone: with g = d(loss)/d(kappa,
// phi0, cot, d0, z0), the derivatives of the loss with respect to what the
// conversion reads -- the first hit, the fitted offsets u0, u1 and curvature
// correction dk of the circle fit, the fitted deviations w0, w1 of the line
// fit, the pre-fit slope t, spacing D0, tangent (tx, ty) and curvature kp.
struct PerigeeBar {
  double P0x, P0y, P0z, wl0, wl1, t, D0, u0, u1, dk, tx, ty, kp;
};

template <int N, class S>
PT_HD inline void perigee_vjp(const State<N, S>& f, const double g[5], PerigeeBar& o) {
  const double tx = double(f.tx), ty = double(f.ty);
  const double tn = sqrt(tx * tx + ty * ty);
  const double ex = tx / tn, ey = ty / tn;
  const double D0 = double(f.D[0]);
  const double u0 = double(f.xc[0]), u1 = double(f.xc[1]);
  double kappa_b = g[0], phi0_b = g[1], cot_b = g[2], d0_b = g[3], z0_b = g[4];
  double P0x_b = 0, P0y_b = 0, P0z_b = 0, wl0_b = 0, wl1_b = 0, t_bd = 0, D0_b = 0;
  double Qx_b = 0, Qy_b = 0, cph_b = 0, sph_b = 0, ex_b = 0, ey_b = 0;
  // z0 = P0z + wl0 - cot ds
  P0z_b += z0_b;
  wl0_b += z0_b;
  cot_b += -z0_b * f.ds;
  const double ds_b = -z0_b * f.cot;
  // cot = t + (wl1 - wl0) / D0
  t_bd += cot_b;
  wl1_b += cot_b / D0;
  wl0_b -= cot_b / D0;
  D0_b += -cot_b * (double(f.wl[1]) - double(f.wl[0])) / (D0 * D0);
  // ds
  double at_b = 0, an_b = 0;
  if (f.kappa != 0.0) {
    const double ang_b = ds_b / f.kappa;
    kappa_b += -ds_b * f.ds / f.kappa;
    const double r2 = f.Xs * f.Xs + f.Ys * f.Ys;
    const double Ys_b = ang_b * f.Xs / r2;
    const double Xs_b = -ang_b * f.Ys / r2;
    kappa_b += Ys_b * f.at + Xs_b * (f.d0 - f.an);
    at_b += Ys_b * f.kappa;
    d0_b += Xs_b * f.kappa;
    an_b -= Xs_b * f.kappa;
  } else {
    at_b += ds_b;
    kappa_b += -ds_b * f.at * (f.d0 - f.an);
  }
  // at = Qx cph + Qy sph, an = -Qx sph + Qy cph
  Qx_b += at_b * f.cph - an_b * f.sph;
  Qy_b += at_b * f.sph + an_b * f.cph;
  cph_b += at_b * f.Qx + an_b * f.Qy;
  sph_b += at_b * f.Qy - an_b * f.Qx;
  // (cph, sph) = (cos, sin) of phi0 = atan2(hy, hx)
  const double phi_b = phi0_b - f.sph * cph_b + f.cph * sph_b;
  const double hn2 = f.hn * f.hn;
  const double hx_b = -phi_b * f.hy / hn2;
  const double hy_b = phi_b * f.hx / hn2;
  // hx = cpsi + kappa Qy, hy = spsi - kappa Qx
  double cpsi_b = hx_b, spsi_b = hy_b;
  kappa_b += hx_b * f.Qy - hy_b * f.Qx;
  Qy_b += hx_b * f.kappa;
  Qx_b -= hy_b * f.kappa;
  // d0 = U / (1 + sqU), sqU = sqrt(1 + kappa U)
  {
    const double den = 1.0 + f.sqU;
    const double U_b = d0_b * (1.0 / den - f.U * f.kappa / (2.0 * f.sqU * den * den));
    kappa_b += d0_b * (-f.U * f.U / (2.0 * f.sqU * den * den));
    // U = kappa (Qx^2 + Qy^2) + 2 (-Qx spsi + Qy cpsi)
    kappa_b += U_b * (f.Qx * f.Qx + f.Qy * f.Qy);
    Qx_b += U_b * (2.0 * f.kappa * f.Qx - 2.0 * f.spsi);
    Qy_b += U_b * (2.0 * f.kappa * f.Qy + 2.0 * f.cpsi);
    spsi_b += -2.0 * U_b * f.Qx;
    cpsi_b += 2.0 * U_b * f.Qy;
  }
  // cpsi = tx ca - ty sa, spsi = ty ca + tx sa
  ex_b += cpsi_b * f.ca + spsi_b * f.sa;
  ey_b += -cpsi_b * f.sa + spsi_b * f.ca;
  const double ca_b = cpsi_b * ex + spsi_b * ey;
  const double sa_b = -cpsi_b * ey + spsi_b * ex;
  // ca = (1 + du0^2)^-1/2, sa = du0 ca
  const double du0_b = f.ca * f.ca * f.ca * (sa_b - f.du0 * ca_b);
  // du0 = (u1 - u0) / D0 - dk D0 / 2
  double xu0_b = -du0_b / D0, xu1_b = du0_b / D0;
  double dk_b = -du0_b * D0 * 0.5;
  D0_b += -du0_b * (u1 - u0) / (D0 * D0) - du0_b * f.dk * 0.5;
  // Qx = P0x - u0 ty, Qy = P0y + u0 tx
  P0x_b += Qx_b;
  P0y_b += Qy_b;
  xu0_b += -Qx_b * ey + Qy_b * ex;
  ey_b += -Qx_b * u0;
  ex_b += Qy_b * u0;
  // (ex, ey) = (tx, ty) / |(tx, ty)|
  const double edot = ex * ex_b + ey * ey_b;
  const double tx_bd = (ex_b - ex * edot) / tn;
  const double ty_bd = (ey_b - ey * edot) / tn;
  // kappa = kp + dk
  double kp_bd = kappa_b;
  dk_b += kappa_b;

  o.P0x = P0x_b;
  o.P0y = P0y_b;
  o.P0z = P0z_b;
  o.wl0 = wl0_b;
  o.wl1 = wl1_b;
  o.t = t_bd;
  o.D0 = D0_b;
  o.u0 = xu0_b;
  o.u1 = xu1_b;
  o.dk = dk_b;
  o.tx = tx_bd;
  o.ty = ty_bd;
  o.kp = kp_bd;
}

// Covariance of (kappa, phi0, cot, d0, z0), the upper triangle row by row in
// cov[15].  The broken-line solutions are linear in the measurements, the
// kinks being zero-mean pseudo-measurements, so the covariance of the circle
// unknowns is the inverse of its normal matrix and that of the line unknowns
// the inverse of its own; the two fits share no measurement.  The perigee
// conversion reads the circle solution only through (u0, u1, dk) and the
// line solution only through (w0, w1), so with Sc and Sl the inverses
// restricted to those unknowns (columns from solves with the Cholesky
// factors) and Jc, Jl the derivatives of the conversion (rows from
// perigee_vjp with unit cotangents), C = Jc Sc Jc^T + Jl Sl Jl^T.  The pre-fit
// is held fixed (it is the point the fit is linearised around).
template <int N, class S>
PT_HD inline void covariance(const State<N, S>& f, double cov[15]) {
  double jc[5][3], jl[5][2];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    double g[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    g[q] = 1.0;
    PerigeeBar pb;
    perigee_vjp<N, S>(f, g, pb);
    jc[q][0] = pb.u0;
    jc[q][1] = pb.u1;
    jc[q][2] = pb.dk;
    jl[q][0] = pb.wl0;
    jl[q][1] = pb.wl1;
  }
  const int ic[3] = {0, 1, N};
  double sc[3][3], sl[2][2];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    S e[N + 1];
#pragma unroll
    for (int i = 0; i <= N; ++i) e[i] = S(0);
    e[ic[j]] = S(1);
    f.circ.solve(e);
#pragma unroll
    for (int i = 0; i < 3; ++i) sc[i][j] = double(e[ic[i]]);
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    S e[N];
#pragma unroll
    for (int i = 0; i < N; ++i) e[i] = S(0);
    e[j] = S(1);
    f.line.solve(e);
    sl[0][j] = double(e[0]);
    sl[1][j] = double(e[1]);
  }
  int q = 0;
#pragma unroll
  for (int a = 0; a < 5; ++a) {
#pragma unroll
    for (int b = a; b < 5; ++b) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) s += jc[a][i] * 0.5 * (sc[i][j] + sc[j][i]) * jc[b][j];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) s += jl[a][i] * 0.5 * (sl[i][j] + sl[j][i]) * jl[b][j];
      cov[q++] = s;
    }
  }
}

// Reverse sweep.  g = d(loss)/d(kappa, phi0, cot, d0, z0, chi2).  On return
// gP[k][c] = d(loss)/d(coordinate c of hit k).
template <int N, class S>
PT_HD inline void backward(const Consts& C, const State<N, S>& f, const double g[6], S gP[N][3]) {
  constexpr int b = N / 2;
  PerigeeBar pb;
  perigee_vjp<N, S>(f, g, pb);
  const double P0x_b = pb.P0x, P0y_b = pb.P0y, P0z_b = pb.P0z, wl0_b = pb.wl0, wl1_b = pb.wl1;
  const double t_bd = pb.t, D0_b = pb.D0, xu0_b = pb.u0, xu1_b = pb.u1, dk_b = pb.dk;
  const double tx_bd = pb.tx, ty_bd = pb.ty, kp_bd = pb.kp;

  // ---------------- the two solves
  const S G2 = S(g[5]);
  S lam[N + 1], mu[N];
#pragma unroll
  for (int k = 0; k <= N; ++k) lam[k] = S(0);
#pragma unroll
  for (int k = 0; k < N; ++k) mu[k] = S(0);
  lam[0] = S(xu0_b);
  lam[1] = S(xu1_b);
  lam[N] = S(dk_b);
  mu[0] = S(wl0_b);
  mu[1] = S(wl1_b);
  f.circ.solve(lam);
  f.line.solve(mu);

  S u_b[N], m_b[N], s_b[N], D_b[N - 1], wZm_b[N], wT_b[N], wZ_b[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    u_b[k] = m_b[k] = s_b[k] = wZm_b[k] = wT_b[k] = wZ_b[k] = S(0);
    if (k + 1 < N) D_b[k] = S(0);
  }
  D_b[0] += S(D0_b);
  S t_b = S(t_bd);
  const S wm = S(1) / S(C.VT);
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const S eu = f.eu[k];
    u_b[k] += wm * (S(2) * G2 * eu + lam[k]);
    const S ez = f.ez[k];
    m_b[k] += f.wZm[k] * (S(2) * G2 * ez + mu[k]);
    wZm_b[k] += G2 * ez * ez + ez * mu[k];
  }
#pragma unroll
  for (int j = 1; j + 1 < N; ++j) {
    const S cm = S(1) / f.D[j - 1], cp = S(1) / f.D[j];
    const S c0 = -(cm + cp);
    const S ck = -(f.D[j - 1] + f.D[j]) * S(0.5);
    {
      const S beta = f.beta[j];
      const S del = cm * lam[j - 1] + c0 * lam[j] + cp * lam[j + 1] + ck * lam[N];
      wT_b[j] += G2 * beta * beta - beta * del;
      const S coef = f.wT[j] * (S(2) * G2 * beta - del);
      const S gl = -f.wT[j] * beta;
      const S gm = coef * f.xc[j - 1] + gl * lam[j - 1];
      const S g0 = coef * f.xc[j] + gl * lam[j];
      const S gp = coef * f.xc[j + 1] + gl * lam[j + 1];
      const S gk = coef * f.xc[N] + gl * lam[N];
      const S cm_b = gm - g0, cp_b = gp - g0;
      D_b[j - 1] += -cm_b * cm * cm - gk * S(0.5);
      D_b[j] += -cp_b * cp * cp - gk * S(0.5);
    }
    {
      const S gam = f.gam[j];
      const S del = cm * mu[j - 1] + c0 * mu[j] + cp * mu[j + 1];
      wZ_b[j] += G2 * gam * gam - gam * del;
      const S coef = f.wZ[j] * (S(2) * G2 * gam - del);
      const S gl = -f.wZ[j] * gam;
      const S gm = coef * f.wl[j - 1] + gl * mu[j - 1];
      const S g0 = coef * f.wl[j] + gl * mu[j];
      const S gp = coef * f.wl[j + 1] + gl * mu[j + 1];
      D_b[j - 1] += -(gm - g0) * cm * cm;
      D_b[j] += -(gp - g0) * cp * cp;
    }
  }

  // ---------------- measurements, scattering, slope, momentum
  S sec2_b = S(0), p_b = S(0);
#pragma unroll
  for (int k = 0; k < N; ++k) {
    if (!f.barrel[k]) {  // wZm = 1 / (VRd t^2)
      t_b += wZm_b[k] * (S(-2) * f.wZm[k] / f.t);
    }
  }
#pragma unroll
  for (int j = 1; j + 1 < N; ++j) {
    S th2_b = -wT_b[j] * f.wT[j] / f.th2[j] - wZ_b[j] * f.wZ[j] / f.th2[j];
    sec2_b += -wT_b[j] * f.wT[j] / f.sec2 - S(2) * wZ_b[j] * f.wZ[j] / f.sec2;
    p_b += th2_b * (S(-2) * f.th2[j] / f.p);
    const S Xm_b = th2_b * (f.th2[j] / f.Xm[j]) * (S(1) + S(2) * S(C.hb) / f.lg[j]);
    const S path_b = Xm_b * S(C.x0);
    sec2_b += path_b * f.path[j] / (S(2) * f.sec2);
    if (!f.barrel[j]) t_b += path_b * (-f.path[j] / f.t);
  }
  S kp_b = S(kp_bd);
  if (!f.capped) {
    const S sqs = m_sqrt(f.sec2);
    const S pT_b = p_b * sqs;
    sec2_b += p_b * f.pT / (S(2) * sqs);
    kp_b += pT_b * (-f.pT / f.kp);
  }
  // m_k = rz_k - t s_k
  S rz_b[N];
#pragma unroll
  for (int k = 0; k < N; ++k) rz_b[k] = S(0);
#pragma unroll
  for (int k = 1; k < N; ++k) {
    rz_b[k] += m_b[k];
    t_b += -m_b[k] * f.s[k];
    s_b[k] += -m_b[k] * f.t;
  }
  t_b += sec2_b * S(2) * f.t;
  // t = rz_{N-1} / s_{N-1}
  rz_b[N - 1] += t_b / f.s[N - 1];
  s_b[N - 1] += -t_b * f.t / f.s[N - 1];
  // D_k = s_{k+1} - s_k
#pragma unroll
  for (int k = 0; k + 1 < N; ++k) {
    s_b[k + 1] += D_b[k];
    s_b[k] -= D_b[k];
  }

  // ---------------- per-hit arc lengths and offsets
  S tx_b = S(tx_bd), ty_b = S(ty_bd);
  S rx_b[N], ry_b[N];
#pragma unroll
  for (int k = 0; k < N; ++k) rx_b[k] = ry_b[k] = S(0);
#pragma unroll
  for (int k = 1; k < N; ++k) {
    const S xt = f.xt[k], xn = f.xn[k];
    S xt_b = S(0), xn_b = S(0);
    // u = A / (1 + sq), sq = sqrt(1 - kp A)
    {
      const S den = S(1) + f.sq[k];
      const S A = f.A[k];
      const S inv = S(1) / (S(2) * f.sq[k] * den * den);
      const S A_b = u_b[k] * (S(1) / den + A * f.kp * inv);
      kp_b += u_b[k] * A * A * inv;
      // A = 2 xn - kp (xt^2 + xn^2)
      xn_b += A_b * (S(2) - S(2) * f.kp * xn);
      xt_b += A_b * (S(-2) * f.kp * xt);
      kp_b += -A_b * (xt * xt + xn * xn);
    }
    // s = atan2(kp xt, 1 - kp xn) / kp
    if (f.kp != S(0)) {
      const S Ys = f.kp * xt, Xs = S(1) - f.kp * xn;
      const S r2 = Xs * Xs + Ys * Ys;
      const S ang_b = s_b[k] / f.kp;
      kp_b += -s_b[k] * f.s[k] / f.kp;
      const S Ys_b = ang_b * Xs / r2;
      const S Xs_b = -ang_b * Ys / r2;
      kp_b += Ys_b * xt - Xs_b * xn;
      xt_b += Ys_b * f.kp;
      xn_b += -Xs_b * f.kp;
    } else {
      xt_b += s_b[k];
      kp_b += s_b[k] * xt * xn;
    }
    // xt = tx rx + ty ry, xn = -ty rx + tx ry
    const S rx = S(f.rx[k]), ry = S(f.ry[k]);
    rx_b[k] += xt_b * f.tx - xn_b * f.ty;
    ry_b[k] += xt_b * f.ty + xn_b * f.tx;
    tx_b += xt_b * rx + xn_b * ry;
    ty_b += xt_b * ry - xn_b * rx;
  }

  // ---------------- pre-fit
  {
    S ux_b = tx_b * f.cb - ty_b * f.sb;
    S uy_b = tx_b * f.sb + ty_b * f.cb;
    const S cb_b = tx_b * f.ux + ty_b * f.uy;
    S sb_b = tx_b * f.uy - ty_b * f.ux;
    if (f.cb > S(0)) sb_b += cb_b * (-f.sb / f.cb);
    kp_b += sb_b * f.lb * S(0.5);
    S lb_b = sb_b * f.kp * S(0.5);
    S bx_b = ux_b / f.lb, by_b = uy_b / f.lb;
    lb_b += -(ux_b * f.ux + uy_b * f.uy) / f.lb;
    const S prod = f.la * f.lb * f.ld;
    const S cr_b = kp_b * S(2) / prod;
    const S la_b = -kp_b * f.kp / f.la;
    lb_b += -kp_b * f.kp / f.lb;
    const S ld_b = -kp_b * f.kp / f.ld;
    S ax_b = la_b * f.ax / f.la, ay_b = la_b * f.ay / f.la;
    bx_b += lb_b * f.bx / f.lb;
    by_b += lb_b * f.by / f.lb;
    const S dx = f.bx - f.ax, dy = f.by - f.ay;
    const S dx_b = ld_b * dx / f.ld, dy_b = ld_b * dy / f.ld;
    bx_b += dx_b;
    by_b += dy_b;
    ax_b -= dx_b;
    ay_b -= dy_b;
    ax_b += cr_b * f.by;
    by_b += cr_b * f.ax;
    ay_b -= cr_b * f.bx;
    bx_b -= cr_b * f.ay;
    rx_b[b] += ax_b;
    ry_b[b] += ay_b;
    rx_b[N - 1] += bx_b;
    ry_b[N - 1] += by_b;
  }

  // ---------------- relative positions -> hits
  S sx = S(0), sy = S(0), sz = S(0);
#pragma unroll
  for (int k = 1; k < N; ++k) {
    gP[k][0] = rx_b[k];
    gP[k][1] = ry_b[k];
    gP[k][2] = rz_b[k];
    sx += rx_b[k];
    sy += ry_b[k];
    sz += rz_b[k];
  }
  gP[0][0] = S(P0x_b) - sx;
  gP[0][1] = S(P0y_b) - sy;
  gP[0][2] = S(P0z_b) - sz;
}

}  // namespace fit
}  // namespace pt
