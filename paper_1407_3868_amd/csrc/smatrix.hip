// Host precompute of the prototype scattering matrix of a smooth star-shaped
// dielectric particle (Section 4): Mueller's second-kind equations
// (eqs. (31)-(32)) on the boundary r(t) = a1 + a2 cos(a3 t) of eq. (50),
// solved for the 2p+1 regular waves J_n(k2 r) e^{in theta}; the outgoing
// coefficients follow eq. (35) with the factor i/4 of G = (i/4) H_0.
//
// Nystrom discretisation on nb equispaced points: the logarithmic part of
// each kernel by Kress's product quadrature, the smooth part by the
// trapezoidal rule; the hypersingular difference T_k2 - T_kp by Maue's
// identity T_k = d/ds S_k d/ds + k^2 n_x . S_k n_y with a spectral derivative.
// The dense system is solved by LU with partial pivoting.
#include <cmath>
#include <complex>
#include <string>
#include <vector>

#include "bie.h"
#include "context.h"

namespace mpsl {

namespace {

using cd = std::complex<double>;
constexpr double kEuler = 0.57721566490153286061;

struct Curve {
  std::vector<double> t, r, x, y, dx, dy, ddx, ddy, speed, nx, ny;
};

Curve star_curve(double a1, double a2, int a3, int nb) {
  Curve c;
  c.t.resize(nb);
  c.r = c.x = c.y = c.dx = c.dy = c.ddx = c.ddy = c.speed = c.nx = c.ny = c.t;
  for (int j = 0; j < nb; ++j) {
    const double t = 2.0 * M_PI * j / nb;
    const double co = std::cos(t), si = std::sin(t);
    const double r = a1 + a2 * std::cos(a3 * t);
    const double rp = -a2 * a3 * std::sin(a3 * t);
    const double rpp = -a2 * a3 * a3 * std::cos(a3 * t);
    c.t[j] = t;
    c.r[j] = r;
    c.x[j] = r * co;
    c.y[j] = r * si;
    c.dx[j] = rp * co - r * si;
    c.dy[j] = rp * si + r * co;
    c.ddx[j] = rpp * co - 2.0 * rp * si - r * co;
    c.ddy[j] = rpp * si + 2.0 * rp * co - r * si;
    c.speed[j] = std::hypot(c.dx[j], c.dy[j]);
    c.nx[j] = c.dy[j] / c.speed[j];   // outward for counter-clockwise traversal
    c.ny[j] = -c.dx[j] / c.speed[j];
  }
  return c;
}

// The single layer S_k, double layer D_k (normal at the source point) and the
// normal derivative N_k of the single layer (normal at the target point), as
// Nystrom matrices (row i: target t_i), plus S_k without the arc-length factor.
void layer_ops(double k, const Curve &c, const std::vector<double> &Rk, std::vector<cd> &S, std::vector<cd> &D,
               std::vector<cd> &N, std::vector<cd> &S0) {
  const int nb = static_cast<int>(c.t.size());
  const double h = 2.0 * M_PI / nb;
  const cd I(0.0, 1.0);
  S.assign(static_cast<size_t>(nb) * nb, 0.0);
  D = N = S0 = S;
  for (int i = 0; i < nb; ++i) {
    const double curv = (c.dy[i] * c.ddx[i] - c.dx[i] * c.ddy[i]) / (c.speed[i] * c.speed[i]);
    for (int j = 0; j < nb; ++j) {
      const size_t ij = static_cast<size_t>(i) * nb + j;
      const double R = Rk[(i - j + nb) % nb];
      if (i == j) {
        const double sp = c.speed[i];
        const double s1 = -sp / (4.0 * M_PI);
        const cd s2 = (cd(0.0, 0.25) - kEuler / (2.0 * M_PI) - std::log(k * sp / 2.0) / (2.0 * M_PI)) * sp;
        S[ij] = R * s1 + h * s2;
        S0[ij] = S[ij] / sp;
        D[ij] = h * curv / (4.0 * M_PI);
        N[ij] = D[ij];
        continue;
      }
      const double ddx = c.x[i] - c.x[j], ddy = c.y[i] - c.y[j];
      const double rr = std::hypot(ddx, ddy);
      const double z = k * rr;
      const double J0 = j0(z), Y0 = y0(z), J1 = j1(z), Y1 = y1(z);
      const double lg = std::log(4.0 * std::pow(std::sin((c.t[i] - c.t[j]) / 2.0), 2));
      // single layer: (i/4) H_0(k r) |x'(tau)|
      const double sp = c.speed[j];
      const cd m = 0.25 * I * cd(J0, Y0) * sp;
      const double m1 = -J0 * sp / (4.0 * M_PI);
      S[ij] = R * m1 + h * (m - m1 * lg);
      S0[ij] = S[ij] / sp;
      // double layer: (ik/4) H_1(k r) nu(tau).(x(t) - x(tau)) / r, |nu| = |x'(tau)|
      const double nud = (c.dy[j] * ddx - c.dx[j] * ddy);
      const cd l = 0.25 * I * k * cd(J1, Y1) * nud / rr;
      const double l1 = -k * J1 * nud / (4.0 * M_PI * rr);
      D[ij] = R * l1 + h * (l - l1 * lg);
      // normal derivative of the single layer: -(ik/4) H_1(k r) n(t).(x(t) - x(tau)) / r |x'(tau)|
      const double nd = (c.nx[i] * ddx + c.ny[i] * ddy);
      const cd q = -0.25 * I * k * cd(J1, Y1) * nd / rr * sp;
      const double q1 = k * J1 * nd / (4.0 * M_PI * rr) * sp;
      N[ij] = R * q1 + h * (q - q1 * lg);
    }
  }
}

// LU with partial pivoting of an n x n row-major matrix, then solve for nrhs
// right-hand sides stored column-major per rhs (B[r * n + i]).
bool lu_solve(int n, std::vector<cd> &A, int nrhs, std::vector<cd> &B) {
  std::vector<int> piv(n);
  for (int k = 0; k < n; ++k) {
    int pr = k;
    double best = std::abs(A[static_cast<size_t>(k) * n + k]);
    for (int i = k + 1; i < n; ++i) {
      const double v = std::abs(A[static_cast<size_t>(i) * n + k]);
      if (v > best) {
        best = v;
        pr = i;
      }
    }
    if (best == 0.0) return false;
    piv[k] = pr;
    if (pr != k)
      for (int j = 0; j < n; ++j) std::swap(A[static_cast<size_t>(k) * n + j], A[static_cast<size_t>(pr) * n + j]);
    const cd inv = 1.0 / A[static_cast<size_t>(k) * n + k];
    for (int i = k + 1; i < n; ++i) {
      cd &lik = A[static_cast<size_t>(i) * n + k];
      lik *= inv;
      const cd f = lik;
      if (f == 0.0) continue;
      cd *ri = &A[static_cast<size_t>(i) * n];
      const cd *rk = &A[static_cast<size_t>(k) * n];
      for (int j = k + 1; j < n; ++j) ri[j] -= f * rk[j];
    }
  }
  for (int r = 0; r < nrhs; ++r) {
    cd *b = &B[static_cast<size_t>(r) * n];
    for (int k = 0; k < n; ++k)
      if (piv[k] != k) std::swap(b[k], b[piv[k]]);
    for (int i = 1; i < n; ++i) {
      cd s = b[i];
      for (int j = 0; j < i; ++j) s -= A[static_cast<size_t>(i) * n + j] * b[j];
      b[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
      cd s = b[i];
      for (int j = i + 1; j < n; ++j) s -= A[static_cast<size_t>(i) * n + j] * b[j];
      b[i] = s / A[static_cast<size_t>(i) * n + i];
    }
  }
  return true;
}

// J_n(x) and J_n'(x) for n >= 0, real x.
void besj(int n, double x, double &j, double &jp) {
  j = jn(n, x);
  jp = (n == 0) ? -jn(1, x) : jn(n - 1, x) - n / x * j;
}

}  // namespace

int star_parts(double a1, double a2, int a3, double k2, int p, int nb, StarParts &sp, std::string &err) {
  if (nb % 2 || nb < 16) {
    err = "n_bdry must be even and >= 16";
    return MPSL_EINVAL;
  }
  const int P = 2 * p + 1, M = 2 * nb;
  const Curve c = star_curve(a1, a2, a3, nb);
  for (int j = 0; j < nb; ++j)
    if (!(c.r[j] > 0.0)) {
      err = "star radius must stay positive";
      return MPSL_EINVAL;
    }
  sp.nb = nb;
  sp.p = p;
  sp.t = c.t;
  sp.r = c.r;
  sp.x = c.x;
  sp.y = c.y;
  sp.dx = c.dx;
  sp.dy = c.dy;
  sp.ddx = c.ddx;
  sp.ddy = c.ddy;
  sp.speed = c.speed;
  sp.nx = c.nx;
  sp.ny = c.ny;
  // Kress weights and the spectral derivative
  const int hn = nb / 2;
  sp.Rk.assign(nb, 0.0);
  for (int k = 0; k < nb; ++k) {
    double s = 0.0;
    for (int m = 1; m < hn; ++m) s += std::cos(m * k * M_PI / hn) / m;
    sp.Rk[k] = -(2.0 * M_PI / hn) * s - (M_PI / (static_cast<double>(hn) * hn)) * std::cos(k * M_PI);
  }
  sp.Fd.assign(static_cast<size_t>(nb) * nb, 0.0);
  for (int i = 0; i < nb; ++i)
    for (int j = 0; j < nb; ++j)
      if (i != j) {
        const int d = i - j;
        sp.Fd[static_cast<size_t>(i) * nb + j] = 0.5 * ((d % 2) ? -1.0 : 1.0) / std::tan(d * M_PI / nb);
      }
  // right-hand sides: -u_inc, -du_inc/dn for u_inc = J_n(k2 r) e^{in theta}
  sp.B.assign(static_cast<size_t>(P) * M, 0.0);
  std::vector<double> Jv(static_cast<size_t>(nb) * (p + 1)), Jd(Jv.size());
  for (int j = 0; j < nb; ++j)
    for (int n = 0; n <= p; ++n) besj(n, k2 * c.r[j], Jv[j * (p + 1) + n], Jd[j * (p + 1) + n]);
  auto jval = [&](int j, int n, double &v, double &d) {  // J_n, J_n' with J_{-n} = (-1)^n J_n
    const int a = n < 0 ? -n : n;
    const double sg = (n < 0 && (a & 1)) ? -1.0 : 1.0;
    v = sg * Jv[j * (p + 1) + a];
    d = sg * Jd[j * (p + 1) + a];
  };
  const double h = 2.0 * M_PI / nb;
  sp.Fs.assign(static_cast<size_t>(P) * nb, 0.0);
  sp.Fm = sp.Fs;
  for (int r = 0; r < P; ++r) {
    const int n = r - p;
    for (int j = 0; j < nb; ++j) {
      double v, dv;
      jval(j, n, v, dv);
      const double th = c.t[j];
      const double nr = c.nx[j] * std::cos(th) + c.ny[j] * std::sin(th);
      const double nt = -c.nx[j] * std::sin(th) + c.ny[j] * std::cos(th);
      const cd e = std::polar(1.0, n * th);
      sp.B[static_cast<size_t>(r) * M + j] = -v * e;
      sp.B[static_cast<size_t>(r) * M + nb + j] = -e * (k2 * dv * nr + cd(0.0, n / c.r[j]) * v * nt);
      // eq. (35): beta^n_l = (i/4) sum_j w_j [J_l e^{-il theta} sigma + d/dn(J_l e^{-il theta}) mu]
      const int l = n;
      const cd em = std::polar(1.0, -l * th);
      const cd w = cd(0.0, 0.25) * (h * c.speed[j]);
      sp.Fs[static_cast<size_t>(r) * nb + j] = w * (v * em);
      sp.Fm[static_cast<size_t>(r) * nb + j] = w * (em * (k2 * dv * nr - cd(0.0, l / c.r[j]) * v * nt));
    }
  }
  return MPSL_OK;
}

int star_smatrix(double a1, double a2, int a3, double k2, double kp, int p, int nb, int pol, std::vector<zc> &Sout,
                 std::string &err) {
  StarParts sp;
  int rc = star_parts(a1, a2, a3, k2, p, nb, sp, err);
  if (rc) return rc;
  const int P = 2 * p + 1;
  Curve c;
  c.t = sp.t;
  c.r = sp.r;
  c.x = sp.x;
  c.y = sp.y;
  c.dx = sp.dx;
  c.dy = sp.dy;
  c.ddx = sp.ddx;
  c.ddy = sp.ddy;
  c.speed = sp.speed;
  c.nx = sp.nx;
  c.ny = sp.ny;
  const std::vector<double> &Rk = sp.Rk, &Fd = sp.Fd;
  std::vector<cd> S2, D2, N2, S02, Sp, Dp, Np, S0p;
  layer_ops(k2, c, Rk, S2, D2, N2, S02);
  layer_ops(kp, c, Rk, Sp, Dp, Np, S0p);
  // difference of the hypersingular operators by Maue's identity
  std::vector<cd> dS0(static_cast<size_t>(nb) * nb), tmp(dS0.size()), T(dS0.size());
  for (size_t i = 0; i < dS0.size(); ++i) dS0[i] = S02[i] - S0p[i];
  for (int i = 0; i < nb; ++i)  // tmp = dS0 * Fd
    for (int j = 0; j < nb; ++j) {
      cd s = 0.0;
      for (int k = 0; k < nb; ++k) s += dS0[static_cast<size_t>(i) * nb + k] * Fd[static_cast<size_t>(k) * nb + j];
      tmp[static_cast<size_t>(i) * nb + j] = s;
    }
  for (int i = 0; i < nb; ++i)  // T = diag(1/speed) Fd tmp + (n_i . n_j)(k2^2 S2 - kp^2 Sp)
    for (int j = 0; j < nb; ++j) {
      cd s = 0.0;
      for (int k = 0; k < nb; ++k) s += Fd[static_cast<size_t>(i) * nb + k] * tmp[static_cast<size_t>(k) * nb + j];
      const size_t ij = static_cast<size_t>(i) * nb + j;
      const double nn = c.nx[i] * c.nx[j] + c.ny[i] * c.ny[j];
      T[ij] = s / c.speed[i] + nn * (k2 * k2 * S2[ij] - kp * kp * Sp[ij]);
    }
  // TE: (1/k^2) du/dn continuous.  With rho = k2^2 / kp^2 the interior field
  // is S_p sigma + D_p mu / rho, which keeps the difference T2 - Tp and moves
  // rho into the identity, Dp and Np terms (rho = 1: the TM system).
  const double rho = (pol == MPSL_TE) ? (k2 * k2) / (kp * kp) : 1.0;
  const double id_mu = 0.5 * (1.0 + 1.0 / rho), id_sig = 0.5 * (1.0 + rho);
  const int M = 2 * nb;
  std::vector<cd> A(static_cast<size_t>(M) * M, 0.0);
  for (int i = 0; i < nb; ++i)
    for (int j = 0; j < nb; ++j) {
      const size_t ij = static_cast<size_t>(i) * nb + j;
      const double id = (i == j) ? 1.0 : 0.0;
      A[static_cast<size_t>(i) * M + j] = S2[ij] - Sp[ij];
      A[static_cast<size_t>(i) * M + nb + j] = id_mu * id + D2[ij] - Dp[ij] / rho;
      A[static_cast<size_t>(nb + i) * M + j] = -id_sig * id + N2[ij] - rho * Np[ij];
      A[static_cast<size_t>(nb + i) * M + nb + j] = T[ij];
    }
  std::vector<cd> B = sp.B;
  if (!lu_solve(M, A, P, B)) {
    err = "singular boundary-integral system";
    return MPSL_ENUMERIC;
  }
  Sout.assign(static_cast<size_t>(P) * P, 0.0);
  for (int li = 0; li < P; ++li)
    for (int r = 0; r < P; ++r) {
      cd s = 0.0;
      const cd *sig = &B[static_cast<size_t>(r) * M];
      const cd *mu = sig + nb;
      for (int j = 0; j < nb; ++j)
        s += sp.Fs[static_cast<size_t>(li) * nb + j] * sig[j] + sp.Fm[static_cast<size_t>(li) * nb + j] * mu[j];
      Sout[static_cast<size_t>(li) * P + r] = s;
    }
  return MPSL_OK;
}

}  // namespace mpsl
