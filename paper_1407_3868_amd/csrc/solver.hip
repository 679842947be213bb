// Right-hand side, GMRES (FP64, and FP32 matvecs inside FP64 iterative
// refinement) and field evaluation.
#include <chrono>
#include <cmath>
#include <vector>

#include "kernels.h"

using mpsl::DBuf;
using mpsl::zc;

namespace mpsl {

namespace {

int cdiv(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }

// rhs = S a for one source, into dev (double2[n*P]).
int rhs_dev(mpsl_ctx *ctx, const double *src, void *dev) {
  int rc = build_tables(ctx);
  if (rc) return rc;
  const int cb = chunks_s2l(ctx);
  if ((rc = launch_reflect(ctx, nullptr, src, ctx->sigma.p))) return rc;
  if ((rc = launch_s2l_coef(ctx, ctx->sigma.p))) return rc;
  if ((rc = launch_s2l(ctx, MPSL_FP64, ctx->part.p, cb))) return rc;
  return launch_sapply(ctx, MPSL_FP64, nullptr, ctx->part.p, cb, dev);
}

// ||v||_2 of a device vector (FP64 complex), synchronous.
int norm2(mpsl_ctx *ctx, const void *v, int64_t len, double &out, void *hbuf) {
  int rc = launch_dotc_multi(ctx, v, 0, 1, v, len, hbuf);
  if (rc) return rc;
  double2 h;
  MPSL_HIP_TRY(ctx, hipMemcpyAsync(&h, hbuf, sizeof(double2), hipMemcpyDeviceToHost, ctx->stream));
  MPSL_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  out = std::sqrt(std::max(h.x, 0.0));
  return MPSL_OK;
}

struct Gm {
  double2 *V = nullptr;     // (m+1) x len
  double2 *w = nullptr;     // len
  double2 *h = nullptr;     // (m+1)
  double2 *h2 = nullptr;    // (m+1)
  float2 *x32 = nullptr;    // len
  float2 *y32 = nullptr;    // len
  double2 *r = nullptr;     // len (residual)
  double2 *xs = nullptr;    // len (solution)
  double2 *b = nullptr;     // len (rhs)
  double2 *d = nullptr;     // len (correction)
};

int gm_alloc(mpsl_ctx *ctx, int m, int64_t len, Gm &g) {
  const size_t c = sizeof(double2);
  const size_t bytes = (static_cast<size_t>(m + 1) + 5) * len * c + 2 * (m + 2) * c + 2 * len * sizeof(float2) + 4096;
  int rc = dev_alloc(ctx, ctx->gm, bytes);
  if (rc) return rc;
  char *p = static_cast<char *>(ctx->gm.p);
  auto take = [&](size_t nb) {
    char *q = p;
    p += (nb + 255) / 256 * 256;
    return q;
  };
  g.V = reinterpret_cast<double2 *>(take((m + 1) * len * c));
  g.w = reinterpret_cast<double2 *>(take(len * c));
  g.r = reinterpret_cast<double2 *>(take(len * c));
  g.xs = reinterpret_cast<double2 *>(take(len * c));
  g.b = reinterpret_cast<double2 *>(take(len * c));
  g.d = reinterpret_cast<double2 *>(take(len * c));
  g.h = reinterpret_cast<double2 *>(take((m + 2) * c));
  g.h2 = reinterpret_cast<double2 *>(take((m + 2) * c));
  g.x32 = reinterpret_cast<float2 *>(take(len * sizeof(float2)));
  g.y32 = reinterpret_cast<float2 *>(take(len * sizeof(float2)));
  return MPSL_OK;
}

// w = A v in precision prec (v, w FP64 device vectors).
int op(mpsl_ctx *ctx, int prec, const double2 *v, double2 *w, Gm &g, int64_t len) {
  if (prec == MPSL_FP64) return matvec(ctx, MPSL_FP64, v, w);
  int rc;
  if ((rc = launch_to_fp32(ctx, v, g.x32, len))) return rc;
  if ((rc = matvec(ctx, MPSL_FP32, g.x32, g.y32))) return rc;
  return launch_to_fp64(ctx, g.y32, w, len);
}

// Restarted GMRES on A x = rhs with x0 = 0 (x written to xout).  Arnoldi by
// classical Gram-Schmidt applied twice, FP64; Givens rotations on the host.
// Stops when the estimated relative residual is below tol or after maxit
// matvecs.  Returns the number of matvecs through *its.
int gmres(mpsl_ctx *ctx, int prec, const double2 *rhs, double2 *xout, int64_t len, double tol, int maxit,
          int m, Gm &g, int *its, std::vector<double> &hist) {
  int rc;
  MPSL_HIP_TRY(ctx, hipMemsetAsync(xout, 0, len * sizeof(double2), ctx->stream));
  double bn;
  if ((rc = norm2(ctx, rhs, len, bn, g.h))) return rc;
  *its = 0;
  if (bn == 0.0) return MPSL_OK;
  int total = 0;
  bool first = true;
  while (total < maxit) {
    // r = rhs - A x
    double beta0;
    if (first) {
      if ((rc = launch_scale(ctx, g.V, len, 1.0, rhs))) return rc;
      beta0 = bn;
    } else {
      if ((rc = op(ctx, prec, xout, g.w, g, len))) return rc;
      ++total;
      if ((rc = launch_scale(ctx, g.V, len, 1.0, rhs))) return rc;
      if ((rc = launch_axpy_c(ctx, g.V, g.w, len, -1.0, 0.0))) return rc;
      if ((rc = norm2(ctx, g.V, len, beta0, g.h))) return rc;
    }
    first = false;
    if (!std::isfinite(beta0)) return set_err(ctx, MPSL_ENUMERIC, "non-finite residual");
    if (beta0 / bn < tol) break;
    if ((rc = launch_scale(ctx, g.V, len, 1.0 / beta0, g.V))) return rc;
    std::vector<zc> H(static_cast<size_t>(m + 1) * m, zc(0, 0)), cs(m), sn(m), gv(m + 1, zc(0, 0));
    gv[0] = beta0;
    int j = 0;
    double res = beta0 / bn;
    for (; j < m && total < maxit; ++j) {
      double2 *vj = g.V + j * len;
      double2 *vn = g.V + (j + 1) * len;
      if ((rc = op(ctx, prec, vj, vn, g, len))) return rc;
      ++total;
      // two passes of classical Gram-Schmidt
      std::vector<double2> hh(j + 1), hh2(j + 1);
      if ((rc = launch_dotc_multi(ctx, g.V, len, j + 1, vn, len, g.h))) return rc;
      if ((rc = launch_gemv_sub(ctx, g.V, len, j + 1, g.h, vn, len))) return rc;
      if ((rc = launch_dotc_multi(ctx, g.V, len, j + 1, vn, len, g.h2))) return rc;
      if ((rc = launch_gemv_sub(ctx, g.V, len, j + 1, g.h2, vn, len))) return rc;
      MPSL_HIP_TRY(ctx, hipMemcpyAsync(hh.data(), g.h, (j + 1) * sizeof(double2), hipMemcpyDeviceToHost, ctx->stream));
      MPSL_HIP_TRY(ctx, hipMemcpyAsync(hh2.data(), g.h2, (j + 1) * sizeof(double2), hipMemcpyDeviceToHost, ctx->stream));
      double hn;
      if ((rc = norm2(ctx, vn, len, hn, g.h))) return rc;
      for (int i = 0; i <= j; ++i) H[i * m + j] = zc(hh[i].x + hh2[i].x, hh[i].y + hh2[i].y);
      H[(j + 1) * m + j] = hn;
      if (!std::isfinite(hn)) return set_err(ctx, MPSL_ENUMERIC, "non-finite Arnoldi norm");
      if (hn > 0.0 && (rc = launch_scale(ctx, vn, len, 1.0 / hn, vn))) return rc;
      // apply previous rotations, then a new one
      for (int i = 0; i < j; ++i) {
        const zc a = H[i * m + j], b = H[(i + 1) * m + j];
        H[i * m + j] = std::conj(cs[i]) * a + std::conj(sn[i]) * b;
        H[(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
      }
      const zc a = H[j * m + j], b = H[(j + 1) * m + j];
      const double den = std::sqrt(std::norm(a) + std::norm(b));
      if (den == 0.0) {
        cs[j] = 1.0;
        sn[j] = 0.0;
      } else {
        cs[j] = a / den;
        sn[j] = b / den;
      }
      H[j * m + j] = std::conj(cs[j]) * a + std::conj(sn[j]) * b;
      H[(j + 1) * m + j] = 0.0;
      gv[j + 1] = -sn[j] * gv[j];
      gv[j] = std::conj(cs[j]) * gv[j];
      res = std::abs(gv[j + 1]) / bn;
      hist.push_back(res);
      if (res < tol || hn == 0.0) {
        ++j;
        break;
      }
    }
    // back substitution, x += V y
    std::vector<zc> y(j);
    for (int i = j - 1; i >= 0; --i) {
      zc s = gv[i];
      for (int k = i + 1; k < j; ++k) s -= H[i * m + k] * y[k];
      y[i] = s / H[i * m + i];
    }
    std::vector<double2> yd(j);
    for (int i = 0; i < j; ++i) yd[i] = make_double2(-y[i].real(), -y[i].imag());
    MPSL_HIP_TRY(ctx, hipMemcpyAsync(g.h, yd.data(), j * sizeof(double2), hipMemcpyHostToDevice, ctx->stream));
    if ((rc = launch_gemv_sub(ctx, g.V, len, j, g.h, xout, len))) return rc;  // x -= V (-y)
    MPSL_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (res < tol) break;
  }
  *its = total;
  return MPSL_OK;
}

}  // namespace
}  // namespace mpsl

extern "C" {

int mpsl_rhs(mpsl_ctx *ctx, const double *src, mpsl_c128 *rhs) {
  if (!ctx || !src || !rhs) return MPSL_EINVAL;
  MPSL_HIP_TRY(ctx, hipSetDevice(ctx->device));
  int rc = mpsl::build_tables(ctx);
  if (rc) return rc;
  if (!(src[1] > 0.0)) return mpsl::set_err(ctx, MPSL_EINVAL, "the source must lie in the top layer (y > 0)");
  const size_t bytes = static_cast<size_t>(ctx->n) * (2 * ctx->p + 1) * sizeof(double2);
  if ((rc = mpsl::dev_alloc(ctx, ctx->ybuf, bytes))) return rc;
  if ((rc = mpsl::rhs_dev(ctx, src, ctx->ybuf.p))) return rc;
  MPSL_HIP_TRY(ctx, hipMemcpyAsync(rhs, ctx->ybuf.p, bytes, hipMemcpyDeviceToHost, ctx->stream));
  MPSL_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return MPSL_OK;
}

int mpsl_solve(mpsl_ctx *ctx, int n_rhs, const double *src_xy, const mpsl_opts *opts, mpsl_c128 *beta_out,
               mpsl_info *info) {
  if (!ctx || !src_xy || !beta_out || n_rhs <= 0) return MPSL_EINVAL;
  MPSL_HIP_TRY(ctx, hipSetDevice(ctx->device));
  int rc = mpsl::build_tables(ctx);
  if (rc) return rc;
  mpsl_opts o = {MPSL_FP64, 1e-10, 500, 0, 0.0};
  if (opts) o = *opts;
  if (o.precision != MPSL_FP64 && o.precision != MPSL_FP32) return MPSL_EINVAL;
  if (!(o.tol > 0.0) || o.maxiter <= 0) return mpsl::set_err(ctx, MPSL_EINVAL, "tol > 0 and maxiter > 0");
  const int m = (o.restart > 0 && o.restart < o.maxiter) ? o.restart : o.maxiter;
  const int64_t len = ctx->n * static_cast<int64_t>(2 * ctx->p + 1);
  mpsl::Gm g;
  if ((rc = mpsl::gm_alloc(ctx, m, len, g))) return rc;
  int status = MPSL_OK;
  for (int r = 0; r < n_rhs; ++r) {
    const double *src = src_xy + 2 * r;
    if (!(src[1] > 0.0)) return mpsl::set_err(ctx, MPSL_EINVAL, "the source must lie in the top layer (y > 0)");
    const auto t0 = std::chrono::steady_clock::now();
    ctx->hist.clear();
    if ((rc = mpsl::rhs_dev(ctx, src, g.b))) return rc;
    double bn;
    if ((rc = mpsl::norm2(ctx, g.b, len, bn, g.h))) return rc;
    int iters = 0, fp64mv = 0, refin = 0;
    double relres = 0.0;
    if (o.precision == MPSL_FP64) {
      int its = 0;
      if ((rc = mpsl::gmres(ctx, MPSL_FP64, g.b, g.xs, len, o.tol, o.maxiter, m, g, &its, ctx->hist))) return rc;
      iters = its;
      fp64mv = its;
    } else {
      // FP64 iterative refinement around an FP32-matvec GMRES
      const double itol = o.inner_tol > 0.0 ? o.inner_tol : 1e-5;
      MPSL_HIP_TRY(ctx, hipMemsetAsync(g.xs, 0, len * sizeof(double2), ctx->stream));
      if ((rc = mpsl::launch_scale(ctx, g.r, len, 1.0, g.b))) return rc;
      int budget = o.maxiter;
      for (;;) {
        double rn;
        if ((rc = mpsl::norm2(ctx, g.r, len, rn, g.h))) return rc;
        if (!std::isfinite(rn)) return mpsl::set_err(ctx, MPSL_ENUMERIC, "non-finite refinement residual");
        ctx->hist.push_back(rn / bn);
        if (rn / bn < o.tol || budget <= 0 || refin >= 50) break;
        int its = 0;
        std::vector<double> inner;
        if ((rc = mpsl::gmres(ctx, MPSL_FP32, g.r, g.d, len, itol, budget, m, g, &its, inner))) return rc;
        budget -= its;
        iters += its;
        ++refin;
        if ((rc = mpsl::launch_axpy_c(ctx, g.xs, g.d, len, 1.0, 0.0))) return rc;
        // r = b - A64 x
        if ((rc = mpsl::matvec(ctx, MPSL_FP64, g.xs, g.w))) return rc;
        ++fp64mv;
        if ((rc = mpsl::launch_scale(ctx, g.r, len, 1.0, g.b))) return rc;
        if ((rc = mpsl::launch_axpy_c(ctx, g.r, g.w, len, -1.0, 0.0))) return rc;
      }
    }
    // true FP64 residual
    if ((rc = mpsl::matvec(ctx, MPSL_FP64, g.xs, g.w))) return rc;
    ++fp64mv;
    if ((rc = mpsl::launch_scale(ctx, g.r, len, 1.0, g.b))) return rc;
    if ((rc = mpsl::launch_axpy_c(ctx, g.r, g.w, len, -1.0, 0.0))) return rc;
    double rn;
    if ((rc = mpsl::norm2(ctx, g.r, len, rn, g.h))) return rc;
    relres = bn > 0 ? rn / bn : 0.0;
    MPSL_HIP_TRY(ctx, hipMemcpyAsync(beta_out + r * len, g.xs, len * sizeof(double2), hipMemcpyDeviceToHost,
                                     ctx->stream));
    MPSL_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    const auto t1 = std::chrono::steady_clock::now();
    if (info) {
      info->iterations = iters;
      info->fp64_matvecs = fp64mv;
      info->refinements = refin;
      info->rel_residual = relres;
      info->seconds = std::chrono::duration<double>(t1 - t0).count();
      info->history = ctx->hist.data();
      info->history_len = static_cast<int>(ctx->hist.size());
    }
    if (!(relres < o.tol * 10.0)) status = MPSL_ENOCONV;
  }
  return status;
}

int mpsl_eval_field(mpsl_ctx *ctx, const double *src, const mpsl_c128 *beta, int64_t n_rcv, const double *rcv,
                    mpsl_c128 *u_out) {
  if (!ctx || !src || !beta || !rcv || !u_out || n_rcv <= 0) return MPSL_EINVAL;
  MPSL_HIP_TRY(ctx, hipSetDevice(ctx->device));
  int rc = mpsl::build_tables(ctx);
  if (rc) return rc;
  const int ns = ctx->ns;
  const int64_t len = ctx->n * static_cast<int64_t>(2 * ctx->p + 1);
  if ((rc = mpsl::dev_alloc(ctx, ctx->xbuf, len * sizeof(double2)))) return rc;
  MPSL_HIP_TRY(ctx, hipMemcpyAsync(ctx->xbuf.p, beta, len * sizeof(double2), hipMemcpyHostToDevice, ctx->stream));
  if ((rc = mpsl::launch_m2s(ctx, MPSL_FP64, ctx->xbuf.p, ctx->spec.p))) return rc;
  if ((rc = mpsl::launch_reflect(ctx, ctx->spec.p, src, ctx->sigma.p))) return rc;
  std::vector<zc> spec(2 * ns), sig(2 * ns);
  MPSL_HIP_TRY(ctx, hipMemcpyAsync(spec.data(), ctx->spec.p, 2 * ns * sizeof(double2), hipMemcpyDeviceToHost, ctx->stream));
  MPSL_HIP_TRY(ctx, hipMemcpyAsync(sig.data(), ctx->sigma.p, 2 * ns * sizeof(double2), hipMemcpyDeviceToHost, ctx->stream));
  MPSL_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  // sigma_1 and sigma_3 from the interface conditions at y = 0 and y = -d
  std::vector<zc> sig4(4 * ns);
  const zc I(0.0, 1.0);
  for (int q = 0; q < ns; ++q) {
    const zc lam = ctx->lam[q];
    auto br = [](zc l, zc k) {
      zc g = std::sqrt(l * l - k * k);
      if (g.real() < 0.0) g = -g;
      if (g.real() == 0.0 && g.imag() > 0.0) g = -g;
      return g;
    };
    const zc g1 = br(lam, ctx->k1), g2 = br(lam, ctx->k2), g3 = br(lam, ctx->k3);
    const zc E = std::exp(-g2 * ctx->d);
    const zc gs = std::exp(-I * lam * src[0] - g1 * src[1]);
    const zc sp = sig[q], sm = sig[ns + q], Pp = spec[q], Pm = spec[ns + q];
    sig4[q] = g1 * (sp + E * sm + Pp) / g2 - gs;
    sig4[ns + q] = sp;
    sig4[2 * ns + q] = sm;
    sig4[3 * ns + q] = g3 * (E * sp + sm + Pm) / g2;
  }
  const size_t rb = static_cast<size_t>(n_rcv) * sizeof(double2);
  if ((rc = mpsl::dev_alloc(ctx, ctx->ybuf, rb * 2 + 4 * ns * sizeof(double2)))) return rc;
  char *base = static_cast<char *>(ctx->ybuf.p);
  void *d_rcv = base;
  void *d_u = base + rb;
  void *d_sig = base + 2 * rb;
  MPSL_HIP_TRY(ctx, hipMemcpyAsync(d_rcv, rcv, rb, hipMemcpyHostToDevice, ctx->stream));
  MPSL_HIP_TRY(ctx, hipMemcpyAsync(d_sig, sig4.data(), 4 * ns * sizeof(double2), hipMemcpyHostToDevice, ctx->stream));
  if ((rc = mpsl::launch_field(ctx, ctx->xbuf.p, d_sig, src, n_rcv, d_rcv, d_u))) return rc;
  MPSL_HIP_TRY(ctx, hipMemcpyAsync(u_out, d_u, rb, hipMemcpyDeviceToHost, ctx->stream));
  MPSL_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  for (int64_t i = 0; i < n_rcv; ++i)
    if (std::isnan(u_out[i].re)) return mpsl::set_err(ctx, MPSL_EINSIDE, "receiver inside an enclosing disk");
  return MPSL_OK;
}

}  // extern "C"
