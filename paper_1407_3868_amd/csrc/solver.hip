// Right-hand side, GMRES (FP64, and FP32 matvecs inside FP64 iterative
// refinement) and field evaluation.
#include <chrono>
#include <cmath>
#include <vector>

#include "solve_sm.h"

using mpsl::DBuf;
using mpsl::zc;

namespace mpsl {

// rhs = S a for one source, into dev (double2[n*P]).
int rhs_device(mpsl_ctx *ctx, const double *src, void *dev) {
  int rc = build_tables(ctx);
  if (rc) return rc;
  const int cb = chunks_s2l(ctx, 1, MPSL_FP64);
  if ((rc = launch_reflect(ctx, nullptr, src, ctx->sigma.p))) return rc;
  if ((rc = launch_s2l_coef(ctx, ctx->sigma.p))) return rc;
  if ((rc = launch_s2l(ctx, MPSL_FP64, ctx->part.p, cb))) return rc;
  if ((rc = launch_fold_parts(ctx, MPSL_FP64, ctx->part.p, cb))) return rc;
  return launch_sapply(ctx, MPSL_FP64, nullptr, ctx->part.p, dev);
}

namespace {


}  // namespace

SolveSM::~SolveSM() {
  if (hh_) (void)hipHostFree(hh_);
}

int SolveSM::init(mpsl_ctx *ctx, const mpsl_opts &o, const void *b_dev) {
  ctx_ = ctx;
  o_ = o;
  if (o_.inner_tol <= 0.0) o_.inner_tol = 1e-5;
  len_ = ctx->n * static_cast<int64_t>(2 * ctx->p + 1);
  m_ = (o.restart > 0 && o.restart < o.maxiter) ? o.restart : o.maxiter;
  if (m_ > kMaxKrylov)
    return set_err(ctx, MPSL_EINVAL, "Krylov dimension (restart, or maxiter without restart) above " +
                                         std::to_string(kMaxKrylov));
  const size_t c = sizeof(double2);
  // the Arnoldi dot products reduce m + 1 rows of partial sums at once
  int rc = dev_alloc(ctx, ctx->scal, dotc_scratch_bytes(m_ + 2));
  if (rc) return rc;
  vp_ = o_.precision == MPSL_FP32 ? MPSL_FP32 : MPSL_FP64;
  const size_t vb = vp_ == MPSL_FP32 ? sizeof(float2) : sizeof(double2);
  const size_t bytes = static_cast<size_t>(m_ + 1) * len_ * vb + 6 * len_ * c + 4 * static_cast<size_t>(m_ + 2) * c +
                       2 * len_ * sizeof(float2) + 8192;
  rc = dev_alloc(ctx, ctx->gm, bytes);
  if (rc) return rc;
  char *p = static_cast<char *>(ctx->gm.p);
  auto take = [&](size_t nb) {
    char *q = p;
    p += (nb + 255) / 256 * 256;
    return q;
  };
  V_ = take((m_ + 1) * len_ * vb);
  u_ = reinterpret_cast<double2 *>(take(len_ * c));
  w_ = reinterpret_cast<double2 *>(take(len_ * c));
  r_ = reinterpret_cast<double2 *>(take(len_ * c));
  xs_ = reinterpret_cast<double2 *>(take(len_ * c));
  b_ = reinterpret_cast<double2 *>(take(len_ * c));
  d_ = reinterpret_cast<double2 *>(take(len_ * c));
  h_ = reinterpret_cast<double2 *>(take((m_ + 2) * c));
  h2_ = reinterpret_cast<double2 *>(take((m_ + 2) * c));
  nrm_ = reinterpret_cast<double2 *>(take((m_ + 2) * c));
  q_ = reinterpret_cast<double2 *>(take((m_ + 2) * c));
  skip_ = reinterpret_cast<int32_t *>(take(256));
  x32_ = reinterpret_cast<float2 *>(take(len_ * sizeof(float2)));
  y32_ = reinterpret_cast<float2 *>(take(len_ * sizeof(float2)));
  if (hh_) (void)hipHostFree(hh_);
  hh_ = nullptr;
  // pinned staging: h (m+2), h2 (m+2), norm (1), y (m+1), second-pass flag (1)
  if (hipHostMalloc(reinterpret_cast<void **>(&hh_), (3 * static_cast<size_t>(m_ + 2) + 2) * c) != hipSuccess) {
    hh_ = nullptr;
    return set_err(ctx, MPSL_ENOMEM, "pinned host allocation failed");
  }
  pc_ = ctx->pc_kind == MPSL_PRECOND_CLUSTER;
  pc_s_ = 0.0;
  if (pc_) {
    const double before = ctx->pc_setup_s;
    if ((rc = precond_build(ctx, o_.precision))) return rc;
    pc_s_ = ctx->pc_setup_s - before;
  }
  status_ = kRunning;
  inner_mv_ = fp64_mv_ = refin_ = 0;
  k0_ = base_ = cycles_ = reorth_ = 0;
  R0_.clear();
  Cs_.clear();
  hist_.clear();
  MPSL_HIP_TRY(ctx, hipMemcpyAsync(b_, b_dev, len_ * c, hipMemcpyDeviceToDevice, ctx->stream));
  MPSL_HIP_TRY(ctx, hipMemsetAsync(xs_, 0, len_ * c, ctx->stream));
  if ((rc = launch_scale(ctx, r_, len_, 1.0, b_))) return rc;
  if ((rc = launch_dotc_multi(ctx, b_, 0, 1, b_, len_, nrm_))) return rc;
  MPSL_HIP_TRY(ctx, hipMemcpyAsync(hh_ + 2 * (m_ + 2), nrm_, c, hipMemcpyDeviceToHost, ctx->stream));
  MPSL_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  bn_ = std::sqrt(std::max(hh_[2 * (m_ + 2)].x, 0.0));
  if (!std::isfinite(bn_)) return set_err(ctx, MPSL_ENUMERIC, "non-finite right-hand side");
  if (bn_ == 0.0) {
    status_ = kConverged;
    rel_res_ = 0.0;
    return MPSL_OK;
  }
  rn_ = bn_;
  rel_res_ = 1.0;
  hist_.push_back(1.0);
  return begin_inner();
}

std::vector<zc> SolveSM::w_coords(const std::vector<zc> &s) const {
  std::vector<zc> t(s);
  for (int i = 0; i < k0_; ++i) {  // Omega = G_{k-1} ... G_0
    const zc a = t[i], b = t[i + 1];
    t[i] = std::conj(cs0_[i]) * a + std::conj(sn0_[i]) * b;
    t[i + 1] = -sn0_[i] * a + cs0_[i] * b;
  }
  t.resize(k0_);
  return t;
}

void SolveSM::keep_first_cycle() {
  const int k = j_, m = m_;
  k0_ = k;
  R0_.assign(static_cast<size_t>(k) * k, zc(0.0, 0.0));
  for (int a = 0; a < k; ++a)
    for (int b = a; b < k; ++b) R0_[static_cast<size_t>(a) * k + b] = H_[static_cast<size_t>(a) * m + b];
  cs0_.assign(cs_.begin(), cs_.begin() + k);
  sn0_.assign(sn_.begin(), sn_.begin() + k);
}

int SolveSM::begin_inner() {
  mpsl_ctx *ctx = ctx_;
  const size_t c = sizeof(double2);
  inner_abs_ = (o_.precision == MPSL_FP64) ? o_.tol * bn_ : std::max(o_.inner_tol * rn_, 0.5 * o_.tol * bn_);
  int rc;
  double rn = rn_;
  base_ = k0_ > 0 ? k0_ + 1 : 0;
  yC_.assign(k0_, zc(0.0, 0.0));
  Cs_.clear();
  if (k0_ > 0) {  // r <- (I - W W^H) r (twice), yC = W^H r
    for (int pass = 0; pass < 2; ++pass) {
      if ((rc = launch_dotc_multi(ctx, V_, len_, k0_ + 1, r_, len_, h_, nullptr, vp_)) ||
          (rc = launch_proj_fix(ctx, h_, q_, k0_ + 1)) ||
          (rc = launch_gemv_sub(ctx, V_, len_, k0_ + 1, h_, r_, len_, nullptr, vp_)))
        return rc;
      MPSL_HIP_TRY(ctx, hipMemcpyAsync(hh_, h_, (k0_ + 1) * c, hipMemcpyDeviceToHost, ctx->stream));
      MPSL_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
      std::vector<zc> sv(k0_ + 1);
      for (int i = 0; i <= k0_; ++i) sv[i] = zc(hh_[i].x, hh_[i].y);
      const std::vector<zc> f = w_coords(sv);
      for (int i = 0; i < k0_; ++i) yC_[i] += f[i];
    }
    if ((rc = launch_dotc_multi(ctx, r_, 0, 1, r_, len_, nrm_))) return rc;
    MPSL_HIP_TRY(ctx, hipMemcpyAsync(hh_ + 2 * (m_ + 2), nrm_, c, hipMemcpyDeviceToHost, ctx->stream));
    MPSL_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    rn = std::sqrt(std::max(hh_[2 * (m_ + 2)].x, 0.0));
  }
  H_.assign(static_cast<size_t>(m_ + 1) * m_, zc(0.0, 0.0));
  cs_.assign(m_, zc(0.0, 0.0));
  sn_.assign(m_, zc(0.0, 0.0));
  gv_.assign(m_ + 1, zc(0.0, 0.0));
  gv_[0] = rn;
  j_ = 0;
  phase_ = kInner;
  if (!(rn > 0.0)) return finish_cycle();  // the recycled space already holds the correction
  return store_basis(base_, 1.0 / rn, r_);
}

int SolveSM::store_basis(int j, double s, const double2 *src) {
  if (vp_ == MPSL_FP32) return launch_scale_to_fp32(ctx_, vslot(j), len_, s, src);
  return launch_scale(ctx_, vslot(j), len_, s, src);
}

int SolveSM::launch() {
  if (status_ != kRunning) return MPSL_OK;
  mpsl_ctx *ctx = ctx_;
  const size_t c = sizeof(double2);
  int rc;
  if (phase_ == kInner) {
    const int nb = base_ + j_ + 1;
    const void *vj = vslot(base_ + j_);
    // the new vector w = A M^{-1} v_j (FP64)
    double2 *vn = vp_ == MPSL_FP32 ? u_ : static_cast<double2 *>(vslot(nb));
    if (o_.precision == MPSL_FP64) {
      if (pc_) {
        if ((rc = precond_apply(ctx, MPSL_FP64, vj, w_))) return rc;
        vj = w_;
      }
      if ((rc = matvec(ctx, MPSL_FP64, vj, vn))) return rc;
    } else {
      if (pc_ && ((rc = launch_to_fp64(ctx, vj, w_, len_)) || (rc = precond_apply(ctx, MPSL_FP32, w_, d_)) ||
                  (rc = launch_to_fp32(ctx, d_, x32_, len_))))
        return rc;
      if ((rc = matvec(ctx, MPSL_FP32, pc_ ? x32_ : vj, y32_)) || (rc = launch_to_fp64(ctx, y32_, vn, len_)))
        return rc;
    }
    // classical Gram-Schmidt over [V_{k0+1} | this cycle's basis] (the
    // recycled part projected onto W only), repeated once when the first pass
    // removed more than 1 - 1/2 of ||w||^2 (decided on the device: the second
    // pass's kernels read the flag); then the norm.  With an FP64 basis the
    // first pass's dots include w itself (it follows the basis in V_), giving
    // ||w||^2; with an FP32 basis w is apart and has its own dot product.
    if (vp_ == MPSL_FP32) {
      if ((rc = launch_dotc_multi(ctx, vn, 0, 1, vn, len_, h_ + nb)) ||
          (rc = launch_dotc_multi(ctx, V_, len_, nb, vn, len_, h_, nullptr, vp_)))
        return rc;
    } else if ((rc = launch_dotc_multi(ctx, V_, len_, nb + 1, vn, len_, h_))) {
      return rc;
    }
    if (k0_ > 0 && (rc = launch_proj_fix(ctx, h_, q_, k0_ + 1))) return rc;
    if ((rc = launch_gemv_sub(ctx, V_, len_, nb, h_, vn, len_, nullptr, vp_)) ||
        (rc = launch_dotc_multi(ctx, vn, 0, 1, vn, len_, nrm_)) ||
        (rc = launch_reorth_flag(ctx, h_ + nb, nrm_, 0.5, skip_)))
      return rc;
    if ((rc = launch_dotc_multi(ctx, V_, len_, nb, vn, len_, h2_, skip_, vp_))) return rc;
    if (k0_ > 0 && (rc = launch_proj_fix(ctx, h2_, q_, k0_ + 1))) return rc;
    if ((rc = launch_gemv_sub(ctx, V_, len_, nb, h2_, vn, len_, skip_, vp_)) ||
        (rc = launch_dotc_multi(ctx, vn, 0, 1, vn, len_, nrm_)))
      return rc;
    MPSL_HIP_TRY(ctx, hipMemcpyAsync(hh_ + 3 * (m_ + 2) + 1, skip_, sizeof(int32_t), hipMemcpyDeviceToHost,
                                     ctx->stream));
    MPSL_HIP_TRY(ctx, hipMemcpyAsync(hh_, h_, nb * c, hipMemcpyDeviceToHost, ctx->stream));
    MPSL_HIP_TRY(ctx, hipMemcpyAsync(hh_ + (m_ + 2), h2_, nb * c, hipMemcpyDeviceToHost, ctx->stream));
  } else {
    if ((rc = matvec(ctx, MPSL_FP64, xs_, w_)) || (rc = launch_scale(ctx, r_, len_, 1.0, b_)) ||
        (rc = launch_axpy_c(ctx, r_, w_, len_, -1.0, 0.0)) ||
        (rc = launch_dotc_multi(ctx, r_, 0, 1, r_, len_, nrm_)))
      return rc;
  }
  MPSL_HIP_TRY(ctx, hipMemcpyAsync(hh_ + 2 * (m_ + 2), nrm_, c, hipMemcpyDeviceToHost, ctx->stream));
  return MPSL_OK;
}

int SolveSM::complete() {
  if (status_ != kRunning) return MPSL_OK;
  mpsl_ctx *ctx = ctx_;
  MPSL_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  const double nn = std::sqrt(std::max(hh_[2 * (m_ + 2)].x, 0.0));
  int rc;
  if (phase_ == kInner) {
    ++inner_mv_;
    if (o_.precision == MPSL_FP64) ++fp64_mv_;
    const int j = j_, m = m_, b0 = base_;
    if (!std::isfinite(nn)) return set_err(ctx, MPSL_ENUMERIC, "non-finite Arnoldi norm");
    if (*reinterpret_cast<const int32_t *>(hh_ + 3 * (m_ + 2) + 1) == 0) ++reorth_;
    for (int i = 0; i <= j; ++i)
      H_[i * m + j] = zc(hh_[b0 + i].x + hh_[m + 2 + b0 + i].x, hh_[b0 + i].y + hh_[m + 2 + b0 + i].y);
    for (int i = 0; b0 > 0 && i <= k0_; ++i)  // coefficients on V_{k0+1} (projected onto W)
      Cs_.push_back(zc(hh_[i].x + hh_[m + 2 + i].x, hh_[i].y + hh_[m + 2 + i].y));
    H_[(j + 1) * m + j] = nn;
    if (nn > 0.0 &&
        (rc = store_basis(b0 + j + 1, 1.0 / nn, vp_ == MPSL_FP32 ? u_ : static_cast<const double2 *>(vslot(b0 + j + 1)))))
      return rc;
    for (int i = 0; i < j; ++i) {  // previous rotations, then a new one
      const zc a = H_[i * m + j], b = H_[(i + 1) * m + j];
      H_[i * m + j] = std::conj(cs_[i]) * a + std::conj(sn_[i]) * b;
      H_[(i + 1) * m + j] = -sn_[i] * a + cs_[i] * b;
    }
    const zc a = H_[j * m + j], b = H_[(j + 1) * m + j];
    const double den = std::sqrt(std::norm(a) + std::norm(b));
    if (den == 0.0) {
      cs_[j] = 1.0;
      sn_[j] = 0.0;
    } else {
      cs_[j] = a / den;
      sn_[j] = b / den;
    }
    H_[j * m + j] = std::conj(cs_[j]) * a + std::conj(sn_[j]) * b;
    H_[(j + 1) * m + j] = 0.0;
    gv_[j + 1] = -sn_[j] * gv_[j];
    gv_[j] = std::conj(cs_[j]) * gv_[j];
    const double res = std::abs(gv_[j + 1]);
    hist_.push_back(res / bn_);
    j_ = j + 1;
    if (res < inner_abs_ || j_ == m_ - base_ || nn == 0.0 || inner_mv_ >= o_.maxiter) return finish_cycle();
    return MPSL_OK;
  }
  // residual phase
  ++fp64_mv_;
  if (!std::isfinite(nn)) return set_err(ctx, MPSL_ENUMERIC, "non-finite residual");
  rn_ = nn;
  rel_res_ = rn_ / bn_;
  if (rel_res_ < o_.tol) {
    status_ = kConverged;
    return MPSL_OK;
  }
  if (inner_mv_ >= o_.maxiter || refin_ >= 100) {
    status_ = kExhausted;
    return MPSL_OK;
  }
  return begin_inner();
}

int SolveSM::finish_cycle() {
  mpsl_ctx *ctx = ctx_;
  const int j = j_, m = m_;
  std::vector<zc> y(j);
  for (int i = j - 1; i >= 0; --i) {
    zc s = gv_[i];
    for (int k = i + 1; k < j; ++k) s -= H_[i * m + k] * y[k];
    y[i] = s / H_[i * m + i];
  }
  // coefficients of the correction over V_[0 .. base_ + j): with a recycled
  // first cycle, V_k R^{-1} (yC - E z) on its k0 vectors (E z = (Omega sum Cs_i y_i)[:k0])
  const int nb = base_ + j;
  std::vector<zc> coef(nb, zc(0.0, 0.0));
  if (base_ > 0) {
    const int k = k0_;
    std::vector<zc> e(k + 1, zc(0.0, 0.0));
    for (int i = 0; i < j; ++i)
      for (int t = 0; t <= k; ++t) e[t] += Cs_[static_cast<size_t>(i) * (k + 1) + t] * y[i];
    const std::vector<zc> f = w_coords(e);
    for (int a = k - 1; a >= 0; --a) {
      zc s = yC_[a] - f[a];
      for (int bb = a + 1; bb < k; ++bb) s -= R0_[static_cast<size_t>(a) * k + bb] * coef[bb];
      coef[a] = s / R0_[static_cast<size_t>(a) * k + a];
    }
  }
  for (int i = 0; i < j; ++i) coef[base_ + i] = y[i];
  double2 *hy = hh_ + 2 * (m_ + 2) + 1;  // pinned, separate from the D2H staging
  for (int i = 0; i < nb; ++i) hy[i] = make_double2(-coef[i].real(), -coef[i].imag());
  MPSL_HIP_TRY(ctx, hipMemcpyAsync(h_, hy, nb * sizeof(double2), hipMemcpyHostToDevice, ctx->stream));
  MPSL_HIP_TRY(ctx, hipMemsetAsync(d_, 0, len_ * sizeof(double2), ctx->stream));
  int rc;
  if ((rc = launch_gemv_sub(ctx, V_, len_, nb, h_, d_, len_, nullptr, vp_))) return rc;  // d = V coef
  if (pc_) {  // the correction is M^{-1} V y
    if ((rc = precond_apply(ctx, o_.precision, d_, w_)) || (rc = launch_axpy_c(ctx, xs_, w_, len_, 1.0, 0.0)))
      return rc;
  } else if ((rc = launch_axpy_c(ctx, xs_, d_, len_, 1.0, 0.0))) {
    return rc;
  }
  // the first cycle's space is kept for the later ones while the basis has room
  if (cycles_ == 0 && j >= 1 && m_ - (j + 1) >= kMinCycle && inner_mv_ < o_.maxiter) {
    keep_first_cycle();
    std::vector<zc> qv(k0_ + 1, zc(0.0, 0.0));  // q = Omega^H e_k
    qv[k0_] = 1.0;
    for (int i = k0_ - 1; i >= 0; --i) {
      const zc a = qv[i], b = qv[i + 1];
      qv[i] = cs0_[i] * a - std::conj(sn0_[i]) * b;
      qv[i + 1] = sn0_[i] * a + std::conj(cs0_[i]) * b;
    }
    MPSL_HIP_TRY(ctx, hipMemcpyAsync(q_, qv.data(), (k0_ + 1) * sizeof(double2), hipMemcpyHostToDevice, ctx->stream));
    MPSL_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  }
  ++cycles_;
  ++refin_;
  phase_ = kResidual;
  return MPSL_OK;
}

namespace {
}  // namespace
}  // namespace mpsl

extern "C" {

int mpsl_rhs(mpsl_ctx *ctx, const double *src, mpsl_c128 *rhs) {
  if (!ctx || !src || !rhs) return MPSL_EINVAL;
  MPSL_HIP_TRY(ctx, hipSetDevice(ctx->device));
  int rc = mpsl::build_tables(ctx);
  if (rc) return rc;
  if (!(src[1] > ctx->yint[0]))
    return mpsl::set_err(ctx, MPSL_EINVAL, "the source must lie in the top half-space (above the top interface)");
  const size_t bytes = static_cast<size_t>(ctx->n) * (2 * ctx->p + 1) * sizeof(double2);
  if ((rc = mpsl::dev_alloc(ctx, ctx->ybuf, bytes))) return rc;
  if ((rc = mpsl::rhs_device(ctx, src, ctx->ybuf.p))) return rc;
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
  const int64_t len = ctx->n * static_cast<int64_t>(2 * ctx->p + 1);
  int status = MPSL_OK;
  for (int r = 0; r < n_rhs; ++r) {
    const double *src = src_xy + 2 * r;
    if (!(src[1] > ctx->yint[0]))
      return mpsl::set_err(ctx, MPSL_EINVAL, "the source must lie in the top half-space (above the top interface)");
    const auto t0 = std::chrono::steady_clock::now();
    if ((rc = mpsl::dev_alloc(ctx, ctx->ybuf, len * sizeof(double2)))) return rc;
    if ((rc = mpsl::rhs_device(ctx, src, ctx->ybuf.p))) return rc;
    mpsl::SolveSM sm;
    if ((rc = sm.init(ctx, o, ctx->ybuf.p))) return rc;
    while (sm.status() == mpsl::SolveSM::kRunning) {
      if ((rc = sm.launch()) || (rc = sm.complete())) return rc;
    }
    MPSL_HIP_TRY(ctx, hipMemcpyAsync(beta_out + r * len, sm.x(), len * sizeof(double2), hipMemcpyDeviceToHost,
                                     ctx->stream));
    MPSL_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    const auto t1 = std::chrono::steady_clock::now();
    ctx->hist = sm.history();
    if (info) {
      info->iterations = sm.iterations();
      info->fp64_matvecs = sm.fp64_matvecs();
      info->refinements = sm.refinements();
      info->rel_residual = sm.rel_residual();
      info->seconds = std::chrono::duration<double>(t1 - t0).count();
      info->history = ctx->hist.data();
      info->history_len = static_cast<int>(ctx->hist.size());
      info->precond_seconds = sm.precond_seconds();
      info->reorthogonalizations = sm.reorthogonalizations();
    }
    if (sm.status() != mpsl::SolveSM::kConverged) status = MPSL_ENOCONV;
  }
  return status;
}

namespace {

// Total field of one source and its coefficients at n_rcv receivers.
int eval_field_one(mpsl_ctx *ctx, const double *src, const mpsl_c128 *beta, int64_t n_rcv, const double *rcv,
                   mpsl_c128 *u_out) {
  int rc = MPSL_OK;
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
  // amplitudes of every layer from the interface conditions, outward from the
  // particle layer (source amplitude referenced to the top interface)
  const int L = static_cast<int>(ctx->ks.size());
  std::vector<zc> gl(static_cast<size_t>(L) * ns), amp(static_cast<size_t>(2 * L) * ns);
  std::vector<zc> A(L), B(L), g(L);
  const zc I(0.0, 1.0);
  for (int q = 0; q < ns; ++q) {
    const zc lam = ctx->lam[q];
    const zc g0 = mpsl::gamma_branch(lam, ctx->k1);
    const zc gs = std::exp(-I * lam * src[0] - g0 * (src[1] - ctx->yint[0]));
    mpsl::stack_amplitudes(ctx, lam, gs, sig[q], sig[ns + q], spec[q], spec[ns + q], A.data(), B.data(), g.data());
    for (int j = 0; j < L; ++j) {
      gl[static_cast<size_t>(j) * ns + q] = g[j];
      amp[static_cast<size_t>(2 * j) * ns + q] = A[j];
      amp[static_cast<size_t>(2 * j + 1) * ns + q] = B[j];
    }
  }
  const size_t rb = static_cast<size_t>(n_rcv) * sizeof(double2);
  const size_t gb = gl.size() * sizeof(double2), ab = amp.size() * sizeof(double2);
  if ((rc = mpsl::dev_alloc(ctx, ctx->ybuf, 2 * rb + gb + ab + (L - 1) * sizeof(double)))) return rc;
  char *base = static_cast<char *>(ctx->ybuf.p);
  void *d_rcv = base;
  void *d_u = base + rb;
  void *d_gl = base + 2 * rb;
  void *d_amp = base + 2 * rb + gb;
  void *d_yint = base + 2 * rb + gb + ab;
  MPSL_HIP_TRY(ctx, hipMemcpyAsync(d_rcv, rcv, rb, hipMemcpyHostToDevice, ctx->stream));
  MPSL_HIP_TRY(ctx, hipMemcpyAsync(d_gl, gl.data(), gb, hipMemcpyHostToDevice, ctx->stream));
  MPSL_HIP_TRY(ctx, hipMemcpyAsync(d_amp, amp.data(), ab, hipMemcpyHostToDevice, ctx->stream));
  MPSL_HIP_TRY(ctx, hipMemcpyAsync(d_yint, ctx->yint.data(), (L - 1) * sizeof(double), hipMemcpyHostToDevice,
                                   ctx->stream));
  if ((rc = mpsl::launch_field(ctx, ctx->xbuf.p, d_gl, d_amp, d_yint, src, n_rcv, d_rcv, d_u))) return rc;
  MPSL_HIP_TRY(ctx, hipMemcpyAsync(u_out, d_u, rb, hipMemcpyDeviceToHost, ctx->stream));
  MPSL_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  for (int64_t i = 0; i < n_rcv; ++i)
    if (std::isnan(u_out[i].re)) return mpsl::set_err(ctx, MPSL_EINSIDE, "receiver inside an enclosing disk");
  return MPSL_OK;
}

}  // namespace

int mpsl_eval_field(mpsl_ctx *ctx, int n_rhs, const double *src_xy, const mpsl_c128 *beta, int64_t n_rcv,
                    const double *rcv_xy, mpsl_c128 *u_out) {
  if (!ctx || n_rhs < 1 || !src_xy || !beta || !rcv_xy || !u_out || n_rcv <= 0) return MPSL_EINVAL;
  MPSL_HIP_TRY(ctx, hipSetDevice(ctx->device));
  int rc = mpsl::build_tables(ctx);
  if (rc) return rc;
  for (int r = 0; r < n_rhs; ++r)
    if (!(src_xy[2 * r + 1] > ctx->yint[0]))
      return mpsl::set_err(ctx, MPSL_EINVAL, "every source must lie in the top half-space (above the top interface)");
  const int64_t len = ctx->n * static_cast<int64_t>(2 * ctx->p + 1);
  bool inside = false;
  for (int r = 0; r < n_rhs; ++r) {
    rc = eval_field_one(ctx, src_xy + 2 * r, beta + r * len, n_rcv, rcv_xy, u_out + r * n_rcv);
    if (rc == MPSL_EINSIDE) {
      inside = true;
    } else if (rc) {
      return rc;
    }
  }
  return inside ? mpsl::set_err(ctx, MPSL_EINSIDE, "receiver inside an enclosing disk") : MPSL_OK;
}

}  // extern "C"
