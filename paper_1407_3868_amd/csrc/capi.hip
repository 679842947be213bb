// C ABI of the mpsl library: context, problem setup (contour, Mie matrix,
// device tables) and the matvec and its steps.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <set>

#include "bie.h"
#include "kernels.h"

using mpsl::DBuf;
using mpsl::zc;

namespace mpsl {

int set_err(mpsl_ctx *ctx, int code, const std::string &msg) {
  if (ctx) ctx->err = msg;
  return code;
}

int check_unpinned(mpsl_ctx *ctx) {
  if (ctx->pinned > 0)
    return set_err(ctx, MPSL_ESTATE,
                   "a batch holds this context's buffers: destroy the batch before changing the context");
  return MPSL_OK;
}

int dev_alloc(mpsl_ctx *ctx, DBuf &b, size_t bytes) {
  if (bytes <= b.bytes && b.p) return MPSL_OK;
  // a captured batch reads the tables and matvec work buffers by address; only
  // the host-call staging and the solver's own buffers may move meanwhile
  if (ctx->pinned > 0 && &b != &ctx->xbuf && &b != &ctx->ybuf && &b != &ctx->gm && &b != &ctx->scal &&
      &b != &ctx->pc_blk && &b != &ctx->pc_blk32 && &b != &ctx->pc_idx && &b != &ctx->pc_part && &b != &ctx->pc_flag)
    return check_unpinned(ctx);
  dev_free(b);
  if (bytes == 0) return MPSL_OK;
  if (ctx->hbm_budget > 0 && ctx->hbm_used + bytes > ctx->hbm_budget)
    return set_err(ctx, MPSL_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes would exceed the " +
                                         "context's HBM budget (" + std::to_string(ctx->hbm_used) + " of " +
                                         std::to_string(ctx->hbm_budget) + " bytes in use)");
  if (hipMalloc(&b.p, bytes) != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    return set_err(ctx, MPSL_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  b.bytes = bytes;
  b.used = &ctx->hbm_used;
  ctx->hbm_used += bytes;
  return MPSL_OK;
}

void dev_free(DBuf &b) {
  if (b.p) {
    (void)hipFree(b.p);
    if (b.used) *b.used -= b.bytes;
  }
  b.p = nullptr;
  b.bytes = 0;
  b.used = nullptr;
}

namespace {

// 16-point Gauss-Legendre rule on [-1, 1] by Newton's method on P_16,
// ascending, symmetrised.
void gauss_legendre16(double *x, double *w) {
  const int n = 16;
  for (int i = 0; i < n / 2; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    const double wi = 2.0 / ((1.0 - z * z) * dp * dp);
    x[n - 1 - i] = z;  // z > 0 here
    x[i] = -z;
    w[n - 1 - i] = wi;
    w[i] = wi;
  }
}

// Panel end points on [0, t_max] for Gamma_1 (rule stated in mpsl.h).
bool panel_rule(int n_pan, double b, double t_max, const std::vector<double> &ks,
                std::vector<std::pair<double, double>> &panels) {
  std::vector<double> sing;
  for (double k : ks)
    if (k > 0.0 && k < t_max && std::find(sing.begin(), sing.end(), k) == sing.end()) sing.push_back(k);
  std::sort(sing.begin(), sing.end());
  std::vector<double> edges = {0.0, t_max};
  for (double s : sing) edges.push_back(s);
  std::sort(edges.begin(), edges.end());
  panels.clear();
  for (size_t i = 0; i + 1 < edges.size(); ++i) panels.emplace_back(edges[i], edges[i + 1]);
  if (static_cast<int>(panels.size()) > n_pan) return false;
  while (static_cast<int>(panels.size()) < n_pan) {
    int best = -1;
    double best_score = -1.0;
    for (size_t i = 0; i < panels.size(); ++i) {
      const double a = panels[i].first, c = panels[i].second;
      const double len = c - a;
      double dist = INFINITY;
      for (double s : sing) {
        const double dd = (s < a) ? (a - s) : ((s > c) ? (s - c) : 0.0);
        dist = std::min(dist, dd);
      }
      const double score = len / std::max(dist, b);
      // panels are kept sorted by left end, so the first maximum has the smallest a
      if (score > best_score) {
        best_score = score;
        best = static_cast<int>(i);
      }
    }
    const double a = panels[best].first, c = panels[best].second;
    const double mid = (a + c) / 2.0;
    panels.erase(panels.begin() + best);
    panels.emplace_back(a, mid);
    panels.emplace_back(mid, c);
    std::sort(panels.begin(), panels.end());
  }
  return true;
}


// Bessel J_n, Y_n of real argument for n >= 0 (C library), and derivatives.
void bessel_jy(int n, double x, double &j, double &y, double &jp, double &yp) {
  j = jn(n, x);
  y = yn(n, x);
  const double jm = (n == 0) ? -jn(1, x) : jn(n - 1, x);
  const double ym = (n == 0) ? -yn(1, x) : yn(n - 1, x);
  // Z_n' = Z_{n-1} - (n/x) Z_n
  jp = (n == 0) ? -jn(1, x) : jm - n / x * j;
  yp = (n == 0) ? -yn(1, x) : ym - n / x * y;
}

void invalidate(mpsl_ctx *ctx) {
  ctx->tables_ok = false;
  ctx->pc_ok = ctx->pc_ok32 = false;
}

}  // namespace

// Diagonal Mie scattering matrix of a disk (Section 3.1, eq. (18) with the
// denominator read as J_n(kp R)); S_{-n} = S_n.  TE weights the derivative
// condition by 1/k^2 of each side, so k2 and kp become 1/k2 and 1/kp where
// they multiply a derivative.
int disk_smatrix(double R, double k2, mpsl_c128 kp, int p, int pol, std::vector<zc> &S, std::string &err) {
  if (!(R > 0.0) || !(kp.re > 0.0) || p < kMinP || p > kMaxP) {
    err = "disk needs R > 0, kp > 0 and 1 <= p <= 20";
    return MPSL_EINVAL;
  }
  if (kp.im != 0.0) {
    err = "disk particles need a real kp";
    return MPSL_EUNSUPPORTED;
  }
  if (pol != MPSL_TM && pol != MPSL_TE) {
    err = "polarization must be MPSL_TM or MPSL_TE";
    return MPSL_EINVAL;
  }
  const int P = 2 * p + 1;
  const double kpr = kp.re;
  // derivative factors: k (TM) or k / k^2 (TE)
  const double c2 = (pol == MPSL_TE) ? 1.0 / k2 : k2, cp = (pol == MPSL_TE) ? 1.0 / kpr : kpr;
  S.assign(static_cast<size_t>(P) * P, zc(0.0, 0.0));
  for (int n = 0; n <= p; ++n) {
    double ja, ya, jap, yap, jb, yb, jbp, ybp;
    bessel_jy(n, k2 * R, ja, ya, jap, yap);
    bessel_jy(n, kpr * R, jb, yb, jbp, ybp);
    const zc H(ja, ya), Hp(jap, yap);
    const zc num = cp * ja * jbp - c2 * jap * jb;
    const zc den = c2 * Hp * jb - cp * jbp * H;
    const zc s = num / den;
    S[static_cast<size_t>(p + n) * P + (p + n)] = s;
    S[static_cast<size_t>(p - n) * P + (p - n)] = s;
  }
  return MPSL_OK;
}

int star_smatrix(double a1, double a2, int a3, double k2, double kp, int p, int nb, int pol, std::vector<zc> &S,
                 std::string &err);

// Argument rules of the star precompute; on success nb holds the boundary points.
int star_args(double a1, double a2, int a3, mpsl_c128 kp, int p, int n_bdry, int pol, int &nb, std::string &err) {
  if (pol != MPSL_TM && pol != MPSL_TE) {
    err = "polarization must be MPSL_TM or MPSL_TE";
    return MPSL_EINVAL;
  }
  if (!(a1 > 0.0) || !(std::fabs(a2) < a1) || a3 < 0 || !(kp.re > 0.0) || p < kMinP || p > kMaxP) {
    err = "star needs a1 > |a2|, a3 >= 0, kp > 0 and 1 <= p <= 20";
    return MPSL_EINVAL;
  }
  if (kp.im != 0.0) {
    err = "star particles need a real kp";
    return MPSL_EUNSUPPORTED;
  }
  nb = n_bdry > 0 ? n_bdry : 256;
  if (nb % 2 || nb < 64 || nb > 2048) {
    err = "n_bdry must be even, 64..2048";
    return MPSL_EINVAL;
  }
  return MPSL_OK;
}

int star_smatrix_checked(double a1, double a2, int a3, double k2, mpsl_c128 kp, int p, int n_bdry, int pol,
                         std::vector<zc> &S, std::string &err) {
  int nb = 0;
  const int rc = star_args(a1, a2, a3, kp, p, n_bdry, pol, nb, err);
  if (rc) return rc;
  return star_smatrix(a1, a2, a3, k2, kp.re, p, nb, pol, S, err);
}

// Gauss-Legendre nodes on the Gamma_1 panels, the mirrored Gamma_3 and the
// two Gamma_2 panels, in path order.
void assemble_contour(const std::vector<std::pair<double, double>> &pan, double b, std::vector<zc> &lam,
                      std::vector<zc> &w) {
  double gx[16], gwt[16];
  gauss_legendre16(gx, gwt);
  std::vector<double> t1, w1;
  for (const auto &pc : pan) {
    const double a = pc.first, c = pc.second;
    for (int i = 0; i < 16; ++i) {
      t1.push_back((a + c) / 2.0 + (c - a) / 2.0 * gx[i]);
      w1.push_back((c - a) / 2.0 * gwt[i]);
    }
  }
  const int n1 = static_cast<int>(t1.size());
  lam.clear();
  w.clear();
  for (int i = n1 - 1; i >= 0; --i) {  // Gamma_3: mirror of Gamma_1, path order
    lam.emplace_back(-t1[i], b);
    w.emplace_back(w1[i], 0.0);
  }
  for (int hh = 0; hh < 2; ++hh)  // Gamma_2: lambda = -i s, s in [-b, 0] then [0, b]
    for (int i = 0; i < 16; ++i) {
      const double s = (hh == 0 ? -b / 2.0 : b / 2.0) + b / 2.0 * gx[i];
      lam.emplace_back(0.0, -s);
      w.emplace_back(0.0, -b / 2.0 * gwt[i]);
    }
  for (int i = 0; i < n1; ++i) {
    lam.emplace_back(t1[i], -b);
    w.emplace_back(w1[i], 0.0);
  }
}

// Contour nodes and weights in path order (rule stated in mpsl.h).
int make_contour(const std::vector<double> &ks, int n_nodes, double b, double t_max, std::vector<zc> &lam,
                 std::vector<zc> &w, std::string &err) {
  if (n_nodes < 96 || (n_nodes - 32) % 32 != 0 || !(b > 0.0) || !(t_max > 0.0)) {
    err = "n_nodes = 32 + 32 m (m >= 2), b > 0, t_max > 0";
    return MPSL_EINVAL;
  }
  std::vector<std::pair<double, double>> pan;
  if (!panel_rule((n_nodes - 32) / 32, b, t_max, ks, pan)) {
    err = "too few nodes for the branch-point breakpoints";
    return MPSL_EINVAL;
  }
  assemble_contour(pan, b, lam, w);
  return MPSL_OK;
}

// Panels of bounded length on [0, t_max] (span rule stated in mpsl.h):
// branch-point breakpoints, grading towards each branch point from b, then
// every piece split into equal panels no longer than h_max.  Returns the
// panel count; fills pan only when it stays within max_panels.
int64_t span_panels(const std::vector<double> &ks, double b, double t_max, double h_max, int64_t max_panels,
                    std::vector<std::pair<double, double>> &pan) {
  std::set<double> sing, edges{0.0, t_max};
  for (double k : ks)
    if (k > 0.0 && k < t_max) sing.insert(k);
  edges.insert(sing.begin(), sing.end());
  std::vector<double> e(edges.begin(), edges.end());
  int64_t count = 0;
  pan.clear();
  for (size_t g = 0; g + 1 < e.size(); ++g) {
    const double a = e[g], c = e[g + 1], m = (a + c) / 2.0;
    const bool ga = sing.count(a) > 0, gc = sing.count(c) > 0;
    std::set<double> cuts{a, c};
    if (ga)
      for (double h = b; a + h < m; h *= 2.0) cuts.insert(a + h);
    if (gc)
      for (double h = b; c - h > m; h *= 2.0) cuts.insert(c - h);
    if (ga || gc) cuts.insert(m);
    std::vector<double> pts(cuts.begin(), cuts.end());
    for (size_t i = 0; i + 1 < pts.size(); ++i) {
      const double u = pts[i], v = pts[i + 1];
      const int64_t k = static_cast<int64_t>(std::ceil((v - u) / h_max));
      count += k;
      if (count > max_panels) continue;
      for (int64_t j = 0; j < k; ++j)
        pan.emplace_back(u + (v - u) * static_cast<double>(j) / static_cast<double>(k),
                         u + (v - u) * static_cast<double>(j + 1) / static_cast<double>(k));
    }
  }
  return count;
}

int make_contour_span(const std::vector<double> &ks, double b, double t_max, double h_max, std::vector<zc> &lam,
                      std::vector<zc> &w, std::string &err) {
  if (!(b > 0.0) || !(t_max > 0.0) || !(h_max > 0.0) || !std::isfinite(b) || !std::isfinite(t_max) ||
      !std::isfinite(h_max)) {
    err = "b, t_max and h_max must be positive and finite";
    return MPSL_EINVAL;
  }
  std::vector<std::pair<double, double>> pan;
  const int64_t max_panels = (kMaxNodes - 32) / 32;
  if (span_panels(ks, b, t_max, h_max, max_panels, pan) > max_panels) {
    err = "the span rule needs more than " + std::to_string(kMaxNodes) + " contour nodes";
    return MPSL_EINVAL;
  }
  assemble_contour(pan, b, lam, w);
  return MPSL_OK;
}

// gamma = sqrt(lam^2 - k^2), Re >= 0, and Im <= 0 on Re == 0.
zc gamma_branch(zc lam, zc k) {
  zc g = std::sqrt(lam * lam - k * k);
  if (g.real() < 0.0) g = -g;
  if (g.real() == 0.0 && g.imag() > 0.0) g = -g;
  return g;
}

// M2S order weights -4i (-i)^nu u^nu (side +) and -4i (-i)^nu v^nu (side -), and
// the S2L powers i^n u^n, i^n v^n, n = -p..p, with u = (lam - g2)/k2 and
// v = (lam + g2)/k2 = 1/u (Theorem 5.1, Lemma 5.1).  The larger of lam +- g2 is
// taken directly and the other as k2^2 / (...) to avoid cancellation.
void order_weights(zc lam, zc g2, zc k2, int p, zc *Wp, zc *Wm, zc *Up, zc *Um) {
  const zc I(0.0, 1.0);
  const int P = 2 * p + 1;
  zc u, v;
  if (std::abs(lam + g2) >= std::abs(lam - g2)) {
    v = (lam + g2) / k2;
    u = k2 / (lam + g2);
  } else {
    u = (lam - g2) / k2;
    v = k2 / (lam - g2);
  }
  // powers u^nu, v^nu for nu = -p..p by repeated multiplication from nu = 0
  std::vector<zc> up(P), vp(P);
  up[p] = vp[p] = 1.0;
  for (int j = 1; j <= p; ++j) {
    up[p + j] = up[p + j - 1] * u;
    up[p - j] = up[p - j + 1] * v;
    vp[p + j] = vp[p + j - 1] * v;
    vp[p - j] = vp[p - j + 1] * u;
  }
  for (int j = 0; j < P; ++j) {
    const int nu = j - p;
    const zc mi = std::pow(-I, nu), pi = std::pow(I, nu);  // (-i)^nu and i^nu
    Wp[j] = -4.0 * I * mi * up[j];
    Wm[j] = -4.0 * I * mi * vp[j];
    Up[j] = pi * up[j];
    Um[j] = pi * vp[j];
  }
}

// Contour tables (host, FP64) and geometry tables (device).
int build_tables(mpsl_ctx *ctx) {
  if (!ctx->has_layers || !ctx->has_particle || !ctx->has_geom || !ctx->has_contour)
    return set_err(ctx, MPSL_ESTATE, "layers, particle, geometry and contour must all be set");
  if (ctx->tables_ok) return MPSL_OK;
  if (ctx->somm_method == MPSL_SOMM_DIRECT && ctx->n * static_cast<int64_t>(ctx->ns) > kMaxPlaneWaves)
    return set_err(ctx, MPSL_EUNSUPPORTED,
                   "particles x contour nodes above " + std::to_string(kMaxPlaneWaves) + " (plane-wave tables)");
  const int ns = ctx->ns;
  const int p = ctx->p;
  const int P = 2 * p + 1;
  const int64_t n = ctx->n;
  const zc k1 = ctx->k1, k2 = ctx->k2, k3 = ctx->k3;

  std::vector<zc> R(4 * ns), sf(2 * ns), gw(4 * ns), cq(ns), W(2 * ns * P), U(2 * ns * P);
  for (int q = 0; q < ns; ++q) {
    const zc lam = ctx->lam[q];
    const zc g1 = gamma_branch(lam, k1), g2 = gamma_branch(lam, k2), g3 = gamma_branch(lam, k3);
    gw[q] = g1;
    gw[ns + q] = g2;
    gw[2 * ns + q] = g3;
    gw[3 * ns + q] = ctx->w[q];
    zc m[6];
    layer_map(ctx, lam, m);
    for (int i = 0; i < 4; ++i) R[4 * q + i] = m[i];
    sf[2 * q + 0] = m[4];
    sf[2 * q + 1] = m[5];
    cq[q] = ctx->w[q] / (4.0 * M_PI * g2);
    order_weights(lam, g2, k2, p, &W[(0 * ns + q) * P], &W[(1 * ns + q) * P], &U[(0 * ns + q) * P],
                  &U[(1 * ns + q) * P]);
  }
  auto up64 = [&](DBuf &b, const std::vector<zc> &v) -> int {
    int rc = dev_alloc(ctx, b, v.size() * sizeof(double2));
    if (rc) return rc;
    MPSL_HIP_TRY(ctx, hipMemcpy(b.p, v.data(), v.size() * sizeof(double2), hipMemcpyHostToDevice));
    return MPSL_OK;
  };
  auto up32 = [&](DBuf &b, const std::vector<zc> &v) -> int {
    std::vector<float2> f(v.size());
    for (size_t i = 0; i < v.size(); ++i)
      f[i] = make_float2(static_cast<float>(v[i].real()), static_cast<float>(v[i].imag()));
    int rc = dev_alloc(ctx, b, f.size() * sizeof(float2));
    if (rc) return rc;
    MPSL_HIP_TRY(ctx, hipMemcpy(b.p, f.data(), f.size() * sizeof(float2), hipMemcpyHostToDevice));
    return MPSL_OK;
  };
  int rc;
  if ((rc = up64(ctx->ct.R, R)) || (rc = up64(ctx->ct.srcfac, sf)) || (rc = up64(ctx->ct.lam, ctx->lam)) ||
      (rc = up64(ctx->ct.gw, gw)) || (rc = up64(ctx->ct.cq, cq)) || (rc = up64(ctx->ct.W64, W)) ||
      (rc = up32(ctx->ct.W32, W)) || (rc = up64(ctx->ct.U64, U)))
    return rc;

  // rotation phases e^{i n psi_l}
  std::vector<zc> rot(static_cast<size_t>(n) * P);
  for (int64_t l = 0; l < n; ++l)
    for (int j = 0; j < P; ++j) {
      const double a = (j - p) * ctx->rot[l];
      rot[l * P + j] = zc(std::cos(a), std::sin(a));
    }
  if ((rc = up64(ctx->gt.rot64, rot)) || (rc = up32(ctx->gt.rot32, rot))) return rc;

  if (ctx->somm_method == MPSL_SOMM_DIRECT) {  // per (particle, node) plane-wave tables
    const size_t tab = 2ull * static_cast<size_t>(n) * ns;
    if ((rc = dev_alloc(ctx, ctx->gt.E64, tab * sizeof(double2))) ||
        (rc = dev_alloc(ctx, ctx->gt.F64, tab * sizeof(double2))) ||
        (rc = dev_alloc(ctx, ctx->gt.E32, tab * sizeof(float2))) ||
        (rc = dev_alloc(ctx, ctx->gt.F32, tab * sizeof(float2))))
      return rc;
    if ((rc = launch_geom_tables(ctx))) return rc;
  } else {
    const DBuf *tabs[] = {&ctx->gt.E64, &ctx->gt.F64, &ctx->gt.E32, &ctx->gt.F32};
    for (const DBuf *t : tabs) dev_free(*const_cast<DBuf *>(t));
  }
  if ((rc = somm_build(ctx))) return rc;
  if (fmm_wanted(ctx)) {
    if ((rc = fmm_build(ctx))) return rc;
  } else if (!ctx->gt.pairs_ok) {
    const size_t np = static_cast<size_t>(n) * static_cast<size_t>(n) * 4;
    if ((rc = dev_alloc(ctx, ctx->gt.pair64, np * sizeof(double2))) ||
        (rc = dev_alloc(ctx, ctx->gt.pair32, np * sizeof(float2))))
      return rc;
    if ((rc = launch_pair_tables(ctx))) return rc;
    ctx->gt.pairs_ok = true;
  }
  if (!fmm_wanted(ctx)) ctx->fmm.active = false;
  MPSL_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  ctx->tables_ok = true;
  return ensure_work(ctx);
}

int ensure_work(mpsl_ctx *ctx) {
  const int P = 2 * ctx->p + 1;
  const size_t len = static_cast<size_t>(ctx->n) * P;
  const int ca = std::max(chunks_m2l(ctx, MPSL_FP64), chunks_m2l(ctx, MPSL_FP32));
  const int cb = std::max(chunks_s2l(ctx, 1, MPSL_FP64), chunks_s2l(ctx, 1, MPSL_FP32));
  const int cc = std::max(chunks_m2s(ctx, 1, MPSL_FP64), chunks_m2s(ctx, 1, MPSL_FP32));
  int rc;
  if ((rc = dev_alloc(ctx, ctx->part, (ca + cb) * len * sizeof(double2))) ||
      (rc = dev_alloc(ctx, ctx->m2s_part, 2ull * cc * ctx->ns * sizeof(double2))) ||
      (rc = dev_alloc(ctx, ctx->spec, 2ull * ctx->ns * sizeof(double2))) ||
      (rc = dev_alloc(ctx, ctx->sigma, 4ull * ctx->ns * sizeof(double2))) ||
      (rc = dev_alloc(ctx, ctx->Up64, 2ull * ctx->ns * P * sizeof(double2))) ||
      (rc = dev_alloc(ctx, ctx->Up32, 2ull * ctx->ns * P * sizeof(float2))) ||
      (rc = dev_alloc(ctx, ctx->scal, 64ull * 1024 * sizeof(double2))))
    return rc;
  return MPSL_OK;
}

// Y = X - S (T + T_R) X for nrhs right-hand sides ([nrhs][n][P]) on device
// buffers.  Work buffers grow on demand (never during graph capture: callers
// that capture run one call first).
int matvec(mpsl_ctx *ctx, int prec, const void *x, void *y, int nrhs) {
  int rc = build_tables(ctx);
  if (rc) return rc;
  if (nrhs < 1) return set_err(ctx, MPSL_EINVAL, "nrhs must be >= 1");
  // the right-hand-side dimension already multiplies the grid: fewer chunks
  // (the FMM writes its own partials: near-field chunks and far field)
  const bool fmm = ctx->fmm.active;
  // many FP32 right-hand sides: one Toeplitz GEMM per pair on the matrix cores
  const bool mrhs = !fmm && prec == MPSL_FP32 && nrhs >= kMrhsMin;
  const int ca = fmm ? fmm_slots(ctx)
                     : (mrhs ? chunks_m2l_mrhs(ctx, nrhs) : std::max(1, chunks_m2l(ctx, prec) / nrhs));
  const int cb = chunks_s2l(ctx, nrhs, prec);
  const int cc = chunks_m2s(ctx, nrhs, prec);
  const int P = 2 * ctx->p + 1;
  const size_t esz = prec == MPSL_FP64 ? sizeof(double2) : sizeof(float2);
  const int64_t len = ctx->n * static_cast<int64_t>(P);
  const int64_t pstride = static_cast<int64_t>(ca + cb) * len;
  if ((rc = dev_alloc(ctx, ctx->part, static_cast<size_t>(pstride) * nrhs * esz)) ||
      (rc = dev_alloc(ctx, ctx->m2s_part, 2ull * nrhs * cc * ctx->ns * sizeof(double2))) ||
      (rc = dev_alloc(ctx, ctx->spec, 2ull * nrhs * ctx->ns * sizeof(double2))) ||
      (rc = dev_alloc(ctx, ctx->sigma, std::max(4ull, 2ull * nrhs) * ctx->ns * sizeof(double2))) ||
      (rc = dev_alloc(ctx, ctx->Up64, 2ull * nrhs * ctx->ns * P * sizeof(double2))) ||
      (rc = dev_alloc(ctx, ctx->Up32, 2ull * nrhs * ctx->ns * P * sizeof(float2))))
    return rc;
  char *part = static_cast<char *>(ctx->part.p);
  char *part_b = part + static_cast<size_t>(ca) * len * esz;
  if ((rc = launch_m2s(ctx, prec, x, ctx->spec.p, nrhs))) return rc;
  if ((rc = launch_reflect(ctx, ctx->spec.p, nullptr, ctx->sigma.p, nrhs))) return rc;
  if ((rc = launch_s2l_coef(ctx, ctx->sigma.p, nrhs))) return rc;
  if ((rc = launch_s2l(ctx, prec, part_b, cb, nrhs, pstride))) return rc;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ctx->prof) {
    MPSL_HIP_TRY(ctx, hipEventCreate(&e0));
    MPSL_HIP_TRY(ctx, hipEventCreate(&e1));
    MPSL_HIP_TRY(ctx, hipEventRecord(e0, ctx->stream));
  }
  if (fmm) {
    for (int r = 0; r < nrhs; ++r)
      if ((rc = fmm_apply(ctx, prec, static_cast<const char *>(x) + static_cast<size_t>(r) * len * esz,
                          part + static_cast<size_t>(r) * pstride * esz)))
        return rc;
  } else if (mrhs) {
    if ((rc = launch_m2l_mrhs(ctx, x, part, ca, nrhs, pstride))) return rc;
  } else if ((rc = launch_m2l(ctx, prec, x, part, ca, -1, nrhs, pstride))) {
    return rc;
  }
  if (ctx->prof) {
    MPSL_HIP_TRY(ctx, hipEventRecord(e1, ctx->stream));
    ctx->ev_start.push_back(e0);
    ctx->ev_stop.push_back(e1);
  }
  if ((rc = launch_fold_parts(ctx, prec, part, ca + cb, nrhs, pstride))) return rc;
  return launch_sapply(ctx, prec, x, part, y, nrhs, pstride);
}

int matvec(mpsl_ctx *ctx, int prec, const void *x, void *y) { return matvec(ctx, prec, x, y, 1); }

}  // namespace mpsl

// ---------------------------------------------------------------------------
// Fixed device scratch of the allocation-free M2L (mpsl_m2l_dev_noalloc): the
// partial local expansions of its source chunks.  Each device holds its own
// copy for the life of the process; host code uses only the address that
// hipGetSymbolAddress returns for the current device (the array's name is a
// host-side stand-in there).
namespace {
constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB
static __device__ __align__(256) double2 scratch[kScratchBytes / sizeof(double2)];
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchDevices] = {};

// Look the array up once per device, with that device current.
int scratch_setup(int device) {
  if (device < 0 || device >= kScratchDevices) return MPSL_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return MPSL_OK;
  void *p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
    (void)hipGetLastError();
    return MPSL_EHIP;
  }
  g_scratch_ptr[device] = p;
  return MPSL_OK;
}

void *scratch_ptr(int device) {
  if (device < 0 || device >= kScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}
}  // namespace

// ===========================================================================
extern "C" {

const char *mpsl_status_string(int s) {
  switch (s) {
    case MPSL_OK: return "ok";
    case MPSL_EINVAL: return "invalid argument";
    case MPSL_ENOMEM: return "out of memory";
    case MPSL_EHIP: return "HIP runtime error";
    case MPSL_ESTATE: return "missing setup call";
    case MPSL_EGEOM: return "invalid geometry";
    case MPSL_ENOCONV: return "GMRES did not converge";
    case MPSL_EUNSUPPORTED: return "unsupported parameters";
    case MPSL_EINSIDE: return "receiver inside an enclosing disk";
    case MPSL_ENUMERIC: return "non-finite value in iteration";
    default: return "unknown status";
  }
}

const char *mpsl_last_error(const mpsl_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int mpsl_create(mpsl_ctx **out, int device, size_t hbm_budget) {
  if (!out) return MPSL_EINVAL;
  *out = nullptr;
  int cnt = 0;
  if (hipGetDeviceCount(&cnt) != hipSuccess || cnt <= 0) {
    (void)hipGetLastError();
    return MPSL_EHIP;
  }
  if (device < 0 || device >= cnt) return MPSL_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return MPSL_EHIP;
  if (const int rc = scratch_setup(device)) return rc;
  mpsl_ctx *ctx = new (std::nothrow) mpsl_ctx();
  if (!ctx) return MPSL_ENOMEM;
  ctx->device = device;
  ctx->hbm_budget = hbm_budget;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
    ctx->n_cu = cus;
  (void)hipGetLastError();
  *out = ctx;
  return MPSL_OK;
}

int mpsl_get_memory(const mpsl_ctx *ctx, size_t *bytes_in_use, size_t *hbm_budget) {
  if (!ctx) return MPSL_EINVAL;
  if (bytes_in_use) *bytes_in_use = ctx->hbm_used;
  if (hbm_budget) *hbm_budget = ctx->hbm_budget;
  return MPSL_OK;
}

void mpsl_destroy(mpsl_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto e : ctx->ev_start) (void)hipEventDestroy(e);
  for (auto e : ctx->ev_stop) (void)hipEventDestroy(e);
  DBuf *bufs[] = {&ctx->bt, &ctx->S64, &ctx->S32, &ctx->types_dev, &ctx->rtype_dev, &ctx->ct.R, &ctx->ct.srcfac, &ctx->ct.lam, &ctx->ct.gw,
                  &ctx->ct.cq, &ctx->ct.W64, &ctx->ct.W32, &ctx->ct.U64, &ctx->gt.xy, &ctx->gt.rot64,
                  &ctx->gt.rot32, &ctx->gt.pair64, &ctx->gt.pair32, &ctx->gt.E64, &ctx->gt.E32, &ctx->gt.F64, &ctx->gt.F32, &ctx->part,
                  &ctx->m2s_part, &ctx->spec, &ctx->sigma, &ctx->Up64, &ctx->Up32, &ctx->xbuf,
                  &ctx->ybuf, &ctx->gm, &ctx->scal, &ctx->pc_blk, &ctx->pc_blk32, &ctx->pc_idx, &ctx->pc_part,
                  &ctx->pc_flag};
  for (DBuf *b : bufs) mpsl::dev_free(*b);
  mpsl::fmm_free(ctx);
  mpsl::somm_free(ctx);
  delete ctx;
}

int mpsl_set_stream(mpsl_ctx *ctx, void *stream) {
  if (!ctx) return MPSL_EINVAL;
  ctx->stream = static_cast<hipStream_t>(stream);
  return MPSL_OK;
}

int mpsl_set_layer_stack(mpsl_ctx *ctx, int n_layers, const mpsl_c128 *k, const double *thickness,
                         int particle_layer) {
  if (!ctx) return MPSL_EINVAL;
  if (const int pe = mpsl::check_unpinned(ctx)) return pe;
  std::string err;
  const int rc = mpsl::assign_stack(ctx, n_layers, k, thickness, particle_layer, err);
  if (rc) return mpsl::set_err(ctx, rc, err);
  ctx->has_layers = true;
  ctx->gt.pairs_ok = false;
  mpsl::invalidate(ctx);
  return MPSL_OK;
}

int mpsl_compute_layer_map(int n_layers, const mpsl_c128 *k, const double *thickness, int particle_layer,
                           int polarization, int n_lam, const mpsl_c128 *lam, mpsl_c128 *map) {
  if (!lam || !map || n_lam <= 0) return MPSL_EINVAL;
  if (polarization != MPSL_TM && polarization != MPSL_TE) return MPSL_EINVAL;
  mpsl_ctx tmp;
  tmp.pol = polarization;
  std::string err;
  const int rc = mpsl::assign_stack(&tmp, n_layers, k, thickness, particle_layer, err);
  if (rc) return rc;
  for (int q = 0; q < n_lam; ++q) {
    const zc l(lam[q].re, lam[q].im);
    if (!std::isfinite(l.real()) || !std::isfinite(l.imag())) return MPSL_EINVAL;
    zc m[6];
    mpsl::layer_map(&tmp, l, m);
    for (int i = 0; i < 6; ++i) map[6 * q + i] = {m[i].real(), m[i].imag()};
  }
  return MPSL_OK;
}

int mpsl_set_polarization(mpsl_ctx *ctx, int polarization) {
  if (!ctx) return MPSL_EINVAL;
  if (const int pe = mpsl::check_unpinned(ctx)) return pe;
  if (polarization != MPSL_TM && polarization != MPSL_TE)
    return mpsl::set_err(ctx, MPSL_EINVAL, "polarization must be MPSL_TM or MPSL_TE");
  if (polarization == ctx->pol) return MPSL_OK;
  ctx->pol = polarization;
  ctx->has_particle = false;  // its scattering matrix belongs to the other polarisation
  mpsl::invalidate(ctx);
  return MPSL_OK;
}

int mpsl_get_polarization(const mpsl_ctx *ctx) { return ctx ? ctx->pol : MPSL_EINVAL; }

int mpsl_set_layers(mpsl_ctx *ctx, mpsl_c128 k1, mpsl_c128 k2, mpsl_c128 k3, double d) {
  if (!ctx) return MPSL_EINVAL;
  const mpsl_c128 ks[3] = {k1, k2, k3};
  const double th[3] = {0.0, d, 0.0};
  return mpsl_set_layer_stack(ctx, 3, ks, th, 1);
}

static int upload_S(mpsl_ctx *ctx) {
  const size_t PP = ctx->S.size();
  std::vector<float2> f(PP);
  for (size_t i = 0; i < PP; ++i)
    f[i] = make_float2(static_cast<float>(ctx->S[i].real()), static_cast<float>(ctx->S[i].imag()));
  int rc;
  if ((rc = mpsl::dev_alloc(ctx, ctx->S64, PP * sizeof(double2))) ||
      (rc = mpsl::dev_alloc(ctx, ctx->S32, PP * sizeof(float2))))
    return rc;
  MPSL_HIP_TRY(ctx, hipMemcpy(ctx->S64.p, ctx->S.data(), PP * sizeof(double2), hipMemcpyHostToDevice));
  MPSL_HIP_TRY(ctx, hipMemcpy(ctx->S32.p, f.data(), PP * sizeof(float2), hipMemcpyHostToDevice));
  return MPSL_OK;
}

// Install n_types prototype matrices (n_types x P x P in S) with their
// enclosing radii.  A geometry whose type ids no longer fit is dropped.
static int install_prototypes(mpsl_ctx *ctx, int p, int n_types, const std::vector<double> &r_type,
                              std::vector<zc> &&S) {
  ctx->p = p;
  ctx->n_types = n_types;
  ctx->r_type = r_type;
  ctx->r_enc = *std::max_element(r_type.begin(), r_type.end());
  ctx->S = std::move(S);
  int rc = upload_S(ctx);
  if (rc) return rc;
  if ((rc = mpsl::dev_alloc(ctx, ctx->rtype_dev, n_types * sizeof(double)))) return rc;
  MPSL_HIP_TRY(ctx, hipMemcpy(ctx->rtype_dev.p, r_type.data(), n_types * sizeof(double), hipMemcpyHostToDevice));
  for (int32_t t : ctx->ptype)
    if (t >= n_types) {
      ctx->ptype.clear();
      ctx->has_geom = false;
      break;
    }
  ctx->has_particle = true;
  mpsl::invalidate(ctx);
  return MPSL_OK;
}

int mpsl_set_particle_disk(mpsl_ctx *ctx, double R, mpsl_c128 kp, int p) {
  if (!ctx) return MPSL_EINVAL;
  if (const int pe = mpsl::check_unpinned(ctx)) return pe;
  if (!ctx->has_layers) return mpsl::set_err(ctx, MPSL_ESTATE, "set_layers first");
  std::vector<zc> S;
  std::string err;
  const int rc0 = mpsl::disk_smatrix(R, ctx->k2.real(), kp, p, ctx->pol, S, err);
  if (rc0) return mpsl::set_err(ctx, rc0, err);
  return install_prototypes(ctx, p, 1, {R}, std::move(S));
}

int mpsl_set_particle_star(mpsl_ctx *ctx, double a1, double a2, int a3, mpsl_c128 kp, int p, int n_bdry) {
  if (!ctx) return MPSL_EINVAL;
  if (const int pe = mpsl::check_unpinned(ctx)) return pe;
  if (!ctx->has_layers) return mpsl::set_err(ctx, MPSL_ESTATE, "set_layers first");
  std::vector<zc> S;
  std::string err;
  int nb = 0;
  int rc0 = mpsl::star_args(a1, a2, a3, kp, p, n_bdry, ctx->pol, nb, err);
  if (rc0) return mpsl::set_err(ctx, rc0, err);
  // host boundary tables, device assembly and solve
  mpsl::StarParts parts;
  MPSL_HIP_TRY(ctx, hipSetDevice(ctx->device));
  if ((rc0 = mpsl::star_parts(a1, a2, a3, ctx->k2.real(), p, nb, parts, err)) ||
      (rc0 = mpsl::star_smatrix_device(ctx, parts, ctx->k2.real(), kp.re, ctx->pol, S, err)))
    return mpsl::set_err(ctx, rc0, err);
  return install_prototypes(ctx, p, 1, {a1 + std::fabs(a2)}, std::move(S));
}

int mpsl_compute_disk_smatrix(double R, mpsl_c128 k2, mpsl_c128 kp, int p, int polarization, mpsl_c128 *S) {
  if (!S || k2.im != 0.0 || !(k2.re > 0.0)) return MPSL_EINVAL;
  std::vector<zc> v;
  std::string err;
  const int rc = mpsl::disk_smatrix(R, k2.re, kp, p, polarization, v, err);
  if (rc) return rc;
  for (size_t i = 0; i < v.size(); ++i) S[i] = {v[i].real(), v[i].imag()};
  return MPSL_OK;
}

int mpsl_compute_star_smatrix(double a1, double a2, int a3, mpsl_c128 k2, mpsl_c128 kp, int p, int n_bdry,
                              int polarization, mpsl_c128 *S) {
  if (!S || k2.im != 0.0 || !(k2.re > 0.0)) return MPSL_EINVAL;
  std::vector<zc> v;
  std::string err;
  const int rc = mpsl::star_smatrix_checked(a1, a2, a3, k2.re, kp, p, n_bdry, polarization, v, err);
  if (rc) return rc;
  for (size_t i = 0; i < v.size(); ++i) S[i] = {v[i].real(), v[i].imag()};
  return MPSL_OK;
}

int mpsl_set_particle_types(mpsl_ctx *ctx, int n_types, int p, const double *r_enclose, const mpsl_c128 *S) {
  if (!ctx || !S || !r_enclose) return MPSL_EINVAL;
  if (const int pe = mpsl::check_unpinned(ctx)) return pe;
  if (n_types < 1 || n_types > mpsl::kMaxTypes)
    return mpsl::set_err(ctx, MPSL_EINVAL, "need 1 to " + std::to_string(mpsl::kMaxTypes) + " particle types");
  if (p < mpsl::kMinP || p > mpsl::kMaxP) return mpsl::set_err(ctx, MPSL_EINVAL, "need 1 <= p <= 20");
  std::vector<double> r(r_enclose, r_enclose + n_types);
  for (double v : r)
    if (!(v > 0.0) || !std::isfinite(v)) return mpsl::set_err(ctx, MPSL_EINVAL, "enclosing radii must be > 0");
  const int P = 2 * p + 1;
  std::vector<zc> v(static_cast<size_t>(n_types) * P * P);
  for (size_t i = 0; i < v.size(); ++i) {
    if (!std::isfinite(S[i].re) || !std::isfinite(S[i].im))
      return mpsl::set_err(ctx, MPSL_EINVAL, "scattering matrix has non-finite entries");
    v[i] = zc(S[i].re, S[i].im);
  }
  return install_prototypes(ctx, p, n_types, r, std::move(v));
}

int mpsl_set_scattering_matrix(mpsl_ctx *ctx, int p, double r_enclose, const mpsl_c128 *S) {
  return mpsl_set_particle_types(ctx, 1, p, &r_enclose, S);
}

int mpsl_set_geometry_typed(mpsl_ctx *ctx, int64_t n, const double *xy, const double *rot, const int32_t *type) {
  if (!ctx || !xy || n <= 0) return MPSL_EINVAL;
  if (const int pe = mpsl::check_unpinned(ctx)) return pe;
  if (!ctx->has_layers || !ctx->has_particle) return mpsl::set_err(ctx, MPSL_ESTATE, "layers and particle first");
  if (n > (int64_t(1) << 30)) return mpsl::set_err(ctx, MPSL_EINVAL, "too many particles");
  const double d = ctx->d, rmax = ctx->r_enc;
  std::vector<int32_t> ty(static_cast<size_t>(n), 0);
  if (type)
    for (int64_t j = 0; j < n; ++j) {
      if (type[j] < 0 || type[j] >= ctx->n_types)
        return mpsl::set_err(ctx, MPSL_EINVAL, "particle " + std::to_string(j) + " has no such type");
      ty[j] = type[j];
    }
  auto rad = [&](int64_t j) { return ctx->r_type[ty[j]]; };
  for (int64_t j = 0; j < n; ++j) {
    const double x = xy[2 * j], y = xy[2 * j + 1];
    if (!std::isfinite(x) || !std::isfinite(y) || (rot && !std::isfinite(rot[j])))
      return mpsl::set_err(ctx, MPSL_EINVAL, "non-finite centre or rotation");
    if (y + rad(j) > 0.0 || y - rad(j) < -d)
      return mpsl::set_err(ctx, MPSL_EGEOM, "particle " + std::to_string(j) + " leaves the middle layer");
  }
  // enclosing disks must be disjoint: sweep in x
  std::vector<int64_t> ord(n);
  for (int64_t j = 0; j < n; ++j) ord[j] = j;
  std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return xy[2 * a] < xy[2 * b]; });
  for (int64_t a = 0; a < n; ++a) {
    const int64_t i = ord[a];
    for (int64_t b = a + 1; b < n; ++b) {
      const int64_t j = ord[b];
      const double dx = xy[2 * j] - xy[2 * i];
      if (dx >= rad(i) + rmax) break;
      const double dy = xy[2 * j + 1] - xy[2 * i + 1];
      const double rr = rad(i) + rad(j);
      if (dx * dx + dy * dy < rr * rr)
        return mpsl::set_err(ctx, MPSL_EGEOM,
                             "enclosing disks of particles " + std::to_string(i) + " and " + std::to_string(j) +
                                 " overlap");
    }
  }
  ctx->n = n;
  ctx->xy.assign(xy, xy + 2 * n);
  ctx->rot.assign(static_cast<size_t>(n), 0.0);
  if (rot) ctx->rot.assign(rot, rot + n);
  int rc = mpsl::dev_alloc(ctx, ctx->gt.xy, static_cast<size_t>(n) * sizeof(double2));
  if (rc) return rc;
  MPSL_HIP_TRY(ctx, hipMemcpy(ctx->gt.xy.p, xy, static_cast<size_t>(n) * sizeof(double2), hipMemcpyHostToDevice));
  ctx->ptype.clear();
  if (ctx->n_types > 1) {
    ctx->ptype = ty;
    if ((rc = mpsl::dev_alloc(ctx, ctx->types_dev, static_cast<size_t>(n) * sizeof(int32_t)))) return rc;
    MPSL_HIP_TRY(ctx, hipMemcpy(ctx->types_dev.p, ty.data(), static_cast<size_t>(n) * sizeof(int32_t),
                                hipMemcpyHostToDevice));
  }
  ctx->has_geom = true;
  ctx->gt.pairs_ok = false;
  mpsl::invalidate(ctx);
  return MPSL_OK;
}

int mpsl_set_geometry(mpsl_ctx *ctx, int64_t n, const double *xy, const double *rot) {
  return mpsl_set_geometry_typed(ctx, n, xy, rot, nullptr);
}

int mpsl_set_contour(mpsl_ctx *ctx, int n_nodes, double b, double t_max) {
  if (!ctx) return MPSL_EINVAL;
  if (const int pe = mpsl::check_unpinned(ctx)) return pe;
  if (!ctx->has_layers) return mpsl::set_err(ctx, MPSL_ESTATE, "set_layers first");
  std::vector<zc> lam, w;
  std::string err;
  std::vector<double> kr;
  for (const zc &k : ctx->ks) kr.push_back(k.real());
  const int rc = mpsl::make_contour(kr, n_nodes, b, t_max, lam, w, err);
  if (rc) return mpsl::set_err(ctx, rc, err);
  ctx->lam = lam;
  ctx->w = w;
  ctx->ns = n_nodes;
  ctx->has_contour = true;
  mpsl::invalidate(ctx);
  return MPSL_OK;
}

int mpsl_compute_contour(mpsl_c128 k1, mpsl_c128 k2, mpsl_c128 k3, int n_nodes, double b, double t_max,
                         mpsl_c128 *lam, mpsl_c128 *w) {
  if (!lam || !w) return MPSL_EINVAL;
  std::vector<zc> l, ww;
  std::string err;
  const int rc = mpsl::make_contour({k1.re, k2.re, k3.re}, n_nodes, b, t_max, l, ww, err);
  if (rc) return rc;
  for (int i = 0; i < n_nodes; ++i) {
    lam[i] = {l[i].real(), l[i].imag()};
    w[i] = {ww[i].real(), ww[i].imag()};
  }
  return MPSL_OK;
}

int mpsl_set_contour_span(mpsl_ctx *ctx, double b, double t_max, double h_max) {
  if (!ctx) return MPSL_EINVAL;
  if (const int pe = mpsl::check_unpinned(ctx)) return pe;
  if (!ctx->has_layers) return mpsl::set_err(ctx, MPSL_ESTATE, "set_layers first");
  std::vector<zc> lam, w;
  std::string err;
  std::vector<double> kr;
  for (const zc &k : ctx->ks) kr.push_back(k.real());
  const int rc = mpsl::make_contour_span(kr, b, t_max, h_max, lam, w, err);
  if (rc) return mpsl::set_err(ctx, rc, err);
  ctx->lam = lam;
  ctx->w = w;
  ctx->ns = static_cast<int>(lam.size());
  ctx->has_contour = true;
  mpsl::invalidate(ctx);
  return MPSL_OK;
}

int mpsl_span_contour_params(double x_extent, double tol, double *b, double *h_max) {
  if (!b || !h_max || !std::isfinite(x_extent) || !(tol > 0.0) || !std::isfinite(tol)) return MPSL_EINVAL;
  const double X = std::max(x_extent, 1.0);
  *b = std::min(0.2, 2.0 / X);
  *h_max = (tol <= 1e-8 ? 6.0 : 12.0) / X;
  return MPSL_OK;
}

int mpsl_set_sommerfeld_method(mpsl_ctx *ctx, int method) {
  if (!ctx) return MPSL_EINVAL;
  if (const int pe = mpsl::check_unpinned(ctx)) return pe;
  if (method != MPSL_SOMM_DIRECT && method != MPSL_SOMM_INTERP)
    return mpsl::set_err(ctx, MPSL_EINVAL, "method must be MPSL_SOMM_DIRECT or MPSL_SOMM_INTERP");
  if (method == ctx->somm_method) return MPSL_OK;
  ctx->somm_method = method;
  mpsl::invalidate(ctx);
  return MPSL_OK;
}

int mpsl_compute_contour_span(int n_k, const double *re_k, double b, double t_max, double h_max, int capacity,
                              mpsl_c128 *lam, mpsl_c128 *w, int *n_nodes) {
  if (!re_k || n_k <= 0 || !n_nodes) return MPSL_EINVAL;
  std::vector<double> kr(re_k, re_k + n_k);
  std::vector<zc> l, ww;
  std::string err;
  const int rc = mpsl::make_contour_span(kr, b, t_max, h_max, l, ww, err);
  if (rc) return rc;
  *n_nodes = static_cast<int>(l.size());
  if (!lam && !w) return MPSL_OK;
  if (!lam || !w || capacity < *n_nodes) return MPSL_EINVAL;
  for (int i = 0; i < *n_nodes; ++i) {
    lam[i] = {l[i].real(), l[i].imag()};
    w[i] = {ww[i].real(), ww[i].imag()};
  }
  return MPSL_OK;
}

int mpsl_set_contour_nodes(mpsl_ctx *ctx, int n_nodes, const mpsl_c128 *lam, const mpsl_c128 *w) {
  if (!ctx || !lam || !w || n_nodes <= 0) return MPSL_EINVAL;
  if (const int pe = mpsl::check_unpinned(ctx)) return pe;
  if (n_nodes > mpsl::kMaxNodes) return mpsl::set_err(ctx, MPSL_EINVAL, "too many contour nodes");
  ctx->lam.resize(n_nodes);
  ctx->w.resize(n_nodes);
  for (int i = 0; i < n_nodes; ++i) {
    ctx->lam[i] = zc(lam[i].re, lam[i].im);
    ctx->w[i] = zc(w[i].re, w[i].im);
  }
  ctx->ns = n_nodes;
  ctx->has_contour = true;
  mpsl::invalidate(ctx);
  return MPSL_OK;
}

int mpsl_get_contour(const mpsl_ctx *ctx, int n_nodes, mpsl_c128 *lam, mpsl_c128 *w) {
  if (!ctx || !ctx->has_contour || n_nodes != ctx->ns) return MPSL_EINVAL;
  for (int i = 0; i < n_nodes; ++i) {
    if (lam) lam[i] = {ctx->lam[i].real(), ctx->lam[i].imag()};
    if (w) w[i] = {ctx->w[i].real(), ctx->w[i].imag()};
  }
  return MPSL_OK;
}

int mpsl_get_scattering_matrix(const mpsl_ctx *ctx, int p, mpsl_c128 *S) {
  if (!ctx || !S || !ctx->has_particle || p != ctx->p) return MPSL_EINVAL;
  for (size_t i = 0; i < ctx->S.size(); ++i) S[i] = {ctx->S[i].real(), ctx->S[i].imag()};
  return MPSL_OK;
}

int mpsl_get_sizes(const mpsl_ctx *ctx, int64_t *n, int *p, int *n_nodes) {
  if (!ctx) return MPSL_EINVAL;
  if (n) *n = ctx->n;
  if (p) *p = ctx->p;
  if (n_nodes) *n_nodes = ctx->ns;
  return MPSL_OK;
}

int mpsl_apply_dev(mpsl_ctx *ctx, int prec, const void *x, void *y) {
  if (!ctx || !x || !y || (prec != MPSL_FP64 && prec != MPSL_FP32)) return MPSL_EINVAL;
  MPSL_HIP_TRY(ctx, hipSetDevice(ctx->device));
  return mpsl::matvec(ctx, prec, x, y);
}

int mpsl_apply_batch_dev(mpsl_ctx *ctx, int prec, int nrhs, const void *x, void *y) {
  if (!ctx || !x || !y || nrhs < 1 || (prec != MPSL_FP64 && prec != MPSL_FP32)) return MPSL_EINVAL;
  MPSL_HIP_TRY(ctx, hipSetDevice(ctx->device));
  return mpsl::matvec(ctx, prec, x, y, nrhs);
}

int mpsl_apply(mpsl_ctx *ctx, int prec, const void *x, void *y) {
  if (!ctx || !x || !y || (prec != MPSL_FP64 && prec != MPSL_FP32)) return MPSL_EINVAL;
  MPSL_HIP_TRY(ctx, hipSetDevice(ctx->device));
  int rc = mpsl::build_tables(ctx);
  if (rc) return rc;
  const size_t bytes = static_cast<size_t>(ctx->n) * (2 * ctx->p + 1) *
                       (prec == MPSL_FP64 ? sizeof(double2) : sizeof(float2));
  if ((rc = mpsl::dev_alloc(ctx, ctx->xbuf, bytes)) || (rc = mpsl::dev_alloc(ctx, ctx->ybuf, bytes))) return rc;
  MPSL_HIP_TRY(ctx, hipMemcpyAsync(ctx->xbuf.p, x, bytes, hipMemcpyHostToDevice, ctx->stream));
  if ((rc = mpsl::matvec(ctx, prec, ctx->xbuf.p, ctx->ybuf.p))) return rc;
  MPSL_HIP_TRY(ctx, hipMemcpyAsync(y, ctx->ybuf.p, bytes, hipMemcpyDeviceToHost, ctx->stream));
  MPSL_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return MPSL_OK;
}

int mpsl_m2l_dev(mpsl_ctx *ctx, int prec, const void *beta, void *alpha) {
  if (!ctx || !beta || !alpha || (prec != MPSL_FP64 && prec != MPSL_FP32)) return MPSL_EINVAL;
  MPSL_HIP_TRY(ctx, hipSetDevice(ctx->device));
  int rc = mpsl::build_tables(ctx);
  if (rc) return rc;
  const bool fmm = ctx->fmm.active;
  const int ca = fmm ? mpsl::fmm_slots(ctx) : mpsl::chunks_m2l(ctx, prec);
  const size_t esz = prec == MPSL_FP64 ? sizeof(double2) : sizeof(float2);
  if ((rc = mpsl::dev_alloc(ctx, ctx->part, static_cast<size_t>(ca) * ctx->n * (2 * ctx->p + 1) * esz))) return rc;
  if (fmm) {
    if ((rc = mpsl::fmm_apply(ctx, prec, beta, ctx->part.p))) return rc;
  } else if ((rc = mpsl::launch_m2l(ctx, prec, beta, ctx->part.p, ca))) {
    return rc;
  }
  return mpsl::launch_sum_parts(ctx, prec, ctx->part.p, ca, alpha);
}

int mpsl_m2l_dev_noalloc(mpsl_ctx *ctx, int prec, const void *beta, void *alpha) {
  if (!ctx || !beta || !alpha || (prec != MPSL_FP64 && prec != MPSL_FP32)) return MPSL_EINVAL;
  MPSL_HIP_TRY(ctx, hipSetDevice(ctx->device));
  if (!ctx->has_layers || !ctx->has_particle || !ctx->has_geom)
    return mpsl::set_err(ctx, MPSL_ESTATE, "layers, particle and geometry first");
  const size_t esz = prec == MPSL_FP64 ? sizeof(double2) : sizeof(float2);
  const size_t slot = static_cast<size_t>(ctx->n) * (2 * ctx->p + 1) * esz;
  if (slot > kScratchBytes)
    return mpsl::set_err(ctx, MPSL_EINVAL,
                         "N P = " + std::to_string(ctx->n * (2 * ctx->p + 1)) + " needs " + std::to_string(slot) +
                             " bytes per partial expansion, above the " + std::to_string(kScratchBytes) +
                             "-byte scratch of the allocation-free M2L");
  if (!ctx->tables_ok || !ctx->gt.pairs_ok)
    return mpsl::set_err(ctx, MPSL_ESTATE, "tables not built: call mpsl_m2l_dev or mpsl_apply_dev once first");
  if (ctx->fmm.active)
    return mpsl::set_err(ctx, MPSL_EUNSUPPORTED, "the allocation-free M2L is the direct all-pairs form (FMM active)");
  void *scr = scratch_ptr(ctx->device);
  if (!scr) return mpsl::set_err(ctx, MPSL_ESTATE, "device scratch not set up");
  // as many source chunks as the default launch shape asks for, while their
  // partial slots fit; every slot is written in full by the M2L (empty
  // chunks write zeros), so nothing needs clearing
  const int ca = static_cast<int>(std::max<size_t>(
      1, std::min<size_t>(static_cast<size_t>(mpsl::chunks_m2l(ctx, prec)), kScratchBytes / slot)));
  int rc;
  if ((rc = mpsl::launch_m2l(ctx, prec, beta, scr, ca))) return rc;
  return mpsl::launch_sum_parts(ctx, prec, scr, ca, alpha);
}

int mpsl_m2s_dev(mpsl_ctx *ctx, int prec, const void *beta, void *spec) {
  if (!ctx || !beta || !spec || (prec != MPSL_FP64 && prec != MPSL_FP32)) return MPSL_EINVAL;
  MPSL_HIP_TRY(ctx, hipSetDevice(ctx->device));
  int rc = mpsl::build_tables(ctx);
  if (rc) return rc;
  return mpsl::launch_m2s(ctx, prec, beta, spec);
}

int mpsl_reflect_dev(mpsl_ctx *ctx, const void *spec, const double *src, void *sigma) {
  if (!ctx || !sigma || (!spec && !src)) return MPSL_EINVAL;
  MPSL_HIP_TRY(ctx, hipSetDevice(ctx->device));
  int rc = mpsl::build_tables(ctx);
  if (rc) return rc;
  return mpsl::launch_reflect(ctx, spec, src, sigma);
}

int mpsl_s2l_dev(mpsl_ctx *ctx, int prec, const void *sigma, void *alpha) {
  if (!ctx || !sigma || !alpha || (prec != MPSL_FP64 && prec != MPSL_FP32)) return MPSL_EINVAL;
  MPSL_HIP_TRY(ctx, hipSetDevice(ctx->device));
  int rc = mpsl::build_tables(ctx);
  if (rc) return rc;
  const int cb = mpsl::chunks_s2l(ctx, 1, prec);
  if ((rc = mpsl::launch_s2l_coef(ctx, sigma))) return rc;
  if ((rc = mpsl::launch_s2l(ctx, prec, ctx->part.p, cb))) return rc;
  return mpsl::launch_sum_parts(ctx, prec, ctx->part.p, cb, alpha);
}

int mpsl_sapply_dev(mpsl_ctx *ctx, int prec, const void *x, const void *alpha, void *y) {
  if (!ctx || !alpha || !y || (prec != MPSL_FP64 && prec != MPSL_FP32)) return MPSL_EINVAL;
  MPSL_HIP_TRY(ctx, hipSetDevice(ctx->device));
  int rc = mpsl::build_tables(ctx);
  if (rc) return rc;
  return mpsl::launch_sapply(ctx, prec, x, alpha, y);
}

int mpsl_profile(mpsl_ctx *ctx, int enable) {
  if (!ctx) return MPSL_EINVAL;
  for (auto e : ctx->ev_start) (void)hipEventDestroy(e);
  for (auto e : ctx->ev_stop) (void)hipEventDestroy(e);
  ctx->ev_start.clear();
  ctx->ev_stop.clear();
  ctx->prof = enable != 0;
  return MPSL_OK;
}

int mpsl_profile_read(mpsl_ctx *ctx, double *ms_avg, int *count) {
  if (!ctx) return MPSL_EINVAL;
  MPSL_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  double tot = 0.0;
  int c = 0;
  for (size_t i = 0; i < ctx->ev_start.size(); ++i) {
    float ms = 0.f;
    MPSL_HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->ev_start[i], ctx->ev_stop[i]));
    tot += ms;
    ++c;
  }
  if (ms_avg) *ms_avg = c ? tot / c : 0.0;
  if (count) *count = c;
  return MPSL_OK;
}

int mpsl_set_tuning(mpsl_ctx *ctx, int prec, int variant, int chunks) {
  if (!ctx || (prec != MPSL_FP64 && prec != MPSL_FP32) || variant < mpsl::kM2LWhole || variant > mpsl::kM2LMfmaWide ||
      chunks < 0)
    return MPSL_EINVAL;
  if (const int pe = mpsl::check_unpinned(ctx)) return pe;
  auto &t = ctx->tune[prec == MPSL_FP64 ? 0 : 1];
  t.variant = variant;
  t.chunks = chunks;
  t.ms = 0.0;
  return MPSL_OK;
}

int mpsl_get_tuning(const mpsl_ctx *ctx, int prec, int *variant, int *chunks, double *ms) {
  if (!ctx || (prec != MPSL_FP64 && prec != MPSL_FP32)) return MPSL_EINVAL;
  const auto &t = ctx->tune[prec == MPSL_FP64 ? 0 : 1];
  if (variant) *variant = t.variant >= 0 ? t.variant : mpsl::m2l_default_variant(ctx->p, prec);
  if (chunks) *chunks = mpsl::chunks_m2l(ctx, prec);
  if (ms) *ms = t.ms;
  return MPSL_OK;
}

int mpsl_autotune(mpsl_ctx *ctx, int prec) {
  if (!ctx || (prec != MPSL_FP64 && prec != MPSL_FP32)) return MPSL_EINVAL;
  if (const int pe = mpsl::check_unpinned(ctx)) return pe;
  MPSL_HIP_TRY(ctx, hipSetDevice(ctx->device));
  int rc = mpsl::build_tables(ctx);
  if (rc) return rc;
  if (ctx->fmm.active) return MPSL_OK;  // the direct kernel is not used
  auto &t = ctx->tune[prec == MPSL_FP64 ? 0 : 1];
  t.chunks = 0;
  const int base = mpsl::chunks_m2l(ctx, prec);
  const int P = 2 * ctx->p + 1;
  const size_t esz = prec == MPSL_FP64 ? sizeof(double2) : sizeof(float2);
  const size_t len = static_cast<size_t>(ctx->n) * P;
  if ((rc = mpsl::dev_alloc(ctx, ctx->xbuf, len * esz))) return rc;
  if ((rc = mpsl::launch_fill_hash(ctx, prec, ctx->xbuf.p, static_cast<int64_t>(len), 12345u))) return rc;
  // the default count first: the others must beat it by more than 1 % (at 5000
  // particles half the default ties with it once the smaller partial sum is
  // counted, while its own launch fills the last wave of blocks worse)
  const int cands[3] = {base, std::max(1, base / 2), static_cast<int>(std::min<int64_t>(2LL * base, ctx->n))};
  hipEvent_t e0, e1;
  MPSL_HIP_TRY(ctx, hipEventCreate(&e0));
  MPSL_HIP_TRY(ctx, hipEventCreate(&e1));
  double best = 1e300;
  int bv = mpsl::kM2LWhole, bc = base;
  for (int variant = mpsl::kM2LWhole; variant <= mpsl::kM2LMfmaWide && !rc; ++variant)
    for (int c : cands) {
      if (variant >= mpsl::kM2LMfma && ctx->p > mpsl::kM2LMfmaMaxP) break;
      if ((rc = mpsl::dev_alloc(ctx, ctx->part, static_cast<size_t>(c) * len * esz))) break;
      // timed with the fold of its c partial slots, which grows with c
      auto run = [&]() {
        int e = mpsl::launch_m2l(ctx, prec, ctx->xbuf.p, ctx->part.p, c, variant);
        return e ? e : mpsl::launch_fold_parts(ctx, prec, ctx->part.p, c);
      };
      if ((rc = run())) break;  // warm-up
      if (hipEventRecord(e0, ctx->stream) != hipSuccess) { rc = MPSL_EHIP; break; }
      const int reps = 5;
      for (int r = 0; r < reps && !rc; ++r) rc = run();
      if (rc) break;
      float ms = 0.f;
      if (hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        rc = MPSL_EHIP;
        break;
      }
      const double avg = ms / reps;
      // a later candidate must win by more than 1 %: near-ties keep the earlier
      // one and the choice stays stable run to run
      if (avg < 0.99 * best) {
        best = avg;
        bv = variant;
        bc = c;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return mpsl::set_err(ctx, rc, "autotune failed: " + ctx->err);
  t.variant = bv;
  t.chunks = bc;
  t.ms = best;
  return mpsl::ensure_work(ctx);
}

}  // extern "C"
