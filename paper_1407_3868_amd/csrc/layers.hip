// Layer stacks of any number of layers around the particle layer (host, FP64),
// TM or TE polarisation.
//
// The three-layer system of Section 2, eq. (10), couples the two particle-layer
// densities through one reflection coefficient per interface.  With more
// layers, the interface conditions (8)-(9) at every interface above the
// particle layer collapse, for a wave travelling up in it, into one generalized
// reflection coefficient, and likewise below; the 2 x 2 coupling of the
// densities keeps its form.  The coefficients come from the standard recursion
// over the layers, outward from the half-spaces:
//   R_j = (r + rho) / (1 + r rho),   rho = R_{j-1} e^{-2 gamma_{j-1} h_{j-1}},
// with r the single-interface coefficient; every factor is bounded because
// Re gamma >= 0 on the contour.  TE weights du/dy by 1/k^2 of its layer
// (permittivity piecewise constant, permeability constant), which enters r
// and t through kappa gamma.
#include <cmath>

#include "context.h"

namespace mpsl {

namespace {

// Single-interface coefficient for a wave in the layer with weighted gamma
// za = kappa_a gamma_a meeting the layer with zb: reflected / incident
// (amplitudes divided by gamma; kappa = 1 for TM, 1/k^2 for TE).
inline zc refl(zc za, zc zb) { return (za - zb) / (za + zb); }

struct StackWork {
  std::vector<zc> g, e, ru, tau, rd;
  std::vector<double> kap;  // weight of du/dy per layer
};

// Recursions above and below the particle layer c; ru[j], tau[j] for
// 1 <= j <= c, rd[j] for c <= j <= L-2.
void stack_recursion(const mpsl_ctx *ctx, zc lam, StackWork &w) {
  const int L = static_cast<int>(ctx->ks.size()), c = ctx->layer_c;
  w.g.resize(L);
  w.e.assign(L, zc(0.0, 0.0));
  w.ru.assign(L, zc(0.0, 0.0));
  w.tau.assign(L, zc(0.0, 0.0));
  w.rd.assign(L, zc(0.0, 0.0));
  w.kap.assign(L, 1.0);
  for (int j = 0; j < L; ++j) {
    w.g[j] = gamma_branch(lam, ctx->ks[j]);
    if (ctx->pol == MPSL_TE) w.kap[j] = 1.0 / (ctx->ks[j].real() * ctx->ks[j].real());
  }
  for (int j = 1; j < L - 1; ++j) w.e[j] = std::exp(-w.g[j] * ctx->thick[j]);
  const std::vector<double> &kp = w.kap;
  // above: layer 1 under the top half-space, then one finite layer at a time;
  // the transmitted amplitude follows from u and kappa du/dy continuous:
  // t = 2 kappa_j gamma_{j+1} / (kappa_j gamma_j + kappa_{j+1} gamma_{j+1})
  w.ru[1] = refl(kp[1] * w.g[1], kp[0] * w.g[0]);
  w.tau[1] = 2.0 * kp[0] * w.g[1] / (kp[0] * w.g[0] + kp[1] * w.g[1]);
  for (int j = 1; j < c; ++j) {
    const zc r = refl(kp[j + 1] * w.g[j + 1], kp[j] * w.g[j]);
    const zc t = 2.0 * kp[j] * w.g[j + 1] / (kp[j] * w.g[j] + kp[j + 1] * w.g[j + 1]);
    const zc rho = w.ru[j] * w.e[j] * w.e[j];
    const zc den = 1.0 + r * rho;
    w.ru[j + 1] = (r + rho) / den;
    w.tau[j + 1] = t * w.e[j] * w.tau[j] / den;
  }
  // below: layer L-2 over the bottom half-space, then upwards
  w.rd[L - 2] = refl(kp[L - 2] * w.g[L - 2], kp[L - 1] * w.g[L - 1]);
  for (int j = L - 3; j >= c; --j) {
    const zc r = refl(kp[j] * w.g[j], kp[j + 1] * w.g[j + 1]);
    const zc rho = w.rd[j + 1] * w.e[j + 1] * w.e[j + 1];
    w.rd[j] = (r + rho) / (1.0 + r * rho);
  }
}

}  // namespace

void stack_node(const mpsl_ctx *ctx, zc lam, zc &Rup, zc &Rdn, zc &T) {
  StackWork w;
  stack_recursion(ctx, lam, w);
  Rup = w.ru[ctx->layer_c];
  Rdn = w.rd[ctx->layer_c];
  T = w.tau[ctx->layer_c];
}

void layer_map(const mpsl_ctx *ctx, zc lam, zc m[6]) {
  // closed-form solution of the interface system for the particle-layer
  // densities: sigma+ - r1 E sigma- = t g + r1 P+,  sigma- - r3 E sigma+ = r3 P-
  // (eq. (10) for three layers; r1, r3, t the generalized coefficients otherwise)
  zc r1, r3, tg;
  stack_node(ctx, lam, r1, r3, tg);
  const zc g2 = gamma_branch(lam, ctx->k2);
  const zc E = std::exp(-g2 * ctx->d);
  const zc det = 1.0 - r1 * r3 * E * E;
  m[0] = r1 / det;
  m[1] = r1 * r3 * E / det;
  m[2] = r1 * r3 * E / det;
  m[3] = r3 / det;
  m[4] = tg / det;
  m[5] = tg * r3 * E / det;
}

int assign_stack(mpsl_ctx *ctx, int n_layers, const mpsl_c128 *k, const double *thickness, int particle_layer,
                 std::string &err) {
  if (!k || !thickness || n_layers < 3 || n_layers > kMaxLayers) {
    err = "need 3 to " + std::to_string(kMaxLayers) + " layers";
    return MPSL_EINVAL;
  }
  const int L = n_layers, c = particle_layer;
  if (c < 1 || c > L - 2) {
    err = "the particle layer must be a finite layer";
    return MPSL_EINVAL;
  }
  for (int j = 0; j < L; ++j) {
    if (!(k[j].re > 0.0) || !(k[j].im >= 0.0) || !std::isfinite(k[j].re) || !std::isfinite(k[j].im)) {
      err = "wavenumbers need Re k > 0 and Im k >= 0";
      return MPSL_EINVAL;
    }
    if (k[j].im != 0.0) {
      err = "this build supports real layer wavenumbers only";
      return MPSL_EUNSUPPORTED;
    }
  }
  for (int j = 1; j < L - 1; ++j)
    if (!(thickness[j] > 0.0) || !std::isfinite(thickness[j])) {
      err = "layer thickness must be > 0";
      return MPSL_EINVAL;
    }
  ctx->ks.resize(L);
  ctx->thick.assign(L, 0.0);
  for (int j = 0; j < L; ++j) ctx->ks[j] = zc(k[j].re, k[j].im);
  for (int j = 1; j < L - 1; ++j) ctx->thick[j] = thickness[j];
  // interface i separates layer i from layer i + 1; the particle layer's top is y = 0
  ctx->yint.assign(L - 1, 0.0);
  for (int i = c - 2; i >= 0; --i) ctx->yint[i] = ctx->yint[i + 1] + ctx->thick[i + 1];
  for (int i = c; i < L - 1; ++i) ctx->yint[i] = ctx->yint[i - 1] - ctx->thick[i];
  ctx->layer_c = c;
  ctx->k1 = ctx->ks[0];
  ctx->k2 = ctx->ks[c];
  ctx->k3 = ctx->ks[L - 1];
  ctx->d = ctx->thick[c];
  return MPSL_OK;
}

void stack_amplitudes(const mpsl_ctx *ctx, zc lam, zc gs, zc sp, zc sm, zc Pp, zc Pm, zc *A, zc *B, zc *g) {
  StackWork w;
  stack_recursion(ctx, lam, w);
  const int L = static_cast<int>(ctx->ks.size()), c = ctx->layer_c;
  for (int j = 0; j < L; ++j) {
    g[j] = w.g[j];
    A[j] = B[j] = zc(0.0, 0.0);
  }
  A[c] = sp;
  B[c] = sm;
  // upwards: (up a, down b) at the top interface of layer j + 1
  zc a = w.e[c] * sm + Pp, b = sp;
  for (int j = c - 1; j >= 1; --j) {
    // u and du/dy continuous across interface j give the upgoing wave at the
    // bottom of layer j; its downgoing wave follows from the layers above
    const zc s = w.g[j] / w.g[j + 1] * (a + b), dl = (w.kap[j + 1] / w.kap[j]) * (b - a);
    B[j] = 0.5 * (s - dl);
    a = B[j] * w.e[j];
    b = w.ru[j] * a + w.tau[j] * gs;
    A[j] = b;
  }
  B[0] = w.g[0] / w.g[1] * (a + b) - gs;
  // downwards: (down dn, up up) at the bottom interface of layer j - 1
  zc dn = w.e[c] * sp + Pm, up = sm;
  for (int j = c + 1; j <= L - 2; ++j) {
    A[j] = 0.5 * (w.g[j] / w.g[j - 1] * (dn + up) + (w.kap[j - 1] / w.kap[j]) * (dn - up));
    dn = A[j] * w.e[j];
    up = w.rd[j] * dn;
    B[j] = up;
  }
  A[L - 1] = w.g[L - 1] / w.g[L - 2] * (dn + up);
}

}  // namespace mpsl
