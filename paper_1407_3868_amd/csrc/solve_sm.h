// Resumable solver for eq. (49): restarted GMRES (Arnoldi by classical
// Gram-Schmidt, FP64, a second pass where the first cancelled much of the
// vector; Givens rotations on the host) inside an
// FP64 residual loop, optionally right-preconditioned by the cluster blocks
// (the Krylov operator is A M^{-1}; corrections are M^{-1} V y).
//
// Cycles after the first recycle the first cycle's Krylov space (augmented
// GMRES in the GCRO form).  The first cycle leaves A M^{-1} V_k = V_{k+1} H_k
// with H_k = Q [R; 0] (Q the product of its Givens rotations), so
// W = V_{k+1} Q[:, :k] is an orthonormal basis of A U for U = M^{-1} V_k R^{-1}.
// A later cycle starts from r - W W^H r, orthogonalises every new vector
// against W as well as its own basis, and its correction is
// M^{-1} (V_k R^{-1} (W^H r - E z) + V' z), E the W-coefficients of the new
// vectors, z its least-squares solution.  In V_{k+1} coordinates the
// projector onto W is s -> s - q (q^H s), q the last column of Q, so both
// bases are swept in one pass.  With FP32 matvecs the later (refinement)
// cycles then keep the convergence the first cycle built up instead of
// starting their Krylov space from scratch.  In FP64 mode the inner matvecs are FP64 and the loop
// is plain restarted GMRES with a final true-residual check; in FP32 mode the
// inner matvecs are complex64 (iterative refinement: x += d, r = b - A x in
// FP64 after every inner solve).
//
// Each step is split into launch() (asynchronous work on the context stream)
// and complete() (waits for that stream, then host bookkeeping), so a caller
// can keep the steps of many solves in flight on their own streams.
#pragma once

#include <vector>

#include "kernels.h"

namespace mpsl {

// Right-hand side S a of eq. (49) for one point source into dev (FP64, n*P).
int rhs_device(mpsl_ctx *ctx, const double *src, void *dev);

class SolveSM {
 public:
  // smallest room (basis vectors) left for a later cycle to recycle the first
  static constexpr int kMinCycle = 16;
  enum Status { kRunning = 0, kConverged = 1, kExhausted = 2 };

  ~SolveSM();
  // Prepare for a solve of A x = b; b_dev (FP64, n*P) is copied.
  int init(mpsl_ctx *ctx, const mpsl_opts &o, const void *b_dev);
  int launch();
  int complete();
  int status() const { return status_; }
  const double2 *x() const { return xs_; }
  int iterations() const { return inner_mv_; }
  int fp64_matvecs() const { return fp64_mv_; }
  int refinements() const { return refin_; }
  double rel_residual() const { return rel_res_; }
  double precond_seconds() const { return pc_s_; }
  int reorthogonalizations() const { return reorth_; }
  const std::vector<double> &history() const { return hist_; }

 private:
  void *vslot(int j) const {
    return static_cast<char *>(V_) + static_cast<size_t>(j) * len_ * (vp_ == MPSL_FP32 ? sizeof(float2) : sizeof(double2));
  }
  // V_'s slot j = s src (src FP64)
  int store_basis(int j, double s, const double2 *src);
  int begin_inner();
  int finish_cycle();
  void keep_first_cycle();  // record W of the first cycle for the later ones
  // (Omega s)[:k0] for a V_{k+1}-coordinate vector s (Omega = Q^H)
  std::vector<zc> w_coords(const std::vector<zc> &s) const;

  enum Phase { kInner, kResidual };
  mpsl_ctx *ctx_ = nullptr;
  mpsl_opts o_{};
  int64_t len_ = 0;
  int m_ = 0;
  int phase_ = kInner;
  int status_ = kRunning;
  // device (inside ctx->gm).  The basis V_ is FP64, or FP32 in the mixed
  // solve (vp_): its inner solve only reaches inner_tol, and the refinement
  // recomputes the residual in FP64.  u_ holds the new Arnoldi vector in FP64
  // while it is orthogonalised (in FP64 mode it is V_'s next slot itself).
  void *V_ = nullptr;
  int vp_ = MPSL_FP64;
  double2 *u_ = nullptr, *w_ = nullptr, *r_ = nullptr, *xs_ = nullptr, *b_ = nullptr, *d_ = nullptr;
  double2 *h_ = nullptr, *h2_ = nullptr, *nrm_ = nullptr;
  float2 *x32_ = nullptr, *y32_ = nullptr;
  // pinned host staging
  double2 *hh_ = nullptr;  // pinned: h, h2 (m + 2 each), norm, y (m + 1), second-pass flag
  // host Hessenberg state
  std::vector<zc> H_, cs_, sn_, gv_;
  int j_ = 0;
  double bn_ = 0.0, rn_ = 0.0, inner_abs_ = 0.0, rel_res_ = 1.0;
  int inner_mv_ = 0, fp64_mv_ = 0, refin_ = 0;
  bool pc_ = false;     // cluster-block right preconditioner active
  double pc_s_ = 0.0;   // seconds spent building its blocks in init
  // recycled first-cycle space (k0_ = 0: none); base_ = first vector of the
  // current cycle's basis in V_
  int k0_ = 0, base_ = 0, cycles_ = 0;
  std::vector<zc> R0_, cs0_, sn0_;  // R (k0 x k0, row-major) and rotations of the first cycle
  std::vector<zc> yC_;              // W^H r of the current cycle
  std::vector<zc> Cs_;              // V_{k+1} coefficients of the new vectors, [j][k0 + 1]
  double2 *q_ = nullptr;            // device: last column of Q (k0 + 1)
  int32_t *skip_ = nullptr;         // device: second Gram-Schmidt pass not needed
  int reorth_ = 0;                  // iterations that needed the second pass
  std::vector<double> hist_;
};

}  // namespace mpsl
