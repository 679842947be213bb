// Launchers of the device kernels (implemented in kernels.hip).
#pragma once

#include "context.h"

namespace mpsl {

// Largest supported expansion order and the range instantiated.
constexpr int kMinP = 1;
constexpr int kMaxP = 20;
// Largest contour, and largest particles x nodes product (the plane-wave
// factor tables hold 2 N N_S entries per precision).
constexpr int kMaxNodes = 1 << 20;
// Largest number of particle types (prototype scattering matrices).
constexpr int kMaxTypes = 1024;
constexpr int64_t kMaxPlaneWaves = int64_t(1) << 29;

// Row a0: per-particle plane-wave factor tables of the contour (E, F) and
// rotation phases.  FP64 master tables and FP32 copies.
int launch_geom_tables(mpsl_ctx *ctx);
// Row a0 (pairs): H_0, H_1, direction and 2/z of every ordered particle pair.
int launch_pair_tables(mpsl_ctx *ctx);

// Row a1: partial local expansions of the all-pairs M2L into
// part[0 .. chunks).  variant: kM2LWhole, kM2LHalves, kM2LMfma, kM2LMfmaWide
// (matrix cores, 16 or 32 targets per wave, p <= kM2LMfmaMaxP), or -1 for the
// tuned one.
constexpr int kM2LWhole = 0;
constexpr int kM2LHalves = 1;
constexpr int kM2LMfma = 2;
constexpr int kM2LMfmaWide = 3;
constexpr int kM2LMfmaMaxP = 16;
// Variant used before any tuning: by expansion order and precision.
int m2l_default_variant(int p, int prec);
// nrhs right-hand sides: beta [nrhs][n][P]; part of rhs r at part + r * pstride.
int launch_m2l(mpsl_ctx *ctx, int prec, const void *beta, void *part, int chunks, int variant = -1,
               int nrhs = 1, int64_t pstride = 0);
// Row a1, many right-hand sides (FP32, MFMA): beta [nrhs][n][P]; partials
// of right-hand side r at part + r * pstride, chunks slots each.
int launch_m2l_mrhs(mpsl_ctx *ctx, const void *beta, void *part, int chunks, int nrhs, int64_t pstride);
int chunks_m2l_mrhs(const mpsl_ctx *ctx, int nrhs);
// Right-hand sides from which the multi-RHS M2L runs on the matrix cores.
constexpr int kMrhsMin = 16;
// FMM near field (pairs in the same or adjacent leaf boxes) into out [n][P].
int launch_fmm_near(mpsl_ctx *ctx, int prec, const void *beta, void *out);
// Row b1: M2S partial spectra and their reduction to spec (double2[2*ns]).
// spec: double2[nrhs][2][ns].
int launch_m2s(mpsl_ctx *ctx, int prec, const void *beta, void *spec, int nrhs = 1);
// Row b2: sigma = R spec (+ source), and the scaled S2L coefficient tables.
// spec, sigma: double2[nrhs][2][ns] (spec may be null; src the same for every rhs).
int launch_reflect(mpsl_ctx *ctx, const void *spec, const double *src, void *sigma, int nrhs = 1);
// S2L coefficient tables from sigma (both precisions).
int launch_s2l_coef(mpsl_ctx *ctx, const void *sigma, int nrhs = 1);
// Row b3: partial local expansions of the layer field into part[0 .. chunks).
int launch_s2l(mpsl_ctx *ctx, int prec, void *part, int chunks, int nrhs = 1, int64_t pstride = 0);
// Sum of partial buffers: alpha = sum_{c < chunks} part[c].
int launch_sum_parts(mpsl_ctx *ctx, int prec, const void *part, int chunks, void *alpha);
// Partial buffers of each right-hand side summed in place into slot 0
// (part + r * pstride holds chunks slots of n P entries).
int launch_fold_parts(mpsl_ctx *ctx, int prec, void *part, int chunks, int nrhs = 1, int64_t pstride = 0);
// Row a2 (MFMA): y = x - S_rot alpha  (x may be null: y = S_rot alpha);
// alpha of right-hand side r at alpha + r * astride.
int launch_sapply(mpsl_ctx *ctx, int prec, const void *x, const void *alpha, void *y, int nrhs = 1,
                  int64_t astride = 0);

// GMRES helpers (FP64 complex vectors of length len; the k vectors of V in
// FP64, or FP32 when v_prec is MPSL_FP32, with FP64 products and sums).  skip
// (device, may be null): when *skip != 0 the dot products come out zero and
// the update does nothing (a second Gram-Schmidt pass found unnecessary on the
// device).
int launch_dotc_multi(mpsl_ctx *ctx, const void *V, int64_t ld, int k, const void *w, int64_t len,
                      void *h_out, const int32_t *skip = nullptr, int v_prec = MPSL_FP64);
int launch_gemv_sub(mpsl_ctx *ctx, const void *V, int64_t ld, int k, const void *h, void *w,
                    int64_t len, const int32_t *skip = nullptr, int v_prec = MPSL_FP64);
// v32 = s src, rounded to complex64.
int launch_scale_to_fp32(mpsl_ctx *ctx, void *v32, int64_t len, double s, const void *src);
// skip = ||after||^2 >= eta2 ||before||^2 (both the real part of a dot product).
int launch_reorth_flag(mpsl_ctx *ctx, const void *before, const void *after, double eta2, int32_t *skip);
int launch_scale(mpsl_ctx *ctx, void *v, int64_t len, double s, const void *src);
// h[i] -= q[i] (q^H h) for i < k (one block): the projection onto span(W)
// in V coordinates used when a GMRES cycle recycles the first cycle's space.
int launch_proj_fix(mpsl_ctx *ctx, void *h, const void *q, int k);
// Bytes of ctx->scal that launch_dotc_multi needs for k dot products.
size_t dotc_scratch_bytes(int k);
// Largest Krylov dimension of the GMRES solver (basis vectors kept at once).
constexpr int kMaxKrylov = 20000;
int launch_axpy_c(mpsl_ctx *ctx, void *y, const void *x, int64_t len, double a_re, double a_im);
int launch_to_fp32(mpsl_ctx *ctx, const void *x64, void *x32, int64_t len);
int launch_to_fp64(mpsl_ctx *ctx, const void *x32, void *x64, int64_t len);
// Deterministic pseudo-random complex vector (n_complex entries) in precision prec.
int launch_fill_hash(mpsl_ctx *ctx, int prec, void *v, int64_t n_complex, uint32_t seed);

// Row a7: field at receivers.  gl: double2[L][ns] gamma per layer; amp:
// double2[L][2][ns] downgoing amplitude at the top and upgoing at the bottom
// of each layer; yint: double[L-1] interface heights (all device).
int launch_field(mpsl_ctx *ctx, const void *beta, const void *gl, const void *amp, const void *yint,
                 const double *src, int64_t nr, const void *rcv, void *u);

// Source chunks of the M2L grid for precision prec (tuned, set, or automatic).
int chunks_m2l(const mpsl_ctx *ctx, int prec);
// Sources per chunk of the matrix-core M2L for a grid of `chunks` chunks
// (whole groups of four sources).
int m2l_mfma_chunk_len(int n, int chunks);
// Partial buffers written by one M2L launch.
inline int m2l_slots(const mpsl_ctx *ctx, int prec) { return chunks_m2l(ctx, prec); }
// Node chunks of the S2L grid for precision prec (its particle tiles differ).
int chunks_s2l(const mpsl_ctx *ctx, int nrhs, int prec);
// Particle chunks of the M2S grid for precision prec.
int chunks_m2s(const mpsl_ctx *ctx, int nrhs, int prec);

// Sommerfeld transforms by tile-local interpolation (somm.hip): M2S spectra
// into spec ([nrhs][2][ns], FP64) and S2L local expansions into one part slot
// per chunk of coarse nodes and right-hand side.
int launch_m2s_interp(mpsl_ctx *ctx, int prec, const void *beta, void *spec, int nrhs);
int launch_s2l_interp(mpsl_ctx *ctx, int prec, void *part, int chunks, int nrhs, int64_t pstride);

}  // namespace mpsl
