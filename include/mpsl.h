/*
 * mpsl.h -- C ABI of the MI355X multi-particle scattering library for a
 * three-layer medium (Lai, Kobayashi, Greengard, "A fast solver for
 * multi-particle scattering in a layered medium").
 *
 * Problem (Section 1): 2D TM scattering, Helmholtz wavenumbers k1 (y > 0),
 * k2 (-d < y < 0), k3 (y < -d); N identical particles of wavenumber kp in the
 * middle layer, each a rotated copy of one prototype; a unit point source
 * G_{k1}(x, x_s) = (i/4) H_0^(1)(k1 |x - x_s|) at x_s in the top layer.
 * Outgoing waves use H^(1) (time dependence e^{-i omega t}).
 *
 * Unknowns (Section 3): for particle l, the coefficients beta^l_n of its
 * multipole expansion sum_n beta_n H_n(k2 r) e^{in theta}, n = -p..p, stored
 * at slot n + p; P = 2p + 1 per particle.  The library solves the
 * Schur-complement system of Section 5.4, eq. (49), in the form
 *
 *     (I - S (T + T_R)) beta = S a
 *
 * T   : all-pairs free-space multipole-to-local translation (Lemma 3.1),
 * T_R : reflected field of the layers, S2L o R o M2S (Sections 5.2-5.3),
 * S   : prototype scattering matrix rotated per particle (Section 4.1),
 * a   : local expansions of the source's layer-2 field.
 *
 * Conventions.
 *  - Complex numbers are interleaved (re, im); mpsl_c128 is two doubles
 *    (binary compatible with C99 double _Complex), mpsl_c64 two floats.
 *  - Coefficient arrays are [particle][n + p], row-major, P per particle;
 *    with several right-hand sides, [rhs][particle][n + p].
 *  - Angles are radians, counter-clockwise.
 *  - Pointers named *_dev are device pointers on the context's device;
 *    all other pointers are host pointers.  The caller owns every buffer
 *    it passes; the library copies what it keeps.
 *  - Every call returns MPSL_OK (0) or a negative MPSL_E* status; no call
 *    aborts.  mpsl_last_error() gives a message for the last failure.
 *  - A context is used by one host thread at a time.
 */
#ifndef MPSL_H
#define MPSL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } mpsl_c128;
typedef struct { float re, im; } mpsl_c64;

typedef struct mpsl_ctx mpsl_ctx;

enum {
  MPSL_OK = 0,
  MPSL_EINVAL = -1,        /* bad argument (null pointer, size, range)         */
  MPSL_ENOMEM = -2,        /* device or host allocation failed                 */
  MPSL_EHIP = -3,          /* a HIP runtime call failed                        */
  MPSL_ESTATE = -4,        /* a required set_* call has not been made          */
  MPSL_EGEOM = -5,         /* particles overlap or leave the middle layer     */
  MPSL_ENOCONV = -6,       /* GMRES stopped above tolerance (result written)   */
  MPSL_EUNSUPPORTED = -7,  /* parameters outside what this build implements    */
  MPSL_EINSIDE = -8,       /* receiver inside an enclosing disk (value NaN)    */
  MPSL_ENUMERIC = -9,      /* NaN/Inf met in the iteration                     */
  MPSL_PENDING = 1         /* server: the request has not finished yet          */
};

/* Polarisation (Section 1): with the permeability constant and the
 * permittivity piecewise constant, TM keeps u and du/dn continuous across
 * every interface and particle boundary (eqs. (8)-(9)); TE keeps u and
 * (1/k^2) du/dn continuous. */
enum {
  MPSL_TM = 0,   /* the paper's case (default) */
  MPSL_TE = 1
};

/* Arithmetic of the hot path. */
enum {
  MPSL_FP64 = 0,   /* complex128 translations, FP64 accumulation            */
  MPSL_FP32 = 1    /* complex64 translations and sums, FP32 accumulation    */
};

const char *mpsl_status_string(int status);
const char *mpsl_last_error(const mpsl_ctx *ctx);

/* Create a context on HIP device `device`.  Owns all device memory and one
 * stream (the null stream of the device unless mpsl_set_stream is called).
 * hbm_budget: device bytes the context may hold at once (tables, work buffers,
 * Krylov basis, preconditioner blocks); a call whose allocation would exceed
 * it fails with MPSL_ENOMEM (that buffer is not allocated; the context stays
 * valid).  0 = no limit beyond the device's memory. */
int mpsl_create(mpsl_ctx **out, int device, size_t hbm_budget);
void mpsl_destroy(mpsl_ctx *ctx);

/* Device bytes the context holds now and its budget (0: none); either output
 * pointer may be NULL. */
int mpsl_get_memory(const mpsl_ctx *ctx, size_t *bytes_in_use, size_t *hbm_budget);

/* Run all later device work on `stream` (a hipStream_t, e.g. torch's current
 * stream); NULL selects the device's null stream. */
int mpsl_set_stream(mpsl_ctx *ctx, void *stream);

/* Polarisation of the context (MPSL_TM or MPSL_TE; MPSL_EINVAL otherwise).
 * It enters the reflection map of the layers and the scattering matrices of
 * disks and stars, so a change clears the particle: call
 * mpsl_set_particle_* (or mpsl_set_scattering_matrix with a matrix of this
 * polarisation) again afterwards.  The matvec's kernels are the same. */
int mpsl_set_polarization(mpsl_ctx *ctx, int polarization);
int mpsl_get_polarization(const mpsl_ctx *ctx);

/* Layer wavenumbers and middle-layer thickness d > 0 (Section 1, Fig. 1):
 * the three-layer case of mpsl_set_layer_stack (k = {k1, k2, k3}, particle
 * layer 1, interfaces y = 0 and y = -d).  Real k > 0 (this build requires
 * Im k == 0 for every layer). */
int mpsl_set_layers(mpsl_ctx *ctx, mpsl_c128 k1, mpsl_c128 k2, mpsl_c128 k3, double d);

/* A stack of n_layers (3..64) layers, top to bottom, TM polarisation: the
 * extension of Section 2 to any number of layers that the Introduction names,
 * with u and du/dy continuous across every interface (eqs. (8)-(9)).
 * k[j] (host, n_layers entries): wavenumber of layer j, real and > 0.
 * thickness[j] (host, n_layers entries): thickness of the finite layer j
 * (1 <= j <= n_layers - 2, > 0); entries 0 and n_layers - 1 (the two
 * half-spaces) are ignored.  particle_layer c (1..n_layers - 2): the finite
 * layer holding the particles; its top interface is y = 0 and its bottom
 * y = -thickness[c], so particle geometry is given as for three layers and
 * the other interfaces sit at y_i = sum of the thicknesses in between.  The
 * point source of mpsl_rhs / mpsl_solve / mpsl_eval_field lies in layer 0,
 * above the top interface.  The particle layer's densities keep the 2 x 2
 * coupling of eq. (10) through generalized reflection coefficients of the
 * layers above and below (host FP64 per contour node); the matvec's kernels
 * and cost do not depend on n_layers.  Returns MPSL_EINVAL for a bad count,
 * layer index, thickness or wavenumber, MPSL_EUNSUPPORTED for Im k != 0. */
int mpsl_set_layer_stack(mpsl_ctx *ctx, int n_layers, const mpsl_c128 *k, const double *thickness,
                         int particle_layer);

/* Host, no device: the per-node map that mpsl_set_layer_stack's stack gives
 * the particle layer's densities (Section 2, eq. (10) and its extension to
 * more layers), for n_lam nodes lam (host).  map (host, 6 * n_lam entries):
 * map[6q + 0..3] = the 2 x 2 matrix, row-major, taking the particles' spectra
 * (P+, P-) on the two interfaces of the particle layer to (sigma+, sigma-);
 * map[6q + 4..5] = (sigma+, sigma-) per unit source amplitude at the top
 * interface.  These are the values the device reflection step applies.
 * Same argument rules and errors as mpsl_set_layer_stack. */
int mpsl_compute_layer_map(int n_layers, const mpsl_c128 *k, const double *thickness, int particle_layer,
                           int polarization, int n_lam, const mpsl_c128 *lam, mpsl_c128 *map);

/* Circular particles of radius R and wavenumber kp (real, > 0): the diagonal
 * Mie scattering matrix of Section 3.1, eqs. (17)-(18), order p (1..32).
 * Requires mpsl_set_layers first (uses k2).  Enclosing radius = R. */
int mpsl_set_particle_disk(mpsl_ctx *ctx, double R, mpsl_c128 kp, int p);

/* Star-shaped particles r(t) = a1 + a2 cos(a3 t), t the polar angle (Section 6,
 * eq. (50)), wavenumber kp (real, > 0): prototype scattering matrix from
 * Mueller's second-kind integral equations (Section 4, eqs. (31)-(32); outgoing
 * coefficients by eq. (35)), Nystrom discretisation on n_bdry equispaced
 * boundary points (even, 64..2048; 0 selects 256) with Kress's logarithmic
 * product quadrature and Maue's identity for the hypersingular difference.
 * Host FP64 precompute, O(n_bdry^3).  Enclosing radius a1 + |a2|.  Requires
 * mpsl_set_layers first (uses k2). */
int mpsl_set_particle_star(mpsl_ctx *ctx, double a1, double a2, int a3, mpsl_c128 kp, int p, int n_bdry);

/* Caller-supplied prototype scattering matrix (Section 4.1): S is P x P
 * row-major, S[(l + p) * P + (n + p)] maps incoming alpha_n to outgoing
 * beta_l, for the prototype at rotation 0.  r_enclose is the radius of the
 * disk enclosing the prototype (used by geometry checks). */
int mpsl_set_scattering_matrix(mpsl_ctx *ctx, int p, double r_enclose, const mpsl_c128 *S);

/* Several particle types (Section 4.2, Remark): n_types (1..1024) prototype
 * scattering matrices, S[t * P * P + (l + p) * P + (n + p)] for type t (the
 * layout of mpsl_set_scattering_matrix per type), with enclosing radii
 * r_enclose[t] > 0 (host arrays, copied).  All types share the order p.
 * Particles get their types from mpsl_set_geometry_typed (mpsl_set_geometry:
 * all type 0).  A geometry whose types no longer exist is dropped (set it
 * again).  The scattering-matrix apply visits, per tile of 16 particles, only
 * the types present in it: ordering particles by type keeps it one pass. */
int mpsl_set_particle_types(mpsl_ctx *ctx, int n_types, int p, const double *r_enclose, const mpsl_c128 *S);

/* mpsl_set_geometry with a type per particle: type[j] in 0..n_types-1 (host,
 * n entries; NULL: all type 0).  The geometry checks use each particle's own
 * enclosing radius. */
int mpsl_set_geometry_typed(mpsl_ctx *ctx, int64_t n, const double *xy, const double *rot, const int32_t *type);

/* Particle centres xy[2 * j], xy[2 * j + 1] and CCW rotations rot[j] (NULL
 * for all zero), j < n.  Fails with MPSL_EGEOM when two enclosing disks
 * overlap or an enclosing disk crosses y = 0 or y = -d.  Requires layers and
 * particle.  Builds the per-particle device tables (rotation phases, plane-
 * wave factors of the contour) when a contour is set. */
int mpsl_set_geometry(mpsl_ctx *ctx, int64_t n, const double *xy, const double *rot);

/* Sommerfeld contour of Section 5.1, eq. (37): Gamma_3 u Gamma_2 u Gamma_1 with
 * offset b > 0, truncated at t_max, 16-point Gauss-Legendre panels; n_nodes
 * = 32 + 32 m (m >= 2).  Panel rule: two panels on Gamma_2; on [0, t_max]
 * breakpoints at 0, t_max and Re k_i, then the panel with the largest
 * length / max(distance to nearest Re k_i, b) is halved until (n_nodes-32)/32
 * panels exist; Gamma_3 mirrors Gamma_1.  Requires layers. */
int mpsl_set_contour(mpsl_ctx *ctx, int n_nodes, double b, double t_max);

/* Context-free host computations (no device needed), same arithmetic as the
 * set_* calls above: the disk and star scattering matrices (P x P, row-major)
 * for polarization MPSL_TM or MPSL_TE (TE: Mie coefficients with the
 * derivative condition weighted by 1/k^2; Mueller's system with the interior
 * double layer scaled by kp^2/k2^2 so that T2 - Tp stays weakly singular),
 * and the contour nodes and weights for layer wavenumbers k1, k2, k3. */
int mpsl_compute_disk_smatrix(double R, mpsl_c128 k2, mpsl_c128 kp, int p, int polarization, mpsl_c128 *S);
int mpsl_compute_star_smatrix(double a1, double a2, int a3, mpsl_c128 k2, mpsl_c128 kp, int p, int n_bdry,
                              int polarization, mpsl_c128 *S);
int mpsl_compute_contour(mpsl_c128 k1, mpsl_c128 k2, mpsl_c128 k3, int n_nodes, double b, double t_max,
                         mpsl_c128 *lam, mpsl_c128 *w);

/* Sommerfeld contour of Section 5.1, eq. (37), with panels of bounded length
 * instead of a fixed node count (span rule), for layouts spread laterally:
 * the sums over nodes carry e^{i lambda (x_l - x_m)}, and |x_l - x_m| up to the
 * lateral extent X of particles and sources must be resolved.  On
 * [0, t_max]: breakpoints 0, t_max and every Re k_i in between; in each gap
 * [a, c] with midpoint m, an end that is a Re k_i is graded (cuts at
 * a + b 2^j while below m, at c - b 2^j while above m, and at m); every piece
 * between cuts splits into ceil(length / h_max) equal 16-point Gauss-Legendre
 * panels.  Gamma_2 (two panels) and Gamma_3 (mirror) as in mpsl_set_contour.
 * Guide: b = min(0.2, 2 / X); h_max = 6 / X gives about 1e-11 on the layered
 * interaction of two particles X apart, h_max = 12 / X about 1e-6; t_max
 * such that e^{-sqrt(t_max^2 - max k^2) dy} is negligible for the smallest
 * vertical distance dy of a reflected path (24 for dy >= 2 and k <= 12).
 * N_S = 32 + 32 * (panels), at most 2^20; the matvec needs N * N_S <= 2^29
 * (MPSL_EUNSUPPORTED otherwise).  Requires layers. */
int mpsl_set_contour_span(mpsl_ctx *ctx, double b, double t_max, double h_max);

/* How M2S and S2L (Sections 5.2.1 and 5.3) sum over the contour nodes:
 * MPSL_SOMM_DIRECT: every particle with every node (O(N N_S P), default);
 * MPSL_SOMM_INTERP: particles grouped in tiles of 8 x 4 (lengths); per tile
 * the part of the plane waves that varies slowly in lambda (the phase
 * relative to the tile centre and the order weights) is evaluated at 24
 * Chebyshev nodes of each lambda-interval of length 1 and interpolated to the
 * contour nodes (barycentric form); nodes within 0.3 of +-k2 and on the
 * vertical segment are summed directly.  Work O(N N_C P + N_S T 24) for N_C
 * coarse nodes and T tiles instead of O(N N_S P); accurate to about 1e-13 in
 * the M2S spectra for the calibrated case (k2 = 9, p = 16, span-rule contour),
 * as the paper's NUFFT forms (Section 5.2.2, 5.3.1) are for large N_S.  This
 * replaces the paper's FFT grids by interpolation, which maps to dense GPU
 * loops.  MPSL_EINVAL for other values. */
enum { MPSL_SOMM_DIRECT = 0, MPSL_SOMM_INTERP = 1 };
int mpsl_set_sommerfeld_method(mpsl_ctx *ctx, int method);

/* Shape of the MPSL_SOMM_INTERP plan of the current problem (after a first
 * apply or solve; MPSL_ESTATE before): active = 1 when the interpolated
 * transforms are in use, particle tiles, lambda-intervals, coarse nodes
 * (24 per interval plus one per direct node) and direct contour nodes.
 * Any output pointer may be NULL. */
int mpsl_get_somm_info(const mpsl_ctx *ctx, int *active, int *tiles, int *intervals, int *coarse_nodes,
                       int *direct_nodes);

/* Host, no device: the span rule's nodes and weights for the real parts
 * re_k[0 .. n_k) of the layer wavenumbers.  *n_nodes receives the count;
 * with lam and w NULL nothing else is written, otherwise both must hold
 * capacity >= *n_nodes entries (MPSL_EINVAL if not). */
int mpsl_compute_contour_span(int n_k, const double *re_k, double b, double t_max, double h_max, int capacity,
                              mpsl_c128 *lam, mpsl_c128 *w, int *n_nodes);

/* Explicit contour: nodes lam[q] and weights w[q] (d lambda included). */
int mpsl_set_contour_nodes(mpsl_ctx *ctx, int n_nodes, const mpsl_c128 *lam, const mpsl_c128 *w);

/* Copy the current contour out (host arrays of n_nodes entries). */
int mpsl_get_contour(const mpsl_ctx *ctx, int n_nodes, mpsl_c128 *lam, mpsl_c128 *w);

/* Copy the prototype scattering matrix out (P x P, host). */
int mpsl_get_scattering_matrix(const mpsl_ctx *ctx, int p, mpsl_c128 *S);

/* Sizes of the current problem (any pointer may be NULL). */
int mpsl_get_sizes(const mpsl_ctx *ctx, int64_t *n, int *p, int *n_nodes);

/* ---- one preconditioned Schur matvec (the GMRES operator) ----------------
 * y = x - S (T + T_R) x   (Section 5.4, eq. (49); Section 3.2 preconditioning)
 * x, y: N*P complex, precision `prec` (mpsl_c128 for MPSL_FP64, mpsl_c64 for
 * MPSL_FP32).  _dev: device pointers, asynchronous on the context stream;
 * the host variant copies in and out and synchronises.  x and y must not
 * overlap. */
int mpsl_apply(mpsl_ctx *ctx, int prec, const void *x, void *y);
int mpsl_apply_dev(mpsl_ctx *ctx, int prec, const void *x_dev, void *y_dev);

/* Batched matvec: nrhs right-hand sides X, Y laid out [nrhs][N][P] (device,
 * precision prec), one launch per step for all of them. */
int mpsl_apply_batch_dev(mpsl_ctx *ctx, int prec, int nrhs, const void *x_dev, void *y_dev);

/* Multi-configuration batch: item i is one (possibly batched) matvec of
 * context ctxs[i] in precision precs[i] with nrhs[i] right-hand sides (nrhs may
 * be NULL: one each) on device buffers x[i] -> y[i].  mpsl_batch_create runs
 * every item once (building tables and work buffers), then captures all of
 * them into one HIP graph with one parallel branch per item; mpsl_batch_launch
 * replays the whole batch with a single graph launch on `stream` (a
 * hipStream_t, NULL for the null stream), reading the current contents of the
 * x buffers.  The graph holds the addresses of each context's tables and work
 * buffers, so while a batch exists its contexts are pinned: calls that would
 * rebuild or move them (mpsl_set_layers, _layer_stack, _polarization,
 * _particle_*, _particle_types, _scattering_matrix, _geometry*, _contour*,
 * _sommerfeld_method, _far_field, _tuning, mpsl_autotune, and a batched matvec
 * with more right-hand sides than any call before) return MPSL_ESTATE until
 * mpsl_batch_destroy.  Solves, right-hand sides, field evaluation and matvecs
 * of the sizes already used stay allowed.  A context appearing twice in one
 * batch is rejected (MPSL_EINVAL: its work buffers are shared).  The x and y
 * buffers must stay allocated, and every batch must be destroyed before its
 * contexts.  Results are bitwise those of mpsl_apply_batch_dev on each item. */
typedef struct mpsl_batch mpsl_batch;
int mpsl_batch_create(mpsl_batch **out, int n_items, mpsl_ctx *const *ctxs, const int *precs, const int *nrhs,
                      const void *const *x, void *const *y);
int mpsl_batch_launch(mpsl_batch *batch, void *stream);
void mpsl_batch_destroy(mpsl_batch *batch);

/* ---- the steps of the matvec, each on device buffers ---------------------
 * Row a1, free-space all-pairs M2L (Lemma 3.1, eq. (24), Graf's theorem):
 *   alpha^l_{n'} = sum_{m != l} sum_nu H_{nu-n'}(k2 rho_lm) e^{i (nu-n') phi_lm} beta^m_nu,
 *   rho_lm, phi_lm = polar form of x_l - x_m.
 * beta_dev, alpha_dev: N*P complex in precision prec; alpha is overwritten. */
int mpsl_m2l_dev(mpsl_ctx *ctx, int prec, const void *beta_dev, void *alpha_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the M2L of
 * mpsl_m2l_dev, with the same arguments and result, that allocates nothing.
 * Its partial expansions live in a fixed 64 MiB device array of the library
 * (one per device, held until the process ends), so N P times 16 bytes
 * (FP64) or 8 bytes (FP32) must fit in 64 MiB (MPSL_EINVAL otherwise); the
 * number of source chunks is the default one capped by that room.  The
 * context's tables must already exist (MPSL_ESTATE until a call such as
 * mpsl_m2l_dev or mpsl_apply_dev has built them) and the far field must be
 * direct (MPSL_EUNSUPPORTED with the FMM active).  All calls on one device
 * share the array: calls that overlap in time on one device (other streams,
 * other host threads or contexts) race and must be serialised by the caller. */
int mpsl_m2l_dev_noalloc(mpsl_ctx *ctx, int prec, const void *beta_dev, void *alpha_dev);

/* Row b1, multipole-to-Sommerfeld (Theorem 5.1, factor as derived from the
 * Sommerfeld form (3) of H_0): P+/P- spectra of all multipoles on y = 0 and
 * y = -d, reduced over particles:
 *   P+(lam_q) = -4i sum_m e^{-i lam x_m + g2 y_m}       sum_nu beta^m_nu (-i)^nu ((lam - g2)/k2)^nu
 *   P-(lam_q) = -4i sum_m e^{-i lam x_m - g2 (d + y_m)} sum_nu beta^m_nu (-i)^nu ((lam + g2)/k2)^nu
 * spec_dev: 2*N_S mpsl_c128 (P+ then P-), FP64 for both precisions (the
 * FP32 path sums each particle chunk in FP32, the chunks in FP64). */
int mpsl_m2s_dev(mpsl_ctx *ctx, int prec, const void *beta_dev, void *spec_dev);

/* Row b2, three-layer reflection per node (eq. (10) solved for the
 * middle-layer densities): sigma2+/- = R(lam_q) [P+; P-] (+ source term when
 * src_xy != NULL, a host pointer to one source position).  FP64 always.
 * spec_dev: 2*N_S mpsl_c128 in; sigma_dev: 2*N_S mpsl_c128 out (sigma2+ then
 * sigma2-).  spec_dev may be NULL (source only). */
int mpsl_reflect_dev(mpsl_ctx *ctx, const void *spec_dev, const double *src_xy, void *sigma_dev);

/* Row b3, Sommerfeld-to-local (Lemma 5.1, eq. (40), exact Jacobi-Anger form):
 *   alpha^l_n = (1/4pi) sum_q (w_q/g2) e^{i lam x_l} i^n [sigma2+ e^{g2 y_l} ((lam-g2)/k2)^n
 *                                                      + sigma2- e^{-g2(y_l+d)} ((lam+g2)/k2)^n]
 * sigma_dev: 2*N_S mpsl_c128; alpha_dev: N*P in precision prec, overwritten. */
int mpsl_s2l_dev(mpsl_ctx *ctx, int prec, const void *sigma_dev, void *alpha_dev);

/* Row a2, scattering-matrix apply (Section 3.2 eq. (21), Section 4.1):
 *   y^l = x^l - S_l alpha^l,  S_l[n, n'] = e^{i (n' - n) psi_l} S[n, n'].
 * x_dev may be NULL (then y = S alpha, used for right-hand sides). */
int mpsl_sapply_dev(mpsl_ctx *ctx, int prec, const void *x_dev, const void *alpha_dev, void *y_dev);

/* ---- right-hand side, solve, field ----------------------------------------- */

/* rhs = S a for a unit point source at src_xy (host, 2 doubles): the local
 * expansions a of the source's layer-2 field (Section 5.4, right side of
 * eq. (49)), FP64.  rhs: host array of N*P mpsl_c128. */
int mpsl_rhs(mpsl_ctx *ctx, const double *src_xy, mpsl_c128 *rhs);

typedef struct {
  int precision;      /* MPSL_FP64: FP64 GMRES; MPSL_FP32: FP32 matvecs inside
                         FP64 iterative refinement; the inner Krylov basis
                         is stored in complex64 (orthogonalisation sums in
                         FP64), the residual and solution in FP64           */
  double tol;         /* relative residual target ||r|| / ||b||             */
  int maxiter;        /* total matvec budget of the Krylov solver           */
  int restart;        /* Krylov dimension before restart (0: maxiter, i.e.
                         unrestarted).  At most 20000 (MPSL_EINVAL above);
                         the basis holds (dimension + 1) N P complex128
                         (complex64 with MPSL_FP32) in device memory
                         (MPSL_ENOMEM when it does not fit)                 */
  double inner_tol;   /* MPSL_FP32 only: inner GMRES tolerance (0: 1e-5)   */
} mpsl_opts;

/* ---- preconditioning of the solve ------------------------------------------
 * Section 3.2 writes the system with the scattering matrices applied, which
 * makes the diagonal block of each particle the identity; with
 * MPSL_PRECOND_NONE (default) mpsl_solve runs GMRES on eq. (49) in that form.
 * MPSL_PRECOND_CLUSTER extends the exact diagonal block from one particle to
 * a cluster of nearby particles, for dense packings of high-contrast
 * inclusions (where the Conclusions note that convergence degrades): the
 * centres are cut by recursive coordinate bisection (a set of more than
 * cluster_size particles is ordered by the coordinate of its longer extent,
 * x on equal extents and particle index on equal coordinates, and cut after
 * floor(n/2)) into clusters of at most cluster_size (0: 160) particles; per
 * cluster c the free-space system of its own particles, K_c = I - S_c T_cc
 * (Lemma 3.1 translations between them, their rotated scattering matrices),
 * is assembled and inverted on the device in FP64, and GMRES solves
 * (I - S (T + T_R)) M^{-1} u = S a with M = blockdiag_c K_c, returning
 * beta = M^{-1} u.  This is right preconditioning: the solution and the
 * residual reported are those of eq. (49).  MPSL_FP32 solves apply an FP32
 * copy of the blocks (FP64 arithmetic) and release the FP64 blocks once the
 * copy is made (an FP64 solve afterwards builds them again).  The blocks are
 * built at the first solve or apply after a change of particle, layers or
 * geometry: device memory n_clusters m^2 16 bytes (FP64) or 8 bytes (FP32),
 * m = 64 ceil(largest cluster * P / 64), at most 16384 (MPSL_EINVAL above).
 * A block whose inversion meets a zero pivot or a non-finite value is
 * replaced by the identity (counted by mpsl_get_precond_info).
 * MPSL_EINVAL for another kind or a negative size. */
enum { MPSL_PRECOND_NONE = 0, MPSL_PRECOND_CLUSTER = 1 };
int mpsl_set_preconditioner(mpsl_ctx *ctx, int kind, int cluster_size);

/* Host, no device: cluster_of[j] (n entries) = cluster of particle j under
 * the bisection rule above for centres xy (2n doubles), clusters numbered
 * depth first (first half before second half); *n_clusters = their count.
 * Either output may be NULL, not both.  MPSL_EINVAL for n <= 0, size < 1 or a
 * non-finite coordinate. */
int mpsl_compute_clusters(int64_t n, const double *xy, int cluster_size, int32_t *cluster_of, int *n_clusters);

/* y = M^{-1} x for device vectors of N P complex128 (x, y distinct), with the
 * blocks of precision prec (MPSL_FP32: the FP32 copy, FP64 arithmetic);
 * builds the blocks when needed.  Asynchronous on the context stream after
 * the build.  MPSL_ESTATE without MPSL_PRECOND_CLUSTER. */
int mpsl_precond_apply_dev(mpsl_ctx *ctx, int prec, const void *x_dev, void *y_dev);

/* Shape of the current blocks (zeros before they are built): clusters,
 * particles of the largest, block dimension m, blocks replaced by the
 * identity; and the seconds spent building blocks in this context so far.
 * Any output may be NULL. */
int mpsl_get_precond_info(const mpsl_ctx *ctx, int *n_clusters, int *max_cluster, int *block_dim, int *replaced,
                          double *setup_seconds);

typedef struct {
  int iterations;         /* matvecs of the working precision               */
  int fp64_matvecs;       /* FP64 matvecs (refinement residuals included)   */
  int refinements;        /* outer refinement steps (MPSL_FP32)             */
  double rel_residual;    /* final ||b - A x|| / ||b|| in FP64              */
  double seconds;         /* wall time of the solve                         */
  const double *history;  /* residual history, context-owned, valid until
                             the next call on the context                  */
  int history_len;
  double precond_seconds; /* part of seconds spent building preconditioner
                             blocks (0 when they were already built)       */
  int reorthogonalizations; /* Arnoldi steps that needed a second classical
                             Gram-Schmidt pass (the first removed more than
                             half of the new vector's squared norm)        */
} mpsl_info;

/* Solve eq. (49) for n_rhs sources src_xy[2*r], src_xy[2*r+1] (host).
 * beta_out: host, n_rhs*N*P mpsl_c128 ([rhs][particle][n+p]).  info may be
 * NULL (for n_rhs > 1 it describes the last right-hand side).  Returns
 * MPSL_ENOCONV when the tolerance was not met (beta is still written). */
int mpsl_solve(mpsl_ctx *ctx, int n_rhs, const double *src_xy, const mpsl_opts *opts,
               mpsl_c128 *beta_out, mpsl_info *info);

/* Total field (eq. (36)) at n_rcv receivers rcv_xy (host, 2 doubles each) for
 * n_rhs sources src_xy[2*r], src_xy[2*r+1] and their coefficients beta (host,
 * n_rhs*N*P mpsl_c128, [rhs][particle][n+p], as mpsl_solve writes them):
 * layer 1: G + u_1^s; layer 2: u_2^t + u_2^b + sum of multipoles; layer 3: u_3^s.
 * u_out: host, n_rhs*n_rcv ([rhs][receiver]).  Every source must lie above the
 * top interface (MPSL_EINVAL otherwise, nothing written).  Receivers inside an
 * enclosing disk get NaN and the call returns MPSL_EINSIDE after filling all
 * other values. */
int mpsl_eval_field(mpsl_ctx *ctx, int n_rhs, const double *src_xy, const mpsl_c128 *beta,
                    int64_t n_rcv, const double *rcv_xy, mpsl_c128 *u_out);

/* Launch-shape tuning of the M2L kernel (row a1), per precision.  Variants:
 * 0 = one lane per target holding all P accumulators; 1 = two lanes per target
 * (output halves, the upper half through the mirror symmetry of the Toeplitz
 * translation) for more waves per SIMD at twice the recurrence work;
 * 2, 3 = matrix cores (the translation as a GEMM over (source, order shift)
 * with the source coefficients in shifted form, 16 or 32 targets per wave),
 * for p <= 16 only (a stored 2 or 3 runs as 0 at larger p, and the autotuner
 * skips them there).
 * mpsl_autotune times the variants at 1, 1/2 and 2 times the default number
 * of source chunks, in that order, on the current problem (pseudo-random
 * input, HIP events on the context stream, each launch with the summation of
 * its partial slots) and keeps the fastest (a later candidate must be more
 * than 1 % faster, so near-ties keep the default); mpsl_set_tuning forces a choice
 * (chunks 0 = default).  Tuning is kept until changed; it never changes
 * results beyond floating-point summation order. */
int mpsl_autotune(mpsl_ctx *ctx, int prec);
int mpsl_set_tuning(mpsl_ctx *ctx, int prec, int variant, int chunks);
int mpsl_get_tuning(const mpsl_ctx *ctx, int prec, int *variant, int *chunks, double *m2l_ms);

/* Far field of the free-space M2L (row a1) for large N: a 2D Helmholtz fast
 * multipole method (the O(M (2p+1)^2) acceleration of the GMRES matvec
 * named in Section 3.2 and used for the large-M runs of Section 6.1) on a
 * uniform quadtree of the particle centres.  Pairs in the
 * same or adjacent leaf boxes are summed directly as in row a1; all other
 * pairs go particle -> leaf multipole (Graf, J-shift), multipole ->
 * multipole, multipole -> local between well-separated boxes of one level
 * (the Toeplitz Graf translation of eq. (24) at box scale), local -> local,
 * local -> particle.  Orders per level follow from tol (relative accuracy of
 * the free-space field as the scattering matrix sees it; FP32 uses
 * max(tol, 1e-7)).
 *   method: MPSL_FAR_AUTO   FMM when N > 8000, else direct (default);
 *           MPSL_FAR_DIRECT all pairs directly;
 *           MPSL_FAR_FMM    FMM at any N.
 *   tol:    1e-13 <= tol <= 1e-3 (0 keeps the current value, default 1e-10).
 * The choice takes effect at the next call that builds tables.  With the FMM
 * active mpsl_autotune leaves the tuning unchanged, and mpsl_profile times
 * the whole FMM sequence in place of the M2L kernel. */
enum { MPSL_FAR_AUTO = 0, MPSL_FAR_DIRECT = 1, MPSL_FAR_FMM = 2 };
int mpsl_set_far_field(mpsl_ctx *ctx, int method, double tol);

/* Shape of the FMM built for the current problem (after a first apply or
 * solve): active = 1 when the FMM replaces the direct sum; levels, leaf box
 * side, orders of the leaf and top level in precision prec, true near-field
 * pair count and the translation work (complex MACs) of one apply in prec.
 * Any output pointer may be NULL. */
int mpsl_get_fmm_info(const mpsl_ctx *ctx, int prec, int *active, int *levels, double *leaf_side,
                      int *p_leaf, int *p_top, int64_t *near_pairs, double *tree_cmac);

/* Average duration (ms) of the last `count` launches of the M2L kernel
 * recorded with HIP events on the context stream (0 when not recorded);
 * enable recording with mpsl_profile(ctx, 1). */
int mpsl_profile(mpsl_ctx *ctx, int enable);
int mpsl_profile_read(mpsl_ctx *ctx, double *m2l_ms_avg, int *count);

/* ---- serving: continuous batching of design-loop solves ------------------- */

enum { MPSL_PARTICLE_DISK = 0, MPSL_PARTICLE_STAR = 1, MPSL_PARTICLE_MATRIX = 2 };

/* Contour rule of a request: MPSL_CONTOUR_COUNT as mpsl_set_contour
 * (n_nodes, b, t_max); MPSL_CONTOUR_SPAN as mpsl_set_contour_span
 * (b, t_max, h_max). */
enum { MPSL_CONTOUR_COUNT = 0, MPSL_CONTOUR_SPAN = 1 };

/* Host, no device: the span-rule parameters the comment of
 * mpsl_set_contour_span recommends for a layout of lateral extent x_extent
 * (particles and sources; values below 1 count as 1):
 * b = min(0.2, 2 / X), h_max = 6 / X for tol <= 1e-8 (about 1e-11 on the
 * layered interaction of two particles X apart), else 12 / X (about 1e-6).
 * MPSL_EINVAL for non-finite or non-positive arguments. */
int mpsl_span_contour_params(double x_extent, double tol, double *b, double *h_max);

/* One self-contained solve request (the library copies every array).  A
 * zero-filled tail (contour .. cluster_size) selects the count-rule contour,
 * direct Sommerfeld sums and no cluster preconditioner. */
typedef struct {
  mpsl_c128 k1, k2, k3;    /* layer wavenumbers (see mpsl_set_layers)          */
  double d;                /* middle-layer thickness                           */
  int particle;            /* MPSL_PARTICLE_*                                  */
  double shape[3];         /* disk: R; star: a1, a2, a3                        */
  mpsl_c128 kp;            /* particle wavenumber (disk, star)                 */
  int p;                   /* expansion order                                  */
  int n_bdry;              /* star boundary points (0: 256)                    */
  const mpsl_c128 *S;      /* MPSL_PARTICLE_MATRIX: P x P prototype matrix     */
  double r_enclose;        /* MPSL_PARTICLE_MATRIX: enclosing radius           */
  int64_t n;               /* particles                                        */
  const double *xy;        /* 2n centres                                       */
  const double *rot;       /* n rotations or NULL                              */
  int n_nodes;             /* Sommerfeld nodes (see mpsl_set_contour)          */
  double b, t_max;         /* contour offset and truncation                    */
  double src[2];           /* point source in layer 1                          */
  mpsl_opts opts;          /* precision, tol, maxiter, restart, inner_tol      */
  int contour;             /* MPSL_CONTOUR_COUNT or MPSL_CONTOUR_SPAN          */
  double h_max;            /* MPSL_CONTOUR_SPAN: longest panel                 */
  int sommerfeld;          /* MPSL_SOMM_DIRECT or MPSL_SOMM_INTERP             */
  int precond;             /* MPSL_PRECOND_NONE or MPSL_PRECOND_CLUSTER        */
  int cluster_size;        /* MPSL_PRECOND_CLUSTER: largest cluster (0: 160)   */
} mpsl_request;

typedef struct {
  int status;                 /* MPSL_OK, MPSL_ENOCONV or the request's error   */
  int64_t n;
  int p;
  const mpsl_c128 *beta;      /* n*P coefficients, owned by the server until
                                 mpsl_server_release (NULL on error)          */
  int iterations, fp64_matvecs, refinements;
  double rel_residual;
  double t_submit, t_admit, t_start, t_finish;  /* seconds on the server clock:
                                 queued, admitted (memory reserved), prepared,
                                 finished                                      */
  size_t hbm_bytes;           /* device memory reserved for the request        */
  const char *error;          /* message of a failed request ("" otherwise),
                                 owned by the server until mpsl_server_release */
} mpsl_result;

typedef struct mpsl_server mpsl_server;

/* A server on `device` that keeps at most max_active requests and at most
 * hbm_budget bytes (estimated per request from N, p, N_S and the Krylov
 * dimension) admitted at once.  Admission is in arrival order.  Each admitted
 * request gets its own context and stream; the worker advances all prepared
 * requests by one solver step per tick, so their device work overlaps.
 * Results are identical whatever else is in flight (own buffers, fixed launch
 * shapes, deterministic reductions). */
int mpsl_server_create(mpsl_server **out, int device, size_t hbm_budget, int max_active);
/* Queue a request; returns at once with a ticket.  MPSL_ENOMEM when the request
 * alone exceeds the budget. */
int mpsl_server_submit(mpsl_server *s, const mpsl_request *req, uint64_t *ticket);
/* MPSL_OK and the result when finished, MPSL_PENDING otherwise. */
int mpsl_server_poll(mpsl_server *s, uint64_t ticket, mpsl_result *res);
/* Block until finished (timeout_s < 0: no limit); MPSL_PENDING on timeout. */
int mpsl_server_wait(mpsl_server *s, uint64_t ticket, double timeout_s, mpsl_result *res);
/* Free a finished request's result. */
int mpsl_server_release(mpsl_server *s, uint64_t ticket);
int mpsl_server_stats(mpsl_server *s, int *queued, int *active, uint64_t *completed, size_t *bytes_in_use);
/* Cancel requests not yet admitted (status MPSL_ESTATE), finish the admitted
 * ones, stop the threads and free everything. */
void mpsl_server_destroy(mpsl_server *s);

#ifdef __cplusplus
}
#endif
#endif /* MPSL_H */
