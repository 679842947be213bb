// Internal state of an mpsl context: host copies of the problem, device
// tables and work buffers.
#pragma once

#include <complex>
#include <string>
#include <vector>

#include "common.h"

namespace mpsl {

using zc = std::complex<double>;

// A growable device allocation owned by the context.
struct DBuf {
  void *p = nullptr;
  size_t bytes = 0;
  size_t *used = nullptr;  // the owning context's count of device bytes in use
};

// Device tables derived from the contour alone (FP64 master + FP32 copy).
struct ContourTables {
  // per node q: 2x2 reflection map and source factors (FP64), weights c_q
  DBuf R;        // double2[4 * ns]: R11, R12, R21, R22
  DBuf srcfac;   // double2[2 * ns]: sigma2+/- per unit source density g_q
  DBuf lam;      // double2[ns]
  DBuf gw;       // double2[4 * ns]: g1, g2, g3 (branch Re >= 0), w
  DBuf cq;       // double2[ns]: w_q / (4 pi g2_q)
  DBuf W64, W32; // [2][ns][P]: -4i (-i)^nu u^nu (side +), with v for side -
  DBuf U64;      // double2 [2][ns][P]: i^n u^n, i^n v^n (S2L, before sigma)
};

// Device tables derived from geometry and contour.
struct GeomTables {
  DBuf xy;              // double2[n]
  DBuf rot64, rot32;    // [n][P] e^{i n psi_l}
  DBuf E64, E32;        // [2][n][ns]: e^{-i lam x_m + g2 y_m}, e^{-i lam x_m - g2 (d + y_m)}
  DBuf F64, F32;        // [2][ns][n]: e^{ i lam x_l + g2 y_l}, e^{ i lam x_l - g2 (y_l + d)}
  DBuf pair64, pair32;  // [m][l][4]: H_0, H_1, e^{i phi}, (2/z, 0) of the pair x_l - x_m
  bool pairs_ok = false;
};

// One level of the FMM quadtree (uniform boxes of side s on a common origin;
// level 0 holds the leaves, every level above halves the box count per axis).
struct FmmLevel {
  int nx = 0, ny = 0;
  double s = 0.0;
  int p[2] = {0, 0};          // expansion order per precision [FP64, FP32]
  int64_t moff[2] = {0, 0};   // multipole block in the expansion buffer (complex units)
  int64_t loff[2] = {0, 0};   // local block
  std::vector<uint8_t> occ;   // box holds at least one particle
};

// One launch of the translation kernel: groups of boxes, each writing one
// expansion per box as a sum of Toeplitz products over the group's terms.
struct FmmStage {
  int tasks = 0;                       // groups launched (one block per output window)
  int pout = 0;                        // output expansion length
  int G = 0;                           // boxes per group
  int tiles = 1;                       // output windows of the translation block
  int tj = 64;                         // input tile length
  int64_t task_off = 0;                // first group in FmmPlan::groups
  int nchunk = 1;                      // partial-local chunks summed after the launch
  int64_t sum_off = 0, sum_len = 0;    // chunk 0 and the length of one chunk
};

// Sommerfeld transforms by tile-local interpolation in lambda (M2S and S2L at
// large node counts).  Particles are grouped in rectangular tiles; per tile the
// smooth factor of the plane-wave sums is sampled at Chebyshev nodes of short
// lambda-intervals and interpolated to the contour nodes; nodes near +-k2 and
// on the vertical segment are kept as their own coarse nodes.
struct SommPlan {
  bool active = false;
  int nT = 0, nc = 0, nint = 0, ndir = 0, nfb = 0;
  double tile_w = 0.0, tile_h = 0.0, L_I = 0.0, d_dir = 0.0;
  DBuf perm;        // int32[n]: particles ordered by tile
  DBuf tstart;      // int32[nT + 1]
  DBuf txy;         // double2[nT]: tile centres
  DBuf ptile;       // int32[n]: tile of each particle
  DBuf lamc, gc;    // double2[nc]: coarse nodes and gamma2 there
  DBuf Wc64, Wc32;  // [2][nc][P]: M2S weights at the coarse nodes
  DBuf Zc64, Zc32;  // [2][nc][P]: S2L powers at the coarse nodes
  DBuf Lw;          // double[ns][kSommNc]: interpolation weights
  DBuf ivl;         // int32[nint][4]: fine start (in fperm), fine count, coarse start, unused
  DBuf fperm;       // int32[ns]: contour nodes of the intervals, interval by interval
  DBuf dir;         // int32[ndir][2]: contour node and coarse node of each direct node
  DBuf G;           // work [nrhs][2][nT][nc] in the matvec precision
  DBuf fblk;        // M2S interval-node blocks: (interval, first node)
  DBuf trow;        // int32[nT]: tiles in row-major order (by y, then x)
  DBuf Fx;          // double2[ns]: e^{i lam_q w}, the factor between horizontally adjacent tiles
  DBuf Bp;          // S2L node-chunk partials [chunk][nrhs][2][nT][24 nint] in the matvec precision
  const void *sigma = nullptr;  // S2L densities recorded by the coefficient step
};

struct FmmPlan {
  bool active = false;
  int top = 0;                // index of the top level
  double x0 = 0.0, y0 = 0.0;  // origin of the box grid
  std::vector<FmmLevel> lv;
  // particles sorted by leaf box (row-major leaf index)
  std::vector<int32_t> perm_h, start_h;
  DBuf perm;                  // int32[n]: sorted position -> particle
  DBuf start;                 // int32[leaf boxes + 1]
  // per precision: translation tables, tasks and terms, expansion buffer
  DBuf tab[2];
  DBuf groups[2], terms[2], ins[2], outs[2];
  std::vector<FmmStage> up[2];    // M2M, level 0 -> 1, ...
  std::vector<FmmStage> down[2];  // M2L (+ L2L), top level first
  int64_t p2m_off[2] = {0, 0}, l2p_off[2] = {0, 0};  // per-particle rows in tab
  int64_t xlen[2] = {0, 0};
  DBuf xb;                    // expansion buffer (sized for FP64)
  // near field: padded lists of neighbour sources per sorted target
  int near_k = 0;
  int near_chunks = 1;        // partial slots of the near field
  DBuf near_src;              // int32[near_k][n] source particle (padding: the target)
  DBuf near_cnt;              // int32[n]: true list length
  DBuf near_wave;             // int32[waves]: loop count of each 64-target wave
  DBuf near64, near32;        // [near_k][n][4]: H_0, H_1, e^{i phi}, (2/z, 0)
  int64_t near_pairs = 0;     // true neighbour pairs
  double tree_cmac[2] = {0.0, 0.0};  // translation work per apply
};

}  // namespace mpsl

struct mpsl_ctx {
  int device = 0;
  int n_cu = 256;          // compute units of the device (launch-shape rules)
  size_t hbm_budget = 0;   // device bytes the context may hold (0: no limit)
  size_t hbm_used = 0;     // device bytes it holds now
  hipStream_t stream = nullptr;
  std::string err;

  // layers, top to bottom: wavenumbers, thicknesses of the finite layers
  // (half-space entries unused), interface heights y_0 > ... > y_{L-2}, and
  // the particle layer c whose interfaces are y = 0 and y = -d
  bool has_layers = false;
  std::vector<mpsl::zc> ks;
  std::vector<double> thick, yint;
  int layer_c = 1;
  int pol = MPSL_TM;    // MPSL_TE: (1/k^2) du/dn continuous instead of du/dn
  mpsl::zc k1, k2, k3;  // top half-space, particle layer, bottom half-space
  double d = 0.0;       // particle-layer thickness

  // particle
  bool has_particle = false;
  int p = 0;
  double r_enc = 0.0;
  std::vector<mpsl::zc> S;  // n_types x P x P row-major
  mpsl::DBuf S64, S32;
  // several particle types (one prototype matrix each); r_enc is their maximum
  int n_types = 1;
  std::vector<double> r_type;       // enclosing radius per type
  std::vector<int32_t> ptype;       // type per particle (empty: all type 0)
  mpsl::DBuf types_dev, rtype_dev;  // int32[n] (only with n_types > 1), double[n_types]

  // geometry
  bool has_geom = false;
  int64_t n = 0;
  std::vector<double> xy, rot;

  // contour
  bool has_contour = false;
  int ns = 0;
  std::vector<mpsl::zc> lam, w;

  bool tables_ok = false;  // contour + geometry tables current
  // far field of the free-space M2L: direct all pairs or FMM
  int far_method = MPSL_FAR_AUTO;
  double far_tol = 1e-10;
  mpsl::FmmPlan fmm;
  int somm_method = MPSL_SOMM_DIRECT;
  mpsl::SommPlan somm;
  mpsl::ContourTables ct;
  mpsl::GeomTables gt;

  // work buffers
  mpsl::DBuf part;        // M2L + S2L partial local expansions
  mpsl::DBuf m2s_part;    // M2S partial spectra
  mpsl::DBuf spec;        // double2[2 * ns]
  mpsl::DBuf sigma;       // double2[2 * ns]
  mpsl::DBuf Up64, Up32;  // [2][ns][P]: S2L coefficients scaled by c_q sigma
  mpsl::DBuf xbuf, ybuf;  // host-pointer apply staging
  mpsl::DBuf bt;          // multi-RHS M2L: beta transposed to [n][P][r]
  mpsl::DBuf gm;          // GMRES workspace
  mpsl::DBuf scal;        // reductions
  // cluster-block right preconditioner of the solve (precond.hip)
  int pc_kind = MPSL_PRECOND_NONE;
  int pc_size = 160;      // largest cluster (particles)
  bool pc_ok = false;     // FP64 blocks current for geometry and particle
  bool pc_ok32 = false;   // FP32 copy current
  int pc_nc = 0, pc_mp = 0, pc_m = 0, pc_replaced = 0;
  double pc_setup_s = 0.0;
  mpsl::DBuf pc_blk;      // double2 [nc][m][m]: inverse cluster blocks
  mpsl::DBuf pc_blk32;    // float2 copy
  mpsl::DBuf pc_idx;      // int32 [nc][mp] members, then [nc] counts
  mpsl::DBuf pc_part;     // apply partial sums
  mpsl::DBuf pc_flag;     // inversion failure flags

  // launch shapes
  int m2l_chunks = 0;     // source chunks of the M2L grid (0: automatic)
  struct Tune {
    int variant = -1;     // M2L variant (kM2LWhole ... kM2LMfmaWide), -1 = by order and precision
    int chunks = 0;       // M2L source chunks (0: automatic)
    double ms = 0.0;      // measured M2L time of the choice
  } tune[2];              // [0]: FP64, [1]: FP32
  int s2l_chunks = 0;
  int m2s_chunks = 0;

  // batches (captured HIP graphs) holding raw pointers to this context's
  // tables and matvec work buffers; while > 0 nothing they read may move
  int pinned = 0;

  // profiling of the M2L kernel
  bool prof = false;
  std::vector<hipEvent_t> ev_start, ev_stop;
  std::vector<double> hist;
};

namespace mpsl {
int dev_alloc(mpsl_ctx *ctx, DBuf &b, size_t bytes);
void dev_free(DBuf &b);
// MPSL_ESTATE (with a message) when a batch holds the context, else MPSL_OK.
int check_unpinned(mpsl_ctx *ctx);
int set_err(mpsl_ctx *ctx, int code, const std::string &msg);
int disk_smatrix(double R, double k2, mpsl_c128 kp, int p, int pol, std::vector<zc> &S, std::string &err);
int star_args(double a1, double a2, int a3, mpsl_c128 kp, int p, int n_bdry, int pol, int &nb, std::string &err);
int star_smatrix_checked(double a1, double a2, int a3, double k2, mpsl_c128 kp, int p, int n_bdry, int pol,
                         std::vector<zc> &S, std::string &err);
// Layer stack per contour node lam (host, FP64).  Rup: generalized
// reflection of the layers above the particle layer for an upgoing wave at
// y = 0; Rdn: that of the layers below for a downgoing wave at y = -d; T:
// downgoing amplitude at y = 0 per unit source amplitude at the top interface
// when nothing comes up from below.  Amplitudes are divided by gamma of their
// layer, as in the spectral representation of Section 5.2.
void stack_node(const mpsl_ctx *ctx, zc lam, zc &Rup, zc &Rdn, zc &T);
// Per-layer plane-wave amplitudes for field evaluation: A[j] the downgoing
// wave at the top interface of layer j, B[j] the upgoing one at its bottom
// (A[0] = B[L-1] = 0), g[j] gamma of layer j, from the particle-layer
// densities sp, sm, the particle spectra Pp, Pm and the source amplitude gs.
void stack_amplitudes(const mpsl_ctx *ctx, zc lam, zc gs, zc sp, zc sm, zc Pp, zc Pm, zc *A, zc *B, zc *g);
// The 2 x 2 map (P+, P-) -> (sigma+, sigma-) row-major in m[0..3] and the
// source factors in m[4..5] (sigma+/- per unit source amplitude).
void layer_map(const mpsl_ctx *ctx, zc lam, zc m[6]);
// Validate a layer stack and store it with its interface heights in ctx.
int assign_stack(mpsl_ctx *ctx, int n_layers, const mpsl_c128 *k, const double *thickness, int particle_layer,
                 std::string &err);
zc gamma_branch(zc lam, zc k);
constexpr int kMaxLayers = 64;
int somm_build(mpsl_ctx *ctx);
void somm_free(mpsl_ctx *ctx);
constexpr int kSommNc = 24;  // Chebyshev nodes per lambda-interval
// M2S weights and S2L powers of one node (P entries each): see capi.hip.
void order_weights(zc lam, zc g2, zc k2, int p, zc *Wp, zc *Wm, zc *Up, zc *Um);
// Contour under the span rule (panels of length <= h_max).
int make_contour_span(const std::vector<double> &ks, double b, double t_max, double h_max, std::vector<zc> &lam,
                      std::vector<zc> &w, std::string &err);
int make_contour(const std::vector<double> &ks, int n_nodes, double b, double t_max, std::vector<zc> &lam,
                 std::vector<zc> &w, std::string &err);
int build_tables(mpsl_ctx *ctx);
// Cluster-block preconditioner: build the inverse blocks (FP64, plus the FP32
// copy for prec == MPSL_FP32) and apply y = M^{-1} x on FP64 device vectors.
int precond_build(mpsl_ctx *ctx, int prec);
int precond_apply(mpsl_ctx *ctx, int prec, const void *x, void *y);
// Clusters of the bisection rule for n centres: count and largest size.
int cluster_shape(int64_t n, const double *xy, int size, int *nc, int *mp);
constexpr int kPcDefaultSize = 160;
constexpr int kPcMaxDim = 16384;
int ensure_work(mpsl_ctx *ctx);
int matvec(mpsl_ctx *ctx, int prec, const void *x, void *y, int nrhs);
int matvec(mpsl_ctx *ctx, int prec, const void *x, void *y);
bool fmm_wanted(const mpsl_ctx *ctx);
int fmm_build(mpsl_ctx *ctx);
void fmm_free(mpsl_ctx *ctx);
// Free-space M2L by the FMM into fmm_slots() partial slots of len = n P
// complex entries: the near field split over near_chunks slots, then the far
// field.
int fmm_apply(mpsl_ctx *ctx, int prec, const void *beta, void *part);
inline int fmm_slots(const mpsl_ctx *ctx) { return ctx->fmm.near_chunks + 1; }
}  // namespace mpsl
