// Fast multipole method for the free-space far field of the M2L (row a1),
// the O(M (2p+1)^2) acceleration of the GMRES matvec that Section 3.2 names
// and Section 6.1 uses for large M.
//
// Tree: uniform boxes of side s_0 on a common origin (leaf level 0); level
// l + 1 merges 2x2 boxes of level l.  Expansions about box centres use the
// conventions of the particle expansions (multipole sum_n M_n H_n(k r)
// e^{i n theta}, local sum_n L_n J_n(k r) e^{i n theta}) with per-level
// orders p_l.  Every translation is a Toeplitz product
//   out_{j'} += sum_j tab[j - j' + P_out - 1] in_j       (slots j = n + p)
// with the entries of tab (q the index difference of the translation):
//   P2M, M2M  J_q(k rho) e^{-i q phi},  q = -idx + p_in + p_out,  rho, phi = polar(x_in - c_out)
//   M2L       H_q(k rho) e^{ i q phi},  q = idx - 2 p,            rho, phi = polar(c_out - c_in)
//   L2L, L2P  J_q(k rho) e^{ i q phi},  q = idx - p_in - p_out,   rho, phi = polar(x_out - c_in)
// (Graf's addition theorem in its three forms; the M2L is eq. (24) between
// box centres).  Pairs of particles in the same or adjacent leaf boxes are
// summed directly by the particle M2L kernel over padded neighbour lists.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "kernels.h"

namespace mpsl {

namespace {

constexpr int kMaxBoxOrder = 600;     // largest box order
constexpr int kAutoThreshold = 8000;  // MPSL_FAR_AUTO: FMM above this many particles

constexpr int kTargetBlocks = 2048;    // blocks a translation launch aims for (8 per CU)
constexpr int kMaxChunks = 64;         // term chunks of one stage

struct FmmGroup {
  int64_t outs;  // first of the group's output offsets (one per box)
  int nbox;      // boxes in the group
  int t0, t1;    // term range
  int pad;
};
struct FmmGTerm {
  int64_t tab;   // first entry of the table row
  int64_t ins;   // first of the per-box input offsets (G of them, -1: absent)
  int pin;       // input length
  int pad;
};

__host__ __device__ inline int cdiv(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }

// ---------------------------------------------------------------------------
// Host Bessel sequences (FP64).

// J_q(x) for q = 0..qmax (qmax >= 1): backward recurrence
// J_{q-1} = (2q/x) J_q - J_{q+1} from well above max(qmax, x), rescaled on
// the way down and normalised with the libm J_0(x) or J_1(x).
void bessel_j_seq(double x, int qmax, double *J) {
  std::fill(J, J + qmax + 1, 0.0);
  if (x == 0.0) {
    J[0] = 1.0;
    return;
  }
  const double big = std::max(static_cast<double>(qmax), x);
  const int top = static_cast<int>(big) + 30 + static_cast<int>(std::sqrt(40.0 * (big + 10.0)));
  double jp1 = 0.0, jc = 1e-200;
  for (int q = top; q >= 1; --q) {
    const double jm1 = (2.0 * q / x) * jc - jp1;
    jp1 = jc;
    jc = jm1;
    if (q - 1 <= qmax) J[q - 1] = jc;
    if (std::fabs(jc) > 1e200) {
      jc *= 1e-200;
      jp1 *= 1e-200;
      for (int i = q - 1; i <= qmax; ++i) J[i] *= 1e-200;
    }
  }
  const double a0 = j0(x), a1 = j1(x);
  const double scale = std::fabs(a0) >= std::fabs(a1) ? a0 / J[0] : a1 / J[1];
  for (int i = 0; i <= qmax; ++i) J[i] *= scale;
}

// Y_q(x) for q = 0..qmax by the (stable) upward recurrence.
void bessel_y_seq(double x, int qmax, double *Y) {
  Y[0] = y0(x);
  if (qmax >= 1) Y[1] = y1(x);
  for (int q = 1; q < qmax; ++q) Y[q + 1] = (2.0 * q / x) * Y[q] - Y[q - 1];
}

// Table row of a J-shift (P2M/M2M with sign = -1, L2L/L2P with sign = +1):
// row[idx] = J_q(k rho) e^{i sign q phi}, q = sign (idx - p_in - p_out).
void jshift_row(double k, double dx, double dy, int p_in, int p_out, int sign, zc *row) {
  const int len = 2 * p_in + 2 * p_out + 1;
  const int qmax = std::max(1, p_in + p_out);
  std::vector<double> J(qmax + 1);
  const double rho = std::hypot(dx, dy);
  const double phi = rho > 0.0 ? std::atan2(dy, dx) : 0.0;
  bessel_j_seq(k * rho, qmax, J.data());
  for (int idx = 0; idx < len; ++idx) {
    const int q = sign * (idx - p_in - p_out);
    const int aq = std::abs(q);
    const double jq = (q < 0 && (aq & 1)) ? -J[aq] : J[aq];
    const double a = sign * q * phi;
    row[idx] = zc(jq * std::cos(a), jq * std::sin(a));
  }
}

// M2L row of order p: row[idx] = H_q(k rho) e^{i q phi}, q = idx - 2p,
// rho, phi = polar(dx, dy) (target centre minus source centre).
void m2l_row(double k, double dx, double dy, int p, zc *row) {
  const int qmax = std::max(1, 2 * p);
  std::vector<double> J(qmax + 1), Y(qmax + 1);
  const double rho = std::hypot(dx, dy);
  const double phi = std::atan2(dy, dx);
  bessel_j_seq(k * rho, qmax, J.data());
  bessel_y_seq(k * rho, qmax, Y.data());
  for (int idx = 0; idx <= 4 * p; ++idx) {
    const int q = idx - 2 * p;
    const int aq = std::abs(q);
    zc h(J[aq], Y[aq]);
    if (q < 0 && (aq & 1)) h = -h;
    const double a = q * phi;
    row[idx] = h * zc(std::cos(a), std::sin(a));
  }
}

// ---------------------------------------------------------------------------
// Order per box size: p = max(p_a(D), k s + c(D), p_particle), D = -log10 eps.
// Fitted to the worst-case chain P2M -> M2L (offset 2 boxes) -> L2P with
// both ends weighted by the decay of a scattering matrix, plus margin.
int box_order(double ks, double eps, int p_particle) {
  const double D = -std::log10(eps);
  const int a = static_cast<int>(std::ceil(3.5 * D + 13.0));
  const int b = static_cast<int>(std::ceil(ks + 2.0 * D - 4.0));
  return std::max(std::max(a, b), p_particle);
}

struct Shape {
  double s0 = 0.0;
  int top = 0;
  double cost = 0.0;
};

// Uniform leaf grid of side s0 and the box counts of every level above it.
struct Grid {
  double x0 = 0.0, y0 = 0.0, s0 = 0.0;
  std::vector<int> nx, ny;
  std::vector<std::vector<uint8_t>> occ;
  std::vector<int> leaf;  // leaf box of each particle
};

Grid make_grid(const std::vector<double> &xy, int64_t n, double s0) {
  Grid g;
  double xmin = xy[0], xmax = xy[0], ymin = xy[1], ymax = xy[1];
  for (int64_t i = 1; i < n; ++i) {
    xmin = std::min(xmin, xy[2 * i]);
    xmax = std::max(xmax, xy[2 * i]);
    ymin = std::min(ymin, xy[2 * i + 1]);
    ymax = std::max(ymax, xy[2 * i + 1]);
  }
  g.s0 = s0;
  g.x0 = xmin - 1e-9 * s0;
  g.y0 = ymin - 1e-9 * s0;
  int nx = std::max(1, static_cast<int>(std::floor((xmax - g.x0) / s0)) + 1);
  int ny = std::max(1, static_cast<int>(std::floor((ymax - g.y0) / s0)) + 1);
  g.leaf.resize(n);
  std::vector<uint8_t> occ(static_cast<size_t>(nx) * ny, 0);
  for (int64_t i = 0; i < n; ++i) {
    const int ix = std::min(nx - 1, static_cast<int>(std::floor((xy[2 * i] - g.x0) / s0)));
    const int iy = std::min(ny - 1, static_cast<int>(std::floor((xy[2 * i + 1] - g.y0) / s0)));
    g.leaf[i] = iy * nx + ix;
    occ[g.leaf[i]] = 1;
  }
  g.nx.push_back(nx);
  g.ny.push_back(ny);
  g.occ.push_back(occ);
  while (nx > 1 || ny > 1) {
    const int px = (nx + 1) / 2, py = (ny + 1) / 2;
    std::vector<uint8_t> po(static_cast<size_t>(px) * py, 0);
    for (int iy = 0; iy < ny; ++iy)
      for (int ix = 0; ix < nx; ++ix)
        if (g.occ.back()[iy * nx + ix]) po[(iy / 2) * px + ix / 2] = 1;
    nx = px;
    ny = py;
    g.nx.push_back(nx);
    g.ny.push_back(ny);
    g.occ.push_back(po);
  }
  return g;
}

inline bool adjacent(int ax, int ay, int bx, int by) { return std::abs(ax - bx) <= 1 && std::abs(ay - by) <= 1; }

// Source boxes of the M2L of box (ix, iy) at level l (top: all non-adjacent).
template <typename F>
void for_interactions(const Grid &g, int l, bool top, int ix, int iy, F f) {
  const int nx = g.nx[l], ny = g.ny[l];
  const auto &occ = g.occ[l];
  if (top) {
    for (int jy = 0; jy < ny; ++jy)
      for (int jx = 0; jx < nx; ++jx)
        if (occ[jy * nx + jx] && !adjacent(ix, iy, jx, jy)) f(jx, jy);
    return;
  }
  const int px = ix / 2, py = iy / 2;
  for (int jy = std::max(0, 2 * (py - 1)); jy <= std::min(ny - 1, 2 * (py + 1) + 1); ++jy)
    for (int jx = std::max(0, 2 * (px - 1)); jx <= std::min(nx - 1, 2 * (px + 1) + 1); ++jx)
      if (occ[jy * nx + jx] && !adjacent(ix, iy, jx, jy)) f(jx, jy);
}

// Cost (complex MACs, spread over 256 compute units, the largest single
// task counted in full) of the tree part for a given top level.
double tree_cost(const Grid &g, const std::vector<int> &P, int top, int64_t n, int Pp) {
  const double cus = 256.0;
  double cost = 2.0 * n * Pp * P[0] / cus;  // P2M + L2P
  for (int l = 0; l <= top; ++l) {
    const int nx = g.nx[l], ny = g.ny[l];
    double work = 0.0, maxtask = 0.0;
    int64_t nonempty = 0;
    for (int iy = 0; iy < ny; ++iy)
      for (int ix = 0; ix < nx; ++ix) {
        if (!g.occ[l][iy * nx + ix]) continue;
        ++nonempty;
        int64_t terms = 0;
        for_interactions(g, l, l == top, ix, iy, [&](int, int) { ++terms; });
        const double w = static_cast<double>(terms) * P[l] * P[l];
        work += w;
        maxtask = std::max(maxtask, w);
      }
    maxtask /= std::min(16.0, std::max(1.0, std::ceil(1024.0 / std::max<int64_t>(1, nonempty))));
    cost += std::max(work / cus, maxtask);
    if (l < top) cost += 2.0 * nonempty * P[l] * P[l + 1] / cus;  // M2M + L2L
  }
  return cost;
}

double near_cost(const Grid &g, int64_t n, int Pp) {
  const int nx = g.nx[0], ny = g.ny[0];
  std::vector<int64_t> cnt(static_cast<size_t>(nx) * ny, 0);
  for (int64_t i = 0; i < n; ++i) ++cnt[g.leaf[i]];
  double pairs = 0.0;
  for (int iy = 0; iy < ny; ++iy)
    for (int ix = 0; ix < nx; ++ix) {
      const int64_t c = cnt[iy * nx + ix];
      if (!c) continue;
      int64_t nb = 0;
      for (int jy = std::max(0, iy - 1); jy <= std::min(ny - 1, iy + 1); ++jy)
        for (int jx = std::max(0, ix - 1); jx <= std::min(nx - 1, ix + 1); ++jx) nb += cnt[jy * nx + jx];
      pairs += static_cast<double>(c) * (nb - 1);
    }
  return pairs * Pp * Pp / 256.0;
}

}  // namespace

// ---------------------------------------------------------------------------
// Device kernels.

// P2M: one block per leaf box, one lane per output slot of the box multipole.
template <typename T>
__global__ void k_fmm_p2m(const cv_t<T> *__restrict__ beta, const int *__restrict__ perm,
                          const int *__restrict__ start, const cv_t<T> *__restrict__ tab, int P, int P0,
                          cv_t<T> *__restrict__ mout) {
  __shared__ cx<T> bs[2 * kMaxP + 1];
  const int b = blockIdx.x;
  const int i0 = start[b], i1 = start[b + 1];
  if (i0 == i1) return;
  const int tl = P0 + P - 1;
  const int nrounds = cdiv(P0, blockDim.x);
  for (int r = 0; r < nrounds; ++r) {
    const int jo = r * blockDim.x + threadIdx.x;
    cx<T> acc = mk<T>(0, 0);
    for (int i = i0; i < i1; ++i) {
      __syncthreads();
      if (threadIdx.x < P) bs[threadIdx.x] = ld<T>(beta[static_cast<int64_t>(perm[i]) * P + threadIdx.x]);
      __syncthreads();
      if (jo < P0) {
        const cv_t<T> *row = tab + static_cast<int64_t>(i) * tl + (P0 - 1) - jo;
        for (int j = 0; j < P; ++j) cmac(acc, ld<T>(row[j]), bs[j]);
      }
    }
    if (jo < P0) mout[static_cast<int64_t>(b) * P0 + jo] = st(acc);
  }
}

// L2P: one block per leaf box; lanes over (particle, output slot).
template <typename T>
__global__ void k_fmm_l2p(const cv_t<T> *__restrict__ lin, const int *__restrict__ perm,
                          const int *__restrict__ start, const cv_t<T> *__restrict__ tab, int P, int P0,
                          cv_t<T> *__restrict__ out) {
  extern __shared__ __align__(16) unsigned char l2p_smem[];
  cx<T> *Ls = reinterpret_cast<cx<T> *>(l2p_smem);
  const int b = blockIdx.x;
  const int i0 = start[b], i1 = start[b + 1];
  if (i0 == i1) return;
  for (int j = threadIdx.x; j < P0; j += blockDim.x) Ls[j] = ld<T>(lin[static_cast<int64_t>(b) * P0 + j]);
  __syncthreads();
  const int tl = P0 + P - 1;
  const int tot = (i1 - i0) * P;
  for (int t = threadIdx.x; t < tot; t += blockDim.x) {
    const int i = i0 + t / P, jo = t % P;
    const cv_t<T> *row = tab + static_cast<int64_t>(i) * tl + (P - 1) - jo;
    cx<T> acc = mk<T>(0, 0);
    for (int j = 0; j < P0; ++j) cmac(acc, ld<T>(row[j]), Ls[j]);
    out[static_cast<int64_t>(perm[i]) * P + jo] = st(acc);
  }
}

// Translation of a group of boxes on the matrix cores (one block per group
// task and window of output slots).  The boxes of a group (one parity class)
// share every table row of the task's terms.  For one term (a table row T
// shared by the group's boxes) the group's outputs form a GEMM
//   Y[j'][b] += sum_j T[j - j' + P_out - 1] X_b[j]
// with M = output slot, K = input slot, N = box of the group (16 NB boxes).
// Each wave owns 16 consecutive output slots and all box columns; the block
// (kFmmMfmaWaves waves) a window of 16 kFmmMfmaWaves slots (blockIdx.y).  Per
// term and input tile of tj slots the block stages the group's inputs
// X[j][b] and the window of T its slots reach in LDS (real and imaginary
// parts apart); lane i supplies A[i % 16][i / 16] = T of its output slot and
// input slot and B[i / 16][i % 16] = X of that input slot and box.  Complex
// products take three real MFMAs (Gauss): P1 = sum Ar Br, P2 = sum Ai Bi,
// P3 = sum (Ar + Ai)(Br + Bi); re = P1 - P2, im = P3 - P1 - P2.  Absent
// inputs (ins < 0) and input slots past the term's length are staged as
// zeros.  The input rows are 16 mod 64 words apart (NB = 1) or 48 (NB = 2),
// so that the four rows one B read touches lie in different LDS banks.  The
// block's term list is cached in LDS at the start, and the next tile's
// operands are loaded into registers while the current tile's MFMAs run.
constexpr int kFmmMfmaWaves = 4;
constexpr int kFmmMfmaRows = 16 * kFmmMfmaWaves;  // output slots per block
constexpr int kFmmGroup = 16;                     // boxes per group (16 NB)
constexpr int kFmmTileMax = 128;                  // longest input tile (registers of the prefetch)
constexpr size_t kFmmLds = 40 * 1024;             // LDS of one translation block

constexpr int kFmmTermCache = 32;                 // terms of one block, at most

// LDS bytes of a block's term list (per term: nc input offsets, the table
// offset and the input length).
__host__ __device__ constexpr size_t fmm_term_cache_bytes(int nc) {
  return static_cast<size_t>(kFmmTermCache) * (nc * sizeof(int64_t) + sizeof(int64_t) + sizeof(int));
}

// LDS bytes of the matrix-core translation block for input tiles of tj slots
// (element size esz): the term list, inputs [tj][16 or 48] and the table
// window [tj + rows], real and imaginary parts apart.
inline size_t fmm_mfma_lds(int tj, size_t esz) {
  const int sx = kFmmGroup == 16 ? 16 : 48;
  return fmm_term_cache_bytes(kFmmGroup) +
         (2 * static_cast<size_t>(tj) * sx + 2 * static_cast<size_t>(tj + kFmmMfmaRows)) * esz;
}

template <typename T, int NB>
__global__ __launch_bounds__(64 * kFmmMfmaWaves) void k_fmm_group_mfma(const FmmGroup *__restrict__ groups,
                                                                       const FmmGTerm *__restrict__ terms,
                                                                       const int64_t *__restrict__ ins,
                                                                       const int64_t *__restrict__ outs,
                                                                       const cv_t<T> *__restrict__ xin,
                                                                       const cv_t<T> *__restrict__ tabs,
                                                                       cv_t<T> *__restrict__ xout, int pout, int tj) {
  constexpr int NC = 16 * NB;               // box columns of a group
  constexpr int SX = NB == 1 ? 16 : 48;     // LDS row stride of the staged inputs
  constexpr int RB = kFmmMfmaRows;
  constexpr int NT = 64 * kFmmMfmaWaves;
  static_assert(NT % NC == 0, "each thread stages one box column");
  typedef typename mfma4<T>::v4 v4;
  extern __shared__ __align__(16) unsigned char fgm_smem[];
  // the block's terms (at most kFmmTermCache): per-box input offsets, table
  // offset and input length, read from LDS by every tile's prefetch
  int64_t *Cin = reinterpret_cast<int64_t *>(fgm_smem);  // [kFmmTermCache][NC]
  int64_t *Ctab = Cin + kFmmTermCache * NC;                // [kFmmTermCache]
  int *Cpin = reinterpret_cast<int *>(Ctab + kFmmTermCache);
  T *Xr = reinterpret_cast<T *>(fgm_smem + fmm_term_cache_bytes(NC));  // [tj][SX]
  T *Xi = Xr + tj * SX;
  T *Hr = Xi + tj * SX;                     // [tj + RB]
  T *Hi = Hr + tj + RB;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = lane & 15, kq = lane >> 4;
  const FmmGroup gr = groups[blockIdx.x];
  const int nterm = gr.t1 - gr.t0;          // <= kFmmTermCache (host-checked)
  for (int e = threadIdx.x; e < nterm * NC; e += 64 * kFmmMfmaWaves) {
    const FmmGTerm tm = terms[gr.t0 + e / NC];
    Cin[e] = ins[tm.ins + e % NC];
  }
  for (int e = threadIdx.x; e < nterm; e += 64 * kFmmMfmaWaves) {
    const FmmGTerm tm = terms[gr.t0 + e];
    Ctab[e] = tm.tab;
    Cpin[e] = tm.pin;
  }
  __syncthreads();
  const int ob = blockIdx.y * RB;           // first output slot of the block
  const int sb = threadIdx.x % NC;          // box column this thread stages
  const int sj = threadIdx.x / NC;          // first input row it stages
  constexpr int RS = NT / NC;               // input rows staged per pass
  constexpr int RPT = kFmmTileMax / RS;     // staged input rows per thread, at most
  constexpr int WPT = (kFmmTileMax + RB + NT - 1) / NT;  // staged window entries per thread, at most
  static_assert(RPT <= 32 && WPT <= 32, "bit masks of the staged entries");
  v4 P1[NB], P2[NB], P3[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) P1[nb] = P2[nb] = P3[nb] = v4{0, 0, 0, 0};
  // operands of the next (term, input tile), fetched into registers while
  // the matrix cores work on the current one.  Loads are clamped into range
  // and issued unconditionally; which of them count is kept as bit masks and
  // applied when the values go to LDS, so that nothing waits for the loads
  // before then.
  cx<T> xs[RPT], hs[WPT];
  uint32_t xok = 0, hok = 0;
  auto fetch = [&](int t, int j0) {
    const int tc = t - gr.t0;
    const int tpin = Cpin[tc];
    const int64_t ttab = Ctab[tc];
    const int tl = tpin + pout - 1;
    const int64_t in = sb < gr.nbox ? Cin[tc * NC + sb] : -1;
    // window entry x holds table row kb + x, kb = j0 - ob - (RB - 1) + P_out - 1
    const int kb = j0 - ob - (RB - 1) + pout - 1;
    hok = 0;
#pragma unroll
    for (int r = 0; r < WPT; ++r) {
      const int x = threadIdx.x + r * NT, k = kb + x;
      hs[r] = ld<T>(tabs[ttab + min(max(k, 0), tl - 1)]);
      hok |= static_cast<uint32_t>(x < tj + RB && k >= 0 && k < tl) << r;
    }
    const int64_t ib = in >= 0 ? in : 0;
    xok = 0;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int j = sj + r * RS;
      xs[r] = ld<T>(xin[ib + min(j0 + j, tpin - 1)]);
      xok |= static_cast<uint32_t>(j < tj && in >= 0 && j0 + j < tpin) << r;
    }
  };
  if (gr.t0 < gr.t1) fetch(gr.t0, 0);
  for (int t = gr.t0, j0 = 0; t < gr.t1;) {
    const int pin = Cpin[t - gr.t0];
    __syncthreads();  // the previous tile consumed
#pragma unroll
    for (int r = 0; r < WPT; ++r) {
      const int x = threadIdx.x + r * NT;
      if (x < tj + RB) {
        const bool ok = (hok >> r) & 1;
        Hr[x] = ok ? hs[r].re : T(0);
        Hi[x] = ok ? hs[r].im : T(0);
      }
    }
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int j = sj + r * RS;
      if (j < tj) {
        const bool ok = (xok >> r) & 1;
        Xr[j * SX + sb] = ok ? xs[r].re : T(0);
        Xi[j * SX + sb] = ok ? xs[r].im : T(0);
      }
    }
    __syncthreads();
    int tn = t, jn = j0 + tj;
    if (jn >= pin) {
      ++tn;
      jn = 0;
    }
    if (tn < gr.t1) fetch(tn, jn);
    // k steps of 4 input slots in groups of KU (tj is a multiple of 4 KU, and
    // the staged rows past the term's input are zeros)
    constexpr int KU = 4;
    const int kgroups = (min(tj, pin - j0) + 4 * KU - 1) / (4 * KU);
    // output slot ob + 16 w + i and input slot j0 + jl meet at window entry
    // jl - 16 w - i + RB - 1
    const int xo = RB - 1 - 16 * w - i;
    // a wave whose 16 output slots all lie past P_out (the last window of a
    // stage) stages its share and meets the barriers but multiplies nothing
    const int kgw = ob + 16 * w < pout ? kgroups : 0;
    for (int kg = 0; kg < kgw; ++kg) {
      T ar[KU], ai[KU], br[KU][NB], bi[KU][NB];
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int jl = 4 * (KU * kg + u) + kq;
        ar[u] = Hr[jl + xo];
        ai[u] = Hi[jl + xo];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          br[u][nb] = Xr[jl * SX + 16 * nb + i];
          bi[u][nb] = Xi[jl * SX + 16 * nb + i];
        }
      }
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const T as = ar[u] + ai[u];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          P1[nb] = mfma4<T>::mac(ar[u], br[u][nb], P1[nb]);
          P2[nb] = mfma4<T>::mac(ai[u], bi[u][nb], P2[nb]);
          P3[nb] = mfma4<T>::mac(as, br[u][nb] + bi[u][nb], P3[nb]);
        }
      }
    }
    t = tn;
    j0 = jn;
  }
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int b = 16 * nb + i;
    if (b >= gr.nbox) continue;
    const int64_t o = outs[gr.outs + b];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int slot = ob + 16 * w + mfma4<T>::row(lane, j);
      const T p1 = P1[nb][j], p2 = P2[nb][j], p3 = P3[nb][j];
      if (slot < pout) xout[o + slot] = st(mk<T>(p1 - p2, p3 - p1 - p2));
    }
  }
}

// Partial locals of a chunked level: x[i] = sum_c x[c len + i], in order.
template <typename T>
__global__ void k_fmm_chunk_sum(cv_t<T> *__restrict__ x, int64_t len, int nchunk) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= len) return;
  cx<T> s = ld<T>(x[i]);
  for (int c = 1; c < nchunk; ++c) s = s + ld<T>(x[c * len + i]);
  x[i] = st(s);
}

// Near-field pair entries in the layout of the all-pairs table:
// [j][i][4] = H_0, H_1, e^{i phi}, (2/z, 0) of target perm[i] and source
// src[j][i]; zeros for padding (j >= cnt[i]).
__global__ void k_near_tables(const double2 *__restrict__ xy, const int *__restrict__ perm,
                              const int *__restrict__ src, const int *__restrict__ cnt, int n, int K,
                              double k2, double2 *__restrict__ t64, float2 *__restrict__ t32) {
  const int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (e >= static_cast<int64_t>(K) * n) return;
  const int j = static_cast<int>(e / n), i = static_cast<int>(e % n);
  double2 v[4] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0), make_double2(0.0, 0.0),
                  make_double2(0.0, 0.0)};
  if (j < cnt[i]) {
    const int l = perm[i], m = src[e];
    const double dx = xy[l].x - xy[m].x, dy = xy[l].y - xy[m].y;
    const double rho = sqrt(dx * dx + dy * dy);
    const double z = k2 * rho;
    v[0] = make_double2(j0(z), y0(z));
    v[1] = make_double2(j1(z), y1(z));
    v[2] = make_double2(dx / rho, dy / rho);
    v[3] = make_double2(2.0 / z, 0.0);
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    t64[4 * e + c] = v[c];
    t32[4 * e + c] = make_float2(static_cast<float>(v[c].x), static_cast<float>(v[c].y));
  }
}

// ---------------------------------------------------------------------------
// Host: plan.

bool fmm_wanted(const mpsl_ctx *ctx) {
  if (ctx->far_method == MPSL_FAR_FMM) return true;
  if (ctx->far_method == MPSL_FAR_DIRECT) return false;
  return ctx->n > kAutoThreshold;
}

void fmm_free(mpsl_ctx *ctx) {
  FmmPlan &f = ctx->fmm;
  for (int i = 0; i < 2; ++i) {
    dev_free(f.tab[i]);
    dev_free(f.groups[i]);
    dev_free(f.terms[i]);
    dev_free(f.ins[i]);
    dev_free(f.outs[i]);
  }
  dev_free(f.perm);
  dev_free(f.start);
  dev_free(f.xb);
  dev_free(f.near_src);
  dev_free(f.near_cnt);
  dev_free(f.near_wave);
  dev_free(f.near64);
  dev_free(f.near32);
  f.active = false;
}

namespace {

template <typename V>
int upload(mpsl_ctx *ctx, DBuf &b, const std::vector<V> &v) {
  int rc = dev_alloc(ctx, b, std::max<size_t>(1, v.size()) * sizeof(V));
  if (rc) return rc;
  if (!v.empty()) MPSL_HIP_TRY(ctx, hipMemcpy(b.p, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice));
  return MPSL_OK;
}

// Tables, tasks and terms of one precision.  Returns false when a table
// entry is not representable (then the shape is rejected).
bool build_precision(mpsl_ctx *ctx, const Grid &g, int top, int pi, std::vector<zc> &tab,
                     std::vector<FmmGroup> &groups, std::vector<FmmGTerm> &terms, std::vector<int64_t> &ins,
                     std::vector<int64_t> &outs, std::string &why) {
  FmmPlan &f = ctx->fmm;
  const double k = ctx->k2.real();
  const int p = ctx->p, P = 2 * p + 1;
  const int64_t n = ctx->n;
  std::vector<int> Pl(top + 1);
  for (int l = 0; l <= top; ++l) Pl[l] = 2 * f.lv[l].p[pi] + 1;

  // launch shape of every stage (matrix-core translation kernel): output
  // windows of kFmmMfmaRows slots, groups of kFmmGroup boxes, term chunks
  // (partial expansions summed afterwards in a fixed order) so that every
  // launch has enough blocks to fill the chip, and input tiles that split the
  // longest input evenly within the LDS budget
  const size_t esz = pi == 0 ? sizeof(double) : sizeof(float);
  auto plan = [&](int pout, int pin_max, const std::vector<int64_t> &cls, int nterms) {
    FmmStage s;
    s.pout = pout;
    s.tiles = cdiv(pout, kFmmMfmaRows);
    s.G = kFmmGroup;
    int64_t blocks = 0;
    for (auto c : cls) blocks += cdiv(c, s.G);
    blocks *= s.tiles;
    s.nchunk = std::min({kMaxChunks, std::max(1, nterms), std::max(1, cdiv(kTargetBlocks, std::max<int64_t>(1, blocks)))});
    s.nchunk = std::max(s.nchunk, cdiv(std::max(1, nterms), kFmmTermCache));  // chunks fit the term cache
    int cap = kFmmTileMax;
    while (cap > 16 && fmm_mfma_lds(cap, esz) > kFmmLds) cap -= 16;
    const int ntile = cdiv(std::max(1, pin_max), cap);
    s.tj = cdiv(cdiv(std::max(1, pin_max), ntile), 16) * 16;  // whole groups of four k steps
    return s;
  };
  std::vector<FmmStage> shp_up(top + 1), shp_dn(top + 1);
  for (int l = 0; l <= top; ++l) {
    std::vector<int64_t> cls(4, 0);
    int64_t nonempty = 0;
    for (int b = 0; b < g.nx[l] * g.ny[l]; ++b)
      if (g.occ[l][b]) {
        ++cls[l < top ? ((b % g.nx[l]) & 1) + 2 * ((b / g.nx[l]) & 1) : 0];
        ++nonempty;
      }
    // terms of one group: 27 interaction offsets of a parity class and the
    // parent's L2L below the top; at the top every offset of the level's
    // box grid outside the 3 x 3 neighbourhood may occur
    const int top_terms = std::max(1, (2 * g.nx[l] - 1) * (2 * g.ny[l] - 1) - 9);
    shp_dn[l] = plan(Pl[l], l < top ? std::max(Pl[l], Pl[l + 1]) : Pl[l], cls, l < top ? 28 : top_terms);
    if (l > 0) shp_up[l] = plan(Pl[l], Pl[l - 1], {nonempty}, 4);
  }

  // expansion buffer: multipoles of every level, then locals (chunk copies)
  int64_t off = 0;
  for (int l = 0; l <= top; ++l) {
    f.lv[l].moff[pi] = off;
    off += static_cast<int64_t>(g.nx[l]) * g.ny[l] * Pl[l] * (l > 0 ? shp_up[l].nchunk : 1);
  }
  for (int l = 0; l <= top; ++l) {
    f.lv[l].loff[pi] = off;
    off += static_cast<int64_t>(g.nx[l]) * g.ny[l] * Pl[l] * shp_dn[l].nchunk;
  }
  f.xlen[pi] = off;

  tab.clear();
  // M2L rows: offset (dx, dy) = source - target in boxes, |dx| <= Dx, |dy| <= Dy
  std::vector<int64_t> m2l_base(top + 1);
  std::vector<int> Dx(top + 1), Dy(top + 1);
  for (int l = 0; l <= top; ++l) {
    Dx[l] = l == top ? g.nx[l] - 1 : std::min(3, g.nx[l] - 1);
    Dy[l] = l == top ? g.ny[l] - 1 : std::min(3, g.ny[l] - 1);
    m2l_base[l] = static_cast<int64_t>(tab.size());
    const int L = 2 * Pl[l] - 1;
    const int p_l = f.lv[l].p[pi];
    const double s = f.lv[l].s;
    tab.resize(tab.size() + static_cast<size_t>(2 * Dy[l] + 1) * (2 * Dx[l] + 1) * L, zc(0.0, 0.0));
    for (int dy = -Dy[l]; dy <= Dy[l]; ++dy)
      for (int dx = -Dx[l]; dx <= Dx[l]; ++dx) {
        if (std::abs(dx) <= 1 && std::abs(dy) <= 1) continue;
        zc *row = tab.data() + m2l_base[l] + ((dy + Dy[l]) * (2 * Dx[l] + 1) + (dx + Dx[l])) * static_cast<int64_t>(L);
        m2l_row(k, -dx * s, -dy * s, p_l, row);
      }
  }
  // M2M (child -> parent) and L2L (parent -> child), child position c = 2 b + a
  std::vector<int64_t> up_base(top), dn_base(top);
  for (int l = 0; l < top; ++l) {
    const int pa = f.lv[l].p[pi], pb = f.lv[l + 1].p[pi];
    const int L = 2 * pa + 2 * pb + 1;
    const double s = f.lv[l].s;
    up_base[l] = static_cast<int64_t>(tab.size());
    tab.resize(tab.size() + 4 * static_cast<size_t>(L));
    for (int c = 0; c < 4; ++c)
      jshift_row(k, ((c & 1) - 0.5) * s, ((c >> 1) - 0.5) * s, pa, pb, -1, tab.data() + up_base[l] + c * L);
    dn_base[l] = static_cast<int64_t>(tab.size());
    tab.resize(tab.size() + 4 * static_cast<size_t>(L));
    for (int c = 0; c < 4; ++c)
      jshift_row(k, ((c & 1) - 0.5) * s, ((c >> 1) - 0.5) * s, pb, pa, +1, tab.data() + dn_base[l] + c * L);
  }
  // per sorted particle: P2M and L2P rows
  const int p0 = f.lv[0].p[pi];
  const int Lp = P + Pl[0] - 1;
  f.p2m_off[pi] = static_cast<int64_t>(tab.size());
  tab.resize(tab.size() + static_cast<size_t>(n) * Lp);
  f.l2p_off[pi] = static_cast<int64_t>(tab.size());
  tab.resize(tab.size() + static_cast<size_t>(n) * Lp);
  const int nx0 = g.nx[0];
  for (int64_t i = 0; i < n; ++i) {
    const int m = f.perm_h[i];
    const int b = g.leaf[m];
    const double cx0 = f.x0 + ((b % nx0) + 0.5) * f.lv[0].s, cy0 = f.y0 + ((b / nx0) + 0.5) * f.lv[0].s;
    const double dx = ctx->xy[2 * m] - cx0, dy = ctx->xy[2 * m + 1] - cy0;
    jshift_row(k, dx, dy, p, p0, -1, tab.data() + f.p2m_off[pi] + i * Lp);
    jshift_row(k, dx, dy, p0, p, +1, tab.data() + f.l2p_off[pi] + i * Lp);
  }
  const double lim = pi == 0 ? 1e300 : 1e37;
  for (const zc &v : tab)
    if (!(std::fabs(v.real()) < lim && std::fabs(v.imag()) < lim)) {
      why = "translation table entry out of range";
      return false;
    }

  // groups and terms
  groups.clear();
  terms.clear();
  ins.clear();
  outs.clear();
  f.up[pi].clear();
  f.down[pi].clear();
  auto shape = [&](FmmStage &st, const FmmStage &from) {
    st = from;
    st.tasks = 0;
    st.task_off = static_cast<int64_t>(groups.size());
  };
  // one term: table row, input length, per-box inputs (G entries)
  auto add_term = [&](int64_t tab_row, int pin, const std::vector<int64_t> &in) {
    FmmGTerm t{};
    t.tab = tab_row;
    t.ins = static_cast<int64_t>(ins.size());
    t.pin = pin;
    ins.insert(ins.end(), in.begin(), in.end());
    terms.push_back(t);
  };
  auto add_group = [&](FmmStage &st, const std::vector<int64_t> &out_rows, int t0, int t1) {
    FmmGroup gr{};
    gr.outs = static_cast<int64_t>(outs.size());
    gr.nbox = static_cast<int>(out_rows.size());
    gr.t0 = t0;
    gr.t1 = t1;
    outs.insert(outs.end(), out_rows.begin(), out_rows.end());
    groups.push_back(gr);
    ++st.tasks;
  };
  // M2M, level l -> l + 1: groups of parents; terms are the four child positions
  for (int l = 0; l < top; ++l) {
    FmmStage st;
    shape(st, shp_up[l + 1]);
    const int nxa = g.nx[l], nya = g.ny[l], nxb = g.nx[l + 1], nyb = g.ny[l + 1];
    const int64_t nbb = static_cast<int64_t>(nxb) * nyb;
    std::vector<int> par;
    for (int b = 0; b < nxb * nyb; ++b)
      if (g.occ[l + 1][b]) par.push_back(b);
    for (size_t g0 = 0; g0 < par.size(); g0 += st.G) {
      const size_t g1 = std::min(par.size(), g0 + st.G);
      const int t0 = static_cast<int>(terms.size());
      for (int c = 0; c < 4; ++c) {
        std::vector<int64_t> in(st.G, -1);
        bool any = false;
        for (size_t i = g0; i < g1; ++i) {
          const int cx = 2 * (par[i] % nxb) + (c & 1), cy = 2 * (par[i] / nxb) + (c >> 1);
          if (cx >= nxa || cy >= nya || !g.occ[l][cy * nxa + cx]) continue;
          in[i - g0] = f.lv[l].moff[pi] + static_cast<int64_t>(cy * nxa + cx) * Pl[l];
          any = true;
        }
        if (any) add_term(up_base[l] + c * static_cast<int64_t>(Pl[l] + Pl[l + 1] - 1), Pl[l], in);
      }
      const int t1 = static_cast<int>(terms.size());
      for (int ch = 0; ch < st.nchunk; ++ch) {  // even split: sizes differ by at most one
        std::vector<int64_t> rows;
        for (size_t i = g0; i < g1; ++i) rows.push_back(f.lv[l + 1].moff[pi] + (ch * nbb + par[i]) * Pl[l + 1]);
        add_group(st, rows, t0 + ch * (t1 - t0) / st.nchunk, t0 + (ch + 1) * (t1 - t0) / st.nchunk);
      }
    }
    st.sum_off = f.lv[l + 1].moff[pi];
    st.sum_len = nbb * Pl[l + 1];
    f.up[pi].push_back(st);
  }
  // M2L (+ L2L from the parent), top level first: groups of boxes of one
  // parity class (top level: one class); terms are the offsets of the union
  // of the group's interaction lists
  for (int l = top; l >= 0; --l) {
    FmmStage st;
    shape(st, shp_dn[l]);
    const int nx = g.nx[l], ny = g.ny[l];
    const int64_t nbl = static_cast<int64_t>(nx) * ny;
    const int L = 2 * Pl[l] - 1;
    const int ncls = l < top ? 4 : 1;
    std::vector<std::vector<int>> cls(ncls);
    for (int b = 0; b < nx * ny; ++b)
      if (g.occ[l][b]) cls[l < top ? ((b % nx) & 1) + 2 * ((b / nx) & 1) : 0].push_back(b);
    for (int c = 0; c < ncls; ++c) {
      const auto &bx = cls[c];
      for (size_t g0 = 0; g0 < bx.size(); g0 += st.G) {
        const size_t g1 = std::min(bx.size(), g0 + st.G);
        const int t0 = static_cast<int>(terms.size());
        if (l < top) {
          std::vector<int64_t> in(st.G, -1);
          for (size_t i = g0; i < g1; ++i) {
            const int ix = bx[i] % nx, iy = bx[i] / nx;
            in[i - g0] = f.lv[l + 1].loff[pi] + static_cast<int64_t>((iy / 2) * g.nx[l + 1] + ix / 2) * Pl[l + 1];
          }
          add_term(dn_base[l] + c * static_cast<int64_t>(Pl[l] + Pl[l + 1] - 1), Pl[l + 1], in);
        }
        for (int dy = -Dy[l]; dy <= Dy[l]; ++dy)
          for (int dx = -Dx[l]; dx <= Dx[l]; ++dx) {
            if (std::abs(dx) <= 1 && std::abs(dy) <= 1) continue;
            std::vector<int64_t> in(st.G, -1);
            bool any = false;
            for (size_t i = g0; i < g1; ++i) {
              const int ix = bx[i] % nx, iy = bx[i] / nx;
              const int jx = ix + dx, jy = iy + dy;
              if (jx < 0 || jx >= nx || jy < 0 || jy >= ny || !g.occ[l][jy * nx + jx]) continue;
              if (l < top && (std::abs(jx / 2 - ix / 2) > 1 || std::abs(jy / 2 - iy / 2) > 1)) continue;
              in[i - g0] = f.lv[l].moff[pi] + static_cast<int64_t>(jy * nx + jx) * Pl[l];
              any = true;
            }
            if (any)
              add_term(m2l_base[l] + ((dy + Dy[l]) * (2 * Dx[l] + 1) + (dx + Dx[l])) * static_cast<int64_t>(L), Pl[l],
                       in);
          }
        const int t1 = static_cast<int>(terms.size());
        for (int ch = 0; ch < st.nchunk; ++ch) {  // even split: sizes differ by at most one
          std::vector<int64_t> rows;
          for (size_t i = g0; i < g1; ++i) rows.push_back(f.lv[l].loff[pi] + (ch * nbl + bx[i]) * Pl[l]);
          add_group(st, rows, t0 + ch * (t1 - t0) / st.nchunk, t0 + (ch + 1) * (t1 - t0) / st.nchunk);
        }
      }
    }
    st.sum_off = f.lv[l].loff[pi];
    st.sum_len = nbl * Pl[l];
    f.down[pi].push_back(st);
  }
  // every access of the translation kernel stays inside its buffers
  const int64_t tsz = static_cast<int64_t>(tab.size());
  double cm = 2.0 * static_cast<double>(n) * P * Pl[0];  // P2M + L2P
  for (int s = 0; s < 2; ++s) {
    const auto &stages = s == 0 ? f.up[pi] : f.down[pi];
    for (const auto &st : stages) {
      if (st.nchunk > 1 && (st.sum_off < 0 || st.sum_off + st.nchunk * st.sum_len > f.xlen[pi])) {
        why = "chunked locals outside the expansion buffer";
        return false;
      }
      for (int64_t gi = 0; gi < st.tasks; ++gi) {
        const FmmGroup &gr = groups[st.task_off + gi];
        if (gr.nbox < 1 || gr.nbox > st.G || gr.t0 > gr.t1 || gr.t1 > static_cast<int>(terms.size()) ||
            gr.t1 - gr.t0 > kFmmTermCache ||
            gr.outs + gr.nbox > static_cast<int64_t>(outs.size())) {
          why = "group outside its lists";
          return false;
        }
        for (int i = 0; i < gr.nbox; ++i)
          if (outs[gr.outs + i] < 0 || outs[gr.outs + i] + st.pout > f.xlen[pi]) {
            why = "group output outside the expansion buffer";
            return false;
          }
        for (int t = gr.t0; t < gr.t1; ++t) {
          const FmmGTerm &tm = terms[t];
          if (tm.pin < 1 || tm.tab < 0 || tm.tab + tm.pin + st.pout - 1 > tsz || tm.ins < 0 ||
              tm.ins + st.G > static_cast<int64_t>(ins.size())) {
            why = "term outside its buffers";
            return false;
          }
          for (int i = 0; i < st.G; ++i) {
            const int64_t v = ins[tm.ins + i];
            if (v >= 0 && v + tm.pin > f.xlen[pi]) {
              why = "term input outside the expansion buffer";
              return false;
            }
            if (v >= 0 && i < gr.nbox) cm += static_cast<double>(tm.pin) * st.pout;
          }
        }
      }
    }
  }
  if (f.p2m_off[pi] + static_cast<int64_t>(n) * Lp > tsz || f.l2p_off[pi] + static_cast<int64_t>(n) * Lp > tsz) {
    why = "particle rows outside the table";
    return false;
  }
  f.tree_cmac[pi] = cm;
  return true;
}

}  // namespace

int fmm_build(mpsl_ctx *ctx) {
  FmmPlan &f = ctx->fmm;
  f.active = false;
  const int64_t n = ctx->n;
  const int p = ctx->p, P = 2 * p + 1;
  const double k = ctx->k2.real();
  const double eps[2] = {ctx->far_tol, std::max(ctx->far_tol, 1e-7)};
  if (n > (int64_t(1) << 30) / 64) return set_err(ctx, MPSL_EUNSUPPORTED, "too many particles for the FMM");

  // candidate shapes: leaf side (k s0 from 8 to 96) x top level
  std::vector<Shape> cands;
  for (double ks0 : {8.0, 12.0, 16.0, 24.0, 32.0, 48.0, 64.0, 96.0}) {
    const double s0 = ks0 / k;
    const Grid g = make_grid(ctx->xy, n, s0);
    const double nc = near_cost(g, n, P);
    const int nlev = static_cast<int>(g.nx.size());
    std::vector<int> Pl(nlev);
    for (int l = 0; l < nlev; ++l) Pl[l] = 2 * box_order(k * s0 * std::ldexp(1.0, l), eps[0], p) + 1;
    for (int top = 0; top < nlev; ++top) {
      if (Pl[top] > 2 * kMaxBoxOrder + 1) break;
      int64_t nb = static_cast<int64_t>(g.nx[top]) * g.ny[top];
      if (nb > 1024) continue;
      const double offs = static_cast<double>(2 * g.nx[top] - 1) * (2 * g.ny[top] - 1);
      if (offs * (2 * Pl[top] - 1) > 2e7) continue;
      Shape sh;
      sh.s0 = s0;
      sh.top = top;
      sh.cost = nc + 1.5 * tree_cost(g, Pl, top, n, P);
      cands.push_back(sh);
    }
  }
  std::sort(cands.begin(), cands.end(), [](const Shape &a, const Shape &b) { return a.cost < b.cost; });
  if (cands.empty()) return set_err(ctx, MPSL_EUNSUPPORTED, "no FMM tree shape fits the problem");

  std::string why;
  for (const Shape &sh : cands) {
    const Grid g = make_grid(ctx->xy, n, sh.s0);
    const int top = sh.top;
    f.top = top;
    f.x0 = g.x0;
    f.y0 = g.y0;
    f.lv.assign(top + 1, FmmLevel());
    bool ok = true;
    for (int l = 0; l <= top; ++l) {
      FmmLevel &L = f.lv[l];
      L.nx = g.nx[l];
      L.ny = g.ny[l];
      L.s = sh.s0 * std::ldexp(1.0, l);
      L.occ = g.occ[l];
      for (int pi = 0; pi < 2; ++pi) L.p[pi] = box_order(k * L.s, eps[pi], p);
      if (L.p[0] > kMaxBoxOrder) ok = false;
    }
    if (!ok) continue;
    // sort particles by leaf box (counting sort, stable)
    const int nb0 = g.nx[0] * g.ny[0];
    f.start_h.assign(nb0 + 1, 0);
    for (int64_t i = 0; i < n; ++i) ++f.start_h[g.leaf[i] + 1];
    for (int b = 0; b < nb0; ++b) f.start_h[b + 1] += f.start_h[b];
    f.perm_h.assign(n, 0);
    {
      std::vector<int32_t> fill(f.start_h.begin(), f.start_h.end() - 1);
      for (int64_t i = 0; i < n; ++i) f.perm_h[fill[g.leaf[i]]++] = static_cast<int32_t>(i);
    }
    std::vector<zc> tab[2];
    std::vector<FmmGroup> groups[2];
    std::vector<FmmGTerm> terms[2];
    std::vector<int64_t> ins[2], outs[2];
    for (int pi = 0; pi < 2 && ok; ++pi)
      ok = build_precision(ctx, g, top, pi, tab[pi], groups[pi], terms[pi], ins[pi], outs[pi], why);
    if (!ok) continue;

    // near field: padded neighbour lists over the 3 x 3 leaf boxes
    const int nx0 = g.nx[0], ny0 = g.ny[0];
    std::vector<int32_t> cnt(n, 0);
    int K = 0;
    int64_t pairs = 0;
    for (int64_t i = 0; i < n; ++i) {
      const int b = g.leaf[f.perm_h[i]];
      const int ix = b % nx0, iy = b / nx0;
      int c = 0;
      for (int jy = std::max(0, iy - 1); jy <= std::min(ny0 - 1, iy + 1); ++jy)
        c += f.start_h[jy * nx0 + std::min(nx0 - 1, ix + 1) + 1] - f.start_h[jy * nx0 + std::max(0, ix - 1)];
      cnt[i] = c - 1;
      K = std::max(K, c - 1);
      pairs += c - 1;
    }
    K = std::max(K, 1);
    std::vector<int32_t> src(static_cast<size_t>(K) * n);
    for (int64_t i = 0; i < n; ++i) {
      const int self = f.perm_h[i];
      const int b = g.leaf[self];
      const int ix = b % nx0, iy = b / nx0;
      int j = 0;
      for (int jy = std::max(0, iy - 1); jy <= std::min(ny0 - 1, iy + 1); ++jy) {
        const int a0 = f.start_h[jy * nx0 + std::max(0, ix - 1)];
        const int a1 = f.start_h[jy * nx0 + std::min(nx0 - 1, ix + 1) + 1];
        for (int a = a0; a < a1; ++a)
          if (f.perm_h[a] != self) src[static_cast<size_t>(j++) * n + i] = f.perm_h[a];
      }
      for (; j < K; ++j) src[static_cast<size_t>(j) * n + i] = self;
    }
    const int64_t waves = 2 * static_cast<int64_t>(cdiv(n, 128));  // whole blocks of the near kernel
    std::vector<int32_t> wave(waves, 0);
    for (int64_t i = 0; i < n; ++i) wave[i / 64] = std::max(wave[i / 64], cnt[i]);
    f.near_k = K;
    f.near_pairs = pairs;
    // split the neighbour lists over several partial slots when one lane
    // per target leaves the chip short of waves
    f.near_chunks = std::max(1, std::min({8, K, cdiv(2048, cdiv(n, 128))}));

    int rc;
    if ((rc = upload(ctx, f.perm, f.perm_h)) || (rc = upload(ctx, f.start, f.start_h)) ||
        (rc = upload(ctx, f.near_src, src)) || (rc = upload(ctx, f.near_cnt, cnt)) ||
        (rc = upload(ctx, f.near_wave, wave)))
      return rc;
    for (int pi = 0; pi < 2; ++pi) {
      if ((rc = upload(ctx, f.groups[pi], groups[pi])) || (rc = upload(ctx, f.terms[pi], terms[pi])) ||
          (rc = upload(ctx, f.ins[pi], ins[pi])) || (rc = upload(ctx, f.outs[pi], outs[pi])))
        return rc;
      if (pi == 0) {
        std::vector<double2> t(tab[0].size());
        for (size_t i = 0; i < t.size(); ++i) t[i] = make_double2(tab[0][i].real(), tab[0][i].imag());
        if ((rc = upload(ctx, f.tab[0], t))) return rc;
      } else {
        std::vector<float2> t(tab[1].size());
        for (size_t i = 0; i < t.size(); ++i)
          t[i] = make_float2(static_cast<float>(tab[1][i].real()), static_cast<float>(tab[1][i].imag()));
        if ((rc = upload(ctx, f.tab[1], t))) return rc;
      }
    }
    const size_t xb = std::max(static_cast<size_t>(f.xlen[0]) * sizeof(double2),
                               static_cast<size_t>(f.xlen[1]) * sizeof(float2));
    if ((rc = dev_alloc(ctx, f.xb, xb))) return rc;
    const size_t ne = static_cast<size_t>(K) * n * 4;
    if ((rc = dev_alloc(ctx, f.near64, ne * sizeof(double2))) || (rc = dev_alloc(ctx, f.near32, ne * sizeof(float2))))
      return rc;
    const int64_t tot = static_cast<int64_t>(K) * n;
    hipLaunchKernelGGL(k_near_tables, dim3(cdiv(tot, 256)), dim3(256), 0, ctx->stream,
                       static_cast<const double2 *>(ctx->gt.xy.p), static_cast<const int *>(f.perm.p),
                       static_cast<const int *>(f.near_src.p), static_cast<const int *>(f.near_cnt.p),
                       static_cast<int>(n), K, k, static_cast<double2 *>(f.near64.p),
                       static_cast<float2 *>(f.near32.p));
    MPSL_HIP_TRY(ctx, hipGetLastError());
    f.active = true;
    return MPSL_OK;
  }
  return set_err(ctx, MPSL_EUNSUPPORTED, "no FMM tree shape fits the problem: " + why);
}

// ---------------------------------------------------------------------------
// Host: apply.

namespace {

template <typename T>
int launch_stage(mpsl_ctx *ctx, int pi, const FmmStage &st) {
  if (st.tasks == 0) return MPSL_OK;
  FmmPlan &f = ctx->fmm;
  const size_t lds = fmm_mfma_lds(st.tj, sizeof(T));
  if (st.G != kFmmGroup || st.tj < 16 || st.tj % 16 || st.tj > kFmmTileMax || lds > kFmmLds)
    return set_err(ctx, MPSL_EUNSUPPORTED, "FMM translation shape outside the kernel's limits");
  hipLaunchKernelGGL((k_fmm_group_mfma<T, kFmmGroup / 16>), dim3(st.tasks, st.tiles), dim3(64 * kFmmMfmaWaves), lds,
                     ctx->stream, static_cast<const FmmGroup *>(f.groups[pi].p) + st.task_off,
                     static_cast<const FmmGTerm *>(f.terms[pi].p), static_cast<const int64_t *>(f.ins[pi].p),
                     static_cast<const int64_t *>(f.outs[pi].p), static_cast<const cv_t<T> *>(f.xb.p),
                     static_cast<const cv_t<T> *>(f.tab[pi].p), static_cast<cv_t<T> *>(f.xb.p), st.pout, st.tj);
  MPSL_HIP_TRY(ctx, hipGetLastError());
  if (st.nchunk > 1) {
    hipLaunchKernelGGL(k_fmm_chunk_sum<T>, dim3(cdiv(st.sum_len, 256)), dim3(256), 0, ctx->stream,
                       static_cast<cv_t<T> *>(f.xb.p) + st.sum_off, st.sum_len, st.nchunk);
    MPSL_HIP_TRY(ctx, hipGetLastError());
  }
  return MPSL_OK;
}

template <typename T>
int fmm_apply_t(mpsl_ctx *ctx, int pi, const void *beta, void *part) {
  FmmPlan &f = ctx->fmm;
  const int P = 2 * ctx->p + 1;
  const int P0 = 2 * f.lv[0].p[pi] + 1;
  const int nb0 = f.lv[0].nx * f.lv[0].ny;
  const cv_t<T> *b = static_cast<const cv_t<T> *>(beta);
  cv_t<T> *xb = static_cast<cv_t<T> *>(f.xb.p);
  const cv_t<T> *tab = static_cast<const cv_t<T> *>(f.tab[pi].p);
  const int bs = std::min(256, cdiv(P0, 64) * 64);
  hipLaunchKernelGGL(k_fmm_p2m<T>, dim3(nb0), dim3(bs), 0, ctx->stream, b, static_cast<const int *>(f.perm.p),
                     static_cast<const int *>(f.start.p), tab + f.p2m_off[pi], P, P0, xb + f.lv[0].moff[pi]);
  MPSL_HIP_TRY(ctx, hipGetLastError());
  int rc;
  for (const auto &st : f.up[pi])
    if ((rc = launch_stage<T>(ctx, pi, st))) return rc;
  for (const auto &st : f.down[pi])
    if ((rc = launch_stage<T>(ctx, pi, st))) return rc;
  const int64_t len = ctx->n * static_cast<int64_t>(P);
  cv_t<T> *far = static_cast<cv_t<T> *>(part) + f.near_chunks * len;
  hipLaunchKernelGGL(k_fmm_l2p<T>, dim3(nb0), dim3(256), P0 * sizeof(cx<T>), ctx->stream,
                     static_cast<const cv_t<T> *>(xb + f.lv[0].loff[pi]), static_cast<const int *>(f.perm.p),
                     static_cast<const int *>(f.start.p), tab + f.l2p_off[pi], P, P0, far);
  MPSL_HIP_TRY(ctx, hipGetLastError());
  return launch_fmm_near(ctx, pi == 0 ? MPSL_FP64 : MPSL_FP32, beta, part);
}

}  // namespace

int fmm_apply(mpsl_ctx *ctx, int prec, const void *beta, void *part) {
  if (!ctx->fmm.active) return set_err(ctx, MPSL_ESTATE, "FMM not built");
  return prec == MPSL_FP64 ? fmm_apply_t<double>(ctx, 0, beta, part) : fmm_apply_t<float>(ctx, 1, beta, part);
}

}  // namespace mpsl

// ===========================================================================
extern "C" {

int mpsl_set_far_field(mpsl_ctx *ctx, int method, double tol) {
  if (!ctx) return MPSL_EINVAL;
  if (const int pe = mpsl::check_unpinned(ctx)) return pe;
  if (method != MPSL_FAR_AUTO && method != MPSL_FAR_DIRECT && method != MPSL_FAR_FMM)
    return mpsl::set_err(ctx, MPSL_EINVAL, "unknown far-field method");
  if (tol != 0.0 && !(tol >= 1e-13 && tol <= 1e-3))
    return mpsl::set_err(ctx, MPSL_EINVAL, "FMM tolerance must lie in [1e-13, 1e-3]");
  ctx->far_method = method;
  if (tol != 0.0) ctx->far_tol = tol;
  ctx->tables_ok = false;
  return MPSL_OK;
}

int mpsl_get_fmm_info(const mpsl_ctx *ctx, int prec, int *active, int *levels, double *leaf_side, int *p_leaf,
                      int *p_top, int64_t *near_pairs, double *tree_cmac) {
  if (!ctx || (prec != MPSL_FP64 && prec != MPSL_FP32)) return MPSL_EINVAL;
  if (!ctx->tables_ok) return MPSL_ESTATE;
  const mpsl::FmmPlan &f = ctx->fmm;
  const int pi = prec == MPSL_FP64 ? 0 : 1;
  if (active) *active = f.active ? 1 : 0;
  if (levels) *levels = f.active ? f.top + 1 : 0;
  if (leaf_side) *leaf_side = f.active ? f.lv[0].s : 0.0;
  if (p_leaf) *p_leaf = f.active ? f.lv[0].p[pi] : 0;
  if (p_top) *p_top = f.active ? f.lv[f.top].p[pi] : 0;
  if (near_pairs) *near_pairs = f.active ? f.near_pairs : 0;
  if (tree_cmac) *tree_cmac = f.active ? f.tree_cmac[pi] : 0.0;
  return MPSL_OK;
}

}  // extern "C"
