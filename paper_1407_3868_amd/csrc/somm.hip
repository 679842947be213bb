// M2S and S2L by tile-local interpolation in lambda (Sections 5.2.1, 5.3).
//
// The direct transforms couple every particle m with every contour node q
// through e^{-i lam_q x_m +- g2_q y_m} (M2S) and e^{i lam_q x_l +- g2_q y_l}
// (S2L).  With the particles grouped in tiles of centre (x_T, y_T) the factor
// splits into a tile part e^{-+i lam x_T +- g2 y_T} and a local part whose
// phase is at most |lam| times the tile size: together with the order weights
// (powers of (lam -+ g2)/k2) the local part is smooth in lambda away from
// lam = +-k2.  Per tile it is evaluated at kSommNc Chebyshev nodes of each
// lambda-interval of length L_I on the contour's lines and interpolated to the
// contour nodes in barycentric form; nodes within d_dir of +-k2 and the nodes
// of the vertical segment are their own coarse nodes (interpolation weight 1).
//
//   M2S: G[T][c]   = sum_{m in T} local_m(c) (beta_m . W(c))
//        spec[q]   = sum_T E_T(q) sum_k L[q][k] G[T][c0(q) + k]
//   S2L: B[T][c]   = sum_{q in run(c)} L[q][k(c)] c_q sigma(q) E'_T(q)
//        alpha_l[n] = sum_c local_l(c) B[T(l)][c] Z_n(c)
//
// Exponentials are evaluated in FP64 (their phases reach |lam| times the strip
// width); sums run in the matvec precision.  The paper's NUFFT forms
// (Sections 5.2.2, 5.3.1) reach the same O(N + N_S) scaling with FFT grids;
// interpolation keeps every step a dense loop.
#include <algorithm>
#include <cmath>
#include <map>

#include "kernels.h"

namespace mpsl {

namespace {

constexpr double kTileW = 8.0, kTileH = 4.0, kIntervalL = 1.0, kDirect = 0.3;

// the expansion orders instantiated (1..20)
#define SOMM_P_CASES(X) \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) X(19) X(20)

// sin and cos of r, |r| <= pi / 4, by their Taylor series (terms up to r^9
// and r^10 in FP32, r^17 and r^18 in FP64: the first term left out is below
// 2e-10 and 1e-19 there).
__device__ inline void sincos_quarter(float r, float &s, float &c) {
  const float r2 = r * r;
  s = r * (1.0f + r2 * (-1.0f / 6 + r2 * (1.0f / 120 + r2 * (-1.0f / 5040 + r2 * (1.0f / 362880)))));
  c = 1.0f + r2 * (-0.5f + r2 * (1.0f / 24 + r2 * (-1.0f / 720 + r2 * (1.0f / 40320 + r2 * (-1.0f / 3628800)))));
}
__device__ inline void sincos_quarter(double r, double &s, double &c) {
  const double r2 = r * r;
  double ps = 1.0 / 355687428096000.0, pc = 1.0 / 6402373705728000.0;  // 1/17!, 1/18!
  ps = 1.0 / 1307674368000.0 - r2 * ps;   // 1/15!
  ps = 1.0 / 6227020800.0 - r2 * ps;      // 1/13!
  ps = 1.0 / 39916800.0 - r2 * ps;        // 1/11!
  ps = 1.0 / 362880.0 - r2 * ps;          // 1/9!
  ps = 1.0 / 5040.0 - r2 * ps;
  ps = 1.0 / 120.0 - r2 * ps;
  ps = 1.0 / 6.0 - r2 * ps;
  s = r * (1.0 - r2 * ps);
  pc = 1.0 / 20922789888000.0 - r2 * pc;  // 1/16!
  pc = 1.0 / 87178291200.0 - r2 * pc;     // 1/14!
  pc = 1.0 / 479001600.0 - r2 * pc;       // 1/12!
  pc = 1.0 / 3628800.0 - r2 * pc;         // 1/10!
  pc = 1.0 / 40320.0 - r2 * pc;
  pc = 1.0 / 720.0 - r2 * pc;
  pc = 1.0 / 24.0 - r2 * pc;
  pc = 0.5 - r2 * pc;
  c = 1.0 - r2 * pc;
}

// e^{a + i b} in the matvec precision.  The phase b (up to |lambda| times the
// strip width) is reduced in FP64 to r = b - k pi/2, |r| <= pi/4, with a
// two-term pi/2 (Cody and Waite); sin and cos of r come from the series
// above in T and are rotated by k quarter turns; exp(a) in T.  In FP32 the
// relative error is ~2e-7 (the result is rounded to FP32 anyway); in FP64 a
// few units in the last place.  No large-argument path: every lane runs the
// same instructions.
template <typename T> __device__ inline cx<T> cexpT(double a, double b) {
  constexpr double kHalfPiHi = 1.5707963267948966, kHalfPiLo = 6.123233995736766e-17;
  const double k = rint(b * 0.6366197723675814);
  const double r = fma(-k, kHalfPiLo, fma(-k, kHalfPiHi, b));
  T sr, cr;
  sincos_quarter(static_cast<T>(r), sr, cr);
  const int qd = static_cast<int>(static_cast<long long>(k) & 3);
  const T sn = qd == 0 ? sr : qd == 1 ? cr : qd == 2 ? -sr : -cr;
  const T cs = qd == 0 ? cr : qd == 1 ? -sr : qd == 2 ? -cr : sr;
  const T e = exp(static_cast<T>(a));
  return {e * cs, e * sn};
}
__device__ inline cx<double> cexp64(double a, double b) { return cexpT<double>(a, b); }
template <typename T> __device__ inline cx<T> cvt(cx<double> v) { return {static_cast<T>(v.re), static_cast<T>(v.im)}; }
template <typename T> __device__ inline cx<double> up(cx<T> v) { return {static_cast<double>(v.re), static_cast<double>(v.im)}; }



// M2S, step 1 (FP32): one lane per (tile, coarse node), blockIdx.z = 2 rhs + side.
// (The matrix-core form below is slower in FP32 at ~10 particles per tile.)
template <typename T, int p>
__global__ __launch_bounds__(256) void k_si_tileG(const cv_t<T> *__restrict__ beta, const double2 *__restrict__ xy,
                                                  const int *__restrict__ perm, const int *__restrict__ tstart,
                                                  const double2 *__restrict__ txy, const double2 *__restrict__ lamc,
                                                  const double2 *__restrict__ gc, const cv_t<T> *__restrict__ Wc,
                                                  int n, int nT, int nc, cv_t<T> *__restrict__ G) {
  constexpr int P = 2 * p + 1;
  const int c = blockIdx.x * 256 + threadIdx.x;
  const int t = blockIdx.y;
  const int s = blockIdx.z & 1, r = blockIdx.z >> 1;
  if (c >= nc) return;
  beta += static_cast<int64_t>(r) * n * P;
  const double lr = lamc[c].x, li = lamc[c].y, gr = gc[c].x, gi = gc[c].y;
  const cv_t<T> *W = Wc + (static_cast<int64_t>(s) * nc + c) * P;
  cx<T> w[P];
#pragma unroll
  for (int j = 0; j < P; ++j) w[j] = ld<T>(W[j]);
  const double sg = s == 0 ? 1.0 : -1.0;
  const double xT = txy[t].x, yT = txy[t].y;
  cx<T> acc = mk<T>(0, 0);
  for (int k = tstart[t]; k < tstart[t + 1]; ++k) {
    const int m = perm[k];
    const double dx = xy[m].x - xT, dy = xy[m].y - yT;
    // e^{-i lam dx + sg g2 dy}
    const cx<T> e = cexpT<T>(li * dx + sg * gr * dy, -lr * dx + sg * gi * dy);
    const cv_t<T> *b = beta + static_cast<int64_t>(m) * P;
    cx<T> bw = mk<T>(0, 0);
#pragma unroll
    for (int j = 0; j < P; ++j) cmac(bw, ld<T>(b[j]), w[j]);
    cmac(acc, e, bw);
  }
  G[((static_cast<int64_t>(r) * 2 + s) * nT + t) * nc + c] = st(acc);
}

// M2S, step 2, interval nodes, on the matrix cores: per interval
//   H[T][q] = sum_k G[T][c0 + k] L[q][k]      (M = tile, N = node, K = 24)
//   spec[q] = sum_T e^{-i lam_q x_T + g2_q yy_T} H[T][q]
// One wave per 16 nodes of a block's run of kSiFineNodes (from fblk), all
// tiles in steps of 16: lane i supplies A[i % 16][i / 16] = G of tile
// tb + i % 16 (complex, two real MFMAs) and B[i / 16][i % 16] = L of node
// i % 16 (loaded once).  The result rows a lane holds are four tiles of its
// node column; along a column their factors change by e^{-g2 h} per tile
// height in the direction in which they shrink (down on side 0, up on side
// 1; no FP32 overflow), and the four tiles are walked in that order with an
// exponential where a column starts.  Each lane sums per step in the matvec
// precision and across steps in FP64; the four row groups are added at the end.
constexpr int kSiFineSplit = 4;   // waves per block
constexpr int kSiFineNodes = 64;  // nodes per block (16 per wave)
template <typename T>
__global__ __launch_bounds__(64 * kSiFineSplit) void k_si_fine(
    const cv_t<T> *__restrict__ G, const double2 *__restrict__ lam, const double2 *__restrict__ g2,
    const double2 *__restrict__ txy, const int *__restrict__ ivl, const int *__restrict__ fperm,
    const int *__restrict__ fblk, const double *__restrict__ Lw, int ns, int nT, int nc, double d,
    double tile_h, double2 *__restrict__ spec) {
  static_assert(kSiFineNodes == 16 * kSiFineSplit, "16 nodes per wave");
  typedef typename mfma4<T>::v4 v4;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  // XCD-aware order: blocks are dealt to the 8 XCDs round-robin, so block b
  // takes run x q + min(x, rem) + b / 8 (x = b % 8) and each XCD works
  // through consecutive runs of the same intervals
  const int nb = gridDim.x, xq = nb / 8, xr = nb % 8, x = blockIdx.x % 8;
  const int fb = x * xq + min(x, xr) + blockIdx.x / 8;
  const int iv = fblk[2 * fb], off = fblk[2 * fb + 1] + 16 * w;
  const int f0 = ivl[4 * iv], nf = ivl[4 * iv + 1], c0 = ivl[4 * iv + 2];
  if (off >= nf) return;  // the whole wave lies past the interval's nodes (no barriers below)
  const int s = blockIdx.y & 1, rr = blockIdx.y >> 1;
  const bool qv = off + r < nf;
  const int q = fperm[f0 + (qv ? off + r : off)];
  T bl[6];  // B operand of the six K steps: L[q][4 ks + g]
#pragma unroll
  for (int ks = 0; ks < 6; ++ks) bl[ks] = qv ? static_cast<T>(Lw[static_cast<int64_t>(q) * kSommNc + 4 * ks + g]) : T(0);
  const double lr = lam[q].x, li = lam[q].y, gr = g2[q].x, gi = g2[q].y;
  const cx<T> Fd = cexpT<T>(-gr * tile_h, -gi * tile_h);
  const double ih = 1.0 / tile_h;
  const int jbeg = s == 0 ? 3 : 0, jstep = s == 0 ? -1 : 1;
  const cv_t<T> *Gs = G + ((static_cast<int64_t>(rr) * 2 + s) * nT) * nc + c0;
  cx<double> acc = mk(0.0, 0.0);
  for (int tb = 0; tb < nT; tb += 16) {
    const int ta = tb + r;
    const bool av = ta < nT;
    const cv_t<T> *Ga = Gs + static_cast<int64_t>(av ? ta : 0) * nc + g;
    v4 hr = v4{0, 0, 0, 0}, hi = v4{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < 6; ++ks) {
      const cx<T> a = av ? ld<T>(Ga[4 * ks]) : mk<T>(0, 0);
      hr = mfma4<T>::mac(a.re, bl[ks], hr);
      hi = mfma4<T>::mac(a.im, bl[ks], hi);
    }
    cx<T> E = mk<T>(0, 0), blk = mk<T>(0, 0);
    double xp = 0.0, yp = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = jbeg + jstep * u;
      const int t = tb + mfma4<T>::row(lane, j);
      if (t < nT) {
        const double xT = txy[t].x, yT = txy[t].y;
        const int k = u > 0 && xT == xp ? static_cast<int>(lrint(fabs(yT - yp) * ih)) : 0;
        if (k >= 1 && k <= 4) {
          for (int v = 0; v < k; ++v) E = E * Fd;
        } else {
          const double yy = s == 0 ? yT : -(d + yT);
          E = cexpT<T>(li * xT + gr * yy, -lr * xT + gi * yy);
        }
        xp = xT;
        yp = yT;
        cmac(blk, E, mk<T>(hr[j], hi[j]));
      }
    }
    acc = acc + up<T>(blk);
  }
  acc.re += __shfl_xor(acc.re, 16);
  acc.im += __shfl_xor(acc.im, 16);
  acc.re += __shfl_xor(acc.re, 32);
  acc.im += __shfl_xor(acc.im, 32);
  if (g == 0 && qv) spec[(static_cast<int64_t>(rr) * 2 + s) * ns + q] = st(acc);
}

// M2S, step 2, direct nodes (their own coarse node, weight 1): one lane per
// node and tile share as above.
template <typename T>
__global__ __launch_bounds__(kSiFineNodes *kSiFineSplit) void k_si_fine_dir(
    const cv_t<T> *__restrict__ G, const double2 *__restrict__ lam, const double2 *__restrict__ g2,
    const double2 *__restrict__ txy, const int *__restrict__ dir, int ndir, int ns, int nT, int nc, double d,
    double2 *__restrict__ spec) {
  __shared__ double2 red[kSiFineSplit][kSiFineNodes];
  const int j = threadIdx.x / kSiFineNodes, ql = threadIdx.x - j * kSiFineNodes;
  const int i = blockIdx.x * kSiFineNodes + ql;
  const bool act = i < ndir;
  const int q = act ? dir[2 * i] : 0, c = act ? dir[2 * i + 1] : 0;
  const int s = blockIdx.y & 1, r = blockIdx.y >> 1;
  const double lr = lam[q].x, li = lam[q].y, gr = g2[q].x, gi = g2[q].y;
  const cv_t<T> *Gs = G + ((static_cast<int64_t>(r) * 2 + s) * nT) * nc + c;
  cx<double> acc = mk(0.0, 0.0);
  if (act) {
    for (int t = j; t < nT; t += kSiFineSplit) {
      const double xT = txy[t].x, yT = txy[t].y;
      const double yy = s == 0 ? yT : -(d + yT);
      acc = acc + up<T>(cexpT<T>(li * xT + gr * yy, -lr * xT + gi * yy)) * up<T>(ld<T>(Gs[static_cast<int64_t>(t) * nc]));
    }
  }
  red[j][ql] = st(acc);
  __syncthreads();
  if (j == 0 && act) {
    cx<double> sum = ld<double>(red[0][ql]);
#pragma unroll
    for (int u = 1; u < kSiFineSplit; ++u) sum = sum + ld<double>(red[u][ql]);
    spec[(static_cast<int64_t>(r) * 2 + s) * ns + q] = st(sum);
  }
}


// Sum of the node-chunk partials of k_si_coarseB into B[rhs, side][t][c],
// c < nci, in chunk order.
template <typename T>
__global__ void k_si_coarseB_sum(const cv_t<T> *__restrict__ Bp, int nchunk, int64_t rows, int nT, int nc, int nci,
                                 cv_t<T> *__restrict__ B) {
  const int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (e >= rows * nci) return;
  const int64_t row = e / nci;  // (rhs, side, tile)
  const int c = static_cast<int>(e - row * nci);
  const int64_t plane = rows * nci;
  cx<T> a = ld<T>(Bp[e]);
  for (int cz = 1; cz < nchunk; ++cz) a = a + ld<T>(Bp[cz * plane + e]);
  B[row * nc + c] = st(a);
}

// S2L, step 1 for the direct nodes: one lane per (direct node, tile).
template <typename T>
__global__ __launch_bounds__(256) void k_si_coarseB_dir(const double2 *__restrict__ sigma,
                                                        const double2 *__restrict__ cq,
                                                        const double2 *__restrict__ lam,
                                                        const double2 *__restrict__ g2,
                                                        const double2 *__restrict__ txy, const int *__restrict__ dir,
                                                        int ndir, int ns, int nT, int nc, double d,
                                                        cv_t<T> *__restrict__ B) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int t = blockIdx.y, s = blockIdx.z & 1, r = blockIdx.z >> 1;
  if (i >= ndir) return;
  sigma += static_cast<int64_t>(r) * 2 * ns;
  const int q = dir[2 * i], c = dir[2 * i + 1];
  const double xT = txy[t].x, yT = txy[t].y;
  const double yy = s == 0 ? yT : -(yT + d);
  const double lr = lam[q].x, li = lam[q].y, gr = g2[q].x, gi = g2[q].y;
  const cx<T> v = cvt<T>(ld<double>(cq[q]) * ld<double>(sigma[s * ns + q])) *
                  cexpT<T>(-li * xT + gr * yy, lr * xT + gi * yy);
  B[((static_cast<int64_t>(r) * 2 + s) * nT + t) * nc + c] = st(v);
}


inline int cdv(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }

// S2L, step 2 on the matrix cores: alpha_l[n] = sum_c e_l(c) Z_n(c) with
// e_l(c) = e^{i lam_c dx_l + sg g2_c dy_l} B[T(l)][c] is a GEMM with M =
// particle, N = order, K = (side, coarse node).  Each 16x16x4 MFMA takes 16
// particles and four coarse nodes: lane i forms e for (particle i % 16, node
// i / 16) — one FP64 exponential per (particle, node), as before — and loads
// Z_n(c) for (node i / 16, order i % 16) as the B operand.  Complex products in
// three real MFMAs (Gauss).  One wave per 16 particles, kSiAlphaWaves waves per
// block; blockIdx.y takes a chunk of the (side, coarse node) pairs and writes
// its own partial slot.
constexpr int kSiAlphaWaves = 4;

template <typename T, int p>
__global__ __launch_bounds__(64 * kSiAlphaWaves) void k_si_alpha_mfma(
    const cv_t<T> *__restrict__ B, const double2 *__restrict__ xy, const int *__restrict__ ptile,
    const double2 *__restrict__ txy, const double2 *__restrict__ lamc, const double2 *__restrict__ gc,
    const cv_t<T> *__restrict__ Zc, int n, int nT, int nc, int chunk_len, cv_t<T> *__restrict__ part,
    int64_t pstride) {
  constexpr int P = 2 * p + 1;
  constexpr int NTN = (P + 15) / 16;
  typedef typename mfma4<T>::v4 v4;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  const int ch = blockIdx.y, rr = blockIdx.z;
  const int k0 = ch * chunk_len, k1 = min(2 * nc, k0 + chunk_len);
  const int lw = (blockIdx.x * kSiAlphaWaves + w) * 16;  // first particle of this wave
  const int l = lw + r;                                   // this lane's particle (A row)
  const bool valid = l < n;
  const int lc = valid ? l : 0;
  const int t = ptile[lc];
  const double dx = xy[lc].x - txy[t].x, dy = xy[lc].y - txy[t].y;
  v4 acc[NTN][3];
#pragma unroll
  for (int nt = 0; nt < NTN; ++nt)
#pragma unroll
    for (int k = 0; k < 3; ++k) acc[nt][k] = v4{0, 0, 0, 0};
  for (int kk = k0; kk < k1; kk += 4) {
    const int k = kk + g;  // this lane's coarse node (K index)
    const bool kv = k < k1;
    const int s = kv && k >= nc ? 1 : 0, c = kv ? k - s * nc : 0;
    cx<T> a = mk<T>(0, 0);
    if (kv && valid) {
      // e^{i lam_c dx + sg g2_c dy} B[T][c]
      const double sg = s == 0 ? 1.0 : -1.0;
      const double lr = lamc[c].x, li = lamc[c].y, gr = gc[c].x, gi = gc[c].y;
      a = cexpT<T>(-li * dx + sg * gr * dy, lr * dx + sg * gi * dy) *
          ld<T>(B[((static_cast<int64_t>(rr) * 2 + s) * nT + t) * nc + c]);
    }
    const T as = a.re + a.im;
    const cv_t<T> *z = Zc + (static_cast<int64_t>(s) * nc + c) * P;
#pragma unroll
    for (int nt = 0; nt < NTN; ++nt) {
      const int o = nt * 16 + r;  // this lane's order (B column)
      const cx<T> zz = (kv && o < P) ? ld<T>(z[o]) : mk<T>(0, 0);
      acc[nt][0] = mfma4<T>::mac(a.re, zz.re, acc[nt][0]);
      acc[nt][1] = mfma4<T>::mac(a.im, zz.im, acc[nt][1]);
      acc[nt][2] = mfma4<T>::mac(as, zz.re + zz.im, acc[nt][2]);
    }
  }
  // result register j of lane i: particle lw + row(i, j), order nt * 16 + i % 16
  cv_t<T> *out = part + rr * pstride + static_cast<int64_t>(ch) * n * P;
#pragma unroll
  for (int nt = 0; nt < NTN; ++nt) {
    const int o = nt * 16 + r;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int pl = lw + mfma4<T>::row(lane, j);
      if (pl < n && o < P) {
        const T p1 = acc[nt][0][j], p2 = acc[nt][1][j], p3 = acc[nt][2][j];
        out[static_cast<int64_t>(pl) * P + o] = st(mk<T>(p1 - p2, p3 - p1 - p2));
      }
    }
  }
}

// M2S, step 1 on the matrix cores (FP64): per tile, D[m][c] = sum_n beta_m[n] W_n(c)
// is a GEMM with M = the tile's particles (16 at a time), N = coarse nodes, K =
// orders; then G[T][c] = sum_m e_m(c) D[m][c] with the local factor
// e_m(c) = e^{-i lam_c dx_m + sg g2_c dy_m}, one FP64 exponential per
// (particle, node) as before, summed over the lane's rows and across the four
// row groups.  One wave per 16 coarse nodes, kSiAlphaWaves waves per block;
// grid: (node blocks, tile, 2 rhs + side).
template <typename T, int p>
__global__ __launch_bounds__(64 * kSiAlphaWaves) void k_si_tileG_mfma(
    const cv_t<T> *__restrict__ beta, const double2 *__restrict__ xy, const int *__restrict__ perm,
    const int *__restrict__ tstart, const double2 *__restrict__ txy, const double2 *__restrict__ lamc,
    const double2 *__restrict__ gc, const cv_t<T> *__restrict__ Wc, int n, int nT, int nc,
    cv_t<T> *__restrict__ G) {
  constexpr int P = 2 * p + 1;
  constexpr int KP = (P + 3) / 4 * 4;
  typedef typename mfma4<T>::v4 v4;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  const int t = blockIdx.y;
  const int s = blockIdx.z & 1, rr = blockIdx.z >> 1;
  const int c0 = (blockIdx.x * kSiAlphaWaves + w) * 16;
  const int c = c0 + r;  // this lane's coarse node (B column, output)
  const bool cv = c < nc;
  beta += static_cast<int64_t>(rr) * n * P;
  const cv_t<T> *W = Wc + (static_cast<int64_t>(s) * nc + (cv ? c : 0)) * P;
  const double sg = s == 0 ? 1.0 : -1.0;
  const double xT = txy[t].x, yT = txy[t].y;
  const int m0 = tstart[t], m1 = tstart[t + 1];
  cx<double> acc = mk(0.0, 0.0);
  for (int mb = m0; mb < m1; mb += 16) {
    // A row of this lane: particle mb + r
    const int ma = mb + r < m1 ? perm[mb + r] : -1;
    const cv_t<T> *b = beta + static_cast<int64_t>(ma < 0 ? 0 : ma) * P;
    v4 d0 = v4{0, 0, 0, 0}, d1 = v4{0, 0, 0, 0}, d2 = v4{0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < KP; kk += 4) {
      const int j = kk + g;  // order (K index) of this lane
      const cx<T> a = (ma >= 0 && j < P) ? ld<T>(b[j]) : mk<T>(0, 0);
      const cx<T> z = (cv && j < P) ? ld<T>(W[j]) : mk<T>(0, 0);
      d0 = mfma4<T>::mac(a.re, z.re, d0);
      d1 = mfma4<T>::mac(a.im, z.im, d1);
      d2 = mfma4<T>::mac(a.re + a.im, z.re + z.im, d2);
    }
    if (cv) {
      const double lr = lamc[c].x, li = lamc[c].y, gr = gc[c].x, gi = gc[c].y;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = mb + mfma4<T>::row(lane, q);  // particle of result register q
        if (k < m1) {
          const int m = perm[k];
          const double dx = xy[m].x - xT, dy = xy[m].y - yT;
          const cx<double> e = cexp64(li * dx + sg * gr * dy, -lr * dx + sg * gi * dy);
          const double p1 = d0[q], p2 = d1[q], p3 = d2[q];
          acc = acc + e * mk(p1 - p2, p3 - p1 - p2);
        }
      }
    }
  }
  acc.re += __shfl_xor(acc.re, 16);
  acc.im += __shfl_xor(acc.im, 16);
  acc.re += __shfl_xor(acc.re, 32);
  acc.im += __shfl_xor(acc.im, 32);
  if (g == 0 && cv) G[((static_cast<int64_t>(rr) * 2 + s) * nT + t) * nc + c] = st(cvt<T>(acc));
}

// S2L, step 1 for the Chebyshev intervals on the matrix cores:
// B[T][k] = sum_q V_T(q) L[q][k] with V_T(q) = c_q sigma(q) e^{i lam_q x_T + sg g2_q y_T}
// is a GEMM with M = tile, N = interpolation column k (24, two 16-column
// tiles), K = the interval's fine nodes.  A wave takes 16 RB tiles in
// row-major order (trow) as RB row blocks: lane i owns tiles
// trow[tw + RB (i % 16) + b], b < RB, consecutive in that order and usually
// horizontal neighbours, and forms their V for node i / 16 of the step as the
// A operand of row block b: one exponential for the first, then one complex
// multiply by e^{i lam w} (modulus ~1, table Fx) per tile (an exponential
// again where a row of tiles ends).  L[q][k] for (node i / 16, column i % 16)
// is the B operand, shared by the row blocks; complex A times real B in two
// real MFMAs.  grid: (interval, blocks of 16 RB * kSiAlphaWaves tiles, chunk
// of the interval's nodes + nchunk * (2 rhs + side)); chunk cz writes its own
// partial slot Bp[cz][rhs, side][t][k], k over the intervals' coarse nodes
// (which come first in the coarse-node order), summed in order by
// k_si_coarseB_sum.
template <typename T> constexpr int coarse_rb() { return sizeof(T) == 4 ? 4 : 2; }
template <typename T>
__global__ __launch_bounds__(64 * kSiAlphaWaves) void k_si_coarseB_mfma(
    const double2 *__restrict__ sigma, const double2 *__restrict__ cq, const double2 *__restrict__ lam,
    const double2 *__restrict__ g2, const double2 *__restrict__ Fx, const double2 *__restrict__ txy,
    const int *__restrict__ trow, const int *__restrict__ ivl, const int *__restrict__ fperm,
    const double *__restrict__ Lw, int ns, int nT, int nci, int nchunk, double d, double tile_w,
    cv_t<T> *__restrict__ Bp) {
  constexpr int RB = coarse_rb<T>();
  typedef typename mfma4<T>::v4 v4;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  const int iv = blockIdx.x;
  const int tw = (blockIdx.y * kSiAlphaWaves + w) * 16 * RB;  // first row-major slot of this wave
  const int cz = blockIdx.z % nchunk, rs = blockIdx.z / nchunk;
  const int s = rs & 1, rr = rs >> 1;
  const int f0 = ivl[4 * iv], nf = ivl[4 * iv + 1], c0 = ivl[4 * iv + 2];
  const int i0 = static_cast<int>((static_cast<int64_t>(nf) * cz) / nchunk);
  const int i1 = static_cast<int>((static_cast<int64_t>(nf) * (cz + 1)) / nchunk);
  sigma += static_cast<int64_t>(rr) * 2 * ns;
  // this lane's tiles, their centres, and the steps between them (0: new exponential)
  int tb[RB], kst[RB];
  double xb[RB], yb[RB];
  const double iw = 1.0 / tile_w;
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    const int o = tw + RB * r + b;
    tb[b] = o < nT ? trow[o] : -1;
    const double2 tc = txy[tb[b] >= 0 ? tb[b] : 0];
    xb[b] = tc.x;
    yb[b] = s == 0 ? tc.y : -(tc.y + d);
    const int k = b > 0 && yb[b] == yb[b - 1] ? static_cast<int>(lrint((xb[b] - xb[b - 1]) * iw)) : 0;
    kst[b] = k >= 1 && k <= 4 ? k : 0;
  }
  v4 acc[RB][2][2];
#pragma unroll
  for (int b = 0; b < RB; ++b)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) acc[b][nt][0] = acc[b][nt][1] = v4{0, 0, 0, 0};
  for (int i = i0; i < i1; i += 4) {
    const int ii = i + g;  // this lane's node (K index)
    const bool kv = ii < i1;
    const int q = fperm[f0 + (kv ? ii : i0)];
    const double lr = lam[q].x, li = lam[q].y, gr = g2[q].x, gi = g2[q].y;
    const cx<T> u = kv ? cvt<T>(ld<double>(cq[q]) * ld<double>(sigma[s * ns + q])) : mk<T>(0, 0);
    const cx<T> fx = cvt<T>(ld<double>(Fx[q]));
    const double *L = Lw + static_cast<int64_t>(q) * kSommNc;
    T lq[2];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      const int k = nt * 16 + r;
      lq[nt] = (kv && k < kSommNc) ? static_cast<T>(L[k]) : T(0);
    }
    cx<T> E = mk<T>(0, 0);
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      if (kst[b] > 0) {
        for (int v = 0; v < kst[b]; ++v) E = E * fx;
      } else {
        E = cexpT<T>(-li * xb[b] + gr * yb[b], lr * xb[b] + gi * yb[b]);
      }
      const cx<T> v = tb[b] >= 0 ? u * E : mk<T>(0, 0);
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        acc[b][nt][0] = mfma4<T>::mac(v.re, lq[nt], acc[b][nt][0]);
        acc[b][nt][1] = mfma4<T>::mac(v.im, lq[nt], acc[b][nt][1]);
      }
    }
  }
  // result register j of lane i in row block b: tile trow[tw + RB row(i, j) + b], column nt * 16 + i % 16
  cv_t<T> *o = Bp + (static_cast<int64_t>(cz) * (gridDim.z / nchunk) + rs) * nT * static_cast<int64_t>(nci) + c0;
#pragma unroll
  for (int b = 0; b < RB; ++b)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      const int k = nt * 16 + r;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int os = tw + RB * mfma4<T>::row(lane, j) + b;
        if (os < nT && k < kSommNc)
          o[static_cast<int64_t>(trow[os]) * nci + k] = st(mk<T>(acc[b][nt][0][j], acc[b][nt][1][j]));
      }
    }
}

template <typename T>
int ensure_G(mpsl_ctx *ctx, int nrhs) {
  const SommPlan &pl = ctx->somm;
  return dev_alloc(ctx, ctx->somm.G, 2ull * nrhs * pl.nT * pl.nc * sizeof(cv_t<T>));
}

template <typename T>
int m2s_interp_t(mpsl_ctx *ctx, const void *beta, void *spec, int nrhs) {
  SommPlan &pl = ctx->somm;
  int rc = ensure_G<T>(ctx, nrhs);
  if (rc) return rc;
  const bool f64 = std::is_same<T, double>::value;
  const auto *Wc = static_cast<const cv_t<T> *>(f64 ? pl.Wc64.p : pl.Wc32.p);
  auto *G = static_cast<cv_t<T> *>(pl.G.p);
  const int n = static_cast<int>(ctx->n);
  const bool f64m = std::is_same<T, double>::value;  // matrix-core step 1 in FP64 only
  const dim3 g1(cdv(pl.nc, f64m ? 16 * kSiAlphaWaves : 256), pl.nT, 2 * nrhs);
  switch (ctx->p) {
#define X(PP)                                                                                                      \
  case PP:                                                                                                         \
    if (f64m)                                                                                                      \
      hipLaunchKernelGGL((k_si_tileG_mfma<T, PP>), g1, dim3(64 * kSiAlphaWaves), 0, ctx->stream,                  \
                         static_cast<const cv_t<T> *>(beta), static_cast<const double2 *>(ctx->gt.xy.p),            \
                         static_cast<const int *>(pl.perm.p), static_cast<const int *>(pl.tstart.p),                \
                         static_cast<const double2 *>(pl.txy.p), static_cast<const double2 *>(pl.lamc.p),           \
                         static_cast<const double2 *>(pl.gc.p), Wc, n, pl.nT, pl.nc, G);                            \
    else                                                                                                           \
      hipLaunchKernelGGL((k_si_tileG<T, PP>), g1, dim3(256), 0, ctx->stream, static_cast<const cv_t<T> *>(beta),   \
                         static_cast<const double2 *>(ctx->gt.xy.p), static_cast<const int *>(pl.perm.p),           \
                         static_cast<const int *>(pl.tstart.p), static_cast<const double2 *>(pl.txy.p),             \
                         static_cast<const double2 *>(pl.lamc.p), static_cast<const double2 *>(pl.gc.p), Wc, n,    \
                         pl.nT, pl.nc, G);                                                                          \
    break;
    SOMM_P_CASES(X)
#undef X
    default: return set_err(ctx, MPSL_EUNSUPPORTED, "expansion order outside 1..20");
  }
  const auto *lam = static_cast<const double2 *>(ctx->ct.lam.p);
  const auto *g2 = static_cast<const double2 *>(ctx->ct.gw.p) + ctx->ns;  // g2 stored after g1
  const auto *txy = static_cast<const double2 *>(pl.txy.p);
  const dim3 blk(kSiFineNodes * kSiFineSplit);
  if (pl.nfb > 0)
    hipLaunchKernelGGL(k_si_fine<T>, dim3(pl.nfb, 2 * nrhs), blk, 0, ctx->stream, G, lam, g2, txy,
                       static_cast<const int *>(pl.ivl.p), static_cast<const int *>(pl.fperm.p),
                       static_cast<const int *>(pl.fblk.p), static_cast<const double *>(pl.Lw.p), ctx->ns, pl.nT,
                       pl.nc, ctx->d, pl.tile_h, static_cast<double2 *>(spec));
  if (pl.ndir > 0)
    hipLaunchKernelGGL(k_si_fine_dir<T>, dim3(cdv(pl.ndir, kSiFineNodes), 2 * nrhs), blk, 0, ctx->stream, G, lam,
                       g2, txy, static_cast<const int *>(pl.dir.p), pl.ndir, ctx->ns, pl.nT, pl.nc, ctx->d,
                       static_cast<double2 *>(spec));
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_err(ctx, MPSL_EHIP, std::string("interpolated M2S: ") + hipGetErrorString(e));
  return MPSL_OK;
}

template <typename T>
int s2l_interp_t(mpsl_ctx *ctx, void *part, int chunks, int nrhs, int64_t pstride) {
  SommPlan &pl = ctx->somm;
  if (!pl.sigma) return set_err(ctx, MPSL_ESTATE, "interpolated S2L without densities");
  int rc = ensure_G<T>(ctx, nrhs);
  if (rc) return rc;
  const bool f64 = std::is_same<T, double>::value;
  const auto *Zc = static_cast<const cv_t<T> *>(f64 ? pl.Zc64.p : pl.Zc32.p);
  auto *B = static_cast<cv_t<T> *>(pl.G.p);
  const auto *sig = static_cast<const double2 *>(pl.sigma);
  const auto *cq = static_cast<const double2 *>(ctx->ct.cq.p);
  const auto *lam = static_cast<const double2 *>(ctx->ct.lam.p);
  const auto *g2 = static_cast<const double2 *>(ctx->ct.gw.p) + ctx->ns;
  const auto *txy = static_cast<const double2 *>(pl.txy.p);
  if (pl.nint > 0) {
    // node chunks so that the launch has about 2048 blocks
    const int nci = kSommNc * pl.nint, tb = cdv(pl.nT, 16 * coarse_rb<T>() * kSiAlphaWaves);
    const int nchunk = std::max(1, std::min(16, cdv(2048, static_cast<int64_t>(pl.nint) * tb * 2 * nrhs)));
    const int64_t rows = 2ll * nrhs * pl.nT;
    if ((rc = dev_alloc(ctx, pl.Bp, static_cast<size_t>(nchunk) * rows * nci * sizeof(cv_t<T>)))) return rc;
    auto *Bp = static_cast<cv_t<T> *>(pl.Bp.p);
    hipLaunchKernelGGL(k_si_coarseB_mfma<T>, dim3(pl.nint, tb, nchunk * 2 * nrhs), dim3(64 * kSiAlphaWaves), 0,
                       ctx->stream, sig, cq, lam, g2, static_cast<const double2 *>(pl.Fx.p), txy,
                       static_cast<const int *>(pl.trow.p), static_cast<const int *>(pl.ivl.p),
                       static_cast<const int *>(pl.fperm.p), static_cast<const double *>(pl.Lw.p), ctx->ns, pl.nT,
                       nci, nchunk, ctx->d, pl.tile_w, Bp);
    hipLaunchKernelGGL(k_si_coarseB_sum<T>, dim3(cdv(rows * nci, 256)), dim3(256), 0, ctx->stream, Bp, nchunk, rows,
                       pl.nT, pl.nc, nci, B);
  }
  if (pl.ndir > 0)
    hipLaunchKernelGGL(k_si_coarseB_dir<T>, dim3(cdv(pl.ndir, 256), pl.nT, 2 * nrhs), dim3(256), 0, ctx->stream,
                       sig, cq, lam, g2, txy, static_cast<const int *>(pl.dir.p), pl.ndir, ctx->ns, pl.nT, pl.nc,
                       ctx->d, B);
  const int n = static_cast<int>(ctx->n);
  const int chunk_len = cdv(2 * static_cast<int64_t>(pl.nc), chunks);
  const dim3 g2d(cdv(n, 16 * kSiAlphaWaves), chunks, nrhs);
  auto *o = static_cast<cv_t<T> *>(part);
  switch (ctx->p) {
#define X(PP)                                                                                                       \
  case PP:                                                                                                          \
    hipLaunchKernelGGL((k_si_alpha_mfma<T, PP>), g2d, dim3(64 * kSiAlphaWaves), 0, ctx->stream, B,                 \
                       static_cast<const double2 *>(ctx->gt.xy.p), static_cast<const int *>(pl.ptile.p), txy,       \
                       static_cast<const double2 *>(pl.lamc.p), static_cast<const double2 *>(pl.gc.p), Zc, n,       \
                       pl.nT, pl.nc, chunk_len, o, pstride);                                                         \
    break;
    SOMM_P_CASES(X)
#undef X
    default: return set_err(ctx, MPSL_EUNSUPPORTED, "expansion order outside 1..20");
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_err(ctx, MPSL_EHIP, std::string("interpolated S2L: ") + hipGetErrorString(e));
  return MPSL_OK;
}

}  // namespace

int launch_m2s_interp(mpsl_ctx *ctx, int prec, const void *beta, void *spec, int nrhs) {
  return prec == MPSL_FP64 ? m2s_interp_t<double>(ctx, beta, spec, nrhs) : m2s_interp_t<float>(ctx, beta, spec, nrhs);
}

int launch_s2l_interp(mpsl_ctx *ctx, int prec, void *part, int chunks, int nrhs, int64_t pstride) {
  return prec == MPSL_FP64 ? s2l_interp_t<double>(ctx, part, chunks, nrhs, pstride)
                           : s2l_interp_t<float>(ctx, part, chunks, nrhs, pstride);
}

void somm_free(mpsl_ctx *ctx) {
  SommPlan &pl = ctx->somm;
  DBuf *b[] = {&pl.perm, &pl.tstart, &pl.txy, &pl.ptile, &pl.lamc, &pl.gc, &pl.Wc64, &pl.Wc32, &pl.Zc64,
               &pl.Zc32, &pl.Lw, &pl.ivl, &pl.fperm, &pl.dir, &pl.G, &pl.Bp, &pl.fblk,
               &pl.trow, &pl.Fx};
  for (DBuf *x : b) dev_free(*x);
  pl.active = false;
  pl.sigma = nullptr;
}

// Tiles, intervals, coarse nodes and interpolation weights (host, FP64).
int somm_build(mpsl_ctx *ctx) {
  somm_free(ctx);
  SommPlan &pl = ctx->somm;
  if (ctx->somm_method != MPSL_SOMM_INTERP) return MPSL_OK;
  const int64_t n = ctx->n;
  const int ns = ctx->ns, p = ctx->p, P = 2 * p + 1;
  pl.tile_w = kTileW;
  pl.tile_h = kTileH;
  pl.L_I = kIntervalL;
  pl.d_dir = kDirect;
  // tiles of the particle bounding box
  double x0 = 1e300, y0 = 1e300;
  for (int64_t m = 0; m < n; ++m) {
    x0 = std::min(x0, ctx->xy[2 * m]);
    y0 = std::min(y0, ctx->xy[2 * m + 1]);
  }
  std::map<std::pair<int64_t, int64_t>, int> tiles;
  std::vector<std::pair<int64_t, int64_t>> key(n);
  for (int64_t m = 0; m < n; ++m) {
    key[m] = {static_cast<int64_t>(std::floor((ctx->xy[2 * m] - x0) / kTileW)),
              static_cast<int64_t>(std::floor((ctx->xy[2 * m + 1] - y0) / kTileH))};
    tiles.emplace(key[m], 0);
  }
  int id = 0;
  std::vector<double2> txy;
  for (auto &kv : tiles) {
    kv.second = id++;
    txy.push_back(make_double2(x0 + (kv.first.first + 0.5) * kTileW, y0 + (kv.first.second + 0.5) * kTileH));
  }
  pl.nT = id;
  // row-major tile order: along it, neighbours are usually horizontally adjacent
  std::vector<int> trow;
  {
    std::vector<std::pair<std::pair<int64_t, int64_t>, int>> byrow;
    for (const auto &kv : tiles) byrow.push_back({{kv.first.second, kv.first.first}, kv.second});
    std::sort(byrow.begin(), byrow.end());
    for (const auto &e : byrow) trow.push_back(e.second);
  }
  std::vector<int> ptile(n), tstart(pl.nT + 1, 0), perm(n);
  for (int64_t m = 0; m < n; ++m) {
    ptile[m] = tiles[key[m]];
    ++tstart[ptile[m] + 1];
  }
  for (int t = 0; t < pl.nT; ++t) tstart[t + 1] += tstart[t];
  {
    std::vector<int> fill(tstart.begin(), tstart.end() - 1);
    for (int64_t m = 0; m < n; ++m) perm[fill[ptile[m]]++] = static_cast<int>(m);
  }
  // contour nodes: direct near +-k2 and on the vertical segment, intervals elsewhere
  const double k2r = ctx->k2.real();
  std::vector<char> direct(ns, 0);
  for (int q = 0; q < ns; ++q) {
    const double tr = ctx->lam[q].real();
    direct[q] = (std::fabs(tr) < 1e-14) || (std::fabs(std::fabs(tr) - k2r) < kDirect);
  }
  std::vector<std::vector<int>> groups;
  for (int q = 0; q < ns;) {
    if (direct[q]) {
      ++q;
      continue;
    }
    const double a = ctx->lam[q].real(), im = ctx->lam[q].imag();
    std::vector<int> g{q};
    int e = q + 1;
    while (e < ns && !direct[e] && ctx->lam[e].imag() == im && (ctx->lam[e].real() > 0) == (a > 0) &&
           std::fabs(ctx->lam[e].real() - a) <= kIntervalL)
      g.push_back(e++);
    if (static_cast<int>(g.size()) <= kSommNc)
      for (int x : g) direct[x] = 1;
    else
      groups.push_back(g);
    q = e;
  }
  // coarse nodes: kSommNc Chebyshev nodes per interval, then one per direct node
  std::vector<zc> lamc;
  std::vector<int> ivl, fperm, dir;
  std::vector<double> Lw(static_cast<size_t>(ns) * kSommNc, 0.0);
  double xs[kSommNc], bw[kSommNc];
  for (int j = 0; j < kSommNc; ++j) {
    xs[j] = std::cos((2 * j + 1) * M_PI / (2.0 * kSommNc));
    bw[j] = ((j & 1) ? -1.0 : 1.0) * std::sin((2 * j + 1) * M_PI / (2.0 * kSommNc));
  }
  for (const auto &g : groups) {
    double a = 1e300, c = -1e300;
    for (int q : g) {
      a = std::min(a, ctx->lam[q].real());
      c = std::max(c, ctx->lam[q].real());
    }
    const double im = ctx->lam[g[0]].imag();
    const int c0 = static_cast<int>(lamc.size());
    double tc[kSommNc];
    for (int j = 0; j < kSommNc; ++j) {
      tc[j] = 0.5 * (a + c) + 0.5 * (c - a) * xs[j];
      lamc.emplace_back(tc[j], im);
    }
    ivl.push_back(static_cast<int>(fperm.size()));
    ivl.push_back(static_cast<int>(g.size()));
    ivl.push_back(c0);
    ivl.push_back(0);
    for (int q : g) {
      fperm.push_back(q);
      const double t = ctx->lam[q].real();
      double *L = &Lw[static_cast<size_t>(q) * kSommNc];
      int hit = -1;
      double sum = 0.0;
      for (int j = 0; j < kSommNc; ++j) {
        const double dd = t - tc[j];
        if (dd == 0.0) hit = j;
        L[j] = (dd == 0.0) ? 0.0 : bw[j] / dd;
        sum += L[j];
      }
      if (hit >= 0) {
        for (int j = 0; j < kSommNc; ++j) L[j] = (j == hit) ? 1.0 : 0.0;
      } else {
        for (int j = 0; j < kSommNc; ++j) L[j] /= sum;
      }
    }
  }
  pl.nint = static_cast<int>(groups.size());
  // blocks of the interval-node M2S step: (interval, first node) per run of kSiFineNodes
  std::vector<int> fblk;
  for (int iv = 0; iv < pl.nint; ++iv)
    for (int o = 0; o < ivl[4 * iv + 1]; o += kSiFineNodes) {
      fblk.push_back(iv);
      fblk.push_back(o);
    }
  pl.nfb = static_cast<int>(fblk.size() / 2);
  for (int q = 0; q < ns; ++q)
    if (direct[q]) {
      const int c = static_cast<int>(lamc.size());
      lamc.push_back(ctx->lam[q]);
      Lw[static_cast<size_t>(q) * kSommNc] = 1.0;
      dir.push_back(q);
      dir.push_back(c);
    }
  pl.ndir = static_cast<int>(dir.size() / 2);
  pl.nc = static_cast<int>(lamc.size());
  // coarse-node tables
  std::vector<zc> gc(pl.nc), Wc(2ull * pl.nc * P), Zc(2ull * pl.nc * P);
  for (int c = 0; c < pl.nc; ++c) {
    gc[c] = gamma_branch(lamc[c], ctx->k2);
    order_weights(lamc[c], gc[c], ctx->k2, p, &Wc[static_cast<size_t>(c) * P],
                  &Wc[(static_cast<size_t>(pl.nc) + c) * P], &Zc[static_cast<size_t>(c) * P],
                  &Zc[(static_cast<size_t>(pl.nc) + c) * P]);
  }
  auto upload = [&](DBuf &b, const void *src, size_t bytes) -> int {
    int rc = dev_alloc(ctx, b, bytes > 0 ? bytes : 16);  // an empty table keeps a valid, unused allocation
    if (rc) return rc;
    if (bytes > 0) MPSL_HIP_TRY(ctx, hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice));
    return MPSL_OK;
  };
  std::vector<float2> Wc32(Wc.size()), Zc32(Zc.size());
  for (size_t i = 0; i < Wc.size(); ++i) {
    Wc32[i] = make_float2(static_cast<float>(Wc[i].real()), static_cast<float>(Wc[i].imag()));
    Zc32[i] = make_float2(static_cast<float>(Zc[i].real()), static_cast<float>(Zc[i].imag()));
  }
  int rc;
  if ((rc = upload(pl.perm, perm.data(), perm.size() * sizeof(int))) ||
      (rc = upload(pl.tstart, tstart.data(), tstart.size() * sizeof(int))) ||
      (rc = upload(pl.txy, txy.data(), txy.size() * sizeof(double2))) ||
      (rc = upload(pl.ptile, ptile.data(), ptile.size() * sizeof(int))) ||
      (rc = upload(pl.lamc, lamc.data(), lamc.size() * sizeof(double2))) ||
      (rc = upload(pl.gc, gc.data(), gc.size() * sizeof(double2))) ||
      (rc = upload(pl.Wc64, Wc.data(), Wc.size() * sizeof(double2))) ||
      (rc = upload(pl.Wc32, Wc32.data(), Wc32.size() * sizeof(float2))) ||
      (rc = upload(pl.Zc64, Zc.data(), Zc.size() * sizeof(double2))) ||
      (rc = upload(pl.Zc32, Zc32.data(), Zc32.size() * sizeof(float2))) ||
      (rc = upload(pl.Lw, Lw.data(), Lw.size() * sizeof(double))) ||
      (rc = upload(pl.ivl, ivl.data(), ivl.size() * sizeof(int))) ||
      (rc = upload(pl.fperm, fperm.data(), fperm.size() * sizeof(int))) ||
      (rc = upload(pl.dir, dir.data(), dir.size() * sizeof(int))) ||
      (rc = upload(pl.fblk, fblk.data(), fblk.size() * sizeof(int))) ||
      (rc = upload(pl.trow, trow.data(), trow.size() * sizeof(int))))
    return rc;

  {  // e^{i lam_q w} per contour node
    std::vector<double2> fx(ns);
    for (int q = 0; q < ns; ++q) {
      const zc v = std::exp(zc(0.0, 1.0) * ctx->lam[q] * kTileW);
      fx[q] = make_double2(v.real(), v.imag());
    }
    if ((rc = upload(pl.Fx, fx.data(), fx.size() * sizeof(double2)))) return rc;
  }
  pl.active = true;
  return MPSL_OK;
}

}  // namespace mpsl

extern "C" int mpsl_get_somm_info(const mpsl_ctx *ctx, int *active, int *tiles, int *intervals, int *coarse_nodes,
                                  int *direct_nodes) {
  if (!ctx) return MPSL_EINVAL;
  if (!ctx->tables_ok) return MPSL_ESTATE;
  const mpsl::SommPlan &pl = ctx->somm;
  if (active) *active = pl.active ? 1 : 0;
  if (tiles) *tiles = pl.active ? pl.nT : 0;
  if (intervals) *intervals = pl.active ? pl.nint : 0;
  if (coarse_nodes) *coarse_nodes = pl.active ? pl.nc : 0;
  if (direct_nodes) *direct_nodes = pl.active ? pl.ndir : 0;
  return MPSL_OK;
}
