// Cluster-block right preconditioner of the GMRES solve of eq. (49).
//
// Section 3.2 multiplies the system by the block-diagonal scattering
// matrices, which makes the block of one particle the identity.  Dense,
// high-contrast packings (which the Conclusions name as the hard case) couple
// near neighbours strongly; here the same idea is applied to clusters of
// nearby particles.  Particles are split by recursive coordinate bisection
// into clusters of at most `size`; per cluster c the free-space system of its
// particles alone, K_c = I - S_c T_cc (translations of Lemma 3.1 between the
// cluster's particles, their rotated scattering matrices), is assembled and
// inverted on the device, and GMRES runs on K M^{-1} with M = blockdiag K_c,
// returning x = M^{-1} u.  The solution of eq. (49) does not change.
//
// Device layout: cluster c holds cnt_c particles (sorted ascending) in
// members[c][0 .. cnt_c) (int32 [nc][mp], -1 past the end); its unknowns are
// ordered (slot s, order n) -> s P + n, padded with identity rows and columns
// to m = ceil(mp P / 64) 64.  Blocks are row-major complex [nc][m][m], FP64
// (and an FP32 copy for the mixed-precision solve).
//
// Kernels:
//  k_pc_assemble  one block per (cluster, row particle): K_c rows of that
//                 particle, -S_a T_ab per column particle b (Hankel recurrence
//                 of the pair in FP64, the P x P product from LDS);
//  k_gj_*         in-place Gauss-Jordan inversion in 64 x 64 block steps
//                 without pivoting across blocks (pivoting inside the
//                 diagonal block): diagonal block inverted in LDS, row panel
//                 D^{-1} A_kj, rank-64 update of every other tile on the FP64
//                 matrix cores (Gauss three-product complex form), column
//                 panel -A_ik D^{-1};
//  k_pc_apply     y = M^{-1} x: per (cluster, 64-row tile, 1024-column chunk)
//                 the gathered input chunk in LDS, one wave per 16 rows
//                 streaming the block rows (HBM-bound), partials summed in a
//                 fixed order by k_pc_apply_sum.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <limits>
#include <vector>

#include "kernels.h"

namespace mpsl {
namespace {

constexpr int kGj = 64;          // block size of the Gauss-Jordan steps
constexpr int kPcPairs = 8;      // column particles per Hankel stage of the assembly
constexpr int kPcCols = 1024;    // columns per chunk of the apply
constexpr int kMaxPP = 2 * kMaxP + 1;
constexpr int kMaxQ = 4 * kMaxP + 1;

inline int cdivi(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }

#define PC_CHECK(ctx)                                                                                           \
  do {                                                                                                          \
    hipError_t e_ = hipGetLastError();                                                                          \
    if (e_ != hipSuccess) return set_err(ctx, MPSL_EHIP, std::string("kernel launch: ") + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// Host: recursive coordinate bisection.  A range of more than `size`
// particles is ordered by the coordinate of its longer extent (x when the
// extents are equal; equal coordinates by particle index) and cut after
// floor(n/2); leaves are emitted depth first, first half first, sorted.
void bisect(const double *xy, std::vector<int64_t> &idx, size_t lo, size_t hi, int size,
            std::vector<std::pair<size_t, size_t>> &out) {
  const size_t n = hi - lo;
  if (n <= static_cast<size_t>(size)) {
    std::sort(idx.begin() + lo, idx.begin() + hi);
    out.emplace_back(lo, hi);
    return;
  }
  double mn[2] = {std::numeric_limits<double>::infinity(), std::numeric_limits<double>::infinity()};
  double mx[2] = {-std::numeric_limits<double>::infinity(), -std::numeric_limits<double>::infinity()};
  for (size_t i = lo; i < hi; ++i)
    for (int a = 0; a < 2; ++a) {
      const double v = xy[2 * idx[i] + a];
      mn[a] = std::min(mn[a], v);
      mx[a] = std::max(mx[a], v);
    }
  const int axis = (mx[0] - mn[0] >= mx[1] - mn[1]) ? 0 : 1;
  std::sort(idx.begin() + lo, idx.begin() + hi, [&](int64_t a, int64_t b) {
    const double va = xy[2 * a + axis], vb = xy[2 * b + axis];
    return va < vb || (va == vb && a < b);
  });
  const size_t h = n / 2;
  bisect(xy, idx, lo, lo + h, size, out);
  bisect(xy, idx, lo + h, hi, size, out);
}

// Members of every cluster in emission order.
void make_clusters(int64_t n, const double *xy, int size, std::vector<int64_t> &idx,
                   std::vector<std::pair<size_t, size_t>> &ranges) {
  idx.resize(n);
  for (int64_t i = 0; i < n; ++i) idx[i] = i;
  ranges.clear();
  bisect(xy, idx, 0, static_cast<size_t>(n), size, ranges);
}

// ---------------------------------------------------------------------------
// Assembly of K_c = I - S_c T_cc.  Block (a, c): row particle a of cluster c.
// T_ab[n'][nu] = h_{nu - n'} with h_q = H_q(k2 rho) e^{i q phi}, rho, phi the
// polar form of x_a - x_b (Lemma 3.1 with the sign corrected), H_q by the
// upward recurrence H_{q+1} = (2q/z) H_q - H_{q-1} from H_0, H_1 and
// h_{-q} = (-1)^q H_q e^{-i q phi}.
__global__ __launch_bounds__(256) void k_pc_assemble(const int32_t *__restrict__ members,
                                                    const int32_t *__restrict__ counts, int mp, int m,
                                                    const double2 *__restrict__ xy,
                                                    const double2 *__restrict__ rot,
                                                    const double2 *__restrict__ S,
                                                    const int32_t *__restrict__ types, double k2, int p,
                                                    double2 *__restrict__ blk) {
  const int c = blockIdx.y, a = blockIdx.x;
  const int cnt = counts[c];
  if (a >= cnt) return;  // padding rows: k_pc_pad
  const int P = 2 * p + 1, Q = 4 * p + 1;
  __shared__ cx<double> Sa[kMaxPP * kMaxPP];
  __shared__ cx<double> H[kPcPairs][kMaxQ];
  const int tid = threadIdx.x;
  const int la = members[static_cast<int64_t>(c) * mp + a];
  const int t = types ? types[la] : 0;
  const cv_t<double> *St = S + static_cast<int64_t>(t) * P * P;
  for (int i = tid; i < P * P; i += blockDim.x) {
    const int n = i / P, n2 = i % P;
    // S_a[n][n'] = e^{i (n' - n) psi_a} S[n][n']
    Sa[i] = conj(ld<double>(rot[static_cast<int64_t>(la) * P + n])) * ld<double>(St[i]) *
            ld<double>(rot[static_cast<int64_t>(la) * P + n2]);
  }
  double2 *row = blk + (static_cast<int64_t>(c) * m + static_cast<int64_t>(a) * P) * m;
  const double xa = xy[la].x, ya = xy[la].y;
  for (int b0 = 0; b0 < cnt; b0 += kPcPairs) {
    const int nb = min(kPcPairs, cnt - b0);
    __syncthreads();  // Sa written / previous H consumed
    if (tid < nb) {
      cx<double> *h = H[tid];
      const int lb = members[static_cast<int64_t>(c) * mp + b0 + tid];
      if (lb == la) {
        for (int q = 0; q < Q; ++q) h[q] = mk(0.0, 0.0);
      } else {
        const double dx = xa - xy[lb].x, dy = ya - xy[lb].y;
        const double rho = sqrt(dx * dx + dy * dy);
        const double z = k2 * rho;
        const cx<double> e = mk(dx / rho, dy / rho);
        cx<double> hm = mk(j0(z), y0(z)), hq = mk(j1(z), y1(z));  // H_0, H_1
        cx<double> ep = e;                                         // e^{i q phi}
        h[2 * p] = hm;
        for (int q = 1; q <= 2 * p; ++q) {
          const cx<double> v = hq * ep;
          h[2 * p + q] = v;
          const cx<double> vm = hq * conj(ep);
          h[2 * p - q] = (q & 1) ? mk(-vm.re, -vm.im) : vm;
          const cx<double> hn = (2.0 * q / z) * hq - hm;
          hm = hq;
          hq = hn;
          ep = ep * e;
        }
      }
    }
    __syncthreads();
    const int w = nb * P;
    for (int i = tid; i < P * w; i += blockDim.x) {
      const int n = i / w, r = i % w;
      const int bl = r / P, nu = r % P;
      const cx<double> *h = H[bl] + nu + 2 * p;  // h[nu - n' + 2p] = h[-n'] from here
      cx<double> s = mk(0.0, 0.0);
      for (int n2 = 0; n2 < P; ++n2) cmac(s, Sa[n * P + n2], h[-n2]);
      const double one = (b0 + bl == a && n == nu) ? 1.0 : 0.0;
      row[static_cast<int64_t>(n) * m + static_cast<int64_t>(b0) * P + r] = make_double2(one - s.re, -s.im);
    }
  }
  const int pad = m - cnt * P;
  for (int i = tid; i < P * pad; i += blockDim.x) {
    const int n = i / pad, col = cnt * P + i % pad;
    row[static_cast<int64_t>(n) * m + col] = make_double2(0.0, 0.0);
  }
}

// Padding rows r >= cnt P: identity rows.
__global__ void k_pc_pad(const int32_t *__restrict__ counts, int m, int P, double2 *__restrict__ blk) {
  const int c = blockIdx.y, r = blockIdx.x;
  if (r < counts[c] * P) return;
  double2 *row = blk + (static_cast<int64_t>(c) * m + r) * m;
  for (int j = threadIdx.x; j < m; j += blockDim.x) row[j] = make_double2(j == r ? 1.0 : 0.0, 0.0);
}

// ---------------------------------------------------------------------------
// Gauss-Jordan step kb, diagonal block: D <- D^{-1} in LDS, row pivoting
// inside D (rows swapped while eliminating, columns swapped back in reverse
// order at the end).  A zero pivot sets flag[c] (the block is later replaced).
__global__ __launch_bounds__(256) void k_gj_diag(double2 *__restrict__ blk, int m, int kb,
                                                int32_t *__restrict__ flag) {
  __shared__ double Dr[kGj][kGj + 1], Di[kGj][kGj + 1];
  __shared__ double fr[kGj], fi[kGj];
  __shared__ int perm[kGj];
  __shared__ int piv_row;
  __shared__ double inv_r, inv_i;
  const int c = blockIdx.x, tid = threadIdx.x;
  double2 *A = blk + static_cast<int64_t>(c) * m * m + static_cast<int64_t>(kb) * kGj * (m + 1);
  for (int i = tid; i < kGj * kGj; i += blockDim.x) {
    const double2 v = A[static_cast<int64_t>(i / kGj) * m + i % kGj];
    Dr[i / kGj][i % kGj] = v.x;
    Di[i / kGj][i % kGj] = v.y;
  }
  bool singular = false;
  __syncthreads();
  for (int t = 0; t < kGj; ++t) {
    if (tid < 64) {  // wave 0: pivot search over rows t..63
      double v = -1.0;
      int idx = tid;
      if (tid >= t) v = Dr[tid][t] * Dr[tid][t] + Di[tid][t] * Di[tid][t];
      for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(v, o);
        const int oi = __shfl_xor(idx, o);
        if (ov > v || (ov == v && oi < idx)) {
          v = ov;
          idx = oi;
        }
      }
      if (tid == 0) {
        piv_row = idx;
        perm[t] = idx;
      }
    }
    __syncthreads();
    const int r = piv_row;
    if (r != t && tid < kGj) {
      const double ar = Dr[t][tid], ai = Di[t][tid];
      Dr[t][tid] = Dr[r][tid];
      Di[t][tid] = Di[r][tid];
      Dr[r][tid] = ar;
      Di[r][tid] = ai;
    }
    __syncthreads();
    if (tid == 0) {
      const double pr = Dr[t][t], pi = Di[t][t];
      const double den = pr * pr + pi * pi;
      if (!(den > 0.0) || !isfinite(den)) {
        singular = true;
        inv_r = 1.0;
        inv_i = 0.0;
      } else {
        inv_r = pr / den;
        inv_i = -pi / den;
      }
    }
    __syncthreads();
    if (tid < kGj) {  // row t: (D[t][j], with 1 at j = t) / pivot
      const double ar = (tid == t) ? 1.0 : Dr[t][tid], ai = (tid == t) ? 0.0 : Di[t][tid];
      Dr[t][tid] = ar * inv_r - ai * inv_i;
      Di[t][tid] = ar * inv_i + ai * inv_r;
      fr[tid] = Dr[tid][t];
      fi[tid] = Di[tid][t];
    }
    __syncthreads();
    for (int i = tid; i < kGj * kGj; i += blockDim.x) {
      const int rr = i / kGj, cc = i % kGj;
      if (rr == t) continue;
      const double br = (cc == t) ? 0.0 : Dr[rr][cc], bi = (cc == t) ? 0.0 : Di[rr][cc];
      const double f_r = (rr == t) ? 0.0 : fr[rr], f_i = fi[rr];
      Dr[rr][cc] = br - (f_r * Dr[t][cc] - f_i * Di[t][cc]);
      Di[rr][cc] = bi - (f_r * Di[t][cc] + f_i * Dr[t][cc]);
    }
    __syncthreads();
  }
  for (int t = kGj - 1; t >= 0; --t) {
    const int r = perm[t];
    if (r != t && tid < kGj) {
      const double ar = Dr[tid][t], ai = Di[tid][t];
      Dr[tid][t] = Dr[tid][r];
      Di[tid][t] = Di[tid][r];
      Dr[tid][r] = ar;
      Di[tid][r] = ai;
    }
    __syncthreads();
  }
  for (int i = tid; i < kGj * kGj; i += blockDim.x)
    A[static_cast<int64_t>(i / kGj) * m + i % kGj] = make_double2(Dr[i / kGj][i % kGj], Di[i / kGj][i % kGj]);
  if (tid == 0 && singular) flag[c] = 1;
}

// Row panel of step kb: A[kb][j] <- D^{-1} A[kb][j] for the columns of one
// 16-column slab outside tile kb.  The slab is staged in LDS; each thread
// forms four outputs of one row with D^{-1} read from the diagonal tile.
__global__ __launch_bounds__(256) void k_gj_row(double2 *__restrict__ blk, int m, int kb) {
  const int slab = blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
  if (slab / (kGj / 16) == kb) return;
  __shared__ cx<double> T[kGj][16];
  double2 *A = blk + static_cast<int64_t>(c) * m * m;
  const int64_t r0 = static_cast<int64_t>(kb) * kGj;
  const int col0 = slab * 16;
  for (int i = tid; i < kGj * 16; i += blockDim.x) T[i / 16][i % 16] = ld<double>(A[(r0 + i / 16) * m + col0 + i % 16]);
  __syncthreads();
  const int r = tid / 4, cg = (tid % 4) * 4;
  const double2 *Dinv = A + r0 * m + r0 + static_cast<int64_t>(r) * m;
  cx<double> o[4] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
  for (int k = 0; k < kGj; ++k) {
    const cx<double> d = ld<double>(Dinv[k]);
#pragma unroll
    for (int j = 0; j < 4; ++j) cmac(o[j], d, T[k][cg + j]);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) A[(r0 + r) * m + col0 + cg + j] = st(o[j]);
}

// Column panel of step kb: A[i][kb] <- -A[i][kb] D^{-1} for the rows of one
// 16-row slab outside tile kb (after the rank-64 update has used them).
__global__ __launch_bounds__(256) void k_gj_col(double2 *__restrict__ blk, int m, int kb) {
  const int slab = blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
  if (slab / (kGj / 16) == kb) return;
  __shared__ cx<double> T[16][kGj];
  double2 *A = blk + static_cast<int64_t>(c) * m * m;
  const int64_t c0 = static_cast<int64_t>(kb) * kGj;
  const int64_t row0 = static_cast<int64_t>(slab) * 16;
  for (int i = tid; i < 16 * kGj; i += blockDim.x) T[i / kGj][i % kGj] = ld<double>(A[(row0 + i / kGj) * m + c0 + i % kGj]);
  __syncthreads();
  const int r = tid / 16, cg = (tid % 16) * 4;
  const double2 *Dinv = A + c0 * m + c0;
  cx<double> o[4] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
  for (int k = 0; k < kGj; ++k) {
    const cx<double> a = T[r][k];
#pragma unroll
    for (int j = 0; j < 4; ++j) cmac(o[j], a, ld<double>(Dinv[static_cast<int64_t>(k) * m + cg + j]));
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) A[(row0 + r) * m + c0 + cg + j] = make_double2(-o[j].re, -o[j].im);
}

// Rank-64 update of step kb on the FP64 matrix cores: for every 64 x 64 tile
// (it, jt) with it, jt != kb,  A[it][jt] -= A[it][kb] A[kb][jt]  (the row
// panel already holds D^{-1} A[kb][jt]).  Four waves, each a 32 x 32 quarter
// as 2 x 2 blocks of 16 x 16; K in chunks of 16 staged in LDS as real,
// imaginary and summed parts so that each complex product takes three real
// MFMAs: P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi); re = P1 - P2,
// im = P3 - P1 - P2.  MFMA 16x16x4 f64: lane i supplies A[i % 16][i / 16] and
// B[i / 16][i % 16]; result register j of lane i is D[i / 16 + 4 j][i % 16].
__global__ __launch_bounds__(256) void k_gj_update(double2 *__restrict__ blk, int m, int kb, int ntile) {
  typedef double v4 __attribute__((ext_vector_type(4)));
  const int it = blockIdx.x / ntile, jt = blockIdx.x % ntile, c = blockIdx.y;
  if (it == kb || jt == kb) return;
  __shared__ double Ar[kGj][17], Ai[kGj][17], As[kGj][17];
  __shared__ double Br[16][kGj], Bi[16][kGj], Bs[16][kGj];
  double2 *A = blk + static_cast<int64_t>(c) * m * m;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  const int64_t arow0 = static_cast<int64_t>(it) * kGj, acol0 = static_cast<int64_t>(kb) * kGj;
  const int64_t brow0 = static_cast<int64_t>(kb) * kGj, bcol0 = static_cast<int64_t>(jt) * kGj;
  v4 P1[2][2], P2[2][2], P3[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      P1[bi][bj] = v4{0, 0, 0, 0};
      P2[bi][bj] = v4{0, 0, 0, 0};
      P3[bi][bj] = v4{0, 0, 0, 0};
    }
  for (int kc = 0; kc < kGj; kc += 16) {
    __syncthreads();  // previous chunk consumed
    for (int i = tid; i < kGj * 16; i += 256) {
      const int r = i / 16, k = i % 16;
      const double2 a = A[(arow0 + r) * m + acol0 + kc + k];
      Ar[r][k] = a.x;
      Ai[r][k] = a.y;
      As[r][k] = a.x + a.y;
      const int kk = i / kGj, cc = i % kGj;
      const double2 b = A[(brow0 + kc + kk) * m + bcol0 + cc];
      Br[kk][cc] = b.x;
      Bi[kk][cc] = b.y;
      Bs[kk][cc] = b.x + b.y;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 16; ks += 4) {
      const int k = ks + (lane >> 4);
      double ar[2], ai[2], as[2], br[2], bim[2], bs[2];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) {
        const int r = wr + bi * 16 + (lane & 15);
        ar[bi] = Ar[r][k];
        ai[bi] = Ai[r][k];
        as[bi] = As[r][k];
      }
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        const int cc = wc + bj * 16 + (lane & 15);
        br[bj] = Br[k][cc];
        bim[bj] = Bi[k][cc];
        bs[bj] = Bs[k][cc];
      }
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
          P1[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[bi], br[bj], P1[bi][bj], 0, 0, 0);
          P2[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[bi], bim[bj], P2[bi][bj], 0, 0, 0);
          P3[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(as[bi], bs[bj], P3[bi][bj], 0, 0, 0);
        }
    }
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t r = arow0 + wr + bi * 16 + (lane >> 4) + 4 * j;
        const int64_t cc = bcol0 + wc + bj * 16 + (lane & 15);
        const double p1 = P1[bi][bj][j], p2 = P2[bi][bj][j], p3 = P3[bi][bj][j];
        double2 v = A[r * m + cc];
        v.x -= p1 - p2;
        v.y -= p3 - p1 - p2;
        A[r * m + cc] = v;
      }
}

// flag[c][slot] = 1 when the slot's share of block c holds a non-finite entry.
__global__ void k_pc_finite(const double2 *__restrict__ blk, int64_t mm, int slots, int32_t *__restrict__ flag) {
  const int c = blockIdx.y, s = blockIdx.x;
  const double2 *B = blk + static_cast<int64_t>(c) * mm;
  const int64_t per = (mm + slots - 1) / slots;
  const int64_t lo = static_cast<int64_t>(s) * per, hi = min(mm, lo + per);
  bool bad = false;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) bad |= !(isfinite(B[i].x) && isfinite(B[i].y));
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) flag[static_cast<int64_t>(c) * slots + s] = bad ? 1 : 0;
}

// Block c <- identity (a block whose inversion failed).
__global__ void k_pc_identity(double2 *__restrict__ blk, int m, int c) {
  const int64_t mm = static_cast<int64_t>(m) * m;
  double2 *B = blk + static_cast<int64_t>(c) * mm;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < mm;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    B[i] = make_double2(i / m == i % m ? 1.0 : 0.0, 0.0);
}

__global__ void k_pc_to32(const double2 *__restrict__ a, float2 *__restrict__ b, int64_t len) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < len;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    b[i] = make_float2(static_cast<float>(a[i].x), static_cast<float>(a[i].y));
}

// y = M^{-1} x, partial sums over column chunks.  Block (row tile, chunk,
// cluster): the chunk's gathered inputs in LDS, wave w of four takes 16 rows,
// each row streamed by 64 lanes (coalesced), reduced across the wave.  Block
// entries in TM, vectors and sums in FP64.
template <typename TM>
__global__ __launch_bounds__(256) void k_pc_apply(const cv_t<TM> *__restrict__ blk,
                                                 const int32_t *__restrict__ members,
                                                 const int32_t *__restrict__ counts, int mp, int m, int P,
                                                 const double2 *__restrict__ x, double2 *__restrict__ part,
                                                 int nchunk) {
  const int rt = blockIdx.x, ch = blockIdx.y, c = blockIdx.z;
  const int rows = counts[c] * P;
  if (rt * 64 >= rows) return;
  __shared__ cx<double> u[kPcCols];
  const int col0 = ch * kPcCols;
  const int ncol = min(kPcCols, m - col0);
  const int tid = threadIdx.x;
  for (int j = tid; j < kPcCols; j += 256) {
    const int col = col0 + j;
    cx<double> v = mk(0.0, 0.0);
    if (col < rows) v = ld<double>(x[static_cast<int64_t>(members[static_cast<int64_t>(c) * mp + col / P]) * P + col % P]);
    u[j] = v;
  }
  __syncthreads();
  const int w = tid >> 6, lane = tid & 63;
  const cv_t<TM> *B = blk + (static_cast<int64_t>(c) * m + static_cast<int64_t>(rt) * 64 + w * 16) * m + col0;
  double2 *out = part + (static_cast<int64_t>(c) * nchunk + ch) * m + rt * 64 + w * 16;
  for (int rr = 0; rr < 16; ++rr) {
    if (rt * 64 + w * 16 + rr >= rows) break;  // wave-uniform
    const cv_t<TM> *br = B + static_cast<int64_t>(rr) * m;
    double sr = 0.0, si = 0.0;
#pragma unroll 8
    for (int j = lane; j < ncol; j += 64) {
      const cv_t<TM> a = br[j];
      const cx<double> b = u[j];
      sr = fma(static_cast<double>(a.x), b.re, sr);
      sr = fma(-static_cast<double>(a.y), b.im, sr);
      si = fma(static_cast<double>(a.x), b.im, si);
      si = fma(static_cast<double>(a.y), b.re, si);
    }
    for (int o = 32; o > 0; o >>= 1) {
      sr += __shfl_xor(sr, o);
      si += __shfl_xor(si, o);
    }
    if (lane == 0) out[rr] = make_double2(sr, si);
  }
}

__global__ void k_pc_apply_sum(const double2 *__restrict__ part, const int32_t *__restrict__ members,
                               const int32_t *__restrict__ counts, int mp, int m, int P, int nchunk,
                               double2 *__restrict__ y) {
  const int c = blockIdx.y;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= counts[c] * P) return;
  const double2 *pp = part + static_cast<int64_t>(c) * nchunk * m + r;
  double sr = 0.0, si = 0.0;
  for (int ch = 0; ch < nchunk; ++ch) {
    sr += pp[static_cast<int64_t>(ch) * m].x;
    si += pp[static_cast<int64_t>(ch) * m].y;
  }
  y[static_cast<int64_t>(members[static_cast<int64_t>(c) * mp + r / P]) * P + r % P] = make_double2(sr, si);
}

}  // namespace

// ---------------------------------------------------------------------------
// Build the FP64 blocks (and the FP32 copy when prec is MPSL_FP32).
int precond_build(mpsl_ctx *ctx, int prec) {
  if (ctx->pc_kind != MPSL_PRECOND_CLUSTER) return MPSL_OK;
  if (prec == MPSL_FP32 ? ctx->pc_ok32 : ctx->pc_ok) return MPSL_OK;
  int rc = build_tables(ctx);
  if (rc) return rc;
  const auto t0 = std::chrono::steady_clock::now();
  const int P = 2 * ctx->p + 1;
  if (!ctx->pc_ok) {
    std::vector<int64_t> idx;
    std::vector<std::pair<size_t, size_t>> ranges;
    make_clusters(ctx->n, ctx->xy.data(), ctx->pc_size, idx, ranges);
    const int nc = static_cast<int>(ranges.size());
    int mp = 0;
    for (auto &r : ranges) mp = std::max(mp, static_cast<int>(r.second - r.first));
    const int m = cdivi(static_cast<int64_t>(mp) * P, kGj) * kGj;
    if (m > kPcMaxDim)
      return set_err(ctx, MPSL_EINVAL, "cluster block of " + std::to_string(m) + " unknowns above " +
                                           std::to_string(kPcMaxDim) + ": lower the cluster size");
    std::vector<int32_t> mem(static_cast<size_t>(nc) * mp + nc, -1);
    for (int c = 0; c < nc; ++c) {
      const auto &r = ranges[c];
      for (size_t i = r.first; i < r.second; ++i) mem[static_cast<size_t>(c) * mp + (i - r.first)] = static_cast<int32_t>(idx[i]);
      mem[static_cast<size_t>(nc) * mp + c] = static_cast<int32_t>(r.second - r.first);
    }
    const int fslots = 64;
    const size_t mm = static_cast<size_t>(m) * m;
    if ((rc = dev_alloc(ctx, ctx->pc_idx, mem.size() * sizeof(int32_t))) ||
        (rc = dev_alloc(ctx, ctx->pc_flag, static_cast<size_t>(nc) * (fslots + 1) * sizeof(int32_t))) ||
        (rc = dev_alloc(ctx, ctx->pc_blk, static_cast<size_t>(nc) * mm * sizeof(double2))))
      return rc;
    MPSL_HIP_TRY(ctx, hipMemcpyAsync(ctx->pc_idx.p, mem.data(), mem.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                     ctx->stream));
    MPSL_HIP_TRY(ctx, hipMemsetAsync(ctx->pc_flag.p, 0, static_cast<size_t>(nc) * (fslots + 1) * sizeof(int32_t),
                                     ctx->stream));
    const auto *members = static_cast<const int32_t *>(ctx->pc_idx.p);
    const auto *counts = members + static_cast<size_t>(nc) * mp;
    auto *blk = static_cast<double2 *>(ctx->pc_blk.p);
    auto *flag = static_cast<int32_t *>(ctx->pc_flag.p);
    const bool typed = ctx->n_types > 1 && !ctx->ptype.empty();
    hipLaunchKernelGGL(k_pc_assemble, dim3(mp, nc), dim3(256), 0, ctx->stream, members, counts, mp, m,
                       static_cast<const double2 *>(ctx->gt.xy.p), static_cast<const double2 *>(ctx->gt.rot64.p),
                       static_cast<const double2 *>(ctx->S64.p),
                       typed ? static_cast<const int32_t *>(ctx->types_dev.p) : nullptr, ctx->k2.real(), ctx->p, blk);
    PC_CHECK(ctx);
    hipLaunchKernelGGL(k_pc_pad, dim3(m, nc), dim3(256), 0, ctx->stream, counts, m, P, blk);
    PC_CHECK(ctx);
    const int nt = m / kGj;
    for (int kb = 0; kb < nt; ++kb) {
      hipLaunchKernelGGL(k_gj_diag, dim3(nc), dim3(256), 0, ctx->stream, blk, m, kb, flag + static_cast<size_t>(nc) * fslots);
      PC_CHECK(ctx);
      if (nt > 1) {
        hipLaunchKernelGGL(k_gj_row, dim3(m / 16, nc), dim3(256), 0, ctx->stream, blk, m, kb);
        PC_CHECK(ctx);
        hipLaunchKernelGGL(k_gj_update, dim3(nt * nt, nc), dim3(256), 0, ctx->stream, blk, m, kb, nt);
        PC_CHECK(ctx);
        hipLaunchKernelGGL(k_gj_col, dim3(m / 16, nc), dim3(256), 0, ctx->stream, blk, m, kb);
        PC_CHECK(ctx);
      }
    }
    hipLaunchKernelGGL(k_pc_finite, dim3(fslots, nc), dim3(256), 0, ctx->stream, blk, static_cast<int64_t>(mm), fslots,
                       flag);
    PC_CHECK(ctx);
    std::vector<int32_t> hf(static_cast<size_t>(nc) * (fslots + 1));
    MPSL_HIP_TRY(ctx, hipMemcpyAsync(hf.data(), flag, hf.size() * sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    MPSL_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    int replaced = 0;
    for (int c = 0; c < nc; ++c) {
      bool bad = hf[static_cast<size_t>(nc) * fslots + c] != 0;
      for (int s = 0; s < fslots; ++s) bad |= hf[static_cast<size_t>(c) * fslots + s] != 0;
      if (bad) {
        hipLaunchKernelGGL(k_pc_identity, dim3(1024), dim3(256), 0, ctx->stream, blk, m, c);
        PC_CHECK(ctx);
        ++replaced;
      }
    }
    ctx->pc_nc = nc;
    ctx->pc_mp = mp;
    ctx->pc_m = m;
    ctx->pc_replaced = replaced;
    ctx->pc_ok = true;
  }
  if (prec == MPSL_FP32) {
    // the mixed-precision solve applies only the FP32 copy: the FP64 blocks
    // are released (an FP64 solve on this context rebuilds them)
    const size_t len = static_cast<size_t>(ctx->pc_nc) * ctx->pc_m * ctx->pc_m;
    if ((rc = dev_alloc(ctx, ctx->pc_blk32, len * sizeof(float2)))) return rc;
    hipLaunchKernelGGL(k_pc_to32, dim3(4096), dim3(256), 0, ctx->stream, static_cast<const double2 *>(ctx->pc_blk.p),
                       static_cast<float2 *>(ctx->pc_blk32.p), static_cast<int64_t>(len));
    PC_CHECK(ctx);
    MPSL_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    dev_free(ctx->pc_blk);
    ctx->pc_ok = false;
    ctx->pc_ok32 = true;
  }
  MPSL_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  ctx->pc_setup_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return MPSL_OK;
}

int cluster_shape(int64_t n, const double *xy, int size, int *nc, int *mp) {
  if (n <= 0 || !xy || size < 1) return MPSL_EINVAL;
  std::vector<int64_t> idx;
  std::vector<std::pair<size_t, size_t>> ranges;
  make_clusters(n, xy, size, idx, ranges);
  int big = 0;
  for (auto &r : ranges) big = std::max(big, static_cast<int>(r.second - r.first));
  *nc = static_cast<int>(ranges.size());
  *mp = big;
  return MPSL_OK;
}

// y = M^{-1} x on FP64 vectors (device, N P entries), with the blocks of
// precision prec.  x and y must not overlap.
int precond_apply(mpsl_ctx *ctx, int prec, const void *x, void *y) {
  if (prec == MPSL_FP32 ? !ctx->pc_ok32 : !ctx->pc_ok)
    return set_err(ctx, MPSL_ESTATE, "preconditioner blocks not built");
  const int P = 2 * ctx->p + 1;
  const int nc = ctx->pc_nc, mp = ctx->pc_mp, m = ctx->pc_m;
  const int nchunk = cdivi(m, kPcCols);
  int rc;
  if ((rc = dev_alloc(ctx, ctx->pc_part, static_cast<size_t>(nc) * nchunk * m * sizeof(double2)))) return rc;
  const auto *members = static_cast<const int32_t *>(ctx->pc_idx.p);
  const auto *counts = members + static_cast<size_t>(nc) * mp;
  auto *part = static_cast<double2 *>(ctx->pc_part.p);
  const dim3 grid(cdivi(m, 64), nchunk, nc);
  if (prec == MPSL_FP64)
    hipLaunchKernelGGL(k_pc_apply<double>, grid, dim3(256), 0, ctx->stream, static_cast<const double2 *>(ctx->pc_blk.p),
                       members, counts, mp, m, P, static_cast<const double2 *>(x), part, nchunk);
  else
    hipLaunchKernelGGL(k_pc_apply<float>, grid, dim3(256), 0, ctx->stream, static_cast<const float2 *>(ctx->pc_blk32.p),
                       members, counts, mp, m, P, static_cast<const double2 *>(x), part, nchunk);
  PC_CHECK(ctx);
  hipLaunchKernelGGL(k_pc_apply_sum, dim3(cdivi(m, 256), nc), dim3(256), 0, ctx->stream, part, members, counts, mp, m,
                     P, nchunk, static_cast<double2 *>(y));
  PC_CHECK(ctx);
  return MPSL_OK;
}

}  // namespace mpsl

extern "C" {

int mpsl_compute_clusters(int64_t n, const double *xy, int cluster_size, int32_t *cluster_of, int *n_clusters) {
  if (n <= 0 || !xy || cluster_size < 1 || (!cluster_of && !n_clusters)) return MPSL_EINVAL;
  for (int64_t i = 0; i < 2 * n; ++i)
    if (!std::isfinite(xy[i])) return MPSL_EINVAL;
  std::vector<int64_t> idx;
  std::vector<std::pair<size_t, size_t>> ranges;
  mpsl::make_clusters(n, xy, cluster_size, idx, ranges);
  if (cluster_of)
    for (size_t c = 0; c < ranges.size(); ++c)
      for (size_t i = ranges[c].first; i < ranges[c].second; ++i) cluster_of[idx[i]] = static_cast<int32_t>(c);
  if (n_clusters) *n_clusters = static_cast<int>(ranges.size());
  return MPSL_OK;
}

int mpsl_set_preconditioner(mpsl_ctx *ctx, int kind, int cluster_size) {
  if (!ctx) return MPSL_EINVAL;
  if (kind != MPSL_PRECOND_NONE && kind != MPSL_PRECOND_CLUSTER)
    return mpsl::set_err(ctx, MPSL_EINVAL, "kind must be MPSL_PRECOND_NONE or MPSL_PRECOND_CLUSTER");
  if (cluster_size < 0) return mpsl::set_err(ctx, MPSL_EINVAL, "cluster size must be >= 0");
  const int size = cluster_size == 0 ? mpsl::kPcDefaultSize : cluster_size;
  if (kind != ctx->pc_kind || size != ctx->pc_size) ctx->pc_ok = ctx->pc_ok32 = false;
  ctx->pc_kind = kind;
  ctx->pc_size = size;
  if (kind == MPSL_PRECOND_NONE) {
    mpsl::dev_free(ctx->pc_blk);
    mpsl::dev_free(ctx->pc_blk32);
    mpsl::dev_free(ctx->pc_part);
  }
  return MPSL_OK;
}

int mpsl_precond_apply_dev(mpsl_ctx *ctx, int prec, const void *x_dev, void *y_dev) {
  if (!ctx || !x_dev || !y_dev || (prec != MPSL_FP64 && prec != MPSL_FP32)) return MPSL_EINVAL;
  if (x_dev == y_dev) return mpsl::set_err(ctx, MPSL_EINVAL, "x and y must not overlap");
  MPSL_HIP_TRY(ctx, hipSetDevice(ctx->device));
  if (ctx->pc_kind != MPSL_PRECOND_CLUSTER) return mpsl::set_err(ctx, MPSL_ESTATE, "no preconditioner set");
  int rc = mpsl::precond_build(ctx, prec);
  if (rc) return rc;
  return mpsl::precond_apply(ctx, prec, x_dev, y_dev);
}

int mpsl_get_precond_info(const mpsl_ctx *ctx, int *n_clusters, int *max_cluster, int *block_dim, int *replaced,
                          double *setup_seconds) {
  if (!ctx) return MPSL_EINVAL;
  const bool ok = ctx->pc_kind == MPSL_PRECOND_CLUSTER && (ctx->pc_ok || ctx->pc_ok32);
  if (n_clusters) *n_clusters = ok ? ctx->pc_nc : 0;
  if (max_cluster) *max_cluster = ok ? ctx->pc_mp : 0;
  if (block_dim) *block_dim = ok ? ctx->pc_m : 0;
  if (replaced) *replaced = ok ? ctx->pc_replaced : 0;
  if (setup_seconds) *setup_seconds = ctx->pc_setup_s;
  return MPSL_OK;
}

}  // extern "C"
