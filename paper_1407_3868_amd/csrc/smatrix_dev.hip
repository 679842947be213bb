// Device precompute of the prototype scattering matrix of a star particle
// (Section 4, eqs. (31)-(32) and (35); TE form with rho = k2^2 / kp^2).
//
// The host prepares the O(nb P) parts (boundary samples, quadrature tables,
// right-hand sides, eq. (35) weights: bie.h); the device does the O(nb^2)
// Nystrom assembly with Hankel functions, the two O(nb^3) products of Maue's
// identity, the O(nb^3) LU with partial pivoting of the 2 nb x 2 nb system
// (eliminating all 2p+1 right-hand sides along), back substitution and the
// projection of eq. (35).  Everything is FP64 on the context's stream.
#include <cmath>

#include "bie.h"
#include "context.h"

namespace mpsl {

namespace {

constexpr double kEulerG = 0.57721566490153286061;
constexpr int kTile = 16;

struct DevCurve {
  const double *t, *x, *y, *dx, *dy, *ddx, *ddy, *speed, *nx, *ny;
};

// Nystrom matrices of S_k, D_k, N_k and S_k without |x'(tau)| (row i: target
// t_i), each kernel split as K1 ln(4 sin^2((t - tau)/2)) + K2.
__global__ void k_bie_ops(double k, int nb, DevCurve c, const double *__restrict__ Rk, double2 *__restrict__ S,
                          double2 *__restrict__ D, double2 *__restrict__ N, double2 *__restrict__ S0) {
  const int64_t id = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (id >= static_cast<int64_t>(nb) * nb) return;
  const int i = static_cast<int>(id / nb), j = static_cast<int>(id % nb);
  const double h = 2.0 * M_PI / nb;
  const double R = Rk[(i - j + nb) % nb];
  cx<double> s, d, nn;
  if (i == j) {
    const double sp = c.speed[i];
    const double curv = (c.dy[i] * c.ddx[i] - c.dx[i] * c.ddy[i]) / (sp * sp);
    const double s1 = -sp / (4.0 * M_PI);
    const cx<double> s2 = sp * mk(-kEulerG / (2.0 * M_PI) - log(k * sp / 2.0) / (2.0 * M_PI), 0.25);
    s = mk(R * s1, 0.0) + h * s2;
    d = mk(h * curv / (4.0 * M_PI), 0.0);
    nn = d;
  } else {
    const double ddx = c.x[i] - c.x[j], ddy = c.y[i] - c.y[j];
    const double rr = sqrt(ddx * ddx + ddy * ddy);
    const double z = k * rr;
    const double J0 = j0(z), Y0 = y0(z), J1 = j1(z), Y1 = y1(z);
    const double sn = sin((c.t[i] - c.t[j]) / 2.0);
    const double lg = log(4.0 * sn * sn);
    const double sp = c.speed[j];
    // single layer: (i/4) H_0(k r) |x'(tau)|
    const cx<double> m = (0.25 * sp) * mk(-Y0, J0);
    const double m1 = -J0 * sp / (4.0 * M_PI);
    s = mk(R * m1, 0.0) + h * (m - mk(m1 * lg, 0.0));
    // double layer: (ik/4) H_1(k r) nu(tau).(x(t) - x(tau)) / r
    const double nud = c.dy[j] * ddx - c.dx[j] * ddy;
    const double fl = 0.25 * k * nud / rr;
    const cx<double> l = mk(-fl * Y1, fl * J1);
    const double l1 = -k * J1 * nud / (4.0 * M_PI * rr);
    d = mk(R * l1, 0.0) + h * (l - mk(l1 * lg, 0.0));
    // normal derivative of the single layer: -(ik/4) H_1(k r) n(t).(x(t) - x(tau)) / r |x'(tau)|
    const double nd = c.nx[i] * ddx + c.ny[i] * ddy;
    const double fq = -0.25 * k * nd / rr * sp;
    const cx<double> q = mk(-fq * Y1, fq * J1);
    const double q1 = k * J1 * nd / (4.0 * M_PI * rr) * sp;
    nn = mk(R * q1, 0.0) + h * (q - mk(q1 * lg, 0.0));
  }
  S[id] = st(s);
  D[id] = st(d);
  N[id] = st(nn);
  S0[id] = st((1.0 / c.speed[j]) * s);
}

__global__ void k_bie_sub(int64_t n, const double2 *__restrict__ a, const double2 *__restrict__ b,
                          double2 *__restrict__ out) {
  const int64_t id = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (id < n) out[id] = st(ld<double>(a[id]) - ld<double>(b[id]));
}

// C = X Y for n x n matrices, one of them real (XR: X real, else Y real);
// 16 x 16 tiles through LDS.
template <bool XR>
__global__ void __launch_bounds__(kTile *kTile) k_bie_gemm(int n, const double *__restrict__ Xr,
                                                           const double2 *__restrict__ Xc,
                                                           const double *__restrict__ Yr,
                                                           const double2 *__restrict__ Yc, double2 *__restrict__ C) {
  __shared__ double2 xs[kTile][kTile];
  __shared__ double2 ys[kTile][kTile];
  const int tx = threadIdx.x % kTile, ty = threadIdx.x / kTile;
  const int row = blockIdx.y * kTile + ty, col = blockIdx.x * kTile + tx;
  cx<double> acc = mk(0.0, 0.0);
  for (int k0 = 0; k0 < n; k0 += kTile) {
    const int xc = k0 + tx, yr = k0 + ty;
    double2 xv = make_double2(0.0, 0.0), yv = make_double2(0.0, 0.0);
    if (row < n && xc < n) xv = XR ? make_double2(Xr[static_cast<int64_t>(row) * n + xc], 0.0)
                                   : Xc[static_cast<int64_t>(row) * n + xc];
    if (yr < n && col < n) yv = XR ? Yc[static_cast<int64_t>(yr) * n + col]
                                   : make_double2(Yr[static_cast<int64_t>(yr) * n + col], 0.0);
    xs[ty][tx] = xv;
    ys[ty][tx] = yv;
    __syncthreads();
    for (int k = 0; k < kTile; ++k) cmac(acc, ld<double>(xs[ty][k]), ld<double>(ys[k][tx]));
    __syncthreads();
  }
  if (row < n && col < n) C[static_cast<int64_t>(row) * n + col] = st(acc);
}

// Mueller's system (TE form, rho = 1 for TM), A row-major 2 nb x 2 nb.
__global__ void k_bie_assemble(int nb, double k2, double kp, double rho, const double *__restrict__ speed,
                               const double *__restrict__ nx, const double *__restrict__ ny,
                               const double2 *__restrict__ S2, const double2 *__restrict__ D2,
                               const double2 *__restrict__ N2, const double2 *__restrict__ Sp,
                               const double2 *__restrict__ Dp, const double2 *__restrict__ Np,
                               const double2 *__restrict__ FdT, double2 *__restrict__ A) {
  const int64_t id = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (id >= static_cast<int64_t>(nb) * nb) return;
  const int i = static_cast<int>(id / nb), j = static_cast<int>(id % nb);
  const int64_t M = 2 * static_cast<int64_t>(nb);
  const double idn = (i == j) ? 1.0 : 0.0;
  const double id_mu = 0.5 * (1.0 + 1.0 / rho), id_sig = 0.5 * (1.0 + rho);
  const double nn = nx[i] * nx[j] + ny[i] * ny[j];
  const cx<double> t = (1.0 / speed[i]) * ld<double>(FdT[id]) +
                       nn * ((k2 * k2) * ld<double>(S2[id]) - (kp * kp) * ld<double>(Sp[id]));
  A[i * M + j] = st(ld<double>(S2[id]) - ld<double>(Sp[id]));
  A[i * M + nb + j] = st(mk(id_mu * idn, 0.0) + ld<double>(D2[id]) - (1.0 / rho) * ld<double>(Dp[id]));
  A[(nb + i) * M + j] = st(mk(-id_sig * idn, 0.0) + ld<double>(N2[id]) - rho * ld<double>(Np[id]));
  A[(nb + i) * M + nb + j] = st(t);
}

// Partial pivoting at column k: the row of largest modulus among k..M-1 is
// swapped into row k (columns k..M-1 of A and every right-hand side).
__global__ void __launch_bounds__(256) k_lu_pivot(int M, int P, int k, double2 *__restrict__ A,
                                                  double2 *__restrict__ B, int *__restrict__ info) {
  __shared__ double bv[256];
  __shared__ int bi[256];
  double best = -1.0;
  int arg = k;
  for (int i = k + threadIdx.x; i < M; i += blockDim.x) {
    const double2 a = A[static_cast<int64_t>(i) * M + k];
    const double v = a.x * a.x + a.y * a.y;
    if (v > best) {
      best = v;
      arg = i;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = arg;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const double o = bv[threadIdx.x + s];
      const int oi = bi[threadIdx.x + s];
      if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = o;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const int pr = bi[0];
  if (threadIdx.x == 0 && !(bv[0] > 0.0)) info[0] = 1;
  if (pr == k) return;
  for (int j = k + threadIdx.x; j < M; j += blockDim.x) {
    const double2 a = A[static_cast<int64_t>(k) * M + j];
    A[static_cast<int64_t>(k) * M + j] = A[static_cast<int64_t>(pr) * M + j];
    A[static_cast<int64_t>(pr) * M + j] = a;
  }
  for (int r = threadIdx.x; r < P; r += blockDim.x) {
    const double2 b = B[static_cast<int64_t>(r) * M + k];
    B[static_cast<int64_t>(r) * M + k] = B[static_cast<int64_t>(r) * M + pr];
    B[static_cast<int64_t>(r) * M + pr] = b;
  }
}

// Elimination below the pivot: rows i > k, columns j > k of A and all
// right-hand sides (column k and row k are only read).
__global__ void k_lu_update(int M, int P, int k, double2 *__restrict__ A, double2 *__restrict__ B) {
  const int w = M - k - 1;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = k + 1 + blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= M || c >= w + P) return;
  const cx<double> piv = ld<double>(A[static_cast<int64_t>(k) * M + k]);
  const cx<double> a = ld<double>(A[static_cast<int64_t>(i) * M + k]);
  const double den = piv.re * piv.re + piv.im * piv.im;
  const cx<double> f = (1.0 / den) * (a * conj(piv));
  if (c < w) {
    const int j = k + 1 + c;
    A[static_cast<int64_t>(i) * M + j] =
        st(ld<double>(A[static_cast<int64_t>(i) * M + j]) - f * ld<double>(A[static_cast<int64_t>(k) * M + j]));
  } else {
    const int r = c - w;
    B[static_cast<int64_t>(r) * M + i] =
        st(ld<double>(B[static_cast<int64_t>(r) * M + i]) - f * ld<double>(B[static_cast<int64_t>(r) * M + k]));
  }
}

// Back substitution with the upper triangle, one block per right-hand side.
__global__ void __launch_bounds__(256) k_lu_back(int M, const double2 *__restrict__ A, double2 *__restrict__ B) {
  __shared__ double2 xk;
  double2 *b = B + static_cast<int64_t>(blockIdx.x) * M;
  for (int k = M - 1; k >= 0; --k) {
    if (threadIdx.x == 0) {
      const cx<double> u = ld<double>(A[static_cast<int64_t>(k) * M + k]);
      const double den = u.re * u.re + u.im * u.im;
      const cx<double> x = (1.0 / den) * (ld<double>(b[k]) * conj(u));
      b[k] = st(x);
      xk = st(x);
    }
    __syncthreads();
    const cx<double> x = ld<double>(xk);
    for (int i = threadIdx.x; i < k; i += blockDim.x)
      b[i] = st(ld<double>(b[i]) - ld<double>(A[static_cast<int64_t>(i) * M + k]) * x);
    __syncthreads();
  }
}

// eq. (35): S[l][r] = sum_j Fs[l][j] sigma_r[j] + Fm[l][j] mu_r[j].
__global__ void k_bie_extract(int nb, int P, const double2 *__restrict__ Fs, const double2 *__restrict__ Fm,
                              const double2 *__restrict__ X, double2 *__restrict__ S) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= P * P) return;
  const int l = id / P, r = id % P;
  const double2 *sig = X + static_cast<int64_t>(r) * 2 * nb;
  const double2 *mu = sig + nb;
  cx<double> s = mk(0.0, 0.0);
  for (int j = 0; j < nb; ++j) {
    cmac(s, ld<double>(Fs[static_cast<int64_t>(l) * nb + j]), ld<double>(sig[j]));
    cmac(s, ld<double>(Fm[static_cast<int64_t>(l) * nb + j]), ld<double>(mu[j]));
  }
  S[id] = st(s);
}

inline int cdivi(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }

}  // namespace

int star_smatrix_device(mpsl_ctx *ctx, const StarParts &sp, double k2, double kp, int pol, std::vector<zc> &S,
                        std::string &err) {
  const int nb = sp.nb, P = 2 * sp.p + 1, M = 2 * nb;
  const int64_t nn = static_cast<int64_t>(nb) * nb;
  // one scratch allocation: 10 curve arrays, Rk, Fd | 9 nb^2 complex work | A | B | Fs, Fm | S | info
  const size_t real_cnt = 10 * static_cast<size_t>(nb) + nb + nn;
  const size_t cplx_cnt = 9 * nn + static_cast<size_t>(M) * M + static_cast<size_t>(P) * M +
                          2 * static_cast<size_t>(P) * nb + static_cast<size_t>(P) * P;
  const size_t bytes = real_cnt * sizeof(double) + cplx_cnt * sizeof(double2) + 256;
  DBuf buf;
  int rc = dev_alloc(ctx, buf, bytes);
  if (rc) {
    err = ctx->err;
    return rc;
  }
  double *rbase = static_cast<double *>(buf.p);
  double *cur[10];
  const std::vector<double> *src[10] = {&sp.t, &sp.x, &sp.y, &sp.dx, &sp.dy, &sp.ddx, &sp.ddy, &sp.speed, &sp.nx, &sp.ny};
  for (int a = 0; a < 10; ++a) cur[a] = rbase + static_cast<size_t>(a) * nb;
  double *dRk = rbase + 10 * static_cast<size_t>(nb);
  double *dFd = dRk + nb;
  double2 *cbase = reinterpret_cast<double2 *>(rbase + real_cnt + (real_cnt & 1));
  double2 *S2 = cbase, *D2 = S2 + nn, *N2 = D2 + nn, *S02 = N2 + nn;
  double2 *Sp = S02 + nn, *Dp = Sp + nn, *Np = Dp + nn, *S0p = Np + nn, *tmp = S0p + nn;
  double2 *A = tmp + nn;
  double2 *B = A + static_cast<size_t>(M) * M;
  double2 *Fs = B + static_cast<size_t>(P) * M, *Fm = Fs + static_cast<size_t>(P) * nb;
  double2 *Sd = Fm + static_cast<size_t>(P) * nb;
  int *info = reinterpret_cast<int *>(Sd + static_cast<size_t>(P) * P);
  hipStream_t st_ = ctx->stream;
  auto fail = [&](const char *what, hipError_t e) {
    err = std::string(what) + ": " + hipGetErrorString(e);
    dev_free(buf);
    return MPSL_EHIP;
  };
  hipError_t e = hipSuccess;
  for (int a = 0; a < 10 && e == hipSuccess; ++a)
    e = hipMemcpyAsync(cur[a], src[a]->data(), nb * sizeof(double), hipMemcpyHostToDevice, st_);
  if (e == hipSuccess) e = hipMemcpyAsync(dRk, sp.Rk.data(), nb * sizeof(double), hipMemcpyHostToDevice, st_);
  if (e == hipSuccess) e = hipMemcpyAsync(dFd, sp.Fd.data(), nn * sizeof(double), hipMemcpyHostToDevice, st_);
  if (e == hipSuccess) e = hipMemcpyAsync(B, sp.B.data(), sp.B.size() * sizeof(double2), hipMemcpyHostToDevice, st_);
  if (e == hipSuccess) e = hipMemcpyAsync(Fs, sp.Fs.data(), sp.Fs.size() * sizeof(double2), hipMemcpyHostToDevice, st_);
  if (e == hipSuccess) e = hipMemcpyAsync(Fm, sp.Fm.data(), sp.Fm.size() * sizeof(double2), hipMemcpyHostToDevice, st_);
  if (e == hipSuccess) e = hipMemsetAsync(info, 0, sizeof(int), st_);
  if (e != hipSuccess) return fail("upload", e);
  const DevCurve c{cur[0], cur[1], cur[2], cur[3], cur[4], cur[5], cur[6], cur[7], cur[8], cur[9]};
  const int g1 = cdivi(nn, 256);
  hipLaunchKernelGGL(k_bie_ops, dim3(g1), dim3(256), 0, st_, k2, nb, c, dRk, S2, D2, N2, S02);
  hipLaunchKernelGGL(k_bie_ops, dim3(g1), dim3(256), 0, st_, kp, nb, c, dRk, Sp, Dp, Np, S0p);
  // Maue: T2 - Tp = diag(1/|x'|) Fd (S0_2 - S0_p) Fd + (n_i . n_j)(k2^2 S2 - kp^2 Sp)
  hipLaunchKernelGGL(k_bie_sub, dim3(g1), dim3(256), 0, st_, nn, S02, S0p, S02);
  const dim3 gg(cdivi(nb, kTile), cdivi(nb, kTile));
  hipLaunchKernelGGL(k_bie_gemm<false>, gg, dim3(kTile * kTile), 0, st_, nb, nullptr, S02, dFd, nullptr, tmp);
  hipLaunchKernelGGL(k_bie_gemm<true>, gg, dim3(kTile * kTile), 0, st_, nb, dFd, nullptr, nullptr, tmp, S0p);
  const double rho = (pol == MPSL_TE) ? (k2 * k2) / (kp * kp) : 1.0;
  hipLaunchKernelGGL(k_bie_assemble, dim3(g1), dim3(256), 0, st_, nb, k2, kp, rho, cur[7], cur[8], cur[9], S2, D2,
                     N2, Sp, Dp, Np, S0p, A);
  if ((e = hipGetLastError()) != hipSuccess) return fail("assembly", e);
  for (int k = 0; k < M; ++k) {
    hipLaunchKernelGGL(k_lu_pivot, dim3(1), dim3(256), 0, st_, M, P, k, A, B, info);
    const int w = M - k - 1;
    if (w > 0) {
      const dim3 blk(64, 4);
      const dim3 grd(cdivi(w + P, 64), cdivi(w, 4));
      hipLaunchKernelGGL(k_lu_update, grd, blk, 0, st_, M, P, k, A, B);
    }
  }
  hipLaunchKernelGGL(k_lu_back, dim3(P), dim3(256), 0, st_, M, A, B);
  hipLaunchKernelGGL(k_bie_extract, dim3(cdivi(static_cast<int64_t>(P) * P, 64)), dim3(64), 0, st_, nb, P, Fs, Fm,
                     B, Sd);
  if ((e = hipGetLastError()) != hipSuccess) return fail("solve", e);
  std::vector<double2> out(static_cast<size_t>(P) * P);
  int hinfo = 0;
  e = hipMemcpyAsync(out.data(), Sd, out.size() * sizeof(double2), hipMemcpyDeviceToHost, st_);
  if (e == hipSuccess) e = hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, st_);
  if (e == hipSuccess) e = hipStreamSynchronize(st_);
  if (e != hipSuccess) return fail("download", e);
  dev_free(buf);
  if (hinfo) {
    err = "singular boundary-integral system";
    return MPSL_ENUMERIC;
  }
  S.resize(out.size());
  for (size_t i = 0; i < out.size(); ++i) S[i] = zc(out[i].x, out[i].y);
  return MPSL_OK;
}

}  // namespace mpsl
