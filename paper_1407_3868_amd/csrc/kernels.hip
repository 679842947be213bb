// Device kernels of the layered-medium multiple-scattering matvec.
//
// Layouts (row-major, complex interleaved):
//   beta, alpha, x, y   [n][P]                 P = 2p + 1, slot n + p
//   part                [chunk][n][P]          partial local expansions
//   E (M2S factors)     [2][n][ns]             side 0: upper interface, 1: lower
//   F (S2L factors)     [2][ns][n]
//   W (M2S order sums)  [2][ns][P]
//   Up (S2L coeffs)     [2][ns][P]
//   spec, sigma         [2][ns]                FP64
#include <atomic>
#include <cmath>

#include "kernels.h"

namespace mpsl {

namespace {

constexpr int kThreads = 128;

inline int cdiv(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }

// complex exp(a + i b) in FP64
__device__ inline cx<double> cexp_d(double a, double b) {
  double s, c;
  sincos(b, &s, &c);
  const double e = exp(a);
  return {e * c, e * s};
}

// ---------------------------------------------------------------------------
// Row a0: plane-wave factors of every (particle, node) pair.
//   E+[m][q] = e^{-i lam x_m + g2 y_m}          E-[m][q] = e^{-i lam x_m - g2 (d + y_m)}
//   F+[q][l] = e^{ i lam x_l + g2 y_l}          F-[q][l] = e^{ i lam x_l - g2 (y_l + d)}
__global__ void k_geom_tables(const double2 *__restrict__ xy, const double2 *__restrict__ lam,
                              const double2 *__restrict__ g2, int n, int ns, double d,
                              double2 *__restrict__ E, double2 *__restrict__ F,
                              float2 *__restrict__ E32, float2 *__restrict__ F32) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  const int64_t tot = static_cast<int64_t>(n) * ns;
  if (idx >= tot) return;
  const int m = static_cast<int>(idx / ns);
  const int q = static_cast<int>(idx % ns);
  const double x = xy[m].x, y = xy[m].y;
  const double lr = lam[q].x, li = lam[q].y, gr = g2[q].x, gi = g2[q].y;
  const cx<double> ep = cexp_d(li * x + gr * y, -lr * x + gi * y);
  const cx<double> em = cexp_d(li * x - gr * (d + y), -lr * x - gi * (d + y));
  const cx<double> fp = cexp_d(-li * x + gr * y, lr * x + gi * y);
  const cx<double> fm = cexp_d(-li * x - gr * (y + d), lr * x - gi * (y + d));
  const int64_t e0 = static_cast<int64_t>(m) * ns + q;
  const int64_t f0 = static_cast<int64_t>(q) * n + m;
  E[e0] = st(ep);
  E[tot + e0] = st(em);
  F[f0] = st(fp);
  F[tot + f0] = st(fm);
  E32[e0] = make_float2(static_cast<float>(ep.re), static_cast<float>(ep.im));
  E32[tot + e0] = make_float2(static_cast<float>(em.re), static_cast<float>(em.im));
  F32[f0] = make_float2(static_cast<float>(fp.re), static_cast<float>(fp.im));
  F32[tot + f0] = make_float2(static_cast<float>(fm.re), static_cast<float>(fm.im));
}

// ---------------------------------------------------------------------------
// Row a0 (pairs): per ordered pair (m -> l) the Hankel functions H_0, H_1 of
// z = k2 |x_l - x_m|, the direction e^{i phi} = (x_l - x_m)/|x_l - x_m| and
// 2/z, computed once per geometry in FP64 and stored source-major
// [m][l][4] = {H_0, H_1, e^{i phi}, (2/z, 0)} in FP64 and FP32.  The self
// pair l == m holds zeros.
__global__ void k_pair_tables(const double2 *__restrict__ xy, int n, double k2, double2 *__restrict__ t64,
                              float2 *__restrict__ t32) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= static_cast<int64_t>(n) * n) return;
  const int m = static_cast<int>(idx / n);
  const int l = static_cast<int>(idx % n);
  double2 e[4] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0), make_double2(0.0, 0.0),
                  make_double2(0.0, 0.0)};
  if (l != m) {
    const double dx = xy[l].x - xy[m].x, dy = xy[l].y - xy[m].y;
    const double rho = sqrt(dx * dx + dy * dy);
    const double z = k2 * rho;
    e[0] = make_double2(j0(z), y0(z));
    e[1] = make_double2(j1(z), y1(z));
    e[2] = make_double2(dx / rho, dy / rho);
    e[3] = make_double2(2.0 / z, 0.0);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    t64[4 * idx + k] = e[k];
    t32[4 * idx + k] = make_float2(static_cast<float>(e[k].x), static_cast<float>(e[k].y));
  }
}

// Row a1: all-pairs free-space M2L (Graf's addition theorem).
// One lane per target l; every lane of the grid walks the same source chunk,
// so the source's coefficients are wave-uniform and live in scalar registers.
// Per pair: H_0, H_1 and e^{i phi} from the pair table, the upward recurrence
// H_{q+1} = (2q/z) H_q - H_{q-1}, e^{iq phi} by repeated multiplication,
// h_q = H_q e^{iq phi}, h_{-q} = (-1)^q H_q e^{-iq phi}, and the Toeplitz
// product alpha_{n'} += sum_nu h_{nu - n'} beta_nu consumed in the order the
// recurrence produces h_q.
//
// m2l_block adds the contribution of source slots [V0, V1] to output slots
// [O0, O1].  FP32 does everything in one call (33 accumulators, 66 scalar
// registers of beta at p = 16).  FP64 splits the outputs over two lanes and
// the source coefficients over two calls: 17 accumulators and at most 68
// scalar registers of beta, at the cost of re-running the recurrence.
template <typename T, int p, int O0, int O1, int V0, int V1, bool MIRROR>
__device__ __forceinline__ void m2l_block(cx<T> (&acc)[O1 - O0 + 1], const cv_t<T> *__restrict__ bm, cx<T> h0,
                                          cx<T> h1, cx<T> t, T two_over_z) {
  constexpr int QA = V1 - O0, QB = O1 - V0;
  constexpr int QMAX = (QA > QB ? QA : QB) < 2 * p ? (QA > QB ? QA : QB) : 2 * p;
  cx<T> bv[V1 - V0 + 1];
#pragma unroll
  for (int v = V0; v <= V1; ++v) bv[v - V0] = ld<T>(bm[MIRROR ? 2 * p - v : v]);
#pragma unroll
  for (int v = (V0 > O0 ? V0 : O0); v <= (V1 < O1 ? V1 : O1); ++v) cmac(acc[v - O0], h0, bv[v - V0]);
  cx<T> hprev = h0, hcur = h1, tq = t;
#pragma unroll
  for (int q = 1; q <= QMAX; ++q) {
    if (q >= 2) {
      const cx<T> hn = static_cast<T>(q - 1) * two_over_z * hcur - hprev;
      hprev = hcur;
      hcur = hn;
      tq = tq * t;
    }
    // alpha_{v-q} += h_q beta_v for v - q in [O0, O1]
    if ((V1 < O1 + q ? V1 : O1 + q) >= (V0 > O0 + q ? V0 : O0 + q)) {
      const cx<T> hp = hcur * tq;
#pragma unroll
      for (int v = (V0 > O0 + q ? V0 : O0 + q); v <= (V1 < O1 + q ? V1 : O1 + q); ++v)
        cmac(acc[v - q - O0], hp, bv[v - V0]);
    }
    // alpha_{v+q} += h_{-q} beta_v for v + q in [O0, O1]
    if ((V1 < O1 - q ? V1 : O1 - q) >= (V0 > O0 - q ? V0 : O0 - q)) {
      cx<T> hm = hcur * conj(tq);
      if (q & 1) hm = mk<T>(-hm.re, -hm.im);
#pragma unroll
      for (int v = (V0 > O0 - q ? V0 : O0 - q); v <= (V1 < O1 - q ? V1 : O1 - q); ++v)
        cmac(acc[v + q - O0], hm, bv[v - V0]);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Mirror identity: with reversed indices (alpha~_k = alpha_{-k},
// beta~_nu = beta_{-nu}) the translation keeps its Toeplitz form with
// h~_q = h_{-q} = H_q e^{iq(pi - phi)}, i.e. e^{i phi} -> -conj(e^{i phi}).
// MIRROR = true computes output slots 2p - [O0, O1] that way.
template <typename T, int p, int O0, int O1, int SPLIT, bool MIRROR>
__device__ __forceinline__ void m2l_body(const cv_t<T> *__restrict__ pairs, const cv_t<T> *__restrict__ beta,
                                         cv_t<T> *__restrict__ part, int n, int m0, int m1, int l) {
  constexpr int P = 2 * p + 1;
  constexpr int NO = O1 - O0 + 1;
  const bool valid = l < n;
  const int lc = valid ? l : n - 1;
  cx<T> acc[NO];
#pragma unroll
  for (int i = 0; i < NO; ++i) acc[i] = mk<T>(0, 0);
  if (m0 < m1) {
    const cv_t<T> *pe = pairs + 4 * (static_cast<int64_t>(m0) * n + lc);
    cv_t<T> a0 = pe[0], a1 = pe[1], a2 = pe[2], a3 = pe[3];
    for (int m = m0; m < m1; ++m) {
      cx<T> h0 = ld<T>(a0), h1 = ld<T>(a1);
      cx<T> t = ld<T>(a2);
      if (MIRROR) t.re = -t.re;
      const T two_over_z = a3.x;
      if (m + 1 < m1) {  // prefetch the next source's pair entry
        pe += 4 * static_cast<int64_t>(n);
        a0 = pe[0];
        a1 = pe[1];
        a2 = pe[2];
        a3 = pe[3];
      }
      if (!valid) h0 = h1 = mk<T>(0, 0);
      const cv_t<T> *bm = beta + static_cast<int64_t>(m) * P;
      if (SPLIT) {  // source coefficients in two halves, one scalar-register set each
        m2l_block<T, p, O0, O1, 0, p, MIRROR>(acc, bm, h0, h1, t, two_over_z);
        __builtin_amdgcn_sched_barrier(0);
        m2l_block<T, p, O0, O1, p + 1, P - 1, MIRROR>(acc, bm, h0, h1, t, two_over_z);
        __builtin_amdgcn_sched_barrier(0);
      } else {
        m2l_block<T, p, O0, O1, 0, P - 1, MIRROR>(acc, bm, h0, h1, t, two_over_z);
      }
    }
  }
  if (valid) {
#pragma unroll
    for (int i = 0; i < NO; ++i) part[static_cast<int64_t>(l) * P + (MIRROR ? 2 * p - O0 - i : O0 + i)] = st(acc[i]);
  }
}

// grid: (target blocks, source chunks); part[chunk][n][P].  Two variants:
//  whole  (HALF = -1): one lane holds all P accumulators of its target;
//  halves (HALF = 0, 1, two launches): output slots [0, p] and, through the
//         mirror identity, [p+1, 2p], at most p+1 accumulators per lane and
//         more waves per SIMD, for twice the recurrence work.  The two halves
//         are separate kernels: in one kernel the compiler merges the bodies
//         and doubles the live registers.
// FP64 always takes the source coefficients in two scalar-register halves.
// The launcher runs the variant the autotuner picked (default: whole).
template <typename T, int p, int HALF>
__global__ __launch_bounds__(kThreads) void k_m2l(const cv_t<T> *__restrict__ pairs,
                                                  const cv_t<T> *__restrict__ beta,
                                                  cv_t<T> *__restrict__ part, int n, int chunk_len,
                                                  int64_t bstride, int64_t pstride) {
  constexpr int P = 2 * p + 1;
  const int l = blockIdx.x * kThreads + threadIdx.x;
  const int c = blockIdx.y;
  beta += blockIdx.z * bstride;  // right-hand side
  part += blockIdx.z * pstride;
  const int m0 = c * chunk_len;
  const int m1 = min(n, m0 + chunk_len);
  cv_t<T> *o = part + static_cast<int64_t>(c) * n * P;
  constexpr int SPLIT = std::is_same<T, double>::value ? 1 : 0;
  if (HALF == 0) m2l_body<T, p, 0, p, SPLIT, false>(pairs, beta, o, n, m0, m1, l);
  else if (HALF == 1) m2l_body<T, p, 0, p - 1, SPLIT, true>(pairs, beta, o, n, m0, m1, l);
  else m2l_body<T, p, 0, P - 1, SPLIT, false>(pairs, beta, o, n, m0, m1, l);
}

// FMM near field: the same pair translation restricted to padded neighbour
// lists.  One lane per target in leaf-box order; each lane walks its own
// list of sources (pair entries [j][i][4] as in the all-pairs table, source
// coefficients loaded per lane), and every wave loops to the longest list
// among its 64 targets (padding entries are zeros).  HALF as in k_m2l: -1
// all outputs; 0 / 1 output slots [0, p] / (mirror) [p+1, 2p] in two
// launches, which keeps FP64 within the register file.
template <typename T, int p, int HALF>
__global__ __launch_bounds__(kThreads) void k_fmm_near(const cv_t<T> *__restrict__ pairs,
                                                       const int *__restrict__ src, const int *__restrict__ perm,
                                                       const int *__restrict__ wave_cnt,
                                                       const cv_t<T> *__restrict__ beta, cv_t<T> *__restrict__ out,
                                                       int n, int kc) {
  constexpr int P = 2 * p + 1;
  const int i = blockIdx.x * kThreads + threadIdx.x;
  // list entries [j_lo, j_hi) of this chunk into partial slot blockIdx.y
  const int kw = __builtin_amdgcn_readfirstlane(wave_cnt[i >> 6]);
  const int j_lo = blockIdx.y * kc, j_hi = min(kw, j_lo + kc);
  out += static_cast<int64_t>(blockIdx.y) * n * P;
  const bool valid = i < n;
  const int ic = valid ? i : n - 1;
  constexpr bool MIRROR = HALF == 1;
  constexpr int O1 = HALF == 0 ? p : (HALF == 1 ? p - 1 : P - 1);  // outputs [0, O1]
  cx<T> acc[O1 + 1];
#pragma unroll
  for (int k = 0; k <= O1; ++k) acc[k] = mk<T>(0, 0);
  constexpr int SPLIT = std::is_same<T, double>::value ? 1 : 0;
  for (int j = j_lo; j < j_hi; ++j) {
    const int64_t e = static_cast<int64_t>(j) * n + ic;
    const cv_t<T> *pe = pairs + 4 * e;
    cx<T> h0 = ld<T>(pe[0]), h1 = ld<T>(pe[1]);
    cx<T> t = ld<T>(pe[2]);
    if (MIRROR) t.re = -t.re;
    const T two_over_z = pe[3].x;
    if (!valid) h0 = h1 = mk<T>(0, 0);
    const cv_t<T> *bm = beta + static_cast<int64_t>(src[e]) * P;
    if (SPLIT) {
      m2l_block<T, p, 0, O1, 0, p, MIRROR>(acc, bm, h0, h1, t, two_over_z);
      __builtin_amdgcn_sched_barrier(0);
      m2l_block<T, p, 0, O1, p + 1, P - 1, MIRROR>(acc, bm, h0, h1, t, two_over_z);
      __builtin_amdgcn_sched_barrier(0);
    } else {
      m2l_block<T, p, 0, O1, 0, P - 1, MIRROR>(acc, bm, h0, h1, t, two_over_z);
    }
  }
  if (valid) {
    const int64_t o = static_cast<int64_t>(perm[i]) * P;
#pragma unroll
    for (int k = 0; k <= O1; ++k) out[o + (MIRROR ? 2 * p - k : k)] = st(acc[k]);
  }
}


template <typename T>
__global__ void k_m2s_reduce(const cv_t<T> *__restrict__ part, int ns, int chunks, int nrhs,
                             double2 *__restrict__ spec) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * ns * nrhs) return;
  const int rs = i / ns, q = i % ns;  // rs = 2 * rhs + side
  double re = 0.0, im = 0.0;
  for (int c = 0; c < chunks; ++c) {
    const cv_t<T> v = part[(static_cast<int64_t>(rs) * chunks + c) * ns + q];
    re += static_cast<double>(v.x);
    im += static_cast<double>(v.y);
  }
  spec[i] = make_double2(re, im);
}

// ---------------------------------------------------------------------------
// Row b2: middle-layer densities per node from the particle spectra and the
// point source:  [s+; s-] = R [P+; P-] + g [f+; f-],  g = e^{-i lam x_s - g1 y_s}.
__global__ void k_reflect(const double2 *__restrict__ spec, const double2 *__restrict__ R,
                          const double2 *__restrict__ sf, const double2 *__restrict__ lam,
                          const double2 *__restrict__ g1, int ns, int has_src, double xs, double ys,
                          double2 *__restrict__ sigma) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ns) return;
  sigma += 2 * static_cast<int64_t>(ns) * blockIdx.y;  // right-hand side
  if (spec) spec += 2 * static_cast<int64_t>(ns) * blockIdx.y;
  cx<double> pp = mk(0.0, 0.0), pm = mk(0.0, 0.0);
  if (spec) {
    pp = ld<double>(spec[q]);
    pm = ld<double>(spec[ns + q]);
  }
  cx<double> sp = ld<double>(R[4 * q + 0]) * pp + ld<double>(R[4 * q + 1]) * pm;
  cx<double> sm = ld<double>(R[4 * q + 2]) * pp + ld<double>(R[4 * q + 3]) * pm;
  if (has_src) {
    const double lr = lam[q].x, li = lam[q].y, gr = g1[q].x, gi = g1[q].y;
    const cx<double> g = cexp_d(li * xs - gr * ys, -lr * xs - gi * ys);
    sp = sp + ld<double>(sf[2 * q + 0]) * g;
    sm = sm + ld<double>(sf[2 * q + 1]) * g;
  }
  sigma[q] = st(sp);
  sigma[ns + q] = st(sm);
}

// S2L coefficient tables: Up[s][q][n] = c_q sigma_s[q] U[s][q][n].
__global__ void k_s2l_coef(const double2 *__restrict__ sigma, const double2 *__restrict__ cq,
                           const double2 *__restrict__ U, int ns, int P, int nrhs, double2 *__restrict__ Up64,
                           float2 *__restrict__ Up32) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  const int64_t per = 2LL * ns * P;
  if (i >= per * nrhs) return;
  const int64_t r = i / per, k = i % per;
  const int s = static_cast<int>(k / (static_cast<int64_t>(ns) * P));
  const int q = static_cast<int>((k / P) % ns);
  const cx<double> v = ld<double>(cq[q]) * ld<double>(sigma[(2 * r + s) * ns + q]) * ld<double>(U[k]);
  Up64[i] = st(v);
  Up32[i] = make_float2(static_cast<float>(v.re), static_cast<float>(v.im));
}


// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_sum_parts(const cv_t<T> *__restrict__ part, int chunks, int64_t len,
                            cv_t<T> *__restrict__ out) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= len) return;
  T re = 0, im = 0;
  for (int c = 0; c < chunks; ++c) {
    const cv_t<T> v = part[c * len + i];
    re += v.x;
    im += v.y;
  }
  cv_t<T> o;
  o.x = re;
  o.y = im;
  out[i] = o;
}

// In-place sum of the partial buffers of each right-hand side into slot 0:
// part[r][0][i] = sum_c part[r][c][i]  (one lane per entry, fixed order).
template <typename T>
__global__ void k_fold_parts(cv_t<T> *__restrict__ part, int chunks, int64_t len, int64_t pstride) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= len) return;
  part += blockIdx.y * pstride;
  // eight independent sums (slot c mod 8), so that eight loads are in flight,
  // combined pairwise at the end: a fixed order for every launch
  T re[8] = {0, 0, 0, 0, 0, 0, 0, 0}, im[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int c = 0;
  for (; c + 8 <= chunks; c += 8) {
    cv_t<T> v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(c + u) * len + i];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      re[u] += v[u].x;
      im[u] += v[u].y;
    }
  }
  for (int u = 0; c < chunks; ++c, ++u) {
    const cv_t<T> v = part[c * len + i];
    re[u] += v.x;
    im[u] += v.y;
  }
  cv_t<T> o;
  o.x = ((re[0] + re[1]) + (re[2] + re[3])) + ((re[4] + re[5]) + (re[6] + re[7]));
  o.y = ((im[0] + im[1]) + (im[2] + im[3])) + ((im[4] + im[5]) + (im[6] + im[7]));
  part[i] = o;
}

// Row a2 on the matrix cores: y^l = x^l - e^{-in psi_l} sum_n' S[n][n'] e^{in' psi_l} alpha^l_{n'},
// alpha one buffer per right-hand side (partials folded first).  One block
// per tile of 16 particles: all lanes rotate the tile's expansions (a
// contiguous range of 16 P entries) into LDS as B[K = n'][N = particle];
// wave w < MT then
// multiplies row tile w of the shared S (A[M = n][K = n'], zero-padded to
// 16 MT x KP) by B with 16x16x4 MFMA, the complex product as four real
// chains (re += Sr Br - Si Bi, im += Sr Bi + Si Br); the result goes back
// through LDS for coalesced stores.
//   (MFMA operand layout: mfma4 in common.h.)
constexpr int kSapplyThreads = 256;

template <typename T, int p>
__global__ __launch_bounds__(kSapplyThreads) void k_sapply(const cv_t<T> *__restrict__ x,
                                                           const cv_t<T> *__restrict__ alpha,
                                                           const cv_t<T> *__restrict__ S,
                                                           const cv_t<T> *__restrict__ rot, int n,
                                                           cv_t<T> *__restrict__ y, int64_t astride,
                                                           const int32_t *__restrict__ types, int ntypes) {
  constexpr int P = 2 * p + 1;
  constexpr int MT = (P + 15) / 16;   // row tiles of S
  constexpr int KP = (P + 3) / 4 * 4; // K padded to the MFMA depth
  static_assert(MT <= kSapplyThreads / 64, "one wave per row tile");
  {  // right-hand side
    const int64_t off = static_cast<int64_t>(blockIdx.y) * n * P;
    if (x) x += off;
    y += off;
    alpha += blockIdx.y * astride;
  }
  __shared__ T Sre[MT * 16][KP], Sim[MT * 16][KP];
  __shared__ T Bre[KP][16], Bim[KP][16];
  __shared__ cx<T> Yt[16 * P];
  __shared__ int32_t tt[16];  // particle types of the tile (-1 past the end)
  const int tid = threadIdx.x;
  const int l0 = blockIdx.x * 16;
  for (int i = tid; i < KP * 16; i += kSapplyThreads) {
    Bre[i / 16][i % 16] = 0;
    Bim[i / 16][i % 16] = 0;
  }
  if (tid < 16) tt[tid] = (l0 + tid < n) ? (types ? types[l0 + tid] : 0) : -1;
  __syncthreads();
  const int cnt = min(16, n - l0) * P;  // entries of the tile
  const int64_t base = static_cast<int64_t>(l0) * P;
  for (int i = tid; i < cnt; i += kSapplyThreads) {
    const cx<T> s = ld<T>(alpha[base + i]) * ld<T>(rot[base + i]);
    Bre[i % P][i / P] = s.re;
    Bim[i % P][i / P] = s.im;
  }
  const int w = tid >> 6, lane = tid & 63;
  const int row = w * 16 + (lane & 15);
  const int col = lane & 15;
  typename mfma4<T>::v4 are = {0, 0, 0, 0}, aim = {0, 0, 0, 0};
  // several particle types: one pass per type present in the tile, with the
  // other columns of B masked out, so each column meets its own matrix
  const int nt = types ? ntypes : 1;
  for (int t = 0; t < nt; ++t) {
    if (types) {
      bool present = false;
      for (int c = 0; c < 16; ++c) present |= (tt[c] == t);
      if (!present) continue;  // uniform over the block
    }
    __syncthreads();  // B written (first pass) or the previous S consumed
    const cv_t<T> *St = S + static_cast<int64_t>(t) * P * P;
    for (int i = tid; i < MT * 16 * KP; i += kSapplyThreads) {
      const int r = i / KP, c = i % KP;
      const cx<T> v = (r < P && c < P) ? ld<T>(St[r * P + c]) : mk<T>(0, 0);
      Sre[r][c] = v.re;
      Sim[r][c] = v.im;
    }
    __syncthreads();
    if (w < MT) {
      const bool on = !types || tt[col] == t;
#pragma unroll
      for (int k0 = 0; k0 < KP; k0 += 4) {
        const int k = k0 + (lane >> 4);
        const T sr = Sre[row][k], si = Sim[row][k];
        const T br = on ? Bre[k][col] : T(0), bi = on ? Bim[k][col] : T(0);
        are = mfma4<T>::mac(sr, br, are);
        are = mfma4<T>::mac(-si, bi, are);
        aim = mfma4<T>::mac(sr, bi, aim);
        aim = mfma4<T>::mac(si, br, aim);
      }
    }
  }
  if (w < MT) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int nn = w * 16 + mfma4<T>::row(lane, j);
      if (nn < P) Yt[col * P + nn] = mk<T>(are[j], aim[j]);
    }
  }
  __syncthreads();
  for (int i = tid; i < cnt; i += kSapplyThreads) {
    cx<T> r = conj(ld<T>(rot[base + i])) * Yt[i];
    if (x) r = ld<T>(x[base + i]) - r;
    y[base + i] = st(r);
  }
}

// ---------------------------------------------------------------------------
// Row b1 on the matrix cores: M2S as a GEMM over the particles of a chunk,
//   G[q][nu] = sum_{m in chunk c} E[s][m][q] beta[m][nu]   (M = node, N = order,
// K = particle), then part[r][s][c][q] = sum_nu W[s][q][nu] G[q][nu] in the
// epilogue (a reduction over the 16 lanes that hold one node's orders).  One
// wave per 16 nodes; lane i supplies A[i % 16][i / 16] = E of node q0 + i % 16
// for particle m0 + i / 16 (16 consecutive nodes: coalesced) and
// B[i / 16][i % 16] = beta of that particle and order.  Complex products take
// three real MFMAs (Gauss: P1 = sum Ar Br, P2 = sum Ai Bi, P3 = sum (Ar + Ai)
// (Br + Bi); re = P1 - P2, im = P3 - P1 - P2).
//
// Orders on the matrix cores and on the vector units: full 16-order tiles go
// to the MFMAs; a remainder of one or two orders (p = 16: 33 = 2 x 16 + 1,
// p = 8: 17 = 16 + 1) is accumulated on the vector units instead of a tile of
// which it would fill at most 2/16; a longer remainder gets a padded tile.
template <int P> struct OrderSplit {
  static constexpr int NF = P / 16;
  static constexpr int REM = P - 16 * NF;
  static constexpr bool VALU_REM = REM > 0 && REM <= 2;
  static constexpr int NT = VALU_REM ? NF : (P + 15) / 16;  // MFMA tiles
  static constexpr int NV = VALU_REM ? REM : 0;             // vector-unit orders, slots 16 NT ..
};

constexpr int kM2sWaves = 4;
template <typename T, int p>
__global__ __launch_bounds__(64 * kM2sWaves) void k_m2s_mfma(const cv_t<T> *__restrict__ E,
                                                             const cv_t<T> *__restrict__ beta,
                                                             const cv_t<T> *__restrict__ W,
                                                             cv_t<T> *__restrict__ part, int n, int ns,
                                                             int chunk_len, int chunks) {
  constexpr int P = 2 * p + 1;
  constexpr int NT = OrderSplit<P>::NT, NV = OrderSplit<P>::NV;
  typedef typename mfma4<T>::v4 v4;
  const int c = blockIdx.y;
  const int s = blockIdx.z & 1;   // side
  const int r = blockIdx.z >> 1;  // right-hand side
  beta += static_cast<int64_t>(r) * n * P;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int q0 = (blockIdx.x * kM2sWaves + w) * 16;
  if (q0 >= ns) return;  // the whole wave lies past the last node (no barriers below)
  const int m0 = c * chunk_len;
  const int m1 = min(n, m0 + chunk_len);
  const int qi = q0 + (lane & 15);
  const int qic = min(qi, ns - 1);
  const int kr = lane >> 4;
  const cv_t<T> *Es = E + static_cast<int64_t>(s) * n * ns;
  v4 P1[NT], P2[NT], P3[NT];
  cx<T> vr[NV > 0 ? NV : 1];
#pragma unroll
  for (int t = 0; t < NT; ++t) P1[t] = P2[t] = P3[t] = v4{0, 0, 0, 0};
#pragma unroll
  for (int v = 0; v < (NV > 0 ? NV : 1); ++v) vr[v] = mk<T>(0, 0);
  if (m0 < m1) {
    // operands of particle group mb (loads clamped into range, zeros selected
    // past the chunk), the next group fetched while the current one multiplies
    struct Ops {
      cv_t<T> a, b[NT], bv[NV > 0 ? NV : 1];
    };
    auto fetch = [&](int mb, Ops &o) {
      const int mc = min(mb + kr, m1 - 1);
      o.a = Es[static_cast<int64_t>(mc) * ns + qic];
#pragma unroll
      for (int t = 0; t < NT; ++t) o.b[t] = beta[static_cast<int64_t>(mc) * P + min(t * 16 + (lane & 15), P - 1)];
#pragma unroll
      for (int v = 0; v < NV; ++v) o.bv[v] = beta[static_cast<int64_t>(mc) * P + 16 * NT + v];
    };
    Ops nx;
    fetch(m0, nx);
    for (int mb = m0; mb < m1; mb += 4) {
      const Ops cu = nx;
      if (mb + 4 < m1) fetch(mb + 4, nx);
      const bool mv = mb + kr < m1;
      const T zr = mv ? cu.a.x : T(0), zi = mv ? cu.a.y : T(0), zs = zr + zi;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const bool cv = t * 16 + (lane & 15) < P;  // padded tile (long remainders only)
        const T br = cv ? cu.b[t].x : T(0), bi = cv ? cu.b[t].y : T(0);
        P1[t] = mfma4<T>::mac(zr, br, P1[t]);
        P2[t] = mfma4<T>::mac(zi, bi, P2[t]);
        P3[t] = mfma4<T>::mac(zs, br + bi, P3[t]);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) cmac(vr[v], mk<T>(zr, zi), ld<T>(cu.bv[v]));
    }
  }
  // vector-unit orders: sum over the four particles of each node (lane
  // groups); lane i then holds node q0 + i % 16
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    vr[v].re += __shfl_xor(vr[v].re, 16);
    vr[v].im += __shfl_xor(vr[v].im, 16);
    vr[v].re += __shfl_xor(vr[v].re, 32);
    vr[v].im += __shfl_xor(vr[v].im, 32);
  }
  // epilogue: contract each node's orders with W, reduce over the 16 lanes
  // holding that node's columns, one lane per node stores
  const cv_t<T> *Ws = W + static_cast<int64_t>(s) * ns * P;
  cv_t<T> *o = part + ((2 * static_cast<int64_t>(r) + s) * chunks + c) * ns;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int row = mfma4<T>::row(lane, j);
    const int q = q0 + row;
    const int qc = min(q, ns - 1);
    cx<T> acc = mk<T>(0, 0);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int col = t * 16 + (lane & 15);
      const T p1 = P1[t][j], p2 = P2[t][j], p3 = P3[t][j];
      if (col < P) cmac(acc, mk<T>(p1 - p2, p3 - p1 - p2), ld<T>(Ws[static_cast<int64_t>(qc) * P + col]));
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) {
      acc.re += __shfl_xor(acc.re, off, 16);
      acc.im += __shfl_xor(acc.im, off, 16);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {  // node q's remainder orders live in lane `row`
      const cx<T> g = mk<T>(__shfl(vr[v].re, row), __shfl(vr[v].im, row));
      cmac(acc, g, ld<T>(Ws[static_cast<int64_t>(qc) * P + 16 * NT + v]));
    }
    if ((lane & 15) == 0 && q < ns) o[q] = st(acc);
  }
}

// ---------------------------------------------------------------------------
// Row b3 on the matrix cores: S2L as a GEMM over the nodes of both interfaces,
//   part[c][l][n] = sum_{side, q in chunk c} F[side][q][l] Up[side][q][n]
// (M = particle, N = order, K = node).  One wave per 16 MT particles (MT
// tiles of 16) and all order tiles; lane i supplies A[i % 16][i / 16] = F of
// particle l0 + 16 t + i % 16 at node q0 + i / 16 (16 consecutive particles
// per node: coalesced) and B[i / 16][i % 16] = the S2L coefficient of that
// node and order, loaded once for the MT particle tiles; complex products
// take three real MFMAs (Gauss), and a remainder of one or two orders runs on
// the vector units (OrderSplit).
constexpr int kS2lWaves = 4;
// particle tiles per wave: two in FP32 (the coefficient loads shared by
// both); one in FP64, where a second tile's accumulators would leave one
// wave per SIMD
template <typename T> constexpr int s2l_tiles() { return sizeof(T) == 4 ? 2 : 1; }
template <typename T, int p, int MT>
__global__ __launch_bounds__(64 * kS2lWaves) void k_s2l_mfma(const cv_t<T> *__restrict__ F,
                                                             const cv_t<T> *__restrict__ Up,
                                                             cv_t<T> *__restrict__ part, int n, int ns,
                                                             int chunk_len, int64_t pstride) {
  constexpr int P = 2 * p + 1;
  constexpr int NT = OrderSplit<P>::NT, NV = OrderSplit<P>::NV;
  typedef typename mfma4<T>::v4 v4;
  Up += 2 * static_cast<int64_t>(ns) * P * blockIdx.z;  // right-hand side
  part += blockIdx.z * pstride;
  const int c = blockIdx.y;
  const int q0 = c * chunk_len;
  const int q1 = min(ns, q0 + chunk_len);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l0 = (blockIdx.x * kS2lWaves + w) * 16 * MT;
  if (l0 >= n) return;  // the whole wave lies past the last particle (no barriers below)
  const int kr = lane >> 4;
  int li[MT];
  bool lv[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    li[m] = l0 + 16 * m + (lane & 15);
    lv[m] = li[m] < n;
  }
  v4 P1[MT][NT], P2[MT][NT], P3[MT][NT];
  cx<T> vr[MT][NV > 0 ? NV : 1];
#pragma unroll
  for (int m = 0; m < MT; ++m) {
#pragma unroll
    for (int t = 0; t < NT; ++t) P1[m][t] = P2[m][t] = P3[m][t] = v4{0, 0, 0, 0};
#pragma unroll
    for (int v = 0; v < (NV > 0 ? NV : 1); ++v) vr[m][v] = mk<T>(0, 0);
  }
  if (q0 < q1) {
    // operands of node group qb (loads clamped into range, zeros selected
    // outside it), the next group fetched while the current one multiplies
    struct Ops {
      cv_t<T> a[MT], b[NT], bv[NV > 0 ? NV : 1];
    };
    auto fetch = [&](int side, int qb, Ops &o) {
      const int q = qb + kr;
      const int qc = min(q, q1 - 1);
      const cv_t<T> *f = F + (side * static_cast<int64_t>(ns) + qc) * n;
#pragma unroll
      for (int m = 0; m < MT; ++m) o.a[m] = f[lv[m] ? li[m] : n - 1];
      const cv_t<T> *u = Up + (side * static_cast<int64_t>(ns) + qc) * P;
#pragma unroll
      for (int t = 0; t < NT; ++t) o.b[t] = u[min(t * 16 + (lane & 15), P - 1)];
#pragma unroll
      for (int v = 0; v < NV; ++v) o.bv[v] = u[16 * NT + v];
    };
    Ops nx;
    fetch(0, q0, nx);
    for (int side = 0, qb = q0; side < 2;) {
      const Ops cu = nx;
      const bool qv = qb + kr < q1;
      int ns_side = side, ns_qb = qb + 4;
      if (ns_qb >= q1) {
        ns_side = side + 1;
        ns_qb = q0;
      }
      if (ns_side < 2) fetch(ns_side, ns_qb, nx);
      T br[NT], bi[NT], bs[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const bool cv = qv && (t * 16 + (lane & 15)) < P;
        br[t] = cv ? cu.b[t].x : T(0);
        bi[t] = cv ? cu.b[t].y : T(0);
        bs[t] = br[t] + bi[t];
      }
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        const T zr = (qv && lv[m]) ? cu.a[m].x : T(0), zi = (qv && lv[m]) ? cu.a[m].y : T(0), zs = zr + zi;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          P1[m][t] = mfma4<T>::mac(zr, br[t], P1[m][t]);
          P2[m][t] = mfma4<T>::mac(zi, bi[t], P2[m][t]);
          P3[m][t] = mfma4<T>::mac(zs, bs[t], P3[m][t]);
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) cmac(vr[m][v], mk<T>(zr, zi), ld<T>(cu.bv[v]));
      }
      side = ns_side;
      qb = ns_qb;
    }
  }
  cv_t<T> *o = part + static_cast<int64_t>(c) * n * P;
#pragma unroll
  for (int m = 0; m < MT; ++m) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int col = t * 16 + (lane & 15);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int l = l0 + 16 * m + mfma4<T>::row(lane, j);
        const T p1 = P1[m][t][j], p2 = P2[m][t][j], p3 = P3[m][t][j];
        if (l < n && col < P) o[static_cast<int64_t>(l) * P + col] = st(mk<T>(p1 - p2, p3 - p1 - p2));
      }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {  // sum over the four node lanes of each particle
      cx<T> z = vr[m][v];
      z.re += __shfl_xor(z.re, 16);
      z.im += __shfl_xor(z.im, 16);
      z.re += __shfl_xor(z.re, 32);
      z.im += __shfl_xor(z.im, 32);
      if (lane < 16 && lv[m]) o[static_cast<int64_t>(li[m]) * P + 16 * NT + v] = st(z);
    }
  }
}

// ---------------------------------------------------------------------------
// Row a1 on the matrix cores, one right-hand side.  The translation
// alpha_{n'} = sum_q h_q beta_{n'+q} (q = nu - n', |q| <= 2p) is a product
// with the source coefficients in shifted form: with A_m[n'][q] = beta_m[n'+q]
// (zero where |n' + q| > p) and B[(m, q)][l] = h_q of the pair (m -> l),
//   alpha_l[n'] = sum_{m, q} A_m[n'][q] B[(m, q)][l],
// a GEMM with M = output orders, N = targets and K = (source, q).  Each
// 16x16x4 MFMA takes four sources at one q: lane i runs the Hankel recurrence
// of the pair (source i / 16 of the group -> target i % 16) and supplies its
// h_q as the B operand; A, the shifted coefficients of one 16-row block of
// output orders, is read from LDS.  Orders n' in [-p, -1] ("lo") and [1, p]
// ("hi") are two 16-row blocks (for p < 16 the rows beyond p compute
// values that are never stored; their reads stay inside the row); n' = 0 is
// accumulated on the vector units and summed over the four sources of a
// group at the end.  q runs from 0 to 2p; h_q and h_{-q} go to the blocks
// whose rows they reach: 96 complex MFMAs per group at p = 16, against the
// 66 that the nonzero band of the 32 block rows needs.  Complex products take three real MFMAs
// (Gauss): P1 = sum Ar Br, P2 = sum Ai Bi, P3 = sum (Ar + Ai)(Br + Bi);
// re = P1 - P2, im = P3 - P1 - P2.  LDS holds the coefficients of
// kM2lMfmaBatch sources of the chunk as (re, im, re + im) with zero padding
// on both sides of every row.  Each wave owns NT tiles of 16 targets (NT = 1
// or 2); the A reads are shared across its tiles.
constexpr int kM2lMfmaWaves = 4;
constexpr int kM2lMfmaBatch = 32;

template <typename T, int p, int NT>
__global__ __launch_bounds__(64 * kM2lMfmaWaves) void k_m2l_mfma(const cv_t<T> *__restrict__ pairs,
                                                                 const cv_t<T> *__restrict__ beta,
                                                                 cv_t<T> *__restrict__ part, int n, int chunk_len,
                                                                 int64_t bstride, int64_t pstride) {
  static_assert(p >= 1 && p <= 16, "one 16-row block per sign of n'");
  constexpr int P = 2 * p + 1;
  constexpr int OFS = p - 1;       // LDS index of coefficient slot s (s >= 1 - p)
  // Row length: slots [1 - p, 2p + 15].  FP32 rows are padded to 16 mod 64
  // words, so that the four source rows one read touches start in different
  // LDS banks (a stride of 0 mod 32 words serialises them four ways).
  constexpr int LR0 = 3 * p + 16;
  constexpr int LR = sizeof(T) == 4 ? LR0 + ((16 - LR0) % 64 + 64) % 64 : LR0;
  constexpr int SB = kM2lMfmaBatch;
  typedef typename mfma4<T>::v4 v4;
  __shared__ T sa[3][SB][LR];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  const int c = blockIdx.y;
  beta += blockIdx.z * bstride;
  part += blockIdx.z * pstride;
  const int m0 = c * chunk_len;
  const int m1 = min(n, m0 + chunk_len);
  const int lt0 = (blockIdx.x * kM2lMfmaWaves + w) * 16 * NT;

  for (int e = threadIdx.x; e < 3 * SB * LR; e += 64 * kM2lMfmaWaves) (&sa[0][0][0])[e] = T(0);

  v4 lo[NT][3], hi[NT][3];
  cx<T> zc[NT];
#pragma unroll
  for (int tt = 0; tt < NT; ++tt) {
#pragma unroll
    for (int k = 0; k < 3; ++k) lo[tt][k] = hi[tt][k] = v4{0, 0, 0, 0};
    zc[tt] = mk<T>(0, 0);
  }
  // pair entries of the first group (source m0 + g)
  cv_t<T> pa[NT][4];
  auto load_pairs = [&](int m) {
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) {
      const int l = lt0 + tt * 16 + r;
      if (m < m1 && l < n) {
        const cv_t<T> *pe = pairs + 4 * (static_cast<int64_t>(m) * n + l);
#pragma unroll
        for (int k = 0; k < 4; ++k) pa[tt][k] = pe[k];
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) pa[tt][k] = st(mk<T>(0, 0));
      }
    }
  };
  load_pairs(m0 + g);

  for (int mb = m0; mb < m1; mb += SB) {
    const int sb = min(SB, m1 - mb);
    __syncthreads();  // previous batch consumed (and the zero fill done)
    for (int e = threadIdx.x; e < SB * P; e += 64 * kM2lMfmaWaves) {
      const int s = e / P, v = e - s * P;
      const cx<T> b = s < sb ? ld<T>(beta[static_cast<int64_t>(mb + s) * P + v]) : mk<T>(0, 0);
      sa[0][s][v + OFS] = b.re;
      sa[1][s][v + OFS] = b.im;
      sa[2][s][v + OFS] = b.re + b.im;
    }
    __syncthreads();
    // a wave whose targets all lie past the last particle (the grid's tail)
    // stages its share of the batch and meets the barriers, but multiplies nothing
    for (int g0 = 0; g0 < sb && lt0 < n; g0 += 4) {
      const int s = g0 + g;  // this lane's source within the batch
      cx<T> hp[NT], hc[NT], t[NT], tq[NT];
      T tz[NT];
#pragma unroll
      for (int tt = 0; tt < NT; ++tt) {
        hp[tt] = ld<T>(pa[tt][0]);
        hc[tt] = ld<T>(pa[tt][1]);
        t[tt] = ld<T>(pa[tt][2]);
        tq[tt] = t[tt];
        tz[tt] = pa[tt][3].x;
      }
      load_pairs(mb + s + 4);  // next group's entries in flight
      const T *ar = sa[0][s], *ai = sa[1][s], *as = sa[2][s];
      // A operands of step q.  lo rows: n' = r - p, coefficient slot r + q
      // (h_q) and r - q (h_{-q}); hi rows: n' = r + 1, slots r + 1 + p + q and
      // r + 1 + p - q; row n' = 0: slots p + q and p - q.
      struct Ops {
        T al[3], ah[3], bl[3], bh[3];
        cx<T> bp, bn;
      };
      auto fetch = [&](int q) {
        Ops o;
        const int il = r + q + OFS, ih = r + 1 + p + q + OFS;
        const int jl = r - q + OFS, jh = r + 1 + p - q + OFS;
        o.al[0] = ar[il], o.al[1] = ai[il], o.al[2] = as[il];
        if (q <= p - 1) o.ah[0] = ar[ih], o.ah[1] = ai[ih], o.ah[2] = as[ih];
        if (q >= 1 && q <= p - 1) o.bl[0] = ar[jl], o.bl[1] = ai[jl], o.bl[2] = as[jl];
        if (q >= 1) o.bh[0] = ar[jh], o.bh[1] = ai[jh], o.bh[2] = as[jh];
        if (q <= p) {
          o.bp = mk<T>(ar[p + q + OFS], ai[p + q + OFS]);
          o.bn = mk<T>(ar[p - q + OFS], ai[p - q + OFS]);
        }
        return o;
      };
      Ops cur = fetch(0);
#pragma unroll
      for (int q = 0; q <= 2 * p; ++q) {
        Ops nxt;
        if (q < 2 * p) nxt = fetch(q + 1);  // the next step's LDS reads in flight
        cx<T> hq[NT], hm[NT];
#pragma unroll
        for (int tt = 0; tt < NT; ++tt) {
          if (q == 0) {
            hq[tt] = hp[tt];  // H_0
          } else {
            if (q >= 2) {
              const cx<T> hn = static_cast<T>(q - 1) * tz[tt] * hc[tt] - hp[tt];
              hp[tt] = hc[tt];
              hc[tt] = hn;
              tq[tt] = tq[tt] * t[tt];
            }
            hq[tt] = hc[tt] * tq[tt];
            hm[tt] = hc[tt] * conj(tq[tt]);
            if (q & 1) hm[tt] = mk<T>(-hm[tt].re, -hm[tt].im);
          }
        }
        // n' = 0 on the vector units: alpha_0 += h_q beta_q + h_{-q} beta_{-q}
        if (q <= p) {
#pragma unroll
          for (int tt = 0; tt < NT; ++tt) cmac(zc[tt], hq[tt], cur.bp);
          if (q > 0) {
#pragma unroll
            for (int tt = 0; tt < NT; ++tt) cmac(zc[tt], hm[tt], cur.bn);
          }
        }
        // the two blocks alternate so that no MFMA waits on the one before it
        const bool lom = q >= 1 && q <= p - 1, hip_ = q <= p - 1, him = q >= 1;
#pragma unroll
        for (int tt = 0; tt < NT; ++tt) {
          const T sq = hq[tt].re + hq[tt].im;
          lo[tt][0] = mfma4<T>::mac(cur.al[0], hq[tt].re, lo[tt][0]);
          if (hip_) hi[tt][0] = mfma4<T>::mac(cur.ah[0], hq[tt].re, hi[tt][0]);
          lo[tt][1] = mfma4<T>::mac(cur.al[1], hq[tt].im, lo[tt][1]);
          if (hip_) hi[tt][1] = mfma4<T>::mac(cur.ah[1], hq[tt].im, hi[tt][1]);
          lo[tt][2] = mfma4<T>::mac(cur.al[2], sq, lo[tt][2]);
          if (hip_) hi[tt][2] = mfma4<T>::mac(cur.ah[2], sq, hi[tt][2]);
          if (q >= 1) {
            const T sm = hm[tt].re + hm[tt].im;
            if (him) hi[tt][0] = mfma4<T>::mac(cur.bh[0], hm[tt].re, hi[tt][0]);
            if (lom) lo[tt][0] = mfma4<T>::mac(cur.bl[0], hm[tt].re, lo[tt][0]);
            if (him) hi[tt][1] = mfma4<T>::mac(cur.bh[1], hm[tt].im, hi[tt][1]);
            if (lom) lo[tt][1] = mfma4<T>::mac(cur.bl[1], hm[tt].im, lo[tt][1]);
            if (him) hi[tt][2] = mfma4<T>::mac(cur.bh[2], sm, hi[tt][2]);
            if (lom) lo[tt][2] = mfma4<T>::mac(cur.bl[2], sm, lo[tt][2]);
          }
        }
        cur = nxt;
        // one q step at a time: keeps the live registers to two steps' operands
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  cv_t<T> *o = part + static_cast<int64_t>(c) * n * P;
#pragma unroll
  for (int tt = 0; tt < NT; ++tt) {
    const int l = lt0 + tt * 16 + r;
    cx<T> z = zc[tt];
    z.re += __shfl_xor(z.re, 16);
    z.im += __shfl_xor(z.im, 16);
    z.re += __shfl_xor(z.re, 32);
    z.im += __shfl_xor(z.im, 32);
    if (l >= n) continue;
    if (g == 0) o[static_cast<int64_t>(l) * P + p] = st(z);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = mfma4<T>::row(lane, j);
      if (row < p) {
        const T p1 = lo[tt][0][j], p2 = lo[tt][1][j], p3 = lo[tt][2][j];
        o[static_cast<int64_t>(l) * P + row] = st(mk<T>(p1 - p2, p3 - p1 - p2));
        const T q1 = hi[tt][0][j], q2 = hi[tt][1][j], q3 = hi[tt][2][j];
        o[static_cast<int64_t>(l) * P + p + 1 + row] = st(mk<T>(q1 - q2, q3 - q1 - q2));
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Row a1 for many right-hand sides on the matrix cores (FP32): per pair the
// Toeplitz translation T^{ml}[n'][nu] = h_{nu-n'} is built once and applied to
// the coefficients of 64 right-hand sides as a GEMM  alpha_l[n'][r] +=
// sum_nu T[n'][nu] beta_m[nu][r]  with 16x16x4 MFMA (M = n', K = nu, N = r),
// complex products in three real MFMAs (Gauss).  One wave per target, kMrhsWaves
// targets per block, grid.y source chunks, grid.z groups of 64 right-hand
// sides.  Lanes 0..7 of each wave run the Hankel recurrences of 8 sources
// at a time (from the pair table, as in k_m2l) into zero-padded LDS rows;
// the A operand is read from there.  The B operand, beta transposed to
// [m][nu][r] (r fastest, zero rows and columns as padding), is staged per
// source in LDS for all waves of the block, double-buffered: the next
// source's loads are in flight during the current source's MFMAs.
constexpr int kMrhsWaves = 8;
constexpr int kMrhsBatch = 8;

template <int p>
__global__ __launch_bounds__(64 * kMrhsWaves) void k_m2l_mrhs(const float2 *__restrict__ pairs,
                                                              const float2 *__restrict__ bt,
                                                              float2 *__restrict__ part, int n, int chunk_len,
                                                              int nrhs, int r_pad, int64_t pstride) {
  constexpr int P = 2 * p + 1;
  constexpr int MT = (P + 15) / 16;
  constexpr int KP = (P + 3) / 4 * 4;
  constexpr int NT = 4;                      // 64 right-hand sides per block
  constexpr int OFF = 16 * MT - 1;           // H index of q = k - row is q + OFF
  constexpr int HQ = KP + OFF;               // zero outside |q| <= 2p
  constexpr int BE = KP * 64;                // B entries of one source
  constexpr int BL = (BE + 64 * kMrhsWaves - 1) / (64 * kMrhsWaves);  // loads per thread
  __shared__ float2 H[kMrhsWaves][kMrhsBatch][HQ];
  __shared__ float2 Bs[2][KP][64];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l = blockIdx.x * kMrhsWaves + w;
  const int c = blockIdx.y;
  const int r0 = blockIdx.z * 64;
  const int m0 = c * chunk_len;
  const int m1 = min(n, m0 + chunk_len);
  typedef float v4 __attribute__((ext_vector_type(4)));
  // Gauss: P1 = sum Ar Br, P2 = sum Ai Bi, P3 = sum (Ar + Ai)(Br + Bi)
  v4 P1[MT][NT], P2[MT][NT], P3[MT][NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int ct = 0; ct < NT; ++ct) P1[mt][ct] = P2[mt][ct] = P3[mt][ct] = v4{0, 0, 0, 0};
  const int col = lane & 15, kq = lane >> 4;
  // B of source m: rows k (zero rows k >= P in bt), 64 right-hand sides
  float2 pre[BL];
  auto load_b = [&](int m) {
#pragma unroll
    for (int i = 0; i < BL; ++i) {
      const int e = threadIdx.x + 64 * kMrhsWaves * i;
      pre[i] = (m < m1 && e < BE) ? bt[(static_cast<int64_t>(m) * KP + e / 64) * r_pad + r0 + (e & 63)]
                                  : make_float2(0.f, 0.f);
    }
  };
  auto store_b = [&](int buf) {
#pragma unroll
    for (int i = 0; i < BL; ++i) {
      const int e = threadIdx.x + 64 * kMrhsWaves * i;
      if (e < BE) Bs[buf][e / 64][e & 63] = pre[i];
    }
  };
  load_b(m0);
  int it = 0;
  for (int mb = m0; mb < m1; mb += kMrhsBatch) {
    const int sb = min(kMrhsBatch, m1 - mb);
    for (int i = lane; i < kMrhsBatch * HQ; i += 64) H[w][i / HQ][i % HQ] = make_float2(0.f, 0.f);
    __syncthreads();
    if (lane < sb) {  // h_q of pair (mb + lane -> l), q = -2p..2p
      const int m = mb + lane;
      float2 *h = H[w][lane] + OFF;
      if (l < n && m != l) {
        const float2 *pe = pairs + 4 * (static_cast<int64_t>(m) * n + l);
        cx<float> hp = ld<float>(pe[0]), hc = ld<float>(pe[1]);
        const cx<float> t = ld<float>(pe[2]);
        const float tz = pe[3].x;
        h[0] = st(hp);
        cx<float> tq = t;
        for (int q = 1; q <= 2 * p; ++q) {
          if (q >= 2) {
            const cx<float> hn = static_cast<float>(q - 1) * tz * hc - hp;
            hp = hc;
            hc = hn;
            tq = tq * t;
          }
          h[q] = st(hc * tq);
          cx<float> hm = hc * conj(tq);
          if (q & 1) hm = mk<float>(-hm.re, -hm.im);
          h[-q] = st(hm);
        }
      }
    }
    for (int s = 0; s < sb; ++s, ++it) {
      const int buf = it & 1;
      store_b(buf);          // B of source mb + s (loaded one iteration ahead)
      __syncthreads();
      load_b(mb + s + 1);    // next source's B in flight during the MFMAs
      const float2 *hrow = H[w][s];
#pragma unroll
      for (int k0 = 0; k0 < KP; k0 += 4) {
        const int k = k0 + kq;
        float br[NT], bi[NT], bs[NT];
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) {
          const float2 bv = Bs[buf][k][ct * 16 + col];
          br[ct] = bv.x;
          bi[ct] = bv.y;
          bs[ct] = bv.x + bv.y;
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const float2 a = hrow[k - (mt * 16 + col) + OFF];
          const float as = a.x + a.y;
#pragma unroll
          for (int ct = 0; ct < NT; ++ct) {
            P1[mt][ct] = mfma4<float>::mac(a.x, br[ct], P1[mt][ct]);
            P2[mt][ct] = mfma4<float>::mac(a.y, bi[ct], P2[mt][ct]);
            P3[mt][ct] = mfma4<float>::mac(as, bs[ct], P3[mt][ct]);
          }
        }
      }
    }
    __syncthreads();
  }
  if (l >= n) return;
  // result register j of lane i: row 4 (i / 16) + j, column i % 16
  const int64_t len = static_cast<int64_t>(n) * P;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int ct = 0; ct < NT; ++ct)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = mt * 16 + 4 * kq + j;
        const int r = r0 + ct * 16 + col;
        const float p1 = P1[mt][ct][j], p2 = P2[mt][ct][j], p3 = P3[mt][ct][j];
        if (row < P && r < nrhs)
          part[r * pstride + c * len + static_cast<int64_t>(l) * P + row] = make_float2(p1 - p2, p3 - p1 - p2);
      }
}

// beta [r][m][P] -> bt [m][KP][r_pad] (r fastest; zero rows k >= P and
// zero columns r >= nrhs), FP32.
__global__ void k_rhs_transpose(const float2 *__restrict__ x, float2 *__restrict__ bt, int n, int P, int KP,
                                int nrhs, int r_pad) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  const int64_t rows = static_cast<int64_t>(n) * KP;
  if (i >= rows * r_pad) return;
  const int64_t row = i / r_pad;
  const int r = static_cast<int>(i % r_pad);
  const int m = static_cast<int>(row / KP), k = static_cast<int>(row % KP);
  bt[i] = (r < nrhs && k < P) ? x[r * static_cast<int64_t>(n) * P + static_cast<int64_t>(m) * P + k]
                              : make_float2(0.f, 0.f);
}

// ---------------------------------------------------------------------------
// GMRES helpers, FP64 complex.
constexpr int kDotBlocks = 64;
constexpr int kRed = 256;

// V holds the basis in FP64 (double2) or, for the mixed-precision solve, FP32
// (float2); products and sums are FP64 either way.  Each block takes one
// slice of w and kDotVecs basis vectors, so every w element is loaded once
// for kDotVecs products (w would otherwise be re-read from L2 once per
// vector: at a basis of several hundred vectors that traffic exceeded V's).
// Sums: per thread, then across the wave by xor shuffles, then the four
// waves in order (deterministic).
constexpr int kDotVecs = 8;
template <typename TV>
__global__ __launch_bounds__(kRed) void k_dotc_part(const TV *__restrict__ V, int64_t ld_v, int k,
                                                    const double2 *__restrict__ w, int64_t len,
                                                    double2 *__restrict__ part, const int32_t *__restrict__ skip) {
  if (skip && *skip) return;  // the pass is not needed (k_dotc_final writes zeros)
  const int j0 = blockIdx.y * kDotVecs;
  const int nv = min(kDotVecs, k - j0);
  const int b = blockIdx.x;
  double re[kDotVecs], im[kDotVecs];
#pragma unroll
  for (int u = 0; u < kDotVecs; ++u) re[u] = im[u] = 0.0;
  for (int64_t i = b * static_cast<int64_t>(kRed) + threadIdx.x; i < len;
       i += static_cast<int64_t>(kRed) * gridDim.x) {
    const double2 c = w[i];
#pragma unroll
    for (int u = 0; u < kDotVecs; ++u) {
      if (u < nv) {
        const TV a = V[(j0 + u) * ld_v + i];
        const double ax = a.x, ay = a.y;
        re[u] += ax * c.x + ay * c.y;
        im[u] += ax * c.y - ay * c.x;
      }
    }
  }
  __shared__ double sr[kRed / 64][kDotVecs], si[kRed / 64][kDotVecs];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int u = 0; u < kDotVecs; ++u) {
    double r = re[u], m = im[u];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      r += __shfl_xor(r, o);
      m += __shfl_xor(m, o);
    }
    if (lane == 0) {
      sr[wv][u] = r;
      si[wv][u] = m;
    }
  }
  __syncthreads();
  if (threadIdx.x < nv) {
    const int u = threadIdx.x;
    double r = 0.0, m = 0.0;
#pragma unroll
    for (int v = 0; v < kRed / 64; ++v) {
      r += sr[v][u];
      m += si[v][u];
    }
    part[(j0 + u) * gridDim.x + b] = make_double2(r, m);
  }
}

__global__ void k_dotc_final(const double2 *__restrict__ part, int k, int nb, double2 *__restrict__ h,
                             const int32_t *__restrict__ skip) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  if (skip && *skip) {
    h[j] = make_double2(0.0, 0.0);
    return;
  }
  double re = 0.0, im = 0.0;
  for (int b = 0; b < nb; ++b) {
    re += part[j * nb + b].x;
    im += part[j * nb + b].y;
  }
  h[j] = make_double2(re, im);
}

template <typename TV>
__global__ void k_gemv_sub(const TV *__restrict__ V, int64_t ld_v, int k,
                           const double2 *__restrict__ h, double2 *__restrict__ w, int64_t len,
                           const int32_t *__restrict__ skip) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= len || (skip && *skip)) return;
  cx<double> acc = ld<double>(w[i]);
  int j = 0;
  for (; j + 8 <= k; j += 8) {  // eight loads in flight per lane
    TV a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = V[(j + u) * ld_v + i];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = acc - mk<double>(a[u].x, a[u].y) * ld<double>(h[j + u]);
  }
  for (; j < k; ++j) {
    const TV a = V[j * ld_v + i];
    acc = acc - mk<double>(a.x, a.y) * ld<double>(h[j]);
  }
  w[i] = st(acc);
}

// Second Gram-Schmidt pass only when the first cancelled much of the vector
// (Daniel, Gragg, Kaufman and Stewart): skip = ||w after||^2 >= eta2 ||w before||^2.
__global__ void k_reorth_flag(const double2 *__restrict__ before, const double2 *__restrict__ after, double eta2,
                              int32_t *__restrict__ skip) {
  if (threadIdx.x == 0 && blockIdx.x == 0) skip[0] = after->x >= eta2 * before->x ? 1 : 0;
}

__global__ __launch_bounds__(kRed) void k_proj_fix(double2 *__restrict__ h, const double2 *__restrict__ q, int k) {
  __shared__ double sr[kRed], si[kRed];
  double re = 0.0, im = 0.0;
  for (int i = threadIdx.x; i < k; i += kRed) {  // q^H h
    re += q[i].x * h[i].x + q[i].y * h[i].y;
    im += q[i].x * h[i].y - q[i].y * h[i].x;
  }
  sr[threadIdx.x] = re;
  si[threadIdx.x] = im;
  __syncthreads();
  for (int o = kRed / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      sr[threadIdx.x] += sr[threadIdx.x + o];
      si[threadIdx.x] += si[threadIdx.x + o];
    }
    __syncthreads();
  }
  const double ar = sr[0], ai = si[0];
  for (int i = threadIdx.x; i < k; i += kRed) {
    const double2 qi = q[i];
    h[i].x -= qi.x * ar - qi.y * ai;
    h[i].y -= qi.x * ai + qi.y * ar;
  }
}

__global__ void k_scale_to32(float2 *__restrict__ v, const double2 *__restrict__ src, int64_t len, double s) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= len) return;
  const double2 a = src[i];
  v[i] = make_float2(static_cast<float>(s * a.x), static_cast<float>(s * a.y));
}

__global__ void k_scale(double2 *__restrict__ v, const double2 *__restrict__ src, int64_t len, double s) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= len) return;
  const double2 a = src[i];
  v[i] = make_double2(s * a.x, s * a.y);
}

__global__ void k_axpy_c(double2 *__restrict__ y, const double2 *__restrict__ x, int64_t len,
                         double ar, double ai) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= len) return;
  const cx<double> r = ld<double>(y[i]) + mk(ar, ai) * ld<double>(x[i]);
  y[i] = st(r);
}

// Deterministic pseudo-random fill in [-1, 1) (tuning input with realistic
// operand switching; zero operands run faster and mislead the tuner).
__global__ void k_fill_hash(double *__restrict__ v, int64_t len, uint32_t seed) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= len) return;
  uint32_t h = static_cast<uint32_t>(i) * 2654435761u ^ seed;
  h ^= h >> 16;
  h *= 2246822519u;
  h ^= h >> 13;
  h *= 3266489917u;
  h ^= h >> 16;
  v[i] = static_cast<double>(h) * (2.0 / 4294967296.0) - 1.0;
}
__global__ void k_fill_hash32(float *__restrict__ v, int64_t len, uint32_t seed) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= len) return;
  uint32_t h = static_cast<uint32_t>(i) * 2654435761u ^ seed;
  h ^= h >> 16;
  h *= 2246822519u;
  h ^= h >> 13;
  h *= 3266489917u;
  h ^= h >> 16;
  v[i] = static_cast<float>(static_cast<double>(h) * (2.0 / 4294967296.0) - 1.0);
}

__global__ void k_to32(const double2 *__restrict__ a, float2 *__restrict__ b, int64_t len) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i < len) b[i] = make_float2(static_cast<float>(a[i].x), static_cast<float>(a[i].y));
}
__global__ void k_to64(const float2 *__restrict__ a, double2 *__restrict__ b, int64_t len) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i < len) b[i] = make_double2(static_cast<double>(a[i].x), static_cast<double>(a[i].y));
}

// ---------------------------------------------------------------------------
// Row a7: total field at receivers (eq. (36)), FP64.
__global__ void k_field(const double2 *__restrict__ xy, const double2 *__restrict__ beta, int n, int p,
                        const double2 *__restrict__ lam, const double2 *__restrict__ w,
                        const double2 *__restrict__ gl, const double2 *__restrict__ amp,
                        const double *__restrict__ yint, int L, int c, int ns, double k0, double kc, double r_enc,
                        const int32_t *__restrict__ types, const double *__restrict__ rtype, double xs, double ys,
                        const double2 *__restrict__ rcv, int64_t nr, double2 *__restrict__ u) {
  const int64_t r = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (r >= nr) return;
  const double X = rcv[r].x, Y = rcv[r].y;
  // layer of the receiver: interfaces above it; the particle layer keeps y = 0
  int layer = 0;
  for (int i = 0; i < L - 1; ++i) layer += (Y < yint[i]) ? 1 : 0;
  if (Y == yint[c - 1]) layer = c;
  const bool hasA = layer > 0, hasB = layer < L - 1;
  const double ta = hasA ? Y - yint[layer - 1] : 0.0;  // <= 0
  const double tb = hasB ? Y - yint[layer] : 0.0;      // >= 0
  const double2 *g = gl + static_cast<int64_t>(layer) * ns;
  const double2 *A = amp + static_cast<int64_t>(2 * layer) * ns;
  const double2 *B = A + ns;
  cx<double> acc = mk(0.0, 0.0);
  for (int q = 0; q < ns; ++q) {
    const double lr = lam[q].x, li = lam[q].y;
    const cx<double> gq = ld<double>(g[q]);
    cx<double> s = mk(0.0, 0.0);
    if (hasA) s = s + ld<double>(A[q]) * cexp_d(-li * X + gq.re * ta, lr * X + gq.im * ta);
    if (hasB) s = s + ld<double>(B[q]) * cexp_d(-li * X - gq.re * tb, lr * X - gq.im * tb);
    const double nn = gq.re * gq.re + gq.im * gq.im;
    acc = acc + (1.0 / nn) * (ld<double>(w[q]) * mk(gq.re, -gq.im) * s);
  }
  acc = (1.0 / (4.0 * M_PI)) * acc;
  bool inside = false;
  if (layer == 0) {
    const double dx = X - xs, dy = Y - ys;
    const double z = k0 * sqrt(dx * dx + dy * dy);
    acc = acc + mk(0.0, 0.25) * mk(j0(z), y0(z));
  } else if (layer == c) {
    const int P = 2 * p + 1;
    for (int m = 0; m < n; ++m) {
      const double dx = X - xy[m].x, dy = Y - xy[m].y;
      const double rr = sqrt(dx * dx + dy * dy);
      if (rr < (types ? rtype[types[m]] : r_enc)) inside = true;
      const double z = kc * rr;
      const cx<double> t = mk(dx / rr, dy / rr);
      const double2 *b = beta + static_cast<int64_t>(m) * P;
      cx<double> hprev = mk(j0(z), y0(z));
      cx<double> hcur = mk(j1(z), y1(z));
      acc = acc + hprev * ld<double>(b[p]);
      cx<double> tq = t;
      for (int q = 1; q <= p; ++q) {
        if (q >= 2) {
          const cx<double> hn = (2.0 * (q - 1) / z) * hcur - hprev;
          hprev = hcur;
          hcur = hn;
          tq = tq * t;
        }
        const double sg = (q & 1) ? -1.0 : 1.0;
        acc = acc + hcur * (tq * ld<double>(b[p + q]) + sg * (conj(tq) * ld<double>(b[p - q])));
      }
    }
  }
  if (inside) acc = mk<double>(NAN, NAN);
  u[r] = st(acc);
}

// ---------------------------------------------------------------------------
// Dispatch over the expansion order.
#define MPSL_P_CASES(X) \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) \
  X(18) X(19) X(20)

}  // namespace

int m2l_default_variant(int p, int prec) {
  // measured crossovers at 5000 particles: the matrix-core form wins from
  // p = 12 in FP32 and at p = 16 in FP64 (its FP64 MFMA rate equals the vector
  // rate, so only the larger translations gain)
  const int from = prec == MPSL_FP64 ? 15 : 12;
  return (p >= from && p <= kM2LMfmaMaxP) ? kM2LMfma : kM2LWhole;
}

static int m2l_variant(const mpsl_ctx *ctx, int prec) {
  int v = ctx->tune[prec == MPSL_FP64 ? 0 : 1].variant;
  if (v < 0) v = m2l_default_variant(ctx->p, prec);
  if (v >= kM2LMfma && ctx->p > kM2LMfmaMaxP) v = kM2LWhole;
  return v;
}

int chunks_m2l(const mpsl_ctx *ctx, int prec) {
  const int tuned = ctx->tune[prec == MPSL_FP64 ? 0 : 1].chunks;
  if (tuned > 0) return static_cast<int>(std::min<int64_t>(tuned, ctx->n));
  if (ctx->m2l_chunks > 0) return static_cast<int>(std::min<int64_t>(ctx->m2l_chunks, ctx->n));
  // about 2560 blocks of 128 lanes, or 10240 of 4 waves on the matrix cores
  const int v = m2l_variant(ctx, prec);
  int c = v >= kM2LMfma ? cdiv(10240, cdiv(ctx->n, 64 * (v == kM2LMfmaWide ? 2 : 1)))
                        : cdiv(2560, cdiv(ctx->n, kThreads));
  c = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(c, ctx->n)));
  // matrix cores: chunks of whole groups of four sources (m2l_mfma_chunk_len),
  // counted so that none is empty
  if (v >= kM2LMfma) c = cdiv(ctx->n, m2l_mfma_chunk_len(static_cast<int>(ctx->n), c));
  return c;
}

// Chunk count for a launch of bpc blocks per chunk whose blocks all carry the
// same work.  With `slots` blocks resident at once on the whole chip
// (compute units x blocks per unit), B blocks run in ceil(B / slots) waves,
// and each block holds 1/c of the work, so the launch takes about
// ceil(bpc c / slots) / c; of the counts in [lo, hi] the smallest within 3 %
// of the best is taken (fewer partial slots to sum).  At 5000 particles and
// 26816 nodes the FP32 S2L's 26 chunks made 1040 blocks for 1024 slots, a
// second wave of 16 blocks (0.82 ms; 50 chunks, 2000 blocks: about 0.63 ms).
static int balanced_chunks(int64_t bpc, int64_t slots, int lo, int hi) {
  lo = std::max(1, lo);
  hi = std::max(lo, hi);
  slots = std::max<int64_t>(1, slots);
  auto cost = [&](int c) { return static_cast<double>((bpc * c + slots - 1) / slots) / c; };
  double best = 1e300;
  for (int c = lo; c <= hi; ++c) best = std::min(best, cost(c));
  for (int c = lo; c <= hi; ++c)
    if (cost(c) <= 1.03 * best) return c;
  return lo;
}

// Blocks of the matrix-core S2L kernel resident per compute unit (occupancy
// query, cached per precision and order; 1 if the query fails).
template <typename T>
static int s2l_resident(int p) {
  static std::atomic<int> cache[kMaxP + 1];
  if (p < kMinP || p > kMaxP) return 1;
  int r = cache[p].load(std::memory_order_relaxed);
  if (r > 0) return r;
  constexpr int MT = s2l_tiles<T>();
  const void *fn = nullptr;
  switch (p) {
#define X(PP) \
  case PP: fn = reinterpret_cast<const void *>(&k_s2l_mfma<T, PP, MT>); break;
    MPSL_P_CASES(X)
#undef X
  }
  int nb = 0;
  if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 64 * kS2lWaves, 0) != hipSuccess || nb < 1) {
    (void)hipGetLastError();
    nb = 1;
  }
  cache[p].store(nb, std::memory_order_relaxed);
  return nb;
}

int chunks_s2l(const mpsl_ctx *ctx, int nrhs, int prec) {
  if (ctx->somm.active) {  // the interpolated S2L: chunks of coarse nodes, one slot each
    const int tb = cdiv(ctx->n, 128) * nrhs;
    return std::max(1, std::min(64, std::min(cdiv(1024, tb), 2 * ctx->somm.nc)));
  }
  if (ctx->s2l_chunks > 0) return std::min(ctx->s2l_chunks, ctx->ns);
  // about 1024 blocks of 128 lanes' worth of particles, at least 8 nodes per
  // chunk; on long contours raised by up to 2x to fill the last wave of
  // blocks (fewer chunks would enlarge the coefficient rows that the resident
  // blocks read at once: at 26816 nodes 19 FP64 chunks ran slower than 26,
  // 29 faster).  Short contours keep it: each chunk adds a partial slot of n P
  // entries to write and sum, about what the better fill gains at 1024 nodes.
  const int tb = cdiv(ctx->n, kThreads) * nrhs;
  const int cmax = std::max(1, ctx->ns / 8);
  const int c0 = std::min(cdiv(1024, tb), cmax);
  if (ctx->ns < 4096) return std::max(1, c0);
  const bool f64 = prec == MPSL_FP64;
  const int64_t bpc =
      static_cast<int64_t>(cdiv(ctx->n, 16 * kS2lWaves * (f64 ? s2l_tiles<double>() : s2l_tiles<float>()))) * nrhs;
  const int64_t slots = static_cast<int64_t>(ctx->n_cu) * (f64 ? s2l_resident<double>(ctx->p) : s2l_resident<float>(ctx->p));
  return balanced_chunks(bpc, slots, std::max(1, c0), std::min(2 * c0, cmax));
}

// Blocks of the matrix-core M2S kernel resident per compute unit (occupancy
// query, cached per precision and order; 1 if the query fails).
template <typename T>
static int m2s_resident(int p) {
  static std::atomic<int> cache[kMaxP + 1];
  if (p < kMinP || p > kMaxP) return 1;
  int r = cache[p].load(std::memory_order_relaxed);
  if (r > 0) return r;
  const void *fn = nullptr;
  switch (p) {
#define X(PP) \
  case PP: fn = reinterpret_cast<const void *>(&k_m2s_mfma<T, PP>); break;
    MPSL_P_CASES(X)
#undef X
  }
  int nb = 0;
  if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 64 * kM2sWaves, 0) != hipSuccess || nb < 1) {
    (void)hipGetLastError();
    nb = 1;
  }
  cache[p].store(nb, std::memory_order_relaxed);
  return nb;
}

int chunks_m2s(const mpsl_ctx *ctx, int nrhs, int prec) {
  if (ctx->m2s_chunks > 0) return static_cast<int>(std::min<int64_t>(ctx->m2s_chunks, ctx->n));
  // about 2048 node-group x chunk tasks, but at least 80 particles per chunk:
  // shorter chunks spend more on the epilogue and on summing the partials
  // than they gain in parallelism (1024 nodes, 5000 particles: 256 -> 63
  // chunks, M2S and partial sum 75 -> about 45 us in FP32)
  const int qb = cdiv(ctx->ns, kThreads) * 2 * nrhs;
  const int c0 = static_cast<int>(std::max<int64_t>(
      1, std::min<int64_t>(std::min<int64_t>(cdiv(2048, qb), cdiv(ctx->n, 80)), ctx->n)));
  // short contours: lowered by up to half to the count whose blocks fill
  // whole waves of the resident slots (1024 nodes, 5000 particles: 63 chunks
  // made 2016 blocks for 1792 FP32 slots; 55 make 1760).  Long contours run
  // many waves already and keep it (3 to 20 chunks within 0.5 % at 26816 nodes).
  if (ctx->ns >= 4096) return c0;
  const bool f64 = prec == MPSL_FP64;
  const int64_t bpc = static_cast<int64_t>(cdiv(ctx->ns, 16 * kM2sWaves)) * 2 * nrhs;
  const int64_t slots = static_cast<int64_t>(ctx->n_cu) * (f64 ? m2s_resident<double>(ctx->p) : m2s_resident<float>(ctx->p));
  return balanced_chunks(bpc, slots, std::max(1, c0 / 2), c0);
}

#define LAUNCH_CHECK(ctx)                                                          \
  do {                                                                             \
    hipError_t e_ = hipGetLastError();                                             \
    if (e_ != hipSuccess) return set_err(ctx, MPSL_EHIP, std::string("kernel launch: ") + hipGetErrorString(e_)); \
  } while (0)

int launch_geom_tables(mpsl_ctx *ctx) {
  const int64_t tot = ctx->n * static_cast<int64_t>(ctx->ns);
  const int threads = 256;
  hipLaunchKernelGGL(k_geom_tables, dim3(cdiv(tot, threads)), dim3(threads), 0, ctx->stream,
                     static_cast<const double2 *>(ctx->gt.xy.p), static_cast<const double2 *>(ctx->ct.lam.p),
                     static_cast<const double2 *>(ctx->ct.gw.p) + ctx->ns,  // g2 stored after g1
                     static_cast<int>(ctx->n), ctx->ns, ctx->d, static_cast<double2 *>(ctx->gt.E64.p),
                     static_cast<double2 *>(ctx->gt.F64.p), static_cast<float2 *>(ctx->gt.E32.p),
                     static_cast<float2 *>(ctx->gt.F32.p));
  LAUNCH_CHECK(ctx);
  return MPSL_OK;
}

int launch_pair_tables(mpsl_ctx *ctx) {
  const int64_t tot = ctx->n * ctx->n;
  hipLaunchKernelGGL(k_pair_tables, dim3(cdiv(tot, 256)), dim3(256), 0, ctx->stream,
                     static_cast<const double2 *>(ctx->gt.xy.p), static_cast<int>(ctx->n), ctx->k2.real(),
                     static_cast<double2 *>(ctx->gt.pair64.p), static_cast<float2 *>(ctx->gt.pair32.p));
  LAUNCH_CHECK(ctx);
  return MPSL_OK;
}

// Sources per chunk of the matrix-core M2L: each MFMA step takes a group of
// four sources, so a chunk length that is not a multiple of 4 leaves a part
// of one group's matrix work on zeros in every chunk (39 sources: 2.5 %
// of the launch at 5000 particles); trailing chunks may come out empty and
// then write zero partials.
int m2l_mfma_chunk_len(int n, int chunks) { return (cdiv(n, chunks) + 3) / 4 * 4; }

template <typename T>
static int launch_m2l_t(mpsl_ctx *ctx, const void *beta, void *part, int chunks, int variant, int nrhs,
                        int64_t pstride) {
  const int n = static_cast<int>(ctx->n);
  const int chunk_len = cdiv(n, chunks);
  const bool f64 = std::is_same<T, double>::value;
  const dim3 grid(cdiv(n, kThreads), chunks, nrhs);
  const auto *pairs = static_cast<const cv_t<T> *>(f64 ? ctx->gt.pair64.p : ctx->gt.pair32.p);
  const auto *b = static_cast<const cv_t<T> *>(beta);
  auto *o = static_cast<cv_t<T> *>(part);
  const int64_t bs = ctx->n * static_cast<int64_t>(2 * ctx->p + 1);
  if (variant == kM2LMfma || variant == kM2LMfmaWide) {
    if (ctx->p > kM2LMfmaMaxP) return set_err(ctx, MPSL_EUNSUPPORTED, "matrix-core M2L needs p <= 16");
    const int nt = variant == kM2LMfma ? 1 : 2;
    const dim3 g(cdiv(n, 16 * nt * kM2lMfmaWaves), chunks, nrhs);
    const dim3 blk(64 * kM2lMfmaWaves);
    const int cl = m2l_mfma_chunk_len(n, chunks);
    switch (ctx->p) {
#define X(PP)                                                                                               \
  case PP:                                                                                                  \
    if constexpr (PP <= kM2LMfmaMaxP) {                                                                     \
      if (nt == 1)                                                                                          \
        hipLaunchKernelGGL((k_m2l_mfma<T, PP, 1>), g, blk, 0, ctx->stream, pairs, b, o, n, cl, bs, pstride); \
      else                                                                                                  \
        hipLaunchKernelGGL((k_m2l_mfma<T, PP, 2>), g, blk, 0, ctx->stream, pairs, b, o, n, cl, bs, pstride); \
    }                                                                                                       \
    break;
      MPSL_P_CASES(X)
#undef X
      default: return set_err(ctx, MPSL_EUNSUPPORTED, "expansion order outside 1..20");
    }
    LAUNCH_CHECK(ctx);
    return MPSL_OK;
  }
  switch (ctx->p) {
#define X(PP)                                                                                               \
  case PP:                                                                                                  \
    if (variant == kM2LHalves) {                                                                            \
      hipLaunchKernelGGL((k_m2l<T, PP, 0>), grid, dim3(kThreads), 0, ctx->stream, pairs, b, o, n, chunk_len, \
                         bs, pstride);                                                                      \
      hipLaunchKernelGGL((k_m2l<T, PP, 1>), grid, dim3(kThreads), 0, ctx->stream, pairs, b, o, n, chunk_len, \
                         bs, pstride);                                                                      \
    } else {                                                                                                \
      hipLaunchKernelGGL((k_m2l<T, PP, -1>), grid, dim3(kThreads), 0, ctx->stream, pairs, b, o, n,           \
                         chunk_len, bs, pstride);                                                           \
    }                                                                                                       \
    break;
    MPSL_P_CASES(X)
#undef X
    default: return set_err(ctx, MPSL_EUNSUPPORTED, "expansion order outside 1..20");
  }
  LAUNCH_CHECK(ctx);
  return MPSL_OK;
}

int launch_m2l(mpsl_ctx *ctx, int prec, const void *beta, void *part, int chunks, int variant, int nrhs,
               int64_t pstride) {
  if (variant < 0) variant = m2l_variant(ctx, prec);  // tuned or default; matrix cores up to p = 16
  return prec == MPSL_FP64 ? launch_m2l_t<double>(ctx, beta, part, chunks, variant, nrhs, pstride)
                           : launch_m2l_t<float>(ctx, beta, part, chunks, variant, nrhs, pstride);
}

int chunks_m2l_mrhs(const mpsl_ctx *ctx, int nrhs) {
  const int64_t blocks = static_cast<int64_t>(cdiv(ctx->n, kMrhsWaves)) * cdiv(nrhs, 64);
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(cdiv(1024, blocks), cdiv(ctx->n, kMrhsBatch))));
}

int launch_m2l_mrhs(mpsl_ctx *ctx, const void *beta, void *part, int chunks, int nrhs, int64_t pstride) {
  const int n = static_cast<int>(ctx->n);
  const int P = 2 * ctx->p + 1;
  const int KP = (P + 3) / 4 * 4;
  const int64_t rows = static_cast<int64_t>(n) * KP;
  const int r_pad = 64 * cdiv(nrhs, 64);
  int rc = dev_alloc(ctx, ctx->bt, static_cast<size_t>(rows) * r_pad * sizeof(float2));
  if (rc) return rc;
  hipLaunchKernelGGL(k_rhs_transpose, dim3(cdiv(rows * r_pad, 256)), dim3(256), 0, ctx->stream,
                     static_cast<const float2 *>(beta), static_cast<float2 *>(ctx->bt.p), n, P, KP, nrhs, r_pad);
  LAUNCH_CHECK(ctx);
  const int chunk_len = cdiv(n, chunks);
  const dim3 grid(cdiv(n, kMrhsWaves), chunks, r_pad / 64);
  const auto *pairs = static_cast<const float2 *>(ctx->gt.pair32.p);
  const auto *bt = static_cast<const float2 *>(ctx->bt.p);
  auto *pp = static_cast<float2 *>(part);
  switch (ctx->p) {
#define X(PP) \
  case PP: hipLaunchKernelGGL((k_m2l_mrhs<PP>), grid, dim3(64 * kMrhsWaves), 0, ctx->stream, pairs, bt, pp, n, chunk_len, nrhs, r_pad, pstride); break;
    MPSL_P_CASES(X)
#undef X
    default: return set_err(ctx, MPSL_EUNSUPPORTED, "expansion order outside 1..20");
  }
  LAUNCH_CHECK(ctx);
  return MPSL_OK;
}

template <typename T>
static int launch_fmm_near_t(mpsl_ctx *ctx, const void *beta, void *out) {
  const FmmPlan &f = ctx->fmm;
  const int n = static_cast<int>(ctx->n);
  const bool f64 = std::is_same<T, double>::value;
  const auto *pairs = static_cast<const cv_t<T> *>(f64 ? f.near64.p : f.near32.p);
  const auto *src = static_cast<const int *>(f.near_src.p);
  const auto *perm = static_cast<const int *>(f.perm.p);
  const auto *wave = static_cast<const int *>(f.near_wave.p);
  const auto *b = static_cast<const cv_t<T> *>(beta);
  auto *o = static_cast<cv_t<T> *>(out);
  const int kc = cdiv(f.near_k, f.near_chunks);
  const dim3 grid(cdiv(n, kThreads), f.near_chunks);
  // FP64: two output halves (register pressure); FP32: one launch
  switch (ctx->p) {
#define X(PP)                                                                                                    \
  case PP:                                                                                                       \
    if constexpr (std::is_same<T, double>::value) {                                                              \
      hipLaunchKernelGGL((k_fmm_near<T, PP, 0>), grid, dim3(kThreads), 0, ctx->stream, pairs, src, perm, wave, b, \
                         o, n, kc);                                                                              \
      hipLaunchKernelGGL((k_fmm_near<T, PP, 1>), grid, dim3(kThreads), 0, ctx->stream, pairs, src, perm, wave, b, \
                         o, n, kc);                                                                              \
    } else {                                                                                                     \
      hipLaunchKernelGGL((k_fmm_near<T, PP, -1>), grid, dim3(kThreads), 0, ctx->stream, pairs, src, perm, wave,   \
                         b, o, n, kc);                                                                           \
    }                                                                                                            \
    break;
    MPSL_P_CASES(X)
#undef X
    default: return set_err(ctx, MPSL_EUNSUPPORTED, "expansion order outside 1..20");
  }
  LAUNCH_CHECK(ctx);
  return MPSL_OK;
}

int launch_fmm_near(mpsl_ctx *ctx, int prec, const void *beta, void *out) {
  return prec == MPSL_FP64 ? launch_fmm_near_t<double>(ctx, beta, out) : launch_fmm_near_t<float>(ctx, beta, out);
}

template <typename T>
static int launch_m2s_t(mpsl_ctx *ctx, const void *beta, void *spec, int nrhs) {
  const int n = static_cast<int>(ctx->n);
  const int chunks = chunks_m2s(ctx, nrhs, std::is_same<T, double>::value ? MPSL_FP64 : MPSL_FP32);
  const int chunk_len = cdiv(n, chunks);
  const dim3 grid(cdiv(ctx->ns, 16 * kM2sWaves), chunks, 2 * nrhs);
  const bool f64 = std::is_same<T, double>::value;
  const auto *E = static_cast<const cv_t<T> *>(f64 ? ctx->gt.E64.p : ctx->gt.E32.p);
  const auto *W = static_cast<const cv_t<T> *>(f64 ? ctx->ct.W64.p : ctx->ct.W32.p);
  const auto *b = static_cast<const cv_t<T> *>(beta);
  auto *part = static_cast<cv_t<T> *>(ctx->m2s_part.p);
  switch (ctx->p) {
#define X(PP) \
  case PP: hipLaunchKernelGGL((k_m2s_mfma<T, PP>), grid, dim3(64 * kM2sWaves), 0, ctx->stream, E, b, W, part, n, ctx->ns, chunk_len, chunks); break;
    MPSL_P_CASES(X)
#undef X
    default: return set_err(ctx, MPSL_EUNSUPPORTED, "expansion order outside 1..20");
  }
  LAUNCH_CHECK(ctx);
  hipLaunchKernelGGL(k_m2s_reduce<T>, dim3(cdiv(2 * ctx->ns * nrhs, 256)), dim3(256), 0, ctx->stream,
                     static_cast<const cv_t<T> *>(part), ctx->ns, chunks, nrhs, static_cast<double2 *>(spec));
  LAUNCH_CHECK(ctx);
  return MPSL_OK;
}

int launch_m2s(mpsl_ctx *ctx, int prec, const void *beta, void *spec, int nrhs) {
  if (ctx->somm.active) return launch_m2s_interp(ctx, prec, beta, spec, nrhs);
  return prec == MPSL_FP64 ? launch_m2s_t<double>(ctx, beta, spec, nrhs)
                           : launch_m2s_t<float>(ctx, beta, spec, nrhs);
}

int launch_reflect(mpsl_ctx *ctx, const void *spec, const double *src, void *sigma, int nrhs) {
  const int ns = ctx->ns;
  hipLaunchKernelGGL(k_reflect, dim3(cdiv(ns, 256), nrhs), dim3(256), 0, ctx->stream,
                     static_cast<const double2 *>(spec), static_cast<const double2 *>(ctx->ct.R.p),
                     static_cast<const double2 *>(ctx->ct.srcfac.p), static_cast<const double2 *>(ctx->ct.lam.p),
                     static_cast<const double2 *>(ctx->ct.gw.p), ns, src ? 1 : 0, src ? src[0] : 0.0,
                     src ? src[1] - ctx->yint[0] : 0.0, static_cast<double2 *>(sigma));
  LAUNCH_CHECK(ctx);
  return MPSL_OK;
}

int launch_s2l_coef(mpsl_ctx *ctx, const void *sigma, int nrhs) {
  if (ctx->somm.active) {  // the interpolated S2L reads the densities directly
    ctx->somm.sigma = sigma;
    return MPSL_OK;
  }
  const int P = 2 * ctx->p + 1;
  const int64_t tot = 2LL * ctx->ns * P * nrhs;
  hipLaunchKernelGGL(k_s2l_coef, dim3(cdiv(tot, 256)), dim3(256), 0, ctx->stream,
                     static_cast<const double2 *>(sigma), static_cast<const double2 *>(ctx->ct.cq.p),
                     static_cast<const double2 *>(ctx->ct.U64.p), ctx->ns, P, nrhs,
                     static_cast<double2 *>(ctx->Up64.p), static_cast<float2 *>(ctx->Up32.p));
  LAUNCH_CHECK(ctx);
  return MPSL_OK;
}

template <typename T>
static int launch_s2l_t(mpsl_ctx *ctx, void *part, int chunks, int nrhs, int64_t pstride) {
  const int n = static_cast<int>(ctx->n);
  const int chunk_len = cdiv(ctx->ns, chunks);
  constexpr int MT = s2l_tiles<T>();
  const dim3 grid(cdiv(n, 16 * MT * kS2lWaves), chunks, nrhs);
  const bool f64 = std::is_same<T, double>::value;
  const auto *F = static_cast<const cv_t<T> *>(f64 ? ctx->gt.F64.p : ctx->gt.F32.p);
  const auto *Up = static_cast<const cv_t<T> *>(f64 ? ctx->Up64.p : ctx->Up32.p);
  auto *o = static_cast<cv_t<T> *>(part);
  switch (ctx->p) {
#define X(PP) \
  case PP: hipLaunchKernelGGL((k_s2l_mfma<T, PP, MT>), grid, dim3(64 * kS2lWaves), 0, ctx->stream, F, Up, o, n, ctx->ns, chunk_len, pstride); break;
    MPSL_P_CASES(X)
#undef X
    default: return set_err(ctx, MPSL_EUNSUPPORTED, "expansion order outside 1..20");
  }
  LAUNCH_CHECK(ctx);
  return MPSL_OK;
}

int launch_s2l(mpsl_ctx *ctx, int prec, void *part, int chunks, int nrhs, int64_t pstride) {
  if (ctx->somm.active) return launch_s2l_interp(ctx, prec, part, chunks, nrhs, pstride);
  return prec == MPSL_FP64 ? launch_s2l_t<double>(ctx, part, chunks, nrhs, pstride)
                           : launch_s2l_t<float>(ctx, part, chunks, nrhs, pstride);
}

int launch_sum_parts(mpsl_ctx *ctx, int prec, const void *part, int chunks, void *alpha) {
  const int64_t len = ctx->n * static_cast<int64_t>(2 * ctx->p + 1);
  if (prec == MPSL_FP64)
    hipLaunchKernelGGL(k_sum_parts<double>, dim3(cdiv(len, 256)), dim3(256), 0, ctx->stream,
                       static_cast<const double2 *>(part), chunks, len, static_cast<double2 *>(alpha));
  else
    hipLaunchKernelGGL(k_sum_parts<float>, dim3(cdiv(len, 256)), dim3(256), 0, ctx->stream,
                       static_cast<const float2 *>(part), chunks, len, static_cast<float2 *>(alpha));
  LAUNCH_CHECK(ctx);
  return MPSL_OK;
}

template <typename T>
static int launch_sapply_t(mpsl_ctx *ctx, const void *x, const void *alpha, void *y, int nrhs, int64_t astride) {
  const int n = static_cast<int>(ctx->n);
  const bool f64 = std::is_same<T, double>::value;
  const auto *S = static_cast<const cv_t<T> *>(f64 ? ctx->S64.p : ctx->S32.p);
  const auto *rot = static_cast<const cv_t<T> *>(f64 ? ctx->gt.rot64.p : ctx->gt.rot32.p);
  const dim3 grid(cdiv(n, 16), nrhs);
  const dim3 block(kSapplyThreads);
  const auto *xx = static_cast<const cv_t<T> *>(x);
  const auto *aa = static_cast<const cv_t<T> *>(alpha);
  auto *yy = static_cast<cv_t<T> *>(y);
  // per-particle types only when several prototypes and a typed geometry
  const bool typed = ctx->n_types > 1 && !ctx->ptype.empty();
  const int32_t *ty = typed ? static_cast<const int32_t *>(ctx->types_dev.p) : nullptr;
  const int nt = typed ? ctx->n_types : 1;
  switch (ctx->p) {
#define X(PP) \
  case PP: hipLaunchKernelGGL((k_sapply<T, PP>), grid, block, 0, ctx->stream, xx, aa, S, rot, n, yy, astride, ty, nt); break;
    MPSL_P_CASES(X)
#undef X
    default: return set_err(ctx, MPSL_EUNSUPPORTED, "expansion order outside 1..20");
  }
  LAUNCH_CHECK(ctx);
  return MPSL_OK;
}

int launch_sapply(mpsl_ctx *ctx, int prec, const void *x, const void *alpha, void *y, int nrhs, int64_t astride) {
  return prec == MPSL_FP64 ? launch_sapply_t<double>(ctx, x, alpha, y, nrhs, astride)
                           : launch_sapply_t<float>(ctx, x, alpha, y, nrhs, astride);
}

int launch_fold_parts(mpsl_ctx *ctx, int prec, void *part, int chunks, int nrhs, int64_t pstride) {
  if (chunks <= 1) return MPSL_OK;
  const int64_t len = ctx->n * static_cast<int64_t>(2 * ctx->p + 1);
  const dim3 grid(cdiv(len, 256), nrhs);
  if (prec == MPSL_FP64)
    hipLaunchKernelGGL(k_fold_parts<double>, grid, dim3(256), 0, ctx->stream, static_cast<double2 *>(part), chunks,
                       len, pstride);
  else
    hipLaunchKernelGGL(k_fold_parts<float>, grid, dim3(256), 0, ctx->stream, static_cast<float2 *>(part), chunks,
                       len, pstride);
  LAUNCH_CHECK(ctx);
  return MPSL_OK;
}

int launch_proj_fix(mpsl_ctx *ctx, void *h, const void *q, int k) {
  hipLaunchKernelGGL(k_proj_fix, dim3(1), dim3(kRed), 0, ctx->stream, static_cast<double2 *>(h),
                     static_cast<const double2 *>(q), k);
  LAUNCH_CHECK(ctx);
  return MPSL_OK;
}

size_t dotc_scratch_bytes(int k) { return static_cast<size_t>(std::max(k, 1)) * kDotBlocks * sizeof(double2); }

int launch_dotc_multi(mpsl_ctx *ctx, const void *V, int64_t ld_v, int k, const void *w, int64_t len,
                      void *h_out, const int32_t *skip, int v_prec) {
  if (ctx->scal.bytes < dotc_scratch_bytes(k))
    return set_err(ctx, MPSL_EINVAL, "reduction scratch too small for " + std::to_string(k) + " dot products");
  auto *scr = static_cast<double2 *>(ctx->scal.p);
  const dim3 grid(kDotBlocks, cdiv(k, kDotVecs));
  if (v_prec == MPSL_FP32)
    hipLaunchKernelGGL(k_dotc_part<float2>, grid, dim3(kRed), 0, ctx->stream, static_cast<const float2 *>(V), ld_v,
                       k, static_cast<const double2 *>(w), len, scr, skip);
  else
    hipLaunchKernelGGL(k_dotc_part<double2>, grid, dim3(kRed), 0, ctx->stream, static_cast<const double2 *>(V), ld_v,
                       k, static_cast<const double2 *>(w), len, scr, skip);
  LAUNCH_CHECK(ctx);
  hipLaunchKernelGGL(k_dotc_final, dim3(cdiv(k, 256)), dim3(256), 0, ctx->stream, scr, k, kDotBlocks,
                     static_cast<double2 *>(h_out), skip);
  LAUNCH_CHECK(ctx);
  return MPSL_OK;
}

int launch_gemv_sub(mpsl_ctx *ctx, const void *V, int64_t ld_v, int k, const void *h, void *w, int64_t len,
                    const int32_t *skip, int v_prec) {
  if (v_prec == MPSL_FP32)
    hipLaunchKernelGGL(k_gemv_sub<float2>, dim3(cdiv(len, 256)), dim3(256), 0, ctx->stream,
                       static_cast<const float2 *>(V), ld_v, k, static_cast<const double2 *>(h),
                       static_cast<double2 *>(w), len, skip);
  else
    hipLaunchKernelGGL(k_gemv_sub<double2>, dim3(cdiv(len, 256)), dim3(256), 0, ctx->stream,
                       static_cast<const double2 *>(V), ld_v, k, static_cast<const double2 *>(h),
                       static_cast<double2 *>(w), len, skip);
  LAUNCH_CHECK(ctx);
  return MPSL_OK;
}

int launch_scale_to_fp32(mpsl_ctx *ctx, void *v32, int64_t len, double s, const void *src) {
  hipLaunchKernelGGL(k_scale_to32, dim3(cdiv(len, 256)), dim3(256), 0, ctx->stream, static_cast<float2 *>(v32),
                     static_cast<const double2 *>(src), len, s);
  LAUNCH_CHECK(ctx);
  return MPSL_OK;
}

int launch_reorth_flag(mpsl_ctx *ctx, const void *before, const void *after, double eta2, int32_t *skip) {
  hipLaunchKernelGGL(k_reorth_flag, dim3(1), dim3(64), 0, ctx->stream, static_cast<const double2 *>(before),
                     static_cast<const double2 *>(after), eta2, skip);
  LAUNCH_CHECK(ctx);
  return MPSL_OK;
}

int launch_scale(mpsl_ctx *ctx, void *v, int64_t len, double s, const void *src) {
  hipLaunchKernelGGL(k_scale, dim3(cdiv(len, 256)), dim3(256), 0, ctx->stream, static_cast<double2 *>(v),
                     static_cast<const double2 *>(src), len, s);
  LAUNCH_CHECK(ctx);
  return MPSL_OK;
}

int launch_axpy_c(mpsl_ctx *ctx, void *y, const void *x, int64_t len, double a_re, double a_im) {
  hipLaunchKernelGGL(k_axpy_c, dim3(cdiv(len, 256)), dim3(256), 0, ctx->stream, static_cast<double2 *>(y),
                     static_cast<const double2 *>(x), len, a_re, a_im);
  LAUNCH_CHECK(ctx);
  return MPSL_OK;
}

int launch_to_fp32(mpsl_ctx *ctx, const void *x64, void *x32, int64_t len) {
  hipLaunchKernelGGL(k_to32, dim3(cdiv(len, 256)), dim3(256), 0, ctx->stream, static_cast<const double2 *>(x64),
                     static_cast<float2 *>(x32), len);
  LAUNCH_CHECK(ctx);
  return MPSL_OK;
}

int launch_fill_hash(mpsl_ctx *ctx, int prec, void *v, int64_t n_complex, uint32_t seed) {
  const int64_t len = 2 * n_complex;
  if (prec == MPSL_FP64)
    hipLaunchKernelGGL(k_fill_hash, dim3(cdiv(len, 256)), dim3(256), 0, ctx->stream, static_cast<double *>(v), len, seed);
  else
    hipLaunchKernelGGL(k_fill_hash32, dim3(cdiv(len, 256)), dim3(256), 0, ctx->stream, static_cast<float *>(v), len, seed);
  LAUNCH_CHECK(ctx);
  return MPSL_OK;
}

int launch_to_fp64(mpsl_ctx *ctx, const void *x32, void *x64, int64_t len) {
  hipLaunchKernelGGL(k_to64, dim3(cdiv(len, 256)), dim3(256), 0, ctx->stream, static_cast<const float2 *>(x32),
                     static_cast<double2 *>(x64), len);
  LAUNCH_CHECK(ctx);
  return MPSL_OK;
}

int launch_field(mpsl_ctx *ctx, const void *beta, const void *gl, const void *amp, const void *yint,
                 const double *src, int64_t nr, const void *rcv, void *u) {
  hipLaunchKernelGGL(k_field, dim3(cdiv(nr, 64)), dim3(64), 0, ctx->stream,
                     static_cast<const double2 *>(ctx->gt.xy.p), static_cast<const double2 *>(beta),
                     static_cast<int>(ctx->n), ctx->p, static_cast<const double2 *>(ctx->ct.lam.p),
                     static_cast<const double2 *>(ctx->ct.gw.p) + 3 * ctx->ns,  // weights stored after g1,g2,g3
                     static_cast<const double2 *>(gl), static_cast<const double2 *>(amp),
                     static_cast<const double *>(yint), static_cast<int>(ctx->ks.size()), ctx->layer_c, ctx->ns,
                     ctx->k1.real(), ctx->k2.real(), ctx->r_enc,
                     (ctx->n_types > 1 && !ctx->ptype.empty()) ? static_cast<const int32_t *>(ctx->types_dev.p)
                                                                : nullptr,
                     static_cast<const double *>(ctx->rtype_dev.p), src[0], src[1],
                     static_cast<const double2 *>(rcv), nr, static_cast<double2 *>(u));
  LAUNCH_CHECK(ctx);
  return MPSL_OK;
}

}  // namespace mpsl
