// Boundary data of the star-particle precompute (Section 4) shared by the
// host and the device solvers: samples of the boundary of eq. (50), the
// quadrature tables, the right-hand sides and the weights of eq. (35).
#pragma once

#include <complex>
#include <string>
#include <vector>

struct mpsl_ctx;

namespace mpsl {

struct StarParts {
  int nb = 0, p = 0;
  // per boundary sample: parameter, radius, point, x', x'', speed, unit outward normal
  std::vector<double> t, r, x, y, dx, dy, ddx, ddy, speed, nx, ny;
  std::vector<double> Rk;                     // Kress weights, indexed by (i - j) mod nb
  std::vector<double> Fd;                     // spectral d/dt, nb x nb row-major
  std::vector<std::complex<double>> B;        // right-hand sides [P][2 nb]: -u_inc, -du_inc/dn
  std::vector<std::complex<double>> Fs, Fm;   // eq. (35) weights [P][nb], (i/4) h |x'| folded in
};

// Host part of the precompute: everything of size O(nb P) and the tables.
int star_parts(double a1, double a2, int a3, double k2, int p, int nb, StarParts &sp, std::string &err);

// Device solve of Mueller's system (assembly, Maue products, LU, eq. (35)) on
// the context's stream; S receives the P x P matrix (row-major, host).
int star_smatrix_device(mpsl_ctx *ctx, const StarParts &sp, double k2, double kp, int pol,
                        std::vector<std::complex<double>> &S, std::string &err);

}  // namespace mpsl
