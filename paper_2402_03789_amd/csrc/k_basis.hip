// Edge basis and its adjoint.
//
// Each edge v<-w carries the displacement d = r_w - r_v (paper section 3.1,
// eq 5 context), evaluated in float64 from float64 positions (ghost
// positions are owner position + image shift).  The edge feature is
// (section 5.1) the real spherical harmonics of d/|d| up to l_sh, in the
// component normalisation |Y^l|^2 = 2l+1 with m ordered -l..l:
//   Y^0 = 1,  Y^1 = sqrt3 (y, z, x),
//   Y^2 = (sqrt15 xy, sqrt15 yz, sqrt5/2 (3z^2-1), sqrt15 xz, sqrt15/2 (x^2-y^2)),
//   Y^3 = (a y(3x^2-y^2), b xyz, c y(5z^2-1), d z(5z^2-3), c x(5z^2-1), b/2 z(x^2-y^2),
//          a x(x^2-3y^2)),  a = sqrt70/4, b = sqrt105, c = sqrt42/4, d = sqrt7/2
//   (l = 3 for the benchmark models of section 4),
// and 8 radial Bessel functions (2/r_c) sin(n pi r / r_c) / r times the
// polynomial envelope u(x) = 1 - (p+1)(p+2)/2 x^p + p(p+2) x^(p+1) - p(p+1)/2 x^(p+2).
//
// The adjoint turns dE/dY and dE/drho, summed over all interaction blocks,
// into the edge gradient g = dE/dd (eq 5 summed over t):
//   g = (sum_n dE/drho_n drho_n/dr) d/r + (I - rr^T)/r grad_rhat (sum_m dE/dY_m Y_m).
#include "kernels.h"

namespace sn {

// l = 3 coefficients
constexpr double kY3a = 2.0916500663351889;  // sqrt(70) / 4
constexpr double kY3b = 10.246950765959598;  // sqrt(105)
constexpr double kY3c = 1.6201851746019651;  // sqrt(42) / 4
constexpr double kY3d = 1.3228756555322954;  // sqrt(7) / 2

template <typename T>
__global__ void k_edge_basis(int64_t E, const int* __restrict__ recv, const int* __restrict__ src,
                             const double* __restrict__ pos_ext, double r_cut, int nb, int p,
                             int l_sh, T* __restrict__ Y, T* __restrict__ rho) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  int i = recv[e], s = src[e];
  double d0 = pos_ext[3 * s] - pos_ext[3 * i];
  double d1 = pos_ext[3 * s + 1] - pos_ext[3 * i + 1];
  double d2 = pos_ext[3 * s + 2] - pos_ext[3 * i + 2];
  double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
  double x = d0 / r, y = d1 / r, z = d2 / r;
  const int NY = (l_sh + 1) * (l_sh + 1);
  T* Ye = Y + e * NY;
  Ye[0] = T(1);
  if (l_sh >= 1) {
    const double s3 = 1.7320508075688772;
    Ye[1] = T(s3 * y);
    Ye[2] = T(s3 * z);
    Ye[3] = T(s3 * x);
  }
  if (l_sh >= 2) {
    const double s15 = 3.872983346207417, s5 = 2.23606797749979;
    Ye[4] = T(s15 * x * y);
    Ye[5] = T(s15 * y * z);
    Ye[6] = T(0.5 * s5 * (3.0 * z * z - 1.0));
    Ye[7] = T(s15 * x * z);
    Ye[8] = T(0.5 * s15 * (x * x - y * y));
  }
  if (l_sh >= 3) {
    Ye[9] = T(kY3a * y * (3.0 * x * x - y * y));
    Ye[10] = T(kY3b * x * y * z);
    Ye[11] = T(kY3c * y * (5.0 * z * z - 1.0));
    Ye[12] = T(kY3d * z * (5.0 * z * z - 3.0));
    Ye[13] = T(kY3c * x * (5.0 * z * z - 1.0));
    Ye[14] = T(0.5 * kY3b * z * (x * x - y * y));
    Ye[15] = T(kY3a * x * (x * x - 3.0 * y * y));
  }
  double xr = r / r_cut;
  double c1 = (p + 1) * (p + 2) / 2.0, c2 = p * (p + 2.0), c3 = p * (p + 1) / 2.0;
  double xp = pow(xr, p);
  double u = (xr < 1.0) ? 1.0 - c1 * xp + c2 * xp * xr - c3 * xp * xr * xr : 0.0;
  const double pi = 3.141592653589793;
  for (int n = 1; n <= nb; ++n) {
    double b = (2.0 / r_cut) * sin(n * pi * r / r_cut) / r;
    rho[e * nb + (n - 1)] = T(b * u);
  }
}

template <typename T>
__global__ void k_edge_grad(int64_t E, const int* __restrict__ recv, const int* __restrict__ src,
                            const double* __restrict__ pos_ext, double r_cut, int nb, int p,
                            int l_sh, const T* __restrict__ dY, const T* __restrict__ drho,
                            double* __restrict__ g) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  int i = recv[e], s = src[e];
  double d0 = pos_ext[3 * s] - pos_ext[3 * i];
  double d1 = pos_ext[3 * s + 1] - pos_ext[3 * i + 1];
  double d2 = pos_ext[3 * s + 2] - pos_ext[3 * i + 2];
  double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
  double x = d0 / r, y = d1 / r, z = d2 / r;
  // radial part
  double xr = r / r_cut;
  double c1 = (p + 1) * (p + 2) / 2.0, c2 = p * (p + 2.0), c3 = p * (p + 1) / 2.0;
  double xp1 = pow(xr, p - 1);
  double xp = xp1 * xr;
  double u = 1.0 - c1 * xp + c2 * xp * xr - c3 * xp * xr * xr;
  double du = (-p * c1 * xp1 + (p + 1) * c2 * xp - (p + 2) * c3 * xp * xr) / r_cut;
  if (xr >= 1.0) {  // skin edges beyond r_c: the envelope and its derivative vanish
    u = 0.0;
    du = 0.0;
  }
  const double pi = 3.141592653589793;
  double dEdr = 0.0;
  for (int n = 1; n <= nb; ++n) {
    double k = n * pi / r_cut;
    double sn = sin(k * r), cs = cos(k * r);
    double b = (2.0 / r_cut) * sn / r;
    double db = (2.0 / r_cut) * (k * cs * r - sn) / (r * r);
    dEdr += (double)drho[e * nb + (n - 1)] * (db * u + b * du);
  }
  // angular part: gradient of sum_m dY_m Y_m(x, y, z) as a polynomial
  const int NY = (l_sh + 1) * (l_sh + 1);
  const T* a = dY + e * NY;
  double vx = 0, vy = 0, vz = 0;
  if (l_sh >= 1) {
    const double s3 = 1.7320508075688772;
    vx += s3 * (double)a[3];
    vy += s3 * (double)a[1];
    vz += s3 * (double)a[2];
  }
  if (l_sh >= 2) {
    const double s15 = 3.872983346207417, s5 = 2.23606797749979;
    double a4 = a[4], a5 = a[5], a6 = a[6], a7 = a[7], a8 = a[8];
    vx += s15 * (a4 * y + a7 * z + a8 * x);
    vy += s15 * (a4 * x + a5 * z - a8 * y);
    vz += s15 * (a5 * y + a7 * x) + 3.0 * s5 * a6 * z;
  }
  if (l_sh >= 3) {  // gradients of the l = 3 polynomials above
    const double a9 = a[9], a10 = a[10], a11 = a[11], a12 = a[12], a13 = a[13], a14 = a[14],
                 a15 = a[15];
    const double q = 5.0 * z * z - 1.0;
    vx += kY3a * (6.0 * x * y * a9 + 3.0 * (x * x - y * y) * a15) + kY3b * y * z * a10 +
          kY3c * q * a13 + kY3b * x * z * a14;
    vy += kY3a * (3.0 * (x * x - y * y) * a9 - 6.0 * x * y * a15) + kY3b * x * z * a10 +
          kY3c * q * a11 - kY3b * y * z * a14;
    vz += kY3b * x * y * a10 + 10.0 * kY3c * z * (y * a11 + x * a13) +
          kY3d * (15.0 * z * z - 3.0) * a12 + 0.5 * kY3b * (x * x - y * y) * a14;
  }
  double vr = vx * x + vy * y + vz * z;
  g[3 * e] = dEdr * x + (vx - vr * x) / r;
  g[3 * e + 1] = dEdr * y + (vy - vr * y) / r;
  g[3 * e + 2] = dEdr * z + (vz - vr * z) / r;
}

template <typename T>
void launch_edge_basis(int64_t E, const int* recv, const int* src, const double* pos_ext,
                       double r_cut, int n_basis, int p, int l_sh, T* Y, T* rho, hipStream_t s) {
  if (E > 0)
    k_edge_basis<T><<<(unsigned)((E + 255) / 256), 256, 0, s>>>(E, recv, src, pos_ext, r_cut,
                                                                n_basis, p, l_sh, Y, rho);
}
template <typename T>
void launch_edge_grad(int64_t E, const int* recv, const int* src, const double* pos_ext,
                      double r_cut, int n_basis, int p, int l_sh, const T* dY, const T* drho,
                      double* g, hipStream_t s) {
  if (E > 0)
    k_edge_grad<T><<<(unsigned)((E + 255) / 256), 256, 0, s>>>(E, recv, src, pos_ext, r_cut,
                                                               n_basis, p, l_sh, dY, drho, g);
}

template void launch_edge_basis<float>(int64_t, const int*, const int*, const double*, double, int,
                                       int, int, float*, float*, hipStream_t);
template void launch_edge_basis<double>(int64_t, const int*, const int*, const double*, double, int,
                                        int, int, double*, double*, hipStream_t);
template void launch_edge_grad<float>(int64_t, const int*, const int*, const double*, double, int,
                                      int, int, const float*, const float*, double*, hipStream_t);
template void launch_edge_grad<double>(int64_t, const int*, const int*, const double*, double, int,
                                       int, int, const double*, const double*, double*, hipStream_t);

}  // namespace sn
