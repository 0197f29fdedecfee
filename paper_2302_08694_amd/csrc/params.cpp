// Plan-time numerics: Kaiser-Bessel kernel, its Fourier transform, the piecewise polynomial fit
// evaluated by the spreading/interpolation kernels, fine-grid sizes and FFT radix plans.
#include <cmath>
#include <vector>

#include "plan.hpp"

namespace fsib {

// Modified Bessel function I0 by its power series sum_k (x^2/4)^k / (k!)^2; every term is
// positive, so the sum is accurate to rounding for the arguments used here (|x| <= 40).
double bessel_i0(double x) {
  const double q = 0.25 * x * x;
  long double term = 1.0L, sum = 1.0L;
  for (int k = 1; k < 500; ++k) {
    term *= (long double)q / ((long double)k * (long double)k);
    sum += term;
    if (term < sum * 1e-21L) break;
  }
  return (double)sum;
}

// Kaiser-Bessel kernel G(z) = I0(beta sqrt(1-z^2)) / I0(beta) on |z| <= 1 (App. A, eq. kernel_KB).
static double kb(double z, double beta) {
  if (std::fabs(z) > 1.0) return 0.0;
  return bessel_i0(beta * std::sqrt(1.0 - z * z)) / bessel_i0(beta);
}

// Its transform int_{-1}^{1} G(z) cos(a z) dz = (2/I0(beta)) sinh(sqrt(beta^2-a^2))/sqrt(beta^2-a^2)
// (App. A, eq. kernel_KB_hat); for a > beta the square root is imaginary and sinh(i s)/(i s) =
// sin(s)/s continues it.
double kb_transform(double a, double beta) {
  const double s2 = beta * beta - a * a;
  double r;
  if (std::fabs(s2) < 1e-14) {
    r = 1.0;
  } else if (s2 > 0) {
    const double s = std::sqrt(s2);
    r = std::sinh(s) / s;
  } else {
    const double s = std::sqrt(-s2);
    r = std::sin(s) / s;
  }
  return 2.0 * r / bessel_i0(beta);
}

// One-dimensional relative error of the oversampled (factor 2) nonuniform transform with the
// Kaiser-Bessel kernel of width w and shape beta = choose_beta(w, 2), measured against direct sums
// on random points (N = 128, M = 2000) when this library's parameters were chosen.
static const double kErr1d[17] = {1, 1,       3.5e-2,  3.3e-3,  3.6e-4,  4.2e-5,  4.4e-6,  4.9e-7, 5.2e-8,
                                  4.9e-9,     5.3e-10, 5.4e-11, 6.2e-12, 6.8e-13, 7.8e-14, 1.5e-14, 1.2e-14};
// The same for oversampling 1.25 with beta = 1.86 w (the best ratio of a scan over beta/w; close to
// beta = pi sqrt((w/sigma)^2 (sigma - 1/2)^2 - 0.8) of Beatty, Nishimura and Pauly, 2005).
static const double kErr1d125[17] = {1, 1,      1.1e-1, 2.6e-2, 5.2e-3, 1.2e-3, 2.7e-4, 6.2e-5, 1.4e-5,
                                     3.5e-6,    7.8e-7, 2.3e-7, 6.2e-8, 1.4e-8, 3.3e-9, 7.3e-10, 1.9e-10};

// The same for oversampling 1.5 with beta = 2.07 w for w >= 5 (1.86, 1.96, 2.04 w below; the best
// ratios of a scan over beta/w in steps of 0.02), measured the same way.
static const double kErr1d15[17] = {1, 1,      6.1e-2, 8.2e-3, 1.3e-3, 2.1e-4, 3.6e-5, 5.3e-6, 7.3e-7,
                                    1.2e-7,    2.2e-8, 4.0e-9, 6.7e-10, 9.5e-11, 1.5e-11, 2.5e-12, 4.0e-13};

int choose_width(double tol, int dim, double sigma) {
  // per-axis errors add up across the dim axes: ask each axis for tol / (2 dim)
  const double target = tol / (2.0 * dim);
  const double* err = sigma < 1.4 ? kErr1d125 : (sigma < 1.75 ? kErr1d15 : kErr1d);
  for (int w = 2; w <= kMaxW; ++w)
    if (err[w] <= target) return w;
  return kMaxW + 1;  // out of reach: the caller rejects the tolerance
}

double choose_beta(int w, double sigma) {
  if (sigma < 1.4) return 1.86 * w;
  if (sigma < 1.75) {
    static const double r15[5] = {0, 0, 1.86, 1.96, 2.04};
    return (w < 5 ? r15[w] : 2.07) * w;
  }
  static const double ratio[6] = {0, 0, 2.143, 2.257, 2.300, 2.329};
  return (w < 6 ? ratio[w] : 2.343) * w;
}

int choose_degree(int w) { return w + 2 < kMaxDeg ? w + 2 : kMaxDeg; }

// Piece j of the kernel, as a function of the point's sub-cell position y in [-1, 1]:
// the support of a point at fine-grid coordinate g starts at cell i0 = ceil(g - w/2); with
// s = i0 - g + w/2 in [0, 1) and y = 2s - 1, cell i0 + j sits at z = 2 (s - w/2 + j) / w.
// Each piece is interpolated at deg+1 Chebyshev points of [-1, 1] and rewritten in monomials of y.
void fit_kernel_pieces(int w, double beta, int deg, double* coef) {
  const int np = deg + 1;
  std::vector<long double> nodes(np), vals(np), cheb(np);
  for (int i = 0; i < np; ++i) nodes[i] = cosl(M_PI * (i + 0.5L) / np);
  for (int j = 0; j < w; ++j) {
    for (int i = 0; i < np; ++i) {
      const double s = 0.5 * ((double)nodes[i] + 1.0);
      vals[i] = kb(2.0 * (s - 0.5 * w + j) / w, beta);
    }
    // Chebyshev coefficients by the discrete orthogonality of T_k at the nodes
    for (int k = 0; k < np; ++k) {
      long double acc = 0;
      for (int i = 0; i < np; ++i) acc += vals[i] * cosl(M_PI * k * (i + 0.5L) / np);
      cheb[k] = acc * (k == 0 ? 1.0L : 2.0L) / np;
    }
    // monomial coefficients: accumulate c_k T_k(y), T_{k+1} = 2 y T_k - T_{k-1}
    std::vector<long double> tkm1(np, 0), tk(np, 0), tkp1(np, 0), mono(np, 0);
    tkm1[0] = 1;  // T_0
    if (np > 1) tk[1] = 1;  // T_1
    for (int i = 0; i < np; ++i) mono[i] += cheb[0] * tkm1[i];
    if (np > 1)
      for (int i = 0; i < np; ++i) mono[i] += cheb[1] * tk[i];
    for (int k = 1; k + 1 < np; ++k) {
      for (int i = 0; i < np; ++i) tkp1[i] = (i > 0 ? 2 * tk[i - 1] : 0) - tkm1[i];
      for (int i = 0; i < np; ++i) mono[i] += cheb[k + 1] * tkp1[i];
      tkm1 = tk;
      tk = tkp1;
    }
    for (int i = 0; i < np; ++i) coef[i * w + j] = (double)mono[i];
  }
}

static bool smooth235(int64_t n) {
  for (int64_t f : {2, 3, 5})
    while (n % f == 0) n /= f;
  return n == 1;
}

int64_t smooth_at_least(int64_t n, int64_t multiple) {
  int64_t m = n < 1 ? 1 : n;
  while (!(smooth235(m) && m % multiple == 0)) ++m;
  return m;
}

// Radices for a length-n Stockham FFT: 8 first, then 4, 2, 3, 5; returns the stage count (0 if n
// has another prime factor or needs too many stages).
int radix_plan(int n, int* radix) {
  int ns = 0;
  int m = n;
  while (m % 8 == 0 && ns < kMaxStages) { radix[ns++] = 8; m /= 8; }
  while (m % 4 == 0 && ns < kMaxStages) { radix[ns++] = 4; m /= 4; }
  while (m % 2 == 0 && ns < kMaxStages) { radix[ns++] = 2; m /= 2; }
  while (m % 3 == 0 && ns < kMaxStages) { radix[ns++] = 3; m /= 3; }
  while (m % 5 == 0 && ns < kMaxStages) { radix[ns++] = 5; m /= 5; }
  return m == 1 ? ns : 0;
}

}  // namespace fsib
