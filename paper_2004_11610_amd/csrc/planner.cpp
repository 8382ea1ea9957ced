// Host-side plan parameters (float64): the Kaiser window (sec. 2.1), zeta(eps1)
// by Newton (sec. 2.2), the number of extra components s(zeta, eps2) (sec. 2.2)
// and the block partition of the block method (sec. 3, Table 1).
//
// Readings of the paper used here:
//  * Newton is applied to I0(zeta) - 1/eps1 (the same root as 1/I0 = eps1).
//  * s is the smallest s >= 1 with w_s^{zeta, W-1+2s} >= eps2, the window value
//    at the first retained column of a width-W row extended by s on each side.
//  * a block of width W uses its first s columns as left extras and s more
//    columns on the right: length L = W + s, window w^{zeta, L-1}; the next
//    block has width s; recursion stops when the width is <= min_block or when
//    s >= W, and those columns are multiplied directly.
//  * L is rounded up to the smallest even length whose half is 2^a 3^b 5^c
//    (sec. 5.1 recommends a slightly larger s for a fast FFT length).

#include "planner.hpp"

#include <cmath>

namespace spt {

// I0(z) = sum_k ((z/2)^k / k!)^2  (all terms positive: no cancellation)
double bessel_i0(double z) {
  const double q = 0.25 * z * z;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 1000; ++k) {
    term *= q / ((double)k * (double)k);
    sum += term;
    if (term < 1e-17 * sum) break;
  }
  return sum;
}

// I1(z) = sum_k (z/2)^{2k+1} / (k! (k+1)!)
double bessel_i1(double z) {
  const double q = 0.25 * z * z;
  double term = 0.5 * z, sum = term;
  for (int k = 1; k < 1000; ++k) {
    term *= q / ((double)k * (double)(k + 1));
    sum += term;
    if (term < 1e-17 * sum) break;
  }
  return sum;
}

double zeta_of_eps(double eps1) {
  double z = 50.0;
  for (int it = 0; it < 500; ++it) {
    const double dz = (bessel_i0(z) - 1.0 / eps1) / bessel_i1(z);
    z -= dz;
    if (std::fabs(dz) <= 1e-14 * z) break;
  }
  return z;
}

double kaiser(double n, double M, double zeta) {
  const double t = 2.0 * n / M - 1.0;
  const double a = 1.0 - t * t;
  return bessel_i0(zeta * std::sqrt(a > 0.0 ? a : 0.0)) / bessel_i0(zeta);
}

int64_t extra_count(int64_t W, double zeta, double eps2) {
  int64_t s = 1;
  while (kaiser((double)s, (double)(W - 1 + 2 * s), zeta) < eps2) ++s;
  return s;
}

static bool smooth5(int64_t n) {
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

int64_t fft_length(int64_t lmin) {
  int64_t L = lmin < 2 ? 2 : lmin + (lmin & 1);
  while (!smooth5(L / 2)) L += 2;
  return L;
}

void partition_one_sided(int64_t N, double zeta, double eps2, int64_t min_block, bool round_fft,
                         std::vector<BlockGeom>& blocks, int64_t& tail) {
  blocks.clear();
  int64_t W = N;
  while (W > min_block) {
    int64_t s = extra_count(W, zeta, eps2);
    int64_t L = W + s;
    if (round_fft) {
      L = fft_length(L);
      s = L - W;
    }
    if (s >= W) break;
    blocks.push_back(BlockGeom{(int)L, 0, (int)s, (int)W});
    W = s;
  }
  tail = W;
}

void partition_two_sided(int64_t N, double zeta, double eps2, bool round_fft,
                         std::vector<BlockGeom>& blocks, int64_t& tail) {
  const int64_t s = extra_count(N, zeta, eps2);
  int64_t L = N + 2 * s;
  if (round_fft) L = fft_length(L);
  blocks.assign(1, BlockGeom{(int)L, (int)-s, (int)s, (int)(s + N)});
  tail = 0;
}

}  // namespace spt
