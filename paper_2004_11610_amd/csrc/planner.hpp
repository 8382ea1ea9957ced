// Host-side plan parameters (see planner.cpp).
#pragma once

#include <stdint.h>

#include <vector>

namespace spt {

// One compressed block: columns c = 0 .. L-1 hold degrees m = c + m_off, the
// columns [c_lo, c_hi) carry the input, the others are extra components.
struct BlockGeom {
  int L;
  int m_off;
  int c_lo;
  int c_hi;
};

double bessel_i0(double z);
double bessel_i1(double z);
double zeta_of_eps(double eps1);
double kaiser(double n, double M, double zeta);
int64_t extra_count(int64_t W, double zeta, double eps2);
int64_t fft_length(int64_t lmin);
void partition_one_sided(int64_t N, double zeta, double eps2, int64_t min_block, bool round_fft,
                         std::vector<BlockGeom>& blocks, int64_t& tail);
void partition_two_sided(int64_t N, double zeta, double eps2, bool round_fft,
                         std::vector<BlockGeom>& blocks, int64_t& tail);

}  // namespace spt
