// Gaussian DRM factors drawn by the library from a 64-bit seed (host code).
//
// Algorithm PSTT draws its dimension reduction maps with i.i.d. standard
// Gaussian entries (Section 3.2).  When the caller passes no factors, entry j
// of the packed factor buffer (the layout pstt2_desc.drm_factors documents)
// is the standard normal
//   p = j / 2, (x0, x1, x2, x3) = Philox4x32-10(counter (p mod 2^32, p / 2^32, 0, 0),
//                                                key (seed mod 2^32, seed / 2^32))
//   u1 = 1 - ((x0 >> 5) 2^26 + (x1 >> 6)) 2^-53        in (0, 1]
//   u2 =     ((x2 >> 5) 2^26 + (x3 >> 6)) 2^-53        in [0, 1)
//   entry 2p = sqrt(-2 ln u1) cos(2 pi u2), entry 2p + 1 = sqrt(-2 ln u1) sin(2 pi u2)
// Philox4x32-10 is the counter-based generator of Salmon, Moraes, Dror and
// Shaw ("Parallel random numbers: as easy as 1, 2, 3", SC 2011): ten rounds of
// two 32x32 -> 64-bit multiplies with the Weyl key schedule; the normals are
// the Box-Muller transform of the two 53-bit uniforms.  Every entry depends
// only on (seed, j), so any sub-range can be drawn independently.
#include <cmath>
#include <cstdint>

#include "internal.h"

namespace pstt2 {

namespace {
constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;   // round multipliers
constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;   // key increments

void philox4x32_10(const uint32_t in[4], uint32_t k0, uint32_t k1, uint32_t out[4]) {
  uint32_t c0 = in[0], c1 = in[1], c2 = in[2], c3 = in[3];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += kW0;
      k1 += kW1;
    }
    const uint64_t p0 = (uint64_t)kM0 * c0, p1 = (uint64_t)kM1 * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

double unit53(uint32_t a, uint32_t b) {
  return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}
}  // namespace

void philox_block(uint64_t seed, uint64_t counter, uint32_t out[4]) {
  const uint32_t ctr[4] = {(uint32_t)counter, (uint32_t)(counter >> 32), 0u, 0u};
  philox4x32_10(ctr, (uint32_t)seed, (uint32_t)(seed >> 32), out);
}

void gaussian_fill(uint64_t seed, int64_t first, int64_t count, double* out) {
  const double two_pi = 2.0 * M_PI;
  for (int64_t t = 0; t < count; ++t) {
    const int64_t j = first + t;
    uint32_t x[4];
    philox_block(seed, (uint64_t)(j >> 1), x);
    const double u1 = 1.0 - unit53(x[0], x[1]);
    const double u2 = unit53(x[2], x[3]);
    const double rad = std::sqrt(-2.0 * std::log(u1));
    out[t] = (j & 1) ? rad * std::sin(two_pi * u2) : rad * std::cos(two_pi * u2);
  }
}

}  // namespace pstt2
