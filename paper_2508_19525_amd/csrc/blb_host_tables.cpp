// Host-only tables that need quad precision (compiled by the host C++ compiler):
// double-double twiddles of the encoder and the Gaussian sampler's CDT.
#include <quadmath.h>
#include <stdint.h>

namespace {
void dd_split(__float128 v, double* hi, double* lo) {
  *hi = (double)v;
  *lo = (double)(v - (__float128)(*hi));
}
}  // namespace

// tw: [N/4][4] = (re_hi, re_lo, im_hi, im_lo) of eta^k, eta = exp(2 pi i / (N/2));
// twist: [N/2][4] of zeta^-k, zeta = exp(i pi / N).
extern "C" void blb_host_enc_tables(int log_n, double* tw, double* twist) {
  const int n = 1 << log_n, M = n / 2;
  for (int k = 0; k < M / 2; ++k) {
    const __float128 ang = 2 * M_PIq * (__float128)k / (__float128)M;
    dd_split(cosq(ang), &tw[k * 4 + 0], &tw[k * 4 + 1]);
    dd_split(sinq(ang), &tw[k * 4 + 2], &tw[k * 4 + 3]);
  }
  for (int k = 0; k < M; ++k) {
    const __float128 ang = M_PIq * (__float128)k / (__float128)n;
    dd_split(cosq(ang), &twist[k * 4 + 0], &twist[k * 4 + 1]);
    dd_split(-sinq(ang), &twist[k * 4 + 2], &twist[k * 4 + 3]);
  }
}

// Cumulative distribution of |x| for the rounded Gaussian (sigma 3.2, |x| <= 19) as 63-bit
// thresholds floor(2^63 P(|x| <= k)); the last bucket takes the remainder.
extern "C" void blb_host_cdt(uint64_t out[20]) {
  __float128 rho[20], z = 0;
  const __float128 sigma = 3.2Q;
  for (int x = 0; x < 20; ++x) {
    rho[x] = expq(-((__float128)x * x) / (2 * sigma * sigma));
    z += (x ? 2 : 1) * rho[x];
  }
  __float128 acc = 0;
  const __float128 scale = 9223372036854775808.0Q;
  for (int x = 0; x < 20; ++x) {
    acc += (x ? 2 : 1) * rho[x] / z;
    const __float128 t = floorq(acc * scale);
    out[x] = t >= scale ? 0x7FFFFFFFFFFFFFFFull : (uint64_t)t;
  }
  out[19] = 0x7FFFFFFFFFFFFFFFull;
}
