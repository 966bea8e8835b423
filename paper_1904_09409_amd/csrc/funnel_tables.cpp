// funnel_tables.cpp -- host tables of the chirp-z NVMT, computed in FP64 and
// rounded to FP32 once.
#include <cmath>
#include <complex>
#include <vector>

#include "funnel_internal.hpp"

namespace funnel {
namespace {

using cd = std::complex<double>;

// y[k] = sum_j x[j xs] exp(-2 pi i j k / n), k < n, by recursive decimation in
// time over the smallest prime factor; root[t] = exp(-2 pi i t / Ln) with
// n | Ln; scratch holds 2n values.
void dft_rec(const cd* x, size_t xs, cd* y, int n, const std::vector<cd>& root, int Ln, cd* scratch) {
  if (n == 1) {
    y[0] = x[0];
    return;
  }
  int p = 2;
  while (n % p) ++p;
  const int m = n / p;
  cd* sub = scratch;
  for (int r = 0; r < p; ++r) dft_rec(x + r * xs, xs * p, sub + (size_t)r * m, m, root, Ln, scratch + n);
  const int step = Ln / n;
  for (int k = 0; k < n; ++k) {
    cd acc = 0.0;
    for (int r = 0; r < p; ++r) acc += sub[(size_t)r * m + k % m] * root[(size_t)((long long)r * k % n) * step];
    y[k] = acc;
  }
}

}  // namespace

// Row n2 has ratio s = 2 n2 / Np.  Chirp phases pi s k^2 / W = 2 pi (n2 k^2) / (Np W)
// are reduced modulo Np W in integers before the cosine and sine.
//   wz[n2-1][i] = exp(-j pi s x^2 / W), x = i - W/2
//   cz[n2-1][k] = (s / L) DFT_L(c')[k], L = 2W, c'[k] = c'[L-k] = exp(+j pi s k^2 / W)
//                 for 0 <= k < W, c'[W] = 0 (the lags of a linear convolution of
//                 two length-W sequences, placed cyclically)
void chirp_tables(int W, int Np, int h, float2* cz, float2* wz) {
  const int L = 2 * W;
  const long long period = (long long)Np * W;
  std::vector<cd> root(L), c(L), C(L), scratch(2 * (size_t)L);
  for (int t = 0; t < L; ++t) {
    const double a = -2.0 * M_PI * (double)t / (double)L;
    root[t] = cd(std::cos(a), std::sin(a));
  }
  for (int n2 = 1; n2 <= h; ++n2) {
    const double s = 2.0 * n2 / Np;
    auto chirp = [&](long long k) {
      const long long q = (long long)n2 * ((k * k) % period) % period;
      const double a = 2.0 * M_PI * (double)q / (double)period;
      return cd(std::cos(a), std::sin(a));
    };
    for (int k = 0; k < L; ++k) c[k] = 0.0;
    for (int k = 0; k < W; ++k) c[k] = chirp(k);
    for (int k = 1; k < W; ++k) c[L - k] = c[k];
    dft_rec(c.data(), 1, C.data(), L, root, L, scratch.data());
    float2* czr = cz + (size_t)(n2 - 1) * L;
    for (int k = 0; k < L; ++k) {
      const cd v = C[k] * (s / L);
      czr[k] = make_float2((float)v.real(), (float)v.imag());
    }
    float2* wzr = wz + (size_t)(n2 - 1) * W;
    for (int i = 0; i < W; ++i) {
      const cd v = std::conj(chirp(i - W / 2));
      wzr[i] = make_float2((float)v.real(), (float)v.imag());
    }
  }
}

}  // namespace funnel
