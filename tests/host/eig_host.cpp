// Host build of the library's PSD projection (bfc_eig.h) for CPU tests:
// reads count, n, then count upper-triangle matrices (doubles) from stdin's
// file argument, writes the projected upper triangles.
#include <cmath>
#include <cstdio>
#include <xmmintrin.h>
#include <pmmintrin.h>
#include <cstdlib>
#include <vector>

#include "bfc_eig.h"

// tol < 0: the single-precision projection of the mixed mode (the matrix
// scaled by its largest entry, projected in float with QR steps stopping at
// 1e-6 of |A|, scaled back); tol < -1.5 also flushes denormals to zero, as
// the device does in single precision.
template <int N> static void run(std::FILE* in, std::FILE* out, long count, double tol) {
  constexpr int M = N * (N + 1) / 2;
  std::vector<double> a(M), p(M);
  std::vector<float> af(M), pf(M);
  for (long c = 0; c < count; ++c) {
    if (std::fread(a.data(), sizeof(double), M, in) != (size_t)M) std::exit(3);
    if (tol >= 0.0) {
      bfc::psd_project<N>(a.data(), p.data(), tol);
    } else {
      double amax = 0.0;
      for (int k = 0; k < M; ++k) amax = std::fmax(amax, std::fabs(a[k]));
      if (amax > 0.0) {
        for (int k = 0; k < M; ++k) {
          const double y = a[k] / amax;
          af[k] = std::fabs(y) < 1e-18 ? 0.0f : (float)y;
        }
        bfc::psd_project<N, float>(af.data(), pf.data(), 1e-6f);
        for (int k = 0; k < M; ++k) p[k] = (double)pf[k] * amax;
      } else {
        for (int k = 0; k < M; ++k) p[k] = 0.0;
      }
    }
    std::fwrite(p.data(), sizeof(double), M, out);
  }
}

int main(int argc, char** argv) {
  if (argc != 4) return 2;
  std::FILE* in = std::fopen(argv[1], "rb");
  std::FILE* out = std::fopen(argv[2], "wb");
  if (!in || !out) return 2;
  double tol = std::atof(argv[3]);
  if (tol < -1.5) {  // as the device treats single precision: denormal inputs and results flushed to zero
    _MM_SET_FLUSH_ZERO_MODE(_MM_FLUSH_ZERO_ON);
    _MM_SET_DENORMALS_ZERO_MODE(_MM_DENORMALS_ZERO_ON);
  }
  long hdr[2];
  if (std::fread(hdr, sizeof(long), 2, in) != 2) return 3;
  if (hdr[1] == 6) run<6>(in, out, hdr[0], tol);
  else if (hdr[1] == 9) run<9>(in, out, hdr[0], tol);
  else return 4;
  std::fclose(in);
  std::fclose(out);
  return 0;
}
