// Host build of the library's PSD projection (bfc_eig.h) for CPU tests:
// reads count, n, then count upper-triangle matrices (doubles) from stdin's
// file argument, writes the projected upper triangles.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "bfc_eig.h"

template <int N> static void run(std::FILE* in, std::FILE* out, long count, double tol) {
  constexpr int M = N * (N + 1) / 2;
  std::vector<double> a(M), p(M);
  for (long c = 0; c < count; ++c) {
    if (std::fread(a.data(), sizeof(double), M, in) != (size_t)M) std::exit(3);
    bfc::psd_project<N>(a.data(), p.data(), tol);
    std::fwrite(p.data(), sizeof(double), M, out);
  }
}

int main(int argc, char** argv) {
  if (argc != 4) return 2;
  std::FILE* in = std::fopen(argv[1], "rb");
  std::FILE* out = std::fopen(argv[2], "wb");
  if (!in || !out) return 2;
  double tol = std::atof(argv[3]);
  long hdr[2];
  if (std::fread(hdr, sizeof(long), 2, in) != 2) return 3;
  if (hdr[1] == 6) run<6>(in, out, hdr[0], tol);
  else if (hdr[1] == 9) run<9>(in, out, hdr[0], tol);
  else return 4;
  std::fclose(in);
  std::fclose(out);
  return 0;
}
