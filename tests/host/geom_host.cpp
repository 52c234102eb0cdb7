// Host build of the library's exact threshold decisions (bfc_geom.h) for
// CPU tests.  Input file: count, then per record: code (as a double), the
// pair's four vertices X[12], the threshold T as two doubles (hi, lo).
// Output per record: the sign of D - T from exact FP64 evaluation (2 when
// some operation rounds), from expansions (2 when they outgrow their room),
// the double-double comparison (-1, 0, 1), and from the point-edge fixed-point
// sum (2 when it does not apply).
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "bfc_geom.h"

int main(int argc, char** argv) {
  if (argc != 3) return 2;
  std::FILE* in = std::fopen(argv[1], "rb");
  std::FILE* out = std::fopen(argv[2], "wb");
  if (!in || !out) return 2;
  long n = 0;
  if (std::fread(&n, sizeof(long), 1, in) != 1) return 3;
  std::vector<double> ws(bfc::XP_WS);
  for (long r = 0; r < n; ++r) {
    double rec[15];
    if (std::fread(rec, sizeof(double), 15, in) != 15) return 3;
    const int code = (int)rec[0];
    bfc::d3 P[4];
    for (int k = 0; k < 4; ++k) P[k] = {rec[1 + 3 * k], rec[2 + 3 * k], rec[3 + 3 * k]};
    const bfc::dd T = {rec[13], rec[14]};
    double o[4];
    o[0] = bfc::exact_in_double(code, P, T);
    o[1] = bfc::xp_sign_sq_minus(code, P[0], P[1], P[2], P[3], T, ws.data());
    bfc::q3 Q[4] = {bfc::q3_of(P[0]), bfc::q3_of(P[1]), bfc::q3_of(P[2]), bfc::q3_of(P[3])};
    const bfc::dd Dq = bfc::sqd_case<bfc::dd>(code, Q);
    o[2] = bfc::dd_lt(Dq, T) ? -1.0 : (bfc::dd_lt(T, Dq) ? 1.0 : 0.0);
    o[3] = bfc::pe_sign_code(code, P, T);
    std::fwrite(o, sizeof(double), 4, out);
  }
  std::fclose(in);
  std::fclose(out);
  return 0;
}
