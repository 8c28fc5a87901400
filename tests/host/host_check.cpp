// Test driver for the host-side scan-path and geometry logic of the
// library (tl_host.cpp), built with g++ under AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_logic.py.  Reads queries on
// stdin and prints the library's answers, one line each:
//   T n, then n lines "x0 y0 x1 y1 speed power radius absorptivity depth"
//   S t_start
//   L t                                  -> "L on xc yc P R eta k"
//   W t hx hy nx ny wx wy have I0 J0     -> "W I0 J0"
//   B t0 t1                              -> "B n" and n lines
//                                           "x_lo x_hi y_lo y_hi depth q"
//   G nq                                 -> "G x0 w0 x1 w1 ..."
#include <cstdio>
#include <vector>

#include "tl_internal.h"

using namespace tl;

int main() {
  std::vector<TrackH> tr;
  double t_start = 0.0;
  char op[4];
  while (std::scanf("%3s", op) == 1) {
    if (op[0] == 'T') {
      int n;
      if (std::scanf("%d", &n) != 1) return 2;
      tr.resize(n);
      for (TrackH& a : tr)
        if (std::scanf("%lf %lf %lf %lf %lf %lf %lf %lf %lf", &a.x0, &a.y0,
                       &a.x1, &a.y1, &a.speed, &a.power, &a.radius,
                       &a.absorptivity, &a.depth) != 9)
          return 2;
    } else if (op[0] == 'S') {
      if (std::scanf("%lf", &t_start) != 1) return 2;
    } else if (op[0] == 'L') {
      double t, xc = 0, yc = 0, P = 0, R = 0, eta = 0;
      int k = -1;
      if (std::scanf("%lf", &t) != 1) return 2;
      const int on = laser_at(tr.data(), (int)tr.size(), t_start, t, &xc, &yc,
                              &P, &R, &eta, &k);
      std::printf("L %d %.17g %.17g %.17g %.17g %.17g %d\n", on, xc, yc, P, R,
                  eta, k);
    } else if (op[0] == 'W') {
      double t, hx, hy;
      int nx, ny, wx, wy, have, ci, cj, I0, J0;
      if (std::scanf("%lf %lf %lf %d %d %d %d %d %d %d", &t, &hx, &hy, &nx,
                     &ny, &wx, &wy, &have, &ci, &cj) != 10)
        return 2;
      window_origin(tr.data(), (int)tr.size(), t_start, t, hx, hy, nx, ny, wx,
                    wy, have, ci, cj, &I0, &J0);
      std::printf("W %d %d\n", I0, J0);
    } else if (op[0] == 'B') {
      double t0, t1;
      if (std::scanf("%lf %lf", &t0, &t1) != 2) return 2;
      BoxSet bs;
      const int n = swept_boxes(tr.data(), (int)tr.size(), t_start, t0, t1, &bs);
      std::printf("B %d\n", n);
      for (int q = 0; q < n; ++q)
        std::printf("%.17g %.17g %.17g %.17g %.17g %.17g\n", bs.b[q].x_lo,
                    bs.b[q].x_hi, bs.b[q].y_lo, bs.b[q].y_hi, bs.b[q].depth,
                    bs.b[q].q);
    } else if (op[0] == 'G') {
      int nq;
      if (std::scanf("%d", &nq) != 1) return 2;
      double x[4], w[4];
      gauss01(nq, x, w);
      std::printf("G");
      for (int q = 0; q < nq; ++q) std::printf(" %.17g %.17g", x[q], w[q]);
      std::printf("\n");
    } else {
      return 2;
    }
  }
  return 0;
}
