// Host-side geometry and scan-path logic of the two-level solver: the laser
// position along the scan path, the window placement rule, micro-step times,
// Gauss-Legendre rules and the structured-grid descriptor.  Built without
// floating-point contraction so that every decision that depends on these
// values (laser on/off, window cell) is reproducible.
#include <algorithm>
#include <cmath>

#include "tl_internal.h"

namespace tl {

// Beam position at time t (paper Section 5.2: the laser moves along the scan
// tracks at constant speed).  Tracks run back to back from t_start; the beam
// is off before t_start and after the last track ends.
int laser_at(const TrackH* tr, int n, double t_start, double t, double* xc,
             double* yc, double* P, double* R, double* eta, int* k) {
  if (n <= 0 || t < t_start) return 0;
  double tk = t_start;
  int found = -1;
  double t_found = 0.0;
  double t_end = t_start;
  for (int q = 0; q < n; ++q) {
    double len = std::hypot(tr[q].x1 - tr[q].x0, tr[q].y1 - tr[q].y0);
    double t_next = tk + len / tr[q].speed;
    if (found < 0 && (q == n - 1 || t < t_next)) {
      found = q;
      t_found = tk;
    }
    tk = t_next;
  }
  t_end = tk;
  if (t > t_end) return 0;
  const TrackH& a = tr[found];
  double len = std::hypot(a.x1 - a.x0, a.y1 - a.y0);
  double s = (t - t_found) * a.speed;
  double frac = len > 0.0 ? s / len : 0.0;
  if (frac > 1.0) frac = 1.0;
  *xc = a.x0 + (a.x1 - a.x0) * frac;
  *yc = a.y0 + (a.y1 - a.y0) * frac;
  *P = a.power;
  *R = a.radius;
  *eta = a.absorptivity;
  *k = found;
  return 1;
}

int swept_boxes(const TrackH* tr, int n, double t_start, double t0, double t1,
                BoxSet* out) {
  out->n = 0;
  double ts = t_start;
  for (int k = 0; k < n; ++k) {
    const TrackH& a = tr[k];
    const double len = std::hypot(a.x1 - a.x0, a.y1 - a.y0);
    const double te = ts + len / a.speed;
    const double lo = std::max(t0, ts), hi = std::min(t1, te);
    if (hi > lo && len > 0.0) {
      if (out->n == kMaxBoxes) return -1;
      const double ux = (a.x1 - a.x0) / len, uy = (a.y1 - a.y0) / len;
      const double xa = a.x0 + ux * a.speed * (lo - ts);
      const double ya = a.y0 + uy * a.speed * (lo - ts);
      const double xb = a.x0 + ux * a.speed * (hi - ts);
      const double yb = a.y0 + uy * a.speed * (hi - ts);
      Box& b = out->b[out->n++];
      if (std::fabs(uy) < 1e-12) {   // along x
        b.x_lo = std::min(xa, xb);
        b.x_hi = std::max(xa, xb);
        b.y_lo = ya - 0.5 * a.radius;
        b.y_hi = ya + 0.5 * a.radius;
      } else {                       // along y
        b.x_lo = xa - 0.5 * a.radius;
        b.x_hi = xa + 0.5 * a.radius;
        b.y_lo = std::min(ya, yb);
        b.y_hi = std::max(ya, yb);
      }
      b.depth = a.depth;
      b.q = a.absorptivity * a.power / (a.radius * a.depth * a.speed * (t1 - t0));
    }
    ts = te;
  }
  return out->n;
}

// Window placement: whole coarse cells, flush with the top, centred on the
// beam across the scan direction; along it the beam at time t sits one third
// of the window length behind the leading edge; clamped to the plate; kept
// in place while the beam is off (the paper moves the local mesh with the
// laser, Section 5.2, without fixing a rule).
void window_origin(const TrackH* tr, int n, double t_start, double t,
                   double hx, double hy, int nx, int ny, int wx, int wy,
                   int have_current, int cur_I0, int cur_J0, int* I0, int* J0) {
  double xc, yc, P, R, eta;
  int k = 0;
  if (!laser_at(tr, n, t_start, t, &xc, &yc, &P, &R, &eta, &k)) {
    if (have_current) {
      *I0 = cur_I0;
      *J0 = cur_J0;
      return;
    }
    xc = tr[0].x0;
    yc = tr[0].y0;
    k = 0;
  }
  double dx = tr[k].x1 - tr[k].x0, dy = tr[k].y1 - tr[k].y0;
  double wx_len = wx * hx, wy_len = wy * hy;
  double x_lo, y_lo;
  if (std::fabs(dx) >= std::fabs(dy)) {
    double lead = dx >= 0 ? (2.0 / 3.0) : (1.0 / 3.0);
    x_lo = xc - lead * wx_len;
    y_lo = yc - 0.5 * wy_len;
  } else {
    double lead = dy >= 0 ? (2.0 / 3.0) : (1.0 / 3.0);
    x_lo = xc - 0.5 * wx_len;
    y_lo = yc - lead * wy_len;
  }
  int i0 = (int)std::floor(x_lo / hx + 0.5);
  int j0 = (int)std::floor(y_lo / hy + 0.5);
  if (i0 > nx - wx) i0 = nx - wx;
  if (i0 < 0) i0 = 0;
  if (j0 > ny - wy) j0 = ny - wy;
  if (j0 < 0) j0 = 0;
  *I0 = i0;
  *J0 = j0;
}

double micro_time(double t_start, double dt, int m, long n, int j) {
  return t_start + (double)n * dt + (double)j * (dt / (double)m);
}

// Gauss-Legendre rules on [0, 1] for 1..4 points (closed forms).
void gauss01(int nq, double* x, double* w) {
  double p[4] = {0, 0, 0, 0}, q[4] = {0, 0, 0, 0};
  if (nq == 1) {
    p[0] = 0.0; q[0] = 2.0;
  } else if (nq == 2) {
    double a = 1.0 / std::sqrt(3.0);
    p[0] = -a; p[1] = a; q[0] = q[1] = 1.0;
  } else if (nq == 3) {
    double a = std::sqrt(3.0 / 5.0);
    p[0] = -a; p[1] = 0.0; p[2] = a;
    q[0] = q[2] = 5.0 / 9.0; q[1] = 8.0 / 9.0;
  } else {
    double s = 2.0 / 7.0 * std::sqrt(6.0 / 5.0);
    double a = std::sqrt(3.0 / 7.0 - s), b = std::sqrt(3.0 / 7.0 + s);
    double wa = (18.0 + std::sqrt(30.0)) / 36.0, wb = (18.0 - std::sqrt(30.0)) / 36.0;
    p[0] = -b; p[1] = -a; p[2] = a; p[3] = b;
    q[0] = wb; q[1] = wa; q[2] = wa; q[3] = wb;
  }
  for (int i = 0; i < nq; ++i) {
    x[i] = 0.5 * (p[i] + 1.0);
    w[i] = 0.5 * q[i];
  }
}

// Q1 element stiffness of an hx x hy x hz box, indexed by the xor pattern of
// the two corners (bit 0: x differs, bit 1: y, bit 2: z):
//   (hy hz/hx) K1 M1 M1 + (hx hz/hy) M1 K1 M1 + (hx hy/hz) M1 M1 K1,
// K1 = [[1,-1],[-1,1]], M1 = [[1/3,1/6],[1/6,1/3]].
Geo make_geo(int ncx, int ncy, int ncz, double hx, double hy, double hz,
             double x0, double y0) {
  Geo g;
  g.nx = ncx + 1;
  g.ny = ncy + 1;
  g.nz = ncz + 1;
  g.px = (g.nx + 2 + 31) / 32 * 32;
  g.pxy = g.px * (g.ny + 2);
  g.nreal = g.nx * g.ny * g.nz;
  g.npad = (long)g.pxy * (g.nz + 2);
  g.hx = hx;
  g.hy = hy;
  g.hz = hz;
  g.x0 = x0;
  g.y0 = y0;
  g.vol8 = hx * hy * hz / 8.0;
  double cx = hy * hz / hx, cy = hx * hz / hy, cz = hx * hy / hz;
  for (int p = 0; p < 8; ++p) {
    int dx = p & 1, dy = (p >> 1) & 1, dz = (p >> 2) & 1;
    double kx = dx ? -1.0 : 1.0, ky = dy ? -1.0 : 1.0, kz = dz ? -1.0 : 1.0;
    double mx = dx ? 1.0 / 6.0 : 1.0 / 3.0, my = dy ? 1.0 / 6.0 : 1.0 / 3.0,
           mz = dz ? 1.0 / 6.0 : 1.0 / 3.0;
    g.w[p] = cx * kx * my * mz + cy * mx * ky * mz + cz * mx * my * kz;
  }
  return g;
}

}  // namespace tl
