// Solid x-intervals of a convex body along lattice rows, and the node
// windows around their ends that a moving body's advance visits (host and
// device: the host bounds the list the kernel builds from the same windows).
#pragma once
#include <math.h>

#include "geom.hpp"

namespace lbm {

// Solid x-interval [a, b] of the row (y, z) at pose p (the body is convex in
// x); false if the row misses the body. Rounding of a and b is absorbed by
// the margin of the windows built from them; the status itself always comes
// from shape_phi.
__host__ __device__ inline bool row_chord(const BodyShape& b, const Pose& p, int y, int z, double& a, double& bb) {
  const double dy = y - p.X[1], dz = b.D == 3 ? z - p.X[2] : 0.0;
  if (b.shape == SHAPE_CIRCLE) {
    const double q = b.R * b.R - dy * dy - dz * dz;
    if (q < 0.0) return false;
    const double h = sqrt(q);
    a = p.X[0] - h;
    bb = p.X[0] + h;
    return true;
  }
  const double A = p.ct * p.ct * b.ia2 + p.st * p.st * b.ib2;
  const double Bh = dy * p.ct * p.st * (b.ia2 - b.ib2);
  const double C = dy * dy * (p.st * p.st * b.ia2 + p.ct * p.ct * b.ib2) + dz * dz * b.ic2 - 1.0;
  const double disc = Bh * Bh - A * C;
  if (disc < 0.0) return false;
  const double h = sqrt(disc);
  a = p.X[0] + (-Bh - h) / A;
  bb = p.X[0] + (-Bh + h) / A;
  return true;
}

// Extent of the solid x-intervals over a set of (row, pose) chords: the
// lowest and highest start and end, whether any chord hits the body and
// whether any misses it.
struct RowExtent {
  double amin = 1e300, amax = -1e300, bmin = 1e300, bmax = -1e300;
  bool any = false, gap = false;
  __host__ __device__ void add(bool hit, double a, double bb) {
    if (hit) {
      any = true;
      amin = fmin(amin, a);
      amax = fmax(amax, a);
      bmin = fmin(bmin, bb);
      bmax = fmax(bmax, bb);
    } else {
      gap = true;
    }
  }
};

// Node windows [w0,w1] and [w2,w3] (x, inclusive) of a row from the extent
// of its chords and those of its lattice neighbour rows at both poses,
// widened by `m` nodes and clipped to [xlo, xhi]. Returns the number of
// windows.
__host__ __device__ inline int windows_of(const RowExtent& e, int m, int xlo, int xhi, int w[4]) {
  if (!e.any) return 0;
  int n;
  if (e.gap) {  // a cap row: one window over the whole hull
    w[0] = (int)floor(e.amin) - m;
    w[1] = (int)ceil(e.bmax) + m;
    n = 1;
  } else {
    w[0] = (int)floor(e.amin) - m;
    w[1] = (int)ceil(e.amax) + m;
    w[2] = (int)floor(e.bmin) - m;
    w[3] = (int)ceil(e.bmax) + m;
    n = 2;
    if (w[2] <= w[1] + 1) {
      w[1] = w[3];
      n = 1;
    }
  }
  for (int k = 0; k < n; ++k) {
    w[2 * k] = w[2 * k] < xlo ? xlo : w[2 * k];
    w[2 * k + 1] = w[2 * k + 1] > xhi ? xhi : w[2 * k + 1];
  }
  return n;
}

// Node windows of row (y,z) outside which nothing can change between poses
// P0 and P1, nor hold a link at P1: around both ends of the solid interval,
// over the row and its lattice neighbour rows, widened by `m` nodes.
__host__ __device__ inline int row_windows(const BodyShape& b, const Pose& P0, const Pose& P1, int y, int z, int D, int m,
                                  int xlo, int xhi, int w[4]) {
  RowExtent e;
  for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int k = 0; k < 2; ++k) {
        double a = 0, bb = 0;
        const bool hit = row_chord(b, k ? P1 : P0, y + dy, z + dz, a, bb);
        e.add(hit, a, bb);
      }
  return windows_of(e, m, xlo, xhi, w);
}

}  // namespace lbm
