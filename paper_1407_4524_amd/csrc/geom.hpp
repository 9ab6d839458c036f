// Domain layout, body poses and the shape function of the GPU path.
//
// Everything here is shared by the host layer and the kernels. The shape
// function and the link root are evaluated with FP contraction off, in the
// left-to-right order that include/lbm.h fixes, so the solid/fluid decision
// and Delta are reproducible bit for bit wherever they are computed.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

enum { FACE_PERIODIC = 0, FACE_WALL = 1, FACE_INLET = 2, FACE_OUTLET = 3, FACE_OUTLET_VELOCITY = 4,
       FACE_ZOUHE_VELOCITY = 5, FACE_ZOUHE_PRESSURE = 6 };
enum { SRC_NONE = 0, SRC_WALL = 1, SRC_INLET = 2, SRC_OUTLET = 3, SRC_OUTVEL = 4 };
enum { SHAPE_CIRCLE = 0, SHAPE_ELLIPSE = 1, SHAPE_OUTER_CIRCLE = 2 };
enum { MASK_FLUID = 0, MASK_WALL = 1, MASK_BODY0 = 2 };

// Padded structure-of-arrays layout. Node (x,y,z), with each coordinate in
// [-1, n] (one halo layer), lives at element base + x + y*sy + z*sz of every
// population array; population i starts at i*S. Interior node x = 0 sits on a
// 128-byte boundary.
struct Geom {
  int nx, ny, nz, D;
  int64_t sy, sz, S, base;
  int face[6];
  // active (non-wall) index ranges, inclusive
  int lo[3], hi[3];
  __host__ __device__ int64_t idx(int x, int y, int z) const { return base + x + y * sy + z * sz; }
};

// Physical parameters of the update.
struct Phys {
  double tau, omega, rho0;
  int eq;  // 0 standard, 1 quasi-incompressible
  int inlet_profile;
  double inlet_u;
  // parabolic inlet: 4 / (n - 2)^2 across the y and z wall pairs
  double inlet_ky, inlet_kz;
};

// Pose of a body at one step: 16 doubles on the device.
struct Pose {
  double X[3];
  double ct, st;
  double V[3];
  double Om;
  double theta;
  double lo[3], hi[3];  // region (inclusive node box) that holds the body and its links
};

struct BodyShape {
  int shape, D;
  double R;              // radius (circle/sphere, outer circle)
  double ia2, ib2, ic2;  // 1/(a*a), 1/(b*b), 1/(c*c)
  int refill;            // REFILL_* rule for the nodes the body uncovers
};

enum { REFILL_MEAN = 0, REFILL_AIDUN = 1, REFILL_EXTRAPOLATE = 2 };

// cos and sin of the angle of a body whose motion the simulation computes
// (include/lbm.h fixes the steps so that every evaluation gives the same
// bits): reduction by pi/2 in two parts (Cody-Waite), then the Taylor series
// of sin through r^17/17! and of cos through r^18/18! in Horner form.
__host__ __device__ inline void free_trig(double theta, double& c, double& s) {
#pragma clang fp contract(off)
  const double k = rint(theta * 0.63661977236758134);
  const double r = (theta - k * 1.5707963267948966) - k * 6.123233995736766e-17;
  const double z = r * r;
  double ps = 1.0 / 355687428096000.0;
  ps = -1.0 / 1307674368000.0 + z * ps;
  ps = 1.0 / 6227020800.0 + z * ps;
  ps = -1.0 / 39916800.0 + z * ps;
  ps = 1.0 / 362880.0 + z * ps;
  ps = -1.0 / 5040.0 + z * ps;
  ps = 1.0 / 120.0 + z * ps;
  ps = -1.0 / 6.0 + z * ps;
  const double sr = r + (r * z) * ps;
  double pc = 1.0 / 6402373705728000.0;
  pc = -1.0 / 20922789888000.0 + z * pc;
  pc = 1.0 / 87178291200.0 + z * pc;
  pc = -1.0 / 479001600.0 + z * pc;
  pc = 1.0 / 3628800.0 + z * pc;
  pc = -1.0 / 40320.0 + z * pc;
  pc = 1.0 / 720.0 + z * pc;
  pc = -1.0 / 24.0 + z * pc;
  pc = 0.5 + z * pc;
  const double cr = 1.0 - z * pc;
  const long long q = ((long long)k) & 3;
  c = q == 0 ? cr : (q == 1 ? -sr : (q == 2 ? -cr : sr));
  s = q == 0 ? sr : (q == 1 ? cr : (q == 2 ? -sr : -cr));
}

// Outward normal (gradient of phi up to a factor 2) of the body at node
// (x, y, z), the direction Lallemand & Luo's refill extrapolates along
__host__ __device__ inline void shape_normal(const BodyShape& b, const Pose& p, double x, double y, double z,
                                             double n[3]) {
#pragma clang fp contract(off)
  const double dx = x - p.X[0], dy = y - p.X[1], dz = b.D == 3 ? z - p.X[2] : 0.0;
  if (b.shape == SHAPE_ELLIPSE) {
    const double xi = p.ct * dx + p.st * dy, eta = p.ct * dy - p.st * dx;
    n[0] = xi * p.ct * b.ia2 - eta * p.st * b.ib2;
    n[1] = xi * p.st * b.ia2 + eta * p.ct * b.ib2;
    n[2] = b.D == 3 ? dz * b.ic2 : 0.0;
  } else {
    const double sg = b.shape == SHAPE_OUTER_CIRCLE ? -1.0 : 1.0;
    n[0] = sg * dx;
    n[1] = sg * dy;
    n[2] = sg * dz;
  }
}

// Node box of a pose: the body plus two layers (links and their
// neighbours); the whole active box for an outer circle. axes: radius or
// semi-axes; lo, hi: the active index ranges of the domain.
__host__ __device__ inline void pose_box(int shape, const double* axes, int D, const int* glo, const int* ghi,
                                         Pose& p) {
#pragma clang fp contract(off)
  if (shape == SHAPE_OUTER_CIRCLE) {
    for (int a = 0; a < 3; ++a) {
      p.lo[a] = glo[a];
      p.hi[a] = ghi[a];
    }
    return;
  }
  double h[3];
  if (shape == SHAPE_CIRCLE) {
    h[0] = h[1] = h[2] = axes[0];
  } else {
    const double a = axes[0], bb = axes[1];
    h[0] = sqrt(a * a * p.ct * p.ct + bb * bb * p.st * p.st);
    h[1] = sqrt(a * a * p.st * p.st + bb * bb * p.ct * p.ct);
    h[2] = axes[2];
  }
  for (int a = 0; a < 3; ++a) {
    if (a >= D) {
      p.lo[a] = p.hi[a] = 0;
      continue;
    }
    p.lo[a] = floor(p.X[a] - h[a]) - 2.0;
    p.hi[a] = ceil(p.X[a] + h[a]) + 2.0;
  }
}

__host__ __device__ inline double shape_phi(const BodyShape& b, const Pose& p, double x, double y, double z) {
#pragma clang fp contract(off)
  double dx = x - p.X[0], dy = y - p.X[1], dz = z - p.X[2];
  if (b.shape == SHAPE_CIRCLE || b.shape == SHAPE_OUTER_CIRCLE) {
    double r2 = (b.D == 3) ? dx * dx + dy * dy + dz * dz : dx * dx + dy * dy;
    return b.shape == SHAPE_CIRCLE ? r2 - b.R * b.R : b.R * b.R - r2;
  }
  double xi = p.ct * dx + p.st * dy;
  double eta = p.ct * dy - p.st * dx;
  if (b.D == 3) return xi * xi * b.ia2 + eta * eta * b.ib2 + dz * dz * b.ic2 - 1.0;
  return xi * xi * b.ia2 + eta * eta * b.ib2 - 1.0;
}

// Fractional wall distance of the link from fluid node xF toward xF - c:
// the root in (0,1] of phi(xF - s c) = A s^2 + 2 B s + C, C = phi(xF) > 0,
// as C / (-B + sqrt(B^2 - A C)).
__host__ __device__ inline double link_delta(const BodyShape& b, const Pose& p, double x, double y, double z,
                                             int cxi, int cyi, int czi) {
#pragma clang fp contract(off)
  double dx = x - p.X[0], dy = y - p.X[1], dz = z - p.X[2];
  double cx = cxi, cy = cyi, cz = czi;
  double A, B;
  double C = shape_phi(b, p, x, y, z);
  if (b.shape == SHAPE_CIRCLE) {
    A = (b.D == 3) ? cx * cx + cy * cy + cz * cz : cx * cx + cy * cy;
    B = -((b.D == 3) ? dx * cx + dy * cy + dz * cz : dx * cx + dy * cy);
  } else if (b.shape == SHAPE_OUTER_CIRCLE) {
    A = -((b.D == 3) ? cx * cx + cy * cy + cz * cz : cx * cx + cy * cy);
    B = (b.D == 3) ? dx * cx + dy * cy + dz * cz : dx * cx + dy * cy;
  } else {
    double xi = p.ct * dx + p.st * dy;
    double eta = p.ct * dy - p.st * dx;
    double xic = p.ct * cx + p.st * cy;
    double etac = p.ct * cy - p.st * cx;
    if (b.D == 3) {
      A = xic * xic * b.ia2 + etac * etac * b.ib2 + cz * cz * b.ic2;
      B = -(xi * xic * b.ia2 + eta * etac * b.ib2 + dz * cz * b.ic2);
    } else {
      A = xic * xic * b.ia2 + etac * etac * b.ib2;
      B = -(xi * xic * b.ia2 + eta * etac * b.ib2);
    }
  }
  double disc = B * B - A * C;
  if (disc < 0.0) disc = 0.0;
  double s = C / (-B + sqrt(disc));
  return s > 1.0 ? 1.0 : s;
}

// One boundary link: fluid node (x,y,z) at padded index `cell`, direction
// `dir` pointing out of the body, fractional distance delta.
struct Link {
  int32_t cell;
  int16_t x, y, z;
  int16_t dir;
  double delta;
};
static_assert(sizeof(Link) == 24, "link record layout");

}  // namespace lbm
