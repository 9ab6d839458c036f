/*
 * lbm_oracle.c -- TEST INFRASTRUCTURE: plain FP64 CPU reference of one
 * lattice-Boltzmann time step with momentum-exchange force and torque
 * (Giovacchini & Ortiz, arXiv:1407.4524). Only tests, the smoke check and the
 * benchmark's CPU-baseline leg use it; the product never does.
 *
 * Storage is array-of-structures f[node*Q + i] and the step is written as
 * collide-then-push, in the order of the paper's two-stage update
 * (Sec. II, Eqs. collision and streaming). Every formula below cites the
 * passage it follows. Where the paper leaves a choice open, the choice is
 * named "reading" in a comment.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off (no fused multiply-add, so the
 * solid/fluid decision is the plainly rounded IEEE value of the shape
 * function).
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_PI 3.14159265358979323846

/* ---------------------------------------------------------------------- */
/* Lattice tables. The paper uses D2Q9 (Sec. IV) but never lists its
 * velocities or weights; these are the textbook tables. Reading: numbering
 * D2Q9 0 rest, 1..4 the axis directions counter-clockwise from +x, 5..8 the
 * diagonals counter-clockwise from (1,1) (so c_1 is an axis and c_5 a
 * diagonal, as in the paper's Fig. 2). D3Q19: 0 rest, 1..6 the axis
 * directions in opposite pairs, 7..18 the face diagonals in opposite pairs. */

typedef struct {
  int D, Q;
  int c[19][3];
  double w[19];
  int opp[19];
} lattice_t;

static const int C_D2Q9[9][3] = {{0, 0, 0},  {1, 0, 0},  {0, 1, 0},   {-1, 0, 0}, {0, -1, 0},
                                 {1, 1, 0},  {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
static const int C_D3Q19[19][3] = {
    {0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
    {-1, 0, 1}, {0, 1, 1},   {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static int lattice_init(lattice_t* L, int kind) {
  memset(L, 0, sizeof(*L));
  if (kind == ORA_D2Q9) {
    L->D = 2;
    L->Q = 9;
    for (int i = 0; i < 9; ++i) {
      for (int a = 0; a < 3; ++a) L->c[i][a] = C_D2Q9[i][a];
      L->w[i] = (i == 0) ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
  } else if (kind == ORA_D3Q19) {
    L->D = 3;
    L->Q = 19;
    for (int i = 0; i < 19; ++i) {
      for (int a = 0; a < 3; ++a) L->c[i][a] = C_D3Q19[i][a];
      L->w[i] = (i == 0) ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
  } else {
    return -1;
  }
  /* opposite index: the direction with c = -c_i */
  for (int i = 0; i < L->Q; ++i)
    for (int j = 0; j < L->Q; ++j)
      if (L->c[j][0] == -L->c[i][0] && L->c[j][1] == -L->c[i][1] && L->c[j][2] == -L->c[i][2])
        L->opp[i] = j;
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Bodies and prescribed motion (Sec. III: Omega(t) is a given function of t). */

typedef struct {
  double X[3];   /* centre */
  double theta;  /* orientation about z */
  double ct, st; /* cos, sin of theta */
  double V[3];   /* centre velocity */
  double Om;     /* angular velocity about z */
  double drive[4]; /* FREE: flow force and torque z that moved the body here */
} pose_t;

typedef struct {
  int active;
  ora_body_desc d;
  double* table; /* owned copy of a TABLE motion */
  double ia2, ib2, ic2;
  /* FREE motion: poses of steps traj_t0 .. traj_t0 + traj_n - 1, and the
     previous step's accelerations (linear, angular) for Adams-Bashforth */
  pose_t* traj;
  int64_t traj_t0, traj_n, traj_cap;
  double a_prev[4];
  int have_prev;
} body_t;

/* cos and sin of theta for FREE bodies, whose angle the simulation
 * produces: Cody-Waite reduction by pi/2 (the double nearest pi/2 plus its
 * remainder) to |r| <= pi/4, then the Taylor series of sin and cos through
 * r^17 / 17! and r^18 / 18! (truncation below 1e-19 there) in Horner form.
 * Every operation is a plain IEEE double operation in a fixed order, so the
 * GPU library, which evaluates the same steps, gets the same bits. */
static void free_trig(double theta, double* c, double* s) {
  const double k = nearbyint(theta * 0.63661977236758134);
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
  const long q = ((long)k) & 3;
  if (q == 0) { *c = cr; *s = sr; }
  else if (q == 1) { *c = -sr; *s = cr; }
  else if (q == 2) { *c = -cr; *s = -sr; }
  else { *c = sr; *s = -cr; }
}

static pose_t body_pose(const body_t* b, int64_t t) {
  pose_t p;
  memset(&p, 0, sizeof(p));
  const ora_body_desc* d = &b->d;
  if (d->motion == ORA_MOTION_FREE) {
    int64_t k = t - b->traj_t0;
    if (k < 0) k = 0;
    if (k >= b->traj_n) k = b->traj_n - 1;
    return b->traj[k];
  }
  for (int a = 0; a < 3; ++a) p.X[a] = d->c0[a];
  p.theta = d->theta0;
  switch (d->motion) {
    case ORA_MOTION_CONST_VEL:
      for (int a = 0; a < 3; ++a) {
        p.X[a] = d->c0[a] + d->vel[a] * (double)t;
        p.V[a] = d->vel[a];
      }
      break;
    case ORA_MOTION_ROTATE:
      p.theta = d->theta0 + d->omega * (double)t;
      p.Om = d->omega;
      break;
    case ORA_MOTION_OSCILLATE: {
      double ph = (2.0 * ORA_PI) * (double)t / d->period;
      double s = sin(ph), c = cos(ph);
      for (int a = 0; a < 3; ++a) {
        p.X[a] = d->c0[a] + d->amp[a] * s;
        p.V[a] = d->amp[a] * ((2.0 * ORA_PI) / d->period) * c;
      }
      break;
    }
    case ORA_MOTION_TABLE: {
      int64_t k = t < b->d.table_count ? t : b->d.table_count - 1;
      const double* r = b->table + 8 * k;
      for (int a = 0; a < 3; ++a) p.X[a] = r[a];
      p.theta = r[3];
      for (int a = 0; a < 3; ++a) p.V[a] = r[4 + a];
      p.Om = r[7];
      break;
    }
    default:
      break;
  }
  p.ct = cos(p.theta);
  p.st = sin(p.theta);
  return p;
}

/* Shape function phi: solid iff phi <= 0 (reading: closed set, so a node
 * exactly on the surface is solid and Delta lies in (0,1]). */
static double body_phi(const body_t* b, const pose_t* p, int D, const double x[3]) {
  double dx = x[0] - p->X[0], dy = x[1] - p->X[1], dz = x[2] - p->X[2];
  double R = b->d.axes[0];
  switch (b->d.shape) {
    case ORA_SHAPE_CIRCLE: {
      double r2 = (D == 3) ? dx * dx + dy * dy + dz * dz : dx * dx + dy * dy;
      return r2 - R * R;
    }
    case ORA_SHAPE_OUTER_CIRCLE: {
      double r2 = (D == 3) ? dx * dx + dy * dy + dz * dz : dx * dx + dy * dy;
      return R * R - r2;
    }
    default: { /* ellipse / ellipsoid, rotated by theta about z */
      double xi = p->ct * dx + p->st * dy;
      double eta = p->ct * dy - p->st * dx;
      if (D == 3) return xi * xi * b->ia2 + eta * eta * b->ib2 + dz * dz * b->ic2 - 1.0;
      return xi * xi * b->ia2 + eta * eta * b->ib2 - 1.0;
    }
  }
}

/* Fractional distance Delta = |x_F - x_B| / |x_F - x_A| (Sec. II.A), the
 * root of phi along x_F - s*c_i, s in (0,1]. Along the link phi is the
 * quadratic A s^2 + 2 B s + C with C = phi(x_F) > 0; the root in (0,1] is
 * C / (-B + sqrt(B^2 - A C)), a form without cancellation. */
static double link_delta(const body_t* b, const pose_t* p, int D, const double xF[3], const int ci[3]) {
  double dx = xF[0] - p->X[0], dy = xF[1] - p->X[1], dz = xF[2] - p->X[2];
  double cx = ci[0], cy = ci[1], cz = ci[2];
  double A, B;
  double C = body_phi(b, p, D, xF);
  switch (b->d.shape) {
    case ORA_SHAPE_CIRCLE:
      A = (D == 3) ? cx * cx + cy * cy + cz * cz : cx * cx + cy * cy;
      B = -((D == 3) ? dx * cx + dy * cy + dz * cz : dx * cx + dy * cy);
      break;
    case ORA_SHAPE_OUTER_CIRCLE:
      A = -((D == 3) ? cx * cx + cy * cy + cz * cz : cx * cx + cy * cy);
      B = (D == 3) ? dx * cx + dy * cy + dz * cz : dx * cx + dy * cy;
      break;
    default: {
      double xi = p->ct * dx + p->st * dy;
      double eta = p->ct * dy - p->st * dx;
      double xic = p->ct * cx + p->st * cy;
      double etac = p->ct * cy - p->st * cx;
      if (D == 3) {
        A = xic * xic * b->ia2 + etac * etac * b->ib2 + cz * cz * b->ic2;
        B = -(xi * xic * b->ia2 + eta * etac * b->ib2 + dz * cz * b->ic2);
      } else {
        A = xic * xic * b->ia2 + etac * etac * b->ib2;
        B = -(xi * xic * b->ia2 + eta * etac * b->ib2);
      }
      break;
    }
  }
  double disc = B * B - A * C;
  if (disc < 0.0) disc = 0.0;
  double s = C / (-B + sqrt(disc));
  if (s > 1.0) s = 1.0;
  return s;
}

/* velocity of the body surface point x: V + Omega e_z x (x - X) */
static void surface_velocity(const pose_t* p, const double x[3], double u[3]) {
  u[0] = p->V[0] - p->Om * (x[1] - p->X[1]);
  u[1] = p->V[1] + p->Om * (x[0] - p->X[0]);
  u[2] = p->V[2];
}

/* ---------------------------------------------------------------------- */
/* Domain */

enum { T_FLUID = 0, T_WALL = 1, T_BODY0 = 2 };
enum { S_INLET = -2, S_OUTLET = -3, S_OUTLET_VEL = -4, S_ZOUHE = -5 };

struct ora_dom {
  lattice_t L;
  int nx, ny, nz;
  int64_t N;
  double tau, rho0;
  int eq;
  int face[6];
  int prof;
  double uin;
  double *f, *fpost, *fnew, *rho, *u;
  int32_t* type;
  unsigned char* solid_new;
  unsigned char* collided; /* node whose populations are already post-collision */
  unsigned char* solid_pred; /* solid set at a free body's predicted pose */
  body_t body[ORA_MAX_BODIES];
  int64_t t;
  int64_t rec_cap;
  double* rec[ORA_MAX_BODIES];
  double* face_rec;
  int error;
};

static int64_t node_index(const ora_dom* d, int x, int y, int z) {
  return (int64_t)x + (int64_t)d->nx * ((int64_t)y + (int64_t)d->ny * z);
}
static void node_pos(const ora_dom* d, int64_t n, int q[3]) {
  q[0] = (int)(n % d->nx);
  q[1] = (int)((n / d->nx) % d->ny);
  q[2] = (int)(n / ((int64_t)d->nx * d->ny));
}

/* Classify the lattice point q (at most one cell outside the box): periodic
 * axes wrap; a point in a wall layer is a wall; otherwise a point beyond -x is
 * the inlet and beyond +x the outlet; inside, the node type decides. Reading:
 * wall layers extend across the inlet/outlet planes and take precedence. */
static int classify(const ora_dom* d, int q[3], int64_t* n) {
  int dims[3] = {d->nx, d->ny, d->nz};
  for (int a = 0; a < d->L.D; ++a)
    if (d->face[2 * a] == ORA_FACE_PERIODIC) q[a] = (q[a] + dims[a]) % dims[a];
  for (int a = 0; a < d->L.D; ++a) {
    if (d->face[2 * a] == ORA_FACE_WALL && q[a] <= 0) return T_WALL;
    if (d->face[2 * a + 1] == ORA_FACE_WALL && q[a] >= dims[a] - 1) return T_WALL;
  }
  if (q[0] < 0) return d->face[0] >= ORA_FACE_ZOUHE_VELOCITY ? S_ZOUHE : S_INLET;
  if (q[0] >= d->nx) {
    if (d->face[1] >= ORA_FACE_ZOUHE_VELOCITY) return S_ZOUHE;
    return d->face[1] == ORA_FACE_OUTLET_VELOCITY ? S_OUTLET_VEL : S_OUTLET;
  }
  *n = node_index(d, q[0], q[1], q[2]);
  return d->type[*n];
}

/* Equilibrium: truncated Maxwellian of Eq. Fillipova_equilibrium
 * w_i rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u); with the quasi-incompressible
 * option of Sec. II (He & Luo) the velocity terms carry rho0 instead. */
static double feq_i(const ora_dom* d, int i, double rho, const double u[3]) {
  const lattice_t* L = &d->L;
  double cu = L->c[i][0] * u[0] + L->c[i][1] * u[1] + L->c[i][2] * u[2];
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  double poly = 3.0 * cu + 4.5 * cu * cu - 1.5 * uu;
  if (d->eq == ORA_EQ_HELUO) return L->w[i] * (rho + d->rho0 * poly);
  return L->w[i] * rho * (1.0 + poly);
}

/* Moments, Eqs. LBMmacroscopics_0 and _1: rho = sum f, rho u = sum c f
 * (u = j / rho0 in the quasi-incompressible option). */
static void moments(const ora_dom* d, const double* fn, double* rho, double u[3]) {
  const lattice_t* L = &d->L;
  double r = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < L->Q; ++i) {
    r += fn[i];
    for (int a = 0; a < 3; ++a) j[a] += L->c[i][a] * fn[i];
  }
  *rho = r;
  double den = (d->eq == ORA_EQ_HELUO) ? d->rho0 : r;
  for (int a = 0; a < 3; ++a) u[a] = j[a] / den;
}

/* density multiplying the velocity in the wall term and in g: rho(x_F) for
 * the standard equilibrium, rho0 for the quasi-incompressible one (reading,
 * chosen so that a uniform flow past a body moving with it is exact). */
static double wall_density(const ora_dom* d, double rhoF) {
  return d->eq == ORA_EQ_HELUO ? d->rho0 : rhoF;
}

static int check_faces(const ora_desc* ds) {
  int D = ds->lattice == ORA_D3Q19 ? 3 : 2;
  for (int a = 0; a < 3; ++a) {
    int lo = ds->face[2 * a], hi = ds->face[2 * a + 1];
    if (a >= D) continue;
    if (lo < 0 || lo > ORA_FACE_ZOUHE_PRESSURE || hi < 0 || hi > ORA_FACE_ZOUHE_PRESSURE) return -1;
    if ((lo == ORA_FACE_PERIODIC) != (hi == ORA_FACE_PERIODIC)) return -1;
    if (a > 0 && (lo >= ORA_FACE_ZOUHE_VELOCITY || hi >= ORA_FACE_ZOUHE_VELOCITY)) return -1;
    if (lo == ORA_FACE_OUTLET || lo == ORA_FACE_OUTLET_VELOCITY || hi == ORA_FACE_INLET) return -1;
    if (a > 0 && (lo == ORA_FACE_INLET || hi == ORA_FACE_OUTLET || hi == ORA_FACE_OUTLET_VELOCITY)) return -1;
  }
  return 0;
}

ora_dom* ora_create(const ora_desc* ds) {
  if (!ds || check_faces(ds) != 0) return NULL;
  ora_dom* d = (ora_dom*)calloc(1, sizeof(ora_dom));
  if (lattice_init(&d->L, ds->lattice) != 0) {
    free(d);
    return NULL;
  }
  d->nx = ds->nx;
  d->ny = ds->ny;
  d->nz = d->L.D == 3 ? ds->nz : 1;
  d->N = (int64_t)d->nx * d->ny * d->nz;
  d->tau = ds->tau;
  d->rho0 = ds->rho0;
  d->eq = ds->eq_model;
  for (int k = 0; k < 6; ++k) d->face[k] = ds->face[k];
  if (d->L.D == 2) d->face[4] = d->face[5] = ORA_FACE_PERIODIC;
  d->prof = ds->inlet_profile;
  d->uin = ds->inlet_u;
  int Q = d->L.Q;
  d->f = (double*)malloc(sizeof(double) * d->N * Q);
  d->fpost = (double*)malloc(sizeof(double) * d->N * Q);
  d->fnew = (double*)malloc(sizeof(double) * d->N * Q);
  d->rho = (double*)malloc(sizeof(double) * d->N);
  d->u = (double*)malloc(sizeof(double) * d->N * 3);
  d->type = (int32_t*)malloc(sizeof(int32_t) * d->N);
  d->solid_new = (unsigned char*)malloc(d->N);
  d->collided = (unsigned char*)calloc((size_t)d->N, 1);
  d->solid_pred = (unsigned char*)calloc((size_t)d->N, 1);
  if (!d->f || !d->fpost || !d->fnew || !d->rho || !d->u || !d->type || !d->solid_new || !d->collided ||
      !d->solid_pred) {
    ora_destroy(d);
    return NULL;
  }
  int dims[3] = {d->nx, d->ny, d->nz};
  for (int64_t n = 0; n < d->N; ++n) {
    int q[3];
    node_pos(d, n, q);
    d->type[n] = T_FLUID;
    for (int a = 0; a < d->L.D; ++a) {
      if (d->face[2 * a] == ORA_FACE_WALL && q[a] == 0) d->type[n] = T_WALL;
      if (d->face[2 * a + 1] == ORA_FACE_WALL && q[a] == dims[a] - 1) d->type[n] = T_WALL;
    }
    double rho = ds->init_rho ? ds->init_rho[n] : ds->rho0;
    double u[3] = {0.0, 0.0, 0.0};
    if (ds->init_u)
      for (int a = 0; a < 3; ++a) u[a] = ds->init_u[3 * n + a];
    if (d->L.D == 2) u[2] = 0.0;
    for (int i = 0; i < Q; ++i)
      d->f[n * Q + i] = (d->type[n] == T_FLUID) ? feq_i(d, i, rho, u) : NAN;
  }
  d->t = 0;
  return d;
}

void ora_destroy(ora_dom* d) {
  if (!d) return;
  free(d->f);
  free(d->fpost);
  free(d->fnew);
  free(d->rho);
  free(d->u);
  free(d->type);
  free(d->solid_new);
  free(d->collided);
  free(d->solid_pred);
  for (int b = 0; b < ORA_MAX_BODIES; ++b) {
    free(d->body[b].table);
    free(d->body[b].traj);
    free(d->rec[b]);
  }
  free(d->face_rec);
  free(d);
}

int64_t ora_time(const ora_dom* d) { return d->t; }

int ora_nthreads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int ora_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

static int ensure_records(ora_dom* d, int64_t upto) {
  if (upto <= d->rec_cap) return 0;
  int64_t cap = d->rec_cap ? d->rec_cap : 1024;
  while (cap < upto) cap *= 2;
  for (int b = 0; b < ORA_MAX_BODIES; ++b) {
    if (!d->body[b].active) continue; /* allocated when the body is placed */
    double* r = (double*)realloc(d->rec[b], sizeof(double) * ORA_REC_LEN * cap);
    if (!r) return -1;
    memset(r + ORA_REC_LEN * d->rec_cap, 0, sizeof(double) * ORA_REC_LEN * (cap - d->rec_cap));
    d->rec[b] = r;
  }
  double* r = (double*)realloc(d->face_rec, sizeof(double) * ORA_FACE_REC_LEN * cap);
  if (!r) return -1;
  memset(r + ORA_FACE_REC_LEN * d->rec_cap, 0, sizeof(double) * ORA_FACE_REC_LEN * (cap - d->rec_cap));
  d->face_rec = r;
  d->rec_cap = cap;
  return 0;
}

int ora_set_body(ora_dom* d, int id, const ora_body_desc* bd) {
  if (!d || id < 0 || id >= ORA_MAX_BODIES || !bd) return -1;
  body_t* b = &d->body[id];
  if (b->active) return -1;
  b->d = *bd;
  b->table = NULL;
  if (bd->motion == ORA_MOTION_TABLE) {
    if (!bd->table || bd->table_count <= 0) return -1;
    b->table = (double*)malloc(sizeof(double) * 8 * bd->table_count);
    memcpy(b->table, bd->table, sizeof(double) * 8 * bd->table_count);
  }
  b->d.table = NULL;
  b->traj = NULL;
  b->traj_n = b->traj_cap = 0;
  b->have_prev = 0;
  if (bd->motion == ORA_MOTION_FREE) {
    if (!(bd->mass > 0.0) || !(bd->inertia > 0.0)) return -1;
    b->traj_cap = 1024;
    b->traj = (pose_t*)calloc((size_t)b->traj_cap, sizeof(pose_t));
    if (!b->traj) return -1;
    pose_t* p0 = &b->traj[0];
    for (int a = 0; a < 3; ++a) {
      p0->X[a] = bd->c0[a];
      p0->V[a] = bd->vel[a];
    }
    if (d->L.D == 2) p0->X[2] = p0->V[2] = 0.0;
    p0->theta = bd->theta0;
    p0->Om = bd->omega;
    free_trig(p0->theta, &p0->ct, &p0->st);
    b->traj_t0 = d->t;
    b->traj_n = 1;
  }
  b->ia2 = 1.0 / (bd->axes[0] * bd->axes[0]);
  b->ib2 = 1.0 / (bd->axes[1] * bd->axes[1]);
  b->ic2 = (d->L.D == 3) ? 1.0 / (bd->axes[2] * bd->axes[2]) : 0.0;
  b->active = 1;
  if (d->rec_cap > 0) {
    d->rec[id] = (double*)calloc((size_t)ORA_REC_LEN * d->rec_cap, sizeof(double));
    if (!d->rec[id]) return -1;
  }
  pose_t p = body_pose(b, d->t);
  for (int64_t n = 0; n < d->N; ++n) {
    if (d->type[n] != T_FLUID) continue;
    int q[3];
    node_pos(d, n, q);
    double x[3] = {q[0], q[1], q[2]};
    if (body_phi(b, &p, d->L.D, x) <= 0.0) {
      d->type[n] = T_BODY0 + id;
      for (int i = 0; i < d->L.Q; ++i) d->f[n * d->L.Q + i] = NAN;
    }
  }
  return 0;
}

static void cross(const double r[3], const double m[3], double out[3]) {
  out[0] = r[1] * m[2] - r[2] * m[1];
  out[1] = r[2] * m[0] - r[0] * m[2];
  out[2] = r[0] * m[1] - r[1] * m[0];
}
static void acc3(double* dst, const double v[3], double sign) {
  for (int a = 0; a < 3; ++a) dst[a] += sign * v[a];
}

/* inlet velocity at the wall point x_B of an inlet link (wall at x = -1/2).
 * Parabolic profile: 4 u (p - 1/2)(n - 3/2 - p) / H^2 along every wall axis
 * (H = n - 2, the no-slip planes of halfway bounce-back on the wall layers at
 * index 0 and n-1). */
static double inlet_speed(const ora_dom* d, const double xB[3]) {
  double u = d->uin;
  if (d->prof == ORA_PROFILE_PARABOLIC) {
    int dims[3] = {d->nx, d->ny, d->nz};
    for (int a = 1; a < d->L.D; ++a) {
      if (d->face[2 * a] != ORA_FACE_WALL) continue;
      double H = dims[a] - 2.0;
      u *= 4.0 * (xB[a] - 0.5) * (dims[a] - 1.5 - xB[a]) / (H * H);
    }
  }
  return u;
}

/* The boundary-condition value of Eq. Fillipova_interpolation for the link
 * from the solid node x_F - c_i to the fluid node x_F, with the Mei-Luo-Shyy
 * choices of u_bf and chi. Halfway bounce-back is the same rule at
 * Delta = 1/2 (chi = 0). Reading: the moving-wall term is taken with the
 * outgoing direction, +6 w_i rho c_i.u_B, i.e. the opposite sign of the
 * printed formula (the printed sign, with the incoming direction, would drive
 * the fluid against the wall). */
static double body_link_value(const ora_dom* d, const body_t* b, const pose_t* p, int64_t nF,
                              const int xFi[3], int i, double fin, double* delta_out, double uB[3]) {
  const lattice_t* L = &d->L;
  const int* ci = L->c[i];
  double xF[3] = {xFi[0], xFi[1], xFi[2]};
  double delta = (b->d.bc == ORA_BC_MLS) ? link_delta(b, p, L->D, xF, ci) : 0.5;
  double xB[3];
  for (int a = 0; a < 3; ++a) xB[a] = xF[a] - delta * ci[a];
  surface_velocity(p, xB, uB);
  if (L->D == 2) uB[2] = 0.0;
  double rhoF = d->rho[nF];
  const double* uF = d->u + 3 * nF;
  double rw = wall_density(d, rhoF);
  double wall = 6.0 * L->w[i] * rw * (ci[0] * uB[0] + ci[1] * uB[1] + ci[2] * uB[2]);
  *delta_out = delta;
  if (b->d.bc == ORA_BC_HALFWAY) return fin + wall;
  double chi, ubf[3];
  if (delta >= 0.5) {
    for (int a = 0; a < 3; ++a) ubf[a] = uF[a] + (3.0 / (2.0 * delta)) * (uB[a] - uF[a]);
    chi = (2.0 * delta - 1.0) / (d->tau + 0.5);
  } else {
    /* u_bf = u(x_F + c_i); reading: fall back to u_F when that node is not fluid */
    int q[3] = {xFi[0] + ci[0], xFi[1] + ci[1], xFi[2] + ci[2]};
    int64_t nG = -1;
    if (classify(d, q, &nG) == T_FLUID) {
      for (int a = 0; a < 3; ++a) ubf[a] = d->u[3 * nG + a];
    } else {
      for (int a = 0; a < 3; ++a) ubf[a] = uF[a];
    }
    chi = (2.0 * delta - 1.0) / (d->tau - 2.0);
  }
  /* fictitious equilibrium g_ibar of Eq. Fillipova_equilibrium, direction c_ibar = -c_i */
  double cb_ubf = -(ci[0] * ubf[0] + ci[1] * ubf[1] + ci[2] * ubf[2]);
  double cb_uF = -(ci[0] * uF[0] + ci[1] * uF[1] + ci[2] * uF[2]);
  double uFuF = uF[0] * uF[0] + uF[1] * uF[1] + uF[2] * uF[2];
  double poly = 3.0 * cb_ubf + 4.5 * cb_uF * cb_uF - 1.5 * uFuF;
  double g = (d->eq == ORA_EQ_HELUO) ? L->w[i] * (rhoF + d->rho0 * poly) : L->w[i] * rhoF * (1.0 + poly);
  return (1.0 - chi) * fin + chi * g + wall;
}

/* The refill of Lallemand & Luo for a node x that a moving body uncovers:
 * every population by quadratic extrapolation along the lattice direction c
 * closest to the body's outward normal at x, from nodes fluid at t and at
 * t+1. Reading: the extrapolation acts on post-collision populations of
 * step t+1, fhat_i(x) = 3 fhat_i(x + c) - 3 fhat_i(x + 2c) + fhat_i(x + 3c)
 * with fhat = f - (f - f^eq)/tau from each node's streamed populations, and
 * x keeps fhat(x) as its post-collision state (its next collision is
 * skipped): the state a fused stream-collide step stores, so that the GPU
 * path can apply the rule without reconstructing pre-collision values
 * (impossible at tau = 1). The normal is the gradient of the shape function
 * phi at x (pose t+1), n = (dx, dy, dz) for a circle/sphere, (xi ct ia2 -
 * eta st ib2, xi st ia2 + eta ct ib2, dz ic2) for an ellipse/ellipsoid; the
 * direction maximises (n . c) / |c| (ties: the smallest (cx, cy, cz) in
 * lexicographic order). Returns 0, leaving x alone, when one of the three
 * nodes is not fluid at both times or lies outside the box (the caller then
 * applies the mean rule). */
static int refill_extrapolate(ora_dom* d, const body_t* b, const pose_t* P, const int p[3],
                              const unsigned char* solid_next, double* out) {
  const lattice_t* L = &d->L;
  const int Q = L->Q, D = L->D;
  const double dx = p[0] - P->X[0], dy = p[1] - P->X[1], dz = D == 3 ? p[2] - P->X[2] : 0.0;
  double nv[3];
  if (b->d.shape == ORA_SHAPE_ELLIPSE) {
    const double xi = P->ct * dx + P->st * dy, eta = P->ct * dy - P->st * dx;
    nv[0] = xi * P->ct * b->ia2 - eta * P->st * b->ib2;
    nv[1] = xi * P->st * b->ia2 + eta * P->ct * b->ib2;
    nv[2] = dz * b->ic2;
  } else {
    const double sgn = b->d.shape == ORA_SHAPE_OUTER_CIRCLE ? -1.0 : 1.0;
    nv[0] = sgn * dx;
    nv[1] = sgn * dy;
    nv[2] = sgn * dz;
  }
  int best = -1;
  double best_s = 0.0;
  for (int i = 1; i < Q; ++i) {
    const int* c = L->c[i];
    const int diag = c[0] * c[0] + c[1] * c[1] + c[2] * c[2] == 2;
    const double sc = (nv[0] * c[0] + nv[1] * c[1] + nv[2] * c[2]) * (diag ? 0.70710678118654757 : 1.0);
    if (best < 0 || sc > best_s) {
      best = i;
      best_s = sc;
    } else if (sc == best_s) {
      const int* cb = L->c[best];
      if (c[0] < cb[0] || (c[0] == cb[0] && (c[1] < cb[1] || (c[1] == cb[1] && c[2] < cb[2])))) best = i;
    }
  }
  int64_t m[3];
  const int dims[3] = {d->nx, d->ny, d->nz};
  for (int k = 1; k <= 3; ++k) {
    int q[3] = {p[0] + k * L->c[best][0], p[1] + k * L->c[best][1], p[2] + k * L->c[best][2]};
    /* reading: the three nodes lie in the box itself (no periodic wrap) */
    for (int a = 0; a < D; ++a)
      if (q[a] < 0 || q[a] >= dims[a]) return 0;
    if (classify(d, q, &m[k - 1]) != T_FLUID || solid_next[m[k - 1]] != 0) return 0;
  }
  double fh[3][32];
  for (int k = 0; k < 3; ++k) {
    double rho, u[3];
    const double* fk = d->fnew + m[k] * Q;
    moments(d, fk, &rho, u);
    for (int i = 0; i < Q; ++i) fh[k][i] = fk[i] - (fk[i] - feq_i(d, i, rho, u)) / d->tau;
  }
  for (int i = 0; i < Q; ++i) out[i] = (3.0 * fh[0][i] - 3.0 * fh[1][i]) + fh[2][i];
  return 1;
}

/* The populations body b's refill rule gives node p (index n), which it
 * uncovers on its way to pose P; solid_next: nonzero for every node solid at
 * that pose (any body). Returns 1 when they are post-collision values
 * (EXTRAPOLATE), 0 for pre-collision ones (the equilibria of MEAN/AIDUN). */
static int refill_values(ora_dom* d, const body_t* b, const pose_t* P, const int p[3],
                         const unsigned char* solid_next, double* out) {
  const lattice_t* L = &d->L;
  const int Q = L->Q, D = L->D;
  double rs = 0.0, us[3] = {0, 0, 0};
  int cnt = 0;
  for (int i = 1; i < Q; ++i) {
    int q[3] = {p[0] + L->c[i][0], p[1] + L->c[i][1], p[2] + L->c[i][2]};
    int64_t m = -1;
    if (classify(d, q, &m) != T_FLUID || solid_next[m] != 0) continue;
    double rho, u[3];
    moments(d, d->fnew + m * Q, &rho, u);
    rs += rho;
    for (int a = 0; a < 3; ++a) us[a] += u[a];
    cnt++;
  }
  if (b->d.refill == ORA_REFILL_EXTRAPOLATE && refill_extrapolate(d, b, P, p, solid_next, out)) return 1;
  double rb, ub[3];
  double x[3] = {p[0], p[1], p[2]};
  if (cnt > 0) {
    rb = rs / cnt;
    for (int a = 0; a < 3; ++a) ub[a] = us[a] / cnt;
  } else {
    rb = d->rho0;
    surface_velocity(P, x, ub);
  }
  if (b->d.refill == ORA_REFILL_AIDUN) surface_velocity(P, x, ub);
  if (D == 2) ub[2] = 0.0;
  for (int i = 0; i < Q; ++i) out[i] = feq_i(d, i, rb, ub);
  return 0;
}

/* The second approximation of Sec. III.B.3 for a free body: the covered and
 * uncovered nodes of step t are taken between pose t and the pose the body
 * would reach moving one step at its velocity of step t, X + V and
 * theta + Omega (cos/sin by free_trig), with the populations of t+1 after
 * streaming and the body's refill rule evaluated there without changing any
 * node: F_nodes = sum_{A+} c f - sum_{A-} c f_refill, the torque about X. */
static void predicted_node_terms(ora_dom* d, int b, const pose_t* P, double F[3], double T[3]) {
  const lattice_t* L = &d->L;
  const int Q = L->Q, D = L->D;
  const body_t* B = &d->body[b];
  pose_t Pp = *P;
  for (int a = 0; a < 3; ++a) Pp.X[a] = P->X[a] + P->V[a];
  Pp.theta = P->theta + P->Om;
  free_trig(Pp.theta, &Pp.ct, &Pp.st);
  unsigned char* pred = d->solid_pred;
  for (int64_t n = 0; n < d->N; ++n) {
    const int ty = d->type[n];
    pred[n] = (unsigned char)(ty >= T_BODY0 && ty != T_BODY0 + b);  /* other bodies where they are */
    if (ty == T_FLUID || ty == T_BODY0 + b) {
      int p[3];
      node_pos(d, n, p);
      double x[3] = {p[0], p[1], p[2]};
      if (body_phi(B, &Pp, D, x) <= 0.0) pred[n] = 1;
    }
  }
  for (int a = 0; a < 3; ++a) F[a] = T[a] = 0.0;
  double vals[32];
  for (int64_t n = 0; n < d->N; ++n) {
    const int ty = d->type[n];
    int sign = 0;
    if (ty == T_FLUID && pred[n]) sign = 1;                 /* covered */
    else if (ty == T_BODY0 + b && !pred[n]) sign = -1;       /* uncovered */
    if (!sign) continue;
    int p[3];
    node_pos(d, n, p);
    const double* f = d->fnew + n * Q;
    if (sign < 0) {
      refill_values(d, B, &Pp, p, pred, vals);
      f = vals;
    }
    double r[3] = {p[0] - P->X[0], p[1] - P->X[1], p[2] - P->X[2]};
    double mom[3] = {0, 0, 0}, tq[3];
    for (int i = 0; i < Q; ++i)
      for (int a = 0; a < 3; ++a) mom[a] += L->c[i][a] * f[i];
    cross(r, mom, tq);
    acc3(F, mom, (double)sign);
    acc3(T, tq, (double)sign);
  }
}

/* Newton-Euler step of a FREE body (Sec. IV: the flow force plus weight and
 * buoyancy move the body; forward Euler, or two-step Adams-Bashforth):
 * a = (F + F_ext) / M and alpha = (T_z + T_ext) / I from the flow force
 * and torque of step t, then V(t+1) = V(t) + a (AB2: + 3/2 a(t) - 1/2 a(t-1),
 * the first step Euler), X(t+1) = X(t) + V(t+1), and likewise Omega and
 * theta about z (reading: the position takes the new velocity, which makes
 * the covered/uncovered sets of step t depend on the force of step t, the
 * implicit case of Sec. III.B.3; the lattice-frame drive then takes one of
 * the paper's two approximations: Aidun et al.'s, the sets of the previous
 * step, F(t) = F_static(t) + [covered/uncovered terms of step t-1]; or the
 * sets of a predicted pose, see predicted_node_terms). Lattice units:
 * dt = 1. */
static pose_t integrate_free(body_t* b, const pose_t* P, const double F[3], double Tz, int D) {
  const ora_body_desc* bd = &b->d;
  double a[4];
  for (int k = 0; k < 3; ++k) a[k] = (F[k] + bd->ext_force[k]) / bd->mass;
  a[3] = (Tz + bd->ext_torque) / bd->inertia;
  if (D == 2) a[2] = 0.0;
  double dv[4];
  for (int k = 0; k < 4; ++k)
    dv[k] = (bd->integrator == ORA_INTEGRATOR_AB2 && b->have_prev) ? 1.5 * a[k] - 0.5 * b->a_prev[k] : a[k];
  pose_t q = *P;
  for (int k = 0; k < 3; ++k) {
    q.V[k] = P->V[k] + dv[k];
    q.X[k] = P->X[k] + q.V[k];
  }
  q.Om = P->Om + dv[3];
  q.theta = P->theta + q.Om;
  free_trig(q.theta, &q.ct, &q.st);
  for (int k = 0; k < 4; ++k) b->a_prev[k] = a[k];
  b->have_prev = 1;
  return q;
}

static void one_step(ora_dom* d) {
  const lattice_t* L = &d->L;
  const int Q = L->Q, D = L->D;
  const int64_t N = d->N;
  const int64_t t = d->t;
  pose_t P0[ORA_MAX_BODIES], P1[ORA_MAX_BODIES];
  for (int b = 0; b < ORA_MAX_BODIES; ++b)
    if (d->body[b].active) {
      P0[b] = body_pose(&d->body[b], t);
      P1[b] = body_pose(&d->body[b], t + 1);
    }
  double* rec[ORA_MAX_BODIES];
  for (int b = 0; b < ORA_MAX_BODIES; ++b) rec[b] = d->body[b].active ? d->rec[b] + ORA_REC_LEN * t : NULL;
  double* frec = d->face_rec + ORA_FACE_REC_LEN * t;

  /* 1. moments and collision on fluid nodes, Eq. collision */
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < N; ++n) {
    if (d->type[n] != T_FLUID) continue;
    double rho, u[3];
    moments(d, d->f + n * Q, &rho, u);
    d->rho[n] = rho;
    for (int a = 0; a < 3; ++a) d->u[3 * n + a] = u[a];
    if (d->collided[n]) { /* already post-collision (extrapolation refill) */
      for (int i = 0; i < Q; ++i) d->fpost[n * Q + i] = d->f[n * Q + i];
      d->collided[n] = 0;
      continue;
    }
    for (int i = 0; i < Q; ++i) {
      double fi = d->f[n * Q + i];
      d->fpost[n * Q + i] = fi - (fi - feq_i(d, i, rho, u)) / d->tau;
    }
  }

  /* 2. streaming between fluid nodes, Eq. streaming (push). Every slot of a
   *    fluid node starts as NaN so that a population nobody supplies shows. */
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < N; ++n)
    for (int i = 0; i < Q; ++i) d->fnew[n * Q + i] = NAN;
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < N; ++n) {
    if (d->type[n] != T_FLUID) continue;
    int p[3];
    node_pos(d, n, p);
    for (int i = 0; i < Q; ++i) {
      int q[3] = {p[0] + L->c[i][0], p[1] + L->c[i][1], p[2] + L->c[i][2]};
      int64_t m = -1;
      if (classify(d, q, &m) == T_FLUID) d->fnew[m * Q + i] = d->fpost[n * Q + i];
    }
  }

  /* 3. populations entering fluid nodes from non-fluid sources: the
   *    boundary links. For a body these are the gained sets G_i of Sec. III
   *    (x_F fluid, x_F - c_i inside the body); the ME sums follow
   *    Eqs. flow_force_2 and flow_torque_2, and the comoving-frame sums
   *    Eqs. ForceInMovementMovingFrame / TorqueInMovementMovingFrame.
   *    Reading of the latter's brackets: the leading minus covers only the
   *    outgoing term, F = sum [-(c_i - v) f_i(x_F - c_i) + (c_ibar - v) f_ibar(x_F)],
   *    which reduces to Eq. flow_force_2 at v = 0. */
  for (int64_t n = 0; n < N; ++n) {
    if (d->type[n] != T_FLUID) continue;
    int p[3];
    node_pos(d, n, p);
    for (int i = 1; i < Q; ++i) {
      const int* ci = L->c[i];
      int q[3] = {p[0] - ci[0], p[1] - ci[1], p[2] - ci[2]};
      int64_t m = -1;
      int s = classify(d, q, &m);
      if (s == T_FLUID || s == S_ZOUHE) continue; /* Zou-He: supplied in step 3b */
      double fin = d->fpost[n * Q + L->opp[i]]; /* post-collision population heading across the link */
      double fbc;
      double xF[3] = {p[0], p[1], p[2]};
      if (s >= T_BODY0) {
        int b = s - T_BODY0;
        const pose_t* P = &P0[b];
        double delta, uB[3];
        fbc = body_link_value(d, &d->body[b], P, n, p, i, fin, &delta, uB);
        double r[3] = {xF[0] - P->X[0], xF[1] - P->X[1], xF[2] - P->X[2]};
        double mom[3], tq[3];
        for (int a = 0; a < 3; ++a) mom[a] = -ci[a] * (fbc + fin);
        cross(r, mom, tq);
        acc3(rec[b] + ORA_REC_F_STATIC, mom, 1.0);
        acc3(rec[b] + ORA_REC_T_STATIC, tq, 1.0);
        for (int a = 0; a < 3; ++a) mom[a] = -(ci[a] - uB[a]) * fbc + (-ci[a] - uB[a]) * fin;
        cross(r, mom, tq);
        acc3(rec[b] + ORA_REC_F_COM, mom, 1.0);
        acc3(rec[b] + ORA_REC_T_COM, tq, 1.0);
      } else {
        int slot;
        if (s == T_WALL) {
          fbc = fin; /* halfway bounce-back at a resting wall */
          slot = 0;
        } else if (s == S_INLET || s == S_OUTLET_VEL) {
          /* velocity bounce-back at x = -1/2 (or x = nx - 1/2 for a velocity
             outlet): the halfway rule with the inlet profile as wall velocity */
          double xB[3] = {xF[0] - 0.5 * ci[0], xF[1] - 0.5 * ci[1], xF[2] - 0.5 * ci[2]};
          double ux = inlet_speed(d, xB);
          fbc = fin + 6.0 * L->w[i] * wall_density(d, d->rho[n]) * (ci[0] * ux);
          slot = (s == S_INLET) ? 6 : 12;
        } else {
          /* zero-gradient outlet: copy from the last column, shifted along the link */
          int o[3] = {d->nx - 1, q[1], q[2]};
          int64_t mo = node_index(d, o[0], o[1], o[2]);
          if (d->type[mo] != T_FLUID) d->error = 3;
          fbc = d->fpost[mo * Q + i];
          slot = 12;
        }
        double mom[3], tq[3];
        for (int a = 0; a < 3; ++a) mom[a] = -ci[a] * (fbc + fin);
        cross(xF, mom, tq);
        acc3(frec + slot, mom, 1.0);
        acc3(frec + slot + 3, tq, 1.0);
      }
      d->fnew[n * Q + i] = fbc;
    }
  }

  /* 3b. Zou-He faces (the boundary method the paper's Sec. IV names for its
   *     faces): at a fluid node of the x = 0 (x = nx-1) plane, every
   *     population with c_ix = +1 (-1) enters through the face and is
   *     rebuilt from the node's other populations, replacing what step 3 put
   *     there. The node is given u = (u_in, 0, 0) (velocity face; u_in the
   *     inlet profile at the node) or rho = rho0 with u_y = u_z = 0
   *     (pressure face); mass and x-momentum give the missing one. The
   *     normal population takes the bounce-back of its non-equilibrium part,
   *     f_i = f_ibar + f^eq_i - f^eq_ibar; each other unknown additionally
   *     takes -c_ia N_a per transverse axis a, with N_a solved from the
   *     node's a-momentum being rho_u u_a. Face momentum exchange is not
   *     recorded for these faces. */
  for (int side = 0; side < 2; ++side) {
    if (d->face[side] < ORA_FACE_ZOUHE_VELOCITY) continue;
    const int sgn = side == 0 ? 1 : -1, x = side == 0 ? 0 : d->nx - 1;
    for (int z = 0; z < d->nz; ++z)
      for (int y = 0; y < d->ny; ++y) {
        int64_t n = node_index(d, x, y, z);
        if (d->type[n] != T_FLUID) continue;
        double* fn = d->fnew + n * Q;
        int known[32];
        for (int i = 0; i < Q; ++i) known[i] = L->c[i][0] != sgn;
        /* sums over the known populations */
        double K = 0.0, Kx = 0.0;
        for (int i = 0; i < Q; ++i)
          if (known[i]) {
            K += fn[i];
            Kx += L->c[i][0] * fn[i];
          }
        /* rho = K + U and j_x = Kx + sgn U, U the sum of the unknowns */
        double rho, u[3] = {0.0, 0.0, 0.0};
        if (d->face[side] == ORA_FACE_ZOUHE_VELOCITY) {
          double xn[3] = {x, y, z};
          u[0] = inlet_speed(d, xn);
          if (d->eq == ORA_EQ_HELUO) rho = K + sgn * (d->rho0 * u[0] - Kx);  /* j_x = rho0 u_x */
          else rho = (K - sgn * Kx) / (1.0 - sgn * u[0]);                    /* j_x = rho u_x */
        } else {
          rho = d->rho0;
          double jx = Kx + sgn * (rho - K);
          u[0] = jx / (d->eq == ORA_EQ_HELUO ? d->rho0 : rho);
        }
        for (int i = 0; i < Q; ++i)
          if (!known[i]) {
            int ib = L->opp[i];
            fn[i] = fn[ib] + feq_i(d, i, rho, u) - feq_i(d, ib, rho, u);
          }
        const double rho_u = d->eq == ORA_EQ_HELUO ? d->rho0 : rho;
        for (int a = 1; a < D; ++a) {
          double ja = 0.0, cc = 0.0;
          for (int i = 0; i < Q; ++i) {
            ja += L->c[i][a] * fn[i];
            if (!known[i]) cc += L->c[i][a] * L->c[i][a];
          }
          double N = (ja - rho_u * u[a]) / cc;
          for (int i = 0; i < Q; ++i)
            if (!known[i]) fn[i] -= L->c[i][a] * N;
        }
      }
  }

  /* 3c. FREE bodies: the pose of t+1 from the flow force of step t */
  for (int b = 0; b < ORA_MAX_BODIES; ++b) {
    body_t* B = &d->body[b];
    if (!B->active || B->d.motion != ORA_MOTION_FREE) continue;
    double F[3], Tz;
    if (B->d.drive == ORA_DRIVE_COMOVING) {
      for (int a = 0; a < 3; ++a) F[a] = rec[b][ORA_REC_F_COM + a];
      Tz = rec[b][ORA_REC_T_COM + 2];
    } else {
      for (int a = 0; a < 3; ++a) F[a] = rec[b][ORA_REC_F_STATIC + a];
      Tz = rec[b][ORA_REC_T_STATIC + 2];
      if (B->d.drive == ORA_DRIVE_LATTICE && B->d.sets == ORA_SETS_PREDICTED) {
        double Fp[3], Tp[3];
        predicted_node_terms(d, b, &P0[b], Fp, Tp);
        for (int a = 0; a < 3; ++a) F[a] += Fp[a];
        Tz += Tp[2];
      } else if (B->d.drive == ORA_DRIVE_LATTICE && t - 1 >= B->traj_t0) {
        const double* prev = d->rec[b] + ORA_REC_LEN * (t - 1);
        for (int a = 0; a < 3; ++a) F[a] += prev[ORA_REC_F_IMP + a];
        Tz += prev[ORA_REC_T_IMP + 2];
      }
    }
    if (B->traj_n == B->traj_cap) {
      pose_t* nt = (pose_t*)realloc(B->traj, sizeof(pose_t) * (size_t)(2 * B->traj_cap));
      if (!nt) {
        d->error = 5;
        return;
      }
      B->traj = nt;
      B->traj_cap *= 2;
    }
    P1[b] = integrate_free(B, &P0[b], F, Tz, D);
    for (int a = 0; a < 3; ++a) P1[b].drive[a] = F[a];
    P1[b].drive[3] = Tz;
    B->traj[B->traj_n++] = P1[b];
  }

  /* 4. moving bodies: covered nodes A+ (fluid at t, solid at t+1) and
   *    uncovered nodes A- (solid at t, fluid at t+1), Sec. III.B.3, taken
   *    forward in time (pose t -> pose t+1; explicit for prescribed motion).
   *    Uncovered nodes are refilled by the body's rule (Sec. III.B.3 names
   *    three): MEAN, the equilibrium at the mean density and mean velocity
   *    of their lattice neighbours that are fluid at both t and t+1 (the
   *    paper's own rule; reading: unweighted means of their t+1 moments;
   *    with no such neighbour, rho0 and the surface velocity); AIDUN, the
   *    equilibrium at that mean density and the surface velocity at the node
   *    (reading of Aidun et al.'s rule); EXTRAPOLATE, Lallemand & Luo's
   *    extrapolation (refill_extrapolate; MEAN where it cannot apply). The
   *    impulsive terms of Eqs. ForceInMovement and
   *    TorqueInMovement are + sum_{A+} c_i f_i(t+1) - sum_{A-} c_i f_i(t+1),
   *    with the lever arm about the body centre X_c(t). */
  memset(d->solid_new, 0, (size_t)N);
  for (int b = 0; b < ORA_MAX_BODIES; ++b) {
    if (!d->body[b].active || d->body[b].d.motion == ORA_MOTION_STATIC) continue;
    for (int64_t n = 0; n < N; ++n) {
      if (d->type[n] == T_WALL) continue;
      int p[3];
      node_pos(d, n, p);
      double x[3] = {p[0], p[1], p[2]};
      if (body_phi(&d->body[b], &P1[b], D, x) <= 0.0) d->solid_new[n] = (unsigned char)(1 + b);
    }
  }
  for (int b = 0; b < ORA_MAX_BODIES; ++b) {
    if (!d->body[b].active) continue;
    int moving = d->body[b].d.motion != ORA_MOTION_STATIC;
    double np = 0.0, nm = 0.0;
    if (moving) {
      for (int64_t n = 0; n < N; ++n) {
        int was = d->type[n] == T_BODY0 + b;
        int will = d->solid_new[n] == 1 + b;
        if (d->type[n] == T_FLUID && will) { /* covered */
          int p[3];
          node_pos(d, n, p);
          double r[3] = {p[0] - P0[b].X[0], p[1] - P0[b].X[1], p[2] - P0[b].X[2]};
          double mom[3] = {0, 0, 0}, tq[3];
          for (int i = 0; i < Q; ++i)
            for (int a = 0; a < 3; ++a) mom[a] += L->c[i][a] * d->fnew[n * Q + i];
          cross(r, mom, tq);
          acc3(rec[b] + ORA_REC_F_IMP, mom, 1.0);
          acc3(rec[b] + ORA_REC_T_IMP, tq, 1.0);
          np += 1.0;
        } else if (was && !will) { /* uncovered */
          if (d->solid_new[n] != 0) d->error = 4; /* would enter another body */
          int p[3];
          node_pos(d, n, p);
          double vals[32];
          if (refill_values(d, &d->body[b], &P1[b], p, d->solid_new, vals)) d->collided[n] = 1;
          for (int i = 0; i < Q; ++i) d->fnew[n * Q + i] = vals[i];
          double r[3] = {p[0] - P0[b].X[0], p[1] - P0[b].X[1], p[2] - P0[b].X[2]};
          double mom[3] = {0, 0, 0}, tq[3];
          for (int i = 0; i < Q; ++i)
            for (int a = 0; a < 3; ++a) mom[a] += L->c[i][a] * d->fnew[n * Q + i];
          cross(r, mom, tq);
          acc3(rec[b] + ORA_REC_F_IMP, mom, -1.0);
          acc3(rec[b] + ORA_REC_T_IMP, tq, -1.0);
          nm += 1.0;
        }
      }
    }
    rec[b][ORA_REC_NPLUS] = np;
    rec[b][ORA_REC_NMINUS] = nm;
  }
  for (int64_t n = 0; n < N; ++n) {
    if (d->type[n] == T_FLUID && d->solid_new[n]) {
      d->type[n] = T_BODY0 + d->solid_new[n] - 1;
      for (int i = 0; i < Q; ++i) d->fnew[n * Q + i] = NAN;
    } else if (d->type[n] >= T_BODY0 && d->body[d->type[n] - T_BODY0].d.motion != ORA_MOTION_STATIC &&
               d->solid_new[n] == 0) {
      d->type[n] = T_FLUID;
    }
  }

  /* self-check: every population of every fluid node was supplied */
  for (int64_t n = 0; n < N; ++n) {
    if (d->type[n] != T_FLUID) continue;
    for (int i = 0; i < Q; ++i)
      if (isnan(d->fnew[n * Q + i])) d->error = 2;
  }
  double* tmp = d->f;
  d->f = d->fnew;
  d->fnew = tmp;
  d->t = t + 1;
}

int ora_step(ora_dom* d, int64_t nsteps) {
  if (!d) return -1;
  if (ensure_records(d, d->t + nsteps) != 0) return -1;
  for (int64_t s = 0; s < nsteps; ++s) {
    one_step(d);
    if (d->error) return -d->error;
  }
  return 0;
}

int ora_body_records(const ora_dom* d, int b, int64_t first, int64_t count, double* out) {
  if (!d || b < 0 || b >= ORA_MAX_BODIES || !d->body[b].active || first < 0 || first + count > d->t) return -1;
  if (count == 0) return 0;
  memcpy(out, d->rec[b] + ORA_REC_LEN * first, sizeof(double) * ORA_REC_LEN * count);
  return 0;
}

int ora_face_records(const ora_dom* d, int64_t first, int64_t count, double* out) {
  if (!d || first < 0 || first + count > d->t) return -1;
  memcpy(out, d->face_rec + ORA_FACE_REC_LEN * first, sizeof(double) * ORA_FACE_REC_LEN * count);
  return 0;
}

int64_t ora_links(const ora_dom* d, int b, int64_t cap, int64_t* node, int32_t* dir, double* delta) {
  if (!d || b < 0 || b >= ORA_MAX_BODIES || !d->body[b].active) return -1;
  const lattice_t* L = &d->L;
  pose_t P = body_pose(&d->body[b], d->t);
  int64_t k = 0;
  for (int64_t n = 0; n < d->N; ++n) {
    if (d->type[n] != T_FLUID) continue;
    int p[3];
    node_pos(d, n, p);
    for (int i = 1; i < L->Q; ++i) {
      int q[3] = {p[0] - L->c[i][0], p[1] - L->c[i][1], p[2] - L->c[i][2]};
      int64_t m = -1;
      if (classify(d, q, &m) != T_BODY0 + b) continue;
      if (k < cap) {
        double xF[3] = {p[0], p[1], p[2]};
        node[k] = n;
        dir[k] = i;
        delta[k] = (d->body[b].d.bc == ORA_BC_MLS) ? link_delta(&d->body[b], &P, L->D, xF, L->c[i]) : 0.5;
      }
      k++;
    }
  }
  return k;
}

int ora_body_pose(const ora_dom* d, int b, int64_t t, double* out) {
  if (!d || b < 0 || b >= ORA_MAX_BODIES || !d->body[b].active || t < 0) return -1;
  const body_t* B = &d->body[b];
  if (B->d.motion == ORA_MOTION_FREE && (t < B->traj_t0 || t >= B->traj_t0 + B->traj_n)) return -1;
  pose_t p = body_pose(&d->body[b], t);
  for (int a = 0; a < 3; ++a) out[a] = p.X[a];
  out[3] = p.theta;
  for (int a = 0; a < 3; ++a) out[4 + a] = p.V[a];
  out[7] = p.Om;
  return 0;
}

int ora_body_drive(const ora_dom* d, int b, int64_t t, double* out) {
  if (!d || b < 0 || b >= ORA_MAX_BODIES || !d->body[b].active) return -1;
  const body_t* B = &d->body[b];
  if (B->d.motion != ORA_MOTION_FREE || t < B->traj_t0 || t + 1 >= B->traj_t0 + B->traj_n) return -1;
  const pose_t* p = &B->traj[t + 1 - B->traj_t0];
  for (int a = 0; a < 4; ++a) out[a] = p->drive[a];
  return 0;
}

int ora_types(const ora_dom* d, int32_t* type) {
  memcpy(type, d->type, sizeof(int32_t) * d->N);
  return 0;
}

int ora_get_f(const ora_dom* d, double* f) {
  memcpy(f, d->f, sizeof(double) * d->N * d->L.Q);
  return 0;
}

int ora_fields(const ora_dom* d, double* rho, double* u) {
  for (int64_t n = 0; n < d->N; ++n) {
    if (d->type[n] != T_FLUID) {
      rho[n] = NAN;
      u[3 * n] = u[3 * n + 1] = u[3 * n + 2] = NAN;
      continue;
    }
    double r, v[3];
    moments(d, d->f + n * d->L.Q, &r, v);
    rho[n] = r;
    for (int a = 0; a < 3; ++a) u[3 * n + a] = v[a];
  }
  return 0;
}

int ora_lattice(int kind, int32_t* c, double* w, int32_t* opp) {
  lattice_t L;
  if (lattice_init(&L, kind) != 0) return -1;
  for (int i = 0; i < L.Q; ++i) {
    for (int a = 0; a < 3; ++a) c[3 * i + a] = L.c[i][a];
    w[i] = L.w[i];
    opp[i] = L.opp[i];
  }
  return L.Q;
}
