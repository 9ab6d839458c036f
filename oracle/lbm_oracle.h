/*
 * lbm_oracle.h -- TEST INFRASTRUCTURE. A plain, slow, FP64 CPU reference of
 * the lattice-Boltzmann time step with momentum-exchange (ME) force and torque
 * from Giovacchini & Ortiz, "Flow force and torque on submerged bodies in
 * lattice-Boltzmann via momentum exchange" (arXiv:1407.4524).
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library. The product path never links or calls it,
 * and this code shares nothing with the GPU path.
 *
 * Lattice units throughout (dx = dt = c = 1, so the factor dx^D/dt of the
 * paper's force sums equals 1). Forces are on the body, by the flow.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORA_D2Q9 = 0, ORA_D3Q19 = 1 };
enum { ORA_EQ_BGK = 0, ORA_EQ_HELUO = 1 };
enum { ORA_FACE_PERIODIC = 0, ORA_FACE_WALL = 1, ORA_FACE_INLET = 2, ORA_FACE_OUTLET = 3,
       ORA_FACE_OUTLET_VELOCITY = 4, ORA_FACE_ZOUHE_VELOCITY = 5, ORA_FACE_ZOUHE_PRESSURE = 6 };
enum { ORA_PROFILE_UNIFORM = 0, ORA_PROFILE_PARABOLIC = 1 };
enum { ORA_SHAPE_CIRCLE = 0, ORA_SHAPE_ELLIPSE = 1, ORA_SHAPE_OUTER_CIRCLE = 2 };
enum { ORA_BC_HALFWAY = 0, ORA_BC_MLS = 1 };
enum { ORA_MOTION_STATIC = 0, ORA_MOTION_CONST_VEL = 1, ORA_MOTION_ROTATE = 2,
       ORA_MOTION_OSCILLATE = 3, ORA_MOTION_TABLE = 4, ORA_MOTION_FREE = 5 };
/* which flow force moves a FREE body (the ME forms the paper compares in
   its Sec. IV sedimentation tests) */
enum { ORA_DRIVE_STATIC = 0, ORA_DRIVE_LATTICE = 1, ORA_DRIVE_COMOVING = 2 };
enum { ORA_INTEGRATOR_EULER = 0, ORA_INTEGRATOR_AB2 = 1 };
/* the covered/uncovered sets a free body moved by the lattice-frame force
   uses at step t (the two approximations of Sec. III.B.3) */
enum { ORA_SETS_PREVIOUS = 0, ORA_SETS_PREDICTED = 1 };
/* value given to the nodes a moving body uncovers */
enum { ORA_REFILL_MEAN = 0, ORA_REFILL_AIDUN = 1, ORA_REFILL_EXTRAPOLATE = 2 };

#define ORA_MAX_BODIES 64
/* per-step record of one body: see ORA_REC_* offsets */
#define ORA_REC_LEN 20
#define ORA_REC_F_STATIC 0   /* Eq. flow_force_2 */
#define ORA_REC_T_STATIC 3   /* Eq. flow_torque_2, about X_c(t) */
#define ORA_REC_F_IMP 6      /* covered/uncovered terms of Eq. ForceInMovement */
#define ORA_REC_T_IMP 9      /* covered/uncovered terms of Eq. TorqueInMovement */
#define ORA_REC_F_COM 12     /* Eq. ForceInMovementMovingFrame without its node terms */
#define ORA_REC_T_COM 15     /* Eq. TorqueInMovementMovingFrame without its node terms */
#define ORA_REC_NPLUS 18
#define ORA_REC_NMINUS 19
/* per-step record of the domain faces: F,T of walls, inlet, outlet (torque about the origin) */
#define ORA_FACE_REC_LEN 18

typedef struct {
  int32_t lattice;          /* ORA_D2Q9 | ORA_D3Q19 */
  int32_t nx, ny, nz;       /* nz = 1 for D2Q9 */
  double tau, rho0;
  int32_t eq_model;         /* ORA_EQ_BGK | ORA_EQ_HELUO */
  int32_t face[6];          /* -x,+x,-y,+y,-z,+z */
  int32_t inlet_profile;
  double inlet_u;
  const double* init_rho;   /* optional, nx*ny*nz, x fastest */
  const double* init_u;     /* optional, 3*nx*ny*nz, (ux,uy,uz) per node */
} ora_desc;

typedef struct {
  int32_t shape;
  double axes[3];           /* radius, or semi-axes a,b(,c) of the ellipse(oid) */
  int32_t bc;               /* ORA_BC_HALFWAY | ORA_BC_MLS */
  int32_t motion;
  double c0[3], theta0;     /* centre and orientation (about z) at t = 0 */
  double vel[3];            /* CONST_VEL velocity */
  double omega;             /* ROTATE angular speed (about z), rad/step */
  double amp[3], period;    /* OSCILLATE: X(t) = c0 + amp*sin(2*pi*t/period) */
  const double* table;      /* TABLE: 8 doubles per step: X[3], theta, V[3], Omega_z */
  int64_t table_count;
  /* FREE: Newton-Euler motion under the flow force plus a constant external
     force/torque, from X = c0, theta = theta0, V = vel, Omega = omega */
  double mass, inertia;     /* inertia about the z axis through X */
  double ext_force[3], ext_torque;
  int32_t drive;            /* ORA_DRIVE_* */
  int32_t integrator;       /* ORA_INTEGRATOR_* */
  int32_t refill;           /* ORA_REFILL_* (every moving body) */
  int32_t sets;             /* FREE with the lattice drive: ORA_SETS_* */
} ora_body_desc;

typedef struct ora_dom ora_dom;

ora_dom* ora_create(const ora_desc* d);
void ora_destroy(ora_dom* dom);
int ora_set_body(ora_dom* dom, int body_id, const ora_body_desc* b);
int ora_step(ora_dom* dom, int64_t nsteps);
int64_t ora_time(const ora_dom* dom);
int ora_nthreads(void);
/* threads of the bulk loops from now on (n > 0); returns the new count */
int ora_set_threads(int n);

/* records: rec[(step - first)*ORA_REC_LEN ...] for steps first..first+count-1 */
int ora_body_records(const ora_dom* dom, int body_id, int64_t first, int64_t count, double* rec);
int ora_face_records(const ora_dom* dom, int64_t first, int64_t count, double* rec);

/* links of body `body_id` at the current step, canonical order (node index, then i).
   node index = x + nx*(y + ny*z). Returns the count; writes at most cap entries. */
int64_t ora_links(const ora_dom* dom, int body_id, int64_t cap, int64_t* node, int32_t* dir, double* delta);

/* pose of body `body_id` at step t (the one the step of time t uses; for a
   FREE body t <= the current step + 1 once that step ran): out = X[3],
   theta, V[3], Omega_z */
int ora_body_pose(const ora_dom* dom, int body_id, int64_t t, double* out);

/* FREE body: the flow force (3) and torque z that moved it from step t to
   t+1 (the form its drive selects, before the external force) */
int ora_body_drive(const ora_dom* dom, int body_id, int64_t t, double* out);

/* node type: 0 fluid, 1 wall layer, 2+b body b */
int ora_types(const ora_dom* dom, int32_t* type);
/* current populations f[node*Q + i] (pre-collision, time t; a node just
   refilled by extrapolation holds its post-collision populations); solid
   nodes hold NaN */
int ora_get_f(const ora_dom* dom, double* f);
/* moments of the current populations; solid nodes get NaN */
int ora_fields(const ora_dom* dom, double* rho, double* u);
/* lattice tables in the oracle's numbering */
int ora_lattice(int lattice, int32_t* c /* Q*3 */, double* w /* Q */, int32_t* opp /* Q */);

#ifdef __cplusplus
}
#endif
#endif
