/*
 * lbm.h -- C ABI of the MI355X lattice-Boltzmann library with
 * momentum-exchange force and torque.
 *
 * The operation: the time step of the lattice-Boltzmann equation (BGK
 * collision then streaming, Sec. II, Eqs. LBE, collision, streaming) for a
 * flow around submerged bodies whose motion is prescribed (Sec. III: Omega(t)
 * is a given function of t, strictly inside the simulated region) or follows
 * from the computed force (Newton-Euler, the tests of Sec. IV), with the
 * interpolated boundary rule of Sec. II.A (Filippova-Haenel with the
 * Mei-Luo-Shyy choices; halfway bounce-back as the special case Delta = 1/2)
 * and the flow force and torque on each body by momentum exchange, every
 * step, in the three forms the paper derives:
 *   static     Eqs. flow_force_2 / flow_torque_2,
 *   lattice    Eqs. ForceInMovement / TorqueInMovement (static sums plus the
 *              covered/uncovered-node terms, sets taken forward in time, or
 *              backward in time as Aidun et al. and Wen et al. take them),
 *   comoving   Eqs. ForceInMovementMovingFrame / TorqueInMovementMovingFrame
 *              (node terms dropped).
 *
 * Units and signs: lattice units (dx = dt = 1). F is the force ON the body BY
 * the flow; T is the torque about the body centre X_c(t). In 2D only Fx, Fy
 * and Tz are non-zero.
 *
 * Lattices (numbering is part of this interface):
 *   D2Q9:  0 (0,0); 1 (1,0); 2 (0,1); 3 (-1,0); 4 (0,-1); 5 (1,1); 6 (-1,1);
 *          7 (-1,-1); 8 (1,-1). Weights 4/9, 1/9 (1..4), 1/36 (5..8).
 *   D3Q19: 0 rest; 1..6 = +x,-x,+y,-y,+z,-z; 7..18 = (1,1,0),(-1,-1,0),
 *          (1,-1,0),(-1,1,0),(1,0,1),(-1,0,-1),(1,0,-1),(-1,0,1),(0,1,1),
 *          (0,-1,-1),(0,1,-1),(0,-1,1). Weights 1/3, 1/18, 1/36.
 *
 * Geometry (part of this interface, so that the solid/fluid decision is
 * reproducible bit for bit): node (x,y,z) sits at the integer point
 * (x,y,z). With d = p - X(t), xi = ct*dx + st*dy, eta = ct*dy - st*dx
 * (ct = cos theta, st = sin theta), a node is solid iff phi <= 0 with
 *   CIRCLE (sphere in 3D):  phi = (dx*dx + dy*dy [+ dz*dz]) - R*R
 *   ELLIPSE (ellipsoid):    phi = xi*xi*ia2 + eta*eta*ib2 [+ dz*dz*ic2] - 1,
 *                           ia2 = 1/(a*a), ib2 = 1/(b*b), ic2 = 1/(c*c)
 *   OUTER_CIRCLE:           phi = R*R - (dx*dx + dy*dy [+ dz*dz])   (solid outside R)
 * every expression evaluated left to right in IEEE double without fused
 * multiply-add. Poses at integer step t (evaluated on the host, libm
 * sin/cos, same rules):
 *   STATIC     X = c0, theta = theta0
 *   CONST_VEL  X = c0 + vel*(double)t, V = vel
 *   ROTATE     theta = theta0 + omega*(double)t, Omega = omega (about z)
 *   OSCILLATE  ph = (2*pi)*(double)t/period; X = c0 + amp*sin(ph);
 *              V = amp*((2*pi)/period)*cos(ph)
 *   TABLE      rows of 8 doubles X[3], theta, V[3], Omega_z per step (the last
 *              row holds after the table ends)
 * The wall velocity at a point x is V + Omega e_z x (x - X).
 *
 * Free bodies (FREE; the sedimentation tests of Sec. IV): the flow force of
 * step t, in the form me_mode selects, plus ext_force and ext_torque, moves
 * the body by Newton-Euler about z: a = (F + ext_force)/mass (a_z = 0 in
 * 2D), alpha = (T_z + ext_torque)/inertia; EULER: dv = a, AB2: dv =
 * 1.5 a - 0.5 a_prev after the first step; V += dv, X += V (the new V),
 * Omega += dalpha, theta += Omega, each operation in that order in IEEE
 * double without fused multiply-add. With LBM_ME_LATTICE (or _BACKWARD) the
 * covered/uncovered terms come from the step before (the approximation of
 * Aidun et al. that Sec. III.B.3 describes, which keeps the step explicit)
 * or, with sets = LBM_SETS_PREDICTED, from a predicted pose (its second
 * approximation).
 * cos/sin of theta are not libm's: k = rint(theta * 0.63661977236758134),
 * r = (theta - k*1.5707963267948966) - k*6.123233995736766e-17, z = r*r,
 * then Horner through 1/17! (sin r = r + (r*z)*p(z)) and 1/18! (cos r =
 * 1 - z*q(z)), quadrant k mod 4. The node box of the new pose must stay
 * inside the interior and |V| below 0.5 (a sticky error otherwise; the body
 * then stops).
 *
 * Faces: -x,+x,-y,+y,-z,+z each PERIODIC (in pairs), WALL (the boundary
 * layer of nodes is solid; halfway bounce-back puts the no-slip plane half
 * way into it), INLET (-x only: velocity bounce-back at x = -1/2 with the
 * inlet profile), OUTLET (+x only: zero gradient, the incoming populations of
 * the last column copied from the column's own outgoing ones shifted along
 * the link) or OUTLET_VELOCITY (+x only: velocity bounce-back at
 * x = nx - 1/2), or, on either x face, ZOUHE_VELOCITY / ZOUHE_PRESSURE (the
 * face nodes x = 0 or nx - 1 are boundary nodes of Zou & He, the reference
 * the paper's Sec. IV set-up uses for its faces: after the pull, the
 * populations entering through the face are rebuilt from the node's others
 * by bounce-back of their non-equilibrium part with the transverse
 * correction, so that the node carries the inlet profile as velocity along x
 * (VELOCITY) or rho0 as density (PRESSURE), with no transverse velocity; on
 * an edge with a WALL face the wall's bounce-back supplies the populations
 * that cross only the wall). A parabolic profile is
 * 4 u (p - 1/2)(n - 3/2 - p)/(n-2)^2 along every WALL axis transverse to x,
 * taken at the wall point of a velocity bounce-back link, at the node itself
 * on a Zou-He face. Face records (face_records = 1) are not kept with a
 * Zou-He face.
 *
 * Ownership and threading: a domain owns its device arrays unless the caller
 * passes device_buffer, which then must outlive the domain. The caller owns
 * every host pointer; the library copies what it keeps. The stream is
 * borrowed. One thread per domain at a time. lbm_step only enqueues work
 * (see lbm_step for the one synchronisation of a domain with moving or
 * several bodies); errors raised on the device surface at the next call
 * that reads results (lbm_force_torque, lbm_records, lbm_get_*). Work the
 * caller enqueues on the stream after lbm_step sees the whole step (see
 * split_schedule for the second stream a domain may use).
 * No exception crosses this interface; every call returns lbm_status and
 * lbm_last_error() gives a thread-local message. An error a kernel reports
 * (instability, an overflowed link or node list, a body meeting a wall or
 * another body while it moves) is sticky: the results from then on are not
 * valid and every later call that synchronises reports it again; destroy the
 * domain. A placement that lbm_set_body finds invalid is undone instead (the
 * body id stays free, the domain usable).
 */
#ifndef LBM_H
#define LBM_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBM_OK = 0,
  LBM_E_INVAL = -1,    /* malformed descriptor or argument */
  LBM_E_NOMEM = -2,    /* device allocation failed or caller buffer too small */
  LBM_E_HIP = -3,      /* HIP runtime error */
  LBM_E_RANGE = -4,    /* body not strictly inside the domain, or record out of the ring */
  LBM_E_UNSTABLE = -5, /* a fluid node's |u| > 0.4 or not a number (flagged on the device by the
                          stream-collide update), or a non-finite force/torque or field */
  LBM_E_STATE = -6     /* call not valid in the current state (e.g. body id in use) */
} lbm_status;

enum { LBM_D2Q9 = 0, LBM_D3Q19 = 1 };
enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F16_SHIFTED = 2 };
enum { LBM_EQ_BGK = 0, LBM_EQ_HELUO = 1 };
enum { LBM_FACE_PERIODIC = 0, LBM_FACE_WALL = 1, LBM_FACE_INLET = 2, LBM_FACE_OUTLET = 3,
       LBM_FACE_OUTLET_VELOCITY = 4, LBM_FACE_ZOUHE_VELOCITY = 5, LBM_FACE_ZOUHE_PRESSURE = 6 };
enum { LBM_PROFILE_UNIFORM = 0, LBM_PROFILE_PARABOLIC = 1 };
enum { LBM_SHAPE_CIRCLE = 0, LBM_SHAPE_ELLIPSE = 1, LBM_SHAPE_OUTER_CIRCLE = 2 };
enum { LBM_BC_HALFWAY = 0, LBM_BC_MLS = 1 };
enum { LBM_ME_STATIC = 0, LBM_ME_LATTICE = 1, LBM_ME_COMOVING = 2, LBM_ME_LATTICE_BACKWARD = 3 };
enum { LBM_MOTION_STATIC = 0, LBM_MOTION_CONST_VEL = 1, LBM_MOTION_ROTATE = 2,
       LBM_MOTION_OSCILLATE = 3, LBM_MOTION_TABLE = 4, LBM_MOTION_FREE = 5 };
enum { LBM_INTEGRATOR_EULER = 0, LBM_INTEGRATOR_AB2 = 1 };
enum { LBM_REFILL_MEAN = 0, LBM_REFILL_AIDUN = 1, LBM_REFILL_EXTRAPOLATE = 2 };
enum { LBM_SETS_PREVIOUS = 0, LBM_SETS_PREDICTED = 1 };

#define LBM_MAX_BODIES 64
/* one per-step record of a body: 20 doubles */
#define LBM_REC_LEN 20
#define LBM_REC_F_STATIC 0 /* Fx,Fy,Fz of Eq. flow_force_2 */
#define LBM_REC_T_STATIC 3 /* Tx,Ty,Tz of Eq. flow_torque_2 */
#define LBM_REC_F_NODES 6  /* covered minus uncovered node momentum (Eq. ForceInMovement) */
#define LBM_REC_T_NODES 9  /* the same for the torque (Eq. TorqueInMovement) */
#define LBM_REC_F_COMOVING 12
#define LBM_REC_T_COMOVING 15
#define LBM_REC_N_COVERED 18
#define LBM_REC_N_UNCOVERED 19

typedef struct lbm_domain_s* lbm_domain;

typedef struct {
  int32_t lattice;          /* LBM_D2Q9 | LBM_D3Q19 */
  int32_t nx, ny, nz;       /* nodes per axis (nz ignored for D2Q9); each >= 3 */
  double tau;               /* BGK relaxation time, > 1/2 */
  double rho0;              /* reference density (rest equilibrium w_i rho0) */
  int32_t storage;          /* LBM_F64 | LBM_F32 | LBM_F16_SHIFTED; populations are stored
                               as deviations f_i - w_i rho0 in this type */
  int32_t eq_model;         /* LBM_EQ_BGK (standard) | LBM_EQ_HELUO (quasi-incompressible) */
  int32_t face[6];          /* -x,+x,-y,+y,-z,+z, LBM_FACE_* */
  int32_t inlet_profile;    /* LBM_PROFILE_* */
  double inlet_u;           /* uniform speed or peak of the parabola */
  const double* init_rho;   /* host, optional: nx*ny*nz densities, x fastest; NULL = rho0 */
  const double* init_u;     /* host, optional: 3 per node (ux,uy,uz); NULL = 0 */
  void* stream;             /* hipStream_t (borrowed); NULL = the default stream */
  void* device_buffer;      /* optional caller-owned device memory; NULL = library allocates */
  size_t device_buffer_bytes;
  int64_t record_capacity;  /* steps kept in each body's record ring; 0 = 65536 */
  int32_t split_schedule;   /* schedule of a domain with a single body (not FREE, not an outer
                               circle). Split: the update of the nodes away from the body
                               runs on a second stream the domain owns (default priority),
                               beside the body's link rule or advance and the update of a
                               near box around it on `stream`, and every call leaves `stream`
                               waiting for it. Plain: the link rule, the stream-collide
                               update and the advance one after another on `stream`.
                               0 (default): a moving body steps as a one-member batch (see
                               lbm_step), a body with fixed links in the plain schedule;
                               1: split; -1: plain. Results are bitwise the same in every
                               schedule. The split costs two cross-stream waits per step on
                               the host, and the far update loses bandwidth to the kernels
                               running beside it, which outweighs the overlap on the
                               domains measured */
  int32_t face_records;     /* 1: the momentum exchange of the domain faces is recorded every
                               step (lbm_face_records, lbm_force_torque with LBM_WALLS); one
                               small kernel per step over the face nodes. 0: not recorded */
  int32_t debug_poison;     /* 1: every population slot of a non-fluid node (wall layers, halo,
                               the solid nodes of a body placed by lbm_set_body) starts as NaN,
                               so a pull that reads a slot no boundary rule wrote shows up as
                               LBM_E_UNSTABLE; results are otherwise unchanged. 0: zeros */
  int32_t max_bodies;       /* body slots: ids 0 .. max_bodies-1 (0 = 4; at most
                               LBM_MAX_BODIES); the record ring keeps one record per slot
                               and step (max_bodies * 160 bytes per step of record_capacity) */
} lbm_domain_desc;

typedef struct {
  int32_t shape;            /* LBM_SHAPE_* */
  double axes[3];           /* radius, or semi-axes a, b (, c) */
  int32_t bc;               /* LBM_BC_HALFWAY | LBM_BC_MLS */
  int32_t me_mode;          /* which form lbm_force_torque returns (LBM_ME_*), and for a FREE
                               body the flow force that moves it */
  int32_t motion;           /* LBM_MOTION_* */
  double c0[3], theta0;
  double vel[3];            /* CONST_VEL velocity; FREE: initial velocity */
  double omega;             /* ROTATE angular speed; FREE: initial angular speed */
  double amp[3], period;
  const double* pose_table; /* TABLE: host rows of 8 doubles, copied */
  int64_t pose_count;
  /* FREE: mass, moment of inertia about z through X, and a constant external
     force and torque (weight minus buoyancy); see "Free bodies" above */
  double mass, inertia;
  double ext_force[3], ext_torque;
  int32_t integrator;       /* FREE: LBM_INTEGRATOR_EULER | LBM_INTEGRATOR_AB2 */
  int32_t refill;           /* moving bodies: LBM_REFILL_*, the value given to a node the body
                               uncovers (Sec. III.B.3): MEAN, the equilibrium at the mean density
                               and velocity of its neighbours fluid at t and t+1 (rho0 and the
                               wall velocity when there are none); AIDUN, the equilibrium at that
                               mean density and the wall velocity at the node; EXTRAPOLATE,
                               every population of the node's post-collision state of t+1 (what
                               a step stores) extrapolated quadratically from the post-collision
                               states of x+c, x+2c, x+3c, 3 f(x+c) - 3 f(x+2c) + f(x+3c),
                               along the lattice direction c that maximises
                               (n.c)/|c| for the outward normal n of the body at the node (the
                               gradient of phi, pose t+1: (dx,dy,dz) for a circle/sphere,
                               (xi ct ia2 - eta st ib2, xi st ia2 + eta ct ib2, dz ic2) for an
                               ellipse/ellipsoid, each left to right; ties to the smallest
                               (cx,cy,cz)), from nodes fluid at t and t+1, else MEAN */
  int32_t sets;             /* FREE with LBM_ME_LATTICE: the covered/uncovered sets of step t,
                               whose pose t+1 depends on that step's force (Sec. III.B.3's two
                               approximations): LBM_SETS_PREVIOUS, those of step t-1 (Aidun
                               et al.); LBM_SETS_PREDICTED, those between pose t and the pose
                               one step ahead at the velocity of step t (X + V, theta +
                               Omega), refilled by the body's rule without changing any node */
} lbm_body_desc;

/* Device bytes a domain with this descriptor needs (for admission by HBM
   footprint and for sizing device_buffer). Each body allocates its own link
   list and pose window at lbm_set_body on top of this: 24 bytes per link of
   capacity (about 16 (Q-1) pi (R+3) links in 2D, 16 (Q-1) pi (R+3)^2 in 3D)
   plus 128 bytes per step of an 8192-step window. */
lbm_status lbm_footprint_bytes(const lbm_domain_desc* desc, size_t* bytes);

/* Device bytes that lbm_set_body allocates for this body in a domain with
   this descriptor (link list, chunk sums, pose window): with
   lbm_footprint_bytes, the admission figure of a request. */
lbm_status lbm_body_footprint_bytes(const lbm_domain_desc* desc, const lbm_body_desc* body, size_t* bytes);

/* Creates the domain and initialises every node to the equilibrium at
   (init_rho, init_u) (Eq. Fillipova_equilibrium's truncated Maxwellian), step
   counter 0. Enqueued on desc->stream. */
lbm_status lbm_create_domain(const lbm_domain_desc* desc, lbm_domain* out);

/* Waits for the domain's stream and frees what the library allocated. */
lbm_status lbm_destroy_domain(lbm_domain dom);

/* Places body `body_id` (0..max_bodies-1 of the domain) at its pose of the
   current step: marks its nodes solid and builds its boundary-link list, the
   gained sets G_i of Sec. III.B (x_F fluid with x_F - c_i inside the body),
   with Delta per link (Sec. II.A). Its bounding box plus two nodes must stay
   inside the non-wall interior at every step that lbm_step reaches
   (LBM_E_RANGE otherwise), except for a static OUTER_CIRCLE. Several bodies
   of one domain (a suspension) are independent: each keeps its own links,
   records and advance. They must stay at least four nodes apart at every
   step (the interpolated rule reads two nodes out from the wall, the refill
   one node around a node that leaves a body, and bodies closer than that
   would make the result depend on the order in which their advances run);
   a body whose nodes meet another body's while it moves is reported as a
   sticky error. Synchronises the stream once. */
lbm_status lbm_set_body(lbm_domain dom, int32_t body_id, const lbm_body_desc* body);

/* Advances nsteps time steps. Enqueue only, except that a domain with two
   or more bodies, or with one body whose solid set moves (none of them
   FREE, no face records, not in a batch, split_schedule 0), is stepped as
   a one-member batch of the domain's own -- the link rule of every body
   with fixed links in one launch, the advance of every moving body in
   another, the nodes away from the bodies updated on a second stream beside
   the body work -- and such a call synchronises the stream once (the launch
   tables' upload). Results are the same bits either way. */
lbm_status lbm_step(lbm_domain dom, int64_t nsteps);

/* Blocks until the domain's queued work is done and reports device errors. */
lbm_status lbm_synchronize(lbm_domain dom);

/* Current step counter (number of steps taken). */
int64_t lbm_time(lbm_domain dom);

/* Force and torque on body `body_id` in its me_mode, for steps
   first_step..first_step+count-1: ft[6*k..6*k+5] = Fx,Fy,Fz,Tx,Ty,Tz.
   LBM_ME_LATTICE_BACKWARD: the static terms of step t plus the covered/
   uncovered terms of step t-1 (nodes that changed between t-1 and t, the
   sets of Aidun et al. and Wen et al. that Sec. III.B.3 contrasts with its
   own forward-in-time sets; zero before the first step).
   body_id LBM_WALLS: the force and torque (about the origin) on the wall
   layers of a domain with face_records (see lbm_face_records).
   Synchronises. LBM_E_RANGE if a step is not in the record ring. */
lbm_status lbm_force_torque(lbm_domain dom, int32_t body_id, int64_t first_step, int64_t count,
                            double* ft);

/* Pose of body `body_id` at steps first_step..first_step+count-1:
   out[8*k ...] = X[3], theta, V[3], Omega_z, for a FREE body from the ring
   its integration fills (steps within record_capacity of the current one,
   up to the current step), for a prescribed motion from its definition.
   Synchronises. LBM_E_RANGE outside that span. */
lbm_status lbm_body_trajectory(lbm_domain dom, int32_t body_id, int64_t first_step, int64_t count,
                               double* out);

/* Full per-step records (LBM_REC_LEN doubles each, layout LBM_REC_*). */
lbm_status lbm_records(lbm_domain dom, int32_t body_id, int64_t first_step, int64_t count,
                       double* rec);

/* The covered (A+, fluid at t and solid at t+1) and uncovered (A-, solid at t
   and fluid at t+1) node counts of body `body_id` between steps `step` and
   step+1 (Sec. III.B.3, the sets of Eqs. ForceInMovement, TorqueInMovement),
   taken forward in time; zero for a body whose solid set does not move.
   The same numbers as LBM_REC_N_COVERED / LBM_REC_N_UNCOVERED of the step's
   record. Synchronises; LBM_E_RANGE if the step is not in the record ring. */
lbm_status lbm_get_moving_sets(lbm_domain dom, int32_t body_id, int64_t step, int64_t* n_plus,
                               int64_t* n_minus);

/* The momentum exchange of the domain faces per step, when the domain was
   created with face_records = 1: rec[18*k ...] = F (3), T (3) of the wall
   layers, then of the inlet, then of the outlet(s), for steps
   first_step..first_step+count-1, T about the origin (node (0,0,0)); the
   force on the faces by the flow, -c_i (f_out + f_in) over every population
   that a face rule supplies (the closed-channel budget behind Eq.
   flow_force_2: at steady state the wall force balances the pressure drop).
   LBM_E_STATE if the domain does not record them; LBM_E_RANGE outside the
   ring. Synchronises. lbm_force_torque with body_id LBM_WALLS returns the
   wall part. */
#define LBM_WALLS (-1)
#define LBM_FACE_REC_LEN 18
lbm_status lbm_face_records(lbm_domain dom, int64_t first_step, int64_t count, double* rec);

/* Boundary links of a body at the current step, canonical order (node index
   x + nx*(y + ny*z) ascending, then direction ascending). Writes at most cap
   entries and the total count to *n. Synchronises. */
lbm_status lbm_get_links(lbm_domain dom, int32_t body_id, int64_t cap, int64_t* node,
                         int32_t* dir, double* delta, int64_t* n);

/* Steady-state test on the device, in FP64, from the record ring: the
   relative change |F_x(t-1) - F_x(t-1-window)| / |F_x(t-1)| of the body's
   drag (the x-force of the momentum-exchange form its me_mode selects) up to
   the current step t; *steady = 1 when that change is below tol, else 0.
   LBM_E_RANGE unless 0 <= t-1-window and window < the record capacity.
   Synchronises. */
lbm_status lbm_steady_state(lbm_domain dom, int32_t body_id, int64_t window, double tol, int32_t* steady,
                            double* rel_change);

/* Density and velocity of every node at the current step (host arrays of
   nx*ny*nz and 3*nx*ny*nz doubles); solid nodes get NaN. Synchronises. */
lbm_status lbm_get_fields(lbm_domain dom, double* rho, double* u);

/* Populations f_i of every node at the current step: f[Q*n + i], node
   n = x + nx*(y + ny*z), direction i in the numbering lbm_lattice gives;
   NaN for non-fluid nodes. Synchronises. For tests and inspection. */
lbm_status lbm_get_populations(lbm_domain dom, double* f);

/* The library's lattice: c[3*i..3*i+2] and w[i] for i < Q (either pointer
   may be NULL); returns Q (9 or 19), or -1 for an unknown lattice. */
int32_t lbm_lattice(int32_t lattice, int32_t* c, double* w);

/* Node types at the current step: 0 fluid, 1 wall layer, 2+b body b. */
lbm_status lbm_get_types(lbm_domain dom, int32_t* type);

/* Kernel timing, for measurement. With every = n >= 1, every n-th launch
   of each kind carries HIP events recorded at the kernel's own start and
   end; every = 0 turns timing off. Kinds: LBM_KERNEL_STREAM_COLLIDE, the
   stream-collide update of all nodes, or of all but the near box of a split
   step; LBM_KERNEL_BODY, the boundary rule + momentum exchange and the
   advance of a moving body; LBM_KERNEL_NEAR_BOX, the update of the near box
   of a split step. Each call waits for the domain's work and restarts the
   totals. lbm_timing_read waits for the events and returns, for one kind and
   since the last enable, the summed duration of the timed launches in
   milliseconds, their number, the node updates they made (zero for the
   body kernels) and the number of launches of that kind issued, timed or
   not (issued may be NULL). */
enum { LBM_KERNEL_STREAM_COLLIDE = 0, LBM_KERNEL_BODY = 1, LBM_KERNEL_NEAR_BOX = 2 };
lbm_status lbm_timing_enable(lbm_domain dom, int32_t every);
lbm_status lbm_timing_read(lbm_domain dom, int32_t kernel, double* total_ms, int64_t* launches,
                           int64_t* nodes, int64_t* issued);

/* Launch shape of a domain's stream-collide update: threads per workgroup x
   nodes per thread, one of (256,1) (256,2) (128,2); memory: bit 0 = the new
   state is written with non-temporal stores, bit 1 = the old state is read
   with non-temporal loads (streaming hints for states larger than the
   256 MB last-level cache); remap 1 = workgroups ordered so that each XCD
   takes a contiguous run of rows. lbm_create_domain picks one from the
   domain's footprint; every shape gives bitwise the same result.
   LBM_E_INVAL for an unsupported shape. Takes effect at the next lbm_step. */
typedef struct {
  int32_t block, cells_per_thread, memory, remap;
} lbm_sweep_config;
lbm_status lbm_get_sweep_config(lbm_domain dom, lbm_sweep_config* cfg);
lbm_status lbm_set_sweep_config(lbm_domain dom, const lbm_sweep_config* cfg);

/* ---------------------------------------------------------------------------
   Batches: many independent domains of one lattice, storage and equilibrium
   advanced by the same launches every step -- one boundary-rule launch over
   all bodies with fixed links, one stream-collide launch over a table of
   row tiles of every member, one launch with a workgroup per moving body.
   The arithmetic of every node and link is the one of lbm_step, so a member
   ends bitwise where lbm_step would have taken it. */
typedef struct lbm_batch_s* lbm_batch;

/* Launch shape of a batch. block x cells_per_thread nodes per tile, one of
   (64,1) (128,1) (256,1) (64,2) (128,2); remap 1 = blocks ordered so that
   each XCD takes a contiguous run of tiles; order 0 = tiles member by
   member, 1 = largest members first, 2 = rows of all members interleaved,
   3 = tiles of `block` consecutive active nodes that run across rows (x,
   then y, then z; largest members first; cells_per_thread 1 only), so that
   short rows leave no lanes idle;
   overlap 1 = each member's nodes near its bodies (the node boxes of the
   poses of the call plus one layer) are updated on the batch's stream
   together with the body work, the rest on a second stream the batch owns
   (default priority), so that the body work overlaps it. us_per_step is
   filled in by lbm_batch_tune. graph 1 = a call of at least 64 steps
   captures 32 steps once into a HIP graph (its kernels take their step from
   a device counter) and replays it, instead of enqueueing every launch from
   the host (not for members with a body too large for the batched advance).
   Every shape gives bitwise the same result. */
typedef struct {
  int32_t block, cells_per_thread, remap, order, overlap, graph;
  double us_per_step;
} lbm_batch_config;

/* Creates an empty batch whose launches go to `stream` (hipStream_t,
   borrowed; NULL = the default stream). */
lbm_status lbm_batch_create(void* stream, lbm_batch* out);

/* Waits for the batch's stream, then releases every member back to its own
   stream and frees the batch (the members stay valid). */
lbm_status lbm_batch_destroy(lbm_batch batch);

/* Adds a domain. From then on all of the domain's work (lbm_step and
   lbm_batch_step alike) and its synchronisation use the batch's stream.
   LBM_E_INVAL if lattice, storage or equilibrium differ from the first
   member's; LBM_E_STATE if the domain already belongs to a batch.
   Destroying a member removes it. */
lbm_status lbm_batch_add(lbm_batch batch, lbm_domain dom);

/* Removes a domain (waits for the batch's stream first); the domain uses its
   own stream again. */
lbm_status lbm_batch_remove(lbm_batch batch, lbm_domain dom);

/* Advances every member by nsteps steps (members may be at different
   steps). Waits for the batch's previous work once, to refresh its device
   tables, then only enqueues. */
lbm_status lbm_batch_step(lbm_batch batch, int64_t nsteps);

/* Sets the launch shape (LBM_E_INVAL for an unsupported one). */
lbm_status lbm_batch_set_config(lbm_batch batch, const lbm_batch_config* cfg);
lbm_status lbm_batch_get_config(lbm_batch batch, lbm_batch_config* cfg);

/* Autotuner: runs trial_steps real steps of the batch under every candidate
   launch shape (the members advance by the sum of the trials' steps), times
   each on the batch's stream with HIP events, then times the best shape in
   ordinary and in graph mode (overlap off and on) over 64-step calls, keeps
   the fastest and returns it in *chosen; up to trial_cap trials are written
   to `trials` (host, may be NULL) and their number to *ntrials. */
lbm_status lbm_batch_tune(lbm_batch batch, int32_t trial_steps, lbm_batch_config* chosen,
                          lbm_batch_config* trials, int32_t trial_cap, int32_t* ntrials);

/* The steady-state test of lbm_steady_state for body 0 of every member, in
   one launch. steady and rel_change are host arrays with one entry per
   member, in the order the members were added; a member without a body or
   with too few steps gets steady = -1 and rel_change = NaN. Synchronises. */
lbm_status lbm_batch_steady_state(lbm_batch batch, int64_t window, double tol, int32_t* steady,
                                  double* rel_change);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the same
   checks and results as lbm_batch_steady_state, with the table of checks and
   their results in a static device array of the library (one per GPU, kept
   until the process ends, about 32 KB) instead of a buffer the batch grows
   with hipMalloc. Host tables live on the caller's stack (about 34 KB). At
   most LBM_STEADY_NOALLOC_MAX members (LBM_E_INVAL beyond). Call with the
   batch's device current. Every call on a GPU shares that GPU's array: calls
   that overlap on one GPU (from several threads) race; each call overwrites
   every entry it reads back, so nothing needs clearing. Synchronises. */
#define LBM_STEADY_NOALLOC_MAX 512
lbm_status lbm_batch_steady_state_noalloc(lbm_batch batch, int64_t window, double tol, int32_t* steady,
                                          double* rel_change);

/* Measurement: a plain device-to-device copy of `bytes` bytes (a multiple of
   16; both addresses 16-byte aligned) by a hand-written kernel, enqueued on
   `stream` (hipStream_t, borrowed). It is the copy ceiling the stream-collide
   kernel is measured against and the reference whose exactly known bytes
   calibrate the HBM traffic counters. variant: 0, 1, 2 = one, two or four
   16-byte vectors per thread over a grid covering the array; 3 = four per
   thread with non-temporal loads and stores; 4, 5 = four or two per thread
   with a fixed grid of 2048 or 4096 workgroups striding over the array.
   Enqueue only; LBM_E_INVAL for a size or alignment that is not a multiple
   of 16 or an unknown variant. Not part of the method. */
lbm_status lbm_copy(const void* src, void* dst, size_t bytes, int32_t variant, void* stream);

/* Thread-local description of the last error. */
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
