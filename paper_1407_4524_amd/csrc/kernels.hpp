// Launchers of the HIP kernels (internal interface of the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "geom.hpp"
#include "lattice.hpp"

namespace lbm {

// Sizes of the single-workgroup body kernels (status box in LDS, two bytes
// per node): the host picks the kernel from them.
constexpr int ADV_LDS_CELLS = 20480;  // 2 bytes each + the window table stay within 64 KB of LDS
constexpr int STEP_ROWS = 1024;       // region rows covered by the window table
constexpr int STEP_LIST = 2048;       // window nodes
constexpr int STEP_CELLS = 20480;     // status box nodes (two bytes each)
constexpr int STEP_LINKS = 8192;      // links held in LDS (the rest go through global memory)
constexpr int LINK_BLOCK = 256;       // threads per block of the link-rule kernel
// Advance of a moving body over many workgroups (bodies too large for the
// single-workgroup kernels): region rows per workgroup, threads per
// workgroup, links of a workgroup held in LDS (the rest go through global
// memory). The body's scratch holds, per workgroup, 20 sums and a link
// count, then one arrival counter (zero between launches).
constexpr int WIDE_ROWS = 16;
constexpr int WIDE_BLOCK = 256;
constexpr int WIDE_LINKS = 4096;
inline size_t wide_scratch_bytes(int slabs) {
  return (size_t)slabs * (20 * sizeof(double) + sizeof(int)) + sizeof(unsigned);
}

struct BulkShape {
  int nbx, nrows, nplanes, nblocks;
};
BulkShape bulk_shape(const Geom& g, int span);

// stream-collide launch shape: threads per block, nodes per thread, memory
// mode (bit 0: non-temporal stores of the new state, bit 1: non-temporal
// loads of the old one), XCD-aware block order; buf (batched sweep): every
// member's population buffer is below 4 GiB, so the loads and stores go
// through raw buffer resources with 32-bit offsets (the single-domain sweep
// decides this from its own buffer)
struct BulkConfig {
  int block, cells_per_thread, nontemporal, remap;
  int buf = 0;
};
enum { MEM_NT_STORE = 1, MEM_NT_LOAD = 2 };
BulkConfig bulk_config(int lat, int st, size_t footprint);

// Node box swept by one stream-collide launch, in tiles of `span`
// consecutive x of one (y, z) row: tile k is span k % nbx of row k / nbx,
// rows running y-fastest. Nodes inside the hole box (x0, x1, y0, y1, z0, z1;
// empty when x0 > x1) are skipped.
struct Sweep {
  int x0, y0, z0, xlast, ny, nbx, ntiles, remap;
  int hole[6];
  // densities of the x-face nodes (x = lo: first half, x = hi: second half;
  // row y + ny z of the active box) of the old state, read by the velocity
  // bounce-back of the faces, and of the new state, written by the sweep;
  // null when the domain has no inlet or velocity outlet (or the
  // quasi-incompressible equilibrium, whose wall term takes rho0)
  const void* rho_in;
  void* rho_out;
  // node status (read only for a node whose speed is out of range) and the
  // word the sweep sets to 1 when a fluid node's |u| exceeds 0.4 or is not a
  // number; null: no check
  const uint8_t* mask;
  int* unstable;
};
Sweep make_sweep(const int lo[3], const int hi[3], int span, const int* hole, int remap);
bool bulk_supported(const BulkConfig& c);

// ev_start/ev_stop (here and below): events recorded at the start and the
// end of the kernel itself by the launch; a start event needs a stop event,
// a stop event alone marks the kernel's completion (in place of a record
// after the launch)
hipError_t launch_stream_collide(int lat, int st, int eq, const void* A, void* B, const Geom& g, const Phys& ph,
                                 hipStream_t s, const BulkConfig& cfg, const Sweep& sw,
                                 hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);

// rho_out (optional): the x-face densities of the initial state (see Sweep)
hipError_t launch_init(int lat, int st, int eq, void* A, uint8_t* mask, const Geom& g, const Phys& ph,
                       const double* rho, const double* u, void* rho_out, hipStream_t s);
hipError_t launch_links(int lat, int st, int eq, void* A, const Link* links, int n_host, const int* n_dev,
                        int grid, const double* pose, int bc, const uint8_t* mask, const Geom& g, const Phys& ph,
                        double* partials, unsigned* counter, double* rec, hipStream_t s, hipEvent_t ev_start = nullptr,
                        hipEvent_t ev_stop = nullptr);
// The link rule + momentum exchange of a body at one step with its chunk
// sums (12 per chunk of 64 links) written to `part`, the step's slot of the
// body's ring; launch_fold later turns the slots of steps t0..t0+nsteps-1
// into records (rec: the body's record of ring slot 0; rec_stride doubles
// between steps). n >= 0 links (none: zero sums).
hipError_t launch_links_part(int lat, int st, int eq, void* A, const Link* links, int n, const double* pose, int bc,
                             const uint8_t* mask, const Geom& g, const Phys& ph, double* part, hipStream_t s,
                             hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
// The momentum exchange of the domain faces at one step from the state A
// (post-collision values of the step), one thread per face node: 18 sums
// (walls, inlet, outlet: F and T about the origin) per wavefront into
// `part`, the step's slot of the face ring (face_chunks(g) chunks);
// launch_fold_faces turns slots into records of 18 doubles.
int face_nodes(const Geom& g);
inline int face_chunks(const Geom& g) { return (face_nodes(g) + 63) / 64; }
hipError_t launch_face_part(int lat, int st, int eq, const void* A, const Geom& g, const Phys& ph, const void* rho_in,
                            double* part, hipStream_t s);
hipError_t launch_fold_faces(const double* ring, int nchunks, int ring_steps, int64_t t0, int64_t nsteps, double* rec,
                             int64_t rec_cap, hipStream_t s);
// NaN into both buffers' slots of the nodes of `body` inside the node box
hipError_t launch_poison_body(int lat, int st, int eq, void* A, void* B, const uint8_t* mask, const Geom& g,
                              const int lo[3], const int hi[3], int body, hipStream_t s);
hipError_t launch_fold(const double* ring, int nchunks, int ring_steps, int64_t t0, int64_t nsteps, double* rec,
                       int64_t rec_cap, int64_t rec_stride, bool zero_nodes, hipStream_t s);
// pose: the poses of t and t+1 on the device; pose_host: the same two on the
// host (read at the call). wide (optional): the body's scratch for the
// many-workgroup advance, of wide_slabs workgroups; an advance (mode 1) of a
// body that is not an outer circle and does not fit the single-workgroup
// list kernel takes it when given.
hipError_t launch_body_advance(int lat, int st, int eq, void* B, uint8_t* mask, uint8_t* mask_next, Link* links,
                               int* n_links, int cap, const double* pose, const double* pose_host, const BodyShape& bs,
                               int bc, int body, int mode, const Geom& g, const Phys& ph, double* rec_t, double* rec_t1,
                               int* err, hipStream_t s, int64_t region_cells, int64_t region_rows, int64_t list_nodes,
                               double* wide = nullptr, int wide_slabs = 0, hipEvent_t ev_start = nullptr,
                               hipEvent_t ev_stop = nullptr);

// The node terms of a FREE body's step t over the covered and uncovered
// nodes between its pose t (pose[0..15], device) and the pose one step at
// its velocity of step t ahead (the second approximation of Sec. III.B.3),
// on the state of t+1 in B, nothing written but out[0..5] (F, T about X).
hipError_t launch_body_predict(int lat, int st, int eq, const void* B, const uint8_t* mask, const double* pose,
                               const BodyShape& bs, int body, const Geom& g, const Phys& ph, double* out,
                               hipStream_t s);

// Steady-state check of one body: relative change of its drag between
// steps t - 1 - window and t - 1 (records of ring `rec`, slot stride
// rec_stride doubles); out[2k] = relative change, out[2k+1] = drag at t - 1.
struct SteadyCheck {
  const double* rec;
  int64_t rec_cap, rec_stride, t, window;
  int me_mode;
};
hipError_t launch_steady(const SteadyCheck* checks, int n, double* out, hipStream_t s);

// True when the per-step advance of a moving body whose region (node box of
// poses t and t+1 plus a margin) has this many nodes and rows, and whose
// near-surface node list has at most list_nodes entries, runs in the
// single-workgroup LDS kernel (the batched path needs it).
bool body_step_fits(int64_t region_cells, int64_t region_rows, int64_t list_nodes);
// Upper bound of the near-surface node list of the advance between poses
// P0 and P1 (the row windows of the single-workgroup kernel; host only).
int64_t step_list_nodes(const BodyShape& bs, const Pose& P0, const Pose& P1, int D);

// ---------------------------------------------------------------------------
// batches of domains advanced by the same launches

constexpr int POSE_DOUBLES = 16;  // doubles per Pose record

// one member domain; the source buffer of batch step s is buf[s & 1];
// hole: its near box (x0, x1, y0, y1, z0, z1; empty when x0 > x1), skipped by
// the far launch and covered by the near launch of a split batch step
struct BatchDomain {
  Geom g;
  Phys ph;
  void* buf[2];
  void* rho[2];  // x-face densities of the state in buf[k] (see Sweep)
  const uint8_t* mask;  // node status and instability word (see Sweep)
  int* unstable;
  int hole[6];
};

// one block of the batched stream-collide launch: span bx of row `row` of
// member `dom` (rows numbered as in RowRange)
struct BatchTile {
  uint16_t dom, bx;
  int32_t row;
};

// one body of a member domain
struct BatchBody {
  int dom, body, bc, cap, n_host;
  Link* links;
  int* n_links;
  const double* pose;  // device pose window; record k is step pose_base + k
  int64_t pose_base;
  BodyShape bs;
  uint8_t* mask;
  double* rec;         // this body's record in ring slot 0
  int64_t rec_cap, rec_stride;
  double* partials;
  unsigned* counter;
  int* err;
  int64_t t0;          // the member's step at batch step 0
  double* wide;        // scratch of the many-workgroup advance (wide_scratch_bytes(wide_slabs))
  int wide_slabs;
};

// (block, nodes per thread) of the batched stream-collide variants
constexpr int BATCH_BULK_VARIANTS[5][2] = {{64, 1}, {128, 1}, {256, 1}, {64, 2}, {128, 2}};
bool batch_bulk_supported(int block, int cells_per_thread);

// part: 0 every node of the tiles' rows, 1 the same but the members' near
// boxes, 2 near-box tiles (rows numbered within the box)
// sbase (optional, device): added to `step` by the kernels, for step
// sequences captured once and replayed
// flat (parts 0 and 1): tile.row is the first of `block` consecutive active
// nodes of the member in x, y, z order (a span may cross rows; one node per
// thread)
hipError_t launch_batch_bulk(int lat, int st, int eq, const BatchDomain* doms, const BatchTile* tiles, int ntiles,
                             const BulkConfig& cfg, int64_t step, hipStream_t s, int part = 0,
                             hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr,
                             const int64_t* sbase = nullptr, int flat = 0);
// blocks per body of the batched link-rule launch for bodies of up to
// max_links links (2D: one workgroup; 3D: one wavefront per chunk of 64)
int batch_link_grid(int lat, int max_links);
hipError_t launch_batch_links(int lat, int st, int eq, const BatchDomain* doms, const BatchBody* bodies, int nbodies,
                              int grid, int64_t step, hipStream_t s, const int64_t* sbase = nullptr);
// 2D batches: the advance of the moving bodies after batch step `step` and
// the link rule of step+1 for the bodies with fixed links, in one launch
hipError_t launch_batch_body_links(int lat, int st, int eq, const BatchDomain* doms, const BatchBody* moving,
                                   int n_moving, const BatchBody* fixed, int n_fixed, int64_t max_region_cells,
                                   int64_t step, hipStream_t s, const int64_t* sbase = nullptr);
hipError_t launch_batch_body_step(int lat, int st, int eq, const BatchDomain* doms, const BatchBody* bodies,
                                  int nbodies, int64_t max_region_cells, int64_t step, hipStream_t s,
                                  const int64_t* sbase = nullptr);
// the many-workgroup advance of every body in `bodies` after batch step
// `step` (two launches, max_slabs workgroups per body)
hipError_t launch_batch_wide(int lat, int st, int eq, const BatchDomain* doms, const BatchBody* bodies, int nbodies,
                             int max_slabs, int64_t step, hipStream_t s, const int64_t* sbase = nullptr);
// Newton-Euler step of a FREE body (include/lbm.h): from the flow force of
// the record rec_t (and the node terms of rec_tm1, optional) and the pose in
// pose[0..15], the pose of the next step into pose[16..31] and traj[0..7];
// dyn holds the previous accelerations and their flag. One thread.
struct FreeBody {
  double mass, inertia, ext_force[3], ext_torque;
  int integrator, drive, shape, D;
  int predicted;  // the lattice drive takes the predicted node terms (pred) instead of those of t-1
  double axes[3];
  int glo[3], ghi[3];
};
hipError_t launch_body_integrate(const double* rec_t, const double* rec_tm1, const double* pred, double* pose,
                                 double* traj, double* dyn, const FreeBody& fb, int* err, hipStream_t s);

// *counter += k, one thread (closes a captured step sequence); *counter = v
hipError_t launch_add_step(int64_t* counter, int64_t k, hipStream_t s);
hipError_t launch_set_step(int64_t* counter, int64_t v, hipStream_t s);

// ---------------------------------------------------------------------------
// The launches of one (lattice, storage, equilibrium) combination. Defined in
// kernels_impl.hpp and instantiated once per lattice and storage (both
// equilibria) in the inst_*.hip sources, so that the kernel templates compile
// in parallel translation units; the launch_* functions above dispatch to
// them after validating their arguments.
template <class L, class S, int EQ>
struct Ops {
  static void stream_collide(const BulkConfig& c, const void* A, void* B, const Geom& g, const Phys& ph,
                             const Sweep& sw, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
  static void init(void* A, uint8_t* mask, const Geom& g, const Phys& ph, const double* rho, const double* u,
                   void* rho_out, hipStream_t s);
  static void links(void* A, const Link* links, int n_host, const int* n_dev, int grid, const double* pose, int bc,
                    const uint8_t* mask, const Geom& g, const Phys& ph, double* partials, unsigned* counter,
                    double* rec, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
  static void links_part(void* A, const Link* links, int n, const double* pose, int bc, const uint8_t* mask,
                         const Geom& g, const Phys& ph, double* part, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
  static void face_part(const void* A, const Geom& g, const Phys& ph, const void* rho_in, int nnodes, double* part,
                        hipStream_t s);
  static void poison_body(void* A, void* B, const uint8_t* mask, const Geom& g, const int lo[3], const int hi[3],
                          int body, hipStream_t s);
  static void body_advance(void* B, uint8_t* mask, uint8_t* mask_next, Link* links, int* n_links, int cap,
                           const double* pose, const double* pose_host, const BodyShape& bs, int bc, int body,
                           int mode, const Geom& g, const Phys& ph, double* rec_t, double* rec_t1, int* err,
                           hipStream_t s, int64_t region_cells, int64_t region_rows, int64_t list_nodes,
                           double* wide, int wide_slabs, hipEvent_t e0, hipEvent_t e1);
  static void body_predict(const void* B, const uint8_t* mask, const double* pose, const BodyShape& bs, int body,
                           const Geom& g, const Phys& ph, double* out, hipStream_t s);
  static void batch_bulk(const BatchDomain* doms, const BatchTile* tiles, int ntiles, const BulkConfig& cfg,
                         int64_t step, hipStream_t s, int part, hipEvent_t e0, hipEvent_t e1, const int64_t* sbase,
                         int flat);
  static void batch_links(const BatchDomain* doms, const BatchBody* bodies, int nbodies, int grid, int64_t step,
                          hipStream_t s, const int64_t* sbase);
  static void batch_body_links(const BatchDomain* doms, const BatchBody* moving, int n_moving,
                               const BatchBody* fixed, int n_fixed, size_t lds, int64_t step, hipStream_t s,
                               const int64_t* sbase);
  static void batch_body_step(const BatchDomain* doms, const BatchBody* bodies, int nbodies, size_t lds,
                              int64_t step, hipStream_t s, const int64_t* sbase);
  static void batch_wide(const BatchDomain* doms, const BatchBody* bodies, int nbodies, int max_slabs, int64_t step,
                         hipStream_t s, const int64_t* sbase);
};

#define LBM_OPS_FOR(MACRO, Lt, St) \
  MACRO(Lt, St, 0)                 \
  MACRO(Lt, St, 1)
#define LBM_OPS_EXTERN(Lt, St, E) extern template struct Ops<Lt, St, E>;
LBM_OPS_FOR(LBM_OPS_EXTERN, D2Q9, StoreF64)
LBM_OPS_FOR(LBM_OPS_EXTERN, D2Q9, StoreF32)
LBM_OPS_FOR(LBM_OPS_EXTERN, D2Q9, StoreF16)
LBM_OPS_FOR(LBM_OPS_EXTERN, D3Q19, StoreF64)
LBM_OPS_FOR(LBM_OPS_EXTERN, D3Q19, StoreF32)
LBM_OPS_FOR(LBM_OPS_EXTERN, D3Q19, StoreF16)
#undef LBM_OPS_EXTERN

}  // namespace lbm
