// Host-side state of a domain and the helpers shared by the files that
// implement the C ABI (include/lbm.h).
#pragma once
#include <string>
#include <vector>

#include "kernels.hpp"
#include "lbm.h"

namespace lbm {
namespace host {

// records `msg` as the thread's last error and returns `code`
lbm_status fail(lbm_status code, const std::string& msg);

#define HIP_TRY(expr)                                                                                  \
  do {                                                                                                 \
    hipError_t e_ = (expr);                                                                            \
    if (e_ != hipSuccess) return ::lbm::host::fail(LBM_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr double PI = 3.14159265358979323846;
constexpr int POSE_LEN = 16;  // doubles per Pose record
constexpr int LINK_GRID_MAX = 64;
constexpr int64_t POSE_WINDOW = 8192;
constexpr int PART_RING = 64;  // steps of link-rule chunk sums a body keeps before they are folded into records

struct Body {
  bool active = false;
  lbm_body_desc desc{};
  BodyShape shape{};
  bool mask_moves = false;  // the solid set changes with the pose
  std::vector<double> table;
  Link* links = nullptr;
  int* n_links = nullptr;
  double* partials = nullptr;  // one 12-double sum per chunk of 64 links
  int cap = 0;
  int n_host = 0;
  double* pose_dev = nullptr;
  double* pose_pinned = nullptr;
  int64_t pose_base = 0, pose_cap = 0, pose_valid = 0;
  // ring of the link rule's chunk sums (PART_RING steps of ring_chunks x 12
  // doubles) and the steps [part_t0, part_t0 + part_n) not yet folded
  double* ring = nullptr;
  int ring_chunks = 0;
  int64_t part_t0 = 0, part_n = 0;
  bool bc_ready = false;
  // FREE motion: the device fills the pose window step by step; traj is a
  // ring of 8 doubles (X, theta, V, Omega) per step of the record ring, dyn
  // the previous accelerations and their flag (Adams-Bashforth)
  bool free_motion = false;
  double* traj = nullptr;
  double* dyn = nullptr;
  double* pred = nullptr;  // node terms of the predicted pose (LBM_SETS_PREDICTED)
  int64_t t_placed = 0;
  // scratch of the many-workgroup advance (moving bodies that are not outer
  // circles): wide_slabs workgroups of WIDE_ROWS region rows each
  double* wide = nullptr;
  int wide_slabs = 0;
};

}  // namespace host
}  // namespace lbm

struct lbm_domain_s {
  lbm_domain_desc desc{};
  int lat = 0, st = 0, eq = 0, Q = 9, D = 2;
  size_t elem = 8;
  lbm::Geom g{};
  lbm::Phys ph{};
  hipStream_t stream = nullptr;
  hipStream_t own_stream = nullptr;  // the descriptor's stream (a batch may lend its own)
  struct lbm_batch_s* batch = nullptr;  // the batch the domain belongs to, if any
  struct lbm_batch_s* solo = nullptr;   // one-member batch lbm_step uses for several bodies
  char* steady_buf = nullptr;           // device: one SteadyCheck and its two results
  bool owns_pool = false;
  char* pool = nullptr;
  size_t pool_bytes = 0;
  void* A = nullptr;
  void* B = nullptr;
  uint8_t* mask = nullptr;
  uint8_t* mask_next = nullptr;
  double* rec = nullptr;
  int64_t rec_cap = 0;
  int nslots = 4;  // body slots (ids 0 .. nslots-1); records per ring step
  int* err = nullptr;
  unsigned* counters = nullptr;
  int64_t t = 0;
  lbm::host::Body body[LBM_MAX_BODIES];
  lbm::BulkConfig bulk{};  // stream-collide launch shape
  // second stream: the far update of a split step; created on first use
  hipStream_t aux = nullptr;
  hipEvent_t e_near = nullptr, e_far = nullptr;
  // face records (face_records): ring of 18 doubles per step, and the ring of
  // the face kernel's chunk sums with its pending steps
  double* face_rec = nullptr;
  double* face_ring = nullptr;
  int face_chunks = 0;
  int64_t face_part_t0 = 0, face_part_n = 0;
  // densities of the x-face nodes of the states in A and B (see Sweep); null
  // when no face rule needs them
  void* rhoA = nullptr;
  void* rhoB = nullptr;
  // kernel timing ring, by kind (LBM_KERNEL_*), every timing_every-th launch
  // of each kind
  int timing_every = 0;
  int64_t kind_count[3] = {0, 0, 0};
  bool timing = false;
  hipEvent_t ev[2][64] = {};
  int ev_kind[64] = {};
  int64_t timed = 0, folded = 0;
  int64_t kind_launches[3] = {0, 0, 0}, kind_nodes[3] = {0, 0, 0};
  double kind_ms[3] = {0.0, 0.0, 0.0};
};

namespace lbm {
namespace host {

double* rec_slot(lbm_domain d, int64_t t, int b);
// makes the device pose table of body b cover steps [t0, t1]
lbm_status ensure_poses(lbm_domain d, Body& b, int64_t t0, int64_t t1);
const double* pose_at(const Body& b, int64_t t);
const double* pose_host_at(const Body& b, int64_t t);  // host copy of the same pose
// nodes (with the one-node margin) and rows of the region of poses t, t+mode
int64_t region_cells(const Body& b, int D, int64_t t, int mode);
int64_t region_rows(const Body& b, int64_t t, int mode);
// upper bound of the near-surface node list of body b's advance from t
int64_t list_bound(const Body& b, int D, int64_t t);
// whether the advance of a moving body (prescribed motion) from step t runs
// in the single-workgroup list kernel (body_step_fits of its region, rows
// and list); the list is bounded only when the region fits
bool step_fits(const Body& b, int D, int64_t t);
lbm_status check_device_errors(lbm_domain d);
// whether a body may advance in the many-workgroup kernels (it holds their
// scratch), and the slabs its region needs at any pose while it moves less
// than a node per step (free bodies: always) in a domain of n nodes per axis
bool wide_advance(int D, const lbm_body_desc& bd);
int wide_slab_bound(int D, const int n[3], const lbm_body_desc& bd);
// makes the body's scratch hold at least `slabs` slabs; a larger one is
// allocated (and zeroed) after `s` has drained
lbm_status ensure_wide(Body& b, int slabs, hipStream_t s);
// the advance of body `id` from step t to t+1 on the current source buffer
lbm_status launch_advance(lbm_domain d, int id, int64_t t);
// n steps of a domain with several bodies through a one-member batch of its
// own (the domain does not join it: d->batch is untouched), and its release
lbm_status solo_step(lbm_domain d, int64_t n);
void solo_destroy(lbm_domain d);
// the steady-state check of one body (see lbm_steady_state); false when the
// ring does not hold both steps
bool steady_check(lbm_domain d, int id, int64_t window, SteadyCheck& c);
// Second stream for the update of the nodes away from the bodies, beside
// `main`: it may use every CU but one in `every` (spread over the device),
// which stay free for the latency-bound body kernels running beside it. A
// CU-masked stream synchronises with the legacy default stream, so with
// main == the default stream (or when the device takes no CU mask) it is a
// plain non-blocking stream instead.
lbm_status create_far_stream(hipStream_t main, hipStream_t* s, int every);
// start/stop events of the next timed launch of this kind (null when off)
lbm_status timing_slot(lbm_domain d, int kind, int64_t nodes, hipEvent_t& e0, hipEvent_t& e1);

}  // namespace host
}  // namespace lbm
