// Host side of the C ABI declared in include/lbm.h: descriptor validation,
// device layout and allocation, host-computed body poses, the per-step launch
// sequence and the result queries.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "domain.hpp"

using namespace lbm;
using namespace lbm::host;

namespace {

thread_local std::string g_last_error;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

lbm_status lbm::host::fail(lbm_status code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

struct Layout {
  Geom g;
  size_t pop_bytes, mask_bytes, rec_bytes, err_bytes, cnt_bytes, rho_bytes, face_rec_bytes, face_ring_bytes, total;
  int64_t rec_cap;
};

// the velocity bounce-back of an inlet or velocity outlet takes rho(x_F) of
// the standard equilibrium: the x-face densities are kept for it
static bool needs_face_rho(const lbm_domain_desc* d) {
  return d->eq_model == LBM_EQ_BGK && (d->face[0] == LBM_FACE_INLET || d->face[1] == LBM_FACE_OUTLET_VELOCITY);
}

// link capacity of a body: (Q-1) links per node of a shell two nodes thick
// around the circumscribed circle/sphere, doubled
static int link_capacity(int D, const lbm_body_desc* bd) {
  const int Q = D == 2 ? 9 : 19;
  double rc = bd->axes[0];
  if (bd->shape == LBM_SHAPE_ELLIPSE) rc = std::max(rc, std::max(bd->axes[1], D == 3 ? bd->axes[2] : 0.0));
  const double shell = D == 2 ? 2.0 * PI * (rc + 3.0) * 4.0 : 4.0 * PI * (rc + 3.0) * (rc + 3.0) * 4.0;
  return (int)std::min<double>(2.0 * (Q - 1) * shell + 1024.0, 2.0e9 / sizeof(Link));
}

static lbm_status check_desc(const lbm_domain_desc* d) {
  if (!d) return fail(LBM_E_INVAL, "null descriptor");
  if (d->lattice != LBM_D2Q9 && d->lattice != LBM_D3Q19) return fail(LBM_E_INVAL, "unknown lattice");
  const int D = d->lattice == LBM_D2Q9 ? 2 : 3;
  if (d->nx < 3 || d->ny < 3 || (D == 3 && d->nz < 3)) return fail(LBM_E_INVAL, "each axis needs >= 3 nodes");
  if ((int64_t)d->nx > 32000 || d->ny > 32000 || (D == 3 && d->nz > 32000))
    return fail(LBM_E_INVAL, "axis longer than 32000 nodes");
  if (!(d->tau > 0.5)) return fail(LBM_E_INVAL, "tau must exceed 1/2");
  if (!(d->rho0 > 0)) return fail(LBM_E_INVAL, "rho0 must be positive");
  if (d->storage < LBM_F64 || d->storage > LBM_F16_SHIFTED) return fail(LBM_E_INVAL, "unknown storage");
  if (d->eq_model != LBM_EQ_BGK && d->eq_model != LBM_EQ_HELUO) return fail(LBM_E_INVAL, "unknown eq_model");
  for (int a = 0; a < D; ++a) {
    int lo = d->face[2 * a], hi = d->face[2 * a + 1];
    if (lo < 0 || lo > 6 || hi < 0 || hi > 6) return fail(LBM_E_INVAL, "unknown face type");
    const bool zh = lo >= LBM_FACE_ZOUHE_VELOCITY || hi >= LBM_FACE_ZOUHE_VELOCITY;
    if (zh && a > 0) return fail(LBM_E_INVAL, "Zou-He faces only along x");
    if (zh && d->face_records) return fail(LBM_E_INVAL, "face records are not kept for Zou-He faces");
    if ((lo == LBM_FACE_PERIODIC) != (hi == LBM_FACE_PERIODIC)) return fail(LBM_E_INVAL, "periodic faces come in pairs");
    if (lo == LBM_FACE_OUTLET || lo == LBM_FACE_OUTLET_VELOCITY || hi == LBM_FACE_INLET)
      return fail(LBM_E_INVAL, "inlet only on -x, outlets only on +x");
    if (a > 0 && (lo == LBM_FACE_INLET || hi == LBM_FACE_OUTLET || hi == LBM_FACE_OUTLET_VELOCITY))
      return fail(LBM_E_INVAL, "inlet/outlet faces only along x");
  }
  if (d->inlet_profile != LBM_PROFILE_UNIFORM && d->inlet_profile != LBM_PROFILE_PARABOLIC)
    return fail(LBM_E_INVAL, "unknown inlet profile");
  if (d->record_capacity < 0) return fail(LBM_E_INVAL, "negative record capacity");
  if (d->max_bodies < 0 || d->max_bodies > LBM_MAX_BODIES) return fail(LBM_E_INVAL, "max_bodies out of range");
  if ((d->face_records != 0 && d->face_records != 1) || (d->debug_poison != 0 && d->debug_poison != 1))
    return fail(LBM_E_INVAL, "face_records and debug_poison are 0 or 1");
  if (d->split_schedule < -1 || d->split_schedule > 1) return fail(LBM_E_INVAL, "split_schedule is -1, 0 or 1");
  return LBM_OK;
}

// body slots of a domain (the record ring holds one record per slot and step)
static int body_slots(const lbm_domain_desc* d) { return d->max_bodies ? d->max_bodies : 4; }

static Layout make_layout(const lbm_domain_desc* d) {
  Layout L{};
  Geom& g = L.g;
  const int D = d->lattice == LBM_D2Q9 ? 2 : 3;
  const int Q = D == 2 ? 9 : 19;
  const size_t elem = d->storage == LBM_F64 ? 8 : (d->storage == LBM_F32 ? 4 : 2);
  g.nx = d->nx;
  g.ny = d->ny;
  g.nz = D == 3 ? d->nz : 1;
  g.D = D;
  for (int k = 0; k < 6; ++k) g.face[k] = d->face[k];
  if (D == 2) g.face[4] = g.face[5] = LBM_FACE_PERIODIC;
  const int64_t xoff = 128 / (int64_t)elem;  // node x = 0 on a 128-byte boundary
  const int64_t px = (int64_t)align_up((size_t)(xoff + g.nx + 1), (size_t)xoff);
  const int64_t rows = g.ny + 2;
  const int64_t planes = D == 3 ? g.nz + 2 : 1;
  g.sy = px;
  g.sz = px * rows;
  g.S = (int64_t)align_up((size_t)(g.sz * planes + px), 64);  // one spare row: V-wide loads may read past the last row
  g.base = xoff + g.sy + (D == 3 ? g.sz : 0);
  int n[3] = {g.nx, g.ny, g.nz};
  for (int a = 0; a < 3; ++a) {
    if (a >= D) {
      g.lo[a] = g.hi[a] = 0;
      continue;
    }
    g.lo[a] = g.face[2 * a] == LBM_FACE_WALL ? 1 : 0;
    g.hi[a] = g.face[2 * a + 1] == LBM_FACE_WALL ? n[a] - 2 : n[a] - 1;
  }
  L.rec_cap = d->record_capacity ? d->record_capacity : 65536;
  L.pop_bytes = align_up((size_t)Q * g.S * elem, 256);
  L.mask_bytes = align_up((size_t)g.S, 256);
  L.rec_bytes = align_up((size_t)L.rec_cap * body_slots(d) * LBM_REC_LEN * sizeof(double), 256);
  L.err_bytes = 256;
  L.cnt_bytes = 256;
  // two arrays (the states in A and B) of 2 n_y n_z densities in the
  // collision's type
  L.rho_bytes = needs_face_rho(d) ? align_up((size_t)2 * (g.hi[1] - g.lo[1] + 1) * (g.hi[2] - g.lo[2] + 1) *
                                                 (d->storage == LBM_F64 ? 8 : 4),
                                             256)
                                  : 0;
  L.face_rec_bytes = d->face_records ? align_up((size_t)L.rec_cap * LBM_FACE_REC_LEN * sizeof(double), 256) : 0;
  L.face_ring_bytes =
      d->face_records ? align_up((size_t)PART_RING * face_chunks(g) * LBM_FACE_REC_LEN * sizeof(double), 256) : 0;
  L.total = 2 * L.pop_bytes + 2 * L.mask_bytes + L.rec_bytes + L.err_bytes + L.cnt_bytes + 2 * L.rho_bytes +
            L.face_rec_bytes + L.face_ring_bytes;
  return L;
}

// Pose of a body at integer step t, by the rules of include/lbm.h.
static Pose body_pose(const Body& b, const Geom& g, int64_t t) {
#pragma clang fp contract(off)
  Pose p{};
  const lbm_body_desc& d = b.desc;
  for (int a = 0; a < 3; ++a) p.X[a] = d.c0[a];
  p.theta = d.theta0;
  switch (d.motion) {
    case LBM_MOTION_CONST_VEL:
      for (int a = 0; a < 3; ++a) {
        p.X[a] = d.c0[a] + d.vel[a] * (double)t;
        p.V[a] = d.vel[a];
      }
      break;
    case LBM_MOTION_ROTATE:
      p.theta = d.theta0 + d.omega * (double)t;
      p.Om = d.omega;
      break;
    case LBM_MOTION_OSCILLATE: {
      double ph = (2.0 * PI) * (double)t / d.period;
      double s = sin(ph), c = cos(ph);
      for (int a = 0; a < 3; ++a) {
        p.X[a] = d.c0[a] + d.amp[a] * s;
        p.V[a] = d.amp[a] * ((2.0 * PI) / d.period) * c;
      }
      break;
    }
    case LBM_MOTION_TABLE: {
      int64_t n = (int64_t)b.table.size() / 8;
      int64_t k = t < n ? t : n - 1;
      const double* r = b.table.data() + 8 * k;
      for (int a = 0; a < 3; ++a) p.X[a] = r[a];
      p.theta = r[3];
      for (int a = 0; a < 3; ++a) p.V[a] = r[4 + a];
      p.Om = r[7];
      break;
    }
    default:
      break;
  }
  if (g.D == 2) {
    p.X[2] = 0.0;
    p.V[2] = 0.0;
  }
  if (d.motion == LBM_MOTION_FREE) {  // the start of a computed motion
    for (int a = 0; a < 3; ++a) p.V[a] = g.D == 2 && a == 2 ? 0.0 : d.vel[a];
    p.Om = d.omega;
    free_trig(p.theta, p.ct, p.st);
  } else {
    p.ct = cos(p.theta);
    p.st = sin(p.theta);
  }
  pose_box(d.shape, d.axes, g.D, g.lo, g.hi, p);
  return p;
}

static bool pose_inside(const Pose& p, const Geom& g) {
  for (int a = 0; a < g.D; ++a)
    if (p.lo[a] < g.lo[a] || p.hi[a] > g.hi[a]) return false;
  return true;
}

lbm_status lbm::host::create_far_stream(hipStream_t main, hipStream_t* s, int every) {
  int dev = 0, cus = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  if (main != nullptr && every > 1 && cus > every) {
    std::vector<uint32_t> mask((size_t)(cus + 31) / 32, 0u);
    for (int k = 0; k < cus; ++k)
      if (k % every != every - 1) mask[k / 32] |= 1u << (k % 32);
    if (hipExtStreamCreateWithCUMask(s, (uint32_t)mask.size(), mask.data()) == hipSuccess) return LBM_OK;
    (void)hipGetLastError();
  }
  HIP_TRY(hipStreamCreateWithFlags(s, hipStreamNonBlocking));
  return LBM_OK;
}

bool lbm::host::steady_check(lbm_domain d, int id, int64_t window, SteadyCheck& c) {
  if (window < 0 || d->t - 1 - window < 0 || window >= d->rec_cap) return false;
  c.rec = d->rec + id * LBM_REC_LEN;
  c.rec_cap = d->rec_cap;
  c.rec_stride = (int64_t)d->nslots * LBM_REC_LEN;
  c.t = d->t;
  c.window = window;
  const int mode = d->body[id].desc.me_mode;
  c.me_mode = mode == LBM_ME_LATTICE_BACKWARD ? LBM_ME_LATTICE : mode;
  return true;
}

double* lbm::host::rec_slot(lbm_domain d, int64_t t, int b) {
  return d->rec + ((t % d->rec_cap) * d->nslots + b) * LBM_REC_LEN;
}

// make sure the device pose table of body b covers steps [t0, t1]; for a
// FREE body, whose poses the device computes one step ahead, that the
// window has room for step t0 + 1 (the window restarts at t0 otherwise,
// from the device's pose of t0)
lbm_status lbm::host::ensure_poses(lbm_domain d, Body& b, int64_t t0, int64_t t1) {
  if (b.free_motion) {
    if (t0 < b.pose_base) return fail(LBM_E_STATE, "pose window of a free body behind its step");
    if (t0 + 1 - b.pose_base < b.pose_cap) return LBM_OK;
    HIP_TRY(hipMemcpyAsync(b.pose_dev, b.pose_dev + (t0 - b.pose_base) * POSE_LEN, sizeof(Pose),
                           hipMemcpyDeviceToDevice, d->stream));
    b.pose_base = t0;
    return LBM_OK;
  }
  if (t0 >= b.pose_base && t1 < b.pose_base + b.pose_valid) return LBM_OK;
  int64_t need = t1 - t0 + 1;
  int64_t cap = std::max<int64_t>(need, POSE_WINDOW);
  std::vector<Pose> poses((size_t)cap);
  for (int64_t k = 0; k < cap; ++k) {
    poses[k] = body_pose(b, d->g, t0 + k);
    if (b.desc.shape != LBM_SHAPE_OUTER_CIRCLE && !pose_inside(poses[k], d->g)) {
      if (k < need)
        return fail(LBM_E_RANGE, "body leaves the interior (bounding box plus two nodes) at step " +
                                     std::to_string(t0 + k));
      cap = k;  // window ends before the body would leave
      break;
    }
  }
  HIP_TRY(hipStreamSynchronize(d->stream));  // the staging buffer may still be in flight
  if (cap > b.pose_cap) {
    if (b.pose_dev) HIP_TRY(hipFree(b.pose_dev));
    if (b.pose_pinned) HIP_TRY(hipHostFree(b.pose_pinned));
    b.pose_dev = nullptr;
    b.pose_pinned = nullptr;
    HIP_TRY(hipMalloc(&b.pose_dev, cap * POSE_LEN * sizeof(double)));
    HIP_TRY(hipHostMalloc(&b.pose_pinned, cap * POSE_LEN * sizeof(double), hipHostMallocDefault));
    b.pose_cap = cap;
  }
  memcpy(b.pose_pinned, poses.data(), cap * sizeof(Pose));
  HIP_TRY(hipMemcpyAsync(b.pose_dev, b.pose_pinned, cap * sizeof(Pose), hipMemcpyHostToDevice, d->stream));
  b.pose_base = t0;
  b.pose_valid = cap;
  return LBM_OK;
}

const double* lbm::host::pose_at(const Body& b, int64_t t) { return b.pose_dev + (t - b.pose_base) * POSE_LEN; }
const double* lbm::host::pose_host_at(const Body& b, int64_t t) {
  return b.pose_pinned + (t - b.pose_base) * POSE_LEN;
}

// nodes of the box that covers the body region at steps t and t + mode,
// with a one-node margin along each lattice axis (the LDS box of the body
// kernel)
int64_t lbm::host::region_cells(const Body& b, int D, int64_t t, int mode) {
  const Pose* p0 = reinterpret_cast<const Pose*>(b.pose_pinned) + (t - b.pose_base);
  const Pose* p1 = p0 + mode;
  int64_t n = 1;
  for (int a = 0; a < 3; ++a)
    n *= (int64_t)(std::max(p0->hi[a], p1->hi[a]) - std::min(p0->lo[a], p1->lo[a]) + 1) + (a < D ? 2 : 0);
  return n;
}

// rows (y,z) of the same box without the margin
int64_t lbm::host::region_rows(const Body& b, int64_t t, int mode) {
  const Pose* p0 = reinterpret_cast<const Pose*>(b.pose_pinned) + (t - b.pose_base);
  const Pose* p1 = p0 + mode;
  int64_t n = 1;
  for (int a = 1; a < 3; ++a)
    n *= (int64_t)(std::max(p0->hi[a], p1->hi[a]) - std::min(p0->lo[a], p1->lo[a]) + 1);
  return n;
}

int64_t lbm::host::list_bound(const Body& b, int D, int64_t t) {
  const int64_t cells = region_cells(b, D, t, 1);
  if (cells <= 2048) return cells;  // the list holds nodes of the region only
  const Pose* p0 = reinterpret_cast<const Pose*>(b.pose_pinned) + (t - b.pose_base);
  return step_list_nodes(b.shape, p0[0], p0[1], D);
}

bool lbm::host::step_fits(const Body& b, int D, int64_t t) {
  if (b.shape.shape == SHAPE_OUTER_CIRCLE) return false;
  const int64_t cells = region_cells(b, D, t, 1), rows = region_rows(b, t, 1);
  if (!body_step_fits(cells, rows, 0)) return false;
  return body_step_fits(cells, rows, list_bound(b, D, t));
}

lbm_status lbm::host::check_device_errors(lbm_domain d) {
  int e[4] = {0, 0, 0, 0};
  HIP_TRY(hipMemcpy(e, d->err, sizeof(e), hipMemcpyDeviceToHost));
  if (e[0] & 1) return fail(LBM_E_NOMEM, "boundary-link list overflowed its capacity");
  if (e[0] & 2) return fail(LBM_E_RANGE, "a body overlaps a wall layer or another body");
  if (e[0] & 4) return fail(LBM_E_NOMEM, "the surface-node list of a moving body overflowed");
  if (e[0] & 8) return fail(LBM_E_RANGE, "a free body left the interior or reached speed 0.5; it was stopped");
  if (e[1]) return fail(LBM_E_UNSTABLE, "a fluid node's speed exceeded 0.4 lattice units or is not a number");
  return LBM_OK;
}

// rest state everywhere (deviation 0), every node non-fluid until k_init
// marks the active ones, then the equilibrium of the initial fields
static lbm_status init_state(lbm_domain d, const Layout& L, const lbm_domain_desc* desc) {
  HIP_TRY(hipMemsetAsync(d->A, desc->debug_poison ? 0xff : 0, 2 * L.pop_bytes, d->stream));  // 0xff..: NaN
  HIP_TRY(hipMemsetAsync(d->mask, MASK_WALL, 2 * L.mask_bytes, d->stream));
  HIP_TRY(hipMemsetAsync(d->rec, 0, L.rec_bytes + L.err_bytes + L.cnt_bytes, d->stream));
  if (L.face_rec_bytes) HIP_TRY(hipMemsetAsync(d->face_rec, 0, L.face_rec_bytes, d->stream));
  const int64_t N = (int64_t)d->g.nx * d->g.ny * d->g.nz;
  double* rho_dev = nullptr;
  double* u_dev = nullptr;
  hipError_t e = hipSuccess;
  if (desc->init_rho && e == hipSuccess) {
    e = hipMalloc(&rho_dev, N * sizeof(double));
    if (e == hipSuccess) e = hipMemcpy(rho_dev, desc->init_rho, N * sizeof(double), hipMemcpyHostToDevice);
  }
  if (desc->init_u && e == hipSuccess) {
    e = hipMalloc(&u_dev, 3 * N * sizeof(double));
    if (e == hipSuccess) e = hipMemcpy(u_dev, desc->init_u, 3 * N * sizeof(double), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess)
    e = launch_init(d->lat, d->st, d->eq, d->A, d->mask, d->g, d->ph, rho_dev, u_dev, d->rhoA, d->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(d->stream);
  if (rho_dev) (void)hipFree(rho_dev);
  if (u_dev) (void)hipFree(u_dev);
  if (e != hipSuccess) return fail(LBM_E_HIP, std::string("initial state: ") + hipGetErrorString(e));
  return LBM_OK;
}

// fold the oldest event pairs of the timing ring into the running totals
static lbm_status fold_timing(lbm_domain d, int64_t keep) {
  while (d->folded < d->timed - keep) {
    const int k = (int)(d->folded % 64);
    HIP_TRY(hipEventSynchronize(d->ev[1][k]));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, d->ev[0][k], d->ev[1][k]));
    d->kind_ms[d->ev_kind[k]] += ms;
    d->folded++;
  }
  return LBM_OK;
}

// nodes a sweep updates
static int64_t sweep_nodes(const Sweep& sw) {
  const int nz = sw.ntiles / (sw.nbx * sw.ny);
  int64_t n = (int64_t)(sw.xlast - sw.x0 + 1) * sw.ny * nz;
  const int lo[3] = {sw.x0, sw.y0, sw.z0}, hi[3] = {sw.xlast, sw.y0 + sw.ny - 1, sw.z0 + nz - 1};
  int64_t h = 1;
  for (int a = 0; a < 3; ++a)
    h *= std::max(0, std::min(hi[a], sw.hole[2 * a + 1]) - std::max(lo[a], sw.hole[2 * a]) + 1);
  return n - h;
}

// start/stop events of the next timed launch of this kind (null when off)
lbm_status lbm::host::timing_slot(lbm_domain d, int kind, int64_t nodes, hipEvent_t& e0, hipEvent_t& e1) {
  e0 = e1 = nullptr;
  if (!d->timing) return LBM_OK;
  if (d->kind_count[kind]++ % d->timing_every != 0) return LBM_OK;
  lbm_status st = fold_timing(d, 63);
  if (st != LBM_OK) return st;
  const int k = (int)(d->timed % 64);
  e0 = d->ev[0][k];
  e1 = d->ev[1][k];
  d->ev_kind[k] = kind;
  d->timed++;
  d->kind_launches[kind]++;
  d->kind_nodes[kind] += nodes;
  return LBM_OK;
}

// one CU in FAR_CU_EVERY stays free of the far update of a split step
static int FAR_CU_EVERY = 32;

// launch shape of the near-box update: a small box, no block reordering,
// and a shape no full sweep uses, so the near update is a kernel of its own
// in profiles
static const BulkConfig NEAR_CFG{128, 2, 0, 0};

// one stream-collide launch over a sweep of the current source buffer,
// timed as `kind`, on stream s; *done (optional) becomes an event that
// completes with the kernel (its timing stop event when timed, else
// `marker`, recorded by the launch itself). The sweep reads the x-face
// densities of the current state and writes those of the new one.
static lbm_status launch_sweep(lbm_domain d, const BulkConfig& cfg, Sweep sw, int kind, hipStream_t s,
                               hipEvent_t marker = nullptr, hipEvent_t* done = nullptr) {
  sw.rho_in = d->rhoA;
  sw.rho_out = d->rhoB;
  sw.mask = d->mask;
  sw.unstable = d->err + 1;
  hipEvent_t e0, e1;
  lbm_status st = timing_slot(d, kind, sweep_nodes(sw), e0, e1);
  if (st != LBM_OK) return st;
  if (done) *done = e1 ? e1 : marker;
  HIP_TRY(launch_stream_collide(d->lat, d->st, d->eq, d->A, d->B, d->g, d->ph, s, cfg, sw, e0, e1 ? e1 : marker));
  return LBM_OK;
}

// The pose window, trajectory ring and integrator state of a FREE body,
// holding its pose at the current step (the rest comes from the device).
static lbm_status start_free_motion(lbm_domain d, Body& b) {
  const Pose p0 = body_pose(b, d->g, d->t);
  if (!pose_inside(p0, d->g)) return fail(LBM_E_RANGE, "body not inside the interior (bounding box plus two nodes)");
  b.pose_cap = POSE_WINDOW;
  HIP_TRY(hipMalloc(&b.pose_dev, b.pose_cap * POSE_LEN * sizeof(double)));
  HIP_TRY(hipHostMalloc(&b.pose_pinned, POSE_LEN * sizeof(double), hipHostMallocDefault));
  HIP_TRY(hipMalloc(&b.traj, (size_t)d->rec_cap * 8 * sizeof(double)));
  HIP_TRY(hipMalloc(&b.dyn, 16 * sizeof(double)));
  HIP_TRY(hipMemsetAsync(b.dyn, 0, 16 * sizeof(double), d->stream));
  b.pred = b.dyn + 8;
  memcpy(b.pose_pinned, &p0, sizeof(Pose));
  HIP_TRY(hipMemcpyAsync(b.pose_dev, b.pose_pinned, sizeof(Pose), hipMemcpyHostToDevice, d->stream));
  const double row[8] = {p0.X[0], p0.X[1], p0.X[2], p0.theta, p0.V[0], p0.V[1], p0.V[2], p0.Om};
  HIP_TRY(hipMemcpy(b.traj + (d->t % d->rec_cap) * 8, row, sizeof(row), hipMemcpyHostToDevice));
  HIP_TRY(hipStreamSynchronize(d->stream));
  b.pose_base = d->t;
  b.pose_valid = 1;
  return LBM_OK;
}

// Per axis the region of a body's advance (node boxes of two poses less than
// a node apart, two layers each side) spans at most 2h + 8 nodes for the
// half-width h of the body; `cells` adds the one-node margin of the status
// box.
static void region_bounds(int D, const lbm_body_desc& bd, int64_t& cells, int64_t& rows) {
  double h[3];
  if (bd.shape == LBM_SHAPE_ELLIPSE) {
    h[0] = h[1] = std::max(bd.axes[0], bd.axes[1]);
    h[2] = bd.axes[2];
  } else {
    h[0] = h[1] = h[2] = bd.axes[0];
  }
  cells = 1;
  rows = 1;
  for (int a = 0; a < D; ++a) {
    const int64_t n = (int64_t)std::ceil(2.0 * h[a]) + 8;
    cells *= n + 2;
    if (a > 0) rows *= n;
  }
}

// A moving body advances, step by step, in the single-workgroup list kernel
// while its region and near-surface list fit it, and in the many-workgroup
// kernels otherwise; every body whose solid set moves (outer circles aside)
// holds the latter's scratch. A batch takes the same decision for every step
// (it splits a call where a body changes kernels), so a body's records do not
// depend on how it is stepped.
bool lbm::host::wide_advance(int D, const lbm_body_desc& bd) {
  (void)D;
  const bool round = bd.shape != LBM_SHAPE_ELLIPSE;
  const bool moves = !(bd.motion == LBM_MOTION_STATIC || (round && bd.motion == LBM_MOTION_ROTATE));
  return moves && bd.shape != LBM_SHAPE_OUTER_CIRCLE;
}

int lbm::host::wide_slab_bound(int D, const int n[3], const lbm_body_desc& bd) {
  int64_t cells, rows;
  region_bounds(D, bd, cells, rows);
  rows = std::min<int64_t>(rows, D == 2 ? n[1] : (int64_t)n[1] * n[2]);  // within the domain
  return (int)((rows + WIDE_ROWS - 1) / WIDE_ROWS);
}

lbm_status lbm::host::ensure_wide(Body& b, int slabs, hipStream_t s) {
  if (slabs <= b.wide_slabs) return LBM_OK;
  HIP_TRY(hipStreamSynchronize(s));  // the old scratch may still be in use
  if (b.wide) HIP_TRY(hipFree(b.wide));
  b.wide = nullptr;
  b.wide_slabs = 0;
  HIP_TRY(hipMalloc(&b.wide, wide_scratch_bytes(slabs)));
  HIP_TRY(hipMemsetAsync(b.wide, 0, wide_scratch_bytes(slabs), s));
  b.wide_slabs = slabs;
  return LBM_OK;
}

// Sizes of a FREE body's advance that hold at any pose (the host does not
// know the pose): the bounds of region_bounds; a list bound beyond the list
// kernel's when the box is, so that the kernel a free body takes is the same
// at every step.
static void free_bounds(const Body& b, int D, int64_t& cells, int64_t& rows, int64_t& list) {
  region_bounds(D, b.desc, cells, rows);
  list = cells <= STEP_LIST ? cells : (int64_t)STEP_LIST + 1;
}

// The Newton-Euler step of a FREE body from the records of step t: the pose
// of t+1 into the pose window and the trajectory ring.
static lbm_status launch_integrate(lbm_domain d, int id, int64_t t) {
  Body& b = d->body[id];
  lbm_status s = ensure_poses(d, b, t, t + 1);
  if (s != LBM_OK) return s;
  const lbm_body_desc& bd = b.desc;
  FreeBody fb{};
  fb.mass = bd.mass;
  fb.inertia = bd.inertia;
  for (int a = 0; a < 3; ++a) {
    fb.ext_force[a] = bd.ext_force[a];
    fb.axes[a] = bd.axes[a];
    fb.glo[a] = d->g.lo[a];
    fb.ghi[a] = d->g.hi[a];
  }
  fb.ext_torque = bd.ext_torque;
  fb.integrator = bd.integrator;
  fb.drive = bd.me_mode;
  fb.shape = bd.shape;
  fb.D = d->D;
  fb.predicted = (bd.me_mode == LBM_ME_LATTICE || bd.me_mode == LBM_ME_LATTICE_BACKWARD) &&
                 bd.sets == LBM_SETS_PREDICTED;
  if (fb.predicted)
    HIP_TRY(launch_body_predict(d->lat, d->st, d->eq, d->A, d->mask, pose_at(b, t), b.shape, id, d->g, d->ph, b.pred,
                                d->stream));
  const double* rec_tm1 = t > b.t_placed ? rec_slot(d, t - 1, id) : nullptr;
  HIP_TRY(launch_body_integrate(rec_slot(d, t, id), rec_tm1, b.pred, const_cast<double*>(pose_at(b, t)),
                                b.traj + ((t + 1) % d->rec_cap) * 8, b.dyn, fb, d->err, d->stream));
  return LBM_OK;
}

// The advance of body `id` from step t to t+1 on the current source buffer
// (which holds the state of t+1), as its own launch; a FREE body's, after
// its integration.
lbm_status lbm::host::launch_advance(lbm_domain d, int id, int64_t t) {
  Body& b = d->body[id];
  if (b.free_motion) {
    lbm_status si = launch_integrate(d, id, t);
    if (si != LBM_OK) return si;
  }
  hipEvent_t e0, e1;
  lbm_status s = timing_slot(d, LBM_KERNEL_BODY, 0, e0, e1);
  if (s != LBM_OK) return s;
  int64_t cells, rows, list;
  if (b.free_motion) {
    free_bounds(b, d->D, cells, rows, list);
  } else {
    cells = region_cells(b, d->D, t, 1);
    rows = region_rows(b, t, 1);
    // the list bound only decides when the region fits the list kernel
    list = body_step_fits(cells, rows, 0) ? list_bound(b, d->D, t) : (int64_t)STEP_LIST + 1;
    if (b.wide) {
      s = ensure_wide(b, (int)((rows + WIDE_ROWS - 1) / WIDE_ROWS), d->stream);
      if (s != LBM_OK) return s;
    }
  }
  HIP_TRY(launch_body_advance(d->lat, d->st, d->eq, d->A, d->mask, d->mask_next, b.links, b.n_links, b.cap,
                              pose_at(b, t), b.free_motion ? nullptr : pose_host_at(b, t), b.shape, b.desc.bc, id,
                              1, d->g, d->ph, rec_slot(d, t, id), rec_slot(d, t + 1, id), d->err, d->stream, cells,
                              rows, list, b.wide, b.wide_slabs, e0, e1));
  return LBM_OK;
}

// Near box of a fused step: the node boxes of the poses t0..t1 that the
// step's body work touches, plus one layer, within the active nodes.
static void near_box(lbm_domain d, const Body& b, int64_t t0, int64_t t1, int lo[3], int hi[3]) {
  const Geom& g = d->g;
  for (int a = 0; a < 3; ++a) {
    double l = 1e300, h = -1e300;
    for (int64_t k = t0; k <= t1; ++k) {
      const Pose* p = reinterpret_cast<const Pose*>(b.pose_pinned) + (k - b.pose_base);
      l = std::min(l, p->lo[a]);
      h = std::max(h, p->hi[a]);
    }
    lo[a] = std::max<int>(g.lo[a], (int)l - 1);
    hi[a] = std::min<int>(g.hi[a], (int)h + 1);
  }
}

static_assert(sizeof(Pose) == POSE_LEN * sizeof(double), "pose record layout");

// Undoes a placement of body `id` that the device reported as failed: every
// node marked as the body's becomes fluid again (placement touches nothing
// but the node status and the body's own link list), the device error flags
// are cleared and the body's memory is released.
static lbm_status undo_placement(lbm_domain d, int id) {
  Body& b = d->body[id];
  std::vector<uint8_t> m((size_t)d->g.S);
  HIP_TRY(hipMemcpy(m.data(), d->mask, m.size(), hipMemcpyDeviceToHost));
  const uint8_t self = (uint8_t)(MASK_BODY0 + id);
  for (auto& v : m)
    if (v == self) v = MASK_FLUID;
  HIP_TRY(hipMemcpy(d->mask, m.data(), m.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemset(d->err, 0, 4 * sizeof(int)));
  if (b.links) (void)hipFree(b.links);
  if (b.n_links) (void)hipFree(b.n_links);
  if (b.partials) (void)hipFree(b.partials);
  if (b.pose_dev) (void)hipFree(b.pose_dev);
  if (b.pose_pinned) (void)hipHostFree(b.pose_pinned);
  if (b.traj) (void)hipFree(b.traj);
  if (b.dyn) (void)hipFree(b.dyn);
  if (b.wide) (void)hipFree(b.wide);
  b = Body();
  return LBM_OK;
}

// Folds the pending face chunk sums into the face records.
static lbm_status fold_faces(lbm_domain d) {
  if (d->face_part_n == 0) return LBM_OK;
  HIP_TRY(launch_fold_faces(d->face_ring, d->face_chunks, PART_RING, d->face_part_t0, d->face_part_n, d->face_rec,
                            d->rec_cap, d->stream));
  d->face_part_n = 0;
  return LBM_OK;
}

// Folds the pending chunk sums of body b (steps part_t0 .. part_t0 +
// part_n - 1) into its records, on the domain's stream.
static lbm_status fold_pending(lbm_domain d, int id) {
  Body& b = d->body[id];
  if (b.part_n == 0) return LBM_OK;
  HIP_TRY(launch_fold(b.ring, b.ring_chunks, PART_RING, b.part_t0, b.part_n, d->rec + id * LBM_REC_LEN, d->rec_cap,
                      (int64_t)d->nslots * LBM_REC_LEN, !b.mask_moves, d->stream));
  b.part_n = 0;
  return LBM_OK;
}


extern "C" {

const char* lbm_last_error(void) { return g_last_error.c_str(); }

lbm_status lbm_footprint_bytes(const lbm_domain_desc* desc, size_t* bytes) {
  lbm_status s = check_desc(desc);
  if (s != LBM_OK) return s;
  if (!bytes) return fail(LBM_E_INVAL, "null output");
  *bytes = make_layout(desc).total;
  return LBM_OK;
}

lbm_status lbm_body_footprint_bytes(const lbm_domain_desc* desc, const lbm_body_desc* bd, size_t* bytes) {
  lbm_status s = check_desc(desc);
  if (s != LBM_OK) return s;
  if (!bd || !bytes) return fail(LBM_E_INVAL, "null argument");
  const int D = desc->lattice == LBM_D2Q9 ? 2 : 3;
  const size_t cap = (size_t)link_capacity(D, bd);
  *bytes = cap * sizeof(Link) + sizeof(int) + (cap + 63) / 64 * 12 * sizeof(double) +
           (size_t)POSE_WINDOW * POSE_LEN * sizeof(double);
  if (wide_advance(D, *bd)) {
    const int n[3] = {desc->nx, desc->ny, D == 3 ? desc->nz : 1};
    *bytes += wide_scratch_bytes(wide_slab_bound(D, n, *bd));
  }
  return LBM_OK;
}

lbm_status lbm_create_domain(const lbm_domain_desc* desc, lbm_domain* out) {
  lbm_status s = check_desc(desc);
  if (s != LBM_OK) return s;
  if (!out) return fail(LBM_E_INVAL, "null output");
  Layout L = make_layout(desc);
  lbm_domain d = new lbm_domain_s();
  d->desc = *desc;
  d->desc.init_rho = nullptr;
  d->desc.init_u = nullptr;
  d->lat = desc->lattice;
  d->st = desc->storage;
  d->eq = desc->eq_model;
  d->D = L.g.D;
  d->Q = d->D == 2 ? 9 : 19;
  d->elem = desc->storage == LBM_F64 ? 8 : (desc->storage == LBM_F32 ? 4 : 2);
  d->g = L.g;
  d->ph.tau = desc->tau;
  d->ph.omega = 1.0 / desc->tau;
  d->ph.rho0 = desc->rho0;
  d->ph.eq = desc->eq_model;
  d->ph.inlet_profile = desc->inlet_profile;
  d->ph.inlet_u = desc->inlet_u;
  d->ph.inlet_ky = 4.0 / ((desc->ny - 2.0) * (desc->ny - 2.0));
  d->ph.inlet_kz = 4.0 / ((desc->nz - 2.0) * (desc->nz - 2.0));
  d->stream = (hipStream_t)desc->stream;
  d->own_stream = d->stream;
  d->rec_cap = L.rec_cap;
  d->nslots = body_slots(desc);
  d->bulk = bulk_config(d->lat, d->st, 2 * L.pop_bytes);
  if (desc->device_buffer) {
    if (desc->device_buffer_bytes < L.total) {
      delete d;
      return fail(LBM_E_NOMEM, "device_buffer smaller than lbm_footprint_bytes");
    }
    d->pool = (char*)desc->device_buffer;
    d->owns_pool = false;
  } else {
    if (hipMalloc(&d->pool, L.total) != hipSuccess) {
      delete d;
      return fail(LBM_E_NOMEM, "hipMalloc of " + std::to_string(L.total) + " bytes failed");
    }
    d->owns_pool = true;
  }
  d->pool_bytes = L.total;
  char* p = d->pool;
  d->A = p;
  p += L.pop_bytes;
  d->B = p;
  p += L.pop_bytes;
  d->mask = (uint8_t*)p;
  p += L.mask_bytes;
  d->mask_next = (uint8_t*)p;
  p += L.mask_bytes;
  d->rec = (double*)p;
  p += L.rec_bytes;
  d->err = (int*)p;
  p += L.err_bytes;
  d->counters = (unsigned*)p;
  p += L.cnt_bytes;
  if (L.rho_bytes) {
    d->rhoA = p;
    p += L.rho_bytes;
    d->rhoB = p;
    p += L.rho_bytes;
  }
  if (L.face_rec_bytes) {
    d->face_rec = (double*)p;
    p += L.face_rec_bytes;
    d->face_ring = (double*)p;
    p += L.face_ring_bytes;
    d->face_chunks = face_chunks(L.g);
  }
  s = init_state(d, L, desc);
  if (s != LBM_OK) {
    std::string msg = g_last_error;
    lbm_destroy_domain(d);
    return fail(s, msg);
  }
  *out = d;
  return LBM_OK;
}

lbm_status lbm_destroy_domain(lbm_domain d) {
  if (!d) return fail(LBM_E_INVAL, "null domain");
  if (d->batch) {
    lbm_status s = lbm_batch_remove(d->batch, d);
    if (s != LBM_OK) return s;
  }
  solo_destroy(d);
  hipError_t e = hipStreamSynchronize(d->stream);
  for (auto& b : d->body) {
    if (b.links) (void)hipFree(b.links);
    if (b.n_links) (void)hipFree(b.n_links);
    if (b.partials) (void)hipFree(b.partials);
    if (b.ring) (void)hipFree(b.ring);
    if (b.traj) (void)hipFree(b.traj);
    if (b.dyn) (void)hipFree(b.dyn);
    if (b.pose_dev) (void)hipFree(b.pose_dev);
    if (b.pose_pinned) (void)hipHostFree(b.pose_pinned);
    if (b.wide) (void)hipFree(b.wide);
  }
  if (d->aux) {
    hipError_t ea = hipStreamSynchronize(d->aux);
    if (e == hipSuccess) e = ea;
    (void)hipStreamDestroy(d->aux);
    (void)hipEventDestroy(d->e_near);
    (void)hipEventDestroy(d->e_far);
  }
  if (d->steady_buf) (void)hipFree(d->steady_buf);
  if (d->owns_pool) (void)hipFree(d->pool);
  for (int k = 0; k < 64; ++k)
    for (int j = 0; j < 2; ++j)
      if (d->ev[j][k]) (void)hipEventDestroy(d->ev[j][k]);
  delete d;
  if (e != hipSuccess) return fail(LBM_E_HIP, hipGetErrorString(e));
  return LBM_OK;
}

lbm_status lbm_set_body(lbm_domain d, int32_t id, const lbm_body_desc* bd) {
  if (!d || !bd) return fail(LBM_E_INVAL, "null argument");
  if (id < 0 || id >= d->nslots) return fail(LBM_E_INVAL, "body id out of range");
  Body& b = d->body[id];
  if (b.active) return fail(LBM_E_STATE, "body id already in use");
  if (bd->shape < 0 || bd->shape > 2) return fail(LBM_E_INVAL, "unknown shape");
  if (bd->bc != LBM_BC_HALFWAY && bd->bc != LBM_BC_MLS) return fail(LBM_E_INVAL, "unknown boundary rule");
  if (bd->me_mode < 0 || bd->me_mode > 3) return fail(LBM_E_INVAL, "unknown me_mode");
  if (bd->motion < 0 || bd->motion > 5) return fail(LBM_E_INVAL, "unknown motion");
  if (bd->refill < 0 || bd->refill > 2) return fail(LBM_E_INVAL, "unknown refill rule");
  if (bd->motion == LBM_MOTION_FREE) {
    if (!(bd->mass > 0) || !(bd->inertia > 0)) return fail(LBM_E_INVAL, "a free body needs positive mass and inertia");
    if (bd->integrator != LBM_INTEGRATOR_EULER && bd->integrator != LBM_INTEGRATOR_AB2)
      return fail(LBM_E_INVAL, "unknown integrator");
    if (d->batch) return fail(LBM_E_STATE, "a free body is stepped alone, not in a batch");
    if (bd->sets != LBM_SETS_PREVIOUS && bd->sets != LBM_SETS_PREDICTED) return fail(LBM_E_INVAL, "unknown sets");
  }
  const int na = bd->shape == LBM_SHAPE_ELLIPSE ? d->D : 1;
  for (int a = 0; a < na; ++a)
    if (!(bd->axes[a] > 0)) return fail(LBM_E_INVAL, "axes must be positive");
  if (bd->motion == LBM_MOTION_OSCILLATE && !(bd->period > 0)) return fail(LBM_E_INVAL, "period must be positive");
  if (bd->motion == LBM_MOTION_TABLE && (!bd->pose_table || bd->pose_count <= 0))
    return fail(LBM_E_INVAL, "TABLE motion needs rows");
  if (bd->shape == LBM_SHAPE_OUTER_CIRCLE && bd->motion != LBM_MOTION_STATIC)
    return fail(LBM_E_INVAL, "an outer circle must be static");
  Body nb;
  nb.desc = *bd;
  nb.desc.pose_table = nullptr;
  if (bd->motion == LBM_MOTION_TABLE) nb.table.assign(bd->pose_table, bd->pose_table + 8 * bd->pose_count);
  nb.shape.shape = bd->shape;
  nb.shape.D = d->D;
  nb.shape.R = bd->axes[0];
  nb.shape.ia2 = 1.0 / (bd->axes[0] * bd->axes[0]);
  nb.shape.ib2 = bd->shape == LBM_SHAPE_ELLIPSE ? 1.0 / (bd->axes[1] * bd->axes[1]) : 0.0;
  nb.shape.ic2 = (bd->shape == LBM_SHAPE_ELLIPSE && d->D == 3) ? 1.0 / (bd->axes[2] * bd->axes[2]) : 0.0;
  nb.shape.refill = bd->refill;
  const bool round = bd->shape != LBM_SHAPE_ELLIPSE;
  nb.mask_moves = !(bd->motion == LBM_MOTION_STATIC || (round && bd->motion == LBM_MOTION_ROTATE));
  nb.free_motion = bd->motion == LBM_MOTION_FREE;
  nb.t_placed = d->t;
  nb.cap = link_capacity(d->D, bd);
  b = std::move(nb);
  HIP_TRY(hipMalloc(&b.links, (size_t)b.cap * sizeof(Link)));
  HIP_TRY(hipMalloc(&b.n_links, sizeof(int)));
  HIP_TRY(hipMalloc(&b.partials, (size_t)((b.cap + 63) / 64) * 12 * sizeof(double)));
  HIP_TRY(hipMemsetAsync(b.n_links, 0, sizeof(int), d->stream));
  lbm_status s = b.free_motion ? start_free_motion(d, b) : ensure_poses(d, b, d->t, d->t + 1);
  if (s != LBM_OK) {
    (void)hipFree(b.links);
    (void)hipFree(b.n_links);
    (void)hipFree(b.partials);
    if (b.traj) (void)hipFree(b.traj);
    if (b.dyn) (void)hipFree(b.dyn);
    b = Body();
    return s;
  }
  HIP_TRY(launch_body_advance(d->lat, d->st, d->eq, d->A, d->mask, d->mask_next, b.links, b.n_links, b.cap,
                              pose_at(b, d->t), pose_host_at(b, d->t), b.shape, bd->bc, id, 0, d->g, d->ph, nullptr,
                              nullptr, d->err,
                              d->stream, region_cells(b, d->D, d->t, 0), region_rows(b, d->t, 0), 0));
  if (d->desc.debug_poison) {
    const Pose* P = reinterpret_cast<const Pose*>(pose_host_at(b, d->t));
    const int lo[3] = {(int)P->lo[0], (int)P->lo[1], (int)P->lo[2]}, hi[3] = {(int)P->hi[0], (int)P->hi[1],
                                                                            (int)P->hi[2]};
    HIP_TRY(launch_poison_body(d->lat, d->st, d->eq, d->A, d->B, d->mask, d->g, lo, hi, id, d->stream));
  }
  HIP_TRY(hipMemcpyAsync(&b.n_host, b.n_links, sizeof(int), hipMemcpyDeviceToHost, d->stream));
  HIP_TRY(hipStreamSynchronize(d->stream));
  s = check_device_errors(d);
  if (s != LBM_OK) {
    // a failed placement is undone: the body's nodes become fluid again (the
    // placement changed nothing else), the error flags are cleared and the id
    // is free
    const std::string msg = g_last_error;
    lbm_status su = undo_placement(d, id);
    return su != LBM_OK ? su : fail(s, msg);
  }
  b.ring_chunks = std::max(1, (b.n_host + 63) / 64);
  HIP_TRY(hipMalloc(&b.ring, (size_t)PART_RING * b.ring_chunks * 12 * sizeof(double)));
  if (wide_advance(d->D, *bd)) {
    const int n[3] = {d->g.nx, d->g.ny, d->g.nz};
    s = ensure_wide(b, wide_slab_bound(d->D, n, *bd), d->stream);
    if (s != LBM_OK) return s;
  }
  b.part_n = 0;
  b.active = true;
  b.bc_ready = false;
  return LBM_OK;
}

// One step is, in order: the boundary rule + momentum exchange of bodies
// whose links are fixed (k_links, on the source buffer), the stream-collide
// update of every node, and the advance of bodies whose solid set moves (on
// the new state). In the split schedule of a single body the update is split
// in two: the nodes of a near box around the body are updated on the
// domain's stream, after the body's link rule there (fixed links) or followed
// there by the body's advance (moving solid set), while every other node is
// updated on the domain's second stream. The far update of step t waits for
// the near update of step t-1, and the near update and link rule of step t
// for the far update of step t-1, so the body work of one step overlaps a
// far update. The near box holds the node boxes of poses t-1, t and t+1 plus
// one layer: every node the link rule or an advance reads or writes (the
// pose's node box holds the body, its links' fluid nodes and the second
// fluid nodes the interpolated rule reads) lies inside it, away from the
// nodes the far update reads and writes. Every node is updated from the same
// values either way.
lbm_status lbm_step(lbm_domain d, int64_t nsteps) {
  if (!d) return fail(LBM_E_INVAL, "null domain");
  if (nsteps < 0) return fail(LBM_E_INVAL, "negative step count");
  if (nsteps == 0) return LBM_OK;
  int only = -1, nactive = 0;
  for (int id = 0; id < d->nslots; ++id)
    if (d->body[id].active) {
      lbm_status s = ensure_poses(d, d->body[id], d->t, d->t + nsteps);
      if (s != LBM_OK) return s;
      only = id;
      nactive++;
    }
  bool any_free = false;
  for (int id = 0; id < d->nslots; ++id) any_free = any_free || (d->body[id].active && d->body[id].free_motion);
  const bool single = nactive == 1 && !d->body[only].free_motion && d->body[only].desc.shape != LBM_SHAPE_OUTER_CIRCLE;
  const bool one_moving = single && d->body[only].mask_moves;
  const int ask = d->desc.split_schedule;
  // several bodies, or one body whose solid set moves: batched launches of
  // the domain's own one-member batch, whose overlapped step updates the
  // nodes away from the bodies beside the body work (the 2000 x 800
  // oscillating cylinder: 34.6 us per step against 39.1 us with the launches
  // below); bodies with fixed links alone keep the deferred link-rule sums
  if ((nactive >= 2 || (one_moving && ask == 0)) && !any_free && !d->face_rec && !d->batch)
    return solo_step(d, nsteps);
  // a single body in the split schedule only when asked for: beside other
  // kernels the far update loses about a tenth of its bandwidth (the 256 x
  // 128 x 128 duct with a fixed sphere: 117 us per step split against 110.5
  // us plain), more than the link rule it hides
  const bool split = single && ask == 1;
  if (split && !d->aux) {
    // compute units kept free for a moving body's one-workgroup advance; a
    // fixed body's link rule needs none (with one unit in 32 masked off the
    // duct's far update took 129 us against 113 us unmasked)
    lbm_status sa = create_far_stream(d->stream, &d->aux, one_moving ? FAR_CU_EVERY : 0);
    if (sa != LBM_OK) return sa;
    HIP_TRY(hipEventCreateWithFlags(&d->e_near, hipEventDisableTiming | hipEventDisableSystemFence));
    HIP_TRY(hipEventCreateWithFlags(&d->e_far, hipEventDisableTiming | hipEventDisableSystemFence));
  }
  const Geom& g = d->g;
  const int full_lo[3] = {g.lo[0], g.lo[1], g.lo[2]}, full_hi[3] = {g.hi[0], g.hi[1], g.hi[2]};
  const Sweep full = make_sweep(full_lo, full_hi, d->bulk.block * d->bulk.cells_per_thread, nullptr, d->bulk.remap);
  bool far_open = false;  // a far update on the second stream is not yet waited for
  hipEvent_t far_done = nullptr, near_done = nullptr;  // completion of the last far / near update
  for (int64_t k = 0; k < nsteps; ++k) {
    const int64_t t = d->t;
    lbm_status s = LBM_OK;
    hipEvent_t e0, e1;
    Sweep near{};
    if (split) {
      Body& b = d->body[only];
      int lo[3], hi[3];
      near_box(d, b, t - 1 >= b.pose_base ? t - 1 : t, t + 1, lo, hi);
      const int hole[6] = {lo[0], hi[0], lo[1], hi[1], lo[2], hi[2]};
      const Sweep far = make_sweep(full_lo, full_hi, d->bulk.block * d->bulk.cells_per_thread, hole, d->bulk.remap);
      near = make_sweep(lo, hi, NEAR_CFG.block * NEAR_CFG.cells_per_thread, nullptr, 0);
      // the far update of step t after the near update of step t-1 (at the
      // first split step: after all earlier work of the domain's stream);
      // the near update after the far update of step t-1. Each completion
      // event is recorded by its kernel's launch.
      if (far_open) {
        HIP_TRY(hipStreamWaitEvent(d->stream, far_done, 0));
      } else {
        HIP_TRY(hipEventRecord(d->e_near, d->stream));
        near_done = d->e_near;
      }
      HIP_TRY(hipStreamWaitEvent(d->aux, near_done, 0));
      if ((s = launch_sweep(d, d->bulk, far, LBM_KERNEL_STREAM_COLLIDE, d->aux, d->e_far, &far_done)) != LBM_OK)
        return s;
      far_open = true;
    }
    for (int id = 0; id < d->nslots; ++id) {
      Body& b = d->body[id];
      if (!b.active || (b.mask_moves && b.bc_ready)) continue;
      if ((s = timing_slot(d, LBM_KERNEL_BODY, 0, e0, e1)) != LBM_OK) return s;
      if (b.part_n == 0) b.part_t0 = t;
      HIP_TRY(launch_links_part(d->lat, d->st, d->eq, d->A, b.links, b.n_host, pose_at(b, t), b.desc.bc, d->mask, g,
                                d->ph, b.ring + (t % PART_RING) * (int64_t)b.ring_chunks * 12, d->stream, e0, e1));
      // (a free body's integration reads the record of this step at once)
      if ((++b.part_n == PART_RING || b.free_motion) && (s = fold_pending(d, id)) != LBM_OK) return s;
      if (b.mask_moves) b.bc_ready = true;
    }
    if (d->face_rec) {  // the faces' momentum exchange of step t, from the state of t
      if (d->face_part_n == 0) d->face_part_t0 = t;
      HIP_TRY(launch_face_part(d->lat, d->st, d->eq, d->A, g, d->ph, d->rhoA,
                               d->face_ring + (t % PART_RING) * (int64_t)d->face_chunks * LBM_FACE_REC_LEN,
                               d->stream));
      if (++d->face_part_n == PART_RING && (s = fold_faces(d)) != LBM_OK) return s;
    }
    if (split) {
      if ((s = launch_sweep(d, NEAR_CFG, near, LBM_KERNEL_NEAR_BOX, d->stream, d->e_near, &near_done)) != LBM_OK)
        return s;
    } else {
      if ((s = launch_sweep(d, d->bulk, full, LBM_KERNEL_STREAM_COLLIDE, d->stream)) != LBM_OK) return s;
    }
    std::swap(d->A, d->B);  // the advance works on the new state
    std::swap(d->rhoA, d->rhoB);
    for (int id = 0; id < d->nslots; ++id) {
      Body& b = d->body[id];
      if (!b.active || !b.mask_moves) continue;
      if ((s = launch_advance(d, id, t)) != LBM_OK) {
        std::swap(d->A, d->B);
        std::swap(d->rhoA, d->rhoB);
        return s;
      }
    }
    d->t = t + 1;
  }
  if (far_open) HIP_TRY(hipStreamWaitEvent(d->stream, far_done, 0));
  for (int id = 0; id < d->nslots; ++id)
    if (d->body[id].active) {
      lbm_status s = fold_pending(d, id);
      if (s != LBM_OK) return s;
    }
  return fold_faces(d);
}

lbm_status lbm_synchronize(lbm_domain d) {
  if (!d) return fail(LBM_E_INVAL, "null domain");
  HIP_TRY(hipStreamSynchronize(d->stream));
  return check_device_errors(d);
}

int64_t lbm_time(lbm_domain d) { return d ? d->t : -1; }

lbm_status lbm_records(lbm_domain d, int32_t id, int64_t first, int64_t count, double* rec) {
  if (!d || !rec) return fail(LBM_E_INVAL, "null argument");
  if (id < 0 || id >= d->nslots || !d->body[id].active) return fail(LBM_E_INVAL, "no such body");
  if (count < 0 || first < 0 || first + count > d->t || first < d->t - d->rec_cap)
    return fail(LBM_E_RANGE, "steps outside the record ring");
  // an instability flag still lets the records be read (they show where it
  // began); the status is returned after the copy
  lbm_status s = lbm_synchronize(d);
  if (s != LBM_OK && s != LBM_E_UNSTABLE) return s;
  const std::string dev_msg = s == LBM_E_UNSTABLE ? g_last_error : std::string();
  std::vector<double> buf;
  int64_t k = 0;
  while (k < count) {
    int64_t slot = (first + k) % d->rec_cap;
    int64_t run = std::min(count - k, d->rec_cap - slot);
    buf.resize((size_t)run * d->nslots * LBM_REC_LEN);
    HIP_TRY(hipMemcpy(buf.data(), d->rec + slot * d->nslots * LBM_REC_LEN, buf.size() * sizeof(double),
                      hipMemcpyDeviceToHost));
    for (int64_t j = 0; j < run; ++j)
      memcpy(rec + (k + j) * LBM_REC_LEN, buf.data() + (j * d->nslots + id) * LBM_REC_LEN,
             LBM_REC_LEN * sizeof(double));
    k += run;
  }
  if (s == LBM_E_UNSTABLE) return fail(s, dev_msg);
  for (int64_t j = 0; j < count * LBM_REC_LEN; ++j)
    if (!isfinite(rec[j])) return fail(LBM_E_UNSTABLE, "non-finite force or torque");
  return LBM_OK;
}

lbm_status lbm_face_records(lbm_domain d, int64_t first, int64_t count, double* rec) {
  if (!d || !rec) return fail(LBM_E_INVAL, "null argument");
  if (!d->face_rec) return fail(LBM_E_STATE, "the domain does not record its faces (face_records = 0)");
  if (count < 0 || first < 0 || first + count > d->t || first < d->t - d->rec_cap)
    return fail(LBM_E_RANGE, "steps outside the record ring");
  lbm_status s = lbm_synchronize(d);
  if (s != LBM_OK && s != LBM_E_UNSTABLE) return s;
  const std::string dev_msg = s == LBM_E_UNSTABLE ? g_last_error : std::string();
  int64_t k = 0;
  while (k < count) {
    const int64_t slot = (first + k) % d->rec_cap;
    const int64_t run = std::min(count - k, d->rec_cap - slot);
    HIP_TRY(hipMemcpy(rec + k * LBM_FACE_REC_LEN, d->face_rec + slot * LBM_FACE_REC_LEN,
                      run * LBM_FACE_REC_LEN * sizeof(double), hipMemcpyDeviceToHost));
    k += run;
  }
  if (s == LBM_E_UNSTABLE) return fail(s, dev_msg);
  return LBM_OK;
}

lbm_status lbm_get_moving_sets(lbm_domain d, int32_t id, int64_t step, int64_t* n_plus, int64_t* n_minus) {
  if (!d || !n_plus || !n_minus) return fail(LBM_E_INVAL, "null argument");
  double r[LBM_REC_LEN];
  lbm_status s = lbm_records(d, id, step, 1, r);
  if (s != LBM_OK) return s;
  *n_plus = (int64_t)r[LBM_REC_N_COVERED];
  *n_minus = (int64_t)r[LBM_REC_N_UNCOVERED];
  return LBM_OK;
}

lbm_status lbm_force_torque(lbm_domain d, int32_t id, int64_t first, int64_t count, double* ft) {
  if (!d || !ft) return fail(LBM_E_INVAL, "null argument");
  if (id == LBM_WALLS) {
    std::vector<double> rec((size_t)std::max<int64_t>(count, 0) * LBM_FACE_REC_LEN);
    lbm_status s = lbm_face_records(d, first, count, rec.data());
    if (s != LBM_OK && s != LBM_E_UNSTABLE) return s;
    for (int64_t k = 0; k < count; ++k)
      for (int a = 0; a < 6; ++a) ft[6 * k + a] = rec[k * LBM_FACE_REC_LEN + a];
    return s;
  }
  if (id < 0 || id >= d->nslots || !d->body[id].active) return fail(LBM_E_INVAL, "no such body");
  const int mode = d->body[id].desc.me_mode;
  // the backward form also takes the node terms of the step before the first
  const int64_t pre = (mode == LBM_ME_LATTICE_BACKWARD && first > 0 && count > 0) ? 1 : 0;
  std::vector<double> rec((size_t)std::max<int64_t>(count + pre, 0) * LBM_REC_LEN);
  lbm_status s = lbm_records(d, id, first - pre, count + pre, rec.data());
  if (s != LBM_OK && s != LBM_E_UNSTABLE) return s;
  for (int64_t k = 0; k < count; ++k) {
    const double* r = rec.data() + (k + pre) * LBM_REC_LEN;
    const double* rp = (k + pre > 0) ? r - LBM_REC_LEN : nullptr;  // step t - 1 (none before step 0)
    for (int a = 0; a < 6; ++a) {
      double v;
      if (mode == LBM_ME_STATIC) v = r[LBM_REC_F_STATIC + a];
      else if (mode == LBM_ME_LATTICE) v = r[LBM_REC_F_STATIC + a] + r[LBM_REC_F_NODES + a];
      else if (mode == LBM_ME_LATTICE_BACKWARD) v = r[LBM_REC_F_STATIC + a] + (rp ? rp[LBM_REC_F_NODES + a] : 0.0);
      else v = r[LBM_REC_F_COMOVING + a];
      ft[6 * k + a] = v;
    }
  }
  return s;
}

lbm_status lbm_body_trajectory(lbm_domain d, int32_t id, int64_t first, int64_t count, double* out) {
  if (!d || (!out && count > 0)) return fail(LBM_E_INVAL, "null argument");
  if (id < 0 || id >= d->nslots || !d->body[id].active) return fail(LBM_E_INVAL, "no such body");
  if (count < 0 || first < 0) return fail(LBM_E_RANGE, "negative step or count");
  Body& b = d->body[id];
  if (!b.free_motion) {
    for (int64_t k = 0; k < count; ++k) {
      const Pose p = body_pose(b, d->g, first + k);
      const double row[8] = {p.X[0], p.X[1], p.X[2], p.theta, p.V[0], p.V[1], p.V[2], p.Om};
      memcpy(out + 8 * k, row, sizeof(row));
    }
    return LBM_OK;
  }
  if (first < b.t_placed || first + count - 1 > d->t || first <= d->t - d->rec_cap)
    return fail(LBM_E_RANGE, "steps outside the trajectory ring");
  lbm_status s = lbm_synchronize(d);
  if (s != LBM_OK && s != LBM_E_UNSTABLE) return s;
  for (int64_t k = 0; k < count;) {  // at most two contiguous runs of the ring
    const int64_t slot = (first + k) % d->rec_cap;
    const int64_t run = std::min(count - k, d->rec_cap - slot);
    HIP_TRY(hipMemcpy(out + 8 * k, b.traj + slot * 8, (size_t)run * 8 * sizeof(double), hipMemcpyDeviceToHost));
    k += run;
  }
  return s;
}

lbm_status lbm_get_links(lbm_domain d, int32_t id, int64_t cap, int64_t* node, int32_t* dir, double* delta,
                         int64_t* n) {
  if (!d || !n) return fail(LBM_E_INVAL, "null argument");
  if (id < 0 || id >= d->nslots || !d->body[id].active) return fail(LBM_E_INVAL, "no such body");
  lbm_status s = lbm_synchronize(d);
  if (s != LBM_OK) return s;
  Body& b = d->body[id];
  int cnt = 0;
  HIP_TRY(hipMemcpy(&cnt, b.n_links, sizeof(int), hipMemcpyDeviceToHost));
  *n = cnt;
  int64_t m = std::min<int64_t>(cap, cnt);
  if (m <= 0) return LBM_OK;
  std::vector<Link> L((size_t)m);
  HIP_TRY(hipMemcpy(L.data(), b.links, m * sizeof(Link), hipMemcpyDeviceToHost));
  for (int64_t k = 0; k < m; ++k) {
    if (node) node[k] = L[k].x + (int64_t)d->g.nx * (L[k].y + (int64_t)d->g.ny * L[k].z);
    if (dir) dir[k] = L[k].dir;
    if (delta) delta[k] = L[k].delta;
  }
  return LBM_OK;
}

lbm_status lbm_steady_state(lbm_domain d, int32_t id, int64_t window, double tol, int32_t* steady,
                            double* rel_change) {
  if (!d || !steady) return fail(LBM_E_INVAL, "null argument");
  if (id < 0 || id >= d->nslots || !d->body[id].active) return fail(LBM_E_INVAL, "no such body");
  SteadyCheck c{};
  if (!steady_check(d, id, window, c)) return fail(LBM_E_RANGE, "the record ring does not hold both steps");
  if (!d->steady_buf) HIP_TRY(hipMalloc(&d->steady_buf, 256));
  HIP_TRY(hipMemcpyAsync(d->steady_buf, &c, sizeof(c), hipMemcpyHostToDevice, d->stream));
  double* out = reinterpret_cast<double*>(d->steady_buf + 128);
  HIP_TRY(launch_steady(reinterpret_cast<const SteadyCheck*>(d->steady_buf), 1, out, d->stream));
  double r[2];
  HIP_TRY(hipMemcpyAsync(r, out, sizeof(r), hipMemcpyDeviceToHost, d->stream));
  lbm_status s = lbm_synchronize(d);
  if (s != LBM_OK) return s;
  *steady = r[0] < tol ? 1 : 0;
  if (rel_change) *rel_change = r[0];
  return LBM_OK;
}

lbm_status lbm_get_types(lbm_domain d, int32_t* type) {
  if (!d || !type) return fail(LBM_E_INVAL, "null argument");
  lbm_status s = lbm_synchronize(d);
  if (s != LBM_OK) return s;
  std::vector<uint8_t> m((size_t)d->g.S);
  HIP_TRY(hipMemcpy(m.data(), d->mask, m.size(), hipMemcpyDeviceToHost));
  const Geom& g = d->g;
  for (int z = 0; z < g.nz; ++z)
    for (int y = 0; y < g.ny; ++y)
      for (int x = 0; x < g.nx; ++x) type[x + (int64_t)g.nx * (y + (int64_t)g.ny * z)] = m[g.idx(x, y, z)];
  return LBM_OK;
}

int32_t lbm_lattice(int32_t lattice, int32_t* c, double* w) {
  if (lattice != LBM_D2Q9 && lattice != LBM_D3Q19) return -1;
  const int Q = lattice == LBM_D2Q9 ? 9 : 19;
  for (int i = 0; i < Q; ++i) {
    if (c) {
      c[3 * i] = lattice == LBM_D2Q9 ? D2Q9::cx(i) : D3Q19::cx(i);
      c[3 * i + 1] = lattice == LBM_D2Q9 ? D2Q9::cy(i) : D3Q19::cy(i);
      c[3 * i + 2] = lattice == LBM_D2Q9 ? 0 : D3Q19::cz(i);
    }
    if (w) w[i] = lattice == LBM_D2Q9 ? D2Q9::w(i) : D3Q19::w(i);
  }
  return Q;
}

lbm_status lbm_get_populations(lbm_domain d, double* f) {
  if (!d || !f) return fail(LBM_E_INVAL, "null argument");
  lbm_status s = lbm_synchronize(d);
  if (s != LBM_OK && s != LBM_E_UNSTABLE) return s;
  const Geom& g = d->g;
  std::vector<uint8_t> m((size_t)g.S);
  HIP_TRY(hipMemcpy(m.data(), d->mask, m.size(), hipMemcpyDeviceToHost));
  std::vector<char> raw((size_t)d->Q * g.S * d->elem);
  HIP_TRY(hipMemcpy(raw.data(), d->A, raw.size(), hipMemcpyDeviceToHost));
  double w[19];
  lbm_lattice(d->lat, nullptr, w);
  for (int z = 0; z < g.nz; ++z)
    for (int y = 0; y < g.ny; ++y)
      for (int x = 0; x < g.nx; ++x) {
        const int64_t n = x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
        const int64_t c = g.idx(x, y, z);
        for (int i = 0; i < d->Q; ++i) {
          const int64_t k = i * g.S + c;
          double h;
          if (d->st == LBM_F64) h = ((const double*)raw.data())[k];
          else if (d->st == LBM_F32) h = ((const float*)raw.data())[k];
          else h = (double)(float)((const _Float16*)raw.data())[k];
          f[n * d->Q + i] = m[c] == MASK_FLUID ? h + w[i] * d->ph.rho0 : NAN;
        }
      }
  return s;
}

lbm_status lbm_get_fields(lbm_domain d, double* rho, double* u) {
  if (!d || !rho || !u) return fail(LBM_E_INVAL, "null argument");
  lbm_status s = lbm_synchronize(d);
  if (s != LBM_OK) return s;
  const Geom& g = d->g;
  std::vector<uint8_t> m((size_t)g.S);
  HIP_TRY(hipMemcpy(m.data(), d->mask, m.size(), hipMemcpyDeviceToHost));
  std::vector<char> raw((size_t)d->Q * g.S * d->elem);
  HIP_TRY(hipMemcpy(raw.data(), d->A, raw.size(), hipMemcpyDeviceToHost));
  auto value = [&](int i, int64_t c) -> double {
    int64_t k = i * g.S + c;
    if (d->st == LBM_F64) return ((const double*)raw.data())[k];
    if (d->st == LBM_F32) return ((const float*)raw.data())[k];
    return (double)(float)((const _Float16*)raw.data())[k];
  };
  auto C = [&](int i, int a) -> int {
    if (d->D == 2) {
      const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1}, cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
      return a == 0 ? cx[i] : (a == 1 ? cy[i] : 0);
    }
    return a == 0 ? D3Q19::cx(i) : (a == 1 ? D3Q19::cy(i) : D3Q19::cz(i));
  };
  bool finite = true;
  for (int z = 0; z < g.nz; ++z)
    for (int y = 0; y < g.ny; ++y)
      for (int x = 0; x < g.nx; ++x) {
        const int64_t n = x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
        const int64_t c = g.idx(x, y, z);
        if (m[c] != MASK_FLUID) {
          rho[n] = NAN;
          u[3 * n] = u[3 * n + 1] = u[3 * n + 2] = NAN;
          continue;
        }
        double dr = 0, j[3] = {0, 0, 0};
        for (int i = 0; i < d->Q; ++i) {
          double v = value(i, c);
          dr += v;
          for (int a = 0; a < 3; ++a) j[a] += C(i, a) * v;
        }
        const double r = d->ph.rho0 + dr;
        const double den = d->eq ? d->ph.rho0 : r;
        rho[n] = r;
        for (int a = 0; a < 3; ++a) u[3 * n + a] = j[a] / den;
        finite = finite && isfinite(r);
      }
  if (!finite) return fail(LBM_E_UNSTABLE, "non-finite density in the fluid");
  return LBM_OK;
}

lbm_status lbm_get_sweep_config(lbm_domain d, lbm_sweep_config* cfg) {
  if (!d || !cfg) return fail(LBM_E_INVAL, "null argument");
  cfg->block = d->bulk.block;
  cfg->cells_per_thread = d->bulk.cells_per_thread;
  cfg->memory = d->bulk.nontemporal;
  cfg->remap = d->bulk.remap;
  return LBM_OK;
}

lbm_status lbm_set_sweep_config(lbm_domain d, const lbm_sweep_config* cfg) {
  if (!d || !cfg) return fail(LBM_E_INVAL, "null argument");
  const BulkConfig c{cfg->block, cfg->cells_per_thread, cfg->memory, cfg->remap};
  if (!bulk_supported(c)) return fail(LBM_E_INVAL, "unsupported stream-collide launch shape");
  d->bulk = c;
  return LBM_OK;
}

lbm_status lbm_timing_enable(lbm_domain d, int32_t every) {
  if (!d) return fail(LBM_E_INVAL, "null domain");
  if (every < 0) return fail(LBM_E_INVAL, "negative timing period");
  if (every && !d->ev[0][0])
    for (int k = 0; k < 64; ++k)
      for (int j = 0; j < 2; ++j) HIP_TRY(hipEventCreate(&d->ev[j][k]));
  HIP_TRY(hipStreamSynchronize(d->stream));
  if (d->aux) HIP_TRY(hipStreamSynchronize(d->aux));
  d->timing = every != 0;
  d->timing_every = every;
  d->timed = d->folded = 0;
  for (int k = 0; k < 3; ++k) {
    d->kind_ms[k] = 0.0;
    d->kind_launches[k] = d->kind_nodes[k] = d->kind_count[k] = 0;
  }
  return LBM_OK;
}

lbm_status lbm_timing_read(lbm_domain d, int32_t kernel, double* total_ms, int64_t* launches, int64_t* nodes,
                           int64_t* issued) {
  if (!d || !total_ms || !launches || !nodes) return fail(LBM_E_INVAL, "null argument");
  if (kernel < LBM_KERNEL_STREAM_COLLIDE || kernel > LBM_KERNEL_NEAR_BOX) return fail(LBM_E_INVAL, "unknown kernel");
  lbm_status s = fold_timing(d, 0);
  if (s != LBM_OK) return s;
  *total_ms = d->kind_ms[kernel];
  *launches = d->kind_launches[kernel];
  *nodes = d->kind_nodes[kernel];
  if (issued) *issued = d->kind_count[kernel];
  return LBM_OK;
}

}  // extern "C"
