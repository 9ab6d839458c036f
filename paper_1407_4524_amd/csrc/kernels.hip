// Host side of the kernel launches: argument checks, launch shapes and the
// dispatch of each launch to the Ops<lattice, storage, equilibrium>
// instantiation that holds its kernels (inst_*.hip), plus the steady-state
// kernel, which does not depend on the lattice.
#include <vector>

#include "kernels.hpp"
#include "reduce.hpp"
#include "rows.hpp"

#include <hip/hip_ext.h>

#include <algorithm>
#include <type_traits>

namespace lbm {

template <class F>
static void with_types(int lat, int st, int eq, F&& f) {
  auto by_eq = [&](auto Lt, auto St) {
    if (eq) f(Lt, St, std::integral_constant<int, 1>{});
    else f(Lt, St, std::integral_constant<int, 0>{});
  };
  auto by_st = [&](auto Lt) {
    if (st == 0) by_eq(Lt, StoreF64{});
    else if (st == 1) by_eq(Lt, StoreF32{});
    else by_eq(Lt, StoreF16{});
  };
  if (lat == 0) by_st(D2Q9{});
  else by_st(D3Q19{});
}

#define LBM_TYPES                        \
  using L = decltype(Lt);                \
  using S = decltype(St);                \
  constexpr int EQ = decltype(E)::value; \
  using O = Ops<L, S, EQ>;

BulkShape bulk_shape(const Geom& g, int span) {
  BulkShape b;
  b.nbx = (g.hi[0] - g.lo[0] + 1 + span - 1) / span;
  b.nrows = g.hi[1] - g.lo[1] + 1;
  b.nplanes = g.hi[2] - g.lo[2] + 1;
  b.nblocks = b.nbx * b.nrows * b.nplanes;
  return b;
}

// Default launch shape of the stream-collide kernel by footprint, from
// scans of the measured sweep time over every supported shape (block, nodes
// per thread, non-temporal loads / stores, XCD remap) on MI355X: while both
// population buffers fit the 256 MB MALL, plain accesses in hardware block
// order are best (channel 2000x800 FP32: 18.9 us); beyond it the
// non-temporal hint pays on the loads of the D3Q19 sweep (duct 256x128x128
// FP32: 119.7 -> 101.4 us), on the stores of the D2Q9 sweep (8192x8192 FP32:
// 884 us, against 1057 us with two nodes per thread and non-temporal
// loads), and on neither with 2-byte storage (FP16 duct: 58.3 us plain,
// 62.6 with non-temporal stores); the D2Q9 sweep in 2-byte storage takes
// two nodes per thread (8192x8192 FP16: 423 us against 519 us with one).
BulkConfig bulk_config(int lat, int st, size_t footprint) {
  if (footprint <= (size_t)192 << 20) return BulkConfig{256, 1, 0, 0};
  if (st == 2) return lat == 0 ? BulkConfig{128, 2, 0, 0} : BulkConfig{256, 1, 0, 0};
  if (lat == 0) return BulkConfig{256, 1, MEM_NT_STORE, 0};
  return BulkConfig{256, 1, MEM_NT_LOAD, 0};
}

bool bulk_supported(const BulkConfig& c) {
  const int v[3][2] = {{256, 1}, {256, 2}, {128, 2}};
  for (const auto& e : v)
    if (c.block == e[0] && c.cells_per_thread == e[1] && c.nontemporal >= 0 && c.nontemporal <= 3 &&
        (c.remap == 0 || c.remap == 1))
      return true;
  return false;
}

Sweep make_sweep(const int lo[3], const int hi[3], int span, const int* hole, int remap) {
  Sweep sw{};
  sw.x0 = lo[0];
  sw.y0 = lo[1];
  sw.z0 = lo[2];
  sw.xlast = hi[0];
  sw.ny = hi[1] - lo[1] + 1;
  sw.nbx = (hi[0] - lo[0] + span) / span;
  sw.ntiles = sw.nbx * sw.ny * (hi[2] - lo[2] + 1);
  sw.remap = remap;
  for (int k = 0; k < 6; ++k) sw.hole[k] = hole ? hole[k] : (k & 1 ? 0 : 1);
  sw.rho_in = nullptr;
  sw.rho_out = nullptr;
  sw.mask = nullptr;
  sw.unstable = nullptr;
  return sw;
}

hipError_t launch_stream_collide(int lat, int st, int eq, const void* A, void* B, const Geom& g, const Phys& ph,
                                 hipStream_t s, const BulkConfig& cfg, const Sweep& sw, hipEvent_t ev_start,
                                 hipEvent_t ev_stop) {
  if (sw.ntiles <= 0 || !bulk_supported(cfg)) return hipErrorInvalidValue;
  if (sw.x0 < g.lo[0] || sw.xlast > g.hi[0] || sw.y0 < g.lo[1] || sw.z0 < g.lo[2]) return hipErrorInvalidValue;
  if (sw.y0 + sw.ny - 1 > g.hi[1] || sw.z0 + sw.ntiles / (sw.nbx * sw.ny) - 1 > g.hi[2])
    return hipErrorInvalidValue;
  if (sw.nbx != (sw.xlast - sw.x0 + cfg.block * cfg.cells_per_thread) / (cfg.block * cfg.cells_per_thread))
    return hipErrorInvalidValue;
  if (ev_start != nullptr && ev_stop == nullptr) return hipErrorInvalidValue;
  with_types(lat, st, eq, [&](auto Lt, auto St, auto E) {
    LBM_TYPES
    O::stream_collide(cfg, A, B, g, ph, sw, s, ev_start, ev_stop);
  });
  return hipGetLastError();
}

hipError_t launch_init(int lat, int st, int eq, void* A, uint8_t* mask, const Geom& g, const Phys& ph,
                       const double* rho, const double* u, void* rho_out, hipStream_t s) {
  with_types(lat, st, eq, [&](auto Lt, auto St, auto E) {
    LBM_TYPES
    O::init(A, mask, g, ph, rho, u, rho_out, s);
  });
  return hipGetLastError();
}

hipError_t launch_links(int lat, int st, int eq, void* A, const Link* links, int n_host, const int* n_dev,
                        int grid, const double* pose, int bc, const uint8_t* mask, const Geom& g, const Phys& ph,
                        double* partials, unsigned* counter, double* rec, hipStream_t s, hipEvent_t e0,
                        hipEvent_t e1) {
  with_types(lat, st, eq, [&](auto Lt, auto St, auto E) {
    LBM_TYPES
    O::links(A, links, n_host, n_dev, grid, pose, bc, mask, g, ph, partials, counter, rec, s, e0, e1);
  });
  return hipGetLastError();
}

hipError_t launch_links_part(int lat, int st, int eq, void* A, const Link* links, int n, const double* pose, int bc,
                             const uint8_t* mask, const Geom& g, const Phys& ph, double* part, hipStream_t s,
                             hipEvent_t e0, hipEvent_t e1) {
  if (n < 0) return hipErrorInvalidValue;
  with_types(lat, st, eq, [&](auto Lt, auto St, auto E) {
    LBM_TYPES
    O::links_part(A, links, n, pose, bc, mask, g, ph, part, s, e0, e1);
  });
  return hipGetLastError();
}

// The records of steps t0 .. t0 + gridDim.x - 1 from their chunk sums in the
// ring (nchunks chunks of 12 per step, ring_steps steps): lane l adds chunks
// l, l + 64, ... in order, then the lanes are summed by the fixed shuffle
// tree -- the order of the single-launch link kernel's final sum, so the
// records are the same bits. Static and comoving sums go to record entries
// 0..5 and 12..17; with zero_nodes the node terms and counts (6..11, 18, 19)
// are zeroed (a body whose solid set does not move has none).
__global__ __launch_bounds__(64) void k_fold(const double* __restrict__ ring, int nchunks, int ring_steps, int64_t t0,
                                             double* rec, int64_t rec_cap, int64_t rec_stride, int zero_nodes) {
  const int64_t t = t0 + blockIdx.x;
  const int lane = threadIdx.x;
  const double* part = ring + (t % ring_steps) * (int64_t)nchunks * 12;
  double* r = rec + (t % rec_cap) * rec_stride;
  double acc[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int c = lane; c < nchunks; c += 64)
#pragma unroll
    for (int j = 0; j < 12; ++j) acc[j] += part[c * 12 + j];
#pragma unroll
  for (int j = 0; j < 12; ++j) {
    const double v = wave_sum(acc[j]);
    if (lane == j) r[j < 6 ? j : j + 6] = v;
  }
  if (zero_nodes) {
    if (lane >= 12 && lane < 18) r[lane - 6] = 0.0;
    if (lane >= 18 && lane < 20) r[lane] = 0.0;
  }
}

// records of 18 doubles (walls, inlet, outlet) of steps t0 .. from the face
// ring, in the fixed order of k_fold
__global__ __launch_bounds__(64) void k_fold_faces(const double* __restrict__ ring, int nchunks, int ring_steps,
                                                   int64_t t0, double* rec, int64_t rec_cap) {
  const int64_t t = t0 + blockIdx.x;
  const int lane = threadIdx.x;
  const double* part = ring + (t % ring_steps) * (int64_t)nchunks * 18;
  double* r = rec + (t % rec_cap) * 18;
  double acc[18];
#pragma unroll
  for (int j = 0; j < 18; ++j) acc[j] = 0.0;
  for (int c = lane; c < nchunks; c += 64)
#pragma unroll
    for (int j = 0; j < 18; ++j) acc[j] += part[c * 18 + j];
#pragma unroll
  for (int j = 0; j < 18; ++j) {
    const double v = wave_sum(acc[j]);
    if (lane == j) r[j] = v;
  }
}

int face_nodes(const Geom& g) {
  const int64_t n[3] = {g.hi[0] - g.lo[0] + 1, g.hi[1] - g.lo[1] + 1, g.hi[2] - g.lo[2] + 1};
  return (int)(2 * (n[1] * n[2] + n[0] * n[2] + (g.D == 3 ? n[0] * n[1] : 0)));
}

hipError_t launch_face_part(int lat, int st, int eq, const void* A, const Geom& g, const Phys& ph, const void* rho_in,
                            double* part, hipStream_t s) {
  const int n = face_nodes(g);
  if (n <= 0) return hipErrorInvalidValue;
  with_types(lat, st, eq, [&](auto Lt, auto St, auto E) {
    LBM_TYPES
    O::face_part(A, g, ph, rho_in, n, part, s);
  });
  return hipGetLastError();
}

hipError_t launch_fold_faces(const double* ring, int nchunks, int ring_steps, int64_t t0, int64_t nsteps, double* rec,
                             int64_t rec_cap, hipStream_t s) {
  if (nsteps <= 0 || nsteps > ring_steps || nchunks <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_fold_faces, dim3((unsigned)nsteps), dim3(64), 0, s, ring, nchunks, ring_steps, t0, rec, rec_cap);
  return hipGetLastError();
}

hipError_t launch_poison_body(int lat, int st, int eq, void* A, void* B, const uint8_t* mask, const Geom& g,
                              const int lo[3], const int hi[3], int body, hipStream_t s) {
  with_types(lat, st, eq, [&](auto Lt, auto St, auto E) {
    LBM_TYPES
    O::poison_body(A, B, mask, g, lo, hi, body, s);
  });
  return hipGetLastError();
}

hipError_t launch_fold(const double* ring, int nchunks, int ring_steps, int64_t t0, int64_t nsteps, double* rec,
                       int64_t rec_cap, int64_t rec_stride, bool zero_nodes, hipStream_t s) {
  if (nsteps <= 0 || nsteps > ring_steps || nchunks <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_fold, dim3((unsigned)nsteps), dim3(64), 0, s, ring, nchunks, ring_steps, t0, rec, rec_cap,
                     rec_stride, zero_nodes ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_body_advance(int lat, int st, int eq, void* B, uint8_t* mask, uint8_t* mask_next, Link* links,
                               int* n_links, int cap, const double* pose, const double* pose_host, const BodyShape& bs,
                               int bc, int body, int mode, const Geom& g, const Phys& ph, double* rec_t, double* rec_t1,
                               int* err, hipStream_t s, int64_t region_cells, int64_t region_rows, int64_t list_nodes,
                               double* wide, int wide_slabs, hipEvent_t e0, hipEvent_t e1) {
  if (wide && wide_slabs <= 0) return hipErrorInvalidValue;
  with_types(lat, st, eq, [&](auto Lt, auto St, auto E) {
    LBM_TYPES
    O::body_advance(B, mask, mask_next, links, n_links, cap, pose, pose_host, bs, bc, body, mode, g, ph, rec_t,
                    rec_t1, err, s, region_cells, region_rows, list_nodes, wide, wide_slabs, e0, e1);
  });
  return hipGetLastError();
}

__global__ __launch_bounds__(64) void k_body_integrate(const double* __restrict__ rec_t,
                                                       const double* __restrict__ rec_tm1,
                                                       const double* __restrict__ pred, double* pose, double* traj,
                                                       double* dyn, FreeBody fb, int* err) {
#pragma clang fp contract(off)
  if (threadIdx.x != 0) return;
  const Pose P = reinterpret_cast<const Pose*>(pose)[0];
  double F[3], Tz;
  if (fb.drive == 2) {  // comoving frame
    for (int a = 0; a < 3; ++a) F[a] = rec_t[12 + a];
    Tz = rec_t[17];
  } else {  // static terms, plus the node terms of the step before (lattice frame)
    for (int a = 0; a < 3; ++a) F[a] = rec_t[a];
    Tz = rec_t[5];
    if ((fb.drive == 1 || fb.drive == 3) && fb.predicted) {  // node terms of the predicted pose
      for (int a = 0; a < 3; ++a) F[a] += pred[a];
      Tz += pred[5];
    } else if ((fb.drive == 1 || fb.drive == 3) && rec_tm1) {
      for (int a = 0; a < 3; ++a) F[a] += rec_tm1[6 + a];
      Tz += rec_tm1[11];
    }
  }
  double acc[4];
  for (int a = 0; a < 3; ++a) acc[a] = (F[a] + fb.ext_force[a]) / fb.mass;
  acc[3] = (Tz + fb.ext_torque) / fb.inertia;
  if (fb.D == 2) acc[2] = 0.0;
  const bool ab2 = fb.integrator == 1 && dyn[4] != 0.0;
  double dv[4];
  for (int a = 0; a < 4; ++a) dv[a] = ab2 ? 1.5 * acc[a] - 0.5 * dyn[a] : acc[a];
  Pose Q = P;
  for (int a = 0; a < 3; ++a) {
    Q.V[a] = P.V[a] + dv[a];
    Q.X[a] = P.X[a] + Q.V[a];
  }
  Q.Om = P.Om + dv[3];
  Q.theta = P.theta + Q.Om;
  free_trig(Q.theta, Q.ct, Q.st);
  pose_box(fb.shape, fb.axes, fb.D, fb.glo, fb.ghi, Q);
  bool ok = Q.V[0] * Q.V[0] + Q.V[1] * Q.V[1] + Q.V[2] * Q.V[2] < 0.25;
  for (int a = 0; a < fb.D; ++a) ok = ok && Q.lo[a] >= fb.glo[a] && Q.hi[a] <= fb.ghi[a];
  if (!ok) {  // the body stops where it is; the error is sticky
    atomicOr(err, 8);
    Q = P;
    for (int a = 0; a < 3; ++a) Q.V[a] = 0.0;
    Q.Om = 0.0;
  }
  reinterpret_cast<Pose*>(pose)[1] = Q;
  for (int a = 0; a < 3; ++a) traj[a] = Q.X[a];
  traj[3] = Q.theta;
  for (int a = 0; a < 3; ++a) traj[4 + a] = Q.V[a];
  traj[7] = Q.Om;
  for (int a = 0; a < 4; ++a) dyn[a] = acc[a];
  dyn[4] = 1.0;
}

hipError_t launch_body_integrate(const double* rec_t, const double* rec_tm1, const double* pred, double* pose,
                                 double* traj, double* dyn, const FreeBody& fb, int* err, hipStream_t s) {
  if (fb.predicted && !pred) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_body_integrate, dim3(1), dim3(64), 0, s, rec_t, rec_tm1, pred, pose, traj, dyn, fb, err);
  return hipGetLastError();
}

hipError_t launch_body_predict(int lat, int st, int eq, const void* B, const uint8_t* mask, const double* pose,
                               const BodyShape& bs, int body, const Geom& g, const Phys& ph, double* out,
                               hipStream_t s) {
  if (bs.shape == SHAPE_OUTER_CIRCLE) return hipErrorInvalidValue;
  with_types(lat, st, eq, [&](auto Lt, auto St, auto E) {
    LBM_TYPES
    O::body_predict(B, mask, pose, bs, body, g, ph, out, s);
  });
  return hipGetLastError();
}

// steady-state check: relative change of the drag (x-force of the body's
// momentum-exchange form) between steps t - 1 - window and t - 1, in FP64
// from the record rings, one thread per check

__global__ __launch_bounds__(64) void k_steady(const SteadyCheck* __restrict__ checks, int n, double* out) {
  const int k = blockIdx.x * 64 + threadIdx.x;
  if (k >= n) return;
  const SteadyCheck c = checks[k];
  const double* r1 = c.rec + ((c.t - 1) % c.rec_cap) * c.rec_stride;
  const double* r0 = c.rec + ((c.t - 1 - c.window) % c.rec_cap) * c.rec_stride;
  double f1, f0;
  if (c.me_mode == 0) {
    f1 = r1[0];
    f0 = r0[0];
  } else if (c.me_mode == 1) {
    f1 = r1[0] + r1[6];
    f0 = r0[0] + r0[6];
  } else {
    f1 = r1[12];
    f0 = r0[12];
  }
  const double rel = fabs(f1 - f0) / fabs(f1);
  out[2 * k] = rel;
  out[2 * k + 1] = f1;
}

hipError_t launch_steady(const SteadyCheck* checks, int n, double* out, hipStream_t s) {
  if (n <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_steady, dim3((n + 63) / 64), dim3(64), 0, s, checks, n, out);
  return hipGetLastError();
}

bool body_step_fits(int64_t region_cells, int64_t region_rows, int64_t list_nodes) {
  return region_cells > 0 && region_cells <= STEP_CELLS && region_rows <= STEP_ROWS && list_nodes <= STEP_LIST;
}

int64_t step_list_nodes(const BodyShape& bs, const Pose& P0, const Pose& P1, int D) {
  int lo[3], n[3];
  for (int a = 0; a < 3; ++a) {
    const int l = (int)(P0.lo[a] < P1.lo[a] ? P0.lo[a] : P1.lo[a]);
    const int h = (int)(P0.hi[a] > P1.hi[a] ? P0.hi[a] : P1.hi[a]);
    lo[a] = l;
    n[a] = h - l + 1;
  }
  // the chord of every row of the region and the rows around it, at both
  // poses, once; each row's windows then combine those of its neighbour rows
  // exactly as row_windows does (min / max are exact, so the windows are the
  // same)
  const int my = n[1] + 2, mz = D == 3 ? n[2] + 2 : 1, dz0 = D == 3 ? 1 : 0;
  struct Chord {
    double a, b;
    bool hit;
  };
  thread_local std::vector<Chord> ch;
  ch.resize((size_t)2 * my * mz);
  for (int k = 0; k < 2; ++k)
    for (int zz = 0; zz < mz; ++zz)
      for (int yy = 0; yy < my; ++yy) {
        Chord& c = ch[((size_t)k * mz + zz) * my + yy];
        c.a = c.b = 0.0;
        c.hit = row_chord(bs, k ? P1 : P0, lo[1] - 1 + yy, lo[2] - dz0 + zz, c.a, c.b);
      }
  int64_t total = 0;
  for (int r = 0; r < n[1] * n[2]; ++r) {
    const int yy = 1 + r % n[1], zz = dz0 + r / n[1];
    RowExtent e;
    for (int dz = -dz0; dz <= dz0; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int k = 0; k < 2; ++k) {
          const Chord& c = ch[((size_t)k * mz + zz + dz) * my + yy + dy];
          e.add(c.hit, c.a, c.b);
        }
    int w[4] = {0, -1, 0, -1};
    const int nw = windows_of(e, 2, lo[0], lo[0] + n[0] - 1, w);
    for (int q = 0; q < nw; ++q) total += w[2 * q + 1] - w[2 * q] + 1 + 2;  // + 2: rounding of the chord ends
  }
  return total;
}

bool batch_bulk_supported(int block, int cells_per_thread) {
  for (const auto& v : BATCH_BULK_VARIANTS)
    if (v[0] == block && v[1] == cells_per_thread) return true;
  return false;
}

hipError_t launch_batch_bulk(int lat, int st, int eq, const BatchDomain* doms, const BatchTile* tiles, int ntiles,
                             const BulkConfig& cfg, int64_t step, hipStream_t s, int part, hipEvent_t ev_start,
                             hipEvent_t ev_stop, const int64_t* sbase, int flat) {
  if (ntiles <= 0 || !batch_bulk_supported(cfg.block, cfg.cells_per_thread) || part < 0 || part > 2 ||
      (flat && (part == 2 || cfg.cells_per_thread != 1)))
    return hipErrorInvalidValue;
  if (ev_start != nullptr && ev_stop == nullptr) return hipErrorInvalidValue;
  with_types(lat, st, eq, [&](auto Lt, auto St, auto E) {
    LBM_TYPES
    O::batch_bulk(doms, tiles, ntiles, cfg, step, s, part, ev_start, ev_stop, sbase, flat);
  });
  return hipGetLastError();
}

int batch_link_grid(int lat, int max_links) {
  if (lat == 0) return 1;  // 2D: one 1024-thread workgroup per body
  return std::max(1, (max_links + 63) / 64);  // 3D: one wavefront per chunk of 64 links
}

hipError_t launch_batch_links(int lat, int st, int eq, const BatchDomain* doms, const BatchBody* bodies, int nbodies,
                              int grid, int64_t step, hipStream_t s, const int64_t* sbase) {
  if (nbodies <= 0 || grid <= 0 || (lat == 0 && grid != 1)) return hipErrorInvalidValue;
  with_types(lat, st, eq, [&](auto Lt, auto St, auto E) {
    LBM_TYPES
    O::batch_links(doms, bodies, nbodies, grid, step, s, sbase);
  });
  return hipGetLastError();
}

hipError_t launch_batch_body_links(int lat, int st, int eq, const BatchDomain* doms, const BatchBody* moving,
                                   int n_moving, const BatchBody* fixed, int n_fixed, int64_t max_region_cells,
                                   int64_t step, hipStream_t s, const int64_t* sbase) {
  if (lat != 0 || n_moving < 0 || n_fixed < 0 || n_moving + n_fixed <= 0) return hipErrorInvalidValue;
  if (n_moving > 0 && (max_region_cells <= 0 || max_region_cells > STEP_CELLS)) return hipErrorInvalidValue;
  const size_t lds = n_moving > 0 ? ((size_t)2 * max_region_cells + 15) / 16 * 16 : 0;
  with_types(lat, st, eq, [&](auto Lt, auto St, auto E) {
    LBM_TYPES
    O::batch_body_links(doms, moving, n_moving, fixed, n_fixed, lds, step, s, sbase);
  });
  return hipGetLastError();
}

hipError_t launch_batch_body_step(int lat, int st, int eq, const BatchDomain* doms, const BatchBody* bodies,
                                  int nbodies, int64_t max_region_cells, int64_t step, hipStream_t s,
                                  const int64_t* sbase) {
  if (nbodies <= 0 || max_region_cells <= 0 || max_region_cells > STEP_CELLS) return hipErrorInvalidValue;
  const size_t lds = ((size_t)2 * max_region_cells + 15) / 16 * 16;
  with_types(lat, st, eq, [&](auto Lt, auto St, auto E) {
    LBM_TYPES
    O::batch_body_step(doms, bodies, nbodies, lds, step, s, sbase);
  });
  return hipGetLastError();
}

hipError_t launch_batch_wide(int lat, int st, int eq, const BatchDomain* doms, const BatchBody* bodies, int nbodies,
                             int max_slabs, int64_t step, hipStream_t s, const int64_t* sbase) {
  if (nbodies <= 0 || max_slabs <= 0) return hipErrorInvalidValue;
  with_types(lat, st, eq, [&](auto Lt, auto St, auto E) {
    LBM_TYPES
    O::batch_wide(doms, bodies, nbodies, max_slabs, step, s, sbase);
  });
  return hipGetLastError();
}

__global__ void k_add_step(int64_t* counter, int64_t k) {
  if (threadIdx.x == 0) *counter += k;
}

hipError_t launch_add_step(int64_t* counter, int64_t k, hipStream_t s) {
  hipLaunchKernelGGL(k_add_step, dim3(1), dim3(64), 0, s, counter, k);
  return hipGetLastError();
}

__global__ void k_set_step(int64_t* counter, int64_t v) {
  if (threadIdx.x == 0) *counter = v;
}

hipError_t launch_set_step(int64_t* counter, int64_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_step, dim3(1), dim3(64), 0, s, counter, v);
  return hipGetLastError();
}

}  // namespace lbm
