// Batches of domains (include/lbm.h, lbm_batch_*): the member tables the
// batched kernels read, the per-step launch sequence and the autotuner of
// the batched stream-collide launch shape.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "domain.hpp"

using namespace lbm;
using namespace lbm::host;

struct lbm_batch_s {
  hipStream_t stream = nullptr;
  std::vector<lbm_domain> members;
  lbm_batch_config cfg{256, 1, 1, 0, 1, 0, 0.0};
  // second stream of the overlapped step; created on first use
  hipStream_t aux = nullptr;
  hipEvent_t e_near = nullptr, e_far = nullptr;
  // device tables and their pinned staging copy, grown as needed
  char* dev = nullptr;
  size_t dev_cap = 0;
  char* pinned = nullptr;
  size_t pinned_cap = 0;
  // steady-state checks of the members: device checks + results
  char* steady_dev = nullptr;
  size_t steady_cap = 0;
  // graph mode: the device step counter the captured kernels add to their
  // step, and the last executable graph (destroyed at the next call or with
  // the batch, after the stream has drained it)
  int64_t* step_dev = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  hipStream_t cap = nullptr;  // the stream sequences are captured on (the batch's may be the null stream)
};

namespace {

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

bool config_ok(const lbm_batch_config& c) {
  return batch_bulk_supported(c.block, c.cells_per_thread) && (c.remap == 0 || c.remap == 1) && c.order >= 0 &&
         c.order <= 3 && (c.order < 3 || c.cells_per_thread == 1) && (c.overlap == 0 || c.overlap == 1) &&
         (c.graph == 0 || c.graph == 1);
}

// steps per captured sequence of a graph-mode call (even: the buffer parity
// of every replay is the same)
constexpr int64_t GRAPH_STEPS = 32;

int64_t active_nodes(const Geom& g) {
  return (int64_t)(g.hi[0] - g.lo[0] + 1) * (g.hi[1] - g.lo[1] + 1) * (g.hi[2] - g.lo[2] + 1);
}

// row tiles of every member in the configured order
std::vector<BatchTile> make_tiles(const std::vector<lbm_domain>& m, const lbm_batch_config& c) {
  const int span = c.block * c.cells_per_thread;
  std::vector<int> order(m.size());
  std::iota(order.begin(), order.end(), 0);
  if (c.order == 1)
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return active_nodes(m[a]->g) > active_nodes(m[b]->g); });
  auto nbx = [&](int i) { return (m[i]->g.hi[0] - m[i]->g.lo[0] + span) / span; };
  auto nrows = [&](int i) {
    const Geom& g = m[i]->g;
    return (g.hi[1] - g.lo[1] + 1) * (g.hi[2] - g.lo[2] + 1);
  };
  std::vector<BatchTile> tiles;
  if (c.order == 3) {  // spans of `span` consecutive active nodes across rows, largest members first
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return active_nodes(m[a]->g) > active_nodes(m[b]->g); });
    for (int i : order) {
      const int64_t n = active_nodes(m[i]->g);
      for (int64_t f = 0; f < n; f += span) tiles.push_back(BatchTile{(uint16_t)i, 0, (int32_t)f});
    }
  } else if (c.order == 2) {
    int maxrows = 0;
    for (size_t i = 0; i < m.size(); ++i) maxrows = std::max(maxrows, nrows((int)i));
    for (int r = 0; r < maxrows; ++r)
      for (int i : order)
        if (r < nrows(i))
          for (int bx = 0; bx < nbx(i); ++bx) tiles.push_back(BatchTile{(uint16_t)i, (uint16_t)bx, r});
  } else {
    for (int i : order)
      for (int r = 0; r < nrows(i); ++r)
        for (int bx = 0; bx < nbx(i); ++bx) tiles.push_back(BatchTile{(uint16_t)i, (uint16_t)bx, r});
  }
  return tiles;
}

struct Plan {
  std::vector<BatchDomain> doms;
  std::vector<BatchTile> tiles, near_tiles;
  std::vector<BatchBody> links, moving;
  std::vector<BatchBody> wide;                // advanced by the many-workgroup kernels
  std::vector<std::pair<int, int>> fallback;  // (member, body) advanced by its own launches
  int link_grid = 1, max_links = 0, wide_slabs = 0;
  int64_t max_cells = 0;
  size_t off_tiles = 0, off_near = 0, off_links = 0, off_moving = 0, off_wide = 0, bytes = 0;
};

// Near box of a member for the steps t0 .. t0+n-1 of a call: the node boxes
// of every pose its bodies take (t0-1 .. t0+n for a body whose solid set
// moves, t0 for the others) plus one layer (two for a body with fixed links,
// whose link rule of the next step reads nodes two away from its box), within
// the active nodes; empty for a member without bodies. Every node the body
// work of the call reads or writes lies inside it, one layer away from the
// far update.
void near_box_of(lbm_domain d, int64_t n, int hole[6]) {
  const Geom& g = d->g;
  int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
  bool any = false;
  for (const Body& b : d->body) {
    if (!b.active) continue;
    const Pose* P = reinterpret_cast<const Pose*>(b.pose_pinned);
    const int64_t k0 = (b.mask_moves && d->t - 1 >= b.pose_base) ? d->t - 1 : d->t;
    const int64_t k1 = b.mask_moves ? d->t + n : d->t;
    const int m = b.mask_moves ? 1 : 2;
    for (int64_t k = k0; k <= k1; ++k)
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], (int)P[k - b.pose_base].lo[a] - m);
        hi[a] = std::max(hi[a], (int)P[k - b.pose_base].hi[a] + m);
      }
    any = true;
  }
  if (!any) {
    const int none[6] = {1, 0, 1, 0, 1, 0};
    for (int k = 0; k < 6; ++k) hole[k] = none[k];
    return;
  }
  for (int a = 0; a < 3; ++a) {
    hole[2 * a] = std::max<int>(g.lo[a], lo[a]);
    hole[2 * a + 1] = std::min<int>(g.hi[a], hi[a]);
  }
}

BatchBody batch_body(lbm_domain d, int member, int id) {
  Body& b = d->body[id];
  BatchBody bb{};
  bb.dom = member;
  bb.body = id;
  bb.bc = b.desc.bc;
  bb.cap = b.cap;
  bb.n_host = b.n_host;
  bb.links = b.links;
  bb.n_links = b.n_links;
  bb.pose = b.pose_dev;
  bb.pose_base = b.pose_base;
  bb.bs = b.shape;
  bb.mask = d->mask;
  bb.rec = d->rec + id * LBM_REC_LEN;
  bb.rec_cap = d->rec_cap;
  bb.rec_stride = (int64_t)d->nslots * LBM_REC_LEN;
  bb.partials = b.partials;
  bb.counter = d->counters + id;
  bb.err = d->err;
  bb.t0 = d->t;
  return bb;
}

// Poses for the next n steps, the first link rule of moving bodies that have
// not had one, and the tables of this call.
lbm_status make_plan(lbm_batch B, int64_t n, Plan& P) {
  const auto& m = B->members;
  for (lbm_domain d : m)
    for (int id = 0; id < d->nslots; ++id) {
      Body& b = d->body[id];
      if (!b.active) continue;
      lbm_status s = ensure_poses(d, b, d->t, d->t + n);
      if (s != LBM_OK) return s;
      if (b.mask_moves && !b.bc_ready) {
        const int grid = std::max(1, std::min(LINK_GRID_MAX, (b.n_host + 255) / 256));
        HIP_TRY(launch_links(d->lat, d->st, d->eq, d->A, b.links, b.n_host, b.n_links, grid, pose_at(b, d->t),
                             b.desc.bc, d->mask, d->g, d->ph, b.partials, d->counters + id, rec_slot(d, d->t, id),
                             B->stream));
        b.bc_ready = true;
      }
    }
  const int span = B->cfg.block * B->cfg.cells_per_thread;
  for (size_t i = 0; i < m.size(); ++i) {
    lbm_domain d = m[i];
    BatchDomain bd{d->g, d->ph, {d->A, d->B}, {d->rhoA, d->rhoB}, d->mask, d->err + 1, {1, 0, 1, 0, 1, 0}};
    if (B->cfg.overlap) {
      near_box_of(d, n, bd.hole);
      if (bd.hole[0] <= bd.hole[1]) {
        const int nbx = (bd.hole[1] - bd.hole[0] + span) / span;
        const int rows = (bd.hole[3] - bd.hole[2] + 1) * (bd.hole[5] - bd.hole[4] + 1);
        for (int r = 0; r < rows; ++r)
          for (int bx = 0; bx < nbx; ++bx) P.near_tiles.push_back(BatchTile{(uint16_t)i, (uint16_t)bx, r});
      }
    }
    P.doms.push_back(bd);
    for (int id = 0; id < d->nslots; ++id) {
      Body& b = d->body[id];
      if (!b.active) continue;
      BatchBody bb = batch_body(d, (int)i, id);
      if (!b.mask_moves) {
        P.links.push_back(bb);
        P.max_links = std::max(P.max_links, b.n_host);
        continue;
      }
      // every step of the call takes the same kernel (batch_step splits a
      // call where a body changes kernels)
      if (step_fits(b, d->D, d->t)) {
        int64_t cells = 0;
        for (int64_t k = 0; k < n; ++k) cells = std::max(cells, region_cells(b, d->D, d->t + k, 1));
        P.moving.push_back(bb);
        P.max_cells = std::max(P.max_cells, cells);
      } else if (b.wide) {
        int64_t rows = 0;
        for (int64_t k = 0; k < n; ++k) rows = std::max(rows, region_rows(b, d->t + k, 1));
        lbm_status s = ensure_wide(b, (int)((rows + WIDE_ROWS - 1) / WIDE_ROWS), B->stream);
        if (s != LBM_OK) return s;
        bb.wide = b.wide;
        bb.wide_slabs = b.wide_slabs;
        P.wide.push_back(bb);
        P.wide_slabs = std::max(P.wide_slabs, b.wide_slabs);
      } else {
        P.fallback.push_back({(int)i, id});
      }
    }
  }
  P.link_grid = batch_link_grid(m.empty() ? 0 : m[0]->lat, P.max_links);
  P.tiles = make_tiles(m, B->cfg);
  P.off_tiles = align256(P.doms.size() * sizeof(BatchDomain));
  P.off_near = P.off_tiles + align256(P.tiles.size() * sizeof(BatchTile));
  P.off_links = P.off_near + align256(P.near_tiles.size() * sizeof(BatchTile));
  P.off_moving = P.off_links + align256(P.links.size() * sizeof(BatchBody));
  P.off_wide = P.off_moving + align256(P.moving.size() * sizeof(BatchBody));
  P.bytes = P.off_wide + align256(P.wide.size() * sizeof(BatchBody));
  return LBM_OK;
}

// copies the tables to the device (after the previous copy has been used)
lbm_status upload(lbm_batch B, const Plan& P) {
  HIP_TRY(hipStreamSynchronize(B->stream));
  if (P.bytes > B->dev_cap) {
    if (B->dev) HIP_TRY(hipFree(B->dev));
    if (B->pinned) HIP_TRY(hipHostFree(B->pinned));
    B->dev = nullptr;
    B->pinned = nullptr;
    const size_t cap = P.bytes * 2;
    HIP_TRY(hipMalloc(&B->dev, cap));
    HIP_TRY(hipHostMalloc(&B->pinned, cap, hipHostMallocDefault));
    B->dev_cap = B->pinned_cap = cap;
  }
  memcpy(B->pinned, P.doms.data(), P.doms.size() * sizeof(BatchDomain));
  memcpy(B->pinned + P.off_tiles, P.tiles.data(), P.tiles.size() * sizeof(BatchTile));
  memcpy(B->pinned + P.off_near, P.near_tiles.data(), P.near_tiles.size() * sizeof(BatchTile));
  memcpy(B->pinned + P.off_links, P.links.data(), P.links.size() * sizeof(BatchBody));
  memcpy(B->pinned + P.off_moving, P.moving.data(), P.moving.size() * sizeof(BatchBody));
  memcpy(B->pinned + P.off_wide, P.wide.data(), P.wide.size() * sizeof(BatchBody));
  HIP_TRY(hipMemcpyAsync(B->dev, B->pinned, P.bytes, hipMemcpyHostToDevice, B->stream));
  return LBM_OK;
}

// n steps of every member; e0 (optional) is recorded once the tables are on
// their way and e1 after the last launch
// Enqueues batch steps k0 .. k1-1 of a call on stream `main` (the batch's
// stream, or the stream a sequence is captured on) and the batch's second
// stream when split: the step index k goes to the kernels, plus *sbase when
// given (captured sequences). `capture`: completion events are recorded by
// separate calls, not by the launches.
static lbm_status enqueue_steps(lbm_batch B, const Plan& P, int64_t k0, int64_t k1, const int64_t* sbase, bool split,
                                bool capture, hipStream_t main) {
  const lbm_domain first = B->members[0];
  const auto* doms = reinterpret_cast<const BatchDomain*>(B->dev);
  const auto* tiles = reinterpret_cast<const BatchTile*>(B->dev + P.off_tiles);
  const auto* near_tiles = reinterpret_cast<const BatchTile*>(B->dev + P.off_near);
  const auto* links = reinterpret_cast<const BatchBody*>(B->dev + P.off_links);
  const auto* moving = reinterpret_cast<const BatchBody*>(B->dev + P.off_moving);
  const auto* wide = reinterpret_cast<const BatchBody*>(B->dev + P.off_wide);
  // buffer resources while every member's population buffer is below 4 GiB
  size_t largest = 0;
  for (lbm_domain d : B->members) largest = std::max(largest, (size_t)d->Q * d->g.S * d->elem);
  const int buf = largest < ((size_t)1 << 32) ? 1 : 0;
  const BulkConfig bc{B->cfg.block, B->cfg.cells_per_thread, 0, B->cfg.remap, buf};
  const BulkConfig nc{B->cfg.block, B->cfg.cells_per_thread, 0, 0, buf};
  const int flat = B->cfg.order == 3 ? 1 : 0;  // tiles of P.tiles are spans across rows
  // a domain that lbm_step advances through a one-member batch of its own
  // keeps its kernel timing: the update of every node but the near box (or
  // of every node) is its stream-collide launch
  const lbm_domain solo = B->members.size() == 1 && B->members[0]->solo == B ? B->members[0] : nullptr;
  int64_t timed_nodes = 0;
  if (solo) {
    const int* h = P.doms[0].hole;
    timed_nodes = active_nodes(solo->g);
    if (split && h[0] <= h[1])
      timed_nodes -= (int64_t)(h[1] - h[0] + 1) * (h[3] - h[2] + 1) * (h[5] - h[4] + 1);
  }
  const int lat = first->lat, st = first->st, eq = first->eq;
  // 2D: the link rule of the bodies with fixed links for step k+1 joins the
  // advance launch of step k (at the first step of a sequence it runs on its
  // own; at its last, not at all: the next sequence starts with it)
  const bool fuse = lat == 0 && !P.links.empty();
  for (int64_t k = k0; k < k1; ++k) {
    if (split) {
      if (k > k0) HIP_TRY(hipStreamWaitEvent(main, B->e_far, 0));
      else HIP_TRY(hipEventRecord(B->e_near, main));
      HIP_TRY(hipStreamWaitEvent(B->aux, B->e_near, 0));
      hipEvent_t t0 = nullptr, t1 = nullptr;
      if (solo && !capture) {
        lbm_status ts = timing_slot(solo, LBM_KERNEL_STREAM_COLLIDE, timed_nodes, t0, t1);
        if (ts != LBM_OK) return ts;
      }
      HIP_TRY(launch_batch_bulk(lat, st, eq, doms, tiles, (int)P.tiles.size(), bc, k, B->aux, 1, t0,
                                t1 ? t1 : (capture ? nullptr : B->e_far), sbase, flat));
      if (capture || t1) HIP_TRY(hipEventRecord(B->e_far, B->aux));
    }
    if (!P.links.empty() && (!fuse || k == k0))
      HIP_TRY(launch_batch_links(lat, st, eq, doms, links, (int)P.links.size(), P.link_grid, k, main, sbase));
    if (split) {
      HIP_TRY(launch_batch_bulk(lat, st, eq, doms, near_tiles, (int)P.near_tiles.size(), nc, k, main, 2, nullptr,
                                capture ? nullptr : B->e_near, sbase));
      if (capture) HIP_TRY(hipEventRecord(B->e_near, main));
    } else {
      hipEvent_t t0 = nullptr, t1 = nullptr;
      if (solo && !capture) {
        lbm_status ts = timing_slot(solo, LBM_KERNEL_STREAM_COLLIDE, timed_nodes, t0, t1);
        if (ts != LBM_OK) return ts;
      }
      HIP_TRY(launch_batch_bulk(lat, st, eq, doms, tiles, (int)P.tiles.size(), bc, k, main, 0, t0, t1, sbase, flat));
    }
    if (fuse && k + 1 < k1)
      HIP_TRY(launch_batch_body_links(lat, st, eq, doms, moving, (int)P.moving.size(), links, (int)P.links.size(),
                                      P.max_cells, k, main, sbase));
    else if (!P.moving.empty())
      HIP_TRY(launch_batch_body_step(lat, st, eq, doms, moving, (int)P.moving.size(), P.max_cells, k, main,
                                     sbase));
    if (!P.wide.empty())
      HIP_TRY(launch_batch_wide(lat, st, eq, doms, wide, (int)P.wide.size(), P.wide_slabs, k, main, sbase));
    for (const auto& f : P.fallback) {  // never in a captured sequence
      lbm_domain d = B->members[f.first];
      Body& b = d->body[f.second];
      const int64_t t = d->t + k;
      void* cur = (k & 1) ? d->A : d->B;  // the state of t+1
      HIP_TRY(launch_body_advance(d->lat, d->st, d->eq, cur, d->mask, d->mask_next, b.links, b.n_links, b.cap,
                                  pose_at(b, t), pose_host_at(b, t), b.shape, b.desc.bc, f.second, 1, d->g, d->ph,
                                  rec_slot(d, t, f.second),
                                  rec_slot(d, t + 1, f.second), d->err, main, region_cells(b, d->D, t, 1),
                                  region_rows(b, t, 1), list_bound(b, d->D, t)));
    }
  }
  if (split) HIP_TRY(hipStreamWaitEvent(main, B->e_far, 0));
  return LBM_OK;
}

// frees the last executable graph (its launches have completed: called
// after the stream was synchronised)
static void drop_graph(lbm_batch B) {
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  B->exec = nullptr;
  B->graph = nullptr;
}

// The longest run of the next n steps (at least one) over which every
// moving body keeps its advance kernel (the single-workgroup list kernel or
// the many-workgroup one), as lbm_step chooses them step by step.
static lbm_status uniform_steps(lbm_batch B, int64_t n, int64_t& run) {
  run = n;
  for (lbm_domain d : B->members)
    for (int id = 0; id < d->nslots; ++id) {
      Body& b = d->body[id];
      if (!b.active || !b.mask_moves) continue;
      lbm_status s = ensure_poses(d, b, d->t, d->t + n);
      if (s != LBM_OK) return s;
      const bool f0 = step_fits(b, d->D, d->t);
      for (int64_t k = 1; k < run; ++k)
        if (step_fits(b, d->D, d->t + k) != f0) {
          run = k;
          break;
        }
    }
  return LBM_OK;
}

static lbm_status batch_run(lbm_batch B, int64_t n, hipEvent_t e0, hipEvent_t e1);

lbm_status batch_step(lbm_batch B, int64_t n, hipEvent_t e0, hipEvent_t e1) {
  if (n <= 0 || B->members.empty()) return LBM_OK;
  for (int64_t done = 0; done < n;) {
    int64_t run = 0;
    lbm_status s = uniform_steps(B, n - done, run);
    if (s != LBM_OK) return s;
    s = batch_run(B, run, done == 0 ? e0 : nullptr, done + run == n ? e1 : nullptr);
    if (s != LBM_OK) return s;
    done += run;
  }
  return LBM_OK;
}

static lbm_status batch_run(lbm_batch B, int64_t n, hipEvent_t e0, hipEvent_t e1) {
  Plan P;
  lbm_status s = make_plan(B, n, P);  // synchronises the stream (table upload): the last graph is done
  if (s != LBM_OK) return s;
  s = upload(B, P);
  if (s != LBM_OK) return s;
  drop_graph(B);
  // Overlapped step (as the single-domain split of lbm_step): the far update
  // of step k, on the second stream, waits for the near update of step k-1;
  // the near update of step k waits for the far update of step k-1; the body
  // work of a member only touches nodes inside its near box, one layer away
  // from what the far update reads.
  const bool split = B->cfg.overlap && !P.near_tiles.empty();
  if (split && !B->aux) {
    lbm_status sa = create_far_stream(B->stream, &B->aux, 8);  // one CU in 8 for the body kernels
    if (sa != LBM_OK) return sa;
    HIP_TRY(hipEventCreateWithFlags(&B->e_near, hipEventDisableTiming | hipEventDisableSystemFence));
    HIP_TRY(hipEventCreateWithFlags(&B->e_far, hipEventDisableTiming | hipEventDisableSystemFence));
  }
  if (e0) HIP_TRY(hipEventRecord(e0, B->stream));
  // Graph mode: GRAPH_STEPS steps are captured once into a HIP graph whose
  // kernels take their step from a device counter (the last node adds
  // GRAPH_STEPS to it), and the graph is replayed; the steps left over run
  // as ordinary launches. The launches are the same as in ordinary mode, so
  // the results are the same bits. Bodies advanced by their own per-step
  // launches (too large for the batched kernels) keep ordinary mode.
  int64_t done = 0;
  if (B->cfg.graph && P.fallback.empty() && n >= 2 * GRAPH_STEPS) {
    if (!B->step_dev) HIP_TRY(hipMalloc(&B->step_dev, sizeof(int64_t)));
    if (!B->cap) HIP_TRY(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
    HIP_TRY(launch_set_step(B->step_dev, 0, B->stream));
    HIP_TRY(hipStreamBeginCapture(B->cap, hipStreamCaptureModeRelaxed));
    lbm_status sc = enqueue_steps(B, P, 0, GRAPH_STEPS, B->step_dev, split, true, B->cap);
    if (sc == LBM_OK) {
      hipError_t e = launch_add_step(B->step_dev, GRAPH_STEPS, B->cap);
      if (e != hipSuccess) sc = fail(LBM_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    }
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(B->cap, &graph);
    if (sc != LBM_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return sc;
    }
    if (ee != hipSuccess) return fail(LBM_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ee));
    B->graph = graph;
    HIP_TRY(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
    const int64_t reps = n / GRAPH_STEPS;
    for (int64_t r = 0; r < reps; ++r) HIP_TRY(hipGraphLaunch(B->exec, B->stream));
    done = reps * GRAPH_STEPS;
  }
  if (done < n) {
    s = enqueue_steps(B, P, done, n, nullptr, split, false, B->stream);
    if (s != LBM_OK) return s;
  }
  if (e1) HIP_TRY(hipEventRecord(e1, B->stream));
  for (lbm_domain d : B->members) {
    d->t += n;
    if (n & 1) {
      std::swap(d->A, d->B);
      std::swap(d->rhoA, d->rhoB);
    }
  }
  return LBM_OK;
}

}  // namespace

// A domain with several bodies steps them through batched launches (one for
// the link rule of every body with fixed links, one for the advance of every
// moving body) as the only member of a batch of its own, on its own stream.
lbm_status lbm::host::solo_step(lbm_domain d, int64_t n) {
  if (!d->solo) {
    d->solo = new lbm_batch_s();
    d->solo->members.push_back(d);
  }
  d->solo->stream = d->stream;
  return batch_step(d->solo, n, nullptr, nullptr);
}

void lbm::host::solo_destroy(lbm_domain d) {
  if (!d->solo) return;
  d->solo->members.clear();  // the domain's own stream and batch stay as they are
  (void)hipStreamSynchronize(d->stream);
  (void)lbm_batch_destroy(d->solo);
  d->solo = nullptr;
}

extern "C" {

lbm_status lbm_batch_create(void* stream, lbm_batch* out) {
  if (!out) return fail(LBM_E_INVAL, "null output");
  lbm_batch B = new lbm_batch_s();
  B->stream = (hipStream_t)stream;
  *out = B;
  return LBM_OK;
}

lbm_status lbm_batch_destroy(lbm_batch B) {
  if (!B) return fail(LBM_E_INVAL, "null batch");
  hipError_t e = hipStreamSynchronize(B->stream);
  for (lbm_domain d : B->members) {
    d->stream = d->own_stream;
    d->batch = nullptr;
  }
  if (B->aux) {
    (void)hipStreamSynchronize(B->aux);
    (void)hipStreamDestroy(B->aux);
    (void)hipEventDestroy(B->e_near);
    (void)hipEventDestroy(B->e_far);
  }
  drop_graph(B);
  if (B->dev) (void)hipFree(B->dev);
  if (B->pinned) (void)hipHostFree(B->pinned);
  if (B->steady_dev) (void)hipFree(B->steady_dev);
  if (B->step_dev) (void)hipFree(B->step_dev);
  if (B->cap) (void)hipStreamDestroy(B->cap);
  delete B;
  if (e != hipSuccess) return fail(LBM_E_HIP, hipGetErrorString(e));
  return LBM_OK;
}

lbm_status lbm_batch_add(lbm_batch B, lbm_domain d) {
  if (!B || !d) return fail(LBM_E_INVAL, "null argument");
  if (d->batch) return fail(LBM_E_STATE, "the domain already belongs to a batch");
  if (B->members.size() >= 65535) return fail(LBM_E_INVAL, "a batch holds at most 65535 domains");
  if (d->face_rec) return fail(LBM_E_INVAL, "a domain that records its faces is stepped alone, not in a batch");
  if (!B->members.empty()) {
    const lbm_domain f = B->members[0];
    if (f->lat != d->lat || f->st != d->st || f->eq != d->eq)
      return fail(LBM_E_INVAL, "batch members share lattice, storage and equilibrium");
  }
  const Geom& g = d->g;
  if ((g.hi[0] - g.lo[0]) / 64 + 1 > 65535) return fail(LBM_E_INVAL, "rows too long for a batch tile index");
  HIP_TRY(hipStreamSynchronize(d->stream));
  if (d->aux) HIP_TRY(hipStreamSynchronize(d->aux));
  d->stream = B->stream;
  d->batch = B;
  B->members.push_back(d);
  return LBM_OK;
}

lbm_status lbm_batch_remove(lbm_batch B, lbm_domain d) {
  if (!B || !d) return fail(LBM_E_INVAL, "null argument");
  auto it = std::find(B->members.begin(), B->members.end(), d);
  if (it == B->members.end()) return fail(LBM_E_INVAL, "the domain is not a member of this batch");
  HIP_TRY(hipStreamSynchronize(B->stream));
  B->members.erase(it);
  d->stream = d->own_stream;
  d->batch = nullptr;
  return LBM_OK;
}

lbm_status lbm_batch_step(lbm_batch B, int64_t nsteps) {
  if (!B) return fail(LBM_E_INVAL, "null batch");
  if (nsteps < 0) return fail(LBM_E_INVAL, "negative step count");
  return batch_step(B, nsteps, nullptr, nullptr);
}

// The steady-state checks of a batch's members (see lbm_batch_steady_state):
// the table of checks is built in `checks` (host, room for `cap`), uploaded
// to `dev` (device, room for the table and 2 doubles per check after
// align256 of the table), evaluated by one launch and read back into `out`
// (host, 2 per check); slot[i] is member i's check or -1.
static lbm_status batch_steady_into(lbm_batch B, int64_t window, double tol, int32_t* steady, double* rel_change,
                                    SteadyCheck* checks, int* slot, double* out, size_t cap, char* dev) {
  const size_t n = B->members.size();
  size_t nc = 0;
  for (size_t i = 0; i < n; ++i) {
    lbm_domain d = B->members[i];
    SteadyCheck c{};
    slot[i] = -1;
    if (d->body[0].active && steady_check(d, 0, window, c)) {
      if (nc >= cap) return fail(LBM_E_INVAL, "more steady-state checks than the table holds");
      slot[i] = (int)nc;
      checks[nc++] = c;
    }
  }
  if (nc > 0) {
    const size_t off = align256(nc * sizeof(SteadyCheck));
    HIP_TRY(hipMemcpyAsync(dev, checks, nc * sizeof(SteadyCheck), hipMemcpyHostToDevice, B->stream));
    double* dout = reinterpret_cast<double*>(dev + off);
    HIP_TRY(launch_steady(reinterpret_cast<const SteadyCheck*>(dev), (int)nc, dout, B->stream));
    HIP_TRY(hipMemcpyAsync(out, dout, 2 * nc * sizeof(double), hipMemcpyDeviceToHost, B->stream));
    HIP_TRY(hipStreamSynchronize(B->stream));
  }
  for (size_t i = 0; i < n; ++i) {
    if (slot[i] < 0) {
      steady[i] = -1;
      if (rel_change) rel_change[i] = NAN;
      continue;
    }
    const double r = out[2 * slot[i]];
    steady[i] = r < tol ? 1 : 0;
    if (rel_change) rel_change[i] = r;
  }
  for (lbm_domain d : B->members) {
    lbm_status s = check_device_errors(d);
    if (s != LBM_OK) return s;
  }
  return LBM_OK;
}

lbm_status lbm_batch_steady_state(lbm_batch B, int64_t window, double tol, int32_t* steady, double* rel_change) {
  if (!B || !steady) return fail(LBM_E_INVAL, "null argument");
  const size_t n = B->members.size();
  if (n == 0) return LBM_OK;
  std::vector<SteadyCheck> checks(n);
  std::vector<int> slot(n, -1);
  std::vector<double> out(2 * n);
  const size_t need = align256(n * sizeof(SteadyCheck)) + out.size() * sizeof(double);
  if (need > B->steady_cap) {
    if (B->steady_dev) HIP_TRY(hipFree(B->steady_dev));
    B->steady_dev = nullptr;
    HIP_TRY(hipMalloc(&B->steady_dev, 2 * need));
    B->steady_cap = 2 * need;
  }
  return batch_steady_into(B, window, tol, steady, rel_change, checks.data(), slot.data(), out.data(), n,
                           B->steady_dev);
}

// Device memory of lbm_batch_steady_state_noalloc: the table of checks and
// their results, in a static array each GPU holds until the process ends.
// Host code never passes the array's name to a kernel or a copy (on the host
// it is only a stand-in for the symbol): it uses the address that
// hipGetSymbolAddress returns for the current device, looked up once per
// device on the entry point's first call there.
constexpr size_t STEADY_TABLE_BYTES = (LBM_STEADY_NOALLOC_MAX * sizeof(SteadyCheck) + 255) / 256 * 256;
constexpr size_t STEADY_SCRATCH_BYTES = STEADY_TABLE_BYTES + 2 * LBM_STEADY_NOALLOC_MAX * sizeof(double);
static __device__ __align__(256) char scratch[STEADY_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[MAX_DEVICES] = {};

lbm_status scratch_for_current_device(char** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(LBM_E_INVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(LBM_E_HIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[dev] = static_cast<char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return LBM_OK;
}
}  // namespace

lbm_status lbm_batch_steady_state_noalloc(lbm_batch B, int64_t window, double tol, int32_t* steady,
                                          double* rel_change) {
  if (!B || !steady) return fail(LBM_E_INVAL, "null argument");
  const size_t n = B->members.size();
  if (n == 0) return LBM_OK;
  if (n > (size_t)LBM_STEADY_NOALLOC_MAX)
    return fail(LBM_E_INVAL, "lbm_batch_steady_state_noalloc takes at most " +
                                 std::to_string(LBM_STEADY_NOALLOC_MAX) + " members, the batch has " +
                                 std::to_string(n));
  char* dev = nullptr;
  lbm_status st = scratch_for_current_device(&dev);
  if (st != LBM_OK) return st;
  // host tables on the stack: no allocation anywhere on this path
  SteadyCheck checks[LBM_STEADY_NOALLOC_MAX];
  int slot[LBM_STEADY_NOALLOC_MAX];
  double out[2 * LBM_STEADY_NOALLOC_MAX];
  static_assert(STEADY_TABLE_BYTES >= LBM_STEADY_NOALLOC_MAX * sizeof(SteadyCheck), "check table fits");
  return batch_steady_into(B, window, tol, steady, rel_change, checks, slot, out, n, dev);
}

lbm_status lbm_batch_set_config(lbm_batch B, const lbm_batch_config* cfg) {
  if (!B || !cfg) return fail(LBM_E_INVAL, "null argument");
  if (!config_ok(*cfg)) return fail(LBM_E_INVAL, "unsupported batch launch shape");
  B->cfg = *cfg;
  return LBM_OK;
}

lbm_status lbm_batch_get_config(lbm_batch B, lbm_batch_config* cfg) {
  if (!B || !cfg) return fail(LBM_E_INVAL, "null argument");
  *cfg = B->cfg;
  return LBM_OK;
}

lbm_status lbm_batch_tune(lbm_batch B, int32_t trial_steps, lbm_batch_config* chosen, lbm_batch_config* trials,
                          int32_t trial_cap, int32_t* ntrials) {
  if (!B || !chosen) return fail(LBM_E_INVAL, "null argument");
  if (trial_steps <= 0) return fail(LBM_E_INVAL, "trial_steps must be positive");
  if (B->members.empty()) return fail(LBM_E_STATE, "empty batch");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  lbm_batch_config best{};
  best.us_per_step = 1e300;
  int count = 0;
  lbm_status s = LBM_OK;
  for (int overlap = 0; overlap <= 1 && s == LBM_OK; ++overlap)
  for (const auto& v : BATCH_BULK_VARIANTS)
    for (int remap = 0; remap <= 1 && s == LBM_OK; ++remap)
      for (int order = 0; order <= 3 && s == LBM_OK; ++order) {
        if (order == 3 && v[1] != 1) continue;
        B->cfg = lbm_batch_config{v[0], v[1], remap, order, overlap, 0, 0.0};
        s = batch_step(B, trial_steps, e0, e1);
        if (s != LBM_OK) break;
        hipError_t e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
          s = fail(LBM_E_HIP, std::string("autotuner timing: ") + hipGetErrorString(e));
          break;
        }
        B->cfg.us_per_step = ms * 1e3 / trial_steps;
        if (trials && count < trial_cap) trials[count] = B->cfg;
        count++;
        if (B->cfg.us_per_step < best.us_per_step) best = B->cfg;
      }
  // graph mode: the best shape of each overlap setting replayed from a
  // captured sequence, against the best ordinary configuration, over a call
  // long enough to replay the graph (2 GRAPH_STEPS steps)
  if (s == LBM_OK) {
    lbm_batch_config cand[3];
    int nc = 0;
    cand[nc++] = best;
    for (int overlap = 0; overlap <= 1; ++overlap) {
      lbm_batch_config c = best;
      c.overlap = overlap;
      c.graph = 1;
      cand[nc++] = c;
    }
    lbm_batch_config best_long{};
    best_long.us_per_step = 1e300;
    for (int k = 0; k < nc && s == LBM_OK; ++k) {
      B->cfg = cand[k];
      s = batch_step(B, 2 * GRAPH_STEPS, e0, e1);
      if (s != LBM_OK) break;
      hipError_t e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        s = fail(LBM_E_HIP, std::string("autotuner timing: ") + hipGetErrorString(e));
        break;
      }
      B->cfg.us_per_step = ms * 1e3 / (2 * GRAPH_STEPS);
      if (trials && count < trial_cap) trials[count] = B->cfg;
      count++;
      if (B->cfg.us_per_step < best_long.us_per_step) best_long = B->cfg;
    }
    best = best_long;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != LBM_OK) return s;
  B->cfg = best;
  *chosen = best;
  if (ntrials) *ntrials = count;
  return LBM_OK;
}

}  // extern "C"
