// Advance of a moving body spread over many workgroups (the operation of
// k_body_advance, mode 1, for bodies whose region is too large for the
// single-workgroup kernels). Included by kernels_impl.hpp after the link rule,
// the refill and the block sums.
//
// The rows (y, z) of the body's region (the node box of poses t and t+1, rows
// y-fastest) are cut into slabs of WIDE_ROWS consecutive rows, one workgroup
// per slab; within a slab only the row windows of row_windows are visited
// (around the ends of the solid interval at both poses, widened by two nodes:
// outside them no node changes status or holds a link). Two launches per step:
//
//  k_wide_sets   status at t+1 of the slab's window nodes; momentum of the
//                covered nodes (fluid at t, solid at t+1); refill of the
//                uncovered ones (solid at t, fluid at t+1); the number of
//                links of the new pose. Per slab: the 8 node terms and the
//                link count, into the body's scratch. Nothing is written to
//                the node status, so every slab reads the status of t.
//  k_wide_links  the slab's links, in node order, at the offset the counts of
//                the slabs before it give; Delta, the boundary rule and the
//                momentum exchange of step t+1 (12 sums per slab); the new
//                status into the node status; the last workgroup to finish
//                adds the slabs' sums in slab order into the records of t and
//                t+1 and writes the link count.
//
// The status at t+1 of any node follows from its status at t and the shape
// function at the new pose: a fluid or own node is own when phi <= 0 and
// fluid otherwise, any other status stays. Applied to a node whose new status
// is already written the rule gives the same answer, so the second launch may
// commit the status while other workgroups still read it. Every sum is a
// fixed tree over the threads of a slab, then over the slabs in order: the
// records do not depend on the grid, and a body gives the same bits advanced
// alone or in a batch.
#pragma once

namespace lbm {

// per slab: 20 sums (the link rule's 12 at 0..11, the node terms at 12..19)
__device__ __forceinline__ double* wide_part(double* w, int s) { return w + 20 * s; }
__device__ __forceinline__ int* wide_count(double* w, int cap) { return reinterpret_cast<int*>(w + 20 * cap); }
__device__ __forceinline__ unsigned* wide_counter(double* w, int cap) {
  return reinterpret_cast<unsigned*>(wide_count(w, cap) + cap);
}

__device__ __forceinline__ uint8_t status_next(const BodyShape& bs, const Pose& P1, uint8_t self, uint8_t old, int x,
                                               int y, int z) {
  if (old != MASK_FLUID && old != self) return old;
  return shape_phi(bs, P1, (double)x, (double)y, (double)z) <= 0.0 ? self : (uint8_t)MASK_FLUID;
}

struct WideSlab {
  Region R;   // node box of the two poses
  int r0, nr;  // first region row of the slab, rows in it (0: beyond the region)
  int nslab;   // slabs of the region
};

__device__ __forceinline__ WideSlab wide_slab(const Pose& P0, const Pose& P1, int s) {
  WideSlab w;
  for (int a = 0; a < 3; ++a) {
    const int lo = (int)(P0.lo[a] < P1.lo[a] ? P0.lo[a] : P1.lo[a]);
    const int hi = (int)(P0.hi[a] > P1.hi[a] ? P0.hi[a] : P1.hi[a]);
    w.R.lo[a] = lo;
    w.R.n[a] = hi - lo + 1;
  }
  w.R.total = (int64_t)w.R.n[0] * w.R.n[1] * w.R.n[2];
  const int nrow = w.R.n[1] * w.R.n[2];
  w.nslab = (nrow + WIDE_ROWS - 1) / WIDE_ROWS;
  w.r0 = s * WIDE_ROWS;
  w.nr = w.r0 < nrow ? (nrow - w.r0 < WIDE_ROWS ? nrow - w.r0 : WIDE_ROWS) : 0;
  return w;
}

// windows of the slab's rows and the first list entry of each row (the list
// runs over rows, windows and x in order); rowoff[nr] = entries in the slab
struct WideRows {
  int16_t win[WIDE_ROWS][4];
  int8_t nwin[WIDE_ROWS];
  int rowoff[WIDE_ROWS + 1];
};

__device__ __forceinline__ void wide_windows(const BodyShape& bs, const Pose& P0, const Pose& P1, const WideSlab& w,
                                             int D, WideRows& wr) {
  const Region& R = w.R;
  if ((int)threadIdx.x < w.nr) {
    const int r = w.r0 + (int)threadIdx.x;
    int v[4] = {0, -1, 0, -1};
    const int n = row_windows(bs, P0, P1, R.lo[1] + r % R.n[1], R.lo[2] + r / R.n[1], D, 2, R.lo[0],
                              R.lo[0] + R.n[0] - 1, v);
    wr.nwin[threadIdx.x] = (int8_t)n;
#pragma unroll
    for (int q = 0; q < 4; ++q) wr.win[threadIdx.x][q] = (int16_t)v[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int r = 0; r < w.nr; ++r) {
      wr.rowoff[r] = acc;
      if (wr.nwin[r] > 0) acc += wr.win[r][1] - wr.win[r][0] + 1;
      if (wr.nwin[r] > 1) acc += wr.win[r][3] - wr.win[r][2] + 1;
    }
    wr.rowoff[w.nr] = acc;
  }
  __syncthreads();
}

// node of list entry e (0 <= e < rowoff[nr])
__device__ __forceinline__ void wide_node(const WideSlab& w, const WideRows& wr, int e, int& x, int& y, int& z) {
  int lo = 0, hi = w.nr - 1;  // last row whose first entry is <= e
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (wr.rowoff[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  const int o = e - wr.rowoff[lo];
  const int len0 = wr.win[lo][1] - wr.win[lo][0] + 1;
  x = o < len0 ? wr.win[lo][0] + o : wr.win[lo][2] + (o - len0);
  const int r = w.r0 + lo;
  y = w.R.lo[1] + r % w.R.n[1];
  z = w.R.lo[2] + r / w.R.n[1];
}

// status bytes of node c and of its pull sources c - c_i (i = 1 .. Q-1),
// loaded together (one round trip to memory)
template <class L>
__device__ __forceinline__ void gather_status(const uint8_t* mask, const Geom& g, int64_t c, uint8_t st[L::Q]) {
#pragma unroll
  for (int i = 0; i < L::Q; ++i) st[i] = mask[c - (L::cx(i) + L::cy(i) * g.sy + L::cz(i) * g.sz)];
}

// bit i set: the pull source x - c_i of a node fluid at t+1 is own at t+1
// (a link of the new pose), from the gathered status bytes
template <class L>
__device__ __forceinline__ uint32_t link_dirs(const BodyShape& bs, const Pose& P1, uint8_t self,
                                              const uint8_t st[L::Q], int x, int y, int z) {
  uint32_t dirs = 0;
#pragma unroll
  for (int i = 1; i < L::Q; ++i)
    if (status_next(bs, P1, self, st[i], x - L::cx(i), y - L::cy(i), z - L::cz(i)) == self) dirs |= 1u << i;
  return dirs;
}

// first launch, slab s of one body (pose: its poses of t and t+1; B: the
// state of t+1; cap_slabs: the slabs its scratch holds). The slab's window
// nodes go in chunks of WIDE_BLOCK, one per thread.
template <class L, class S, int EQ>
__device__ __forceinline__ void wide_sets(typename S::T* B, const uint8_t* mask, const double* pose,
                                          const BodyShape& bs, int body, const Geom& g, const Phys& ph,
                                          double* scratch, int cap_slabs, int* err, int s) {
  constexpr int NT = WIDE_BLOCK;
  __shared__ WideRows wr;
  __shared__ int scan_sm[NT / 64 + 1];
  __shared__ uint16_t unc[NT];  // uncovered nodes of the current chunk (thread index within it)
  __shared__ double sm[8 * NT / 64];
  const Pose P0 = reinterpret_cast<const Pose*>(pose)[0];
  const Pose P1 = reinterpret_cast<const Pose*>(pose)[1];
  const uint8_t self = (uint8_t)(MASK_BODY0 + body);
  const WideSlab w = wide_slab(P0, P1, s);
  if (w.nslab > cap_slabs) {  // the region outgrew the scratch: reported, nothing done
    if (s == 0 && threadIdx.x == 0) atomicOr(err, 4);
    return;
  }
  if (w.nr == 0) return;
  wide_windows(bs, P0, P1, w, L::D, wr);
  const int nlist = wr.rowoff[w.nr];
  // a node that is fluid at t and t+1 (the refill's neighbours)
  auto fluid_both = [&](int xa, int ya, int za) {
    return mask[g.idx(xa, ya, za)] == MASK_FLUID && shape_phi(bs, P1, (double)xa, (double)ya, (double)za) > 0.0;
  };
  double imp[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // [0..2] F, [3..5] T, [6] covered, [7] uncovered
  int my_links = 0;
  for (int c0 = 0; c0 < nlist; c0 += NT) {
    const int e = c0 + (int)threadIdx.x;
    bool uncovered = false;
    if (e < nlist) {
      int x, y, z;
      wide_node(w, wr, e, x, y, z);
      const int64_t c = g.idx(x, y, z);
      uint8_t st[L::Q];
      gather_status<L>(mask, g, c, st);
      const uint8_t old = st[0];
      const bool solid = shape_phi(bs, P1, (double)x, (double)y, (double)z) <= 0.0;
      if (old != MASK_FLUID && old != self) {
        if (solid) atomicOr(err, 2);
      } else if (solid) {
        if (old == MASK_FLUID) {  // covered
          double m[3] = {0, 0, 0};
#pragma unroll
          for (int i = 1; i < L::Q; ++i) {
            const double v = (double)S::load(B + i * g.S + c);
            m[0] += L::cx(i) * v;
            m[1] += L::cy(i) * v;
            m[2] += L::cz(i) * v;
          }
          const double rr[3] = {x - P0.X[0], y - P0.X[1], z - P0.X[2]};
          imp[0] += m[0];
          imp[1] += m[1];
          imp[2] += m[2];
          imp[3] += rr[1] * m[2] - rr[2] * m[1];
          imp[4] += rr[2] * m[0] - rr[0] * m[2];
          imp[5] += rr[0] * m[1] - rr[1] * m[0];
          imp[6] += 1.0;
        }
      } else {
        uncovered = old == self;
        my_links += __popc(link_dirs<L>(bs, P1, self, st, x, y, z));
      }
    }
    // refill of the chunk's uncovered nodes: a group of G lanes per node,
    // lane j reading the moments of neighbour j + 1, summed by a fixed
    // shuffle tree
    const int pos = block_exclusive_scan<NT>(uncovered ? 1 : 0, scan_sm);
    const int nunc = scan_sm[NT / 64];
    if (uncovered) unc[pos] = (uint16_t)threadIdx.x;
    __syncthreads();
    constexpr int G = L::Q - 1 <= 8 ? 8 : 32;
    const int j = threadIdx.x & (G - 1);
    for (int u = (int)threadIdx.x / G; u < nunc; u += NT / G) {
      int x, y, z;
      wide_node(w, wr, c0 + (int)unc[u], x, y, z);
      double v[5] = {0, 0, 0, 0, 0};  // density, velocity, count
      if (j + 1 < L::Q) {
        const Dir<L> d = dir_of<L>(j + 1);
        const int xn = x + d.cx, yn = y + d.cy, zn = z + d.cz;
        if (fluid_both(xn, yn, zn)) {
          double hn[L::Q], dn, un[3];
          moments_at<L, S>(B, g, g.idx(xn, yn, zn), ph.rho0, EQ, hn, dn, un);
          v[0] = ph.rho0 + dn;
          v[1] = un[0];
          v[2] = un[1];
          v[3] = un[2];
          v[4] = 1.0;
        }
      }
#pragma unroll
      for (int o = G / 2; o > 0; o >>= 1)
#pragma unroll
        for (int q = 0; q < 5; ++q) v[q] += __shfl_xor(v[q], o, G);
      if (j != 0) continue;
      const double us[3] = {v[1], v[2], v[3]};
      refill_node<L, S, EQ>(B, g, ph, P0, P1, bs, x, y, z, v[0], us, v[4], fluid_both, imp);
    }
    __syncthreads();  // unc is refilled by the next chunk
  }
  block_exclusive_scan<NT>(my_links, scan_sm);
  const int nl = scan_sm[NT / 64];
  block_sum<8, NT>(imp, wide_part(scratch, s) + 12, sm);
  if (threadIdx.x == 0) wide_count(scratch, cap_slabs)[s] = nl;
}

// second launch, slab s of one body; every workgroup of the grid (gridDim.x
// of them per body) passes the arrival counter once
template <class L, class S, int EQ>
__device__ __forceinline__ void wide_links(typename S::T* B, uint8_t* mask, Link* links, int* n_links, int cap,
                                           const double* pose, const BodyShape& bs, int bc, int body, const Geom& g,
                                           const Phys& ph, double* scratch, int cap_slabs, double* rec_t,
                                           double* rec_t1, int* err, int s) {
  constexpr int NT = WIDE_BLOCK;
  __shared__ WideRows wr;
  __shared__ int scan_sm[NT / 64 + 1];
  __shared__ uint32_t linfo[WIDE_LINKS];  // the slab's first links: list entry << 8 | direction
  __shared__ double sm[12 * NT / 64];
  __shared__ int last;
  const Pose P0 = reinterpret_cast<const Pose*>(pose)[0];
  const Pose P1 = reinterpret_cast<const Pose*>(pose)[1];
  const uint8_t self = (uint8_t)(MASK_BODY0 + body);
  const WideSlab w = wide_slab(P0, P1, s);
  const bool fits = w.nslab <= cap_slabs;
  const int* cnt = wide_count(scratch, cap_slabs);
  if (fits && w.nr > 0) {
    wide_windows(bs, P0, P1, w, L::D, wr);
    const int nlist = wr.rowoff[w.nr];
    // offset of the slab's links: the counts of the slabs before it
    int before = 0;
    for (int k = (int)threadIdx.x; k < s; k += NT) before += cnt[k];
    block_exclusive_scan<NT>(before, scan_sm);
    const int off = scan_sm[NT / 64];
    // the slab's links in node order, chunk by chunk (one node per thread,
    // a scan over the chunk); the new status is committed on the way
    int nl = 0;
    for (int c0 = 0; c0 < nlist; c0 += NT) {
      const int e = c0 + (int)threadIdx.x;
      uint32_t dirs = 0;
      int x = 0, y = 0, z = 0;
      if (e < nlist) {
        wide_node(w, wr, e, x, y, z);
        const int64_t c = g.idx(x, y, z);
        uint8_t st[L::Q];
        gather_status<L>(mask, g, c, st);
        const uint8_t nw = status_next(bs, P1, self, st[0], x, y, z);
        if (nw != st[0]) mask[c] = nw;
        if (nw == MASK_FLUID) dirs = link_dirs<L>(bs, P1, self, st, x, y, z);
      }
      int b = nl + block_exclusive_scan<NT>(__popc(dirs), scan_sm);
      nl += scan_sm[NT / 64];
      for (uint32_t m = dirs; m; m &= m - 1) {
        const int i = __ffs(m) - 1;
        if (b < WIDE_LINKS) {
          linfo[b] = ((uint32_t)e << 8) | (uint32_t)i;
        } else if (off + b < cap) {  // beyond the LDS list: through global memory
          Link lk;
          lk.cell = (int32_t)g.idx(x, y, z);
          lk.x = (int16_t)x;
          lk.y = (int16_t)y;
          lk.z = (int16_t)z;
          lk.dir = (int16_t)i;
          lk.delta = 0.5;
          links[off + b] = lk;
        }
        b++;
      }
    }
    __syncthreads();
    // one link per thread: Delta, boundary rule, momentum exchange; the link
    // record with its Delta
    double acc[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = (int)threadIdx.x; k < nl && off + k < cap; k += NT) {
      Link lk;
      if (k < WIDE_LINKS) {
        const uint32_t v = linfo[k];
        int x, y, z;
        wide_node(w, wr, (int)(v >> 8), x, y, z);
        lk.cell = (int32_t)g.idx(x, y, z);
        lk.x = (int16_t)x;
        lk.y = (int16_t)y;
        lk.z = (int16_t)z;
        lk.dir = (int16_t)(v & 0xff);
      } else {
        lk = links[off + k];
      }
      const Dir<L> d = dir_of<L>(lk.dir);
      lk.delta = bc ? link_delta(bs, P1, (double)lk.x, (double)lk.y, (double)lk.z, d.cx, d.cy, d.cz) : 0.5;
      const int xn = lk.x + d.cx, yn = lk.y + d.cy, zn = lk.z + d.cz;
      const bool nb = status_next(bs, P1, self, mask[g.idx(xn, yn, zn)], xn, yn, zn) == MASK_FLUID;
      link_rule<L, S, EQ>(B, lk, P1, bc, nb, g, ph, acc);
      links[off + k] = lk;
    }
    block_sum<12, NT>(acc, wide_part(scratch, s), sm);
  }
  // the last workgroup adds the slabs in order
  __threadfence();
  __syncthreads();
  unsigned* counter = wide_counter(scratch, cap_slabs);
  if (threadIdx.x == 0) last = atomicAdd(counter, 1u) == gridDim.x - 1;
  __syncthreads();
  if (!last) return;
  __threadfence();
  if (threadIdx.x == 0) *counter = 0u;
  if (!fits) return;
  const int lane = threadIdx.x & 63;
  for (int k = (int)(threadIdx.x >> 6); k < 20; k += NT / 64) {
    double v = 0.0;
    for (int q = lane; q < w.nslab; q += 64) v += __builtin_nontemporal_load(wide_part(scratch, q) + k);
    v = wave_sum(v);
    if (lane == 0) {
      if (k < 6) rec_t1[k] = v;            // static F, T of t+1
      else if (k < 12) rec_t1[k + 6] = v;  // comoving F, T of t+1
      else if (k < 18) rec_t[k - 6] = v;   // node terms of t
      else rec_t[k] = v;                   // covered, uncovered counts of t
      if (k < 6) rec_t1[6 + k] = 0.0;
      if (k < 2) rec_t1[18 + k] = 0.0;
    }
  }
  int total = 0;
  for (int q = (int)threadIdx.x; q < w.nslab; q += NT) total += __builtin_nontemporal_load(cnt + q);
  block_exclusive_scan<NT>(total, scan_sm);
  if (threadIdx.x == 0) {
    const int nlk = scan_sm[NT / 64];
    *n_links = nlk < cap ? nlk : cap;
    if (nlk > cap) atomicOr(err, 1);
  }
}

template <class L, class S, int EQ>
__global__ __launch_bounds__(WIDE_BLOCK) void k_wide_sets(typename S::T* B, const uint8_t* mask, const double* pose,
                                                          BodyShape bs, int body, Geom g, Phys ph, double* scratch,
                                                          int cap_slabs, int* err) {
  wide_sets<L, S, EQ>(B, mask, pose, bs, body, g, ph, scratch, cap_slabs, err, (int)blockIdx.x);
}

template <class L, class S, int EQ>
__global__ __launch_bounds__(WIDE_BLOCK) void k_wide_links(typename S::T* B, uint8_t* mask, Link* links,
                                                           int* n_links, int cap, const double* pose, BodyShape bs,
                                                           int bc, int body, Geom g, Phys ph, double* scratch,
                                                           int cap_slabs, double* rec_t, double* rec_t1, int* err) {
  wide_links<L, S, EQ>(B, mask, links, n_links, cap, pose, bs, bc, body, g, ph, scratch, cap_slabs, rec_t, rec_t1,
                       err, (int)blockIdx.x);
}

}  // namespace lbm
