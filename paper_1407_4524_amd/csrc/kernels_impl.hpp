#pragma once
// Device code (kernel templates) of the lattice-Boltzmann step with momentum-exchange force and
// torque, for gfx950 (MI355X).
//
// Per time step t the host enqueues, on one stream:
//   k_links         (static bodies, or a moving body's first step) -- the
//                   interpolated boundary rule of Sec. II.A writes the value
//                   leaving the body into the solid node's slot of the source
//                   buffer and sums the momentum exchange of Eqs. flow_force_2,
//                   flow_torque_2 and the comoving-frame forms;
//   k_stream_collide the fused pull streaming + BGK collision (Eqs. LBE,
//                   collision, streaming) over every non-wall node, with
//                   the domain-face rules on the pull side (sweep.hpp);
//   k_body_advance  (moving bodies) covered/uncovered nodes between pose t
//                   and t+1, their momentum (Eqs. ForceInMovement,
//                   TorqueInMovement), refill, the link list of pose t+1 and
//                   the boundary rule + momentum exchange of step t+1.
// Populations are stored as deviations h_i = f_i - w_i rho0 in
// structure-of-arrays layout; momentum exchange accumulates in FP64.
#include "kernels.hpp"
#include "rows.hpp"
#include "reduce.hpp"
#include "sweep.hpp"

#include <hip/hip_ext.h>

#include <algorithm>
#include <type_traits>

namespace lbm {

// initial state: equilibrium deviations at (rho, u) per node, the densities
// of the x-face nodes and the fluid mask
template <class L, class S, int EQ>
__global__ __launch_bounds__(BULK_BLOCK) void k_init(typename S::T* __restrict__ A, uint8_t* __restrict__ mask,
                                                     Geom g, Phys ph, const double* __restrict__ rho_in,
                                                     const double* __restrict__ u_in, typename S::C* rho_out) {
  using C = typename S::C;
  const int x = g.lo[0] + blockIdx.x * BULK_BLOCK + threadIdx.x;
  const int y = g.lo[1] + blockIdx.y;
  const int z = g.lo[2] + blockIdx.z;
  if (x > g.hi[0]) return;
  const int64_t c = g.idx(x, y, z);
  const int64_t node = x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
  double rho = rho_in ? rho_in[node] : ph.rho0;
  double ux = 0, uy = 0, uz = 0;
  if (u_in) {
    ux = u_in[3 * node];
    uy = u_in[3 * node + 1];
    uz = L::D == 3 ? u_in[3 * node + 2] : 0.0;
  }
  const double drho = rho - ph.rho0;
  const double rhoU = EQ ? ph.rho0 : rho;
  const double usq = 1.5 * (ux * ux + uy * uy + uz * uz);
  C dr = 0;
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    double cu = L::cx(i) * ux + L::cy(i) * uy + L::cz(i) * uz;
    double heq = L::w(i) * (drho + rhoU * (3.0 * cu + 4.5 * cu * cu - usq));
    S::store_plain(A + i * g.S + c, heq);
    dr += S::load(A + i * g.S + c);
  }
  mask[c] = MASK_FLUID;
  // the density of the stored state, summed as a sweep sums it
  if (rho_out && (x == g.lo[0] || x == g.hi[0])) rho_out[xface_index(g, x, y, z)] = (C)ph.rho0 + dr;
}
// ---------------------------------------------------------------------------
// boundary links of a body

template <class L>
struct Dir {
  int i, cx, cy, cz, oi;
  double w;
};

template <class L>
__device__ __forceinline__ Dir<L> dir_of(int i) {
  Dir<L> d{0, 0, 0, 0, 0, 0.0};
#pragma unroll
  for (int q = 1; q < L::Q; ++q)
    if (q == i) d = Dir<L>{q, L::cx(q), L::cy(q), L::cz(q), L::opp(q), L::w(q)};
  return d;
}

template <class L, class S>
__device__ __forceinline__ void moments_at(const typename S::T* A, const Geom& g, int64_t c, double rho0, int eq,
                                  double h[L::Q], double& drho, double u[3]) {
  double jx = 0, jy = 0, jz = 0;
  drho = 0;
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    h[q] = (double)S::load(A + q * g.S + c);
    drho += h[q];
    jx += L::cx(q) * h[q];
    jy += L::cy(q) * h[q];
    jz += L::cz(q) * h[q];
  }
  const double rhoU = eq ? rho0 : rho0 + drho;
  u[0] = jx / rhoU;
  u[1] = jy / rhoU;
  u[2] = jz / rhoU;
}

// Moments at node c in the storage's compute type (FP32 for FP32 and FP16
// storage, FP64 for FP64), as the collision takes them.
template <class L, class S>
__device__ __forceinline__ void moments_c(const typename S::T* A, const Geom& g, int64_t c, double rho0, int eq,
                                          typename S::C h[L::Q], typename S::C& drho, typename S::C u[3]) {
  using C = typename S::C;
  C jx = 0, jy = 0, jz = 0;
  drho = 0;
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    h[q] = S::load(A + q * g.S + c);
    drho += h[q];
    jx += (C)L::cx(q) * h[q];
    jy += (C)L::cy(q) * h[q];
    jz += (C)L::cz(q) * h[q];
  }
  const C rhoU = eq ? (C)rho0 : (C)rho0 + drho;
  u[0] = jx / rhoU;
  u[1] = jy / rhoU;
  u[2] = jz / rhoU;
}

// Lattice direction of Lallemand & Luo's extrapolation at node (x, y, z):
// the one that maximises (n . c) / |c| for the outward normal n of pose P
// (ties: the smallest (cx, cy, cz) in lexicographic order).
template <class L>
__device__ __forceinline__ int extrap_dir(const BodyShape& bs, const Pose& P, int x, int y, int z) {
#pragma clang fp contract(off)
  double n[3];
  shape_normal(bs, P, (double)x, (double)y, (double)z, n);
  int best = 1;
  double best_s = 0.0;
#pragma unroll
  for (int i = 1; i < L::Q; ++i) {
    const int cx = L::cx(i), cy = L::cy(i), cz = L::cz(i);
    const bool diag = cx * cx + cy * cy + cz * cz == 2;
    const double sc = (n[0] * (double)cx + n[1] * (double)cy + n[2] * (double)cz) * (diag ? 0.70710678118654757 : 1.0);
    const int bx = L::cx(best), by = L::cy(best), bz = L::cz(best);
    const bool less = cx < bx || (cx == bx && (cy < by || (cy == by && cz < bz)));
    if (i == 1 || sc > best_s || (sc == best_s && less)) {
      best = i;
      best_s = sc;
    }
  }
  return best;
}

// Refill of node (x, y, z), which the body uncovers between poses P0 and P1
// (Sec. III.B.3), by the body's rule (bs.refill): MEAN, the equilibrium at
// the mean density and velocity of its neighbours fluid at t and t+1 (sums
// rs, us over cnt of them; rho0 and the wall velocity when cnt = 0); AIDUN,
// the equilibrium at that mean density and the wall velocity at the node;
// EXTRAPOLATE, h_i = (3 h_i(x+c) - 3 h_i(x+2c)) + h_i(x+3c) along extrap_dir
// when fluid_both says the three nodes are fluid at t and t+1 (MEAN
// otherwise), on the stored post-collision states of step t+1. Writes the node's populations (the state of t+1) and takes
// their momentum off the node terms imp, about X_c(t).
template <class L, class S, int EQ, bool STORE = true, class FluidBoth>
__device__ __forceinline__ void refill_node(typename S::T* B, const Geom& g, const Phys& ph, const Pose& P0,
                                            const Pose& P1, const BodyShape& bs, int x, int y, int z, double rs,
                                            const double us[3], double cnt, FluidBoth fluid_both, double imp[8]) {
  const int64_t c = g.idx(x, y, z);
  double hv[L::Q];
  bool done = false;
  if (bs.refill == REFILL_EXTRAPOLATE) {
    const int i = extrap_dir<L>(bs, P1, x, y, z);
    const int dx = L::cx(i), dy = L::cy(i), dz = L::cz(i);
    if (fluid_both(x + dx, y + dy, z + dz) && fluid_both(x + 2 * dx, y + 2 * dy, z + 2 * dz) &&
        fluid_both(x + 3 * dx, y + 3 * dy, z + 3 * dz)) {
      const int64_t c1 = g.idx(x + dx, y + dy, z + dz), c2 = g.idx(x + 2 * dx, y + 2 * dy, z + 2 * dz),
                    c3 = g.idx(x + 3 * dx, y + 3 * dy, z + 3 * dz);
#pragma unroll
      for (int q = 0; q < L::Q; ++q) {
        const double h1 = (double)S::load(B + q * g.S + c1), h2 = (double)S::load(B + q * g.S + c2),
                     h3 = (double)S::load(B + q * g.S + c3);
        hv[q] = (3.0 * h1 - 3.0 * h2) + h3;
      }
      done = true;
    }
  }
  if (!done) {
    double rb, ub[3];
    const double wall[3] = {P1.V[0] - P1.Om * (y - P1.X[1]), P1.V[1] + P1.Om * (x - P1.X[0]), P1.V[2]};
    if (cnt > 0.0) {
      rb = rs / cnt;
      for (int a = 0; a < 3; ++a) ub[a] = us[a] / cnt;
    } else {
      rb = ph.rho0;
      for (int a = 0; a < 3; ++a) ub[a] = wall[a];
    }
    if (bs.refill == REFILL_AIDUN)
      for (int a = 0; a < 3; ++a) ub[a] = wall[a];
    if (L::D == 2) ub[2] = 0.0;
    const double drb = rb - ph.rho0;
    const double rhoU = EQ ? ph.rho0 : rb;
    const double usq = 1.5 * (ub[0] * ub[0] + ub[1] * ub[1] + ub[2] * ub[2]);
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
      const double cu = L::cx(q) * ub[0] + L::cy(q) * ub[1] + L::cz(q) * ub[2];
      hv[q] = L::w(q) * (drb + rhoU * (3.0 * cu + 4.5 * cu * cu - usq));
    }
  }
  double m[3] = {0, 0, 0};
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    if constexpr (STORE) S::store_plain(B + q * g.S + c, hv[q]);
    const double v = S::round_trip(hv[q]);
    m[0] += L::cx(q) * v;
    m[1] += L::cy(q) * v;
    m[2] += L::cz(q) * v;
  }
  const double r[3] = {x - P0.X[0], y - P0.X[1], z - P0.X[2]};
  imp[0] -= m[0];
  imp[1] -= m[1];
  imp[2] -= m[2];
  imp[3] -= r[1] * m[2] - r[2] * m[1];
  imp[4] -= r[2] * m[0] - r[0] * m[2];
  imp[5] -= r[0] * m[1] - r[1] * m[0];
  imp[7] += 1.0;
}

// The interpolated boundary rule (Eq. Fillipova_interpolation with the
// Mei-Luo-Shyy u_bf and chi; halfway bounce-back when bc == 0) for one link,
// in deviation form, written to the solid node's slot; then the link's
// momentum exchange in FP64:
//   static   m = -c_i (f_i(x_F - c_i) + f_ibar(x_F))            (Eq. flow_force_2)
//   comoving m = -(c_i - v) f_i(x_F - c_i) + (c_ibar - v) f_ibar(x_F)
// with v the wall velocity at the link's wall point, and torques r x m about
// the body centre. The moving-wall term is +6 w_i rho c_i.u_B with c_i the
// outgoing direction (the sign that drives the fluid with the wall).
// nb_fluid: the node x_F + c_i (one step away from the wall) is fluid at t.
// Its populations are loaded together with those of x_F whatever the case
// (the node lies within the halo of the node array), so that the rule costs
// one round trip to memory; they are used only for Delta < 1/2 when it is
// fluid.
// acc: [0..2] F static, [3..5] T static, [6..8] F comoving, [9..11] T comoving.
template <class L, class S, int EQ>
__device__ __forceinline__ void link_rule(typename S::T* A, const Link& lk, const Pose& P, int bc, bool nb_fluid,
                          const Geom& g, const Phys& ph, double acc[12]) {
  using C = typename S::C;
  const Dir<L> d = dir_of<L>(lk.dir);
  const int64_t c = lk.cell;
  const int64_t off = d.cx + d.cy * g.sy + d.cz * g.sz;
  C h[L::Q], drho, uF[3];
  moments_c<L, S>(A, g, c, ph.rho0, EQ, h, drho, uF);
  C hg[L::Q], dg, ug[3];
  moments_c<L, S>(A, g, bc ? c + off : c, ph.rho0, EQ, hg, dg, ug);
  C hin = 0;
#pragma unroll
  for (int q = 0; q < L::Q; ++q)
    if (q == d.oi) hin = h[q];
  const C rhoU = EQ ? (C)ph.rho0 : (C)ph.rho0 + drho;
  const double xF = lk.x, yF = lk.y, zF = lk.z;
  const double dl = lk.delta;
  const double xB = xF - dl * d.cx, yB = yF - dl * d.cy;
  const double uB[3] = {P.V[0] - P.Om * (yB - P.X[1]), P.V[1] + P.Om * (xB - P.X[0]), L::D == 3 ? P.V[2] : 0.0};
  const C uBc[3] = {(C)uB[0], (C)uB[1], (C)uB[2]};
  const C wall = (C)(6.0 * d.w) * rhoU * ((C)d.cx * uBc[0] + (C)d.cy * uBc[1] + (C)d.cz * uBc[2]);
  C hbc;
  if (bc == 0) {
    hbc = hin + wall;
  } else {
    const C dlc = (C)dl;
    C ubf[3], chi;
    if (dl >= 0.5) {
      const C f = (C)1.5 / dlc;
      for (int a = 0; a < 3; ++a) ubf[a] = uF[a] + f * (uBc[a] - uF[a]);
      chi = ((C)2 * dlc - (C)1) / ((C)ph.tau + (C)0.5);
    } else {
      for (int a = 0; a < 3; ++a) ubf[a] = nb_fluid ? ug[a] : uF[a];
      chi = ((C)2 * dlc - (C)1) / ((C)ph.tau - (C)2);
    }
    const C cb_ubf = -((C)d.cx * ubf[0] + (C)d.cy * ubf[1] + (C)d.cz * ubf[2]);
    const C cb_uF = -((C)d.cx * uF[0] + (C)d.cy * uF[1] + (C)d.cz * uF[2]);
    const C uu = uF[0] * uF[0] + uF[1] * uF[1] + uF[2] * uF[2];
    const C gdev = (C)d.w * (drho + rhoU * ((C)3 * cb_ubf + (C)4.5 * cb_uF * cb_uF - (C)1.5 * uu));
    hbc = ((C)1 - chi) * hin + chi * gdev + wall;
  }
  typename S::T* slot = A + d.i * g.S + c - off;
  S::store_plain(slot, hbc);
  const double wr = d.w * ph.rho0;
  const double fbc = S::round_trip(hbc) + wr;
  const double fin = hin + wr;
  const double r[3] = {xF - P.X[0], yF - P.X[1], zF - P.X[2]};
  const double s = fbc + fin;
  const double m[3] = {-d.cx * s, -d.cy * s, -d.cz * s};
  const double mc[3] = {-(d.cx - uB[0]) * fbc + (-d.cx - uB[0]) * fin,
                        -(d.cy - uB[1]) * fbc + (-d.cy - uB[1]) * fin,
                        -(d.cz - uB[2]) * fbc + (-d.cz - uB[2]) * fin};
  acc[0] += m[0];
  acc[1] += m[1];
  acc[2] += m[2];
  acc[3] += r[1] * m[2] - r[2] * m[1];
  acc[4] += r[2] * m[0] - r[0] * m[2];
  acc[5] += r[0] * m[1] - r[1] * m[0];
  acc[6] += mc[0];
  acc[7] += mc[1];
  acc[8] += mc[2];
  acc[9] += r[1] * mc[2] - r[2] * mc[1];
  acc[10] += r[2] * mc[0] - r[0] * mc[2];
  acc[11] += r[0] * mc[1] - r[1] * mc[0];
}

// link_rule with the neighbour status read from the global node mask
template <class L, class S, int EQ>
__device__ __forceinline__ void link_rule_m(typename S::T* A, const Link& lk, const Pose& P, int bc,
                                            const uint8_t* mask, const Geom& g, const Phys& ph, double acc[12]) {
  const Dir<L> d = dir_of<L>(lk.dir);
  const bool nb = mask[lk.cell + d.cx + d.cy * g.sy + d.cz * g.sz] == MASK_FLUID;
  link_rule<L, S, EQ>(A, lk, P, bc, nb, g, ph, acc);
}

// Deterministic block sum of N doubles per thread: xor-shuffle tree inside
// each 64-wide wavefront, then a fixed-order sum over wavefronts.
template <int N, int NT>
__device__ __forceinline__ void block_sum(double v[N], double* out /* shared or global, N */, double* sm /* shared N*NT/64 */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    double x = v[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0) sm[wave * N + k] = x;
  }
  __syncthreads();
  if (threadIdx.x < N) {
    double s = 0;
    for (int w = 0; w < NT / 64; ++w) s += sm[w * N + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// Boundary rule + momentum exchange over a body's link list at step t. The
// last block to finish sums the per-block partials in block order and writes
// the step's record (static and comoving sums; node terms zero): block blk
// of nblk (NTL threads each) working on one body's links. Wave w
// of the grid takes the chunks of 64 consecutive links c = w, w + waves, ...
// and sums each chunk with a fixed shuffle tree into partials[c]; the first
// wave of the last block to finish adds the chunk sums, lane l over chunks
// l, l + 64, ... in order, then across lanes with the same tree. The result
// therefore does not depend on the block size or the grid.
template <class L, class S, int EQ, int NTL>
__device__ __forceinline__ void links_block(typename S::T* A, const Link* __restrict__ links, int n,
                                            const double* __restrict__ pose, int bc,
                                            const uint8_t* __restrict__ mask, const Geom& g, const Phys& ph,
                                            double* partials, unsigned* counter, double* rec, int blk, int nblk) {
  __shared__ int last;
  const Pose P = *reinterpret_cast<const Pose*>(pose);
  const int lane = threadIdx.x & 63;
  const int nchunks = (n + 63) >> 6;
  const int waves = nblk * (NTL / 64);
  for (int c = blk * (NTL / 64) + (int)(threadIdx.x >> 6); c < nchunks; c += waves) {
    double acc[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int k = c * 64 + lane;
    if (k < n) link_rule_m<L, S, EQ>(A, links[k], P, bc, mask, g, ph, acc);
#pragma unroll
    for (int j = 0; j < 12; ++j) {
      const double v = wave_sum(acc[j]);
      if (lane == j) partials[c * 12 + j] = v;
    }
  }
  if (nblk == 1) {  // the block's own chunk sums: no other block to wait for
    __syncthreads();
    if (threadIdx.x == 0) last = 1;
    __syncthreads();
  } else {
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) last = (atomicAdd(counter, 1u) == (unsigned)nblk - 1);
    __syncthreads();
  }
  if (last && threadIdx.x < 64) {
    if (nblk > 1) __threadfence();
    double acc[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int c = lane; c < nchunks; c += 64)
#pragma unroll
      for (int j = 0; j < 12; ++j) acc[j] += __builtin_nontemporal_load(partials + c * 12 + j);
#pragma unroll
    for (int j = 0; j < 12; ++j) {
      const double v = wave_sum(acc[j]);
      if (lane == j) rec[j < 6 ? j : j + 6] = v;  // static -> 0..5, comoving -> 12..17
    }
    if (lane >= 12 && lane < 18) rec[lane - 6] = 0.0;  // node terms 6..11
    if (lane >= 18 && lane < 20) rec[lane] = 0.0;      // counts 18, 19
    if (lane == 0 && nblk > 1) *counter = 0u;
  }
}

template <class L, class S, int EQ>
__global__ __launch_bounds__(LINK_BLOCK) void k_links(typename S::T* A, const Link* __restrict__ links, int n_host,
                                                      const int* __restrict__ n_dev, const double* __restrict__ pose,
                                                      int bc, const uint8_t* __restrict__ mask, Geom g, Phys ph,
                                                      double* partials, unsigned* counter, double* rec) {
  const int n = n_dev ? *n_dev : n_host;
  links_block<L, S, EQ, LINK_BLOCK>(A, links, n, pose, bc, mask, g, ph, partials, counter, rec, blockIdx.x, gridDim.x);
}

// The boundary rule + momentum exchange over a body's link list at step t,
// without the final sum: workgroup w (one wavefront, so that the chunks
// spread over as many compute units as there are chunks: 9.6 -> 7.0 us for
// the 15k links of a radius-16 sphere) takes chunk w of 64 consecutive
// links and writes the chunk's 12 sums (fixed shuffle tree) to part[12 w ..],
// the step's slot of the body's ring of partial sums; k_fold adds the chunks
// later, for many steps in one launch. Two dependent memory round trips per
// step (link record, then the populations) and no grid-wide handshake.
template <class L, class S, int EQ>
__global__ __launch_bounds__(64) void k_links_part(typename S::T* A, const Link* __restrict__ links, int n,
                                                   const double* __restrict__ pose, int bc,
                                                   const uint8_t* __restrict__ mask, Geom g, Phys ph,
                                                   double* __restrict__ part) {
  __shared__ double sm[12 * 64 + 48];
  const int lane = threadIdx.x;
  const int c = (int)blockIdx.x;
  if (c > 0 && c * 64 >= n) return;  // wave-uniform; chunk 0 is written even without links (zero sums)
  const Pose P = *reinterpret_cast<const Pose*>(pose);
  double acc[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  const int k = c * 64 + lane;
  if (k < n) link_rule_m<L, S, EQ>(A, links[k], P, bc, mask, g, ph, acc);
  // the chunk's 12 sums, the bits of wave_sum (the kernel's time is one
  // wavefront's instruction chain, of which the DPP sums took a third)
  const double v = wave_sums_lds<12>(acc, sm);
  if (lane < 12) part[c * 12 + lane] = v;
}

// ---------------------------------------------------------------------------
// momentum exchange of the domain faces (the channel budget behind Eq.
// flow_force_2), and the NaN fill of a debug domain's solid nodes

// Node k of the enumeration of the active nodes next to a face, slab by
// slab: x = lo, x = hi, y = lo, y = hi, then z = lo, z = hi in 3D; a node in
// several slabs belongs to the first. 32-bit index arithmetic.
__device__ __forceinline__ bool face_node(const Geom& g, int k, int& x, int& y, int& z) {
  const int n0 = g.hi[0] - g.lo[0] + 1, n1 = g.hi[1] - g.lo[1] + 1, n2 = g.hi[2] - g.lo[2] + 1;
  const int sx = n1 * n2, sy = n0 * n2, sz = n0 * n1;
  if (k < 2 * sx) {
    const int side = k >= sx, r = side ? k - sx : k;
    x = side ? g.hi[0] : g.lo[0];
    y = g.lo[1] + r % n1;
    z = g.lo[2] + r / n1;
    return !(side && n0 == 1);
  }
  k -= 2 * sx;
  if (k < 2 * sy) {
    const int side = k >= sy, r = side ? k - sy : k;
    x = g.lo[0] + r % n0;
    y = side ? g.hi[1] : g.lo[1];
    z = g.lo[2] + r / n0;
    return !(side && n1 == 1) && x != g.lo[0] && x != g.hi[0];
  }
  k -= 2 * sy;
  if (g.D == 3 && k < 2 * sz) {
    const int side = k >= sz, r = side ? k - sz : k;
    x = g.lo[0] + r % n0;
    y = g.lo[1] + r / n0;
    z = side ? g.hi[2] : g.lo[2];
    return !(side && n2 == 1) && x != g.lo[0] && x != g.hi[0] && y != g.lo[1] && y != g.hi[1];
  }
  return false;
}

// Per face node (one per thread) and direction whose pull crosses a face:
// the value leaving the face is the face rule's (see face_pull; the velocity
// bounce-back term in the collision's type, as in the sweep) and the
// momentum exchanged is -c_i (f_out + f_in) with f = h + w_i rho0, torque
// about the origin. Walls, inlet and outlet(s) are summed apart (18 values)
// and every wavefront writes its 18 sums (fixed shuffle tree) to part, the
// step's slot of the domain's face ring; k_fold_faces adds them later.
template <class L, class S, int EQ>
__global__ __launch_bounds__(256) void k_face_part(const typename S::T* __restrict__ A, Geom g, Phys ph,
                                                   const typename S::C* __restrict__ rho_in, int nnodes,
                                                   double* __restrict__ part) {
  using C = typename S::C;
  const int k = (int)blockIdx.x * 256 + (int)threadIdx.x;
  const int lane = threadIdx.x & 63;
  const int chunk = k >> 6;  // one per wavefront: face_chunks = ceil(nnodes / 64) of them
  if (chunk * 64 >= nnodes) return;  // wave-uniform
  double acc[18];
#pragma unroll
  for (int j = 0; j < 18; ++j) acc[j] = 0.0;
  int x, y, z;
  if (k < nnodes && face_node(g, k, x, y, z)) {
    const int64_t c = g.idx(x, y, z);
    C rho_w = (C)ph.rho0;
    if (!EQ && rho_in && (x == g.lo[0] || x == g.hi[0])) rho_w = rho_in[xface_index(g, x, y, z)];
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
      int st;
      const int64_t off = face_pull<L>(g, x, y, z, c, i, st);
      if (st == SRC_NONE) continue;
      const C fin = S::load(A + L::opp(i) * g.S + c);
      C fbc = st == SRC_OUTLET ? S::load(A + off) : fin;
      if (st == SRC_INLET || st == SRC_OUTVEL)
        fbc += (C)(6.0 * L::w(i) * L::cx(i)) * rho_w *
               inlet_speed<C>(g, ph, (C)y - (C)(0.5 * L::cy(i)), (C)z - (C)(0.5 * L::cz(i)));
      const double sum = (double)fbc + (double)fin + 2.0 * L::w(i) * ph.rho0;
      const double m[3] = {-L::cx(i) * sum, -L::cy(i) * sum, -L::cz(i) * sum};
      const double t[3] = {y * m[2] - z * m[1], z * m[0] - x * m[2], x * m[1] - y * m[0]};
      const double sw = st == SRC_WALL ? 1.0 : 0.0, si = st == SRC_INLET ? 1.0 : 0.0;
      const double so = (st == SRC_OUTLET || st == SRC_OUTVEL) ? 1.0 : 0.0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        acc[a] += sw * m[a];
        acc[3 + a] += sw * t[a];
        acc[6 + a] += si * m[a];
        acc[9 + a] += si * t[a];
        acc[12 + a] += so * m[a];
        acc[15 + a] += so * t[a];
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 18; ++j) {
    const double v = wave_sum(acc[j]);
    if (lane == j) part[chunk * 18 + j] = v;
  }
}

// NaN in every population slot (both buffers) of the nodes of body `self`
// inside the node box lo..hi (debug domains: a pull that reads a solid
// node's slot that no link rule wrote then shows)
template <class L, class S>
__global__ __launch_bounds__(256) void k_poison_body(typename S::T* A, typename S::T* B, const uint8_t* mask, Geom g,
                                                     int lo0, int lo1, int lo2, int n0, int n1, int64_t total,
                                                     uint8_t self) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= total) return;
  const int x = lo0 + (int)(k % n0), y = lo1 + (int)((k / n0) % n1), z = lo2 + (int)(k / ((int64_t)n0 * n1));
  const int64_t c = g.idx(x, y, z);
  if (mask[c] != self) return;
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    S::store_plain(A + i * g.S + c, __builtin_nan(""));
    S::store_plain(B + i * g.S + c, __builtin_nan(""));
  }
}

// ---------------------------------------------------------------------------
// body placement and advance (one workgroup per body)

constexpr int ADV_BLOCK = 1024;

struct Region {
  int lo[3], n[3];
  int64_t total;
  __device__ void at(int64_t k64, int& x, int& y, int& z) const {
    const unsigned k = (unsigned)k64;  // regions hold far fewer than 2^31 nodes
    const unsigned n0 = (unsigned)n[0], n1 = (unsigned)n[1];
    const unsigned r = k / n0;
    x = lo[0] + (int)(k - r * n0);
    const unsigned r2 = r / n1;
    y = lo[1] + (int)(r - r2 * n1);
    z = lo[2] + (int)r2;
  }
  __device__ bool contains(int x, int y, int z) const {
    return x >= lo[0] && x < lo[0] + n[0] && y >= lo[1] && y < lo[1] + n[1] && z >= lo[2] && z < lo[2] + n[2];
  }
};

// Inclusive prefix sum of an int over the 64 lanes of a wavefront: DPP row
// shifts within each row of 16 lanes, then the totals of the rows below
// (read out of lanes 15, 31, 47) added on; no LDS round trip.
__device__ __forceinline__ int wave_inclusive_scan(int x) {
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
  const int lane = threadIdx.x & 63;
  const int r0 = __builtin_amdgcn_readlane(x, 15), r1 = __builtin_amdgcn_readlane(x, 31),
            r2 = __builtin_amdgcn_readlane(x, 47);
  return x + (lane >= 16 ? r0 : 0) + (lane >= 32 ? r1 : 0) + (lane >= 48 ? r2 : 0);
}

// Exclusive prefix sum over the NT threads of a block (thread order); the
// total lands in sm[NT / 64]. Every thread of the block must call it.
template <int NT = 1024>
__device__ inline int block_exclusive_scan(int v, int* sm /* NT/64 + 1 */) {
  static_assert(NT % 64 == 0 && NT / 64 <= 64, "whole wavefronts, at most 64");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int x = wave_inclusive_scan(v);
  if (lane == 63) sm[wave] = x;
  __syncthreads();
  if (wave == 0) {  // the wavefront totals, scanned by the first wavefront
    const int t = lane < NT / 64 ? sm[lane] : 0;
    const int it = wave_inclusive_scan(t);
    if (lane < NT / 64) sm[lane] = it - t;
    if (lane == NT / 64 - 1) sm[NT / 64] = it;
  }
  __syncthreads();
  return sm[wave] + x - v;
}

// mode 0: place the body at pose p0 (mark its nodes, build its links).
// mode 1: advance from pose p0 (step t) to p1 (step t+1) after the bulk
// update of step t wrote the state of t+1 into B: covered nodes A+ (fluid at
// t, solid at t+1) give up their momentum, uncovered nodes A- are refilled
// with the equilibrium at the mean density and velocity of their neighbours
// that are fluid at t and t+1 (rho0 and the wall velocity if there are none);
// rec_t receives sum_{A+} c f - sum_{A-} c f (and r x ..., r about X_c(t))
// and the two counts; then the links of pose t+1 are built and the boundary
// rule and momentum exchange of step t+1 run, into rec_t1.
template <class L, class S, int EQ>
__global__ __launch_bounds__(ADV_BLOCK) void k_body_advance(typename S::T* B, uint8_t* mask, uint8_t* mask_next,
                                                            Link* links, int* n_links, int cap, const double* pose,
                                                            BodyShape bs, int bc, int body, int mode, Geom g,
                                                            Phys ph, double* rec_t, double* rec_t1, int* err) {
  using T = typename S::T;
  __shared__ double sm[20 * ADV_BLOCK / 64];
  __shared__ double red[20];
  __shared__ int scan_sm[ADV_BLOCK / 64 + 1];
  const Pose P0 = reinterpret_cast<const Pose*>(pose)[0];
  const Pose P1 = reinterpret_cast<const Pose*>(pose)[mode];
  const uint8_t self = (uint8_t)(MASK_BODY0 + body);
  Region R;
  for (int a = 0; a < 3; ++a) {
    int lo = (int)(P0.lo[a] < P1.lo[a] ? P0.lo[a] : P1.lo[a]);
    int hi = (int)(P0.hi[a] > P1.hi[a] ? P0.hi[a] : P1.hi[a]);
    R.lo[a] = lo;
    R.n[a] = hi - lo + 1;
  }
  R.total = (int64_t)R.n[0] * R.n[1] * R.n[2];
  const bool outer = bs.shape == SHAPE_OUTER_CIRCLE;
  // imp: [0..2] F nodes, [3..5] T nodes, [6] n+, [7] n-
  double imp[8] = {0, 0, 0, 0, 0, 0, 0, 0};

  // phase A: status at the new pose; momentum of covered nodes
  for (int64_t k = threadIdx.x; k < R.total; k += ADV_BLOCK) {
    int x, y, z;
    R.at(k, x, y, z);
    const int64_t c = g.idx(x, y, z);
    const uint8_t old = mask[c];
    const bool solid = shape_phi(bs, P1, (double)x, (double)y, (double)z) <= 0.0;
    uint8_t nw = old;
    if (old == MASK_FLUID || old == self) {
      nw = solid ? self : MASK_FLUID;
    } else if (solid && !outer) {
      atomicOr(err, 2);
    }
    mask_next[c] = nw;
    if (mode == 1 && old == MASK_FLUID && nw == self) {
      double m[3] = {0, 0, 0};
#pragma unroll
      for (int q = 1; q < L::Q; ++q) {
        const double v = (double)S::load(B + q * g.S + c);
        m[0] += L::cx(q) * v;
        m[1] += L::cy(q) * v;
        m[2] += L::cz(q) * v;
      }
      const double r[3] = {x - P0.X[0], y - P0.X[1], z - P0.X[2]};
      imp[0] += m[0];
      imp[1] += m[1];
      imp[2] += m[2];
      imp[3] += r[1] * m[2] - r[2] * m[1];
      imp[4] += r[2] * m[0] - r[0] * m[2];
      imp[5] += r[0] * m[1] - r[1] * m[0];
      imp[6] += 1.0;
    }
  }
  __syncthreads();

  // phase B: refill uncovered nodes; count links of the new pose (contiguous
  // chunks per thread so that the list comes out in node order)
  const int64_t chunk = (R.total + ADV_BLOCK - 1) / ADV_BLOCK;
  const int64_t k0 = threadIdx.x * chunk;
  const int64_t k1 = (k0 + chunk < R.total) ? k0 + chunk : R.total;
  int my_links = 0;
  for (int64_t k = k0; k < k1; ++k) {
    int x, y, z;
    R.at(k, x, y, z);
    const int64_t c = g.idx(x, y, z);
    const uint8_t nw = mask_next[c];
    if (nw != MASK_FLUID) continue;
    if (mode == 1 && mask[c] == self) {
      double rs = 0, us[3] = {0, 0, 0};
      int cnt = 0;
#pragma unroll
      for (int q = 1; q < L::Q; ++q) {
        const int xn = x + L::cx(q), yn = y + L::cy(q), zn = z + L::cz(q);
        const int64_t cn = g.idx(xn, yn, zn);
        const uint8_t nn = R.contains(xn, yn, zn) ? mask_next[cn] : mask[cn];
        if (mask[cn] != MASK_FLUID || nn != MASK_FLUID) continue;
        double hn[L::Q], dn, un[3];
        moments_at<L, S>(B, g, cn, ph.rho0, EQ, hn, dn, un);
        rs += ph.rho0 + dn;
        us[0] += un[0];
        us[1] += un[1];
        us[2] += un[2];
        cnt++;
      }
      auto fluid_both = [&](int xa, int ya, int za) {
        const int64_t ca = g.idx(xa, ya, za);
        const uint8_t na = R.contains(xa, ya, za) ? mask_next[ca] : mask[ca];
        return mask[ca] == MASK_FLUID && na == MASK_FLUID;
      };
      refill_node<L, S, EQ>(B, g, ph, P0, P1, bs, x, y, z, rs, us, (double)cnt, fluid_both, imp);
    }
#pragma unroll
    for (int q = 1; q < L::Q; ++q) {
      const int xs = x - L::cx(q), ys = y - L::cy(q), zs = z - L::cz(q);
      const int64_t cs = g.idx(xs, ys, zs);
      const uint8_t ns = R.contains(xs, ys, zs) ? mask_next[cs] : mask[cs];
      if (ns == self) my_links++;
    }
  }
  int base = block_exclusive_scan(my_links, scan_sm);
  const int total = scan_sm[ADV_BLOCK / 64];
  for (int64_t k = k0; k < k1; ++k) {
    int x, y, z;
    R.at(k, x, y, z);
    const int64_t c = g.idx(x, y, z);
    if (mask_next[c] != MASK_FLUID) continue;
#pragma unroll
    for (int q = 1; q < L::Q; ++q) {
      const int xs = x - L::cx(q), ys = y - L::cy(q), zs = z - L::cz(q);
      const int64_t cs = g.idx(xs, ys, zs);
      const uint8_t ns = R.contains(xs, ys, zs) ? mask_next[cs] : mask[cs];
      if (ns != self) continue;
      if (base < cap) {
        Link lk;
        lk.cell = (int32_t)c;
        lk.x = (int16_t)x;
        lk.y = (int16_t)y;
        lk.z = (int16_t)z;
        lk.dir = (int16_t)q;
        lk.delta = bc ? link_delta(bs, P1, (double)x, (double)y, (double)z, L::cx(q), L::cy(q), L::cz(q)) : 0.5;
        links[base] = lk;
      }
      base++;
    }
  }
  __syncthreads();
  // commit the new status
  for (int64_t k = threadIdx.x; k < R.total; k += ADV_BLOCK) {
    int x, y, z;
    R.at(k, x, y, z);
    const int64_t c = g.idx(x, y, z);
    mask[c] = mask_next[c];
  }
  if (threadIdx.x == 0) {
    *n_links = total < cap ? total : cap;
    if (total > cap) atomicOr(err, 1);
  }
  __syncthreads();
  if (mode == 0) return;

  // phase C: boundary rule + momentum exchange of step t+1
  const int nl = total < cap ? total : cap;
  double acc[20];
  for (int k = 0; k < 20; ++k) acc[k] = 0.0;
  for (int k = threadIdx.x; k < nl; k += ADV_BLOCK) link_rule_m<L, S, EQ>(B, links[k], P1, bc, mask, g, ph, acc);
  for (int k = 0; k < 8; ++k) acc[12 + k] = imp[k];
  block_sum<20, ADV_BLOCK>(acc, red, sm);
  if (threadIdx.x < 20) {
    const int k = threadIdx.x;
    const double v = red[k];
    if (k < 6) rec_t1[k] = v;
    else if (k < 12) rec_t1[k + 6] = v;
    else if (k < 18) rec_t[k - 6] = v;   // node terms 6..11 of step t
    else rec_t[k] = v;                   // counts 18, 19 of step t
    if (k < 6) rec_t1[6 + k] = 0.0;
    if (k < 2) rec_t1[18 + k] = 0.0;
  }
}



// Same operation as k_body_advance with the old and new node status of the
// region plus a one-node margin held in LDS (two bytes per node), so that
// every neighbour lookup of the link search and of the refill stays on chip;
// only the nodes whose status changes are written back to the global mask.
// Used whenever that box fits the LDS budget.
constexpr int ADV_WIN_ROWS = 2048;

template <class L, class S, int EQ>
__global__ __launch_bounds__(ADV_BLOCK) void k_body_advance_lds(typename S::T* B, uint8_t* mask, Link* links,
                                                                int* n_links, int cap, const double* pose,
                                                                BodyShape bs, int bc, int body, int mode, Geom g,
                                                                Phys ph, double* rec_t, double* rec_t1, int* err) {
  extern __shared__ uint8_t lds[];
  __shared__ double sm[20 * ADV_BLOCK / 64];
  // per region row: x-windows (advance only) outside which nothing changes
  __shared__ int16_t win[ADV_WIN_ROWS][4];
  __shared__ int8_t nwin[ADV_WIN_ROWS];
  __shared__ double red[20];
  __shared__ int scan_sm[ADV_BLOCK / 64 + 1];
  const Pose P0 = reinterpret_cast<const Pose*>(pose)[0];
  const Pose P1 = reinterpret_cast<const Pose*>(pose)[mode];
  const uint8_t self = (uint8_t)(MASK_BODY0 + body);
  Region R, E;  // body region, and the region with a one-node margin
  for (int a = 0; a < 3; ++a) {
    int lo = (int)(P0.lo[a] < P1.lo[a] ? P0.lo[a] : P1.lo[a]);
    int hi = (int)(P0.hi[a] > P1.hi[a] ? P0.hi[a] : P1.hi[a]);
    R.lo[a] = lo;
    R.n[a] = hi - lo + 1;
    const int m = a < L::D ? 1 : 0;
    E.lo[a] = lo - m;
    E.n[a] = R.n[a] + 2 * m;
  }
  R.total = (int64_t)R.n[0] * R.n[1] * R.n[2];
  E.total = (int64_t)E.n[0] * E.n[1] * E.n[2];
  const int total = (int)E.total;
  // lds[k] = status at t, lds[total + k] = status at t+1 of box node k
#define ADV_STATUS(x, y, z, nw) \
  lds[(nw) * total + ((x) - E.lo[0]) + E.n[0] * (((y) - E.lo[1]) + E.n[1] * ((z) - E.lo[2]))]
  const bool outer = bs.shape == SHAPE_OUTER_CIRCLE;
  double imp[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  // advancing a body whose rows fit the window table: a node outside its
  // row's windows (around the ends of the solid interval at both poses,
  // widened by two nodes) can neither change status nor hold a link
  const int nrow = R.n[1] * R.n[2];
  const bool windowed = mode == 1 && !outer && nrow <= ADV_WIN_ROWS;
  if (windowed)
    for (int r = threadIdx.x; r < nrow; r += ADV_BLOCK) {
      int w[4] = {0, -1, 0, -1};
      const int n = row_windows(bs, P0, P1, R.lo[1] + r % R.n[1], R.lo[2] + r / R.n[1], L::D, 2, R.lo[0],
                                R.lo[0] + R.n[0] - 1, w);
      nwin[r] = (int8_t)n;
      for (int q = 0; q < 4; ++q) win[r][q] = (int16_t)w[q];
    }
  auto in_window = [&](int x, int y, int z) -> bool {
    if (!windowed) return true;
    const int r = (y - R.lo[1]) + R.n[1] * (z - R.lo[2]);
    const int n = nwin[r];
    return (n > 0 && x >= win[r][0] && x <= win[r][1]) || (n > 1 && x >= win[r][2] && x <= win[r][3]);
  };

  __syncthreads();
  // phase A: status at the new pose, momentum of covered nodes, commit
  // changes. Each node's old status is read just before it is used: a form
  // that fetched the status bytes of eight nodes ahead gave wrong covered-node
  // sums with 4- and 2-byte storage on gfx950 (FP64 was right; the cause was
  // not found), and this kernel is not on the hot path.
  for (int k = threadIdx.x; k < total; k += ADV_BLOCK) {
    int x, y, z;
    E.at(k, x, y, z);
    const int64_t c = g.idx(x, y, z);
    const uint8_t old = mask[c];
    uint8_t nw = old;
    if (R.contains(x, y, z) && in_window(x, y, z)) {
      const bool solid = shape_phi(bs, P1, (double)x, (double)y, (double)z) <= 0.0;
      if (old == MASK_FLUID || old == self) nw = solid ? self : MASK_FLUID;
      else if (solid && !outer) atomicOr(err, 2);
    }
    lds[k] = old;
    lds[total + k] = nw;
    if (nw != old) mask[c] = nw;
    if (mode == 1 && old == MASK_FLUID && nw == self) {
      double m[3] = {0, 0, 0};
#pragma unroll
      for (int q = 1; q < L::Q; ++q) {
        const double v = (double)S::load(B + q * g.S + c);
        m[0] += L::cx(q) * v;
        m[1] += L::cy(q) * v;
        m[2] += L::cz(q) * v;
      }
      const double r[3] = {x - P0.X[0], y - P0.X[1], z - P0.X[2]};
      imp[0] += m[0];
      imp[1] += m[1];
      imp[2] += m[2];
      imp[3] += r[1] * m[2] - r[2] * m[1];
      imp[4] += r[2] * m[0] - r[0] * m[2];
      imp[5] += r[0] * m[1] - r[1] * m[0];
      imp[6] += 1.0;
    }
  }
  __syncthreads();

  // phase B: refill uncovered nodes and count the links of the new pose over
  // contiguous chunks of the box (node order); margin nodes hold no links
  const int chunk = (total + ADV_BLOCK - 1) / ADV_BLOCK;
  const int k0 = threadIdx.x * chunk;
  const int k1 = k0 + chunk < total ? k0 + chunk : total;
  int my_links = 0;
  for (int k = k0; k < k1; ++k) {
    if (lds[total + k] != MASK_FLUID) continue;
    int x, y, z;
    E.at(k, x, y, z);
    if (!R.contains(x, y, z) || !in_window(x, y, z)) continue;
    if (mode == 1 && lds[k] == self) {
      double rs = 0, us[3] = {0, 0, 0};
      int cnt = 0;
#pragma unroll
      for (int q = 1; q < L::Q; ++q) {
        const int xn = x + L::cx(q), yn = y + L::cy(q), zn = z + L::cz(q);
        if (ADV_STATUS(xn, yn, zn, 0) != MASK_FLUID || ADV_STATUS(xn, yn, zn, 1) != MASK_FLUID) continue;
        double hn[L::Q], dn, un[3];
        moments_at<L, S>(B, g, g.idx(xn, yn, zn), ph.rho0, EQ, hn, dn, un);
        rs += ph.rho0 + dn;
        us[0] += un[0];
        us[1] += un[1];
        us[2] += un[2];
        cnt++;
      }
      // beyond the status box a node keeps its status (the global mask)
      auto fluid_both = [&](int xa, int ya, int za) {
        if (!E.contains(xa, ya, za)) return mask[g.idx(xa, ya, za)] == MASK_FLUID;
        return ADV_STATUS(xa, ya, za, 0) == MASK_FLUID && ADV_STATUS(xa, ya, za, 1) == MASK_FLUID;
      };
      refill_node<L, S, EQ>(B, g, ph, P0, P1, bs, x, y, z, rs, us, (double)cnt, fluid_both, imp);
    }
#pragma unroll
    for (int q = 1; q < L::Q; ++q)
      if (ADV_STATUS(x - L::cx(q), y - L::cy(q), z - L::cz(q), 1) == self) my_links++;
  }
  int base = block_exclusive_scan(my_links, scan_sm);
  const int nlinks = scan_sm[ADV_BLOCK / 64];
  for (int k = k0; k < k1; ++k) {
    if (lds[total + k] != MASK_FLUID) continue;
    int x, y, z;
    E.at(k, x, y, z);
    if (!R.contains(x, y, z) || !in_window(x, y, z)) continue;
#pragma unroll
    for (int q = 1; q < L::Q; ++q) {
      if (ADV_STATUS(x - L::cx(q), y - L::cy(q), z - L::cz(q), 1) != self) continue;
      if (base < cap) {
        Link lk;
        lk.cell = (int32_t)g.idx(x, y, z);
        lk.x = (int16_t)x;
        lk.y = (int16_t)y;
        lk.z = (int16_t)z;
        lk.dir = (int16_t)q;
        lk.delta = 0.5;
        links[base] = lk;
      }
      base++;
    }
  }
#undef ADV_STATUS
  if (threadIdx.x == 0) {
    *n_links = nlinks < cap ? nlinks : cap;
    if (nlinks > cap) atomicOr(err, 1);
  }
  __syncthreads();

  // phase C: Delta per link (FP64), then, when advancing, the boundary rule
  // + momentum exchange of step t+1 -- one link per thread
  const int nl = nlinks < cap ? nlinks : cap;
  double acc[20];
  for (int k = 0; k < 20; ++k) acc[k] = 0.0;
  for (int k = threadIdx.x; k < nl; k += ADV_BLOCK) {
    Link lk = links[k];
    if (bc) {
      const Dir<L> d = dir_of<L>(lk.dir);
      lk.delta = link_delta(bs, P1, (double)lk.x, (double)lk.y, (double)lk.z, d.cx, d.cy, d.cz);
      links[k].delta = lk.delta;
    }
    if (mode == 1) link_rule_m<L, S, EQ>(B, lk, P1, bc, mask, g, ph, acc);
  }
  if (mode == 0) return;
  for (int k = 0; k < 8; ++k) acc[12 + k] = imp[k];
  block_sum<20, ADV_BLOCK>(acc, red, sm);
  if (threadIdx.x < 20) {
    const int k = threadIdx.x;
    const double v = red[k];
    if (k < 6) rec_t1[k] = v;
    else if (k < 12) rec_t1[k + 6] = v;
    else if (k < 18) rec_t[k - 6] = v;
    else rec_t[k] = v;
    if (k < 6) rec_t1[6 + k] = 0.0;
    if (k < 2) rec_t1[18 + k] = 0.0;
  }
}

// Advance of a moving body (the operation of k_body_advance, mode 1) for a
// region whose status box fits LDS: the per-row windows (around the ends of
// the solid x-interval at both poses and in the neighbouring rows, widened
// by two nodes) are gathered into one node list in node order, and every
// per-node phase walks that list only -- a node outside it can neither change
// status nor hold a link. One workgroup (1024 threads in 2D, 512 in 3D, so
// that the per-link work is spread wide without register spills).


// Sum of the 20 record terms over the block: every row of 16 lanes sums its
// lanes (row_sum16), the row totals go to LDS, and one wavefront per term
// adds them (wave_sum) -- all in a fixed order. sm holds N * NT / 16
// doubles. In 2D only Fx, Fy, Tz of each group (and the two counts) can be
// non-zero; the others are written as zero.
template <int NT, int D>
__device__ __forceinline__ void block_sum_ft(double v[20], double* out, double* sm) {
  constexpr int K2[11] = {0, 1, 5, 6, 7, 11, 12, 13, 17, 18, 19};
  constexpr int N = D == 2 ? 11 : 20;
  constexpr int ROWS = NT / 16;
  static_assert(ROWS <= 64, "one wavefront adds the row totals of a term");
  const int lane = threadIdx.x & 63, row = threadIdx.x >> 4;
  if (threadIdx.x < 20) out[threadIdx.x] = 0.0;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const double x = row_sum16(v[D == 2 ? K2[j] : j]);
    if ((threadIdx.x & 15) == 15) sm[j * ROWS + row] = x;
  }
  __syncthreads();
  for (int j = (int)(threadIdx.x >> 6); j < N; j += NT / 64) {
    const double t = wave_sum(lane < ROWS ? sm[j * ROWS + lane] : 0.0);
    if (lane == 0) out[D == 2 ? K2[j] : j] = t;
  }
  __syncthreads();
}

// The node box of a body at two poses (the region of its advance), when the
// caller knows it: the kernel then reads the node status without waiting
// for the poses.
struct StepBox {
  int lo[3], n[3];
};

template <class L, class S, int EQ, int NT, bool BOX>
__device__ __forceinline__ void body_step(typename S::T* B, uint8_t* mask, Link* links, int* n_links, int cap,
                                          const double* pose, const BodyShape& bs, int bc, int body, const Geom& g,
                                          const Phys& ph, double* rec_t, double* rec_t1, int* err, StepBox box) {
  extern __shared__ uint8_t lds[];  // status box: [0,total) at t, [total,2 total) at t+1
  __shared__ double red[20];
  __shared__ int scan_sm[NT / 64 + 1];
  // per region row: x-windows; once the list is built, the LDS list of
  // uncovered nodes, then the block sum's row totals
  __shared__ __align__(16) int16_t win[STEP_ROWS][4];
  __shared__ int8_t nwin[STEP_ROWS];
  __shared__ uint16_t rowoff[STEP_ROWS + 1];  // first list entry of each row
  __shared__ uint32_t list[STEP_LIST];        // window nodes (x - R.lo[0]) | row << 16
  __shared__ uint32_t linfo[STEP_LINKS];      // links of the new pose: list entry << 8 | direction
  __shared__ int list_n;
  static_assert(STEP_ROWS * 8 >= (L::D == 2 ? 11 : 20) * (NT / 16) * 8, "row totals fit the window table");
  static_assert(STEP_ROWS * 4 >= STEP_LIST, "uncovered-node list fits the window table");
  const Pose P0 = reinterpret_cast<const Pose*>(pose)[0];
  const Pose P1 = reinterpret_cast<const Pose*>(pose)[1];
  const uint8_t self = (uint8_t)(MASK_BODY0 + body);
  Region R, E;
  for (int a = 0; a < 3; ++a) {
    if (BOX) {
      R.lo[a] = box.lo[a];
      R.n[a] = box.n[a];
    } else {
      const int lo = (int)(P0.lo[a] < P1.lo[a] ? P0.lo[a] : P1.lo[a]);
      const int hi = (int)(P0.hi[a] > P1.hi[a] ? P0.hi[a] : P1.hi[a]);
      R.lo[a] = lo;
      R.n[a] = hi - lo + 1;
    }
    const int lo = R.lo[a];
    const int m = a < L::D ? 1 : 0;
    E.lo[a] = lo - m;
    E.n[a] = R.n[a] + 2 * m;
  }
  const int total = E.n[0] * E.n[1] * E.n[2];
  const int nrow = R.n[1] * R.n[2];
#define STEP_STATUS(x, y, z, nw) \
  lds[(nw) * total + ((x) - E.lo[0]) + E.n[0] * (((y) - E.lo[1]) + E.n[1] * ((z) - E.lo[2]))]

  // status box at t, copied with 4-byte loads (every box row starts at the
  // same offset modulo 4, since row and plane pitches are multiples of 16)
  {
    const int64_t c00 = g.idx(E.lo[0], E.lo[1], E.lo[2]);
    const int off = (int)(c00 & 3);
    const int wpr = (off + E.n[0] + 3) >> 2;  // words per box row
    const int nrE = E.n[1] * E.n[2];
    const int words = wpr * nrE;
    for (int w0 = 0; w0 < words; w0 += 4 * NT) {
      uint32_t v[4];
      int64_t base[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        int w = w0 + j * NT + threadIdx.x;
        w = w < words ? w : 0;
        const int r = w / wpr, wi = w - r * wpr;
        const int y = E.lo[1] + r % E.n[1], z = E.lo[2] + r / E.n[1];
        base[j] = g.idx(E.lo[0], y, z) - off + 4 * wi;
        v[j] = *reinterpret_cast<const uint32_t*>(mask + base[j]);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int w = w0 + j * NT + threadIdx.x;
        if (w >= words) break;
        const int r = w / wpr, wi = w - r * wpr;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int x = 4 * wi + b - off;
          if (x >= 0 && x < E.n[0]) {
            const uint8_t st = (uint8_t)(v[j] >> (8 * b));
            lds[r * E.n[0] + x] = st;
            lds[total + r * E.n[0] + x] = st;
          }
        }
      }
    }
  }
  // windows of every region row (rows r0 .. r1-1 of this thread, in thread
  // order); the list is laid out in row order, window order, x order, and
  // filled one entry per thread
  int r0, r1, my_cells = 0;
  if constexpr (L::D == 2) {
    // a group of 8 lanes per row: lane j < 6 takes the chord of row y + j%3 - 1
    // at pose j/3, and the group combines them (min / max are exact, so the
    // windows are those of row_windows)
    constexpr int GW = 8;
    const int j = threadIdx.x & (GW - 1), rpg = (nrow + NT / GW - 1) / (NT / GW);
    const int g0 = (threadIdx.x / GW) * rpg, g1 = g0 + rpg < nrow ? g0 + rpg : nrow;
    for (int r = g0; r < g1; ++r) {
      RowExtent e;
      if (j < 6) {
        double a = 0, bb = 0;
        const bool hit = row_chord(bs, j < 3 ? P0 : P1, R.lo[1] + r + j % 3 - 1, R.lo[2], a, bb);
        e.add(hit, a, bb);
      }
      int flags = (e.any ? 1 : 0) | (e.gap ? 2 : 0);
#pragma unroll
      for (int o = GW / 2; o > 0; o >>= 1) {
        e.amin = fmin(e.amin, __shfl_xor(e.amin, o, GW));
        e.amax = fmax(e.amax, __shfl_xor(e.amax, o, GW));
        e.bmin = fmin(e.bmin, __shfl_xor(e.bmin, o, GW));
        e.bmax = fmax(e.bmax, __shfl_xor(e.bmax, o, GW));
        flags |= __shfl_xor(flags, o, GW);
      }
      e.any = flags & 1;
      e.gap = (flags & 2) != 0;
      if (j == 0) {
        int w[4] = {0, -1, 0, -1};
        const int n = windows_of(e, 2, R.lo[0], R.lo[0] + R.n[0] - 1, w);
        nwin[r] = (int8_t)n;
#pragma unroll
        for (int q = 0; q < 4; ++q) win[r][q] = (int16_t)w[q];
        if (n > 0) my_cells += w[1] - w[0] + 1;
        if (n > 1) my_cells += w[3] - w[2] + 1;
      }
    }
    r0 = j == 0 ? g0 : 0;
    r1 = j == 0 ? g1 : 0;
  } else {
    const int rchunk = (nrow + NT - 1) / NT;
    r0 = threadIdx.x * rchunk;
    r1 = r0 + rchunk < nrow ? r0 + rchunk : nrow;
    for (int r = r0; r < r1; ++r) {
      int w[4] = {0, -1, 0, -1};
      const int n = row_windows(bs, P0, P1, R.lo[1] + r % R.n[1], R.lo[2] + r / R.n[1], L::D, 2, R.lo[0],
                                R.lo[0] + R.n[0] - 1, w);
      nwin[r] = (int8_t)n;
#pragma unroll
      for (int q = 0; q < 4; ++q) win[r][q] = (int16_t)w[q];
      if (n > 0) my_cells += w[1] - w[0] + 1;
      if (n > 1) my_cells += w[3] - w[2] + 1;
    }
  }
  int lbase = block_exclusive_scan<NT>(my_cells, scan_sm);
  const int list_total = scan_sm[NT / 64];
  if (threadIdx.x == 0) {
    list_n = list_total;
    if (list_total > STEP_LIST) atomicOr(err, 4);
    rowoff[nrow] = (uint16_t)(list_total < STEP_LIST ? list_total : STEP_LIST);
  }
  for (int r = r0; r < r1; ++r) {
    rowoff[r] = (uint16_t)(lbase < STEP_LIST ? lbase : STEP_LIST);
    if (nwin[r] > 0) lbase += win[r][1] - win[r][0] + 1;
    if (nwin[r] > 1) lbase += win[r][3] - win[r][2] + 1;
  }
  __syncthreads();
  const int nlist = list_n < STEP_LIST ? list_n : STEP_LIST;
  for (int e = threadIdx.x; e < nlist; e += NT) {
    int lo = 0, hi = nrow - 1;  // last row whose first entry is <= e
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if ((int)rowoff[mid] <= e) lo = mid;
      else hi = mid - 1;
    }
    const int o = e - (int)rowoff[lo];
    const int len0 = win[lo][1] - win[lo][0] + 1;
    const int x = o < len0 ? win[lo][0] + o : win[lo][2] + (o - len0);
    list[e] = (uint32_t)(x - R.lo[0]) | ((uint32_t)lo << 16);
  }
  __syncthreads();
  auto node = [&](int k, int& x, int& y, int& z) {
    const uint32_t e = list[k];
    const int r = (int)(e >> 16);
    x = R.lo[0] + (int)(e & 0xffff);
    y = R.lo[1] + r % R.n[1];
    z = R.lo[2] + r / R.n[1];
  };
  double imp[8] = {0, 0, 0, 0, 0, 0, 0, 0};

  // phase A: new status of the listed nodes, momentum of covered ones
  for (int k = threadIdx.x; k < nlist; k += NT) {
    int x, y, z;
    node(k, x, y, z);
    const uint8_t old = STEP_STATUS(x, y, z, 0);
    const bool solid = shape_phi(bs, P1, (double)x, (double)y, (double)z) <= 0.0;
    if (old != MASK_FLUID && old != self) {
      if (solid) atomicOr(err, 2);
      continue;
    }
    const uint8_t nw = solid ? self : MASK_FLUID;
    if (nw == old) continue;
    STEP_STATUS(x, y, z, 1) = nw;
    const int64_t c = g.idx(x, y, z);
    mask[c] = nw;
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
  }
  __syncthreads();

  // phase B: over contiguous runs of the list (node order), the links of the
  // new pose (to the global list, in node order) and the uncovered nodes (to
  // an LDS list), counted together by one scan (links in the low half)
  uint16_t* uncovered = reinterpret_cast<uint16_t*>(&win[0][0]);
  const int kchunk = (nlist + NT - 1) / NT;
  const int k0 = threadIdx.x * kchunk;
  const int k1 = k0 + kchunk < nlist ? k0 + kchunk : nlist;
  int my_links = 0, my_unc = 0;
  for (int k = k0; k < k1; ++k) {
    int x, y, z;
    node(k, x, y, z);
    if (STEP_STATUS(x, y, z, 1) != MASK_FLUID) continue;
    if (STEP_STATUS(x, y, z, 0) == self) my_unc++;
#pragma unroll
    for (int i = 1; i < L::Q; ++i)
      if (STEP_STATUS(x - L::cx(i), y - L::cy(i), z - L::cz(i), 1) == self) my_links++;
  }
  const int packed = block_exclusive_scan<NT>(my_links | (my_unc << 16), scan_sm);
  const int nlinks = scan_sm[NT / 64] & 0xffff, n_unc = scan_sm[NT / 64] >> 16;
  int base = packed & 0xffff, ubase = packed >> 16;
  for (int k = k0; k < k1; ++k) {
    int x, y, z;
    node(k, x, y, z);
    if (STEP_STATUS(x, y, z, 1) != MASK_FLUID) continue;
    if (STEP_STATUS(x, y, z, 0) == self) uncovered[ubase++] = (uint16_t)k;
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
      if (STEP_STATUS(x - L::cx(i), y - L::cy(i), z - L::cz(i), 1) != self) continue;
      if (base < STEP_LINKS) {
        linfo[base] = ((uint32_t)k << 8) | (uint32_t)i;
      } else if (base < cap) {  // beyond the LDS list: through global memory
        Link lk;
        lk.cell = (int32_t)g.idx(x, y, z);
        lk.x = (int16_t)x;
        lk.y = (int16_t)y;
        lk.z = (int16_t)z;
        lk.dir = (int16_t)i;
        lk.delta = 0.5;
        links[base] = lk;
      }
      base++;
    }
  }
  if (threadIdx.x == 0) {
    *n_links = nlinks < cap ? nlinks : cap;
    if (nlinks > cap) atomicOr(err, 1);
  }
  __syncthreads();

  // refill of the uncovered nodes with the equilibrium at the mean density
  // and velocity of their neighbours fluid at t and t+1 (the wall velocity
  // when there are none): a group of G lanes per node, lane j reading the
  // moments of neighbour j + 1, so that all neighbours are read at once;
  // the group sums them with a fixed shuffle tree
  {
    constexpr int G = L::Q - 1 <= 8 ? 8 : 32;
    const int j = threadIdx.x & (G - 1);
    for (int u = threadIdx.x / G; u < n_unc; u += NT / G) {
      int x, y, z;
      node(uncovered[u], x, y, z);
      double v[5] = {0, 0, 0, 0, 0};  // density, velocity, count
      if (j + 1 < L::Q) {
        const Dir<L> d = dir_of<L>(j + 1);
        const int xn = x + d.cx, yn = y + d.cy, zn = z + d.cz;
        if (STEP_STATUS(xn, yn, zn, 0) == MASK_FLUID && STEP_STATUS(xn, yn, zn, 1) == MASK_FLUID) {
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
      // beyond the status box a node keeps its status (the global mask)
      auto fluid_both = [&](int xa, int ya, int za) {
        if (!E.contains(xa, ya, za)) return mask[g.idx(xa, ya, za)] == MASK_FLUID;
        return STEP_STATUS(xa, ya, za, 0) == MASK_FLUID && STEP_STATUS(xa, ya, za, 1) == MASK_FLUID;
      };
      const double us[3] = {v[1], v[2], v[3]};
      refill_node<L, S, EQ>(B, g, ph, P0, P1, bs, x, y, z, v[0], us, v[4], fluid_both, imp);
    }
  }
  __syncthreads();

  // phase C: Delta, boundary rule and momentum exchange of step t+1, one
  // link per thread; the status of x_F + c_i comes from the status box. The
  // link list of the new pose is written out here, with its Delta.
  const int nl = nlinks < cap ? nlinks : cap;
  double acc[20];
#pragma unroll
  for (int k = 0; k < 20; ++k) acc[k] = 0.0;
  for (int k = threadIdx.x; k < nl; k += NT) {
    Link lk;
    if (k < STEP_LINKS) {
      const uint32_t e = linfo[k];
      int x, y, z;
      node((int)(e >> 8), x, y, z);
      lk.cell = (int32_t)g.idx(x, y, z);
      lk.x = (int16_t)x;
      lk.y = (int16_t)y;
      lk.z = (int16_t)z;
      lk.dir = (int16_t)(e & 0xff);
    } else {
      lk = links[k];
    }
    const Dir<L> d = dir_of<L>(lk.dir);
    lk.delta = bc ? link_delta(bs, P1, (double)lk.x, (double)lk.y, (double)lk.z, d.cx, d.cy, d.cz) : 0.5;
    const bool nb = STEP_STATUS(lk.x + d.cx, lk.y + d.cy, lk.z + d.cz, 1) == MASK_FLUID;
    link_rule<L, S, EQ>(B, lk, P1, bc, nb, g, ph, acc);
    links[k] = lk;
  }
#undef STEP_STATUS
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[12 + k] = imp[k];
  block_sum_ft<NT, L::D>(acc, red, reinterpret_cast<double*>(&win[0][0]));
  if (threadIdx.x < 20) {
    const int k = threadIdx.x;
    const double v = red[k];
    if (k < 6) rec_t1[k] = v;
    else if (k < 12) rec_t1[k + 6] = v;
    else if (k < 18) rec_t[k - 6] = v;
    else rec_t[k] = v;
    if (k < 6) rec_t1[6 + k] = 0.0;
    if (k < 2) rec_t1[18 + k] = 0.0;
  }
}

template <class L, class S, int EQ, int NT>
__global__ __launch_bounds__(NT) void k_body_step(typename S::T* B, uint8_t* mask, Link* links, int* n_links,
                                                  int cap, const double* pose, BodyShape bs, int bc, int body,
                                                  Geom g, Phys ph, double* rec_t, double* rec_t1, int* err,
                                                  StepBox box) {
  body_step<L, S, EQ, NT, true>(B, mask, links, n_links, cap, pose, bs, bc, body, g, ph, rec_t, rec_t1, err, box);
}

// the same for a body whose poses only the device knows (FREE motion): the
// region comes from the two poses
template <class L, class S, int EQ, int NT>
__global__ __launch_bounds__(NT) void k_body_step_free(typename S::T* B, uint8_t* mask, Link* links, int* n_links,
                                                       int cap, const double* pose, BodyShape bs, int bc, int body,
                                                       Geom g, Phys ph, double* rec_t, double* rec_t1, int* err) {
  body_step<L, S, EQ, NT, false>(B, mask, links, n_links, cap, pose, bs, bc, body, g, ph, rec_t, rec_t1, err,
                                 StepBox{});
}

}  // namespace lbm
#include "wide.hpp"
namespace lbm {

// Node terms of a free body over the covered and uncovered nodes between
// its pose t and the predicted pose X + V, theta + Omega (cos/sin by
// free_trig), on the state of t+1, written to out[0..5]: one workgroup
// scans the node box of pose t (it holds both bodies and the layer around
// them, the body moving less than a node per step); statuses at the
// predicted pose come from the shape inside the box and from the mask
// beyond it. The refill rule of the body gives the uncovered nodes' values
// (computed, not stored).
template <class L, class S, int EQ>
__global__ __launch_bounds__(ADV_BLOCK) void k_body_predict(const typename S::T* B, const uint8_t* mask,
                                                            const double* pose, BodyShape bs, int body, Geom g,
                                                            Phys ph, double* out) {
#pragma clang fp contract(off)
  __shared__ double sm[6 * ADV_BLOCK / 64];
  __shared__ double red[6];
  const Pose P = reinterpret_cast<const Pose*>(pose)[0];
  Pose Pp = P;
  for (int a = 0; a < 3; ++a) Pp.X[a] = P.X[a] + P.V[a];
  Pp.theta = P.theta + P.Om;
  free_trig(Pp.theta, Pp.ct, Pp.st);
  const uint8_t self = (uint8_t)(MASK_BODY0 + body);
  Region R;
  for (int a = 0; a < 3; ++a) {
    R.lo[a] = (int)P.lo[a];
    R.n[a] = (int)P.hi[a] - (int)P.lo[a] + 1;
  }
  R.total = (int64_t)R.n[0] * R.n[1] * R.n[2];
  auto next = [&](int x, int y, int z) -> uint8_t {  // status at the predicted pose
    const uint8_t m = mask[g.idx(x, y, z)];
    if (!R.contains(x, y, z) || (m != MASK_FLUID && m != self)) return m;
    return shape_phi(bs, Pp, (double)x, (double)y, (double)z) <= 0.0 ? self : (uint8_t)MASK_FLUID;
  };
  auto fluid_both = [&](int x, int y, int z) {
    return mask[g.idx(x, y, z)] == MASK_FLUID && next(x, y, z) == MASK_FLUID;
  };
  double imp[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t k = threadIdx.x; k < R.total; k += ADV_BLOCK) {
    int x, y, z;
    R.at(k, x, y, z);
    const int64_t c = g.idx(x, y, z);
    const uint8_t old = mask[c];
    if (old != MASK_FLUID && old != self) continue;
    const bool will = shape_phi(bs, Pp, (double)x, (double)y, (double)z) <= 0.0;
    if (old == MASK_FLUID && will) {  // covered
      double m[3] = {0, 0, 0};
#pragma unroll
      for (int q = 1; q < L::Q; ++q) {
        const double v = (double)S::load(B + q * g.S + c);
        m[0] += L::cx(q) * v;
        m[1] += L::cy(q) * v;
        m[2] += L::cz(q) * v;
      }
      const double r[3] = {x - P.X[0], y - P.X[1], z - P.X[2]};
      imp[0] += m[0];
      imp[1] += m[1];
      imp[2] += m[2];
      imp[3] += r[1] * m[2] - r[2] * m[1];
      imp[4] += r[2] * m[0] - r[0] * m[2];
      imp[5] += r[0] * m[1] - r[1] * m[0];
    } else if (old == self && !will) {  // uncovered
      double rs = 0, us[3] = {0, 0, 0}, cnt = 0;
#pragma unroll
      for (int q = 1; q < L::Q; ++q) {
        const int xn = x + L::cx(q), yn = y + L::cy(q), zn = z + L::cz(q);
        if (!fluid_both(xn, yn, zn)) continue;
        double hn[L::Q], dn, un[3];
        moments_at<L, S>(B, g, g.idx(xn, yn, zn), ph.rho0, EQ, hn, dn, un);
        rs += ph.rho0 + dn;
        us[0] += un[0];
        us[1] += un[1];
        us[2] += un[2];
        cnt += 1.0;
      }
      refill_node<L, S, EQ, false>(const_cast<typename S::T*>(B), g, ph, P, Pp, bs, x, y, z, rs, us, cnt, fluid_both,
                                   imp);
    }
  }
  block_sum<6, ADV_BLOCK>(imp, red, sm);
  if (threadIdx.x < 6) out[threadIdx.x] = red[threadIdx.x];
}

// ---------------------------------------------------------------------------
// batches: many domains per launch; every argument that differs between
// domains comes from a device table, the batch step s from the launch

__device__ __forceinline__ double* batch_rec(const BatchBody& b, int64_t t) {
  return b.rec + (t % b.rec_cap) * b.rec_stride;
}

// part 0: tile rows of every node; 1: the same without the members' near
// boxes; 2: tiles of the near boxes (rows numbered within the box)
template <class L, class S, int EQ, int BX, int CPT, int MEM, bool BUF>
__global__ __launch_bounds__(BX) void k_stream_collide_batch(const BatchDomain* __restrict__ doms,
                                                             const BatchTile* __restrict__ tiles, int ntiles,
                                                             int remap, int64_t s, int part,
                                                             const int64_t* __restrict__ sbase, int flat) {
  s += sbase ? *sbase : 0;  // a captured step sequence takes its first step from the device
  const int blk = remap ? xcd_block(blockIdx.x, ntiles) : blockIdx.x;
  const BatchTile tl = tiles[blk];
  const BatchDomain& D = doms[tl.dom];
  const Geom g = D.g;
  const Phys ph = D.ph;
  using C = typename S::C;
  const auto* A = (const typename S::T*)D.buf[s & 1];
  auto* B = (typename S::T*)D.buf[(s + 1) & 1];
  const auto* rin = (const C*)D.rho[s & 1];
  auto* rout = (C*)D.rho[(s + 1) & 1];
  const int no_hole[6] = {1, 0, 1, 0, 1, 0};
  if (part == 2) {
    const int nrows = D.hole[3] - D.hole[2] + 1;
    const int y = D.hole[2] + tl.row % nrows;
    const int z = D.hole[4] + tl.row / nrows;
    stream_collide_span<L, S, EQ, BX, CPT, MEM, BUF>(A, B, g, ph, D.hole[0] + tl.bx * (BX * CPT) + threadIdx.x, y,
                                                     z, D.hole[1], no_hole, rin, rout, D.mask, D.unstable);
    return;
  }
  const int nrows = g.hi[1] - g.lo[1] + 1;
  if (flat) {  // node tl.row + t of the member's active nodes (x fastest); past the last one: no update
    const int nxa = g.hi[0] - g.lo[0] + 1;
    const int64_t total = (int64_t)nxa * nrows * (g.hi[2] - g.lo[2] + 1);
    const int64_t f = (int64_t)tl.row + threadIdx.x;
    const int ff = (int)(f < total ? f : total - 1);
    const int r = ff / nxa;
    const int x = f < total ? g.lo[0] + (ff - r * nxa) : g.hi[0] + 1;
    stream_collide_span<L, S, EQ, BX, 1, MEM, BUF>(A, B, g, ph, x, g.lo[1] + r % nrows, g.lo[2] + r / nrows, g.hi[0],
                                                 part == 1 ? D.hole : no_hole, rin, rout, D.mask, D.unstable);
    return;
  }
  const int y = g.lo[1] + tl.row % nrows;
  const int z = g.lo[2] + tl.row / nrows;
  stream_collide_span<L, S, EQ, BX, CPT, MEM, BUF>(A, B, g, ph, g.lo[0] + tl.bx * (BX * CPT) + threadIdx.x, y, z,
                                                   g.hi[0], part == 1 ? D.hole : no_hole, rin, rout, D.mask,
                                                   D.unstable);
}

// grid (blocks per body, bodies), NTL threads per block: the boundary rule +
// momentum exchange of batch step s before its bulk update, on the source
// buffer
template <class L, class S, int EQ, int NTL>
__global__ __launch_bounds__(NTL) void k_links_batch(const BatchDomain* __restrict__ doms,
                                                     const BatchBody* __restrict__ bodies, int64_t s,
                                                     const int64_t* __restrict__ sbase) {
  s += sbase ? *sbase : 0;
  const BatchBody& b = bodies[blockIdx.y];
  const BatchDomain& D = doms[b.dom];
  const int64_t t = b.t0 + s;
  links_block<L, S, EQ, NTL>((typename S::T*)D.buf[s & 1], b.links, b.n_host, b.pose + (t - b.pose_base) * POSE_DOUBLES,
                        b.bc, b.mask, D.g, D.ph, b.partials, b.counter, batch_rec(b, t), blockIdx.x, gridDim.x);
}

// The link rule of batch step s in two launches, without a grid-wide
// handshake: k_links_batch_part writes every chunk's 12 sums (as the waves of
// links_block do), k_fold_batch adds them per body in the order of
// links_block's last block, so the records are the same bits. Used in 3D,
// where a body's links span many workgroups (a device-scope fence per
// workgroup costs far more than the second launch).
template <class L, class S, int EQ>
__global__ __launch_bounds__(64) void k_links_batch_part(const BatchDomain* __restrict__ doms,
                                                         const BatchBody* __restrict__ bodies, int64_t s,
                                                         const int64_t* __restrict__ sbase) {
  s += sbase ? *sbase : 0;
  const BatchBody& b = bodies[blockIdx.y];
  const int c = (int)blockIdx.x;  // chunk of 64 links
  if (c * 64 >= b.n_host) return;
  const BatchDomain& D = doms[b.dom];
  const int64_t t = b.t0 + s;
  const Pose P = *reinterpret_cast<const Pose*>(b.pose + (t - b.pose_base) * POSE_DOUBLES);
  const int lane = threadIdx.x;
  __shared__ double sm[12 * 64 + 48];
  double acc[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  const int k = c * 64 + lane;
  if (k < b.n_host) link_rule_m<L, S, EQ>((typename S::T*)D.buf[s & 1], b.links[k], P, b.bc, b.mask, D.g, D.ph, acc);
  const double v = wave_sums_lds<12>(acc, sm);  // the bits of wave_sum, lane j value j
  if (lane < 12) b.partials[c * 12 + lane] = v;
}

template <class L>
__global__ __launch_bounds__(64) void k_fold_batch(const BatchBody* __restrict__ bodies, int64_t s,
                                                   const int64_t* __restrict__ sbase) {
  s += sbase ? *sbase : 0;
  const BatchBody& b = bodies[blockIdx.x];
  const int lane = threadIdx.x;
  const int nchunks = (b.n_host + 63) >> 6;
  double acc[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int c = lane; c < nchunks; c += 64)
#pragma unroll
    for (int j = 0; j < 12; ++j) acc[j] += b.partials[c * 12 + j];
  double* rec = batch_rec(b, b.t0 + s);
#pragma unroll
  for (int j = 0; j < 12; ++j) {
    const double v = wave_sum(acc[j]);
    if (lane == j) rec[j < 6 ? j : j + 6] = v;  // static -> 0..5, comoving -> 12..17
  }
  if (lane >= 12 && lane < 18) rec[lane - 6] = 0.0;  // node terms 6..11
  if (lane >= 18 && lane < 20) rec[lane] = 0.0;      // counts 18, 19
}

// one workgroup per moving body: its advance after batch step s's bulk update
template <class L, class S, int EQ, int NT>
__global__ __launch_bounds__(NT) void k_body_step_batch(const BatchDomain* __restrict__ doms,
                                                        const BatchBody* __restrict__ bodies, int64_t s,
                                                        const int64_t* __restrict__ sbase) {
  s += sbase ? *sbase : 0;
  const BatchBody& b = bodies[blockIdx.x];
  const BatchDomain& D = doms[b.dom];
  const int64_t t = b.t0 + s;
  body_step<L, S, EQ, NT, false>((typename S::T*)D.buf[(s + 1) & 1], b.mask, b.links, b.n_links, b.cap,
                                 b.pose + (t - b.pose_base) * POSE_DOUBLES, b.bs, b.bc, b.body, D.g, D.ph,
                                 batch_rec(b, t), batch_rec(b, t + 1), b.err, StepBox{});
}

// After batch step s's bulk update, one launch for all the body work that
// follows it: blocks [0, n_moving) advance the moving bodies (as
// k_body_step_batch), the others apply the link rule of step s+1 for the
// bodies with fixed links (as k_links_batch, one workgroup per body). That
// rule reads the new state only within two nodes of its body, inside the
// body's near box, so it may run beside the far update of step s.
template <class L, class S, int EQ, int NT>
__global__ __launch_bounds__(NT) void k_body_links_batch(const BatchDomain* __restrict__ doms,
                                                         const BatchBody* __restrict__ moving, int n_moving,
                                                         const BatchBody* __restrict__ fixed, int64_t s,
                                                         const int64_t* __restrict__ sbase) {
  s += sbase ? *sbase : 0;
  if ((int)blockIdx.x < n_moving) {
    const BatchBody& b = moving[blockIdx.x];
    const BatchDomain& D = doms[b.dom];
    const int64_t t = b.t0 + s;
    body_step<L, S, EQ, NT, false>((typename S::T*)D.buf[(s + 1) & 1], b.mask, b.links, b.n_links, b.cap,
                                   b.pose + (t - b.pose_base) * POSE_DOUBLES, b.bs, b.bc, b.body, D.g, D.ph,
                                   batch_rec(b, t), batch_rec(b, t + 1), b.err, StepBox{});
    return;
  }
  const BatchBody& b = fixed[blockIdx.x - n_moving];
  const BatchDomain& D = doms[b.dom];
  const int64_t t = b.t0 + s + 1;
  links_block<L, S, EQ, NT>((typename S::T*)D.buf[(s + 1) & 1], b.links, b.n_host,
                            b.pose + (t - b.pose_base) * POSE_DOUBLES, b.bc, b.mask, D.g, D.ph, b.partials, b.counter,
                            batch_rec(b, t), 0, 1);
}

// the many-workgroup advance of the bodies of a batch after batch step s:
// workgroup (x, y) is slab x of body y
template <class L, class S, int EQ>
__global__ __launch_bounds__(WIDE_BLOCK) void k_wide_sets_batch(const BatchDomain* __restrict__ doms,
                                                                const BatchBody* __restrict__ bodies, int64_t s,
                                                                const int64_t* __restrict__ sbase) {
  s += sbase ? *sbase : 0;
  const BatchBody& b = bodies[blockIdx.y];
  const BatchDomain& D = doms[b.dom];
  const int64_t t = b.t0 + s;
  wide_sets<L, S, EQ>((typename S::T*)D.buf[(s + 1) & 1], b.mask, b.pose + (t - b.pose_base) * POSE_DOUBLES, b.bs,
                      b.body, D.g, D.ph, b.wide, b.wide_slabs, b.err, (int)blockIdx.x);
}

template <class L, class S, int EQ>
__global__ __launch_bounds__(WIDE_BLOCK) void k_wide_links_batch(const BatchDomain* __restrict__ doms,
                                                                 const BatchBody* __restrict__ bodies, int64_t s,
                                                                 const int64_t* __restrict__ sbase) {
  s += sbase ? *sbase : 0;
  const BatchBody& b = bodies[blockIdx.y];
  const BatchDomain& D = doms[b.dom];
  const int64_t t = b.t0 + s;
  wide_links<L, S, EQ>((typename S::T*)D.buf[(s + 1) & 1], b.mask, b.links, b.n_links, b.cap,
                       b.pose + (t - b.pose_base) * POSE_DOUBLES, b.bs, b.bc, b.body, D.g, D.ph, b.wide,
                       b.wide_slabs, batch_rec(b, t), batch_rec(b, t + 1), b.err, (int)blockIdx.x);
}

// ---------------------------------------------------------------------------
// launches for one (lattice, storage, equilibrium); instantiated once per
// lattice and storage in the inst_*.hip sources

template <class K, class... Args>
static void launch_timed(K kern, dim3 grid, dim3 block, size_t lds, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                         Args... args) {
  if (e0 || e1) hipExtLaunchKernelGGL(kern, grid, block, (uint32_t)lds, s, e0, e1, 0, args...);
  else hipLaunchKernelGGL(kern, grid, block, lds, s, args...);
}

template <class L, class S, int EQ, int BX, int CPT, int MEM>
static void launch_bulk_variant(const void* A, void* B, const Geom& g, const Phys& ph, const Sweep& sw,
                                hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const auto* a = (const typename S::T*)A;
  auto* o = (typename S::T*)B;
  // raw buffer accesses whenever a population buffer is below 4 GiB
  const bool buf = (uint64_t)L::Q * g.S * sizeof(typename S::T) < ((uint64_t)1 << 32);
  if (buf) launch_timed(k_stream_collide<L, S, EQ, BX, CPT, MEM, true>, dim3(sw.ntiles), dim3(BX), 0, s, e0, e1, a, o,
                        g, ph, sw);
  else launch_timed(k_stream_collide<L, S, EQ, BX, CPT, MEM, false>, dim3(sw.ntiles), dim3(BX), 0, s, e0, e1, a, o,
                    g, ph, sw);
}

template <class L, class S, int EQ>
void Ops<L, S, EQ>::stream_collide(const BulkConfig& c, const void* A, void* B, const Geom& g, const Phys& ph,
                                   const Sweep& sw, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
#define LBM_BULK_CASE(BX_, CPT_)                                                                    \
  if (c.block == BX_ && c.cells_per_thread == CPT_) {                                               \
    switch (c.nontemporal) {                                                                        \
      case 0: return launch_bulk_variant<L, S, EQ, BX_, CPT_, 0>(A, B, g, ph, sw, s, e0, e1);       \
      case 1: return launch_bulk_variant<L, S, EQ, BX_, CPT_, 1>(A, B, g, ph, sw, s, e0, e1);       \
      case 2: return launch_bulk_variant<L, S, EQ, BX_, CPT_, 2>(A, B, g, ph, sw, s, e0, e1);       \
      default: return launch_bulk_variant<L, S, EQ, BX_, CPT_, 3>(A, B, g, ph, sw, s, e0, e1);      \
    }                                                                                               \
  }
  LBM_BULK_CASE(256, 1)
  LBM_BULK_CASE(256, 2)
  LBM_BULK_CASE(128, 2)
#undef LBM_BULK_CASE
}

template <class L, class S, int EQ>
void Ops<L, S, EQ>::init(void* A, uint8_t* mask, const Geom& g, const Phys& ph, const double* rho, const double* u,
                         void* rho_out, hipStream_t s) {
  BulkShape b = bulk_shape(g, BULK_BLOCK);
  hipLaunchKernelGGL((k_init<L, S, EQ>), dim3(b.nbx, b.nrows, b.nplanes), dim3(BULK_BLOCK), 0, s,
                     (typename S::T*)A, mask, g, ph, rho, u, (typename S::C*)rho_out);
}

template <class L, class S, int EQ>
void Ops<L, S, EQ>::links(void* A, const Link* links, int n_host, const int* n_dev, int grid, const double* pose,
                          int bc, const uint8_t* mask, const Geom& g, const Phys& ph, double* partials,
                          unsigned* counter, double* rec, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  launch_timed(k_links<L, S, EQ>, dim3(grid), dim3(LINK_BLOCK), 0, s, e0, e1, (typename S::T*)A, links, n_host,
               n_dev, pose, bc, mask, g, ph, partials, counter, rec);
}

template <class L, class S, int EQ>
void Ops<L, S, EQ>::links_part(void* A, const Link* links, int n, const double* pose, int bc, const uint8_t* mask,
                               const Geom& g, const Phys& ph, double* part, hipStream_t s, hipEvent_t e0,
                               hipEvent_t e1) {
  const int chunks = n > 0 ? (n + 63) / 64 : 1;
  launch_timed(k_links_part<L, S, EQ>, dim3(chunks), dim3(64), 0, s, e0, e1, (typename S::T*)A, links, n, pose,
               bc, mask, g, ph, part);
}

template <class L, class S, int EQ>
void Ops<L, S, EQ>::face_part(const void* A, const Geom& g, const Phys& ph, const void* rho_in, int nnodes,
                              double* part, hipStream_t s) {
  hipLaunchKernelGGL((k_face_part<L, S, EQ>), dim3((unsigned)((nnodes + 255) / 256)), dim3(256), 0, s,
                     (const typename S::T*)A, g, ph, (const typename S::C*)rho_in, nnodes, part);
}

template <class L, class S, int EQ>
void Ops<L, S, EQ>::poison_body(void* A, void* B, const uint8_t* mask, const Geom& g, const int lo[3], const int hi[3],
                                int body, hipStream_t s) {
  const int n0 = hi[0] - lo[0] + 1, n1 = hi[1] - lo[1] + 1, n2 = hi[2] - lo[2] + 1;
  const int64_t total = (int64_t)n0 * n1 * n2;
  if (total <= 0) return;
  hipLaunchKernelGGL((k_poison_body<L, S>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     (typename S::T*)A, (typename S::T*)B, mask, g, lo[0], lo[1], lo[2], n0, n1, total,
                     (uint8_t)(MASK_BODY0 + body));
}

template <class L, class S, int EQ>
void Ops<L, S, EQ>::body_advance(void* B, uint8_t* mask, uint8_t* mask_next, Link* links, int* n_links, int cap,
                                 const double* pose, const double* pose_host, const BodyShape& bs, int bc, int body,
                                 int mode, const Geom& g, const Phys& ph, double* rec_t, double* rec_t1, int* err,
                                 hipStream_t s, int64_t region_cells, int64_t region_rows, int64_t list_nodes,
                                 double* wide, int wide_slabs, hipEvent_t e0, hipEvent_t e1) {
  auto* b = (typename S::T*)B;
  const size_t lds = ((size_t)2 * region_cells + 15) / 16 * 16;
  const bool fits = body_step_fits(region_cells, region_rows, list_nodes);
  if (mode == 1 && wide && bs.shape != SHAPE_OUTER_CIRCLE && !fits) {
    if (e0) (void)hipEventRecord(e0, s);
    hipLaunchKernelGGL((k_wide_sets<L, S, EQ>), dim3(wide_slabs), dim3(WIDE_BLOCK), 0, s, b, mask, pose, bs, body,
                       g, ph, wide, wide_slabs, err);
    hipLaunchKernelGGL((k_wide_links<L, S, EQ>), dim3(wide_slabs), dim3(WIDE_BLOCK), 0, s, b, mask, links, n_links,
                       cap, pose, bs, bc, body, g, ph, wide, wide_slabs, rec_t, rec_t1, err);
    if (e1) (void)hipEventRecord(e1, s);
  } else if (mode == 1 && !pose_host && bs.shape != SHAPE_OUTER_CIRCLE && fits) {
    constexpr int NT = L::D == 2 ? 1024 : 512;
    launch_timed(k_body_step_free<L, S, EQ, NT>, dim3(1), dim3(NT), lds, s, e0, e1, b, mask, links, n_links, cap,
                 pose, bs, bc, body, g, ph, rec_t, rec_t1, err);
  } else if (mode == 1 && bs.shape != SHAPE_OUTER_CIRCLE && fits) {
    constexpr int NT = L::D == 2 ? 1024 : 512;  // 2D fits the 128 VGPRs of 1024-thread blocks
    const Pose* P = reinterpret_cast<const Pose*>(pose_host);  // the same two poses, host copy
    StepBox box;
    for (int a = 0; a < 3; ++a) {
      const int lo = (int)(P[0].lo[a] < P[1].lo[a] ? P[0].lo[a] : P[1].lo[a]);
      const int hi = (int)(P[0].hi[a] > P[1].hi[a] ? P[0].hi[a] : P[1].hi[a]);
      box.lo[a] = lo;
      box.n[a] = hi - lo + 1;
    }
    launch_timed(k_body_step<L, S, EQ, NT>, dim3(1), dim3(NT), lds, s, e0, e1, b, mask, links, n_links, cap, pose,
                 bs, bc, body, g, ph, rec_t, rec_t1, err, box);
  } else if (region_cells > 0 && region_cells <= ADV_LDS_CELLS) {
    launch_timed(k_body_advance_lds<L, S, EQ>, dim3(1), dim3(ADV_BLOCK), lds, s, e0, e1, b, mask, links, n_links,
                 cap, pose, bs, bc, body, mode, g, ph, rec_t, rec_t1, err);
  } else {
    launch_timed(k_body_advance<L, S, EQ>, dim3(1), dim3(ADV_BLOCK), 0, s, e0, e1, b, mask, mask_next, links,
                 n_links, cap, pose, bs, bc, body, mode, g, ph, rec_t, rec_t1, err);
  }
}

template <class L, class S, int EQ>
void Ops<L, S, EQ>::body_predict(const void* B, const uint8_t* mask, const double* pose, const BodyShape& bs,
                                 int body, const Geom& g, const Phys& ph, double* out, hipStream_t s) {
  hipLaunchKernelGGL((k_body_predict<L, S, EQ>), dim3(1), dim3(ADV_BLOCK), 0, s, (const typename S::T*)B, mask, pose,
                     bs, body, g, ph, out);
}

template <class L, class S, int EQ>
void Ops<L, S, EQ>::batch_bulk(const BatchDomain* doms, const BatchTile* tiles, int ntiles, const BulkConfig& cfg,
                               int64_t step, hipStream_t s, int part, hipEvent_t e0, hipEvent_t e1,
                               const int64_t* sbase, int flat) {
  // buffer-resource accesses with 32-bit offsets, or plain global accesses
  // when a member's buffer is 4 GiB or more (plain memory mode either way:
  // non-temporal loads, the choice for a single D3Q19 domain beyond the
  // last-level cache, made the served mix of many small 3D members slower)
#define LBM_BATCH_LAUNCH(BX_, CPT_, BUF_)                                                                     \
  launch_timed(k_stream_collide_batch<L, S, EQ, BX_, CPT_, 0, BUF_>, dim3(ntiles), dim3(BX_), 0, s, e0, e1, doms, \
               tiles, ntiles, cfg.remap, step, part, sbase, flat)
#define LBM_BATCH_CASE(BX_, CPT_)                         \
  if (cfg.block == BX_ && cfg.cells_per_thread == CPT_) { \
    if (cfg.buf) LBM_BATCH_LAUNCH(BX_, CPT_, true);       \
    else LBM_BATCH_LAUNCH(BX_, CPT_, false);              \
    return;                                               \
  }
  LBM_BATCH_CASE(64, 1)
  LBM_BATCH_CASE(128, 1)
  LBM_BATCH_CASE(256, 1)
  LBM_BATCH_CASE(64, 2)
  LBM_BATCH_CASE(128, 2)
#undef LBM_BATCH_CASE
#undef LBM_BATCH_LAUNCH
}

template <class L, class S, int EQ>
void Ops<L, S, EQ>::batch_links(const BatchDomain* doms, const BatchBody* bodies, int nbodies, int grid, int64_t step,
                                hipStream_t s, const int64_t* sbase) {
  if constexpr (L::D == 2) {
    hipLaunchKernelGGL((k_links_batch<L, S, EQ, 1024>), dim3(1, nbodies), dim3(1024), 0, s, doms, bodies, step, sbase);
  } else {
    // grid: chunks of 64 links of the largest body
    hipLaunchKernelGGL((k_links_batch_part<L, S, EQ>), dim3(grid, nbodies), dim3(64), 0, s, doms, bodies, step, sbase);
    hipLaunchKernelGGL(k_fold_batch<L>, dim3(nbodies), dim3(64), 0, s, bodies, step, sbase);
  }
}

template <class L, class S, int EQ>
void Ops<L, S, EQ>::batch_body_links(const BatchDomain* doms, const BatchBody* moving, int n_moving,
                                     const BatchBody* fixed, int n_fixed, size_t lds, int64_t step, hipStream_t s,
                                     const int64_t* sbase) {
  if constexpr (L::D == 2)
    hipLaunchKernelGGL((k_body_links_batch<L, S, EQ, 1024>), dim3(n_moving + n_fixed), dim3(1024), lds, s, doms,
                       moving, n_moving, fixed, step, sbase);
}

template <class L, class S, int EQ>
void Ops<L, S, EQ>::batch_body_step(const BatchDomain* doms, const BatchBody* bodies, int nbodies, size_t lds,
                                    int64_t step, hipStream_t s, const int64_t* sbase) {
  constexpr int NT = L::D == 2 ? 1024 : 512;
  hipLaunchKernelGGL((k_body_step_batch<L, S, EQ, NT>), dim3(nbodies), dim3(NT), lds, s, doms, bodies, step, sbase);
}

template <class L, class S, int EQ>
void Ops<L, S, EQ>::batch_wide(const BatchDomain* doms, const BatchBody* bodies, int nbodies, int max_slabs,
                               int64_t step, hipStream_t s, const int64_t* sbase) {
  hipLaunchKernelGGL((k_wide_sets_batch<L, S, EQ>), dim3(max_slabs, nbodies), dim3(WIDE_BLOCK), 0, s, doms, bodies,
                     step, sbase);
  hipLaunchKernelGGL((k_wide_links_batch<L, S, EQ>), dim3(max_slabs, nbodies), dim3(WIDE_BLOCK), 0, s, doms, bodies,
                     step, sbase);
}

}  // namespace lbm
