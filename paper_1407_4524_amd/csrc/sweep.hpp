// Device code of the fused pull stream-collide sweep (Eqs. LBE, collision,
// streaming) with the domain-face rules applied on the pull side: the
// dominant kernel of the step, kept in a header of its own (its HBM traffic
// summary is keyed to the hash of this file and the layout headers).
#pragma once
#include "kernels.hpp"

#include <hip/hip_ext.h>

namespace lbm {

// The update's arithmetic: every fused multiply-add is written out
// (fmadd) and the functions that compute a node's new populations let the
// compiler form no other, so that the bits of a node's update do not depend
// on the kernel or launch shape the code is compiled into (left to the
// compiler, the fusions followed the surrounding code).
template <class C>
__device__ __forceinline__ C fmadd(C a, C b, C c) {
  if constexpr (sizeof(C) == 8) return __builtin_fma(a, b, c);
  else return __builtin_fmaf(a, b, c);
}

// ---------------------------------------------------------------------------
// domain faces, applied on the pull side

// Element offset (population plane included) that the pull of direction i
// at the active node (x, y, z), cell c, reads, with the face rules of the
// domain applied on the pull side, and the kind of its source (st):
//  * SRC_WALL, a wall layer: the node's own post-collision value of the
//    opposite direction (halfway bounce-back at a resting wall);
//  * SRC_INLET beyond -x, SRC_OUTVEL beyond a velocity outlet: the same (the
//    wall term 6 w_i rho c_i.u_in is added by the caller: velocity
//    bounce-back at x = -1/2 or nx - 1/2); beyond a Zou-He face the same
//    placeholder, which the caller replaces (zou_he);
//  * SRC_OUTLET beyond a zero-gradient outlet: direction i at the last
//    column, one link back along the transverse axes;
//  * SRC_NONE: the source x - c_i itself, wrapped across periodic faces.
// Periodic axes wrap first and wall layers take precedence (edges and
// corners of the box bounce). Written without branches (bitwise logic and
// selects), so that the loads of all directions stay in one batch.
template <class L>
__device__ __forceinline__ int64_t face_pull(const Geom& g, int x, int y, int z, int64_t c, int i, int& st) {
  int sx = x - L::cx(i), sy = y - L::cy(i), sz = z - L::cz(i);
  const bool px = g.face[0] == FACE_PERIODIC, py = g.face[2] == FACE_PERIODIC, pz = g.face[4] == FACE_PERIODIC;
  sx += (px & (sx < 0)) ? g.nx : ((px & (sx >= g.nx)) ? -g.nx : 0);
  sy += (py & (sy < 0)) ? g.ny : ((py & (sy >= g.ny)) ? -g.ny : 0);
  if (L::D == 3) sz += (pz & (sz < 0)) ? g.nz : ((pz & (sz >= g.nz)) ? -g.nz : 0);
  bool wall = ((g.face[0] == FACE_WALL) & (sx <= 0)) | ((g.face[1] == FACE_WALL) & (sx >= g.nx - 1)) |
              ((g.face[2] == FACE_WALL) & (sy <= 0)) | ((g.face[3] == FACE_WALL) & (sy >= g.ny - 1));
  if (L::D == 3) wall = wall | ((g.face[4] == FACE_WALL) & (sz <= 0)) | ((g.face[5] == FACE_WALL) & (sz >= g.nz - 1));
  const int beyond = sx >= g.nx ? (g.face[1] == FACE_OUTLET ? SRC_OUTLET : SRC_OUTVEL) : SRC_NONE;
  st = wall ? SRC_WALL : (sx < 0 ? SRC_INLET : beyond);
  const bool own = st == SRC_WALL || st == SRC_INLET || st == SRC_OUTVEL;
  const int64_t src = g.idx(st == SRC_OUTLET ? g.nx - 1 : sx, sy, sz);
  return own ? L::opp(i) * g.S + c : i * g.S + src;
}

// Element delta that takes the plain pull of direction i (source x - c_i)
// to the one face_pull gives, at an x-face node of a row that touches no
// other face: at x = lo for c_ix = +1 (lo_side) or x = hi for c_ix = -1.
// Depends on the face type only: bounce-back faces (wall, inlet, velocity
// outlet) read the node's own opposite direction, the zero-gradient outlet
// the last column (one node back), a periodic face the wrapped node.
template <class L>
__device__ __forceinline__ int64_t xface_delta(const Geom& g, int i, bool lo_side) {
  const int64_t off = L::cx(i) + L::cy(i) * g.sy + L::cz(i) * g.sz;
  const int f = lo_side ? g.face[0] : g.face[1];
  const int64_t bounce = (int64_t)(L::opp(i) - i) * g.S + off;
  const int64_t wrap = lo_side ? (int64_t)g.nx : -(int64_t)g.nx;
  return f == FACE_PERIODIC ? wrap : (f == FACE_OUTLET ? (int64_t)-1 : bounce);
}
// Speed of the inlet (or velocity outlet) at the wall point with transverse
// coordinates yB, zB, in the collision's arithmetic type: uniform, or
// 4 u (p - 1/2)(n - 3/2 - p)/(n - 2)^2 along every wall axis (4/(n - 2)^2
// precomputed on the host).
template <class C>
__device__ __forceinline__ C inlet_speed(const Geom& g, const Phys& ph, C yB, C zB) {
#pragma clang fp contract(off)
  C u = (C)ph.inlet_u;
  if (ph.inlet_profile == 1) {
    if (g.face[2] == FACE_WALL) u *= (C)ph.inlet_ky * ((yB - (C)0.5) * ((C)(g.ny - 1.5) - yB));
    if (g.D == 3 && g.face[4] == FACE_WALL) u *= (C)ph.inlet_kz * ((zB - (C)0.5) * ((C)(g.nz - 1.5) - zB));
  }
  return u;
}

// Zou-He face at x = lo (SIDE = +1: the populations with c_ix = +1 are
// unknown) or x = hi (SIDE = -1), on the deviations h of one node after the
// pull (the unknown slots hold placeholders). The node is given either its
// velocity (ux along x, no transverse velocity) or its density (rho0, no
// transverse velocity); mass and x-momentum fix the other one:
//   rho (1 - SIDE ux) = rho0 + K0 + 2 Kb   (standard equilibrium: j = rho u)
//   j_x = rho0 ux                            (quasi-incompressible)
//   j_x = -SIDE (K0 + 2 Kb)                  (given density rho0)
// with K0 the sum over c_ix = 0 and Kb over c_ix = -SIDE. Each unknown i is
// its opposite plus the odd part of the equilibrium difference, 6 w_i c_i.j,
// minus the transverse corrections c_ia N_a, N_a = (1/2) sum_{c_ix=0} c_ia h,
// which give the node zero tangential momentum.
template <class L, int EQ, int SIDE, class C>
__device__ __forceinline__ void zou_he(C* h, bool velocity, C ux, C rho0) {
#pragma clang fp contract(off)
  C k0 = 0, kb = 0, ty = 0, tz = 0;
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    if (L::cx(i) == 0) {
      k0 += h[i];
      if (L::cy(i)) ty += L::cy(i) > 0 ? h[i] : -h[i];
      if (L::D == 3 && L::cz(i)) tz += L::cz(i) > 0 ? h[i] : -h[i];
    } else if (L::cx(i) == -SIDE) {
      kb += h[i];
    }
  }
  const C known = fmadd((C)2, kb, k0);
  C jx;
  if (velocity) jx = EQ ? rho0 * ux : (rho0 + known) / fmadd(-(C)SIDE, ux, (C)1) * ux;
  else jx = -(C)SIDE * known;
  const C ny = (C)0.5 * ty, nz = (C)0.5 * tz;
#pragma unroll
  for (int i = 1; i < L::Q; ++i) {
    if (L::cx(i) != SIDE) continue;
    C v = fmadd((C)(6.0 * L::w(i) * SIDE), jx, h[L::opp(i)]);
    if (L::cy(i)) v += L::cy(i) > 0 ? -ny : ny;
    if (L::D == 3 && L::cz(i)) v += L::cz(i) > 0 ? -nz : nz;
    h[i] = v;
  }
}

// index of an x-face node (x = lo or x = hi) in the arrays of x-face
// densities (the density of the node's state, which the velocity
// bounce-back of the next step takes)
__device__ __forceinline__ int xface_index(const Geom& g, int x, int y, int z) {
  const int n1 = g.hi[1] - g.lo[1] + 1, n2 = g.hi[2] - g.lo[2] + 1;
  return (x == g.lo[0] ? 0 : n1 * n2) + (y - g.lo[1]) + n1 * (z - g.lo[2]);
}

// ---------------------------------------------------------------------------
// fused pull stream + collide

// BGK collision (Eq. collision) of one node in deviation form, h_i = f_i -
// w_i rho0, with the equilibrium of Eq. Fillipova_equilibrium (standard, or
// the quasi-incompressible form when EQ: momentum terms carry rho0 and
// u = j/rho0). Written over the opposite pairs (i, ibar): the moments from
// pair sums and differences, and each pair's equilibria as a common even part
// a and an odd part +-b, so that the arithmetic per node is about 5
// operations per direction (it is what bounds the 2-byte storage sweep).
template <class L, class S, int EQ>
__device__ __forceinline__ void collide(typename S::C* h, typename S::C rho0, typename S::C omega,
                                        typename S::C& rho_out, typename S::C& uu_out) {
#pragma clang fp contract(off)
  using C = typename S::C;
  C drho = h[0], jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int i = 1; i < L::Q; ++i) {
    const int o = L::opp(i);
    if (o < i) continue;
    const C sum = h[i] + h[o], dif = h[i] - h[o];
    drho += sum;
    if (L::cx(i)) jx += L::cx(i) > 0 ? dif : -dif;
    if (L::cy(i)) jy += L::cy(i) > 0 ? dif : -dif;
    if (L::D == 3 && L::cz(i)) jz += L::cz(i) > 0 ? dif : -dif;
  }
  const C rho = rho0 + drho;
  const C rhoU = EQ ? rho0 : rho;
  const C inv = (C)1 / rhoU;
  const C ux = jx * inv, uy = jy * inv, uz = jz * inv;
  const C uu = fmadd(ux, ux, fmadd(uy, uy, uz * uz));
  uu_out = uu;
  // even part common to all directions: drho - rhoU 3/2 u.u
  const C t = fmadd(-rhoU, (C)1.5 * uu, drho);
  const C keep = (C)1 - omega;
  const C r45 = (C)4.5 * rhoU, r3 = (C)3 * rhoU;
  h[0] = fmadd(keep, h[0], omega * ((C)L::w(0) * t));
#pragma unroll
  for (int i = 1; i < L::Q; ++i) {
    const int o = L::opp(i);
    if (o < i) continue;
    C cu = 0;
    if (L::cx(i)) cu += L::cx(i) > 0 ? ux : -ux;
    if (L::cy(i)) cu += L::cy(i) > 0 ? uy : -uy;
    if (L::D == 3 && L::cz(i)) cu += L::cz(i) > 0 ? uz : -uz;
    const C wo = omega * (C)L::w(i);
    const C a = wo * fmadd(r45, cu * cu, t);  // omega times the even part of f^eq_i - w_i rho0
    const C r3cu = r3 * cu;                   // wo r3cu: omega times the odd part
    h[i] = fmadd(keep, h[i], fmadd(wo, r3cu, a));
    h[o] = fmadd(keep, h[o], fmadd(-wo, r3cu, a));
  }
  rho_out = rho;
}

constexpr int BULK_BLOCK = 256;

// Logical block of hardware block hw: hardware block k runs on XCD k % 8, so
// every XCD gets a contiguous run of logical blocks and the cache lines shared
// by neighbouring blocks stay in one L2.
__device__ inline int xcd_block(int hw, int nblocks) {
  const int q = nblocks >> 3, r = nblocks & 7;
  const int xcd = hw & 7, k = hw >> 3;
  return xcd * q + (xcd < r ? xcd : r) + k;
}

// BX*CPT consecutive nodes of one row up to xlast, starting at x0; thread t
// of a block takes x = x0 + k*BX (k < CPT), so every load and store
// instruction of a wavefront covers 64 consecutive nodes. Nodes inside the
// hole box (x0, x1, y0, y1, z0, z1; empty when x0 > x1) are left alone. All
// CPT*Q loads are issued before any arithmetic.
// Face rules on the pull side: in a row that touches a y or z face (FACE_ROW,
// a block-uniform case) every pull goes through face_pull; in any other row
// only the two x-face nodes differ from the plain pull, by an address delta
// per direction (xface_delta) selected per lane, so that the loads stay one
// batch. rho_in / rho_out: densities of the x-face nodes of the old / new
// state (the velocity bounce-back's rho(x_F)); null when no face needs them.
template <class L, class S, int EQ, int BX, int CPT, int MEM, bool FACE_ROW, bool BUF>
__device__ __forceinline__ void stream_collide_row(const typename S::T* __restrict__ A,
                                                   typename S::T* __restrict__ B, const Geom& g, const Phys& ph,
                                                   int x0, int y, int z, int xlast, const int* hole,
                                                   const typename S::C* __restrict__ rho_in,
                                                   typename S::C* __restrict__ rho_out,
                                                   const uint8_t* __restrict__ mask, int* unstable) {
  using C = typename S::C;
  using T = typename S::T;
  const bool hole_row = y >= hole[2] && y <= hole[3] && z >= hole[4] && z <= hole[5];
  bool ok[CPT];
  bool any = false;
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int x = x0 + k * BX;
    ok[k] = x <= xlast && !(hole_row && x >= hole[0] && x <= hole[1]);
    any = any || ok[k];
  }
  if (!any) return;
  const int64_t c0 = g.idx(x0, y, z);
  const bool need_rho = !EQ && rho_in != nullptr;
  // Every load is unconditional (a node that is not updated re-reads node x0)
  // and lands in its own register before any conversion, so that all of them
  // are in flight together; a guarded load would sit in its own basic block
  // and be waited for at the block's end.
  // BUF: raw buffer accesses with 32-bit byte offsets (the host picks this
  // form when a population buffer is below 4 GiB): a plain pull is the
  // node's offset plus a per-direction constant, so the address arithmetic
  // is scalar except where a lane's pull is shifted by a face rule
  constexpr uint32_t ESZ = sizeof(T);
  constexpr int LAUX = (MEM & MEM_NT_LOAD) ? BUF_NT : 0;
  constexpr int SAUX = (MEM & MEM_NT_STORE) ? BUF_NT : 0;
  [[maybe_unused]] const Rsrc ra = make_rsrc(A, (uint64_t)L::Q * g.S * ESZ);
  [[maybe_unused]] const Rsrc rb = make_rsrc(B, (uint64_t)L::Q * g.S * ESZ);
  typename S::R raw[CPT][L::Q];
  C rho_w[CPT];
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int x = ok[k] ? x0 + k * BX : x0;
    const int64_t ck = c0 + (x - x0);
    const bool xlo = x == g.lo[0], xhi = x == g.hi[0];
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
      const int64_t plain = i * g.S - (L::cx(i) + L::cy(i) * g.sy + L::cz(i) * g.sz);  // uniform
      int64_t a;
      if constexpr (FACE_ROW) {
        int st;
        a = i == 0 ? ck : face_pull<L>(g, x, y, z, ck, i, st);
      } else {
        a = plain + ck;
        if (L::cx(i) == 1) a += xlo ? xface_delta<L>(g, i, true) : (int64_t)0;
        if (L::cx(i) == -1) a += xhi ? xface_delta<L>(g, i, false) : (int64_t)0;
      }
      if constexpr (BUF) {
        // 32-bit wrap-around arithmetic: the sum is the offset itself
        if (!FACE_ROW && L::cx(i) == 0)
          raw[k][i] = S::template load_buf<LAUX>(ra, (uint32_t)ck * ESZ, (uint32_t)plain * ESZ);
        else
          raw[k][i] = S::template load_buf<LAUX>(ra, (uint32_t)a * ESZ, 0u);
      } else {
        raw[k][i] = S::template load_raw_mem<(MEM & MEM_NT_LOAD) != 0>(A + a);
      }
    }
    // the x-face density (every lane loads one; only x-face lanes use it)
    rho_w[k] = need_rho ? rho_in[xface_index(g, xhi ? g.hi[0] : g.lo[0], y, z)] : (C)ph.rho0;
  }
  // keep the scheduler from sinking conversions between the loads
  __builtin_amdgcn_sched_barrier(0);
  C h[CPT][L::Q];
#pragma unroll
  for (int k = 0; k < CPT; ++k)
#pragma unroll
    for (int i = 0; i < L::Q; ++i) h[k][i] = S::from_raw(raw[k][i]);
  // velocity bounce-back: the wall term of the inlet (x = lo, c_ix = +1)
  // and velocity outlet (x = hi, c_ix = -1) directions
  const bool inlet = g.face[0] == FACE_INLET, outvel = g.face[1] == FACE_OUTLET_VELOCITY;
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int x = x0 + k * BX;
    const bool xlo = x == g.lo[0], xhi = x == g.hi[0];
    if (!((inlet & xlo) | (outvel & xhi))) continue;
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
      if (!L::cx(i)) continue;
      bool apply;
      if constexpr (FACE_ROW) {
        int st;
        (void)face_pull<L>(g, x, y, z, 0, i, st);
        apply = st == SRC_INLET || st == SRC_OUTVEL;
      } else {
        apply = L::cx(i) == 1 ? (inlet & xlo) : (outvel & xhi);
      }
      if (apply)
        h[k][i] = fmadd((C)(6.0 * L::w(i) * L::cx(i)) * rho_w[k],
                        inlet_speed<C>(g, ph, (C)y - (C)(0.5 * L::cy(i)), (C)z - (C)(0.5 * L::cz(i))), h[k][i]);
    }
  }
  // Zou-He faces: the entering populations of the x-face nodes rebuilt
  const bool zlo = g.face[0] >= FACE_ZOUHE_VELOCITY, zhi = g.face[1] >= FACE_ZOUHE_VELOCITY;
  if (zlo | zhi) {
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      const int x = x0 + k * BX;
      if (zlo & (x == g.lo[0]))
        zou_he<L, EQ, 1>(h[k], g.face[0] == FACE_ZOUHE_VELOCITY, inlet_speed<C>(g, ph, (C)y, (C)z), (C)ph.rho0);
      else if (zhi & (x == g.hi[0]))
        zou_he<L, EQ, -1>(h[k], g.face[1] == FACE_ZOUHE_VELOCITY, inlet_speed<C>(g, ph, (C)y, (C)z), (C)ph.rho0);
    }
  }
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    if (!ok[k]) continue;
    const int x = x0 + k * BX;
    const int64_t c = c0 + k * BX;
    C rho, uu;
    collide<L, S, EQ>(h[k], (C)ph.rho0, (C)ph.omega, rho, uu);
    // instability: a fluid node whose speed exceeds 0.4 or is not a number
    // (the mask is read only for such a node; solid nodes are swept too but
    // their values are never used)
    if (!(uu <= (C)0.16) && unstable && mask[c] == MASK_FLUID) *unstable = 1;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
      if constexpr (BUF) S::template store_buf<SAUX>(rb, (uint32_t)c * ESZ, (uint32_t)(i * g.S) * ESZ, h[k][i]);
      else if constexpr ((MEM & MEM_NT_STORE) != 0) __builtin_nontemporal_store((T)h[k][i], B + i * g.S + c);
      else B[i * g.S + c] = (T)h[k][i];
    }
    if (rho_out && (x == g.lo[0] || x == g.hi[0])) rho_out[xface_index(g, x, y, z)] = rho;
  }
}

template <class L, class S, int EQ, int BX, int CPT, int MEM, bool BUF = false>
__device__ __forceinline__ void stream_collide_span(const typename S::T* __restrict__ A,
                                                    typename S::T* __restrict__ B, const Geom& g, const Phys& ph,
                                                    int x0, int y, int z, int xlast, const int* hole,
                                                    const typename S::C* __restrict__ rho_in,
                                                    typename S::C* __restrict__ rho_out,
                                                    const uint8_t* __restrict__ mask, int* unstable) {
  const bool face_row = (y <= g.lo[1]) | (y >= g.hi[1]) | (L::D == 3 && ((z <= g.lo[2]) | (z >= g.hi[2])));
  if (face_row)
    stream_collide_row<L, S, EQ, BX, CPT, MEM, true, BUF>(A, B, g, ph, x0, y, z, xlast, hole, rho_in, rho_out, mask,
                                                          unstable);
  else
    stream_collide_row<L, S, EQ, BX, CPT, MEM, false, BUF>(A, B, g, ph, x0, y, z, xlast, hole, rho_in, rho_out, mask,
                                                           unstable);
}
// tile k of a sweep: the span of BX*CPT nodes at which thread 0 starts
__device__ __forceinline__ void sweep_tile(const Sweep& sw, int k, int span, int& x, int& y, int& z) {
  const int bx = k % sw.nbx, r = k / sw.nbx;
  x = sw.x0 + bx * span;
  y = sw.y0 + r % sw.ny;
  z = sw.z0 + r / sw.ny;
}

// one block per tile of the sweep
template <class L, class S, int EQ, int BX, int CPT, int MEM, bool BUF>
__global__ __launch_bounds__(BX) void k_stream_collide(const typename S::T* __restrict__ A,
                                                       typename S::T* __restrict__ B, Geom g, Phys ph, Sweep sw) {
  const int blk = sw.remap ? xcd_block(blockIdx.x, sw.ntiles) : blockIdx.x;
  int x, y, z;
  sweep_tile(sw, blk, BX * CPT, x, y, z);
  stream_collide_span<L, S, EQ, BX, CPT, MEM, BUF>(A, B, g, ph, x + threadIdx.x, y, z, sw.xlast, sw.hole,
                                                   (const typename S::C*)sw.rho_in, (typename S::C*)sw.rho_out,
                                                   sw.mask, sw.unstable);
}

}  // namespace lbm
