// Lattice and storage traits of the GPU path.
//
// D2Q9 and D3Q19 velocity sets with the numbering fixed by include/lbm.h.
// The tables are constexpr functions so that, inside fully unrolled loops,
// every c_i, w_i and opposite index folds to an immediate.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// Raw buffer resource over `bytes` bytes at p (stride 0: byte offsets, a
// per-lane one plus a uniform one; lanes whose offset reaches past the end
// read zero and write nothing). Offsets are 32-bit, so a buffer addressed
// this way holds less than 4 GiB.
using Rsrc = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ Rsrc make_rsrc(const void* p, uint64_t bytes) {
  const uint32_t n = bytes > 0xffffffffull ? 0xffffffffu : (uint32_t)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)n, 0x00020000);
}
// cache-policy bits of a buffer access: the non-temporal hint
constexpr int BUF_NT = 2;

struct D2Q9 {
  static constexpr int D = 2;
  static constexpr int Q = 9;
  __host__ __device__ static constexpr int cx(int i) {
    constexpr int t[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    return t[i];
  }
  __host__ __device__ static constexpr int cy(int i) {
    constexpr int t[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    return t[i];
  }
  __host__ __device__ static constexpr int cz(int) { return 0; }
  __host__ __device__ static constexpr int opp(int i) {
    constexpr int t[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    return t[i];
  }
  __host__ __device__ static constexpr double w(int i) {
    return i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
  }
};

struct D3Q19 {
  static constexpr int D = 3;
  static constexpr int Q = 19;
  __host__ __device__ static constexpr int cx(int i) {
    constexpr int t[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return t[i];
  }
  __host__ __device__ static constexpr int cy(int i) {
    constexpr int t[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    return t[i];
  }
  __host__ __device__ static constexpr int cz(int i) {
    constexpr int t[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    return t[i];
  }
  __host__ __device__ static constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
  __host__ __device__ static constexpr double w(int i) {
    return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
};

// Storage of a population deviation h_i = f_i - w_i rho0 and the type the
// bulk collision computes in.
struct StoreF64 {
  using T = double;
  using C = double;
  using R = double;  // register form of a loaded element
  __device__ static R load_raw(const T* p) { return *p; }
  template <bool NT>
  __device__ static R load_raw_mem(const T* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
  }
  template <int AUX>
  __device__ static R load_buf(Rsrc r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, AUX));
  }
  template <int AUX>
  __device__ static void store_buf(Rsrc r, uint32_t voff, uint32_t soff, C v) {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, (int)voff, (int)soff, AUX);
  }
  __device__ static C from_raw(R r) { return r; }
  __device__ static C load(const T* p) { return *p; }
  __device__ static void store_plain(T* p, double v) { *p = v; }
  __device__ static double round_trip(double v) { return v; }
  // the value a store keeps
  __device__ static C stored(C v) { return v; }
};

struct StoreF32 {
  using T = float;
  using C = float;
  using R = float;
  __device__ static R load_raw(const T* p) { return *p; }
  template <bool NT>
  __device__ static R load_raw_mem(const T* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
  }
  template <int AUX>
  __device__ static R load_buf(Rsrc r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, AUX));
  }
  template <int AUX>
  __device__ static void store_buf(Rsrc r, uint32_t voff, uint32_t soff, C v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff, (int)soff, AUX);
  }
  __device__ static C from_raw(R r) { return r; }
  __device__ static C load(const T* p) { return *p; }
  __device__ static void store_plain(T* p, double v) { *p = (float)v; }
  __device__ static double round_trip(double v) { return (double)(float)v; }
  // the value a store keeps
  __device__ static C stored(C v) { return v; }
};

// binary16 deviations, round-to-nearest-even on store, FP32 arithmetic
struct StoreF16 {
  using T = _Float16;
  using C = float;
  // a loaded element is held zero-extended in a full 32-bit register, so
  // that the loads of all populations can be in flight at once (two halves
  // packed into one register would serialise them)
  using R = uint32_t;
  __device__ static R load_raw(const T* p) { return (uint32_t)*reinterpret_cast<const uint16_t*>(p); }
  template <bool NT>
  __device__ static R load_raw_mem(const T* p) {
    const uint16_t* q = reinterpret_cast<const uint16_t*>(p);
    if constexpr (NT) return (uint32_t)__builtin_nontemporal_load(q);
    else return (uint32_t)*q;
  }
  template <int AUX>
  __device__ static R load_buf(Rsrc r, uint32_t voff, uint32_t soff) {
    return (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, AUX);
  }
  template <int AUX>
  __device__ static void store_buf(Rsrc r, uint32_t voff, uint32_t soff, C v) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, (_Float16)v), r, (int)voff, (int)soff, AUX);
  }
  __device__ static C from_raw(R r) { return (float)__builtin_bit_cast(_Float16, (uint16_t)r); }
  __device__ static C load(const T* p) { return (float)*p; }
  __device__ static void store_plain(T* p, double v) { *p = (_Float16)(float)v; }
  __device__ static double round_trip(double v) { return (double)(float)(_Float16)(float)v; }
  // the value a store keeps (rounded to binary16, to nearest even)
  __device__ static C stored(C v) { return (float)(_Float16)v; }
};

}  // namespace lbm
