// Teams: the group of threads that executes one heap (one workgroup of NT
// threads on the GPU; NT = 64 is a single wavefront and needs no barrier).
//
// The paper maps one thread block to one PEM processor whose shared memory is
// the internal memory (Section 4.1).  Here a team is one gfx950 workgroup; its
// LDS holds the small top levels of the heap and the team's scratch.
//
// Every primitive of the heap is written once against this interface
// (pbh_core.h).  Wavefront scans and reductions use DPP row shifts and row
// broadcasts (no LDS traffic); totals are broadcast with v_readlane.
// HostTeam is a one-thread team used only by the CPU tests that drive the same
// schedule logic on adversarial inputs; the GPU library never instantiates it.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define PBH_LDS __attribute__((address_space(3)))
#define PBH_GLB __attribute__((address_space(1)))

namespace bkt {

typedef unsigned long long u64;
typedef unsigned int u32;

// Per-team LDS scratch used by scans, reductions, histograms and the stable
// radix scatter.
template <int NW>
struct TeamShared {
  u32 wsum[NW > 1 ? NW : 1];
  u64 wk[NW > 1 ? NW : 1];
  u64 wk2[NW > 1 ? NW : 1];
  u32 wv[NW > 1 ? NW : 1];
  u32 hist[256];
  u32 base[256];
  u32 wcnt[NW][256];
  u32 b32[4];
  u64 ex0[256];  // first edge of each vertex extracted in a round
  u32 exd[257];  // prefix sums of their out-degrees
  float mlp_h[64];
  float mlp_z[64];
  float mlp_p[NW >= 4 ? 256 : 1];  // partial sums of the second layer (teams of >= 256)
};

// DPP lane moves (gfx9 encodings): row_shr:n = 0x110 + n within rows of 16
// lanes; row_bcast:15 = 0x142 (lane 15 of a row to the next row);
// row_bcast:31 = 0x143 (lane 31 to rows 2 and 3).  Lanes whose source is
// invalid, or whose row is masked off, keep `old`.
template <int CTRL, int RM>
__device__ __forceinline__ u32 dpp_mov(u32 old, u32 x) {
  return (u32)__builtin_amdgcn_update_dpp((int)old, (int)x, CTRL, RM, 0xF, false);
}
template <int CTRL, int RM>
__device__ __forceinline__ u64 dpp_mov64(u64 old, u64 x) {
  u32 lo = dpp_mov<CTRL, RM>((u32)old, (u32)x);
  u32 hi = dpp_mov<CTRL, RM>((u32)(old >> 32), (u32)(x >> 32));
  return ((u64)hi << 32) | lo;
}
__device__ __forceinline__ u64 readlane64(u64 x, int l) {
  u32 lo = __builtin_amdgcn_readlane((u32)x, l), hi = __builtin_amdgcn_readlane((u32)(x >> 32), l);
  return ((u64)hi << 32) | lo;
}

// Inclusive prefix sum over the 64 lanes of a wavefront.
__device__ __forceinline__ u32 wave_incl(u32 x) {
  x += dpp_mov<0x111, 0xF>(0u, x);
  x += dpp_mov<0x112, 0xF>(0u, x);
  x += dpp_mov<0x114, 0xF>(0u, x);
  x += dpp_mov<0x118, 0xF>(0u, x);
  x += dpp_mov<0x142, 0xA>(0u, x);
  x += dpp_mov<0x143, 0xC>(0u, x);
  return x;
}

template <int CTRL, int RM>
__device__ __forceinline__ void kv_step_min(u64& k, u32& v) {
  u64 k2 = dpp_mov64<CTRL, RM>(~0ull, k);
  u32 v2 = dpp_mov<CTRL, RM>(~0u, v);
  bool lt = k2 < k || (k2 == k && v2 < v);
  k = lt ? k2 : k;
  v = lt ? v2 : v;
}
// Minimum (key, id) of the wavefront, in every lane.
__device__ __forceinline__ void wave_min_kv(u64& k, u32& v) {
  kv_step_min<0x111, 0xF>(k, v);
  kv_step_min<0x112, 0xF>(k, v);
  kv_step_min<0x114, 0xF>(k, v);
  kv_step_min<0x118, 0xF>(k, v);
  kv_step_min<0x142, 0xA>(k, v);
  kv_step_min<0x143, 0xC>(k, v);
  k = readlane64(k, 63);
  v = __builtin_amdgcn_readlane(v, 63);
}
template <int CTRL, int RM>
__device__ __forceinline__ void mm_step(u64& lo, u64& hi) {
  u64 a = dpp_mov64<CTRL, RM>(~0ull, lo), b = dpp_mov64<CTRL, RM>(0ull, hi);
  lo = a < lo ? a : lo;
  hi = b > hi ? b : hi;
}
__device__ __forceinline__ void wave_minmax64(u64& lo, u64& hi) {
  mm_step<0x111, 0xF>(lo, hi);
  mm_step<0x112, 0xF>(lo, hi);
  mm_step<0x114, 0xF>(lo, hi);
  mm_step<0x118, 0xF>(lo, hi);
  mm_step<0x142, 0xA>(lo, hi);
  mm_step<0x143, 0xC>(lo, hi);
  lo = readlane64(lo, 63);
  hi = readlane64(hi, 63);
}

// FULL: the team of the large-heap round loop (deep-level workers), whose
// primitives on HBM levels use the LDS staging area, keep more loads in
// flight and select in registers; the default team keeps the plain forms,
// which leave the one-workgroup round loop's registers as they are.
template <int NT, bool FULL = false>
struct DevTeam {
  static constexpr int kNT = NT;
  static constexpr int kNW = NT / 64;
  static constexpr int kE = NT == 64 ? 8 : 4;  // elements per thread per tile
  static constexpr bool kStage = FULL;
  static constexpr int kRU = FULL ? 4 : 1;     // loads in flight per thread in streaming loops
  TeamShared<kNW> PBH_LDS* sh;
  // LDS staging area for merges of arrays in HBM (null: none): two windows of
  // kNT * kE + 2 elements (keys, then ids) and kNT + 1 split points
  u64 PBH_LDS* stk = nullptr;
  u32 PBH_LDS* stv = nullptr;
  u32 PBH_LDS* stp = nullptr;

  __device__ __forceinline__ int tid() const { return (int)threadIdx.x; }
  __device__ __forceinline__ int lane() const { return (int)(threadIdx.x & 63); }
  __device__ __forceinline__ int wave() const { return (int)(threadIdx.x >> 6); }

  // Orders LDS and global accesses of the team.  A single wavefront needs no
  // hardware barrier: its memory operations reach the CU's LDS and L1 in
  // issue order, so a compiler fence is enough.
  __device__ __forceinline__ void sync() const {
    if constexpr (NT == 64) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
      __syncthreads();
    }
  }

  __device__ __forceinline__ u64 ballot(bool p) const { return __ballot(p); }
  // Number of set bits of m in lanes below this one.
  __device__ __forceinline__ u32 count_below(u64 m) const {
    return __builtin_amdgcn_mbcnt_hi((u32)(m >> 32), __builtin_amdgcn_mbcnt_lo((u32)m, 0u));
  }

  // Exclusive prefix sum over the team; *total receives the team sum.
  __device__ __forceinline__ u32 scan_excl(u32 x, u32* total) const {
    u32 inc = wave_incl(x);
    if constexpr (NT == 64) {
      *total = __builtin_amdgcn_readlane(inc, 63);
      return inc - x;
    } else {
      if (lane() == 63) sh->wsum[wave()] = inc;
      __syncthreads();
      u32 pre = 0, tot = 0;
#pragma unroll
      for (int w = 0; w < kNW; ++w) {
        u32 s = sh->wsum[w];
        pre += (w < wave()) ? s : 0u;
        tot += s;
      }
      __syncthreads();
      *total = tot;
      return pre + inc - x;
    }
  }

  __device__ __forceinline__ u32 sum(u32 x) const {
    u32 t;
    scan_excl(x, &t);
    return t;
  }

  __device__ __forceinline__ void minmax64(u64& lo, u64& hi) const {
    wave_minmax64(lo, hi);
    if constexpr (NT > 64) {
      if (lane() == 0) {
        sh->wk[wave()] = lo;
        sh->wk2[wave()] = hi;
      }
      __syncthreads();
      u64 l = sh->wk[0], h = sh->wk2[0];
      for (int w = 1; w < kNW; ++w) {
        l = sh->wk[w] < l ? sh->wk[w] : l;
        h = sh->wk2[w] > h ? sh->wk2[w] : h;
      }
      __syncthreads();
      lo = l;
      hi = h;
    }
  }

  // Team minimum of (k, v) pairs in (key, id) order.
  __device__ __forceinline__ void minkv(u64& k, u32& v) const {
    wave_min_kv(k, v);
    if constexpr (NT > 64) {
      if (lane() == 0) {
        sh->wk[wave()] = k;
        sh->wv[wave()] = v;
      }
      __syncthreads();
      u64 bk = sh->wk[0];
      u32 bv = sh->wv[0];
      for (int w = 1; w < kNW; ++w) {
        u64 k2 = sh->wk[w];
        u32 v2 = sh->wv[w];
        bool lt = k2 < bk || (k2 == bk && v2 < bv);
        bk = lt ? k2 : bk;
        bv = lt ? v2 : bv;
      }
      __syncthreads();
      k = bk;
      v = bv;
    }
  }

  __device__ __forceinline__ void hist_add(u32 PBH_LDS* h, u32 b) const {
    __hip_atomic_fetch_add(h + b, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  __device__ __forceinline__ u64 atomic_min(u64* p, u64 v) const {
    return __hip_atomic_fetch_min((u64 PBH_GLB*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ __forceinline__ u32 atomic_add32(u32* p, u32 v) const {
    return __hip_atomic_fetch_add((u32 PBH_GLB*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ __forceinline__ u64 atomic_exch(u64* p, u64 v) const {
    return __hip_atomic_exchange((u64 PBH_GLB*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ __forceinline__ u32 atomic_or32(u32* p, u32 v) const {
    return __hip_atomic_fetch_or((u32 PBH_GLB*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  // Coherent (L2) reads and writes of values that atomics may have changed.
  __device__ __forceinline__ u64 load_cur(const u64* p) const {
    return __hip_atomic_load((u64 PBH_GLB*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ __forceinline__ u32 load32(const u32* p) const {
    return __hip_atomic_load((u32 PBH_GLB*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ __forceinline__ void store_cur(u64* p, u64 v) const {
    __hip_atomic_store((u64 PBH_GLB*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ __forceinline__ void fence() const { __threadfence(); }
};

// One-thread team for the CPU logic tests; STAGE picks the large-heap forms
// of the primitives (as DevTeam's FULL) or the plain ones.
template <bool STAGE>
struct HostTeamT {
  static constexpr int kNT = 1;
  static constexpr int kNW = 1;
  static constexpr int kE = 4;
  static constexpr bool kStage = STAGE;
  static constexpr int kRU = STAGE ? 4 : 1;
  TeamShared<1>* sh;
  u64* stk = nullptr;  // staging area (as DevTeam's)
  u32* stv = nullptr;
  u32* stp = nullptr;
  int tid() const { return 0; }
  int lane() const { return 0; }
  int wave() const { return 0; }
  void sync() const {}
  u64 ballot(bool p) const { return p ? 1ull : 0ull; }
  u32 count_below(u64) const { return 0; }
  u32 scan_excl(u32 x, u32* total) const {
    *total = x;
    return 0;
  }
  u32 sum(u32 x) const { return x; }
  void minmax64(u64&, u64&) const {}
  void minkv(u64&, u32&) const {}
  void hist_add(u32* h, u32 b) const { h[b] += 1; }
  u64 atomic_min(u64* p, u64 v) const {
    u64 o = *p;
    if (v < o) *p = v;
    return o;
  }
  u32 atomic_or32(u32* p, u32 v) const {
    u32 o = *p;
    *p = o | v;
    return o;
  }
  u32 atomic_add32(u32* p, u32 v) const {
    u32 o = *p;
    *p = o + v;
    return o;
  }
  u64 atomic_exch(u64* p, u64 v) const {
    u64 o = *p;
    *p = v;
    return o;
  }
  u64 load_cur(const u64* p) const { return *p; }
  u32 load32(const u32* p) const { return *p; }
  void store_cur(u64* p, u64 v) const { *p = v; }
  void fence() const {}
};
using HostTeam = HostTeamT<true>;
using HostTeamPlain = HostTeamT<false>;

}  // namespace bkt
