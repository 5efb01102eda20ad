// Teams: the group of threads that executes one heap (one workgroup of NT
// threads on the GPU; NT = 64 is a single wavefront and needs no barrier).
//
// The paper maps one thread block to one PEM processor whose shared memory is
// the internal memory (Section 4.1).  Here a team is one gfx950 workgroup; its
// LDS holds the small top levels of the heap and the team's scratch.
//
// Every primitive of the heap is written once against this interface
// (pbh_core.h).  HostTeam is a one-thread team used only by the CPU tests that
// drive the same schedule logic on adversarial inputs; the GPU library never
// instantiates it.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

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
  u64 b64[2];
  u32 b32[4];
};

template <int NT>
struct DevTeam {
  static constexpr int kNT = NT;
  static constexpr int kNW = NT / 64;
  TeamShared<kNW>* sh;

  __device__ __forceinline__ int tid() const { return (int)threadIdx.x; }
  __device__ __forceinline__ int lane() const { return (int)(threadIdx.x & 63); }
  __device__ __forceinline__ int wave() const { return (int)(threadIdx.x >> 6); }

  // Orders LDS and global accesses of the team.  A single wavefront needs no
  // hardware barrier: its vector memory operations reach the CU's LDS and L1 in
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
  __device__ __forceinline__ u64 lanemask_lt() const { return (1ull << lane()) - 1ull; }

  __device__ __forceinline__ u32 wave_incl(u32 x) const {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      u32 y = __shfl_up(x, o);
      if (lane() >= o) x += y;
    }
    return x;
  }

  // Exclusive prefix sum over the team; *total receives the team sum.  Ends
  // with every thread past the scratch, so calls may follow each other.
  __device__ u32 scan_excl(u32 x, u32* total) const {
    u32 inc = wave_incl(x);
    if constexpr (NT == 64) {
      *total = __shfl(inc, 63);
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

  __device__ u32 sum(u32 x) const {
    u32 t;
    scan_excl(x, &t);
    return t;
  }

  __device__ void minmax64(u64& lo, u64& hi) const {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      u64 a = __shfl_xor(lo, o), b = __shfl_xor(hi, o);
      lo = a < lo ? a : lo;
      hi = b > hi ? b : hi;
    }
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
  __device__ void minkv(u64& k, u32& v) const {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      u64 k2 = __shfl_xor(k, o);
      u32 v2 = __shfl_xor(v, o);
      bool lt = k2 < k || (k2 == k && v2 < v);
      k = lt ? k2 : k;
      v = lt ? v2 : v;
    }
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

  __device__ __forceinline__ void hist_add(u32* h, u32 b) const { atomicAdd(h + b, 1u); }
  __device__ __forceinline__ u64 atomic_min(u64* p, u64 v) const { return atomicMin(p, v); }
  __device__ __forceinline__ u32 atomic_or32(u32* p, u32 v) const { return atomicOr(p, v); }
  __device__ __forceinline__ u32 load32(const u32* p) const {
    return __hip_atomic_load(const_cast<u32*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ __forceinline__ void store_cur(u64* p, u64 v) const {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ __forceinline__ void fence() const { __threadfence(); }
  // Coherent (L2) read of a value that atomics of this team may have changed.
  __device__ __forceinline__ u64 load_cur(const u64* p) const {
    return __hip_atomic_load(const_cast<u64*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ __forceinline__ void store_stat(u64* p, u64 v) const { *p = v; }
};

// One-thread team for the CPU logic tests.
struct HostTeam {
  static constexpr int kNT = 1;
  static constexpr int kNW = 1;
  TeamShared<1>* sh;
  int tid() const { return 0; }
  int lane() const { return 0; }
  int wave() const { return 0; }
  void sync() const {}
  u64 ballot(bool p) const { return p ? 1ull : 0ull; }
  u64 lanemask_lt() const { return 0ull; }
  u32 scan_excl(u32 x, u32* total) const {
    *total = x;
    return 0;
  }
  u32 sum(u32 x) const { return x; }
  void minmax64(u64&, u64&) const {}
  void minkv(u64&, u32&) const {}
  void hist_add(u32* h, u32 b) const { h[b] += 1; }
  u64 load_cur(const u64* p) const { return *p; }
  u32 atomic_or32(u32* p, u32 v) const {
    u32 o = *p;
    *p = o | v;
    return o;
  }
  u32 load32(const u32* p) const { return *p; }
  void store_cur(u64* p, u64 v) const { *p = v; }
  void fence() const {}
  u64 atomic_min(u64* p, u64 v) const {
    u64 o = *p;
    if (v < o) *p = v;
    return o;
  }
  void store_stat(u64* p, u64 v) const { *p = v; }
};

}  // namespace bkt
