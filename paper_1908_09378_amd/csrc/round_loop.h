// The parDijkstra round loop as the SSSP kernels run it (kernels.hip: one
// query on one workgroup; kernels_full.hip: the large-heap form with
// deep-level workers, and many queries in one launch).
#pragma once
#include "pbh_launch.h"

namespace bkt {

// GPU placement of the heap: LDS levels, HBM levels and the state in LDS.
struct DevPolicy {
  using L = ArrT<u64 PBH_LDS*, u32 PBH_LDS*>;
  using G = ArrT<u64 PBH_GLB*, u32 PBH_GLB*>;
  using SP = HeapState PBH_LDS*;
  __device__ __forceinline__ static void on_resolve(const Geom&, SP, int, bool) {}
};

// Synchronisation of the deep-level service (pbh_core.h) between workgroups:
// counters in the control block, read and written with agent-scope atomics
// (the XCDs' L2 caches are not coherent for plain accesses).  Before a team
// counts a request or a completion, every thread waits for its own stores
// and thread 0 issues an agent-scope release, so the level arrays and states
// it wrote are visible to the team that sees the count; a waiting team's
// thread 0 issues an agent-scope acquire once the condition holds.  Waits
// poll with s_sleep and give up at once when another team has failed, or
// with E_TIMEOUT after DEEP_TIMEOUT of the 100 MHz clock without the condition
// (a Resolve never takes that long); a worker waiting for its next request,
// which may not come for the rest of a long run, restarts that clock whenever
// the front's heartbeat (its round count, every 1024 rounds) moves.
constexpr u64 DEEP_TIMEOUT = 1000000000ull;  // 10 s

template <class T>
struct DevDeepSync {
  static constexpr bool kOn = true;
  DeepCtl* c;
  int lim;

  __device__ static u32 ld(const u32* p) {
    return __hip_atomic_load((u32 PBH_GLB*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ static u64 ld64(const u64* p) {
    return __hip_atomic_load((u64 PBH_GLB*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ static u64 add64(u64* p, u64 v) {
    return __hip_atomic_fetch_add((u64 PBH_GLB*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  // Thread 0's value to every thread of the team.
  __device__ static u64 bcast(const T& t, u64 v) {
    if (t.tid() == 0) t.sh->wk2[0] = v;
    t.sync();
    const u64 r = t.sh->wk2[0];
    t.sync();
    return r;
  }
  // Every thread's stores complete, then one agent-scope release.
  __device__ void release(const T& t) const {
    __builtin_amdgcn_s_waitcnt(0);
    t.sync();
    if (t.tid() == 0) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  }
  __device__ void count(const T& t, u32* ctr) const {
    release(t);
    if (t.tid() == 0) __hip_atomic_fetch_add((u32 PBH_GLB*)ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    t.sync();
  }
  __device__ void set_err(int code) const {
    int zero = 0;
    __hip_atomic_compare_exchange_strong((int PBH_GLB*)&c->err, &zero, code, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
  }
  // Thread 0 polls until ready() (true), another team failed or the time ran
  // out (false), or leave_ok and the exit flag is set (false); then acquires.
  template <class F>
  __device__ bool spin(const T& t, F ready, bool leave_ok) const {
    u64 r = 1;
    if (t.tid() == 0) {
      u64 t0 = __builtin_amdgcn_s_memrealtime();
      u32 beat = ld(&c->beat);
      while (!ready()) {
        if (ld((const u32*)&c->err) || (leave_ok && ld(&c->exit))) {
          r = 0;
          break;
        }
        if (leave_ok) {
          const u32 b = ld(&c->beat);
          if (b != beat) {
            beat = b;
            t0 = __builtin_amdgcn_s_memrealtime();
          }
        }
        if (__builtin_amdgcn_s_memrealtime() - t0 > DEEP_TIMEOUT) {
          set_err(E_TIMEOUT);
          r = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    return bcast(t, r) != 0;
  }

  __device__ bool wait_idle(const T& t, int j) const {
    return spin(t, [&] { return ld(&c->done[j]) == ld(&c->req[j]); }, false);
  }
  // A Resolve(j) request is pending (true), or the run is over (false).
  __device__ bool wait_request(const T& t, int j) const {
    return spin(t, [&] { return ld(&c->done[j]) != ld(&c->req[j]); }, true);
  }
  __device__ void post(const T& t, int j) const { count(t, &c->req[j]); }
  __device__ void done(const T& t, int j) const { count(t, &c->done[j]); }
  __device__ void publish(const T& t) const {
    release(t);
    t.sync();
  }
  template <class SP>
  __device__ void get(const T& t, SP st, int j) const {
    if (t.tid() == 0) lvl_store(st, j, lvl_load(c, j));
    t.sync();
  }
  template <class SP>
  __device__ void put(const T& t, SP st, int j) const {
    t.sync();
    if (t.tid() == 0) lvl_store(c, j, lvl_load(st, j));
    t.sync();
  }
  __device__ u64 deeper(const T& t, int j) const { return bcast(t, t.tid() == 0 ? ld64(&c->deeper[j]) : 0ull); }
  __device__ void set_deeper(const T& t, int j, u64 v) const {
    if (t.tid() == 0) __hip_atomic_store((u64 PBH_GLB*)&c->deeper[j], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    t.sync();
  }
  // After Resolve(i) of a worker: `drop` (<= 0) elements left levels i and
  // i+1, level i+1 changed by d1; elements touched and busy ticks so far.
  __device__ void account(const T& t, int i, long long drop, long long d1, u64 elems, u64 busy) const {
    if (t.tid() == 0) {
      if (drop)
        for (int j = lim; j <= i; ++j) add64(&c->deeper[j], (u64)drop);
      if (d1) add64(&c->deeper[i + 1], (u64)d1);
      if (elems) add64(&c->elems, elems);
      c->busy[i] = busy;
    }
    t.sync();
  }
  // After the front's Resolve(lim - 1): level lim changed by d; returns the
  // elements now in the worker levels.
  __device__ u64 front_account(const T& t, int j, long long d) const {
    return bcast(t, t.tid() == 0 ? add64(&c->deeper[j], (u64)d) + (u64)d : 0ull);
  }
  __device__ void fail(const T& t, int code) const {
    if (t.tid() == 0) set_err(code);
    t.sync();
  }
  __device__ int error(const T& t) const { return (int)bcast(t, t.tid() == 0 ? (u64)(u32)ld((const u32*)&c->err) : 0ull); }
  template <class SP>
  __device__ void merge_stats(const T& t, SP st, int lo, int q) const {
    if (t.tid() == 0) {
      st->elems += ld64(&c->elems);
      if (st->prof_on)
        for (int j = lo; j < q; ++j) st->prof[j] += c->busy[j];
    }
    t.sync();
  }
  __device__ void beat(const T& t, u32 rounds) const {
    if (t.tid() == 0) __hip_atomic_store((u32 PBH_GLB*)&c->beat, rounds, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ void leave(const T& t) const {
    release(t);
    if (t.tid() == 0) __hip_atomic_store((u32 PBH_GLB*)&c->exit, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    t.sync();
  }
};

// A deep-level worker: Resolve(lvl) whenever the level above asks, until the
// front has finished (or any team has failed).
template <int NT>
__device__ __attribute__((always_inline)) void deep_worker(DevTeam<NT, true>& t, HeapState PBH_LDS* st,
                                                          unsigned char* dyn, const SsspParams& p,
                            int lvl) {
  Geom g = p.g;
  g.lk = nullptr;  // worker levels are never in LDS
  g.lv = nullptr;
  if (p.stage) stage_setup(t, (unsigned char PBH_LDS*)dyn);
  if (threadIdx.x == 0) {
    state_init(st, g.d, g.q);
    st->prof_on = p.prof;
  }
  t.sync();
  DevDeepSync<DevTeam<NT, true>> sy{p.deep, p.deep_lim};
  while (sy.wait_request(t, lvl)) {
    deep_step<DevTeam<NT, true>, DevPolicy>(t, g, st, p.dist, lvl, sy);
    if (sy.error(t)) break;
  }
}

// One parDijkstra query on one team: heap state in LDS, levels 0..qlds-1 in
// the dynamic LDS block, deeper levels in the query's slice of the HBM arena.
// FULL: the large-heap form (staging for HBM merges, deep-level workers when
// p.deep is set); otherwise the plain form.  SPEC false: the plain rule only.
// Inlined into its kernel: called, it received the kernel's parameters as a
// copy in private (scratch) memory, read back with vector loads in the round
// loop, and the call's register conventions left 248-256 VGPRs and a 350-byte
// stack frame per lane (inlined: 126-193 VGPRs, no stack; learned ring 1.58
// -> 1.37 s, the paper's DAG 2.08 -> 1.68 s, plain ring 11.56 -> 10.56 s).
template <int NT, bool FULL, bool SPEC = true>
__device__ __attribute__((always_inline)) void sssp_query(DevTeam<NT, FULL>& t, HeapState PBH_LDS* st,
                                                         unsigned char* dyn, const SsspParams& p) {
  Geom g = p.g;
  const u64 nl = lvl_off(g.d, g.qlds);
  g.lk = reinterpret_cast<u64*>(dyn);
  g.lv = reinterpret_cast<u32*>(dyn + nl * sizeof(u64));
  // the LDS after the levels: staging for merges of HBM levels (between
  // Resolves it also holds a speculative round's list for its sort)
  if constexpr (FULL)
    if (p.stage) stage_setup(t, (unsigned char PBH_LDS*)(dyn + nl * 12u));
  if (threadIdx.x == 0) {
    state_init(st, g.d, g.q);
    st->prof_on = p.prof;
  }
  t.sync();
  SsspCounters c;
  using TT = DevTeam<NT, FULL>;
  if constexpr (FULL) {
    // the deep-level service is off when it gets no sync object
    DevDeepSync<TT> sy{p.deep, p.deep_lim};
    if (p.deep) {
      // the worker levels start as the front's own levels do (empty, pivots +inf)
      if (threadIdx.x == 0)
        for (int j = p.deep_lim; j < g.q; ++j) p.deep->L[j] = Lvl{0, 0, 0, 0, KINF, VINF, 0};
      sy.publish(t);
    }
    sssp_rounds<TT, DevPolicy, NoHook, DevDeepSync<TT>>(t, g, st, p.off, p.tg, p.wt, p.dist, p.n, p.src, p.sched,
                                                        p.spec, &c, NoHook(), p.deep ? &sy : nullptr,
                                                        p.deep ? p.deep_lim : MAXL);
  } else {
    sssp_rounds<TT, DevPolicy, NoHook, NoDeepSync, SPEC>(t, g, st, p.off, p.tg, p.wt, p.dist, p.n, p.src, p.sched,
                                                         p.spec, &c);
  }
  t.sync();
  if (threadIdx.x == 0) {
    SsspDevStats* o = p.stats;
    o->rounds = c.rounds;
    o->relax = c.relax;
    o->updates = c.updates;
    o->extracted = c.extracted;
    o->last_key = c.last_key;
    o->elems = st->elems;
    o->err = st->err;
    o->ell = st->ell;
    for (int i = 0; i < MAXL; ++i) o->resolves[i] = st->L[i].cnt;
    for (int i = 0; i < PROF_N; ++i) o->prof[i] = st->prof[i];
  }
  t.sync();
}

}  // namespace bkt
