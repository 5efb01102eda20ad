// Kernels of the parallel bucket heap and parDijkstra for gfx950.
//
//  k_sssp          one workgroup (one team) runs all parDijkstra rounds; the
//                  small top levels of the heap live in its LDS, deeper
//                  levels in HBM.  One kernel per query: no host round trip
//                  per round.
//  k_pbh_update    BulkUpdate of a host call (current keys + id bitmap,
//                  then pieces of at most d into S_0, each followed by
//                  Resolve(0) and the schedule).
//  k_pbh_extract   batched ExtractMin of a host call.
//  k_pbh_delete    Delete of a batch of ids of a host call.
//  k_fill_dist, k_check_csr, k_check_update: grid-wide helpers.
#include "pbh_launch.h"

namespace bkt {

// GPU placement of the heap: LDS levels, HBM levels and the state in LDS.
struct DevPolicy {
  using L = ArrT<u64 PBH_LDS*, u32 PBH_LDS*>;
  using G = ArrT<u64 PBH_GLB*, u32 PBH_GLB*>;
  using SP = HeapState PBH_LDS*;
  __device__ __forceinline__ static void on_resolve(const Geom&, SP, int, bool) {}
};

__global__ void k_fill_dist(u64* dist, u32 n, u32 src) {
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x)
    dist[i] = (i == src) ? 0ull : KINF;
}

// offsets[0] == 0, non-decreasing, offsets[n] == m, targets < n; max degree.
__global__ void k_check_csr(const u64* off, const u32* tg, u32 n, u64 m, CsrCheck* out) {
  u64 bad = 0, md = 0;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  const u64 t0 = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  for (u64 u = t0; u < n; u += stride) {
    u64 a = off[u], b = off[u + 1];
    if (b < a) bad = 1;
    else md = (b - a) > md ? (b - a) : md;
  }
  if (t0 == 0 && (off[0] != 0 || off[n] != m)) bad = 1;
  for (u64 e = t0; e < m; e += stride)
    if (tg[e] >= n) bad = 1;
  if (bad) atomicOr(&out->bad, 1ull);
  if (md) atomicMax(&out->maxdeg, md);
}

__global__ void k_zero_u64(u64* p, u64 n) {
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x) p[i] = 0;
}

__global__ void k_check_update(const u64* keys, const u32* ids, u64 count, u32 id_cap, u64* bad) {
  u64 b = 0;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (u64)gridDim.x * blockDim.x)
    if (ids[i] >= id_cap || (keys && keys[i] == KINF)) b = 1;
  if (b) atomicOr(bad, 1ull);
}

// Synchronisation of the deep-level service (pbh_core.h) between workgroups:
// counters in the control block, read and written with agent-scope atomics
// (the XCDs' L2 caches are not coherent for plain accesses).  Before a team
// counts a request or a completion, every thread waits for its own stores
// and thread 0 issues an agent-scope release, so the level arrays and states
// it wrote are visible to the team that sees the count; a waiting team's
// thread 0 issues an agent-scope acquire once the condition holds.  Waits
// poll with s_sleep and give up at once when another team has failed, or
// with E_TIMEOUT after DEEP_TIMEOUT of the 100 MHz clock (a Resolve never takes
// that long) -- or, for a worker waiting for its next request (which may not
// come for the rest of a long run), after DEEP_RUN_LIMIT.
constexpr u64 DEEP_TIMEOUT = 1000000000ull;      // 10 s
constexpr u64 DEEP_RUN_LIMIT = 30000000000ull;   // 300 s

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
  __device__ bool spin(const T& t, F ready, bool leave_ok, u64 limit = DEEP_TIMEOUT) const {
    u64 r = 1;
    if (t.tid() == 0) {
      const u64 t0 = __builtin_amdgcn_s_memrealtime();
      while (!ready()) {
        if (ld((const u32*)&c->err) || (leave_ok && ld(&c->exit))) {
          r = 0;
          break;
        }
        if (__builtin_amdgcn_s_memrealtime() - t0 > limit) {
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
    return spin(t, [&] { return ld(&c->done[j]) != ld(&c->req[j]); }, true, DEEP_RUN_LIMIT);
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
  __device__ void leave(const T& t) const {
    release(t);
    if (t.tid() == 0) __hip_atomic_store((u32 PBH_GLB*)&c->exit, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    t.sync();
  }
};

// A deep-level worker: Resolve(lvl) whenever the level above asks, until the
// front has finished (or any team has failed).
template <int NT>
__device__ void deep_worker(DevTeam<NT>& t, HeapState PBH_LDS* st, unsigned char* dyn, const SsspParams& p,
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
  DevDeepSync<DevTeam<NT>> sy{p.deep, p.deep_lim};
  while (sy.wait_request(t, lvl)) {
    deep_step<DevTeam<NT>, DevPolicy>(t, g, st, p.dist, lvl, sy);
    if (sy.error(t)) break;
  }
}

// One parDijkstra query on one team: heap state in LDS, levels 0..qlds-1 in
// the dynamic LDS block, deeper levels in the query's slice of the HBM arena.
template <int NT>
__device__ void sssp_query(DevTeam<NT>& t, HeapState PBH_LDS* st, unsigned char* dyn, const SsspParams& p) {
  Geom g = p.g;
  const u64 nl = lvl_off(g.d, g.qlds);
  g.lk = reinterpret_cast<u64*>(dyn);
  g.lv = reinterpret_cast<u32*>(dyn + nl * sizeof(u64));
  // the LDS after the levels: staging for merges of HBM levels (between
  // Resolves it also holds a speculative round's list for its sort)
  if (p.stage) stage_setup(t, (unsigned char PBH_LDS*)(dyn + nl * 12u));
  if (threadIdx.x == 0) {
    state_init(st, g.d, g.q);
    st->prof_on = p.prof;
  }
  t.sync();
  SsspCounters c;
  // One instantiation of the round loop serves both cases (with and without
  // deep-level workers); the service is off when it gets no sync object.
  DevDeepSync<DevTeam<NT>> sy{p.deep, p.deep_lim};
  if (p.deep) {
    // the worker levels start as the front's own levels do (empty, pivots +inf)
    if (threadIdx.x == 0)
      for (int j = p.deep_lim; j < g.q; ++j) p.deep->L[j] = Lvl{0, 0, 0, 0, KINF, VINF, 0};
    sy.publish(t);
  }
  sssp_rounds<DevTeam<NT>, DevPolicy, NoHook, DevDeepSync<DevTeam<NT>>>(
      t, g, st, p.off, p.tg, p.wt, p.dist, p.n, p.src, p.sched, p.spec, &c, NoHook(), p.deep ? &sy : nullptr,
      p.deep ? p.deep_lim : MAXL);
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

// Block 0 runs the rounds; with deep-level workers, block b >= 1 is the
// worker of level deep_lim + b - 1.
template <int NT>
__global__ __launch_bounds__(NT) void k_sssp(SsspParams p) {
  extern __shared__ __align__(16) unsigned char dyn[];
  __shared__ TeamShared<NT / 64> ts;
  __shared__ HeapState st_lds;
  DevTeam<NT> t{(TeamShared<NT / 64> PBH_LDS*)&ts};
  if (blockIdx.x == 0)
    sssp_query(t, (HeapState PBH_LDS*)&st_lds, dyn, p);
  else if (p.deep && p.deep_lim + (int)blockIdx.x - 1 < p.g.q)
    deep_worker(t, (HeapState PBH_LDS*)&st_lds, dyn, p, p.deep_lim + (int)blockIdx.x - 1);
}

// Many independent queries in one launch: persistent teams take queries from
// a counter (queries are ordered by decreasing size, so the long ones start
// first); every team leaves once the counter passes the last query.
template <int NT>
__global__ __launch_bounds__(NT) void k_sssp_multi(const SsspParams* qs, u32 nq, u32* counter) {
  extern __shared__ __align__(16) unsigned char dyn[];
  __shared__ TeamShared<NT / 64> ts;
  __shared__ HeapState st_lds;
  __shared__ u32 qnext;
  DevTeam<NT> t{(TeamShared<NT / 64> PBH_LDS*)&ts};
  for (;;) {
    if (threadIdx.x == 0) qnext = atomicAdd(counter, 1u);
    t.sync();
    const u32 qi = qnext;
    t.sync();
    if (qi >= nq) break;
    const SsspParams p = qs[qi];
    sssp_query(t, (HeapState PBH_LDS*)&st_lds, dyn, p);
  }
}

// dist = INF except dist[src] = 0, for every query (blockIdx.y = query).
__global__ void k_fill_multi(const SsspParams* qs, u32 nq, u32* counter) {
  const u32 qi = blockIdx.y;
  if (qi == 0 && blockIdx.x == 0 && threadIdx.x == 0) *counter = 0;
  if (qi >= nq) return;
  u64* dist = qs[qi].dist;
  const u32 n = qs[qi].n, s = qs[qi].src;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x)
    dist[i] = (i == s) ? 0ull : KINF;
}

template <int NT>
__device__ void load_state(DevTeam<NT>& t, HeapState PBH_LDS* st, const HeapState* gst) {
  const u32* s = reinterpret_cast<const u32*>(gst);
  u32 PBH_LDS* d = reinterpret_cast<u32 PBH_LDS*>(st);
  for (u32 i = threadIdx.x; i < sizeof(HeapState) / 4; i += NT) d[i] = s[i];
  t.sync();
}

template <int NT>
__device__ void store_state(DevTeam<NT>& t, const HeapState PBH_LDS* st, HeapState* gst) {
  t.sync();
  const u32 PBH_LDS* s = reinterpret_cast<const u32 PBH_LDS*>(st);
  u32* d = reinterpret_cast<u32*>(gst);
  for (u32 i = threadIdx.x; i < sizeof(HeapState) / 4; i += NT) d[i] = s[i];
}

template <int NT>
__global__ __launch_bounds__(NT) void k_pbh_update(PbhParams p) {
  __shared__ TeamShared<NT / 64> ts;
  __shared__ HeapState st_lds;
  HeapState PBH_LDS* st = (HeapState PBH_LDS*)&st_lds;
  DevTeam<NT> t{(TeamShared<NT / 64> PBH_LDS*)&ts};
  load_state(t, st, p.gst);
  pbh_update_body<DevTeam<NT>, DevPolicy>(t, p.g, st, p);
  store_state(t, st, p.gst);
}

template <int NT>
__global__ __launch_bounds__(NT) void k_pbh_delete(PbhParams p) {
  __shared__ TeamShared<NT / 64> ts;
  __shared__ HeapState st_lds;
  HeapState PBH_LDS* st = (HeapState PBH_LDS*)&st_lds;
  DevTeam<NT> t{(TeamShared<NT / 64> PBH_LDS*)&ts};
  load_state(t, st, p.gst);
  pbh_delete_body<DevTeam<NT>, DevPolicy>(t, p.g, st, p);
  store_state(t, st, p.gst);
}

template <int NT>
__global__ __launch_bounds__(NT) void k_pbh_extract(PbhParams p) {
  __shared__ TeamShared<NT / 64> ts;
  __shared__ HeapState st_lds;
  HeapState PBH_LDS* st = (HeapState PBH_LDS*)&st_lds;
  DevTeam<NT> t{(TeamShared<NT / 64> PBH_LDS*)&ts};
  load_state(t, st, p.gst);
  pbh_extract_body<DevTeam<NT>, DevPolicy>(t, p.g, st, p);
  store_state(t, st, p.gst);
}

static int grid_for(u64 work, int block) {
  u64 g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 4096) g = 4096;
  return (int)g;
}

hipError_t launch_fill_dist(u64* dist, u32 n, u32 src, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_dist, dim3(grid_for(n, 256)), dim3(256), 0, s, dist, n, src);
  return hipGetLastError();
}

hipError_t launch_zero_u64(u64* p, u64 n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_check_csr(const u64* off, const u32* tg, u32 n, u64 m, CsrCheck* out, hipStream_t s) {
  hipLaunchKernelGGL(k_check_csr, dim3(grid_for(m > n ? m : n, 256)), dim3(256), 0, s, off, tg, n, m, out);
  return hipGetLastError();
}

hipError_t launch_check_update(const u64* keys, const u32* ids, u64 count, u32 id_cap, u64* bad,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_check_update, dim3(grid_for(count, 256)), dim3(256), 0, s, keys, ids, count, id_cap, bad);
  return hipGetLastError();
}

size_t sssp_static_lds(int team) {
  size_t hs = sizeof(HeapState);
  switch (team) {
    case 64: return sizeof(TeamShared<1>) + hs;
    case 256: return sizeof(TeamShared<4>) + hs;
    default: return sizeof(TeamShared<16>) + hs;
  }
}

template <int NT>
static hipError_t sssp_go(const SsspParams& p, size_t lds, hipStream_t s) {
  if (lds > 65536 - sssp_static_lds(NT)) {
    hipError_t e = hipFuncSetAttribute((const void*)k_sssp<NT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (p.deep) {
    // the round loop and one workgroup per worker level, resident together
    SsspParams a = p;
    void* args[] = {&a};
    return hipLaunchCooperativeKernel((const void*)k_sssp<NT>, dim3(1 + p.g.q - p.deep_lim), dim3(NT), args, lds, s);
  }
  hipLaunchKernelGGL(k_sssp<NT>, dim3(1), dim3(NT), lds, s, p);
  return hipGetLastError();
}

template <int NT>
static hipError_t multi_go(const SsspParams* qs, u32 nq, u32* counter, size_t lds, int grid, hipStream_t s) {
  if (lds > 65536 - sssp_static_lds(NT)) {
    hipError_t e =
        hipFuncSetAttribute((const void*)k_sssp_multi<NT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_sssp_multi<NT>, dim3(grid), dim3(NT), lds, s, qs, nq, counter);
  return hipGetLastError();
}

hipError_t launch_sssp_multi(int team, const SsspParams* qs, u32 nq, u32* counter, size_t lds, int grid,
                             hipStream_t s) {
  switch (team) {
    case 64: return multi_go<64>(qs, nq, counter, lds, grid, s);
    case 256: return multi_go<256>(qs, nq, counter, lds, grid, s);
    case 1024: return multi_go<1024>(qs, nq, counter, lds, grid, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fill_multi(const SsspParams* qs, u32 nq, u32 maxn, u32* counter, hipStream_t s) {
  u32 bx = (maxn + 255) / 256;
  bx = bx < 1 ? 1 : (bx > 1024 ? 1024 : bx);
  hipLaunchKernelGGL(k_fill_multi, dim3(bx, nq > 0 ? nq : 1), dim3(256), 0, s, qs, nq, counter);
  return hipGetLastError();
}

int multi_occupancy(int team, size_t lds) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (team) {
    case 64: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sssp_multi<64>, 64, lds); break;
    case 256: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sssp_multi<256>, 256, lds); break;
    case 1024: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sssp_multi<1024>, 1024, lds); break;
  }
  return e == hipSuccess ? nb : 0;
}

hipError_t launch_sssp(int team, const SsspParams& p, size_t lds_bytes, hipStream_t s) {
  switch (team) {
    case 64: return sssp_go<64>(p, lds_bytes, s);
    case 256: return sssp_go<256>(p, lds_bytes, s);
    case 1024: return sssp_go<1024>(p, lds_bytes, s);
    default: return hipErrorInvalidValue;
  }
}

// The round loop's MLP inference (mlp_forward) on given feature rows, one
// team per row: y[r] = the model output for features X[8r .. 8r+7].
template <int NT>
__global__ __launch_bounds__(NT) void k_mlp_infer(const float* X, u32 n, const float* blob, float* y) {
  __shared__ TeamShared<NT / 64> ts;
  DevTeam<NT> t{(TeamShared<NT / 64> PBH_LDS*)&ts};
  const u32 r = blockIdx.x;
  if (r >= n) return;
  float f[NFEAT];
#pragma unroll
  for (int i = 0; i < NFEAT; ++i) f[i] = X[(u64)r * NFEAT + i];
  const float v = mlp_forward(t, blob, f);
  if (threadIdx.x == 0) y[r] = v;
}

hipError_t launch_mlp_infer(int team, const float* X, u32 n, const float* blob, float* y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (team == 64)
    hipLaunchKernelGGL(k_mlp_infer<64>, dim3(n), dim3(64), 0, s, X, n, blob, y);
  else
    hipLaunchKernelGGL(k_mlp_infer<256>, dim3(n), dim3(256), 0, s, X, n, blob, y);
  return hipGetLastError();
}

hipError_t launch_pbh_update(const PbhParams& p, hipStream_t s) {
  hipLaunchKernelGGL(k_pbh_update<1024>, dim3(1), dim3(1024), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_pbh_delete(const PbhParams& p, hipStream_t s) {
  hipLaunchKernelGGL(k_pbh_delete<1024>, dim3(1), dim3(1024), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_pbh_extract(const PbhParams& p, hipStream_t s) {
  hipLaunchKernelGGL(k_pbh_extract<1024>, dim3(1), dim3(1024), 0, s, p);
  return hipGetLastError();
}

}  // namespace bkt
