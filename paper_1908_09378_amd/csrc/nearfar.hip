// Near-Far, a GPU form of Delta-stepping (Meyer and Sanders; Davidson et al.,
// IPDPS 2014): the comparison family of the paper (Sections 1.1 and 4.2).
//
// Two buckets: the "near" frontier holds vertices whose tentative distance is
// below a threshold T, the "far" pile the rest.  A relax phase scans every
// out-edge of the near frontier (atomicMin on dist); an improved vertex goes
// to the next near frontier if its new distance is below T, else to the far
// pile.  When the near frontier runs empty, T grows by Delta (or jumps to the
// first Delta step past the smallest far key) and the far vertices now below
// T become the near frontier; vertices whose distance improved since they
// were filed are re-scanned, so the result is exact for any Delta.
//
// One persistent cooperative launch over the whole GPU (one workgroup per
// CU): phases are separated by a software grid barrier whose last arriving
// workgroup also does the bookkeeping (queue sizes, next phase, T) while the
// others wait.  Every word workgroups hand to each other is written and read
// with agent-scope atomics (the XCDs' L2 caches are not coherent for plain
// stores); every wait is bounded by the real-time clock and gives up with an
// error flag, and a phase limit ends a run that would not terminate.
//
// Frontier vertices of low degree are scanned by groups of G lanes (G close
// to the mean degree), vertices of high degree by every workgroup at once.
// Pushes are deduplicated per phase by stamping vertices with the phase
// number (near) or the far pile's epoch (far), so each queue holds at most n.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "../../include/pbh.h"
#include "pbh_team.h"

namespace bkt {
namespace nf {

constexpr u64 KINF = ~0ull;
constexpr u32 NONE = ~0u;
constexpr int NT = 512;          // threads per workgroup
constexpr u32 HEAVY = 1024;      // out-degree above which a vertex is scanned by the whole grid
constexpr u64 TIMEOUT_TICKS = 2000000000ull;  // 20 s of the 100 MHz real-time clock
constexpr u64 RUN_LIMIT_TICKS = 12000000000ull;  // 120 s: a run that long is stopped

enum { RELAX = 0, SPLIT = 1, DONE = 2 };
enum { ERR_TIMEOUT = 1, ERR_OVERFLOW = 2, ERR_PHASES = 4 };

// Phase descriptor, written by the barrier's leader.
struct Phase {
  u32 mode;
  u32 src, dst;     // near queues read (relax) and written
  u32 nl, nh;       // relax: light and heavy vertices in queue src
  u32 fsrc, fdst;   // far piles: split reads fsrc; relax and split append to fdst
  u32 nf;           // split: entries of fsrc
  u32 phase;        // stamp of near pushes in this phase
  u32 epoch;        // stamp of far pushes
  u64 T;            // threshold
};

struct Ctl {
  u32 arrive, gen;
  u32 err;
  u32 cl[2], ch[2];  // near queue sizes (light, heavy)
  u32 cf[2];         // far pile sizes
  u64 fmin[2];       // smallest key filed in each far pile
  u64 relax;         // edges scanned
  u64 t_start;       // real-time clock at the first barrier
  u32 phases, splits;
  u32 nq;            // leader: near queue the current phase writes
  u32 fcur;          // leader: far pile the current phase appends to
  u32 pad_[2];
  Phase ph;
};

struct Args {
  const u64* off;
  const u32* tg;
  const u32* wt;
  u64* dist;
  u32 n;
  u64 delta;
  u32 glog;         // light vertices: groups of 2^glog lanes
  u32* ql[2];       // near queues, light vertices
  u32* qh[2];       // near queues, heavy vertices
  u32* far[2];      // far piles
  u32* nstamp;      // per vertex: phase of its last near push
  u32* fstamp;      // per vertex: epoch of its last far filing
  u64* done_at;     // per vertex: the distance at which its edges were last scanned
  u32 cap;          // capacity of every queue and pile
  u32 max_phases;
  Ctl* c;
};

__device__ __forceinline__ u32 ld32(const u32* p) {
  return __hip_atomic_load((const u32 PBH_GLB*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u64 ld64(const u64* p) {
  return __hip_atomic_load((const u64 PBH_GLB*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st32(u32* p, u32 v) {
  __hip_atomic_store((u32 PBH_GLB*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st64(u64* p, u64 v) {
  __hip_atomic_store((u64 PBH_GLB*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u32 xchg32(u32* p, u32 v) {
  return __hip_atomic_exchange((u32 PBH_GLB*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u64 xchg64(u64* p, u64 v) {
  return __hip_atomic_exchange((u64 PBH_GLB*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u32 add32(u32* p, u32 v) {
  return __hip_atomic_fetch_add((u32 PBH_GLB*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u64 min64(u64* p, u64 v) {
  return __hip_atomic_fetch_min((u64 PBH_GLB*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Appends one element per lane with p set to the queue behind ctr: one atomic
// per wavefront; returns this lane's slot (meaningful where p is set).
__device__ __forceinline__ u32 wave_slot(u32* ctr, bool p) {
  const u64 m = __ballot(p);
  if (m == 0) return 0;
  const int lead = __builtin_ctzll(m);
  u32 base = 0;
  if ((int)(threadIdx.x & 63) == lead) base = add32(ctr, (u32)__builtin_popcountll(m));
  base = __shfl(base, lead, 64);
  return base + __builtin_amdgcn_mbcnt_hi((u32)(m >> 32), __builtin_amdgcn_mbcnt_lo((u32)m, 0u));
}

// Files vertex v with key `key` (improved in this phase): near (below T) or
// far, each at most once per phase / epoch.
__device__ __forceinline__ void file(const Args& a, const Phase& ph, bool imp, u32 v, u64 key) {
  const bool near = imp && key < ph.T;
  const bool fresh_near = near && xchg32(a.nstamp + v, ph.phase) != ph.phase;
  const bool fresh_far = imp && !near && xchg32(a.fstamp + v, ph.epoch) != ph.epoch;
  bool heavy = false;
  if (fresh_near) heavy = a.off[v + 1] - a.off[v] > HEAVY;
  const u32 sl = wave_slot(&a.c->cl[ph.dst], fresh_near && !heavy);
  const u32 sh = wave_slot(&a.c->ch[ph.dst], fresh_near && heavy);
  const u32 sf = wave_slot(&a.c->cf[ph.fdst], fresh_far);
  if (fresh_near) {
    const u32 s = heavy ? sh : sl;
    if (s < a.cap)
      st32((heavy ? a.qh[ph.dst] : a.ql[ph.dst]) + s, v);
    else
      __hip_atomic_fetch_or((u32 PBH_GLB*)&a.c->err, (u32)ERR_OVERFLOW, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (fresh_far) {
    if (sf < a.cap)
      st32(a.far[ph.fdst] + sf, v);
    else
      __hip_atomic_fetch_or((u32 PBH_GLB*)&a.c->err, (u32)ERR_OVERFLOW, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    min64(&a.c->fmin[ph.fdst], key);
  }
}

// Relaxes edge e out of a vertex at distance du; files an improved target.
__device__ __forceinline__ void relax_edge(const Args& a, const Phase& ph, bool in, u64 e, u64 du) {
  u32 v = 0;
  u64 cand = 0;
  bool imp = false;
  if (in) {
    v = a.tg[e];
    cand = du + (u64)a.wt[e];
    imp = cand < min64(a.dist + v, cand);
  }
  file(a, ph, imp, v, cand);
}

// Leader of a grid barrier: turns the queue sizes of the phase that ended
// into the next phase's descriptor (every other workgroup is waiting).
__device__ void lead(const Args& a, Phase& ph) {
  // (the leader changes from phase to phase, so even its own words go
  // through agent-scope atomics)
  Ctl* c = a.c;
  const u32 d = ld32(&c->nq);
  const u32 nl = ld32(&c->cl[d]), nh = ld32(&c->ch[d]);
  const u32 phases = ld32(&c->phases) + 1;
  st32(&c->phases, phases);
  const u64 now = __builtin_amdgcn_s_memrealtime();
  u64 t0 = ld64(&c->t_start);
  if (t0 == 0) st64(&c->t_start, t0 = now);
  if (phases > a.max_phases || now - t0 > RUN_LIMIT_TICKS) {
    __hip_atomic_fetch_or((u32 PBH_GLB*)&c->err, (u32)ERR_PHASES, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    ph.mode = DONE;
    return;
  }
  ph.phase += 1;
  if (nl + nh > 0) {
    ph.mode = RELAX;
    ph.src = d;
    ph.dst = d ^ 1;
    ph.nl = nl < a.cap ? nl : a.cap;
    ph.nh = nh < a.cap ? nh : a.cap;
    st32(&c->cl[d ^ 1], 0u);
    st32(&c->ch[d ^ 1], 0u);
    st32(&c->nq, d ^ 1);
    return;
  }
  const u32 f = ld32(&c->fcur);
  const u32 nf = ld32(&c->cf[f]);
  if (nf == 0) {
    ph.mode = DONE;
    return;
  }
  // Next threshold: one Delta further, or the first multiple of Delta past
  // the smallest key filed in the far pile if that is further.
  const u64 fm = ld64(&c->fmin[f]);
  u64 t = ph.T + a.delta < ph.T ? KINF : ph.T + a.delta;
  if (fm != KINF) {
    const u64 j = (fm / a.delta + 1) * a.delta;
    const u64 jt = j < fm ? KINF : j;  // saturate
    t = jt > t ? jt : t;
  }
  ph.T = t;
  ph.mode = SPLIT;
  ph.dst = d;  // empty: the relax phase that ended filed nothing near
  ph.fsrc = f;
  ph.fdst = f ^ 1;
  ph.nf = nf < a.cap ? nf : a.cap;
  ph.epoch += 1;
  st32(&c->cf[f ^ 1], 0u);
  st64(&c->fmin[f ^ 1], KINF);
  st32(&c->fcur, f ^ 1);
  st32(&c->splits, ld32(&c->splits) + 1);
}

// Grid barrier.  Every thread first waits for its own memory operations;
// one arrival per workgroup; the last one runs lead() and bumps the
// generation the others spin on.  Returns false once the run has failed.
__device__ bool grid_sync(const Args& a, Phase& ph, Phase* sph, u32* sflag) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  Ctl* c = a.c;
  if (threadIdx.x == 0) {
    const u32 g = ld32(&c->gen);
    const u32 prev = add32(&c->arrive, 1u);
    if (prev == gridDim.x - 1) {
      st32(&c->arrive, 0u);
      lead(a, ph);
      Phase* gp = &c->ph;
      u32* src = reinterpret_cast<u32*>(&ph);
      u32* dstp = reinterpret_cast<u32*>(gp);
      for (u32 i = 0; i < sizeof(Phase) / 4; ++i) st32(dstp + i, src[i]);
      __builtin_amdgcn_s_waitcnt(0);
      st32(&c->gen, g + 1);
    } else {
      const u64 t0 = __builtin_amdgcn_s_memrealtime();
      while (ld32(&c->gen) == g) {
        if (ld32(&c->err)) break;
        if (__builtin_amdgcn_s_memrealtime() - t0 > TIMEOUT_TICKS) {
          __hip_atomic_fetch_or((u32 PBH_GLB*)&c->err, (u32)ERR_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      const u32* gp = reinterpret_cast<const u32*>(&c->ph);
      u32* d = reinterpret_cast<u32*>(&ph);
      for (u32 i = 0; i < sizeof(Phase) / 4; ++i) d[i] = ld32(gp + i);
    }
    *sph = ph;
    *sflag = ld32(&c->err);
  }
  __syncthreads();
  ph = *sph;
  return *sflag == 0;
}

__global__ __launch_bounds__(NT) void k_nearfar(Args a) {
  __shared__ Phase sph;
  __shared__ u32 sflag;
  Phase ph;
  if (threadIdx.x == 0) {
    const u32* gp = reinterpret_cast<const u32*>(&a.c->ph);
    u32* d = reinterpret_cast<u32*>(&sph);
    for (u32 i = 0; i < sizeof(Phase) / 4; ++i) d[i] = ld32(gp + i);
  }
  __syncthreads();
  ph = sph;
  const u32 G = 1u << a.glog;
  const u32 gtid = blockIdx.x * NT + threadIdx.x;
  const u32 nthreads = gridDim.x * NT;
  const u32 sub = gtid >> a.glog, nsub = nthreads >> a.glog, lig = threadIdx.x & (G - 1);
  u64 scanned = 0;
  while (ph.mode != DONE) {
    if (ph.mode == RELAX) {
      // light vertices: one group of G lanes per vertex, striding its edges
      const u32 rounds_l = (ph.nl + nsub - 1) / nsub;
      for (u32 r = 0; r < rounds_l; ++r) {
        const u32 j = r * nsub + sub;
        bool have = j < ph.nl;
        const u32 u = have ? ld32(a.ql[ph.src] + j) : 0u;
        const u64 du = have ? ld64(a.dist + u) : 0ull;
        // a vertex already scanned at this distance (filed twice) is skipped
        if (have && lig == 0) have = xchg64(a.done_at + u, du) != du;
        have = __shfl(have ? 1 : 0, (int)((threadIdx.x & 63) & ~(G - 1)), 64) != 0;
        const u64 e0 = have ? a.off[u] : 0ull, e1 = have ? a.off[u + 1] : 0ull;
        const u64 deg = e1 - e0;
        scanned += lig == 0 ? deg : 0;
        // every lane of the wavefront runs the same number of steps (the
        // largest degree in the wavefront), so the ballots stay convergent
        u64 steps = (deg + G - 1) / G;
        for (int o = 32; o > 0; o >>= 1) {
          const u64 s2 = __shfl_xor(steps, o, 64);
          steps = s2 > steps ? s2 : steps;
        }
        for (u64 s = 0; s < steps; ++s) {
          const u64 e = e0 + s * G + lig;
          relax_edge(a, ph, e < e1, e, du);
        }
      }
      // heavy vertices: every workgroup takes a share of each one's edges
      // (always scanned: every workgroup would have to agree on a skip)
      for (u32 h = 0; h < ph.nh; ++h) {
        const u32 u = ld32(a.qh[ph.src] + h);
        const u64 du = ld64(a.dist + u);
        const u64 e0 = a.off[u], e1 = a.off[u + 1];
        if (gtid == 0) scanned += e1 - e0;
        const u64 span = e1 - e0;
        const u64 steps = (span + nthreads - 1) / nthreads;
        for (u64 s = 0; s < steps; ++s) {
          const u64 e = e0 + s * nthreads + gtid;
          relax_edge(a, ph, e < e1, e, du);
        }
      }
    } else {  // SPLIT: far vertices now below T become the near frontier
      const u32 rounds_f = (ph.nf + nthreads - 1) / nthreads;
      for (u32 r = 0; r < rounds_f; ++r) {
        const u32 j = r * nthreads + gtid;
        const bool have = j < ph.nf;
        const u32 v = have ? ld32(a.far[ph.fsrc] + j) : 0u;
        const u64 dv = have ? ld64(a.dist + v) : KINF;
        file(a, ph, have, v, dv);
      }
    }
    if (!grid_sync(a, ph, &sph, &sflag)) break;
  }
  if (scanned) __hip_atomic_fetch_add((u64 PBH_GLB*)&a.c->relax, scanned, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_nf_init(u64* dist, u32* nstamp, u32* fstamp, u64* done_at, u32 n, u32 src) {
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x) {
    dist[i] = i == src ? 0ull : KINF;
    nstamp[i] = NONE;
    fstamp[i] = NONE;
    done_at[i] = KINF;
  }
}

// Maximum out-degree, edge-weight sum and CSR validity (one pass).
struct Scan {
  u64 bad, maxdeg, wsum;
};
__global__ void k_nf_scan(const u64* off, const u32* tg, const u32* wt, u32 n, u64 m, Scan* out) {
  u64 bad = 0, md = 0, ws = 0;
  const u64 stride = (u64)gridDim.x * blockDim.x, t0 = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  for (u64 u = t0; u < n; u += stride) {
    const u64 a = off[u], b = off[u + 1];
    if (b < a)
      bad = 1;
    else
      md = b - a > md ? b - a : md;
  }
  if (t0 == 0 && (off[0] != 0 || off[n] != m)) bad = 1;
  for (u64 e = t0; e < m; e += stride) {
    if (tg[e] >= n) bad = 1;
    ws += wt[e];
  }
  if (bad) atomicOr(&out->bad, 1ull);
  if (md) atomicMax(&out->maxdeg, md);
  if (ws) atomicAdd(&out->wsum, ws);
}

thread_local char g_nferr[256] = "";
std::mutex g_nf_mu;

int nf_fail(int code, const char* msg) {
  snprintf(g_nferr, sizeof g_nferr, "%s", msg);
  return code;
}

}  // namespace nf
}  // namespace bkt

using namespace bkt;
using namespace bkt::nf;

#define NFCHK(expr)                                                                            \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) {                                                                    \
      snprintf(g_nferr, sizeof g_nferr, "%s: %s", #expr, hipGetErrorString(e_));               \
      rc = e_ == hipErrorOutOfMemory ? PBH_ENOMEM : PBH_EDEVICE;                               \
      goto out;                                                                                \
    }                                                                                          \
  } while (0)

extern "C" {

const char* sssp_nearfar_last_error(void) { return g_nferr; }

int sssp_nearfar(const uint64_t* offsets, const uint32_t* targets, const uint32_t* weights, uint32_t n,
                 uint64_t m, uint32_t source, uint64_t* dist_out, uint64_t delta, sssp_nearfar_stats* stats,
                 void* stream) {
  if (stats) std::memset(stats, 0, sizeof *stats);
  if (!offsets || !dist_out || (m > 0 && (!targets || !weights))) return nf_fail(PBH_EINVAL, "NULL array argument");
  if (n == 0 || source >= n) return nf_fail(PBH_EINVAL, "n == 0 or source >= n");
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(g_nf_mu);
  int rc = PBH_OK;
  unsigned char* buf = nullptr;
  Scan sc{};
  Ctl ctl{};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const u64 cap = n;
  const u64 bytes = 256 + ((sizeof(Ctl) + 255) / 256) * 256 + 8ull * n + 4ull * (6 * cap + 2ull * n);
  Args a{};
  int dev = 0, cus = 0, occ = 0;
  float ms = 0.f;
  u64 avgdeg;
  NFCHK(hipMalloc(&buf, bytes));
  {
    Scan* dscan = reinterpret_cast<Scan*>(buf);
    Ctl* dctl = reinterpret_cast<Ctl*>(buf + 256);
    u32* q = reinterpret_cast<u32*>(buf + 256 + ((sizeof(Ctl) + 255) / 256) * 256);
    NFCHK(hipMemsetAsync(dscan, 0, sizeof(Scan), s));
    hipLaunchKernelGGL(k_nf_scan, dim3(1024), dim3(256), 0, s, (const u64*)offsets, targets, weights, n, m, dscan);
    NFCHK(hipGetLastError());
    NFCHK(hipMemcpyAsync(&sc, dscan, sizeof sc, hipMemcpyDeviceToHost, s));
    NFCHK(hipStreamSynchronize(s));
    if (sc.bad) {
      rc = nf_fail(PBH_EINVAL, "malformed CSR (offsets or targets)");
      goto out;
    }
    avgdeg = m / n ? m / n : 1;
    if (delta == 0) {
      // Davidson et al.'s choice: mean weight x wavefront width / mean degree
      const u64 wmean = m ? (sc.wsum + m - 1) / m : 1;
      delta = std::max<u64>(1, wmean * 64 / avgdeg);
    }
    a.off = (const u64*)offsets;
    a.tg = targets;
    a.wt = weights;
    a.dist = (u64*)dist_out;
    a.n = n;
    a.delta = delta;
    a.glog = avgdeg <= 6 ? 2 : avgdeg <= 12 ? 3 : avgdeg <= 24 ? 4 : avgdeg <= 48 ? 5 : 6;
    a.done_at = reinterpret_cast<u64*>(q);
    q += 2ull * n;
    for (int i = 0; i < 2; ++i) {
      a.ql[i] = q + (u64)i * cap;
      a.qh[i] = q + (u64)(2 + i) * cap;
      a.far[i] = q + (u64)(4 + i) * cap;
    }
    a.nstamp = q + 6 * cap;
    a.fstamp = q + 6 * cap + n;
    a.cap = (u32)cap;
    a.max_phases = (u32)std::min<u64>(0xFFFFFFF0ull, 64ull * n + (1ull << 20));
    a.c = dctl;
    hipLaunchKernelGGL(k_nf_init, dim3(std::min<u32>(4096, (n + 255) / 256)), dim3(256), 0, s, (u64*)dist_out,
                       a.nstamp, a.fstamp, a.done_at, n, source);
    NFCHK(hipGetLastError());
    // the source is the first near frontier (heavy if its degree is)
    u64 so[2];
    NFCHK(hipMemcpyAsync(so, offsets + source, sizeof so, hipMemcpyDeviceToHost, s));
    NFCHK(hipStreamSynchronize(s));
    const bool heavy = so[1] - so[0] > HEAVY;
    ctl.cl[0] = heavy ? 0 : 1;
    ctl.ch[0] = heavy ? 1 : 0;
    ctl.fmin[0] = ctl.fmin[1] = KINF;
    ctl.nq = 1;
    ctl.fcur = 0;
    ctl.ph.mode = RELAX;
    ctl.ph.src = 0;
    ctl.ph.dst = 1;
    ctl.ph.nl = heavy ? 0 : 1;
    ctl.ph.nh = heavy ? 1 : 0;
    ctl.ph.fsrc = 1;
    ctl.ph.fdst = 0;
    ctl.ph.phase = 0;
    ctl.ph.epoch = 0;
    ctl.ph.T = delta;
    NFCHK(hipMemcpyAsync(dctl, &ctl, sizeof ctl, hipMemcpyHostToDevice, s));
    const u32 srcv = source;
    NFCHK(hipMemcpyAsync(heavy ? a.qh[0] : a.ql[0], &srcv, sizeof(u32), hipMemcpyHostToDevice, s));
    NFCHK(hipGetDevice(&dev));
    NFCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    NFCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_nearfar, NT, 0));
    if (occ < 1) {
      rc = nf_fail(PBH_EDEVICE, "the near-far kernel cannot be resident");
      goto out;
    }
    NFCHK(hipEventCreate(&e0));
    NFCHK(hipEventCreate(&e1));
    NFCHK(hipEventRecord(e0, s));
    {
      void* args[] = {&a};
      NFCHK(hipLaunchCooperativeKernel((const void*)k_nearfar, dim3(cus), dim3(NT), args, 0, s));
    }
    NFCHK(hipEventRecord(e1, s));
    NFCHK(hipMemcpyAsync(&ctl, dctl, sizeof ctl, hipMemcpyDeviceToHost, s));
    NFCHK(hipStreamSynchronize(s));
    NFCHK(hipEventElapsedTime(&ms, e0, e1));
    if (ctl.err) {
      rc = nf_fail(ctl.err & ERR_TIMEOUT ? PBH_ETIMEOUT : PBH_EINTERNAL,
                   ctl.err & ERR_TIMEOUT ? "a grid barrier wait ran out" :
                   ctl.err & ERR_OVERFLOW ? "a frontier queue overflowed" : "phase or time limit reached");
      goto out;
    }
    if (stats) {
      stats->relaxations = ctl.relax;
      stats->phases = ctl.phases;
      stats->splits = ctl.splits;
      stats->delta = delta;
      stats->workgroups = (uint32_t)cus;
      stats->kernel_ms = ms;
    }
  }
out:
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (buf) {
    (void)hipStreamSynchronize(s);
    (void)hipFree(buf);
  }
  return rc;
}

}  // extern "C"
