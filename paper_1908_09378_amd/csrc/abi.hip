// C ABI of the parallel bucket heap and parDijkstra (include/pbh.h).
//
// Host side only: argument checks, the device arena, growth of the level
// arena, stream handling and error reporting.  All heap and SSSP work runs in
// the kernels of kernels.hip.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "../../include/pbh.h"
#include "pbh_launch.h"

using namespace bkt;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

#define HIPCHK(expr)                                                                 \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(e_ == hipErrorOutOfMemory ? PBH_ENOMEM : PBH_EDEVICE, "%s: %s", #expr, \
                  hipGetErrorString(e_));                                            \
  } while (0)

int ceil_log2(u64 x) {
  int b = 0;
  while (b < 63 && (1ull << b) < x) ++b;
  return b;
}

// Smallest q >= qmin such that the deepest level's nominal bucket 2d*4^(q-1)
// holds `elems` elements.
int levels_for(u32 d, u64 elems, int qmin) {
  int q = qmin;
  while (q < MAXL && nomB(d, q - 1) < elems) ++q;
  return q;
}

// Device arena of levels [0, q) in global memory: keys then ids.
struct Arena {
  u64* k = nullptr;
  u32* v = nullptr;
  u64 elems = 0;
};

int arena_alloc(Arena* a, u64 elems) {
  a->elems = elems;
  if (elems == 0) return PBH_OK;
  HIPCHK(hipMalloc(&a->k, elems * sizeof(u64)));
  hipError_t e = hipMalloc(&a->v, elems * sizeof(u32));
  if (e != hipSuccess) {
    (void)hipFree(a->k);
    a->k = nullptr;
    return fail(PBH_ENOMEM, "hipMalloc of the level arena (%llu elements) failed", (unsigned long long)elems);
  }
  return PBH_OK;
}

void arena_free(Arena* a) {
  if (a->k) (void)hipFree(a->k);
  if (a->v) (void)hipFree(a->v);
  *a = Arena{};
}

}  // namespace

struct pbh {
  u32 id_cap = 0, d = 0;
  int q = 0;
  int sched = 0;
  u64* cur = nullptr;
  u32* bitmap = nullptr;
  u32 nwords = 0;
  Arena arena;
  HeapState* gst = nullptr;
  HeapState host;  // mirror of gst after each call
  u64* ukeys = nullptr;
  u32* uids = nullptr;
  u64 ulist_cap = 0;
  u64* flag = nullptr;
};

namespace {

Geom pbh_geom(const pbh* h) {
  Geom g;
  g.d = h->d;
  g.q = h->q;
  g.qlds = 0;
  g.gk = h->arena.k;
  g.gv = h->arena.v;
  g.lk = nullptr;
  g.lv = nullptr;
  return g;
}

// Adds one level; existing levels keep their offsets, so the old arena is a
// prefix of the new one.
int pbh_grow(pbh* h) {
  if (h->q >= MAXL) return fail(PBH_ECAPACITY, "heap needs more than %d levels", MAXL);
  Arena na;
  int rc = arena_alloc(&na, lvl_off(h->d, h->q + 1));
  if (rc) return rc;
  if (h->arena.elems) {
    HIPCHK(hipMemcpy(na.k, h->arena.k, h->arena.elems * sizeof(u64), hipMemcpyDeviceToDevice));
    HIPCHK(hipMemcpy(na.v, h->arena.v, h->arena.elems * sizeof(u32), hipMemcpyDeviceToDevice));
  }
  arena_free(&h->arena);
  h->arena = na;
  h->q += 1;
  h->host.q = h->q;
  HIPCHK(hipMemcpy(&h->gst->q, &h->host.q, sizeof(int), hipMemcpyHostToDevice));
  return PBH_OK;
}

int pull_state(pbh* h) {
  HIPCHK(hipMemcpy(&h->host, h->gst, sizeof(HeapState), hipMemcpyDeviceToHost));
  return PBH_OK;
}

int push_state(pbh* h) {
  HIPCHK(hipMemcpy(h->gst, &h->host, sizeof(HeapState), hipMemcpyHostToDevice));
  return PBH_OK;
}

int state_error(const HeapState& s) {
  if (s.err == E_CAPACITY) return fail(PBH_ECAPACITY, "a heap level overflowed its allocation");
  if (s.err) return fail(PBH_EINTERNAL, "device-side heap check failed (code %d)", s.err);
  return PBH_OK;
}

}  // namespace

extern "C" {

const char* pbh_last_error(void) { return g_err; }

int pbh_create(pbh_t** out, uint32_t id_capacity, uint32_t d) {
  if (!out) return fail(PBH_EINVAL, "pbh_create: out is NULL");
  *out = nullptr;
  if (id_capacity == 0 || d == 0) return fail(PBH_EINVAL, "pbh_create: id_capacity and d must be > 0");
  pbh* h = new pbh;
  h->id_cap = id_capacity;
  h->d = d;
  // q = ceil(log4(n/d)) + 1 (Section 2.2): the deepest nominal bucket holds n.
  h->q = levels_for(d, id_capacity, 1);
  h->nwords = (id_capacity + 31) / 32;
  int rc = PBH_OK;
  hipError_t e;
  if ((e = hipMalloc(&h->cur, (u64)id_capacity * sizeof(u64))) != hipSuccess ||
      (e = hipMalloc(&h->bitmap, (u64)h->nwords * sizeof(u32))) != hipSuccess ||
      (e = hipMalloc(&h->gst, sizeof(HeapState))) != hipSuccess ||
      (e = hipMalloc(&h->flag, sizeof(u64))) != hipSuccess) {
    rc = fail(e == hipErrorOutOfMemory ? PBH_ENOMEM : PBH_EDEVICE, "pbh_create: %s", hipGetErrorString(e));
  }
  if (!rc) rc = arena_alloc(&h->arena, lvl_off(d, h->q));
  if (!rc) {
    if (hipMemset(h->cur, 0xFF, (u64)id_capacity * sizeof(u64)) != hipSuccess ||
        hipMemset(h->bitmap, 0, (u64)h->nwords * sizeof(u32)) != hipSuccess)
      rc = fail(PBH_EDEVICE, "pbh_create: hipMemset failed");
  }
  if (!rc) {
    state_init(&h->host, d, h->q);
    rc = push_state(h);
  }
  if (rc) {
    pbh_destroy(h);
    return rc;
  }
  *out = h;
  return PBH_OK;
}

int pbh_destroy(pbh_t* h) {
  if (!h) return PBH_OK;
  if (h->cur) (void)hipFree(h->cur);
  if (h->bitmap) (void)hipFree(h->bitmap);
  if (h->gst) (void)hipFree(h->gst);
  if (h->ukeys) (void)hipFree(h->ukeys);
  if (h->uids) (void)hipFree(h->uids);
  if (h->flag) (void)hipFree(h->flag);
  arena_free(&h->arena);
  delete h;
  return PBH_OK;
}

int pbh_bulk_update(pbh_t* h, const uint64_t* keys, const uint32_t* ids, uint64_t count) {
  if (!h) return fail(PBH_EINVAL, "pbh_bulk_update: NULL handle");
  if (count == 0) return PBH_OK;
  if (!keys || !ids) return fail(PBH_EINVAL, "pbh_bulk_update: NULL arrays");
  if (h->host.err) return state_error(h->host);
  HIPCHK(hipMemset(h->flag, 0, sizeof(u64)));
  HIPCHK(launch_check_update((const u64*)keys, ids, count, h->id_cap, h->flag, 0));
  u64 bad = 0;
  HIPCHK(hipMemcpy(&bad, h->flag, sizeof(u64), hipMemcpyDeviceToHost));
  if (bad) return fail(PBH_EINVAL, "pbh_bulk_update: id >= id_capacity or key == UINT64_MAX");
  u64 need = count < h->id_cap ? count : h->id_cap;
  if (need > h->ulist_cap) {
    if (h->ukeys) (void)hipFree(h->ukeys);
    if (h->uids) (void)hipFree(h->uids);
    h->ukeys = nullptr;
    h->uids = nullptr;
    h->ulist_cap = 0;
    HIPCHK(hipMalloc(&h->ukeys, need * sizeof(u64)));
    HIPCHK(hipMalloc(&h->uids, need * sizeof(u32)));
    h->ulist_cap = need;
  }
  h->host.aux[0] = h->host.aux[1] = h->host.aux[3] = 0;
  h->host.progress = 0;
  int rc = push_state(h);
  if (rc) return rc;
  for (;;) {
    PbhParams p{};
    p.g = pbh_geom(h);
    p.gst = h->gst;
    p.cur = h->cur;
    p.bitmap = h->bitmap;
    p.nwords = h->nwords;
    p.id_cap = h->id_cap;
    p.sched = h->sched;
    p.idbits = ceil_log2(h->id_cap) < 1 ? 1 : ceil_log2(h->id_cap);
    p.keys = (const u64*)keys;
    p.ids = ids;
    p.count = count;
    p.ukeys = h->ukeys;
    p.uids = h->uids;
    HIPCHK(launch_pbh_update(p, 0));
    if ((rc = pull_state(h))) return rc;
    if ((rc = state_error(h->host))) return rc;
    if (h->host.aux[3] == 0) break;  // done
    if ((rc = pbh_grow(h))) return rc;
  }
  return PBH_OK;
}

int pbh_extract_min(pbh_t* h, uint64_t k, uint64_t* keys_out, uint32_t* ids_out, uint64_t* count_out) {
  if (!h || !count_out) return fail(PBH_EINVAL, "pbh_extract_min: NULL handle or count_out");
  *count_out = 0;
  if (k == 0) return PBH_OK;
  if (!keys_out || !ids_out) return fail(PBH_EINVAL, "pbh_extract_min: NULL output arrays");
  if (h->host.err) return state_error(h->host);
  h->host.progress = 0;
  h->host.aux[3] = h->host.aux[4] = 0;
  int rc = push_state(h);
  if (rc) return rc;
  for (;;) {
    PbhParams p{};
    p.g = pbh_geom(h);
    p.gst = h->gst;
    p.cur = h->cur;
    p.id_cap = h->id_cap;
    p.sched = h->sched;
    p.idbits = ceil_log2(h->id_cap) < 1 ? 1 : ceil_log2(h->id_cap);
    p.k = k;
    p.okeys = (u64*)keys_out;
    p.oids = ids_out;
    HIPCHK(launch_pbh_extract(p, 0));
    if ((rc = pull_state(h))) return rc;
    if ((rc = state_error(h->host))) return rc;
    if (h->host.aux[3] == 0) break;
    if ((rc = pbh_grow(h))) return rc;
  }
  *count_out = h->host.progress;
  return PBH_OK;
}

int pbh_size(pbh_t* h, uint64_t* size_out) {
  if (!h || !size_out) return fail(PBH_EINVAL, "pbh_size: NULL argument");
  *size_out = h->host.live;
  return PBH_OK;
}

int pbh_debug_levels(pbh_t* h, uint32_t max_levels, uint32_t* levels_out, int32_t* ell_out, uint32_t* nB,
                     uint32_t* nS, uint64_t* p_key, uint32_t* p_id, uint64_t* resolves) {
  if (!h || !levels_out || !ell_out) return fail(PBH_EINVAL, "pbh_debug_levels: NULL argument");
  int rc = pull_state(h);
  if (rc) return rc;
  *levels_out = (u32)h->q;
  *ell_out = h->host.ell;
  for (u32 i = 0; i < max_levels && i < (u32)h->q; ++i) {
    if (nB) nB[i] = h->host.L[i].nB;
    if (nS) nS[i] = h->host.L[i].nS;
    if (p_key) p_key[i] = h->host.L[i].pk;
    if (p_id) p_id[i] = h->host.L[i].pv;
    if (resolves) resolves[i] = h->host.L[i].cnt;
  }
  return PBH_OK;
}

// ------------------------------------------------------------------ sssp

static std::mutex g_sssp_mu;
static Arena g_sssp_arena;        // reused across calls
static SsspDevStats* g_sssp_stats = nullptr;
static CsrCheck* g_csr = nullptr;

int sssp_ex(const uint64_t* offsets, const uint32_t* targets, const uint32_t* weights, uint32_t n, uint64_t m,
            uint32_t source, uint64_t* dist_out, const sssp_opts* opts, sssp_stats* stats, void* stream) {
  if (!offsets || !dist_out || (m > 0 && (!targets || !weights)))
    return fail(PBH_EINVAL, "sssp: NULL array argument");
  if (n == 0) return fail(PBH_EINVAL, "sssp: n == 0");
  if (source >= n) return fail(PBH_EINVAL, "sssp: source %u >= n %u", source, n);
  sssp_opts o{};
  if (opts) o = *opts;
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(g_sssp_mu);
  if (!g_csr) HIPCHK(hipMalloc(&g_csr, sizeof(CsrCheck)));
  if (!g_sssp_stats) HIPCHK(hipMalloc(&g_sssp_stats, sizeof(SsspDevStats)));
  HIPCHK(hipMemsetAsync(g_csr, 0, sizeof(CsrCheck), s));
  HIPCHK(launch_check_csr((const u64*)offsets, targets, n, m, g_csr, s));
  CsrCheck cc;
  HIPCHK(hipMemcpyAsync(&cc, g_csr, sizeof cc, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (cc.bad) return fail(PBH_EINVAL, "sssp: malformed CSR (offsets or targets)");
  u32 d = o.d ? o.d : (u32)(cc.maxdeg ? cc.maxdeg : 1);
  if (cc.maxdeg > d) return fail(PBH_EINVAL, "sssp: opts.d %u below the maximum out-degree %llu", d,
                                 (unsigned long long)cc.maxdeg);
  int team = (int)o.team;
  if (team == 0) team = d <= 256 ? 64 : (d <= 4096 ? 256 : 1024);
  if (team != 64 && team != 256 && team != 1024) return fail(PBH_EINVAL, "sssp: team must be 64, 256 or 1024");
  // Heap capacity: every inserted element is a strict improvement of some
  // vertex, so at most m + 1 elements are ever inserted.  The default starts
  // smaller and retries with that bound if a level overflows.
  u64 safe = m + 1;
  u64 hcap = o.heap_capacity ? o.heap_capacity : (safe < 4ull * n + 4096 ? safe : 4ull * n + 4096);
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  int max_lds = 0;
  HIPCHK(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  for (;;) {
    int q = levels_for(d, hcap, 2);
    size_t budget = (size_t)max_lds - sssp_static_lds(team) - 256;
    int qlds = 0;
    if (o.lds_levels == 0) {
      while (qlds < q && lvl_off(d, qlds + 1) * 12ull <= budget) ++qlds;
    } else if (o.lds_levels != 0xFFFFFFFFu) {
      qlds = (int)o.lds_levels;
    }
    if (qlds > q) qlds = q;
    size_t lds = (size_t)lvl_off(d, qlds) * 12ull;
    if (lds > budget) return fail(PBH_EINVAL, "sssp: %d LDS levels do not fit", qlds);
    u64 gel = lvl_off(d, q) - lvl_off(d, qlds);
    if (g_sssp_arena.elems < gel) {
      arena_free(&g_sssp_arena);
      int rc = arena_alloc(&g_sssp_arena, gel);
      if (rc) return rc;
    }
    SsspParams p{};
    p.off = (const u64*)offsets;
    p.tg = targets;
    p.wt = weights;
    p.dist = (u64*)dist_out;
    p.n = n;
    p.src = source;
    p.sched = (int)o.schedule;
    p.g.d = d;
    p.g.q = q;
    p.g.qlds = qlds;
    p.g.gk = g_sssp_arena.k;
    p.g.gv = g_sssp_arena.v;
    p.stats = g_sssp_stats;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(launch_fill_dist((u64*)dist_out, n, source, s));
    HIPCHK(hipEventRecord(e0, s));
    HIPCHK(launch_sssp(team, p, lds, s));
    HIPCHK(hipEventRecord(e1, s));
    SsspDevStats ds;
    HIPCHK(hipMemcpyAsync(&ds, g_sssp_stats, sizeof ds, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (ds.err == E_CAPACITY && hcap < safe) {
      hcap = safe;
      continue;
    }
    if (ds.err == E_CAPACITY) return fail(PBH_ECAPACITY, "sssp: heap levels overflowed");
    if (ds.err) return fail(PBH_EINTERNAL, "sssp: device-side heap check failed (code %lld)", ds.err);
    if (stats) {
      std::memset(stats, 0, sizeof *stats);
      stats->rounds = ds.rounds;
      stats->relaxations = ds.relax;
      stats->updates = ds.updates;
      stats->heap_elems = ds.elems;
      for (int i = 0; i < 16 && i < MAXL; ++i) stats->resolves[i] = ds.resolves[i];
      stats->levels = (u32)q;
      stats->d = d;
      stats->team = (u32)team;
      stats->lds_levels = (u32)qlds;
      stats->kernel_ms = ms;
    }
    return PBH_OK;
  }
}

int sssp(const uint64_t* offsets, const uint32_t* targets, const uint32_t* weights, uint32_t n, uint64_t m,
         uint32_t source, uint64_t* dist_out) {
  return sssp_ex(offsets, targets, weights, n, m, source, dist_out, nullptr, nullptr, nullptr);
}

}  // extern "C"
