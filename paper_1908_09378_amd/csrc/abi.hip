// C ABI of the parallel bucket heap and parDijkstra (include/pbh.h).
//
// Host side only: argument checks, the device arena, growth of the level
// arena, stream handling and error reporting.  All heap and SSSP work runs in
// the kernels of kernels.hip (one workgroup per operation) and wide.hip (the
// device-wide heap engine for large d).
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <vector>

#include "../../include/pbh.h"
#include "pbh_launch.h"
#include "wide.h"

using namespace bkt;

static_assert(PBH_TRACE_K == TRACE_K, "trace record length of the header and the kernels");
static_assert(PBH_MLP_BLOB == MLP_BLOB, "model size of the header and the kernels");

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

// On failure *a is left empty (elems 0, no pointers), so a later call that
// needs less allocates again instead of using the missing arrays.
int arena_alloc(Arena* a, u64 elems) {
  *a = Arena{};
  if (elems == 0) return PBH_OK;
  u64* k = nullptr;
  u32* v = nullptr;
  if (hipMalloc(&k, elems * sizeof(u64)) != hipSuccess || hipMalloc(&v, elems * sizeof(u32)) != hipSuccess) {
    if (k) (void)hipFree(k);
    (void)hipGetLastError();  // clear the sticky allocation error
    return fail(PBH_ENOMEM, "hipMalloc of the level arena (%llu elements) failed", (unsigned long long)elems);
  }
  a->k = k;
  a->v = v;
  a->elems = elems;
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
  WideScratch* wide = nullptr;  // device-wide engine (state authoritative on the host)
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
  if (h->wide) return PBH_OK;  // the host copy is the state
  HIPCHK(hipMemcpy(&h->host, h->gst, sizeof(HeapState), hipMemcpyDeviceToHost));
  return PBH_OK;
}

int push_state(pbh* h) {
  if (h->wide) return PBH_OK;
  HIPCHK(hipMemcpy(h->gst, &h->host, sizeof(HeapState), hipMemcpyHostToDevice));
  return PBH_OK;
}

int state_error(const HeapState& s) {
  if (s.err == E_CAPACITY) return fail(PBH_ECAPACITY, "a heap level overflowed its allocation");
  if (s.err == E_DEVICE) return fail(PBH_EDEVICE, "a HIP call of the device-wide heap engine failed");
  if (s.err == E_TIMEOUT)
    return fail(PBH_ETIMEOUT, "a step of the device-wide heap engine ended without publishing its results");
  if (s.err) return fail(PBH_EINTERNAL, "device-side heap check failed (code %d)", s.err);
  return PBH_OK;
}

int wide_grow_cb(void* ctx, Geom* g) {
  pbh* h = (pbh*)ctx;
  int rc = pbh_grow(h);
  if (rc) return rc == PBH_ECAPACITY ? E_CAPACITY : E_DEVICE;
  *g = pbh_geom(h);
  return 0;
}

WideHeap wide_view(pbh* h) {
  WideHeap w;
  w.g = pbh_geom(h);
  w.st = &h->host;
  w.cur = h->cur;
  w.nwords = h->nwords;
  w.sched = h->sched;
  w.ukeys = h->ukeys;
  w.uids = h->uids;
  w.grow = wide_grow_cb;
  w.ctx = h;
  return w;
}

// A device-wide engine result -> PBH code; a failed step leaves the heap
// unusable (its error is kept in the state).
int wide_result(pbh* h, int rc) {
  if (rc == 0) return PBH_OK;
  if (!h->host.err) h->host.err = rc;
  return state_error(h->host);
}

// k rule of sssp_opts -> SpecCfg (the list buffers are filled in by the caller).
int spec_from_opts(const sssp_opts& o, u32 d, SpecCfg* sc, u32* kmax_out) {
  std::memset(sc, 0, sizeof *sc);
  if (o.k_rule > 3) return fail(PBH_EINVAL, "sssp: k_rule must be 0..3");
  u32 kmax = o.k_max ? o.k_max : 2 * d;
  if (kmax > (u32)KMAX_ROUND) kmax = KMAX_ROUND;
  if (kmax < 1) kmax = 1;
  // k capped at 1 is the plain rule; its round path is the cheaper one
  sc->rule = kmax == 1 ? 0 : (int)o.k_rule;
  sc->kfix = o.k_fixed ? o.k_fixed : 1;
  sc->kmax = kmax;
  if (o.k_rule == 2 && !o.k_model) return fail(PBH_EINVAL, "sssp: k_rule 2 needs k_model");
  if (o.k_rule == 3 && (!o.k_seq || o.k_seq_len == 0)) return fail(PBH_EINVAL, "sssp: k_rule 3 needs k_seq");
  sc->kseq = o.k_seq;
  sc->kseq_len = o.k_seq_len;
  sc->model = o.k_model;
  sc->stop_key = o.stop_key;
  sc->max_rounds = o.max_rounds;
  sc->kscale = o.k_scale > 0.0f ? o.k_scale : 1.0f;
  sc->kevery = o.k_every > 1 ? o.k_every : 1u;
  *kmax_out = kmax;
  return PBH_OK;
}

bool spec_needs_list(const sssp_opts& o) { return o.k_rule != 0 || o.trace_features != nullptr; }

}  // namespace

extern "C" {

const char* pbh_last_error(void) { return g_err; }

int pbh_create(pbh_t** out, uint32_t id_capacity, uint32_t d) { return pbh_create_ex(out, id_capacity, d, nullptr); }

int pbh_create_ex(pbh_t** out, uint32_t id_capacity, uint32_t d, const pbh_opts* opts) {
  if (!out) return fail(PBH_EINVAL, "pbh_create: out is NULL");
  *out = nullptr;
  if (id_capacity == 0 || d == 0) return fail(PBH_EINVAL, "pbh_create: id_capacity and d must be > 0");
  pbh_opts o{};
  if (opts) o = *opts;
  if (o.engine > 2 || o.schedule > 1) return fail(PBH_EINVAL, "pbh_create_ex: engine must be 0..2, schedule 0..1");
  for (uint32_t r : o.reserved)
    if (r) return fail(PBH_EINVAL, "pbh_create_ex: reserved fields must be zero");
  const bool wide = o.engine == 2 || (o.engine == 0 && d >= 16384);
  pbh* h = new pbh;
  h->sched = (int)o.schedule;
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
  if (!rc && wide) {
    if (wide_create(&h->wide, d) || wide_reserve(h->wide, capB(d, h->q - 1)))
      rc = fail(PBH_ENOMEM, "pbh_create: scratch of the device-wide engine: %s", hipGetErrorString(hipGetLastError()));
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
  if (h->wide) wide_destroy(h->wide);
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
  if (h->wide) {
    WideHeap w = wide_view(h);
    return wide_result(h, wide_bulk_update(h->wide, &w, (const u64*)keys, ids, count));
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

int pbh_delete(pbh_t* h, const uint32_t* ids, uint64_t count) {
  if (!h) return fail(PBH_EINVAL, "pbh_delete: NULL handle");
  if (count == 0) return PBH_OK;
  if (!ids) return fail(PBH_EINVAL, "pbh_delete: NULL ids");
  if (h->host.err) return state_error(h->host);
  HIPCHK(hipMemset(h->flag, 0, sizeof(u64)));
  HIPCHK(launch_check_update(nullptr, ids, count, h->id_cap, h->flag, 0));
  u64 bad = 0;
  HIPCHK(hipMemcpy(&bad, h->flag, sizeof(u64), hipMemcpyDeviceToHost));
  if (bad) return fail(PBH_EINVAL, "pbh_delete: id >= id_capacity");
  if (h->wide) {
    WideHeap w = wide_view(h);
    return wide_result(h, wide_delete(h->wide, &w, ids, count));
  }
  h->host.aux[1] = h->host.aux[3] = 0;
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
    p.ids = ids;
    p.count = count;
    HIPCHK(launch_pbh_delete(p, 0));
    if ((rc = pull_state(h))) return rc;
    if ((rc = state_error(h->host))) return rc;
    if (h->host.aux[3] == 0) break;
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
  if (h->wide) {
    WideHeap w = wide_view(h);
    return wide_result(h, wide_extract_min(h->wide, &w, k, (u64*)keys_out, ids_out, (u64*)count_out));
  }
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

int mlp_infer(const float* X, uint32_t n, const float* blob, uint32_t team, float* y) {
  if (n == 0) return PBH_OK;
  if (!X || !blob || !y) return fail(PBH_EINVAL, "mlp_infer: NULL array");
  if (team != 64 && team != 256) return fail(PBH_EINVAL, "mlp_infer: team must be 64 or 256");
  HIPCHK(launch_mlp_infer((int)team, X, n, blob, y, 0));
  HIPCHK(hipDeviceSynchronize());
  return PBH_OK;
}

int pbh_kernel_profile(pbh_t* h, uint32_t kind, uint64_t* launches, uint64_t* bytes, double* ms) {
  if (!h || !launches || !bytes || !ms) return fail(PBH_EINVAL, "pbh_kernel_profile: NULL argument");
  if (kind >= (uint32_t)WK_COUNT) return fail(PBH_EINVAL, "pbh_kernel_profile: kind %u >= %d", kind, (int)WK_COUNT);
  WideKernelStat k{0, 0, 0.0};
  if (h->wide) wide_kernel_profile(h->wide, (int)kind, &k);
  *launches = k.launches;
  *bytes = k.bytes;
  *ms = k.ms;
  return PBH_OK;
}

const char* pbh_kernel_name(uint32_t kind) { return wide_kernel_name((int)kind); }

int pbh_merge_profile(pbh_t* h, uint64_t* launches, uint64_t* bytes, double* ms) {
  if (!h || !launches || !bytes || !ms) return fail(PBH_EINVAL, "pbh_merge_profile: NULL argument");
  return pbh_kernel_profile(h, WK_MERGE_WRITE, launches, bytes, ms);
}

int pbh_set_profiling(pbh_t* h, int on) {
  if (!h) return fail(PBH_EINVAL, "pbh_set_profiling: NULL handle");
  if (h->wide) wide_set_profiling(h->wide, on != 0);
  return PBH_OK;
}

int pbh_traffic(pbh_t* h, uint64_t* elements_out) {
  if (!h || !elements_out) return fail(PBH_EINVAL, "pbh_traffic: NULL argument");
  int rc = pull_state(h);
  if (rc) return rc;
  *elements_out = h->host.elems;
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
static Arena g_sssp_list;         // round update lists of speculative rounds
static SsspDevStats* g_sssp_stats = nullptr;
static DeepCtl* g_deep_ctl = nullptr;  // control block of the deep-level workers
static CsrCheck* g_csr = nullptr;

}  // extern "C"

namespace {

// A fixed block of device memory that a run carves all of its buffers from
// instead of allocating them (the no-allocation entry point).
struct FixedScratch {
  unsigned char* base;
  u64 bytes;
};

// Bytes of the fixed block a run needs: the CSR check and the statistics
// (one 4096-byte header), the HBM levels (12 B per element) and the
// speculative rounds' update lists.
constexpr u64 FIXED_HEAD = 4096;
constexpr u64 FIXED_DEEP = 1024;  // the deep-level workers' control block inside the header
u64 fixed_bytes(u64 arena_elems, u64 list_elems) { return FIXED_HEAD + 12ull * (arena_elems + list_elems); }

// sssp_ex with the query index that trace records carry (0 for a single
// query; a batch re-running one of its queries passes that query's index).
// With fx, every device buffer comes from that block and nothing is
// allocated (no events either: kernel_ms is then 0).  The caller holds
// g_sssp_mu.
int sssp_run(const uint64_t* offsets, const uint32_t* targets, const uint32_t* weights, uint32_t n, uint64_t m,
             uint32_t source, uint64_t* dist_out, const sssp_opts* opts, sssp_stats* stats, void* stream, u32 qid,
             const FixedScratch* fx = nullptr) {
  if (!offsets || !dist_out || (m > 0 && (!targets || !weights)))
    return fail(PBH_EINVAL, "sssp: NULL array argument");
  if (n == 0) return fail(PBH_EINVAL, "sssp: n == 0");
  if (source >= n) return fail(PBH_EINVAL, "sssp: source %u >= n %u", source, n);
  sssp_opts o{};
  if (opts) o = *opts;
  hipStream_t s = (hipStream_t)stream;
  CsrCheck* csr;
  SsspDevStats* dstats;
  if (fx) {
    csr = reinterpret_cast<CsrCheck*>(fx->base);
    dstats = reinterpret_cast<SsspDevStats*>(fx->base + 256);
    static_assert(256 + sizeof(SsspDevStats) <= FIXED_DEEP, "header of the fixed block");
    static_assert(FIXED_DEEP + sizeof(DeepCtl) <= FIXED_HEAD, "header of the fixed block");
  } else {
    if (!g_csr) HIPCHK(hipMalloc(&g_csr, sizeof(CsrCheck)));
    if (!g_sssp_stats) HIPCHK(hipMalloc(&g_sssp_stats, sizeof(SsspDevStats)));
    csr = g_csr;
    dstats = g_sssp_stats;
  }
  // a fill kernel, not a memset, so that the sequence stays free of memset
  // nodes for callers that record it
  HIPCHK(launch_zero_u64(reinterpret_cast<u64*>(csr), sizeof(CsrCheck) / 8, s));
  HIPCHK(launch_check_csr((const u64*)offsets, targets, n, m, csr, s));
  CsrCheck cc;
  HIPCHK(hipMemcpyAsync(&cc, csr, sizeof cc, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (cc.bad) return fail(PBH_EINVAL, "sssp: malformed CSR (offsets or targets)");
  u32 d = o.d ? o.d : (u32)(cc.maxdeg ? cc.maxdeg : 1) * (o.d_scale > 1 ? o.d_scale : 1u);
  if (cc.maxdeg > d) return fail(PBH_EINVAL, "sssp: opts.d %u below the maximum out-degree %llu", d,
                                 (unsigned long long)cc.maxdeg);
  int team = (int)o.team;
  if (team == 0) team = d <= 256 ? 64 : (d <= 4096 ? 256 : 1024);
  if (team != 64 && team != 256 && team != 1024) return fail(PBH_EINVAL, "sssp: team must be 64, 256 or 1024");
  if (o.deep_level && o.schedule != 0) return fail(PBH_EINVAL, "sssp: deep-level workers need schedule 0");
  // Heap capacity: the arena is sized for hcap elements.  With the plain rule
  // every inserted element is a strict improvement from one scanned edge, so
  // at most m + 1 are ever inserted; rules that pull ahead re-insert vertices
  // whose distance improves again, so their insertions are bounded only by
  // the relaxations.  The default starts at min(m + 1, 4n + 4096); if the
  // deepest level overflows, the run is repeated with at least one more level
  // (the plain rule's bound m + 1 first, then 4x per retry) until it fits or
  // MAXL levels are reached.
  const u64 safe = m + 1;
  u64 hcap = o.heap_capacity ? o.heap_capacity : (safe < 4ull * n + 4096 ? safe : 4ull * n + 4096);
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  int max_lds = 0;
  HIPCHK(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  bool first = true;
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
    const u64 gel = lvl_off(d, q) - lvl_off(d, qlds);
    SsspParams p{};
    u32 kmax = 1;
    {
      int rc = spec_from_opts(o, d, &p.spec, &kmax);
      if (rc) return rc;
    }
    const u64 le = spec_needs_list(o) ? 2ull * kmax * (u64)d : 0ull;
    u64 *ak, *lk;
    u32 *av, *lv;
    if (fx) {
      const u64 need = fixed_bytes(gel, le);
      if (need > fx->bytes) {
        if (first)
          return fail(PBH_EINVAL,
                      "sssp_noalloc: this query needs %llu bytes of scratch (%d heap levels of bulk size %u), "
                      "the fixed scratch holds %llu",
                      (unsigned long long)need, q, d, (unsigned long long)fx->bytes);
        return fail(PBH_ECAPACITY, "sssp_noalloc: the heap outgrew the fixed scratch (%llu bytes needed, %llu held)",
                    (unsigned long long)need, (unsigned long long)fx->bytes);
      }
      // keys (8-byte aligned after the header), then ids, for the arena and the list
      ak = reinterpret_cast<u64*>(fx->base + FIXED_HEAD);
      lk = ak + gel;
      av = reinterpret_cast<u32*>(lk + le);
      lv = av + gel;
    } else {
      if (g_sssp_arena.elems < gel) {
        arena_free(&g_sssp_arena);
        int rc = arena_alloc(&g_sssp_arena, gel);
        if (rc) return rc;
      }
      if (le && g_sssp_list.elems < le) {
        arena_free(&g_sssp_list);
        int rc = arena_alloc(&g_sssp_list, le);
        if (rc) return rc;
      }
      ak = g_sssp_arena.k;
      av = g_sssp_arena.v;
      lk = le ? g_sssp_list.k : nullptr;
      lv = le ? g_sssp_list.v : nullptr;
    }
    first = false;
    if (le) {
      p.spec.uk = lk;
      p.spec.uv = lv;
      p.spec.tk = lk + (u64)kmax * d;
      p.spec.tv = lv + (u64)kmax * d;
      // the LDS left after the levels holds the round's list for the intake
      // sort when it fits (two buffers, 12 B per pair each)
      const u64 room = (budget - lds) / 24u;
      const u64 lcap = std::min<u64>(room, (u64)kmax * d);
      if (lcap >= 256) {
        p.spec.lcap = (u32)lcap;
        lds += (size_t)lcap * 24u;
      }
    }
    p.prof = o.profile ? 1u : 0u;
    // deep_level selects the large-heap form of the round loop: LDS staging
    // for merges of the HBM levels, after the LDS levels (it shares that
    // room with the speculative rounds' list), and the deep-level workers
    p.full = o.deep_level ? 1u : 0u;
    p.stage = 0;
    if (p.full && q > qlds) {
      const u64 sb = stage_bytes(team, team == 64 ? 8 : 4);
      const size_t lvb = (size_t)lvl_off(d, qlds) * 12ull;
      if (lvb + sb <= budget) {
        p.stage = (u32)sb;
        lds = std::max(lds, lvb + (size_t)sb);
      }
    }
    // Deep-level workers: one workgroup per level from max(deep_level, 2,
    // LDS levels) down (none if that is past the deepest level).
    p.deep = nullptr;
    p.deep_lim = MAXL;
    if (o.deep_level) {
      const int lim = std::max<int>(std::max<int>((int)std::min<u32>(o.deep_level, MAXL), 2), qlds);
      if (lim < q) {
        DeepCtl* ctl;
        if (fx) {
          ctl = reinterpret_cast<DeepCtl*>(fx->base + FIXED_DEEP);
        } else {
          if (!g_deep_ctl) HIPCHK(hipMalloc(&g_deep_ctl, (sizeof(DeepCtl) + 7) / 8 * 8));
          ctl = g_deep_ctl;
        }
        HIPCHK(launch_zero_u64(reinterpret_cast<u64*>(ctl), (sizeof(DeepCtl) + 7) / 8, s));
        p.deep = ctl;
        p.deep_lim = lim;
      }
    }
    p.spec.order = o.settle_order;
    p.spec.order_cap = o.settle_order ? o.settle_cap : 0;
    if (o.trace_features) {
      if (!o.trace_keys || !o.trace_ids || !o.trace_count || o.trace_every == 0)
        return fail(PBH_EINVAL, "sssp: trace needs keys, ids, count and trace_every");
      p.spec.trace_f = o.trace_features;
      p.spec.trace_k = (u64*)o.trace_keys;
      p.spec.trace_v = o.trace_ids;
      p.spec.trace_count = o.trace_count;
      p.spec.trace_q = o.trace_query;
      p.spec.qid = qid;
      p.spec.trace_every = o.trace_every;
      p.spec.trace_cap = o.trace_cap;
    }
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
    p.g.gk = ak;
    p.g.gv = av;
    p.stats = dstats;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!fx) {
      HIPCHK(hipEventCreate(&e0));
      HIPCHK(hipEventCreate(&e1));
    }
    HIPCHK(launch_fill_dist((u64*)dist_out, n, source, s));
    if (e0) HIPCHK(hipEventRecord(e0, s));
    HIPCHK(launch_sssp(team, p, lds, s));
    if (e1) HIPCHK(hipEventRecord(e1, s));
    SsspDevStats ds;
    HIPCHK(hipMemcpyAsync(&ds, dstats, sizeof ds, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    float ms = 0.f;
    if (e0) {
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
    }
    if (ds.err == E_CAPACITY && q < MAXL) {
      // at least one more level: the deepest nominal bucket must grow past hcap
      const u64 grown = std::max<u64>(safe, nomB(d, q - 1) * 4ull);
      hcap = std::max<u64>(hcap * 4ull, grown);
      continue;
    }
    if (ds.err == E_CAPACITY) return fail(PBH_ECAPACITY, "sssp: heap levels overflowed at %d levels", q);
    if (ds.err == E_TIMEOUT)
      return fail(PBH_ETIMEOUT, "sssp: a wait between the round loop and a deep-level worker ran out");
    if (ds.err) return fail(PBH_EINTERNAL, "sssp: device-side heap check failed (code %lld)", ds.err);
    if (stats) {
      std::memset(stats, 0, sizeof *stats);
      stats->rounds = ds.rounds;
      stats->relaxations = ds.relax;
      stats->updates = ds.updates;
      stats->heap_elems = ds.elems;
      stats->extracted = ds.extracted;
      stats->last_key = ds.last_key;
      for (int i = 0; i < 16 && i < MAXL; ++i) stats->resolves[i] = ds.resolves[i];
      stats->levels = (u32)q;
      stats->d = d;
      stats->team = (u32)team;
      stats->lds_levels = (u32)qlds;
      stats->kernel_ms = ms;
      if (o.profile) {
        int khz = 0;
        HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
        const double us = khz > 0 ? 1e3 / (double)khz : 0.0;  // microseconds per tick
        for (int i = 0; i < 16 && i < MAXL; ++i) stats->level_us[i] = (double)ds.prof[i] * us;
        for (int i = 0; i < 8 && MAXL + i < PROF_N; ++i) stats->phase_us[i] = (double)ds.prof[MAXL + i] * us;
      }
    }
    return PBH_OK;
  }
}

}  // namespace

extern "C" {

int sssp_ex(const uint64_t* offsets, const uint32_t* targets, const uint32_t* weights, uint32_t n, uint64_t m,
            uint32_t source, uint64_t* dist_out, const sssp_opts* opts, sssp_stats* stats, void* stream) {
  std::lock_guard<std::mutex> lock(g_sssp_mu);
  return sssp_run(offsets, targets, weights, n, m, source, dist_out, opts, stats, stream, 0u);
}

// ------------------------------------------------------------ sssp_noalloc

}  // extern "C"

// Fixed scratch of the no-allocation entry point: one static device array,
// held by every GPU the library runs on until the process ends.  In host code
// `scratch` names a host-side stand-in, never the device memory: its device
// address comes from hipGetSymbolAddress, once per device, and only that
// address is used.
constexpr u64 NOALLOC_SCRATCH_BYTES = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
unsigned char* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// The device address of `scratch` on the current device (set up on the first
// call there).  The caller holds g_sssp_mu.
int scratch_on_device(unsigned char** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(PBH_EDEVICE, "sssp_noalloc: device %d out of range", dev);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(PBH_EDEVICE, "sssp_noalloc: no device address for the scratch array");
    g_scratch_ptr[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return PBH_OK;
}
}  // namespace

extern "C" {

int sssp_noalloc(const uint64_t* offsets, const uint32_t* targets, const uint32_t* weights, uint32_t n, uint64_t m,
                 uint32_t source, uint64_t* dist_out, const sssp_opts* opts, sssp_stats* stats, void* stream) {
  std::lock_guard<std::mutex> lock(g_sssp_mu);
  unsigned char* base = nullptr;
  if (int rc = scratch_on_device(&base)) return rc;
  const FixedScratch fx{base, NOALLOC_SCRATCH_BYTES};
  return sssp_run(offsets, targets, weights, n, m, source, dist_out, opts, stats, stream, 0u, &fx);
}

// ------------------------------------------------------------ sssp_batch

static Arena g_batch_arena;
static Arena g_batch_list;
static SsspParams* g_batch_desc = nullptr;
static u32 g_batch_desc_cap = 0;
static SsspDevStats* g_batch_stats = nullptr;
static CsrCheck* g_batch_csr = nullptr;
static u32 g_batch_csr_cap = 0;
static u32* g_batch_counter = nullptr;

int sssp_batch(const sssp_query* queries, uint32_t nq, const sssp_opts* opts, sssp_stats* stats, void* stream) {
  if (stats) std::memset(stats, 0, sizeof *stats);
  if (nq == 0) return PBH_OK;
  if (!queries) return fail(PBH_EINVAL, "sssp_batch: queries is NULL");
  for (u32 i = 0; i < nq; ++i) {
    const sssp_query& q = queries[i];
    if (!q.offsets || !q.dist_out || (q.m > 0 && (!q.targets || !q.weights)))
      return fail(PBH_EINVAL, "sssp_batch: query %u has a NULL array", i);
    if (q.n == 0 || q.source >= q.n) return fail(PBH_EINVAL, "sssp_batch: query %u has n == 0 or source >= n", i);
  }
  sssp_opts o{};
  if (opts) o = *opts;
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(g_sssp_mu);
  // distinct graphs: validate each once and get its maximum out-degree
  std::map<const uint64_t*, u32> gid;
  std::vector<u32> qg(nq);
  std::vector<u32> grep;
  for (u32 i = 0; i < nq; ++i) {
    auto it = gid.find(queries[i].offsets);
    if (it == gid.end()) {
      it = gid.emplace(queries[i].offsets, (u32)grep.size()).first;
      grep.push_back(i);
    }
    qg[i] = it->second;
  }
  const u32 ng = (u32)grep.size();
  if (ng > g_batch_csr_cap) {
    if (g_batch_csr) (void)hipFree(g_batch_csr);
    g_batch_csr = nullptr;
    g_batch_csr_cap = 0;
    HIPCHK(hipMalloc(&g_batch_csr, ng * sizeof(CsrCheck)));
    g_batch_csr_cap = ng;
  }
  HIPCHK(hipMemsetAsync(g_batch_csr, 0, ng * sizeof(CsrCheck), s));
  for (u32 k = 0; k < ng; ++k) {
    const sssp_query& q = queries[grep[k]];
    HIPCHK(launch_check_csr((const u64*)q.offsets, q.targets, q.n, q.m, g_batch_csr + k, s));
  }
  std::vector<CsrCheck> cc(ng);
  HIPCHK(hipMemcpyAsync(cc.data(), g_batch_csr, ng * sizeof(CsrCheck), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (u32 i = 0; i < nq; ++i) {
    const CsrCheck& c = cc[qg[i]];
    if (c.bad) return fail(PBH_EINVAL, "sssp_batch: query %u: malformed CSR", i);
    if (o.d && c.maxdeg > o.d) return fail(PBH_EINVAL, "sssp_batch: opts.d below a maximum out-degree");
    // every query of a graph must agree on n and m
    const sssp_query& r = queries[grep[qg[i]]];
    if (queries[i].n != r.n || queries[i].m != r.m)
      return fail(PBH_EINVAL, "sssp_batch: queries %u and %u share offsets but not n/m", i, grep[qg[i]]);
  }
  u32 dmax = 1;
  std::vector<u32> qd(nq);
  for (u32 i = 0; i < nq; ++i) {
    u64 md = cc[qg[i]].maxdeg;
    qd[i] = o.d ? o.d : (u32)(md ? md : 1) * (o.d_scale > 1 ? o.d_scale : 1u);
    dmax = std::max(dmax, qd[i]);
  }
  int team = (int)o.team;
  if (team == 0) team = dmax <= 256 ? 64 : (dmax <= 4096 ? 256 : 1024);
  if (team != 64 && team != 256 && team != 1024) return fail(PBH_EINVAL, "sssp_batch: team must be 64, 256 or 1024");
  int dev = 0, max_lds = 0, cus = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  // LDS per team: leave room for two teams per compute unit.
  size_t budget = std::min((size_t)max_lds, (size_t)80 * 1024) - sssp_static_lds(team) - 256;
  // order: largest graphs first (they have the longest round chains)
  std::vector<u32> order(nq);
  std::iota(order.begin(), order.end(), 0u);
  std::stable_sort(order.begin(), order.end(), [&](u32 a, u32 b) { return queries[a].m > queries[b].m; });
  std::vector<SsspParams> desc(nq);
  std::vector<u64> gel(nq);
  u64 total_gel = 0;
  size_t lds = 0;
  u32 maxn = 0;
  for (u32 j = 0; j < nq; ++j) {
    const u32 i = order[j];
    const sssp_query& q = queries[i];
    const u32 d = qd[i];
    // The heap of one query holds its frontier plus copies awaiting deletion;
    // start from max(4096, n) elements and rerun a query alone with the safe
    // bound m + 1 if a level would overflow.
    u64 hcap = o.heap_capacity ? o.heap_capacity : std::min<u64>(q.m + 1, std::max<u64>(4096, q.n));
    int qv = levels_for(d, hcap, 2);
    int qlds = 0;
    if (o.lds_levels == 0) {
      while (qlds < qv && lvl_off(d, qlds + 1) * 12ull <= budget) ++qlds;
    } else if (o.lds_levels != 0xFFFFFFFFu) {
      qlds = std::min((int)o.lds_levels, qv);
      if (lvl_off(d, qlds) * 12ull > budget) return fail(PBH_EINVAL, "sssp_batch: LDS levels do not fit");
    }
    lds = std::max(lds, (size_t)(lvl_off(d, qlds) * 12ull));
    // LDS staging for merges of the HBM levels, after the LDS levels
    u32 stage = 0;
    if (qv > qlds) {
      const u64 sb = stage_bytes(team, team == 64 ? 8 : 4);
      const size_t lvb = (size_t)lvl_off(d, qlds) * 12ull;
      if (lvb + sb <= budget) {
        stage = (u32)sb;
        lds = std::max(lds, lvb + (size_t)sb);
      }
    }
    gel[j] = lvl_off(d, qv) - lvl_off(d, qlds);
    total_gel += gel[j];
    maxn = std::max(maxn, q.n);
    SsspParams& p = desc[j];
    p.off = (const u64*)q.offsets;
    p.tg = q.targets;
    p.wt = q.weights;
    p.dist = (u64*)q.dist_out;
    p.n = q.n;
    p.src = q.source;
    p.sched = (int)o.schedule;
    p.g.d = d;
    p.g.q = qv;
    p.g.qlds = qlds;
    p.stage = stage;
    p.full = 1;
  }
  if (o.trace_features && (!o.trace_keys || !o.trace_ids || !o.trace_count || o.trace_every == 0))
    return fail(PBH_EINVAL, "sssp_batch: trace needs keys, ids, count and trace_every");
  std::vector<u64> lel(nq, 0);
  u64 total_lel = 0;
  for (u32 j = 0; j < nq; ++j) {
    u32 kmax = 1;
    int rc = spec_from_opts(o, desc[j].g.d, &desc[j].spec, &kmax);
    if (rc) return rc;
    if (spec_needs_list(o)) lel[j] = 2ull * kmax * desc[j].g.d;
    total_lel += lel[j];
    if (o.trace_features) {
      desc[j].spec.trace_f = o.trace_features;
      desc[j].spec.trace_k = (u64*)o.trace_keys;
      desc[j].spec.trace_v = o.trace_ids;
      desc[j].spec.trace_count = o.trace_count;
      desc[j].spec.trace_q = o.trace_query;
      desc[j].spec.qid = order[j];
      desc[j].spec.trace_every = o.trace_every;
      desc[j].spec.trace_cap = o.trace_cap;
    }
  }
  if (g_batch_list.elems < total_lel) {
    arena_free(&g_batch_list);
    int rc = arena_alloc(&g_batch_list, total_lel);
    if (rc) return rc;
  }
  {
    u64 lat = 0;
    for (u32 j = 0; j < nq; ++j) {
      if (!lel[j]) continue;
      desc[j].spec.uk = g_batch_list.k + lat;
      desc[j].spec.uv = g_batch_list.v + lat;
      desc[j].spec.tk = g_batch_list.k + lat + lel[j] / 2;
      desc[j].spec.tv = g_batch_list.v + lat + lel[j] / 2;
      lat += lel[j];
    }
  }
  if (g_batch_arena.elems < total_gel) {
    arena_free(&g_batch_arena);
    int rc = arena_alloc(&g_batch_arena, total_gel);
    if (rc) return rc;
  }
  if (nq > g_batch_desc_cap) {
    if (g_batch_desc) (void)hipFree(g_batch_desc);
    if (g_batch_stats) (void)hipFree(g_batch_stats);
    g_batch_desc = nullptr;
    g_batch_stats = nullptr;
    g_batch_desc_cap = 0;
    HIPCHK(hipMalloc(&g_batch_desc, nq * sizeof(SsspParams)));
    HIPCHK(hipMalloc(&g_batch_stats, nq * sizeof(SsspDevStats)));
    g_batch_desc_cap = nq;
  }
  if (!g_batch_counter) HIPCHK(hipMalloc(&g_batch_counter, sizeof(u32)));
  u64 at = 0;
  for (u32 j = 0; j < nq; ++j) {
    desc[j].g.gk = g_batch_arena.k + at;
    desc[j].g.gv = g_batch_arena.v + at;
    desc[j].stats = g_batch_stats + j;
    at += gel[j];
  }
  HIPCHK(hipMemcpyAsync(g_batch_desc, desc.data(), nq * sizeof(SsspParams), hipMemcpyHostToDevice, s));
  int occ = multi_occupancy(team, lds);
  if (occ < 1) return fail(PBH_EDEVICE, "sssp_batch: kernel cannot be resident with %zu bytes of LDS", lds);
  int grid = (int)std::min<u64>(nq, (u64)occ * (u64)cus);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(launch_fill_multi(g_batch_desc, nq, maxn, g_batch_counter, s));
  HIPCHK(hipEventRecord(e0, s));
  HIPCHK(launch_sssp_multi(team, g_batch_desc, nq, g_batch_counter, lds, grid, s));
  HIPCHK(hipEventRecord(e1, s));
  std::vector<SsspDevStats> ds(nq);
  HIPCHK(hipMemcpyAsync(ds.data(), g_batch_stats, nq * sizeof(SsspDevStats), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::vector<u32> redo;
  for (u32 j = 0; j < nq; ++j) {
    if (ds[j].err == E_CAPACITY) {
      redo.push_back(order[j]);
    } else if (ds[j].err) {
      return fail(PBH_EINTERNAL, "sssp_batch: query %u: device-side heap check failed (code %lld)", order[j],
                  ds[j].err);
    }
  }
  if (stats) {
    for (u32 j = 0; j < nq; ++j) {
      if (ds[j].err) continue;  // rerun below
      stats->rounds += ds[j].rounds;
      stats->relaxations += ds[j].relax;
      stats->updates += ds[j].updates;
      stats->heap_elems += ds[j].elems;
      stats->extracted += ds[j].extracted;
      stats->last_key = j == 0 ? ds[j].last_key : std::max(stats->last_key, (uint64_t)ds[j].last_key);
      for (int i = 0; i < 16 && i < MAXL; ++i) stats->resolves[i] += ds[j].resolves[i];
    }
    stats->levels = 0;
    stats->d = dmax;
    stats->team = (u32)team;
    stats->lds_levels = (u32)(lds / 12);
    stats->kernel_ms = ms;
  }
  // Queries whose heap outgrew its slice run again alone, starting from the
  // plain rule's bound m + 1 (and growing further if that overflows too).
  // Their trace records keep the query's index; the records of the rounds
  // the first run traced before it stopped stay as well (the same rounds are
  // traced again, so those rounds appear twice).
  for (u32 i : redo) {
    const sssp_query& q = queries[i];
    sssp_opts o2 = o;
    o2.d = qd[i];
    o2.team = (u32)team;
    o2.heap_capacity = q.m + 1;
    sssp_stats s2;
    int rc = sssp_run(q.offsets, q.targets, q.weights, q.n, q.m, q.source, q.dist_out, &o2, &s2, stream, i);
    if (rc) return rc;
    if (stats) {
      stats->rounds += s2.rounds;
      stats->relaxations += s2.relaxations;
      stats->updates += s2.updates;
      stats->heap_elems += s2.heap_elems;
      stats->extracted += s2.extracted;
      stats->kernel_ms += s2.kernel_ms;
    }
  }
  return PBH_OK;
}

int sssp(const uint64_t* offsets, const uint32_t* targets, const uint32_t* weights, uint32_t n, uint64_t m,
         uint32_t source, uint64_t* dist_out) {
  return sssp_ex(offsets, targets, weights, n, m, source, dist_out, nullptr, nullptr, nullptr);
}

}  // extern "C"

namespace {

// Frontier trials on one query: a plain run of a few rounds gives the
// distance frontier D; every candidate (d = maxdeg * mult, team, k_max) then
// runs until all vertices closer than D are settled -- the same work for
// each -- and is timed.  The three fastest are timed again on a frontier four
// times deeper (the heap and the frontier grow during a run, so the early
// ranking can mislead), and the fastest there wins.
struct TuneCand {
  u32 d, team, kmax;
  double ms;
};

// Ranks candidate settings for one query; *ranked receives at most three,
// fastest first (the two run to the end, when that stage ran, then the third
// of the frontier trials), with their d, team and k_max.
int tune_query(const uint64_t* offsets, const uint32_t* targets, const uint32_t* weights, uint32_t n, uint64_t m,
               uint32_t source, uint64_t* dist_out, const sssp_opts& user, void* stream,
               std::vector<TuneCand>* ranked, u32* maxdeg_out) {
  sssp_opts base = user;
  base.stop_key = 0;
  base.max_rounds = 0;
  base.trace_features = nullptr;
  base.d = 0;
  base.d_scale = 0;
  // frontiers: after n/32 and n/8 plain rounds
  u64 D[2] = {KINF, KINF};
  u32 maxdeg = 1;
  const u32 rounds[2] = {std::min<u32>(65536u, std::max<u32>(256u, n / 32)),
                         std::min<u32>(262144u, std::max<u32>(1024u, n / 8))};
  for (int s = 0; s < 2; ++s) {
    sssp_opts t0 = base;
    t0.k_rule = 0;
    t0.max_rounds = rounds[s];
    sssp_stats s0;
    int rc = sssp_ex(offsets, targets, weights, n, m, source, dist_out, &t0, &s0, stream);
    if (rc) return rc;
    maxdeg = s0.d;
    D[s] = s0.last_key;  // UINT64_MAX: the whole run fits; candidates run to the end
  }
  const bool spec = user.k_rule != 0;
  const u32 kms[3] = {1, 64, 256};  // k_max 1 = the plain rule, for graphs where pulling ahead does not pay
  std::vector<TuneCand> cands;
  for (u32 mult = 1; (u64)maxdeg * mult <= 2048 || mult == 1; mult *= 2) {
    const u32 d = maxdeg * mult;
    std::vector<u32> teams;
    if (user.team)
      teams = {user.team};
    else if (d < 64)
      teams = {64};
    else if (d <= 2048)
      teams = {64, 256};
    else
      teams = {1024};
    for (u32 tm : teams)
      for (int ki = 0; ki < (spec ? 3 : 1); ++ki)
        cands.push_back(TuneCand{d, tm, spec ? kms[ki] : user.k_max, 0.0});
  }
  auto trial = [&](TuneCand& c, u64 stop) -> int {
    sssp_opts t = base;
    t.d = c.d;
    t.team = c.team;
    t.k_max = c.kmax;
    t.stop_key = stop == KINF ? 0 : stop;
    sssp_stats st;
    int rc = sssp_ex(offsets, targets, weights, n, m, source, dist_out, &t, &st, stream);
    c.ms = rc ? 1e300 : st.kernel_ms;
    return rc == PBH_EINVAL ? 0 : rc;  // a candidate whose LDS levels do not fit is skipped
  };
  for (TuneCand& c : cands)
    if (int rc = trial(c, D[0])) return rc;
  std::sort(cands.begin(), cands.end(), [](const TuneCand& a, const TuneCand& b) { return a.ms < b.ms; });
  if (cands.empty() || cands[0].ms >= 1e300) return fail(PBH_EINTERNAL, "sssp_autotune: every candidate failed");
  if (cands.size() > 3) cands.resize(3);
  if (D[0] != KINF) {
    for (TuneCand& c : cands)
      if (int rc = trial(c, D[1])) return rc;
    std::sort(cands.begin(), cands.end(), [](const TuneCand& a, const TuneCand& b) { return a.ms < b.ms; });
    // The frontier trials cover the first n/8 settled vertices at most; the
    // cost of a large d grows with the heap, so the two best are run to the
    // end and the faster of those wins.
    if (D[1] != KINF) {
      std::vector<TuneCand> third(cands.begin() + std::min<size_t>(2, cands.size()), cands.end());
      if (cands.size() > 2) cands.resize(2);
      for (TuneCand& c : cands)
        if (int rc = trial(c, KINF)) return rc;
      std::sort(cands.begin(), cands.end(), [](const TuneCand& a, const TuneCand& b) { return a.ms < b.ms; });
      cands.insert(cands.end(), third.begin(), third.end());
    }
  }
  *ranked = cands;
  *maxdeg_out = maxdeg;
  return PBH_OK;
}

}  // namespace

extern "C" {

int sssp_autotune(const uint64_t* offsets, const uint32_t* targets, const uint32_t* weights, uint32_t n,
                  uint64_t m, uint32_t source, uint64_t* dist_out, sssp_opts* opts, void* stream) {
  if (!opts) return fail(PBH_EINVAL, "sssp_autotune: opts is NULL");
  std::vector<TuneCand> ranked;
  u32 maxdeg = 1;
  int rc = tune_query(offsets, targets, weights, n, m, source, dist_out, *opts, stream, &ranked, &maxdeg);
  if (rc) return rc;
  opts->d = ranked[0].d;
  opts->d_scale = 0;
  opts->k_max = ranked[0].kmax;
  opts->team = ranked[0].team;
  opts->k_scale = opts->k_scale > 0.0f ? opts->k_scale : 1.0f;
  // Learned rule, k_every left to the tuner: the winner (whose time is that
  // of a whole run) also runs with the model every 4th and every 16th round;
  // the fastest of the three stays.
  if (opts->k_rule == 2 && opts->k_every == 0 && ranked[0].kmax != 1) {
    sssp_opts t = *opts;
    t.stop_key = 0;
    t.max_rounds = 0;
    t.trace_features = nullptr;
    double best = ranked[0].ms;
    opts->k_every = 1;
    for (u32 ke : {4u, 16u}) {
      t.k_every = ke;
      sssp_stats st;
      rc = sssp_ex(offsets, targets, weights, n, m, source, dist_out, &t, &st, stream);
      if (rc) return rc;
      if (st.kernel_ms < best) {
        best = st.kernel_ms;
        opts->k_every = ke;
      }
    }
  }
  return PBH_OK;
}

int sssp_batch_autotune(const sssp_query* queries, uint32_t nq, sssp_opts* opts, void* stream) {
  if (!opts) return fail(PBH_EINVAL, "sssp_batch_autotune: opts is NULL");
  if (nq == 0) return PBH_OK;
  if (!queries) return fail(PBH_EINVAL, "sssp_batch_autotune: queries is NULL");
  // The largest query is the batch's critical path: tune on it and apply
  // the same multiple of each query's maximum out-degree to all.
  u32 big = 0;
  for (u32 i = 1; i < nq; ++i)
    if (queries[i].m > queries[big].m) big = i;
  const sssp_query& q = queries[big];
  if (!q.offsets || !q.dist_out || (q.m > 0 && (!q.targets || !q.weights)) || q.n == 0 || q.source >= q.n)
    return fail(PBH_EINVAL, "sssp_batch_autotune: query %u is malformed", big);
  std::vector<TuneCand> ranked;
  u32 maxdeg = 1;
  int rc = tune_query(q.offsets, q.targets, q.weights, q.n, q.m, q.source, q.dist_out, *opts, stream, &ranked,
                      &maxdeg);
  if (rc) return rc;
  // The best settings for the largest query alone need not be the best for
  // the batch (every query runs with the same multiple, and the largest
  // query's ranking of close candidates varies from run to run): its (at most
  // three) best candidates, and every multiple of the maximum out-degree up
  // to d = 2048 with the winner's team and k_max, run the whole batch, and the
  // fastest launch wins.  (Not swept when the winner is the plain rule, whose
  // batch runs are long.)
  if (ranked[0].kmax != 1)
    for (u32 mult = 1; (u64)maxdeg * mult <= 2048 || mult == 1; mult *= 2) {
      TuneCand c{maxdeg * mult, ranked[0].team, ranked[0].kmax, 0.0};
      bool seen = false;
      for (const TuneCand& r : ranked) seen = seen || (r.d == c.d && r.team == c.team && r.kmax == c.kmax);
      if (!seen) ranked.push_back(c);
    }
  size_t best = 0;
  double best_ms = 1e300;
  for (size_t c = 0; c < ranked.size(); ++c) {
    sssp_opts t = *opts;
    t.d = 0;
    t.d_scale = ranked[c].d / maxdeg;
    t.k_max = ranked[c].kmax;
    t.team = ranked[c].team;
    t.stop_key = 0;
    t.max_rounds = 0;
    t.trace_features = nullptr;
    sssp_stats st;
    if ((rc = sssp_batch(queries, nq, &t, &st, stream))) return rc;
    if (st.kernel_ms < best_ms) {
      best_ms = st.kernel_ms;
      best = c;
    }
  }
  opts->d = 0;
  opts->d_scale = ranked[best].d / maxdeg;
  opts->k_max = ranked[best].kmax;
  opts->team = ranked[best].team;
  opts->k_scale = opts->k_scale > 0.0f ? opts->k_scale : 1.0f;
  return PBH_OK;
}

}  // extern "C"
