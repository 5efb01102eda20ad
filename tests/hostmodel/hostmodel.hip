// CPU driver for the heap and parDijkstra logic of the GPU kernels, for tests.
// The heap operations run the plain forms of the primitives (those of the
// one-workgroup kernels), the round loop the large-heap forms (staging,
// register select, more loads in flight).
//
// It instantiates the same team-templated code as kernels.hip with a
// one-thread team on host memory, so that CPU tests can run adversarial
// operation scripts through the exact schedule, capacity and growth logic.
// It is not part of the library and the library never calls it; results from
// here are checked against the oracle like any other implementation.
#include <algorithm>
#include <cmath>
#include <new>
#include <cstring>
#include <type_traits>
#include <vector>

#include "../../paper_1908_09378_amd/csrc/pbh_core.h"

using namespace bkt;
typedef long long i64;

namespace {

int levels_for(u32 d, u64 elems, int qmin) {
  int q = qmin;
  while (q < MAXL && nomB(d, q - 1) < elems) ++q;
  return q;
}

int ceil_log2(u64 x) {
  int b = 0;
  while (b < 63 && (1ull << b) < x) ++b;
  return b < 1 ? 1 : b;
}

// One record per Resolve(i) call, before and after it: the level sizes it
// is about and the deepest non-empty level.
struct ResolveRec {
  int lvl, after, ell, q;
  u32 nB0, nS0, nB1, nS1;  // levels i and i+1 (0 when i+1 does not exist)
  u64 cnt;                 // Resolve(i) executions so far
};
static std::vector<ResolveRec>* g_log = nullptr;

// HostPolicy that records every Resolve (the CPU tests of Algorithm 1's
// pre- and postconditions and of Theorem 1's schedule read the records).
struct TracePolicy {
  using L = Arr;
  using G = Arr;
  using SP = HeapState*;
  static void on_resolve(const Geom& g, HeapState* st, int i, bool after) {
    if (!g_log) return;
    ResolveRec r;
    r.lvl = i;
    r.after = after ? 1 : 0;
    r.ell = st->ell;
    r.q = g.q;
    r.nB0 = st->L[i].nB;
    r.nS0 = st->L[i].nS;
    r.nB1 = i + 1 < g.q ? st->L[i + 1].nB : 0;
    r.nS1 = i + 1 < g.q ? st->L[i + 1].nS : 0;
    r.cnt = st->L[i].cnt;
    g_log->push_back(r);
  }
};

struct HM {
  u32 id_cap, d;
  int q, sched;
  std::vector<u64> cur, ak, uk;
  std::vector<u32> bitmap, av, ui;
  HeapState st;
  TeamShared<1> ts;
  std::vector<ResolveRec> log;
};

// Routes the Resolve records of the operation that follows to h's log.
struct LogScope {
  explicit LogScope(HM* h) { g_log = &h->log; }
  ~LogScope() { g_log = nullptr; }
};

Geom geom(HM* h) {
  Geom g;
  g.d = h->d;
  g.q = h->q;
  g.qlds = 0;
  g.gk = h->ak.data();
  g.gv = h->av.data();
  g.lk = nullptr;
  g.lv = nullptr;
  return g;
}

void grow(HM* h) {
  h->q += 1;
  h->st.q = h->q;
  h->ak.resize(lvl_off(h->d, h->q));
  h->av.resize(lvl_off(h->d, h->q));
}

}  // namespace

extern "C" {

void* hm_create(u32 id_cap, u32 d, int sched) {
  HM* h = new HM;
  h->id_cap = id_cap;
  h->d = d;
  h->sched = sched;
  h->q = levels_for(d, id_cap, 1);
  h->cur.assign(id_cap, KINF);
  h->bitmap.assign((id_cap + 31) / 32, 0u);
  h->ak.resize(lvl_off(d, h->q));
  h->av.resize(lvl_off(d, h->q));
  state_init(&h->st, d, h->q);
  return h;
}

void hm_destroy(void* p) { delete static_cast<HM*>(p); }

int hm_update(void* hp, const u64* keys, const u32* ids, u64 count) {
  HM* h = static_cast<HM*>(hp);
  for (u64 i = 0; i < count; ++i)
    if (ids[i] >= h->id_cap || keys[i] == KINF) return -1;
  if (count == 0) return 0;
  u64 need = count < h->id_cap ? count : h->id_cap;
  h->uk.resize(need);
  h->ui.resize(need);
  h->st.aux[0] = h->st.aux[1] = h->st.aux[3] = 0;
  h->st.progress = 0;
  for (;;) {
    PbhParams p{};
    p.g = geom(h);
    p.cur = h->cur.data();
    p.bitmap = h->bitmap.data();
    p.nwords = (u32)h->bitmap.size();
    p.id_cap = h->id_cap;
    p.sched = h->sched;
    p.idbits = ceil_log2(h->id_cap);
    p.keys = keys;
    p.ids = ids;
    p.count = count;
    p.ukeys = h->uk.data();
    p.uids = h->ui.data();
    HostTeamPlain t{&h->ts};
    LogScope ls(h);
    pbh_update_body<HostTeamPlain, TracePolicy>(t, p.g, &h->st, p);
    if (h->st.err) return h->st.err;
    if (h->st.aux[3] == 0) return 0;
    if (h->q >= MAXL) return -2;
    grow(h);
  }
}

int hm_delete(void* hp, const u32* ids, u64 count) {
  HM* h = static_cast<HM*>(hp);
  for (u64 i = 0; i < count; ++i)
    if (ids[i] >= h->id_cap) return -1;
  if (count == 0) return 0;
  h->st.aux[1] = h->st.aux[3] = 0;
  for (;;) {
    PbhParams p{};
    p.g = geom(h);
    p.cur = h->cur.data();
    p.id_cap = h->id_cap;
    p.sched = h->sched;
    p.idbits = ceil_log2(h->id_cap);
    p.ids = ids;
    p.count = count;
    HostTeamPlain t{&h->ts};
    LogScope ls(h);
    pbh_delete_body<HostTeamPlain, TracePolicy>(t, p.g, &h->st, p);
    if (h->st.err) return h->st.err;
    if (h->st.aux[3] == 0) return 0;
    if (h->q >= MAXL) return -2;
    grow(h);
  }
}

int hm_extract(void* hp, u64 k, u64* ko, u32* io, u64* count) {
  HM* h = static_cast<HM*>(hp);
  h->st.progress = 0;
  *count = 0;
  if (k == 0) return 0;
  for (;;) {
    PbhParams p{};
    p.g = geom(h);
    p.cur = h->cur.data();
    p.id_cap = h->id_cap;
    p.sched = h->sched;
    p.idbits = ceil_log2(h->id_cap);
    p.k = k;
    p.okeys = ko;
    p.oids = io;
    HostTeamPlain t{&h->ts};
    LogScope ls(h);
    pbh_extract_body<HostTeamPlain, TracePolicy>(t, p.g, &h->st, p);
    if (h->st.err) return h->st.err;
    if (h->st.aux[3] == 0) break;
    if (h->q >= MAXL) return -2;
    grow(h);
  }
  *count = h->st.progress;
  return 0;
}

int hm_levels(void* hp, u32* q, int* ell, u32* nB, u32* nS, u64* pk, u32* pv, u64* cnt, u64* live) {
  HM* h = static_cast<HM*>(hp);
  *q = (u32)h->q;
  *ell = h->st.ell;
  *live = h->st.live;
  for (int i = 0; i < h->q; ++i) {
    nB[i] = h->st.L[i].nB;
    nS[i] = h->st.L[i].nS;
    pk[i] = h->st.L[i].pk;
    pv[i] = h->st.L[i].pv;
    cnt[i] = h->st.L[i].cnt;
  }
  return 0;
}

// Copies up to cap Resolve records (ints: lvl, after, ell, q, nB_i, nS_i,
// nB_i+1, nS_i+1, cnt; 9 per record) and clears the log; returns how many
// records there were.
u64 hm_resolve_log(void* hp, long long* out, u64 cap) {
  HM* h = static_cast<HM*>(hp);
  const u64 n = h->log.size();
  for (u64 j = 0; j < n && j < cap; ++j) {
    const ResolveRec& r = h->log[j];
    long long* o = out + 9 * j;
    o[0] = r.lvl, o[1] = r.after, o[2] = r.ell, o[3] = r.q;
    o[4] = r.nB0, o[5] = r.nS0, o[6] = r.nB1, o[7] = r.nS1, o[8] = (long long)r.cnt;
  }
  h->log.clear();
  return n;
}

// Dumps level i's B and S contents (for invariant checks).
int hm_level_items(void* hp, int i, u64* bk, u32* bv, u64* sk, u32* sv) {
  HM* h = static_cast<HM*>(hp);
  Geom g = geom(h);
  const Lvl& L = h->st.L[i];
  Arr B = lbuf(g, i, L.bsel), S = lbuf(g, i, 3 + L.ssel);
  std::memcpy(bk, B.k, L.nB * 8);
  std::memcpy(bv, B.v, L.nB * 4);
  std::memcpy(sk, S.k, L.nS * 8);
  std::memcpy(sv, S.v, L.nS * 4);
  return 0;
}

// The deep-level service of the SSSP kernel with the workers simulated on one
// thread: a worker's Resolve runs when a team waits for its level (mode 1,
// lazy: the workers are as slow as they may be), as soon as it is posted
// (mode 0, eager), or, from the round loop's own synchronisation points, at
// seeded random times (mode 2).  Every order it produces is one the device's
// workgroups can produce, at the granularity of whole Resolves: a Resolve(j)
// only starts when nobody holds level j or j+1.
struct SimDeep {
  static constexpr bool kOn = true;
  DeepCtl c;
  int lim, mode;
  u64 rng;
  int depth = 0;  // worker steps on the stack
  Geom g;
  const u64* cur;
  HeapState wst[MAXL];
  TeamShared<1> wts[MAXL];
  u64 runs = 0;

  bool coin() {
    rng = rng * 6364136223846793005ull + 1442695040888963407ull;
    return (rng >> 33) & 1u;
  }
  u64 wstage[MAXL][32];
  void run(int j) {
    HostTeam wt{&wts[j]};
    static_assert(sizeof(wstage[0]) >= 2 * 6 * 12 + 8, "worker staging (one thread, 4 outputs)");
    stage_setup(wt, reinterpret_cast<unsigned char*>(wstage[j]));
    ++depth;
    ++runs;
    deep_step<HostTeam, HostPolicy>(wt, g, &wst[j], cur, j, *this);
    --depth;
  }
  // Random mode, from the round loop only (no worker step on the stack):
  // run pending Resolves of random levels.
  void maybe_run() {
    if (mode != 2 || depth) return;
    for (int j = g.q - 1; j >= lim; --j)
      while (!c.err && c.done[j] != c.req[j] && coin()) run(j);
  }
  bool wait_idle(const HostTeam&, int j) {
    while (!c.err && c.done[j] != c.req[j]) run(j);
    return c.err == 0;
  }
  void post(const HostTeam&, int j) {
    c.req[j]++;
    if (mode == 0 || (mode == 2 && depth == 0 && coin()))
      while (!c.err && c.done[j] != c.req[j]) run(j);
  }
  void done(const HostTeam&, int j) { c.done[j]++; }
  void publish(const HostTeam&) {}
  void get(const HostTeam&, HeapState* st, int j) { st->L[j] = c.L[j]; }
  void put(const HostTeam&, HeapState* st, int j) { c.L[j] = st->L[j]; }
  u64 deeper(const HostTeam&, int j) { return c.deeper[j]; }
  void set_deeper(const HostTeam&, int j, u64 v) { c.deeper[j] = v; }
  void account(const HostTeam&, int i, long long drop, long long d1, u64 elems, u64) {
    for (int j = lim; j <= i; ++j) c.deeper[j] += (u64)drop;
    c.deeper[i + 1] += (u64)d1;
    c.elems += elems;
  }
  u64 front_account(const HostTeam&, int j, long long d) { return c.deeper[j] += (u64)d; }
  void fail(const HostTeam&, int code) {
    if (!c.err) c.err = code;
  }
  int error(const HostTeam&) { return c.err; }
  void merge_stats(const HostTeam&, HeapState* st, int, int) { st->elems += c.elems; }
  void leave(const HostTeam&) { c.exit = 1; }
  void beat(const HostTeam&, u32 r) { c.beat = r; }
};

// Invariant checks run after every operation of the round loop: the smallest
// live element of the heap (key == dist[id]) sits in B_0; with the plain rule
// every reached vertex is either extracted or live in the heap exactly once;
// and the level order of Section 2.2: every element of B_i is <= p_i, and
// every element of every deeper level is > p_i.  With simulated deep-level
// workers the state checked is the round loop's levels plus the workers'
// published ones (every worker is between Resolves here).  Records the round
// of the first violation.
struct LiveCheck {
  const u64* dist;
  u32 n;
  bool plain;
  int* first_bad;  // -1 if none
  u64* info;       // what was violated: (1, key, id) misplaced minimum, (2, live, reached), (3, level, 0)
  SimDeep* deep;   // null: no workers
  void operator()(const Geom& g, HeapState* st0, const SsspCounters& c) const {
    if (*first_bad >= 0) return;
    HeapState merged;
    HeapState* st = st0;
    if (deep) {
      deep->maybe_run();
      merged = *st0;
      for (int j = deep->lim; j < g.q; ++j) merged.L[j] = deep->c.L[j];
      st = &merged;
    }
    for (int i = 0; i + 1 < g.q; ++i) {
      const KV p{st->L[i].pk, st->L[i].pv};
      if (p.k == KINF) continue;
      bool ok = true;
      Arr B = lbuf(g, i, st->L[i].bsel);
      for (u32 x = 0; x < st->L[i].nB; ++x) ok = ok && kv_le(KV{B.k[x], B.v[x]}, p);
      for (int j = i + 1; j < g.q; ++j)
        for (int w = 0; w < 2; ++w) {
          Arr A = lbuf(g, j, w ? 3 + st->L[j].ssel : st->L[j].bsel);
          const u32 na = w ? st->L[j].nS : st->L[j].nB;
          for (u32 x = 0; x < na; ++x) ok = ok && kv_less(p, KV{A.k[x], A.v[x]});
        }
      if (!ok) {
        *first_bad = (int)c.rounds;
        info[0] = 3, info[1] = (u64)i, info[2] = 0;
        return;
      }
    }
    std::vector<char> seen(n, 0);
    u64 live = 0, mk = KINF, mk0 = KINF;
    u32 mv = VINF, mv0 = VINF;
    for (int i = 0; i < g.q; ++i) {
      const Lvl& L = st->L[i];
      for (int w = 0; w < 2; ++w) {
        Arr A = lbuf(g, i, w ? 3 + L.ssel : L.bsel);
        u32 na = w ? L.nS : L.nB;
        for (u32 x = 0; x < na; ++x) {
          if (dist[A.v[x]] != A.k[x]) continue;
          if (!seen[A.v[x]]) seen[A.v[x]] = 1, ++live;
          if (A.k[x] < mk || (A.k[x] == mk && A.v[x] < mv)) mk = A.k[x], mv = A.v[x];
          if (i == 0 && w == 0 && (A.k[x] < mk0 || (A.k[x] == mk0 && A.v[x] < mv0))) mk0 = A.k[x], mv0 = A.v[x];
        }
      }
    }
    if (mk != KINF && (mk0 != mk || mv0 != mv)) {
      *first_bad = (int)c.rounds;
      info[0] = 1, info[1] = mk, info[2] = mv;
      return;
    }
    if (plain) {
      u64 reached = 0;
      for (u32 v = 0; v < n; ++v) reached += dist[v] != KINF;
      if (live + c.extracted != reached) {
        *first_bad = (int)c.rounds;
        info[0] = 2, info[1] = live, info[2] = reached;
      }
    }
  }
};

// parDijkstra with the kernel's round loop.  qlds levels are placed in a
// separate buffer, standing in for LDS.  stats: rounds, relaxations, updates,
// heap element touches, levels, resolves[0..15].
// deep_lim > 0: levels >= max(deep_lim, 2, qlds) are resolved by simulated
// deep-level workers (SimDeep, deep_mode, deep_seed).
int hm_sssp(const u64* off, const u32* tg, const u32* wt, u32 n, u64 m, u32 src, u64* dist, u32 d_opt,
            int sched, u64 hcap, int qlds, u64* stats, int rule, u32 kfix, u32 kmax, const u32* kseq, u32 kseq_len,
            const float* model, int check_live, u64 stop_key, u32 max_rounds, int deep_lim, int deep_mode,
            u64 deep_seed) {
  u64 md = 0;
  for (u32 u = 0; u < n; ++u) md = off[u + 1] - off[u] > md ? off[u + 1] - off[u] : md;
  u32 d = d_opt ? d_opt : (u32)(md ? md : 1);
  if (hcap == 0) hcap = m + 1;
  int q = levels_for(d, hcap, 2);
  if (qlds > q) qlds = q;
  std::vector<u64> gk(lvl_off(d, q) - lvl_off(d, qlds)), lk(lvl_off(d, qlds));
  std::vector<u32> gv(gk.size()), lv(lk.size());
  Geom g;
  g.d = d;
  g.q = q;
  g.qlds = qlds;
  g.gk = gk.data();
  g.gv = gv.data();
  g.lk = lk.data();
  g.lv = lv.data();
  HeapState st;
  state_init(&st, d, q);
  TeamShared<1> ts;
  HostTeam t{&ts};
  // the kernel's LDS staging for merges of HBM levels (here: every merge of
  // more than one tile goes through it)
  std::vector<u64> stage_buf(stage_bytes(1, HostTeam::kE) / 8 + 1);
  stage_setup(t, reinterpret_cast<unsigned char*>(stage_buf.data()));
  for (u32 v = 0; v < n; ++v) dist[v] = KINF;
  dist[src] = 0;
  SpecCfg sc;
  std::memset(&sc, 0, sizeof sc);
  sc.rule = rule;
  sc.kfix = kfix ? kfix : 1;
  sc.kmax = kmax ? kmax : 2 * d;
  if (sc.kmax > (u32)KMAX_ROUND) sc.kmax = KMAX_ROUND;
  sc.kseq = kseq;
  sc.kseq_len = kseq_len;
  sc.model = model;
  sc.kscale = 1.0f;
  sc.kevery = 1;
  sc.stop_key = stop_key;
  sc.max_rounds = max_rounds;
  std::vector<u64> uk(2ull * sc.kmax * d);
  std::vector<u32> uv(2ull * sc.kmax * d);
  sc.uk = uk.data();
  sc.uv = uv.data();
  sc.tk = uk.data() + (u64)sc.kmax * d;
  sc.tv = uv.data() + (u64)sc.kmax * d;
  SsspCounters c;
  int first_bad = -1;
  u64 info[3] = {0, 0, 0};
  int lim = deep_lim > 0 ? std::max(std::max(deep_lim, 2), qlds) : MAXL;
  SimDeep* sim = nullptr;
  std::vector<char> simbuf;
  if (lim < q) {
    simbuf.assign(sizeof(SimDeep), 0);
    sim = new (simbuf.data()) SimDeep();
    std::memset(&sim->c, 0, sizeof sim->c);
    sim->lim = lim;
    sim->mode = deep_mode;
    sim->rng = deep_seed * 2654435761ull + 1;
    sim->g = g;
    sim->cur = dist;
    for (int j = 0; j < MAXL; ++j) {
      state_init(&sim->wst[j], d, q);
      sim->c.L[j] = Lvl{0, 0, 0, 0, KINF, VINF, 0};
    }
  } else {
    lim = MAXL;
  }
  // The plain rule runs the plain-rule-only instantiation (as the kernel
  // does), the other rules the general one.
  auto run = [&](auto spec_tag) {
    constexpr bool SPEC = decltype(spec_tag)::value;
    if (check_live) {
      LiveCheck hk{dist, n, rule == 0, &first_bad, info, sim};
      if (sim)
        sssp_rounds<HostTeam, HostPolicy, LiveCheck, SimDeep, SPEC>(t, g, &st, off, tg, wt, dist, n, src, sched, sc,
                                                                    &c, hk, sim, lim);
      else
        sssp_rounds<HostTeam, HostPolicy, LiveCheck, NoDeepSync, SPEC>(t, g, &st, off, tg, wt, dist, n, src, sched,
                                                                       sc, &c, hk);
    } else if (sim) {
      sssp_rounds<HostTeam, HostPolicy, NoHook, SimDeep, SPEC>(t, g, &st, off, tg, wt, dist, n, src, sched, sc, &c,
                                                               NoHook(), sim, lim);
    } else {
      sssp_rounds<HostTeam, HostPolicy, NoHook, NoDeepSync, SPEC>(t, g, &st, off, tg, wt, dist, n, src, sched, sc, &c);
    }
  };
  if (rule == 0)
    run(std::false_type());
  else
    run(std::true_type());
  stats[28] = sim ? sim->runs : 0;
  stats[29] = sim ? (u64)sim->lim : 0;
  if (sim) sim->~SimDeep();
  stats[26] = c.last_key;
  stats[27] = c.stopped;
  stats[22] = (u64)(i64)first_bad;
  stats[23] = info[0];
  stats[24] = info[1];
  stats[25] = info[2];
  stats[0] = c.rounds;
  stats[1] = c.relax;
  stats[2] = c.updates;
  stats[3] = st.elems;
  stats[4] = (u64)q;
  for (int i = 0; i < MAXL; ++i) stats[5 + i] = st.L[i].cnt;
  stats[21] = c.extracted;
  return st.err;
}

}  // extern "C"
