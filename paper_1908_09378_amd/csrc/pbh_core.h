// Parallel bucket heap (Section 2.2) and parDijkstra rounds (Section 4.1),
// written once against a "team" (pbh_team.h): every thread of the team runs the
// same control flow on team-uniform values; the data-parallel steps (Merge,
// DeleteDuplicates, Select, PrefixSums, the relaxation) are split across the
// team's threads.
//
// Elements are (key u64, id u32) in structure-of-arrays form, ordered by
// (key, id).  Level i has a bucket B_i and a signal buffer S_i, each kept
// sorted by id (Section 2.1), nominal sizes |B_i| = 2d*4^i and |S_i| = d*4^i
// (Section 2.2), and a pivot p_i with B_i <= p_i < every element deeper.
#pragma once
#include "pbh_team.h"

#define PBH_HD __host__ __device__
#define PBH_INL __host__ __device__ __forceinline__
#define PBH_NOINL __host__ __device__ __attribute__((noinline))

namespace bkt {

constexpr u64 KINF = ~0ull;
constexpr u32 VINF = ~0u;
constexpr int MAXL = 16;

enum { E_OK = 0, E_INVAL = -1, E_CAPACITY = -2, E_INTERNAL = -6 };

struct KV {
  u64 k;
  u32 v;
};
PBH_HD inline bool kv_less(KV a, KV b) { return a.k < b.k || (a.k == b.k && a.v < b.v); }
PBH_HD inline bool kv_le(KV a, KV b) { return !kv_less(b, a); }
PBH_HD inline KV kv_inf() { return KV{KINF, VINF}; }

// A view of an element array: keys and ids.  The pointer types carry the
// address space on the GPU (LDS levels -> ds_* instructions, HBM levels ->
// global_* instructions); the geometry hands out generic views (Arr) that are
// cast to the typed view of the level's placement.
template <class KP, class VP>
struct ArrT {
  KP k;
  VP v;
};
using Arr = ArrT<u64*, u32*>;
template <class A>
PBH_INL A as_arr(Arr a) {
  A r;
  r.k = (decltype(r.k))a.k;
  r.v = (decltype(r.v))a.v;
  return r;
}

// ---------------------------------------------------------------- geometry
// Nominal sizes from Section 2.2, and the allocated buffer sizes.  A level
// stores two B buffers (merge ping-pong, 4d*4^i each), one temporary T (4d*4^i)
// and two S buffers (2d*4^i each): 16d*4^i elements.  The allocated sizes
// leave room for what Algorithm 1 can hold between two Resolve(i): B_i may
// absorb elements of S_i that fall below p_i, and each Resolve(i-1) adds at
// most |S_{i-1}| + |B_{i-1}| to S_i.
PBH_HD inline u64 nomS(u32 d, int i) { return (u64)d << (2 * i); }
PBH_HD inline u64 nomB(u32 d, int i) { return (u64)d << (2 * i + 1); }
PBH_HD inline u64 capS(u32 d, int i) { return (u64)d << (2 * i + 1); }
PBH_HD inline u64 capB(u32 d, int i) { return (u64)d << (2 * i + 2); }
PBH_HD inline u64 lvl_size(u32 d, int i) { return (16ull * d) << (2 * i); }
PBH_HD inline u64 lvl_off(u32 d, int i) { return 16ull * d * (((1ull << (2 * i)) - 1ull) / 3ull); }

struct Geom {
  u32 d;
  int q;     // levels allocated
  int qlds;  // levels 0..qlds-1 live in LDS
  u64* gk;   // global arena (level qlds at offset 0)
  u32* gv;
  u64* lk;   // LDS arena
  u32* lv;
};

// Buffer w of level i: 0/1 = B ping-pong, 2 = T, 3/4 = S ping-pong.
PBH_HD inline Arr lbuf(const Geom& g, int i, int w) {
  u64 cb = capB(g.d, i);
  u64 off = (w < 3) ? (u64)w * cb : 3ull * cb + (u64)(w - 3) * capS(g.d, i);
  if (i < g.qlds) {
    u64 b = lvl_off(g.d, i) + off;
    return Arr{g.lk + b, g.lv + b};
  }
  u64 b = lvl_off(g.d, i) - lvl_off(g.d, g.qlds) + off;
  return Arr{g.gk + b, g.gv + b};
}

struct Lvl {
  u32 nB, nS;    // sizes of B_i and S_i
  u32 bsel;      // which B buffer (0/1) holds B_i
  u32 ssel;      // which S buffer (0/1) holds S_i
  u64 pk;        // pivot p_i = (pk, pv); KINF = +infinity
  u32 pv;
  u32 cnt;       // Resolve(i) executions
};

// Time accounting of a profiled SSSP run (ticks of the device's constant
// real-time clock): prof[i] for i < MAXL is the time inside Resolve(i); the
// other slots split each round into its steps.
enum {
  PROF_DRIVE = MAXL,  // Resolve(0), the schedule and refills after each operation
  PROF_PIECE,         // moving the next piece of a round's update list into S_0
  PROF_PROPOSE,       // features and the MLP (learned rule)
  PROF_EXTRACT,       // choosing and removing the round's minima from B_0
  PROF_RELAX,         // scanning their out-edges (atomicMin on dist)
  PROF_INTAKE,        // the round's updates: filter, sort by id, deduplicate
  PROF_OTHER,
  PROF_WAIT,          // waiting for a deep-level worker (inside PROF_DRIVE)
  PROF_N
};

struct HeapState {
  Lvl L[MAXL];
  int ell;       // deepest non-empty level, -1 if the heap is empty
  int err;
  u32 d;
  int q;
  u64 elems;     // heap elements read + written by level operations
  u64 live;      // elements in the heap (queue size)
  u64 progress;  // resumable progress of a multi-piece operation
  u64 aux[5];
  u32 prof_on;   // time accounting on (SSSP kernels only)
  // Levels resolved by their own workers (the deep-level service of the SSSP
  // kernel): this team's copies of their states are not kept up to date, so
  // the deepest level known to hold elements (-1: none) and the number of
  // elements in the worker levels stand in for them.
  int deep_floor;
  u64 deep_n;
  u64 prof_last;  // clock at the last lap mark
  u64 prof_res;   // clock at the start of the running Resolve
  u64 prof[PROF_N];
};

// The device's constant-rate real-time clock (0 on the host).
PBH_INL u64 pbh_clock() {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_s_memrealtime();
#else
  return 0;
#endif
}

// Lap mark of a profiled run: the time since the previous mark goes to `cat`.
// One thread keeps the books; marks sit after the team's barriers, so the
// time of a step includes its slowest wavefront.
template <class T, class SP>
PBH_INL void prof_lap(const T& t, SP st, int cat) {
  if (t.tid() == 0 && st->prof_on) {
    const u64 now = pbh_clock();
    st->prof[cat] += now - st->prof_last;
    st->prof_last = now;
  }
}

template <class SP>
PBH_HD inline void state_init(SP st, u32 d, int q) {
  for (int i = 0; i < MAXL; ++i) {
    st->L[i].nB = st->L[i].nS = st->L[i].bsel = st->L[i].ssel = st->L[i].cnt = 0;
    st->L[i].pk = KINF;
    st->L[i].pv = VINF;
  }
  st->ell = -1;
  st->err = 0;
  st->d = d;
  st->q = q;
  st->elems = st->live = st->progress = 0;
  for (int i = 0; i < 5; ++i) st->aux[i] = 0;
  st->prof_on = 0;
  st->deep_floor = -1;
  st->deep_n = 0;
  st->prof_last = st->prof_res = 0;
  for (int i = 0; i < PROF_N; ++i) st->prof[i] = 0;
}

// Field-wise copies of a level's state (the state may live in LDS, whose
// objects have no implicit copy into generic memory).
template <class SP>
PBH_INL Lvl lvl_load(SP st, int i) {
  Lvl a;
  a.nB = st->L[i].nB;
  a.nS = st->L[i].nS;
  a.bsel = st->L[i].bsel;
  a.ssel = st->L[i].ssel;
  a.pk = st->L[i].pk;
  a.pv = st->L[i].pv;
  a.cnt = st->L[i].cnt;
  return a;
}
template <class SP>
PBH_INL void lvl_store(SP st, int i, const Lvl& a) {
  st->L[i].nB = a.nB;
  st->L[i].nS = a.nS;
  st->L[i].bsel = a.bsel;
  st->L[i].ssel = a.ssel;
  st->L[i].pk = a.pk;
  st->L[i].pv = a.pv;
  st->L[i].cnt = a.cnt;
}

// Host-side policy: every array and the state live in ordinary memory.  The
// GPU policy (kernels.hip) types LDS levels, HBM levels and the state with
// their address spaces.
struct HostPolicy {
  using L = Arr;
  using G = Arr;
  using SP = HeapState*;
  // called before (after = false) and after every Resolve(i); the CPU tests'
  // policy records the level sizes there, the others do nothing
  template <class SPP>
  PBH_INL static void on_resolve(const Geom&, SPP, int, bool) {}
};

// ---------------------------------------------------------------- primitives

// Merge-path split (Green, McColl, Bader 2012): how many of the first `diag`
// elements of merge(A, B) by id come from A (A first on equal ids).
template <class VA, class VB>
PBH_INL u32 merge_path(VA av, u32 na, VB bv, u32 nb, u32 diag) {
  u32 lo = diag > nb ? diag - nb : 0u, hi = diag < na ? diag : na;
  while (lo < hi) {
    u32 mid = (lo + hi) >> 1;
    if (av[mid] <= bv[diag - 1 - mid])
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Merge + DeleteDuplicates (Algorithm 1; DeleteDuplicates by scan + prefix
// sums as in Lemma 2's proof).  A and B are sorted by id with unique ids; the
// output C (not aliasing A or B) is sorted by id with unique ids.  For a pair
// of copies of one id the one whose key equals cur[id] (the live one) is kept;
// if neither is live both are dropped; without cur the smaller key is kept
// (Section 2.1: duplicates keep the smaller priority).  With filterB, B
// elements that are not live are dropped as well (used when elements move up
// into B_0, so that B_0 holds only live elements).
enum { PREFER_LIVE = 0, PREFER_A = 1, PREFER_B = 2 };

template <class T, int E, class AA, class AB, class AC>
PBH_INL u32 merge_dedup_e(const T& t, AA A, u32 na, AB B, u32 nb, AC C, const u64* cur, bool filterB, int prefer) {
  const u32 total = na + nb;
  u32 out = 0;
  for (u32 base = 0; base < total; base += (u32)T::kNT * E) {
    u32 d0 = base + (u32)t.tid() * E;
    d0 = d0 < total ? d0 : total;
    u32 d1 = d0 + E < total ? d0 + E : total;
    u32 i = merge_path(A.v, na, B.v, nb, d0), j = d0 - i;
    u64 ko[E];
    u32 vo[E];
    u32 keep = 0;
#pragma unroll
    for (int s = 0; s < E; ++s) {
      ko[s] = 0;
      vo[s] = 0;
      if (d0 + s < d1) {
        bool takeA = i < na && (j >= nb || A.v[i] <= B.v[j]);
        if (takeA) {
          u64 ka = A.k[i];
          u32 va = A.v[i];
          bool kp = true;
          if (j < nb && B.v[j] == va) {
            u64 kb = B.k[j];
            if (prefer == PREFER_B) {
              ka = kb;
            } else if (prefer == PREFER_A) {
            } else if (kb != ka) {
              if (cur) {
                u64 c = t.load_cur(cur + va);
                if (ka == c) {
                } else if (kb == c) {
                  ka = kb;
                } else {
                  kp = false;
                }
              } else if (kb < ka) {
                ka = kb;
              }
            }
          }
          ko[s] = ka;
          vo[s] = va;
          keep |= (u32)kp << s;
          ++i;
        } else {
          u64 kb = B.k[j];
          u32 vb = B.v[j];
          bool kp = !(i > 0 && A.v[i - 1] == vb);
          if (kp && filterB && t.load_cur(cur + vb) != kb) kp = false;
          ko[s] = kb;
          vo[s] = vb;
          keep |= (u32)kp << s;
          ++j;
        }
      }
    }
    u32 tot;
    u32 w = out + t.scan_excl((u32)__builtin_popcount(keep), &tot);
#pragma unroll
    for (int s = 0; s < E; ++s)
      if ((keep >> s) & 1u) {
        C.k[w] = ko[s];
        C.v[w] = vo[s];
        ++w;
      }
    out += tot;
  }
  t.sync();
  return out;
}

// Bytes of the staging area of a team of NT threads walking E outputs each.
PBH_HD inline u64 stage_bytes(int nt, int e) {
  const u64 w = (u64)nt * (u64)e + 2u;
  return ((2u * w * 12u + ((u64)nt + 1u) * 4u) + 7u) & ~7ull;
}
// Carves the staging area out of `base` (8-byte aligned).
template <class T, class BP>
PBH_INL void stage_setup(T& t, BP base) {
  const u64 w = (u64)T::kNT * T::kE + 2u;
  t.stk = (decltype(t.stk))base;
  t.stv = (decltype(t.stv))(base + 2u * w * 8u);
  t.stp = (decltype(t.stp))(base + 2u * w * 12u);
}

// Merge + DeleteDuplicates of arrays in HBM through the team's LDS staging
// area, with the same result as merge_dedup_e.  The merge-path split of every
// tile boundary is found first, a team-sized batch of boundaries at a time
// (one binary search per thread, all in flight together), instead of one
// search per thread per tile; then each tile's two input windows are loaded
// into LDS with coalesced reads (plus A's element before the window and B's
// element after it, which the duplicate checks look at), and the per-thread
// merge-path searches and walks run on LDS.
template <class T, class AA, class AB, class AC>
PBH_INL u32 merge_dedup_staged(const T& t, AA A, u32 na, AB B, u32 nb, AC C, const u64* cur, bool filterB,
                               int prefer) {
  constexpr int E = T::kE;
  constexpr u32 TILE = (u32)T::kNT * E;
  constexpr u32 W = TILE + 2u;
  const u32 total = na + nb;
  const auto ka = t.stk;  // window of A: keys ka[0..W), ids va[0..W)
  const auto kb = ka + W;  // window of B
  const auto va = t.stv;
  const auto vb = va + W;
  const auto sp = t.stp;
  u32 out = 0;
  for (u32 cbase = 0; cbase < total; cbase += TILE * (u32)T::kNT) {
    u32 ntile = (total - cbase + TILE - 1) / TILE;
    ntile = ntile < (u32)T::kNT ? ntile : (u32)T::kNT;
    for (u32 j = (u32)t.tid(); j <= ntile; j += (u32)T::kNT) {
      const u64 dg = (u64)cbase + (u64)j * TILE;
      sp[j] = merge_path(A.v, na, B.v, nb, dg < total ? (u32)dg : total);
    }
    t.sync();
    for (u32 k = 0; k < ntile; ++k) {
      const u32 d0 = cbase + k * TILE, d1 = total - d0 < TILE ? total : d0 + TILE;
      const u32 a0 = sp[k], a1 = sp[k + 1], b0 = d0 - a0, b1 = d1 - a1;
      // the windows reach one element past the tile's inputs (the walk
      // compares with the next element of the other array) and A's one
      // before (a B element is checked against A's previous id)
      const u32 abase = a0 > 0 ? a0 - 1 : 0;
      const u32 aend = a1 < na ? a1 + 1 : a1, bend = b1 < nb ? b1 + 1 : b1;
      {
        // every load of both windows in flight before the first LDS store
        constexpr int R = (int)((W + T::kNT - 1) / T::kNT);
        const u32 la = aend - abase, lb = bend - b0;
        u64 xk[R], yk[R];
        u32 xv[R], yv[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const u32 x = (u32)t.tid() + (u32)r * (u32)T::kNT;
          if (x < la) {
            xk[r] = A.k[abase + x];
            xv[r] = A.v[abase + x];
          }
          if (x < lb) {
            yk[r] = B.k[b0 + x];
            yv[r] = B.v[b0 + x];
          }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const u32 x = (u32)t.tid() + (u32)r * (u32)T::kNT;
          if (x < la) {
            ka[x] = xk[r];
            va[x] = xv[r];
          }
          if (x < lb) {
            kb[x] = yk[r];
            vb[x] = yv[r];
          }
        }
      }
      t.sync();
      // this thread's outputs [e0, e1) of the tile, relative to d0
      u32 e0 = (u32)t.tid() * E;
      e0 = e0 < d1 - d0 ? e0 : d1 - d0;
      const u32 e1 = e0 + E < d1 - d0 ? e0 + E : d1 - d0;
      u32 i = a0 + merge_path(va + (a0 - abase), a1 - a0, vb, b1 - b0, e0), j = d0 + e0 - i;
      u64 ko[E];
      u32 vo[E];
      u32 keep = 0;
#pragma unroll
      for (int s = 0; s < E; ++s) {
        ko[s] = 0;
        vo[s] = 0;
        if (e0 + s < e1) {
          const bool takeA = i < na && (j >= nb || va[i - abase] <= vb[j - b0]);
          if (takeA) {
            u64 kx = ka[i - abase];
            const u32 vx = va[i - abase];
            bool kp = true;
            if (j < nb && vb[j - b0] == vx) {
              const u64 ky = kb[j - b0];
              if (prefer == PREFER_B) {
                kx = ky;
              } else if (prefer == PREFER_A) {
              } else if (ky != kx) {
                if (cur) {
                  const u64 c = t.load_cur(cur + vx);
                  if (kx == c) {
                  } else if (ky == c) {
                    kx = ky;
                  } else {
                    kp = false;
                  }
                } else if (ky < kx) {
                  kx = ky;
                }
              }
            }
            ko[s] = kx;
            vo[s] = vx;
            keep |= (u32)kp << s;
            ++i;
          } else {
            const u64 ky = kb[j - b0];
            const u32 vy = vb[j - b0];
            bool kp = !(i > 0 && va[i - 1 - abase] == vy);
            if (kp && filterB && t.load_cur(cur + vy) != ky) kp = false;
            ko[s] = ky;
            vo[s] = vy;
            keep |= (u32)kp << s;
            ++j;
          }
        }
      }
      u32 tot;
      u32 w = out + t.scan_excl((u32)__builtin_popcount(keep), &tot);
#pragma unroll
      for (int s = 0; s < E; ++s)
        if ((keep >> s) & 1u) {
          C.k[w] = ko[s];
          C.v[w] = vo[s];
          ++w;
        }
      out += tot;
      t.sync();  // the next tile overwrites the windows
    }
  }
  t.sync();
  return out;
}

// Arrays that live in LDS are merged in place; the others (HBM) go through
// the staging area when the team has one.
template <class A>
struct in_lds {
  static constexpr bool v = false;
};
template <>
struct in_lds<ArrT<u64 PBH_LDS*, u32 PBH_LDS*>> {
  static constexpr bool v = true;
};

// Merge with the per-thread walk length chosen by size: a long walk amortises
// the merge-path search on big arrays, a short one keeps the chain of
// dependent reads short on the small top levels.  Arrays in HBM larger than a
// tile are merged through the LDS staging area when there is one.
template <class T, class AA, class AB, class AC>
PBH_INL u32 merge_dedup(const T& t, AA A, u32 na, AB B, u32 nb, AC C, const u64* cur, bool filterB,
                        int prefer = PREFER_LIVE) {
  if constexpr (T::kStage && !in_lds<AA>::v && !in_lds<AB>::v) {
    if (t.stk && na + nb > (u32)T::kNT * T::kE)
      return merge_dedup_staged(t, A, na, B, nb, C, cur, filterB, prefer);
  }
  if (T::kE > 2 && na + nb <= 2u * (u32)T::kNT)
    return merge_dedup_e<T, 2>(t, A, na, B, nb, C, cur, filterB, prefer);
  return merge_dedup_e<T, T::kE>(t, A, na, B, nb, C, cur, filterB, prefer);
}

// |{e in A : e <= p}|

template <class T, class AA>
PBH_INL u32 count_le(const T& t, AA A, u32 n, KV p) {
  if (p.k == KINF) return n;
  u32 c = 0;
  for (u32 base = 0; base < n; base += (u32)T::kNT * T::kRU) {
    u64 k[T::kRU];
    u32 v[T::kRU];
#pragma unroll
    for (int r = 0; r < T::kRU; ++r) {
      const u32 x = base + (u32)r * (u32)T::kNT + (u32)t.tid();
      k[r] = x < n ? A.k[x] : KINF;
      v[r] = x < n ? A.v[x] : VINF;
    }
#pragma unroll
    for (int r = 0; r < T::kRU; ++r) {
      const u32 x = base + (u32)r * (u32)T::kNT + (u32)t.tid();
      c += (x < n && kv_le(KV{k[r], v[r]}, p)) ? 1u : 0u;
    }
  }
  return t.sum(c);
}

// Finds the histogram bin where the r-th element (1-based) falls.
template <class T>
PBH_INL void hist_pick(const T& t, u32 r, u32* D, u32* below, u32* cnt) {
  constexpr int BPT = (256 + T::kNT - 1) / T::kNT;
  u32 b0 = (u32)t.tid() * BPT;
  u32 loc = 0;
#pragma unroll
  for (int q = 0; q < BPT; ++q)
    if (b0 + q < 256) loc += t.sh->hist[b0 + q];
  u32 tot;
  u32 pre = t.scan_excl(loc, &tot);
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    u32 b = b0 + q;
    if (b < 256) {
      u32 h = t.sh->hist[b];
      if (pre < r && r <= pre + h) {
        t.sh->b32[0] = b;
        t.sh->b32[1] = pre;
        t.sh->b32[2] = h;
      }
      pre += h;
    }
  }
  t.sync();
  *D = t.sh->b32[0];
  *below = t.sh->b32[1];
  *cnt = t.sh->b32[2];
  t.sync();
}

// r-th smallest by repeated team minima (or the (n-r+1)-th largest by
// repeated maxima) over at most 8 elements per thread held in registers; for
// the small ranks that Resolve asks for when one element leaves B_0.
template <class T, class AA>
PBH_INL KV select_small(const T& t, AA A, u32 n, u32 r) {
  const bool top = (n - r + 1) < r;
  u32 it = top ? n - r + 1 : r;
  u64 kk[8];
  u32 vv[8];
  u32 live = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    u32 x = (u32)t.tid() + (u32)j * (u32)T::kNT;
    kk[j] = 0;
    vv[j] = 0;
    if (x < n) {
      kk[j] = top ? ~A.k[x] : A.k[x];
      vv[j] = top ? ~A.v[x] : A.v[x];
      live |= 1u << j;
    }
  }
  u64 bk = KINF;
  u32 bv = VINF;
  for (u32 s = 0; s < it; ++s) {
    bk = KINF;
    bv = VINF;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if ((live >> j) & 1u) {
        bool lt = kk[j] < bk || (kk[j] == bk && vv[j] < bv);
        bk = lt ? kk[j] : bk;
        bv = lt ? vv[j] : bv;
      }
    t.minkv(bk, bv);
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (((live >> j) & 1u) && kk[j] == bk && vv[j] == bv) live &= ~(1u << j);
  }
  return top ? KV{~bk, ~bv} : KV{bk, bv};
}

// r-th smallest of n <= 2 * team size elements by counting: every element
// (at most two per thread) counts the elements below it; the one with r - 1
// below is the answer ((key, id) pairs are distinct).
template <class T, class AA>
PBH_INL KV select_rank(const T& t, AA A, u32 n, u32 r) {
  const u32 x0 = (u32)t.tid(), x1 = x0 + (u32)T::kNT;
  const u64 k0 = x0 < n ? A.k[x0] : KINF, k1 = x1 < n ? A.k[x1] : KINF;
  const u32 v0 = x0 < n ? A.v[x0] : VINF, v1 = x1 < n ? A.v[x1] : VINF;
  u32 c0 = 0, c1 = 0;
  for (u32 y = 0; y < n; ++y) {
    const u64 ky = A.k[y];
    const u32 vy = A.v[y];
    c0 += (ky < k0 || (ky == k0 && vy < v0)) ? 1u : 0u;
    c1 += (ky < k1 || (ky == k1 && vy < v1)) ? 1u : 0u;
  }
  t.sync();
  if (x0 < n && c0 + 1 == r) {
    t.sh->wk[0] = k0;
    t.sh->wv[0] = v0;
  }
  if (x1 < n && c1 + 1 == r) {
    t.sh->wk[0] = k1;
    t.sh->wv[0] = v1;
  }
  t.sync();
  const KV res{t.sh->wk[0], t.sh->wv[0]};
  t.sync();
  return res;
}

// Select over an array in HBM of at most RS elements per thread: every
// element is read once into registers and the radix passes run there (the
// same passes as select_kth, without re-reading the array for each byte).
constexpr int RS = 16;

template <class T, class AA>
PBH_INL KV select_reg(const T& t, AA A, u32 n, u32 r) {
  u64 k[RS];
  u32 v[RS];
  u64 lo = KINF, hi = 0;
#pragma unroll
  for (int q = 0; q < RS; ++q) {
    const u32 x = (u32)t.tid() + (u32)q * (u32)T::kNT;
    k[q] = x < n ? A.k[x] : KINF;
    v[q] = x < n ? A.v[x] : VINF;
  }
#pragma unroll
  for (int q = 0; q < RS; ++q) {
    const bool in = (u32)t.tid() + (u32)q * (u32)T::kNT < n;
    lo = k[q] < lo ? k[q] : lo;
    hi = (in && k[q] > hi) ? k[q] : hi;
  }
  t.minmax64(lo, hi);
  const u64 span = hi - lo;
  const int nb = span ? 64 - __builtin_clzll(span) : 0;
  const int top = (nb + 7) & ~7;
  u64 prefix = 0;
  u32 cnt = n;
  for (int s = top - 8; s >= 0; s -= 8) {
    for (u32 b = (u32)t.tid(); b < 256; b += (u32)T::kNT) t.sh->hist[b] = 0;
    t.sync();
#pragma unroll
    for (int q = 0; q < RS; ++q) {
      const bool in = (u32)t.tid() + (u32)q * (u32)T::kNT < n;
      const u64 dk = k[q] - lo;
      const bool m = in && ((s + 8 >= 64) ? true : ((dk >> (s + 8)) == prefix));
      if (m) t.hist_add(t.sh->hist, (u32)(dk >> s) & 255u);
    }
    t.sync();
    u32 D, below;
    hist_pick(t, r, &D, &below, &cnt);
    prefix = (prefix << 8) | D;
    r -= below;
  }
  const u64 K = lo + prefix;
  if (cnt == 1) {
#pragma unroll
    for (int q = 0; q < RS; ++q)
      if ((u32)t.tid() + (u32)q * (u32)T::kNT < n && k[q] == K) t.sh->b32[3] = v[q];
    t.sync();
    const u32 id = t.sh->b32[3];
    t.sync();
    return KV{K, id};
  }
  u32 idp = 0;
  for (int s = 24; s >= 0; s -= 8) {
    for (u32 b = (u32)t.tid(); b < 256; b += (u32)T::kNT) t.sh->hist[b] = 0;
    t.sync();
#pragma unroll
    for (int q = 0; q < RS; ++q) {
      const bool in = (u32)t.tid() + (u32)q * (u32)T::kNT < n;
      if (in && k[q] == K && (s == 24 || (v[q] >> (s + 8)) == idp)) t.hist_add(t.sh->hist, (v[q] >> s) & 255u);
    }
    t.sync();
    u32 D, below, c2;
    hist_pick(t, r, &D, &below, &c2);
    idp = (idp << 8) | D;
    r -= below;
  }
  return KV{K, idp};
}

// Select(A, r): the r-th smallest (key, id) of A, 1 <= r <= n.  Radix select,
// most significant byte first, over key - min(key) (only the bytes the key
// range needs), then over the id among elements with the selected key.  The
// paper sorted with a radix sort to select (Section 4.1); a radix select reads
// the candidates once per byte and sorts nothing.  Ranks within two of either
// end of a small array use select_small; other ranks in arrays of at most two
// elements per thread use select_rank; arrays in HBM of at most RS elements
// per thread use select_reg.
template <class T, class AA>
PBH_INL KV select_kth(const T& t, AA A, u32 n, u32 r) {
  if (n <= 8u * (u32)T::kNT && (r <= 2 || n - r + 1 <= 2)) return select_small(t, A, n, r);
  if (n <= 2u * (u32)T::kNT) return select_rank(t, A, n, r);
  if constexpr (T::kStage && !in_lds<AA>::v) {
    if (n <= (u32)RS * (u32)T::kNT) return select_reg(t, A, n, r);
  }
  u64 lo = KINF, hi = 0;
  for (u32 base = 0; base < n; base += (u32)T::kNT * T::kRU) {
    u64 k[T::kRU];
#pragma unroll
    for (int r = 0; r < T::kRU; ++r) {
      const u32 x = base + (u32)r * (u32)T::kNT + (u32)t.tid();
      k[r] = x < n ? A.k[x] : KINF;
    }
#pragma unroll
    for (int r = 0; r < T::kRU; ++r) {
      const u32 x = base + (u32)r * (u32)T::kNT + (u32)t.tid();
      lo = k[r] < lo ? k[r] : lo;
      hi = (x < n && k[r] > hi) ? k[r] : hi;
    }
  }
  t.minmax64(lo, hi);
  u64 span = hi - lo;
  int nb = span ? 64 - __builtin_clzll(span) : 0;
  int top = (nb + 7) & ~7;
  u64 prefix = 0;
  u32 cnt = n;
  for (int s = top - 8; s >= 0; s -= 8) {
    for (u32 b = (u32)t.tid(); b < 256; b += (u32)T::kNT) t.sh->hist[b] = 0;
    t.sync();
    for (u32 base = 0; base < n; base += (u32)T::kNT * T::kRU) {
      u64 k[T::kRU];
#pragma unroll
      for (int r = 0; r < T::kRU; ++r) {
        const u32 x = base + (u32)r * (u32)T::kNT + (u32)t.tid();
        k[r] = x < n ? A.k[x] : 0;
      }
#pragma unroll
      for (int r = 0; r < T::kRU; ++r) {
        const u32 x = base + (u32)r * (u32)T::kNT + (u32)t.tid();
        const u64 dk = k[r] - lo;
        const bool m = x < n && ((s + 8 >= 64) ? true : ((dk >> (s + 8)) == prefix));
        if (m) t.hist_add(t.sh->hist, (u32)(dk >> s) & 255u);
      }
    }
    t.sync();
    u32 D, below;
    hist_pick(t, r, &D, &below, &cnt);
    prefix = (prefix << 8) | D;
    r -= below;
  }
  const u64 K = lo + prefix;
  if (cnt == 1) {
    for (u32 base = 0; base < n; base += (u32)T::kNT * T::kRU) {
      u64 k[T::kRU];
#pragma unroll
      for (int r = 0; r < T::kRU; ++r) {
        const u32 x = base + (u32)r * (u32)T::kNT + (u32)t.tid();
        k[r] = x < n ? A.k[x] : ~K;
      }
#pragma unroll
      for (int r = 0; r < T::kRU; ++r)
        if (k[r] == K) t.sh->b32[3] = A.v[base + (u32)r * (u32)T::kNT + (u32)t.tid()];
    }
    t.sync();
    u32 id = t.sh->b32[3];
    t.sync();
    return KV{K, id};
  }
  u32 idp = 0;
  for (int s = 24; s >= 0; s -= 8) {
    for (u32 b = (u32)t.tid(); b < 256; b += (u32)T::kNT) t.sh->hist[b] = 0;
    t.sync();
    for (u32 base = 0; base < n; base += (u32)T::kNT * T::kRU) {
      u64 k[T::kRU];
      u32 v[T::kRU];
#pragma unroll
      for (int r = 0; r < T::kRU; ++r) {
        const u32 x = base + (u32)r * (u32)T::kNT + (u32)t.tid();
        k[r] = x < n ? A.k[x] : ~K;
        v[r] = x < n ? A.v[x] : 0u;
      }
#pragma unroll
      for (int r = 0; r < T::kRU; ++r)
        if (k[r] == K && (s == 24 || (v[r] >> (s + 8)) == idp)) t.hist_add(t.sh->hist, (v[r] >> s) & 255u);
    }
    t.sync();
    u32 D, below, c2;
    hist_pick(t, r, &D, &below, &c2);
    idp = (idp << 8) | D;
    r -= below;
  }
  return KV{K, idp};
}

// Stable three-way split of A (order by id is kept in each part):
// e <= p1 -> O0, p1 < e <= p2 -> O1, e > p2 -> O2.
template <class T, class AA, class A0, class A1, class A2>
PBH_INL void partition3(const T& t, AA A, u32 n, KV p1, KV p2, A0 O0, A1 O1, A2 O2, u32* n0, u32* n1,
                        u32* n2, const u64* live0 = nullptr) {
  // twice the elements per thread from HBM: more loads in flight per tile
  constexpr int E = (T::kStage && !in_lds<AA>::v) ? 2 * T::kE : T::kE;
  u32 c0t = 0, c1t = 0, c2t = 0;
  for (u32 base = 0; base < n; base += (u32)T::kNT * E) {
    u32 x0 = base + (u32)t.tid() * E;
    u64 kk[E];
    u32 vv[E];
    u32 cl[E];
    u32 c0 = 0, c1 = 0, c2 = 0;
#pragma unroll
    for (int s = 0; s < E; ++s) {
      kk[s] = 0;
      vv[s] = 0;
      cl[s] = 3;
      if (x0 + s < n) {
        kk[s] = A.k[x0 + s];
        vv[s] = A.v[x0 + s];
        KV e{kk[s], vv[s]};
        cl[s] = kv_le(e, p1) ? 0u : (kv_le(e, p2) ? 1u : 2u);
        // With live0, class-0 elements that are not live are dropped.
        if (cl[s] == 0 && live0 && t.load_cur(live0 + vv[s]) != kk[s]) cl[s] = 3;
        c0 += cl[s] == 0;
        c1 += cl[s] == 1;
        c2 += cl[s] == 2;
      }
    }
    u32 tot;
    u32 pre = t.scan_excl(c0 | (c1 << 16), &tot);
    u32 tot2;
    u32 pre2 = live0 ? t.scan_excl(c2, &tot2) : 0u;
    u32 before = x0 < n ? x0 - base : n - base;
    u32 o0 = c0t + (pre & 0xFFFFu), o1 = c1t + (pre >> 16);
    u32 o2 = c2t + (live0 ? pre2 : (before - (pre & 0xFFFFu) - (pre >> 16)));
#pragma unroll
    for (int s = 0; s < E; ++s) {
      if (cl[s] == 0) {
        O0.k[o0] = kk[s];
        O0.v[o0] = vv[s];
        ++o0;
      } else if (cl[s] == 1) {
        O1.k[o1] = kk[s];
        O1.v[o1] = vv[s];
        ++o1;
      } else if (cl[s] == 2) {
        O2.k[o2] = kk[s];
        O2.v[o2] = vv[s];
        ++o2;
      }
    }
    u32 tile = n - base < (u32)T::kNT * E ? n - base : (u32)T::kNT * E;
    u32 t0 = tot & 0xFFFFu, t1 = tot >> 16;
    c0t += t0;
    c1t += t1;
    c2t += live0 ? tot2 : tile - t0 - t1;
  }
  t.sync();
  *n0 = c0t;
  *n1 = c1t;
  *n2 = c2t;
}

struct DigitId {
  int s;
  PBH_INL u32 operator()(u64, u32 v) const { return (v >> s) & 255u; }
};
struct DigitKey {
  int s;
  u64 lo;
  PBH_INL u32 operator()(u64 k, u32) const { return (u32)((k - lo) >> s) & 255u; }
};

// One stable counting-sort pass on an 8-bit digit (LSD radix sort).  Ranks
// among equal digits inside a wavefront come from ballots (peer masks), and
// across wavefronts from per-wave digit counts in LDS.
template <class T, class AS, class AD, class F>
PBH_INL void radix_pass(const T& t, AS src, AD dst, u32 n, F dig) {
  for (u32 b = (u32)t.tid(); b < 256; b += (u32)T::kNT) t.sh->hist[b] = 0;
  t.sync();
  for (u32 x = (u32)t.tid(); x < n; x += (u32)T::kNT) t.hist_add(t.sh->hist, dig(src.k[x], src.v[x]));
  t.sync();
  {
    constexpr int BPT = (256 + T::kNT - 1) / T::kNT;
    u32 b0 = (u32)t.tid() * BPT, loc = 0;
#pragma unroll
    for (int q = 0; q < BPT; ++q)
      if (b0 + q < 256) loc += t.sh->hist[b0 + q];
    u32 tot;
    u32 pre = t.scan_excl(loc, &tot);
#pragma unroll
    for (int q = 0; q < BPT; ++q)
      if (b0 + q < 256) {
        t.sh->base[b0 + q] = pre;
        pre += t.sh->hist[b0 + q];
      }
  }
  t.sync();
  for (u32 tb = 0; tb < n; tb += (u32)T::kNT) {
    u32 x = tb + (u32)t.tid();
    bool valid = x < n;
    u64 k = valid ? src.k[x] : 0;
    u32 v = valid ? src.v[x] : 0;
    u32 dg = valid ? dig(k, v) : 0;
    u64 m = t.ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      bool bit = (dg >> b) & 1u;
      u64 bb = t.ballot(valid && bit);
      m &= bit ? bb : ~bb;
    }
    u32 rank = t.count_below(m);
    u32 cnt = (u32)__builtin_popcountll(m);
    for (u32 z = (u32)t.tid(); z < (u32)T::kNW * 256; z += (u32)T::kNT) t.sh->wcnt[z >> 8][z & 255] = 0;
    t.sync();
    if (valid && rank == 0) t.sh->wcnt[t.wave()][dg] = cnt;
    t.sync();
    for (u32 gd = (u32)t.tid(); gd < 256; gd += (u32)T::kNT) {
      u32 run = t.sh->base[gd];
      for (int w = 0; w < T::kNW; ++w) {
        u32 c = t.sh->wcnt[w][gd];
        t.sh->wcnt[w][gd] = run;
        run += c;
      }
      t.sh->base[gd] = run;
    }
    t.sync();
    if (valid) {
      u32 pos = t.sh->wcnt[t.wave()][dg] + rank;
      dst.k[pos] = k;
      dst.v[pos] = v;
    }
    t.sync();
  }
}

// Sorts n elements by id (idbits significant bits).  Returns true when the
// result ended in tmp (false: in a).
template <class T, class A>
PBH_INL bool sort_by_id(const T& t, A a, A tmp, u32 n, int idbits) {
  bool in_tmp = false;
  for (int s = 0; s < idbits; s += 8) {
    if (in_tmp)
      radix_pass(t, tmp, a, n, DigitId{s});
    else
      radix_pass(t, a, tmp, n, DigitId{s});
    in_tmp = !in_tmp;
  }
  return in_tmp;
}

// Sorts n elements by (key, id); returns true when the result is in tmp.
template <class T, class A>
PBH_INL bool sort_kv(const T& t, A a, A tmp, u32 n, int idbits) {
  bool in_tmp = sort_by_id(t, a, tmp, n, idbits);
  if (n == 0) return in_tmp;
  A src = in_tmp ? tmp : a;
  u64 lo = KINF, hi = 0;
  for (u32 x = (u32)t.tid(); x < n; x += (u32)T::kNT) {
    u64 k = src.k[x];
    lo = k < lo ? k : lo;
    hi = k > hi ? k : hi;
  }
  t.minmax64(lo, hi);
  u64 span = hi - lo;
  int nb = span ? 64 - __builtin_clzll(span) : 0;
  for (int s = 0; s < nb; s += 8) {
    if (in_tmp)
      radix_pass(t, tmp, a, n, DigitKey{s, lo});
    else
      radix_pass(t, a, tmp, n, DigitKey{s, lo});
    in_tmp = !in_tmp;
  }
  return in_tmp;
}

template <class T, class AS, class AD>
PBH_INL void copy_arr(const T& t, AS src, AD dst, u32 n) {
  for (u32 x = (u32)t.tid(); x < n; x += (u32)T::kNT) {
    dst.k[x] = src.k[x];
    dst.v[x] = src.v[x];
  }
  t.sync();
}

// ---------------------------------------------------------------- the heap

// Recomputes ell (deepest non-empty level) and sets p_j = +inf for j >= ell:
// the deepest non-empty level has nothing below it to separate from.
// A deep_floor set by the deep-level service counts as a non-empty level.
template <class SP>
PBH_INL void fix_ell(SP st, int q) {
  int e = -1;
  for (int j = q - 1; j >= 0; --j)
    if (st->L[j].nB + st->L[j].nS) {
      e = j;
      break;
    }
  if (st->deep_floor > e) e = st->deep_floor;
  st->ell = e;
  for (int j = e < 0 ? 0 : e; j < MAXL; ++j) {
    st->L[j].pk = KINF;
    st->L[j].pv = VINF;
  }
}

// Algorithm 1, Resolve(i): empty S_i and fill B_i, with level i's arrays of
// type AI and level i+1's of type AN.
//   EMPTY: B_i <- DeleteDuplicates(Merge(S_i, B_i)); if more than 2d*4^i
//          elements are <= p_i, p_i <- Select(B_i, 2d*4^i); elements > p_i move
//          to S_{i+1} <- Merge(S_{i+1}, B'_i).
//   FILL (if |B_i| < 2d*4^i and i is not the deepest non-empty level):
//          B_{i+1} <- DeleteDuplicates(Merge(B_{i+1}, S_{i+1}));
//          p_i <- Select(B_{i+1}, 2d*4^i - |B_i|); elements <= p_i move up into
//          B_i <- Merge(B_i, B'_{i+1}); elements > p_{i+1} go back to S_{i+1}.
// Readings (documented with the others): EMPTY also runs when B_i holds more
// than 2d*4^i elements with S_i empty (B_i can absorb elements of S_i during
// FILL of level i-1); the new p_i in FILL never exceeds p_{i+1}, so nothing
// deeper than level i+1 can be smaller than an element moved up; the two
// splits at the end of FILL are one three-way split.
template <class T, class P, class AI, class AN>
PBH_INL void resolve_t(T t, Geom g, typename P::SP st, const u64* cur, int i) {
  Lvl a = lvl_load(st, i);
  const bool nx = i + 1 < g.q;
  Lvl b = nx ? lvl_load(st, i + 1) : Lvl{0, 0, 0, 0, KINF, VINF, 0};
  int ell = st->ell;
  KV pi{a.pk, a.pv}, pn{b.pk, b.pv};
  const u32 cB = (u32)nomB(g.d, i);
  u64 touched = 0;
  int err = 0;
  if (a.nS > 0 || a.nB > cB) {
    AI S = as_arr<AI>(lbuf(g, i, 3 + a.ssel)), B = as_arr<AI>(lbuf(g, i, a.bsel)),
       M = as_arr<AI>(lbuf(g, i, a.bsel ^ 1));
    if ((u64)a.nS + a.nB > capB(g.d, i)) {
      err = E_INTERNAL;
      goto done;
    }
    // S_0 holds the latest updates, so at level 0 its copy of an id is the live one.
    u32 m = merge_dedup(t, S, a.nS, B, a.nB, M, cur, false, i == 0 ? PREFER_A : PREFER_LIVE);
    touched += 2ull * (a.nS + a.nB) + m;
    a.bsel ^= 1;
    a.nS = 0;
    a.ssel = 0;
    u32 num = count_le(t, M, m, pi);
    if (num > cB) {
      pi = select_kth(t, M, m, cB);
      num = cB;
      touched += m;
    }
    if (num < m) {
      if (!nx) {
        err = E_CAPACITY;
        goto done;
      }
      AI Lo = as_arr<AI>(lbuf(g, i, a.bsel ^ 1)), Hi = as_arr<AI>(lbuf(g, i, 2));
      u32 n0, n1, n2;
      partition3(t, M, m, pi, kv_inf(), Lo, Hi, Hi, &n0, &n1, &n2);
      touched += 3ull * m;
      a.bsel ^= 1;
      a.nB = n0;
      if ((u64)b.nS + n1 > capS(g.d, i + 1)) {
        err = E_INTERNAL;
        goto done;
      }
      AN Sn = as_arr<AN>(lbuf(g, i + 1, 3 + b.ssel)), Sn2 = as_arr<AN>(lbuf(g, i + 1, 3 + (b.ssel ^ 1)));
      u32 ms = merge_dedup(t, Sn, b.nS, Hi, n1, Sn2, cur, false);
      touched += 2ull * (b.nS + n1) + ms;
      b.ssel ^= 1;
      b.nS = ms;
      if (ell < i + 1) ell = i + 1;
    } else {
      a.nB = m;
    }
  }
  if (a.nB < cB && i < ell && nx) {
    AN Bn = as_arr<AN>(lbuf(g, i + 1, b.bsel)), Sn = as_arr<AN>(lbuf(g, i + 1, 3 + b.ssel)),
       M2 = as_arr<AN>(lbuf(g, i + 1, b.bsel ^ 1));
    if ((u64)b.nB + b.nS > capB(g.d, i + 1)) {
      err = E_INTERNAL;
      goto done;
    }
    u32 m2 = merge_dedup(t, Bn, b.nB, Sn, b.nS, M2, cur, false);
    touched += 2ull * (b.nB + b.nS) + m2;
    b.nS = 0;
    b.ssel = 0;
    b.bsel ^= 1;
    b.nB = m2;
    if (m2 > 0) {
      u32 r = cB - a.nB;
      KV pnew = (r >= m2) ? kv_inf() : select_kth(t, M2, m2, r);
      if (r < m2) touched += m2;
      if (kv_less(pn, pnew)) pnew = pn;
      AI Up = as_arr<AI>(lbuf(g, i, 2));
      AN Bk = as_arr<AN>(lbuf(g, i + 1, b.bsel ^ 1)), Sk = as_arr<AN>(lbuf(g, i + 1, 3));
      u32 nu, nb1, ns1;
      // Elements moving up into B_0 are checked for liveness here, all at once.
      partition3(t, M2, m2, pnew, pn, Up, Bk, Sk, &nu, &nb1, &ns1, i == 0 ? cur : nullptr);
      touched += 3ull * m2;
      b.bsel ^= 1;
      b.nB = nb1;
      b.nS = ns1;
      b.ssel = 0;
      AI Bi = as_arr<AI>(lbuf(g, i, a.bsel)), Bi2 = as_arr<AI>(lbuf(g, i, a.bsel ^ 1));
      u32 mb = merge_dedup(t, Bi, a.nB, Up, nu, Bi2, cur, false, i == 0 && cur != nullptr ? PREFER_B : PREFER_LIVE);
      touched += 2ull * (a.nB + nu) + mb;
      a.bsel ^= 1;
      a.nB = mb;
      pi = pnew;
    }
  }
  a.cnt++;
  a.pk = pi.k;
  a.pv = pi.v;
done:
  t.sync();
  if (t.tid() == 0) {
    if (err) {
      st->err = err;
    } else {
      lvl_store(st, i, a);
      if (nx) lvl_store(st, i + 1, b);
      st->elems += touched;
      fix_ell(st, g.q);
    }
  }
  t.sync();
}

template <class T, class P>
PBH_INL void resolve(const T& t, const Geom& g, typename P::SP st, const u64* cur, int i) {
  P::on_resolve(g, st, i, false);
  if (t.tid() == 0 && st->prof_on) st->prof_res = pbh_clock();
  if (i + 1 < g.qlds)
    resolve_t<T, P, typename P::L, typename P::L>(t, g, st, cur, i);
  else if (i < g.qlds)
    resolve_t<T, P, typename P::L, typename P::G>(t, g, st, cur, i);
  else
    resolve_t<T, P, typename P::G, typename P::G>(t, g, st, cur, i);
  if (t.tid() == 0 && st->prof_on) st->prof[i] += pbh_clock() - st->prof_res;
  P::on_resolve(g, st, i, true);
}

// Can Resolve(j) move its worst case (all of S_j and B_j) into level j+1?
template <class SP>
PBH_INL bool room_below(const Geom& g, SP st, int j) {
  if (j + 1 >= g.q) return true;
  u64 push = (u64)st->L[j].nS + st->L[j].nB;
  u64 bS = st->L[j + 1].nS, bB = st->L[j + 1].nB;
  return bS + push <= capS(g.d, j + 1) && bB + bS + push <= capB(g.d, j + 1);
}

enum { DRIVE_AFTER = 1, DRIVE_ENSURE = 2 };

// The resolution schedule, as one loop with a single call of Resolve (so each
// placement variant of Resolve is instantiated once per kernel).  Requests:
//
// * DRIVE_AFTER -- after an operation: Resolve(0), then the schedule:
//     sched 0 = Theorem 1: Resolve(i+1) after every fourth Resolve(i);
//     sched 1 = on demand (as the sequential bucket heap of Section 2.1 does):
//               Resolve(i+1) only when the next Resolve(i) would otherwise
//               violate its preconditions on level i+1.
// * DRIVE_ENSURE -- then, while B_0 is empty and the heap is not (possible
//     when dead copies thin out the levels below: Resolve(0) drops the dead
//     ones among the elements it moves up), let j be the shallowest non-empty
//     level below 0 and resolve levels j, j-1, ..., 0 (Resolve(j) first, so
//     that S_j elements above p_j move down and B_j is filled).  A cascade
//     puts a live element into B_0 or drops dead ones at level 0; the loop
//     gives up with E_INTERNAL after (elements + 1) * (q + 1) cascades rather
//     than spin.
//
// Every requested Resolve(x) first resolves the levels below x that lack
// room for what Resolve(x) may push down: find the first j >= x whose next
// level can take all of S_j and B_j, then resolve j, j-1, ..., x.  After
// Resolve(j), level j has S_j empty and |B_j| <= 2d*4^j, which always leaves
// room for level j-1.
//
// `res(i)` performs Resolve(i) on `st`: the team's own Resolve in the kernels,
// or the device-wide engine driven from the host.
//
// With the deep-level service (levels >= lim resolved by their own workers,
// Section 2.2.1), this caller never resolves a level >= lim itself: when the
// Theorem 1 schedule reaches Resolve(lim), `post(lim)` hands it to level lim's
// worker and the schedule of this caller ends there (the worker continues
// it); levels lack room only up to lim - 1 here (res(lim - 1) makes room in
// level lim itself); and when B_0 must be refilled but every level below 0
// that this caller holds is empty, `ensure()` refills it from the worker
// levels and the drive ends.  lim >= q: no workers.
template <class T, class SP, class R, class PO, class EN>
PBH_INL void drive_with(const T& t, const Geom& g, SP st, int sched, int what, R&& res, int lim, PO&& post,
                        EN&& ensure) {
  int tgt = -1, chain = -1;  // pending chain: levels chain, chain-1, ..., tgt
  int stage = (what & DRIVE_AFTER) ? 0 : 2;
  int si = 0;                // schedule position
  int ek = -1;               // refill position
  u64 cascades = 0, climit = 0;
  for (;;) {
    if (st->err) break;
    int lvl;
    if (chain >= 0) {
      lvl = chain;
      chain = chain > tgt ? chain - 1 : -1;
    } else {
      int x = -1;
      if (stage == 0) {
        x = 0;
        stage = 1;
        si = 0;
      } else if (stage == 1) {
        bool go = si + 1 < g.q && si + 1 <= st->ell;
        if (go) {
          if (sched == 0) {
            go = (st->L[si].cnt & 3u) == 0;
          } else {
            u64 bS = st->L[si + 1].nS, bB = st->L[si + 1].nB;
            go = bS > nomS(g.d, si + 1) - nomS(g.d, si) ||
                 (si + 1 < st->ell && bB < nomS(g.d, si + 1) + nomS(g.d, si));
          }
        }
        if (go && si + 1 >= lim) {
          post(si + 1);
          stage = 2;
        } else if (go) {
          x = si + 1;
          ++si;
        } else {
          stage = 2;
        }
      }
      if (x < 0 && stage == 2) {
        if (!(what & DRIVE_ENSURE)) break;
        if (ek < 0) {
          const int ell = st->ell;
          if (st->L[0].nB != 0 || ell < 1) break;
          int j = 1;
          u64 tot = 0;
          for (int l = 0; l <= ell; ++l) tot += (u64)st->L[l].nB + st->L[l].nS;
          while (j <= ell && j < lim && st->L[j].nB + st->L[j].nS == 0) ++j;
          if (j >= lim && j <= ell) {
            ensure();
            break;
          }
          if (cascades == 0) climit = (tot + 1) * (u64)(g.q + 1);
          if (j > ell || ++cascades > climit) {
            t.sync();
            if (t.tid() == 0) st->err = E_INTERNAL;
            t.sync();
            break;
          }
          ek = j;
        }
        x = ek--;
      }
      int j = x;
      while (j + 1 < g.q && j + 1 < lim && !room_below(g, st, j)) ++j;
      tgt = x;
      lvl = j;
      chain = j > x ? j - 1 : -1;
    }
    res(lvl);
  }
}

template <class T, class SP, class R>
PBH_INL void drive_with(const T& t, const Geom& g, SP st, int sched, int what, R&& res) {
  drive_with(t, g, st, sched, what, res, MAXL, [](int) {}, [] {});
}

template <class T, class P>
PBH_INL void drive(const T& t, const Geom& g, typename P::SP st, const u64* cur, int sched, int what) {
  drive_with(t, g, st, sched, what, [&](int lvl) { resolve<T, P>(t, g, st, cur, lvl); });
}

// ---------------------------------------------------------------- deep-level service
// Section 2.2.1 and Theorem 1: Resolve(i) only needs levels i and i+1, so
// Resolves of levels two apart can run at the same time.  The paper gives
// every level its own thread block (Section 4.1).  Here the team that runs the
// rounds (the "front") keeps levels 0 .. lim-1 -- among them every level in
// its LDS -- and each level i >= lim has a worker team of its own that runs
// Resolve(i) on request.  Level i+1's owner is idle whenever Resolve(i) runs:
//
//  * the owner of level i-1 (the front for i = lim) posts a request for
//    Resolve(i) after every fourth Resolve(i-1) (Theorem 1), and before each
//    Resolve(i-1) waits until every posted Resolve(i) is done;
//  * worker i, before each Resolve(i), waits until every posted Resolve(i+1)
//    is done; if level i+1 lacks room for what Resolve(i) can push down, it
//    posts an extra Resolve(i+1) and waits for it first.
//
// So Resolve(i) never overlaps Resolve(i-1) or Resolve(i+1), and the levels
// below lim leave the front's critical path: they run while the front goes on
// with its rounds.  A worker posts its own follow-up request (Theorem 1 again)
// before it reports its Resolve done, so "every level idle" is observed
// correctly by a scan from lim downwards.
//
// Whoever runs Resolve(i) sees real states of levels i and i+1 only.  Two
// facts stand in for the levels further down: deeper[j] = the number of
// elements in levels >= j (j >= lim; Resolve(i) moves elements between levels
// i and i+1 and drops dead ones, so it changes deeper[i+1] and lowers
// deeper[lim .. i]; a concurrent drop makes the value an upper bound), and
// HeapState::deep_floor, which makes the deepest-level computation (fix_ell)
// count "something below" as a non-empty level.  An upper bound is safe: a
// pivot stays finite (the last Select result) one Resolve longer than needed,
// which only moves elements down that could have stayed; a pivot never
// becomes +infinity while anything lies below it.
//
// Refilling an empty B_0 from the worker levels, which the schedule does not
// cover, is done by the front with every worker idle (it holds all levels and
// runs the one-team code), as are the final statistics.
struct DeepCtl {
  u32 req[MAXL];          // Resolve(i) requests posted
  u32 done[MAXL];         // Resolve(i) finished
  u64 deeper[MAXL + 1];   // elements in levels >= i, for i >= lim
  Lvl L[MAXL];            // states of the worker levels (level lim: also the front's, while worker lim is idle)
  u64 elems;              // heap elements touched by the workers' Resolves
  u64 busy[MAXL];         // clock ticks inside Resolve(i) of worker i (profiled runs)
  int err;                // first error of any team (E_*), 0 if none
  u32 exit;               // set by the front once every worker is idle at the end
  u32 beat;               // the front's round count, published every 1024 rounds (it is alive)
  u32 beat_pad;
};

enum { E_TIMEOUT = -5 };

template <class SP>
PBH_INL u64 lvl_count(SP st, int i) {
  return (u64)st->L[i].nB + st->L[i].nS;
}

// Worker i: one requested Resolve(i).  `sy` is the synchronisation layer
// (device spin waits and fences in the kernel, a deterministic scheduler in
// the CPU tests): wait_idle(t, j) returns once every posted Resolve(j) is done
// (false on an error), post(t, j) / done(t, j) count a request / completion
// after making this team's writes visible, get/put copy level states from /
// to the control block, deeper(t, j) reads deeper[j], account(...) applies a
// Resolve's changes to deeper[] and the element count.
template <class T, class P, class SY>
PBH_INL void deep_step(const T& t, const Geom& g, typename P::SP st, const u64* cur, int i, SY& sy) {
  const bool nx = i + 1 < g.q;
  if (nx && !sy.wait_idle(t, i + 1)) return;
  for (int tries = 0;; ++tries) {
    sy.get(t, st, i);
    if (nx) sy.get(t, st, i + 1);
    const u64 below = i + 2 < g.q ? sy.deeper(t, i + 2) : 0ull;
    if (t.tid() == 0) {
      st->deep_floor = below ? i + 2 : -1;
      fix_ell(st, g.q);
    }
    t.sync();
    if (!nx || room_below(g, st, i)) break;
    if (tries > 2 * MAXL) {
      sy.fail(t, E_INTERNAL);
      return;
    }
    sy.post(t, i + 1);  // an extra Resolve(i+1) makes room
    if (!sy.wait_idle(t, i + 1)) return;
  }
  const u64 c01 = lvl_count(st, i) + (nx ? lvl_count(st, i + 1) : 0ull);
  const u64 c1 = nx ? lvl_count(st, i + 1) : 0ull;
  const u64 e0 = st->elems;
  // worker levels are never in LDS: only the global placement is needed
  if (t.tid() == 0 && st->prof_on) st->prof_res = pbh_clock();
  resolve_t<T, P, typename P::G, typename P::G>(t, g, st, cur, i);
  if (t.tid() == 0 && st->prof_on) st->prof[i] += pbh_clock() - st->prof_res;
  if (st->err) {
    sy.fail(t, st->err);
    return;
  }
  const u64 n01 = lvl_count(st, i) + (nx ? lvl_count(st, i + 1) : 0ull);
  const u64 n1 = nx ? lvl_count(st, i + 1) : 0ull;
  sy.put(t, st, i);
  if (nx) sy.put(t, st, i + 1);
  sy.account(t, i, (long long)n01 - (long long)c01, (long long)n1 - (long long)c1, st->elems - e0,
             st->prof_on ? st->prof[i] : 0ull);
  if (nx && (st->L[i].cnt & 3u) == 0 && i + 1 <= st->ell) sy.post(t, i + 1);
  sy.done(t, i);
}

// The front's side of the service (levels 0 .. lim-1), handed to the round
// loop.  `sy` null: no workers, every level is the front's.
template <class T, class P, class SY>
struct DeepFront {
  SY* sy;
  int lim;
  bool hold;  // every worker idle and every level held by the front

  // Resolve(lvl) as the front runs it.  Resolve(lim - 1) shares level lim
  // with worker lim: wait until that worker is idle, take level lim's state,
  // make room in it if needed (an extra Resolve(lim) by the worker), and
  // hand the level back afterwards.  (One call of resolve() per kernel: each
  // placement variant of Resolve is instantiated once.)
  PBH_INL void res(const T& t, const Geom& g, typename P::SP st, const u64* cur, int lvl) {
    const bool shared = sy && !hold && lvl == lim - 1;
    u64 c = 0;
    if (shared) {
      if (!take_lim(t, g, st)) return;
      c = lvl_count(st, lim);
    }
    resolve<T, P>(t, g, st, cur, lvl);
    if (shared && !st->err) give_lim(t, g, st, c);
  }

  PBH_INL bool take_lim(const T& t, const Geom& g, typename P::SP st) {
    if (!sy->wait_idle(t, lim)) {
      fail(t, st);
      return false;
    }
    for (int tries = 0;; ++tries) {
      sy->get(t, st, lim);
      const u64 below = lim + 1 < g.q ? sy->deeper(t, lim + 1) : 0ull;
      if (t.tid() == 0) {
        st->deep_floor = below ? lim + 1 : -1;
        fix_ell(st, g.q);
      }
      t.sync();
      if (room_below(g, st, lim - 1)) return true;
      if (tries > 2 * MAXL) {
        sy->fail(t, E_INTERNAL);
        fail(t, st);
        return false;
      }
      sy->post(t, lim);
      if (!sy->wait_idle(t, lim)) {
        fail(t, st);
        return false;
      }
    }
  }

  // After Resolve(lim - 1): level lim (which held c elements) goes back to
  // its worker; the front keeps only the count of the worker levels.
  PBH_INL void give_lim(const T& t, const Geom& g, typename P::SP st, u64 c) {
    const u64 nc = lvl_count(st, lim);
    sy->put(t, st, lim);
    const u64 dn = sy->front_account(t, lim, (long long)nc - (long long)c);
    if (t.tid() == 0) {
      st->L[lim].nB = st->L[lim].nS = 0;
      st->deep_n = dn;
      st->deep_floor = dn ? lim : -1;
      fix_ell(st, g.q);
    }
    t.sync();
  }

  PBH_INL void fail(const T& t, typename P::SP st) {
    t.sync();
    if (t.tid() == 0 && st->err == 0) st->err = sy->error(t);
    t.sync();
  }

  // Every worker idle; the front takes every level's real state.
  PBH_INL bool hold_all(const T& t, const Geom& g, typename P::SP st) {
    for (int j = lim; j < g.q; ++j)
      if (!sy->wait_idle(t, j)) return false;
    for (int j = lim; j < g.q; ++j) sy->get(t, st, j);
    if (t.tid() == 0) {
      st->deep_floor = -1;
      st->deep_n = 0;
      fix_ell(st, g.q);
    }
    t.sync();
    hold = true;
    return true;
  }

  PBH_INL void release_all(const T& t, const Geom& g, typename P::SP st) {
    u64 tot = 0;
    for (int j = g.q - 1; j >= lim; --j) {
      tot += lvl_count(st, j);
      sy->put(t, st, j);
      sy->set_deeper(t, j, tot);
    }
    sy->publish(t);
    if (t.tid() == 0) {
      for (int j = lim; j < g.q; ++j) st->L[j].nB = st->L[j].nS = 0;
      st->deep_n = tot;
      st->deep_floor = tot ? lim : -1;
      fix_ell(st, g.q);
    }
    t.sync();
    hold = false;
  }

  // Resolve(0) and the schedule after an operation (and the refill of B_0).
  // A refill that needs the worker levels makes a second pass with every
  // level held (all workers idle): the one-team refill of drive_with.
  PBH_INL void drive(const T& t, const Geom& g, typename P::SP st, const u64* cur, int sched, int what) {
    if constexpr (!SY::kOn) {
      drive_with(t, g, st, sched, what, [&](int lvl) { resolve<T, P>(t, g, st, cur, lvl); });
    } else {
      int w = what;
      for (int pass = 0; pass < 2; ++pass) {
        bool refill = false;
        drive_with(
            t, g, st, sched, w, [&](int lvl) { res(t, g, st, cur, lvl); }, (sy && !hold) ? lim : MAXL,
            [&](int lvl) { sy->post(t, lvl); }, [&] { refill = true; });
        if (!refill || st->err) break;
        if (!hold_all(t, g, st)) {
          fail(t, st);
          break;
        }
        w = DRIVE_ENSURE;
      }
      if (hold) {
        if (!st->err) release_all(t, g, st);
        hold = false;
      }
    }
  }

  // Every 1024 rounds the front shows it is alive, so that a worker whose
  // level gets no request for a long time can tell that from a stopped front.
  PBH_INL void tick(const T& t, u64 rounds) {
    if constexpr (SY::kOn) {
      if (sy && (rounds & 1023u) == 0) sy->beat(t, (u32)rounds);
    }
  }

  // End of the run: every worker idle, their levels' Resolve counts and
  // element traffic merged into st, then the workers leave.
  PBH_INL void finish(const T& t, const Geom& g, typename P::SP st) {
    if constexpr (SY::kOn) {
      if (!sy) return;
      if (!st->err) {
        if (hold_all(t, g, st)) {
          sy->merge_stats(t, st, lim, g.q);
        } else {
          fail(t, st);
        }
      }
      sy->leave(t);
    }
  }
};

// No workers (every level is the front's).
struct NoDeepSync {
  static constexpr bool kOn = false;
};

// ---------------------------------------------------------------- parDijkstra

PBH_HD inline int bits_for(u32 n) {
  int b = 0;
  while (b < 32 && ((u64)1 << b) < (u64)n) ++b;
  return b < 1 ? 1 : b;
}

// U (relaxation output, n pairs in S) -> sorted by id with one pair per id.
// With rows sorted by target the pairs already are strictly increasing in id
// and nothing is done.  Otherwise each id keeps the pair whose key equals
// dist[id] (the minimum, since dist was lowered by atomicMin) and the rest is
// sorted by id.
template <class T, class A>
PBH_INL u32 intake(const T& t, A S, u32 n, A tmp, A tmp2, const u64* dist, int idbits) {
  u32 bad = 0;
  for (u32 x = (u32)t.tid() + 1; x < n; x += (u32)T::kNT) bad += S.v[x - 1] >= S.v[x];
  bad = t.sum(bad);
  if (bad == 0) return n;
  u32 out = 0;
  for (u32 base = 0; base < n; base += (u32)T::kNT) {
    u32 x = base + (u32)t.tid();
    bool keep = x < n && t.load_cur(dist + S.v[x]) == S.k[x];
    u64 k = x < n ? S.k[x] : 0;
    u32 v = x < n ? S.v[x] : 0;
    u32 tot;
    u32 o = out + t.scan_excl(keep ? 1u : 0u, &tot);
    if (keep) {
      tmp.k[o] = k;
      tmp.v[o] = v;
    }
    out += tot;
  }
  t.sync();
  bool in2 = sort_by_id(t, tmp, tmp2, out, idbits);
  if (in2)
    copy_arr(t, tmp2, S, out);
  else
    copy_arr(t, tmp, S, out);
  return out;
}

// One parDijkstra round (Section 4.1) with level 0 of type A0: extract the
// minimum (key, id) of B_0 -- B_0 holds only live elements, so this is the
// closest unsettled vertex u -- relax all out-edges of u in parallel
// (atomicMin on dist) and compact the improved (dist, v) pairs with a prefix
// sum straight into S_0 (a BulkUpdate of at most d = max out-degree pairs).
// Returns false when the heap is empty.
// LONG: the forms for long rows and a large B_0 in HBM (the plain-rule-only
// kernel, whose registers have room for them; in the kernel that also runs
// speculative rounds they would change the register allocation of those).
template <class T, class P, class A0, bool LONG = false>
PBH_INL bool round_body(const T& t, const Geom& g, typename P::SP st, const u64* off, const u32* tg,
                        const u32* wt, u64* dist, int idbits, u64* relax, u64* upd, u32* order, u64 order_cap,
                        u64 nth) {
  const Lvl a0 = lvl_load(st, 0);
  if (a0.nB == 0) return false;
  A0 B = as_arr<A0>(lbuf(g, 0, a0.bsel));
  u64 mk = KINF;
  u32 mv = VINF;
  if constexpr (!LONG || in_lds<A0>::v) {
    for (u32 x = (u32)t.tid(); x < a0.nB; x += (u32)T::kNT) {
      u64 k = B.k[x];
      u32 v = B.v[x];
      if (k < mk || (k == mk && v < mv)) {
        mk = k;
        mv = v;
      }
    }
  } else {
    // B_0 in HBM (large d): eight loads per thread in flight per pass
    constexpr int U = 8;
    for (u32 base = 0; base < a0.nB; base += (u32)T::kNT * U) {
      u64 k[U];
      u32 v[U];
#pragma unroll
      for (int r = 0; r < U; ++r) {
        const u32 x = base + (u32)r * (u32)T::kNT + (u32)t.tid();
        k[r] = x < a0.nB ? B.k[x] : KINF;
        v[r] = x < a0.nB ? B.v[x] : VINF;
      }
#pragma unroll
      for (int r = 0; r < U; ++r)
        if (k[r] < mk || (k[r] == mk && v[r] < mv)) {
          mk = k[r];
          mv = v[r];
        }
    }
  }
  t.minkv(mk, mv);
  const u64 e0 = off[mv], e1 = off[mv + 1];
  if (order && nth < order_cap && t.tid() == 0) order[nth] = mv;  // the settle order, when asked for
  u32 n0, n1, n2;
  A0 T0 = as_arr<A0>(lbuf(g, 0, 2));
  partition3(t, B, a0.nB, KV{mk, mv}, kv_inf(), T0, as_arr<A0>(lbuf(g, 0, a0.bsel ^ 1)), T0, &n0, &n1, &n2);
  prof_lap(t, st, PROF_EXTRACT);
  A0 S = as_arr<A0>(lbuf(g, 0, 3));
  u32 nu = 0;
  u64 eb = e0;
  // Long rows: four edges per thread per pass, their loads and atomics in
  // flight together (the scans place the improvements in edge order, edge
  // eb + r * NT + tid before those of r + 1).
  constexpr int RE = 4;
  for (; LONG && e1 - eb >= (u64)T::kNT * RE; eb += (u64)T::kNT * RE) {
    u64 cand[RE];
    u32 v[RE];
    bool imp[RE];
#pragma unroll
    for (int r = 0; r < RE; ++r) {
      const u64 e = eb + (u64)r * T::kNT + (u64)t.tid();
      v[r] = tg[e];
      cand[r] = mk + (u64)wt[e];
    }
#pragma unroll
    for (int r = 0; r < RE; ++r) imp[r] = cand[r] < t.atomic_min(dist + v[r], cand[r]);
#pragma unroll
    for (int r = 0; r < RE; ++r) {
      u32 tot;
      const u32 p = t.scan_excl(imp[r] ? 1u : 0u, &tot);
      if (imp[r]) {
        S.k[nu + p] = cand[r];
        S.v[nu + p] = v[r];
      }
      nu += tot;
    }
  }
  for (; eb < e1; eb += (u64)T::kNT) {
    u64 e = eb + (u64)t.tid();
    bool imp = false;
    u64 cand = 0;
    u32 v = 0;
    if (e < e1) {
      v = tg[e];
      cand = mk + (u64)wt[e];
      imp = cand < t.atomic_min(dist + v, cand);
    }
    u32 tot;
    u32 p = t.scan_excl(imp ? 1u : 0u, &tot);
    if (imp) {
      S.k[nu + p] = cand;
      S.v[nu + p] = v;
    }
    nu += tot;
  }
  t.sync();
  prof_lap(t, st, PROF_RELAX);
  nu = intake(t, S, nu, T0, as_arr<A0>(lbuf(g, 0, 4)), dist, idbits);
  if (t.tid() == 0) {
    st->L[0].bsel = a0.bsel ^ 1;
    st->L[0].nB = n1;
    st->L[0].nS = nu;
    st->L[0].ssel = 0;
    st->elems += 3ull * a0.nB + nu;
    if (st->ell < 0 && (n1 + nu) > 0) st->ell = 0;
  }
  t.sync();
  prof_lap(t, st, PROF_INTAKE);
  *relax += e1 - e0;
  *upd += nu;
  return true;
}

// ------------------------------------------------------------ speculative rounds
// A round may extract the k >= 1 smallest live elements of B_0 instead of one
// (the plain rule of Section 4.1 is k = 1).  All out-edges of the k vertices
// are relaxed; any vertex whose distance later improves is re-inserted into the
// heap and relaxed again, so the distances are exact for every choice of k.
// The k of each round comes from a rule: plain, fixed, a given sequence, or a
// small learned model (see mlp_forward).

constexpr int KMAX_ROUND = 256;  // cap on k per round (extracted vertices kept in LDS)
constexpr int TRACE_K = 32;      // key-ordered prefix of B_0 recorded per traced round
constexpr int NFEAT = 8;
constexpr int MLP_H = 64;
// MLP parameters (float32, weights already rounded to bfloat16), in order:
// W1[NFEAT][MLP_H] (input-major), b1[MLP_H], W2[MLP_H][MLP_H] (input-major),
// b2[MLP_H], w3[MLP_H], b3, then the feature normalisation mu[NFEAT],
// sd[NFEAT] and the output scale s (k = 2^(s * y)).
constexpr int MLP_PARAMS = NFEAT * MLP_H + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1;
constexpr int MLP_BLOB = MLP_PARAMS + 2 * NFEAT + 1;

struct SpecCfg {
  int rule;           // 0 plain, 1 fixed, 2 learned, 3 sequence
  u32 kfix, kmax;
  const u32* kseq;
  u32 kseq_len;
  const float* model;  // MLP_BLOB floats (learned rule)
  u64* uk;             // round update list (capacity kmax * d) and a temporary of the same size
  u32* uv;
  u64* tk;
  u32* tv;
  // training traces: every trace_every-th round records NFEAT features and the
  // TRACE_K smallest (key, id) of B_0 in key order
  float* trace_f;
  u64* trace_k;
  u32* trace_v;
  u32 trace_every, trace_cap;
  u32* trace_count;
  u32* trace_q;  // query index of each record
  u32 qid;
  // trial limits: no round starts once the heap's smallest key exceeds
  // stop_key (0 = none) or after max_rounds rounds (0 = none)
  u64 stop_key;
  u32 max_rounds;
  float kscale;  // learned rule: multiplies log2 k
  u32 kevery;    // learned rule: the model runs every kevery-th round (>= 1)
  // LDS room for the round's list after the LDS levels: two buffers of lcap
  // pairs (keys, then ids); 0 = the intake sorts in global memory
  u32 lcap;
  // extracted ids in extraction order (order[j] = the j-th extraction; a
  // round of k > 1 writes its k in id order), first order_cap of them
  u32* order;
  u64 order_cap;
};

struct SsspCounters {
  u64 rounds, relax, updates, extracted;
  u64 last_key;  // smallest key left in the heap when the rounds stopped (KINF: ran empty)
  u32 stopped;   // a trial limit ended the rounds
};

// Smallest key of B_0 (the heap's minimum once B_0 has been refilled).
template <class T, class P>
PBH_INL u64 b0_min_key(const T& t, const Geom& g, typename P::SP st) {
  const Lvl a0 = lvl_load(st, 0);
  Arr Bg = lbuf(g, 0, a0.bsel);
  u64 lo = KINF, hi = 0;
  if (g.qlds > 0) {
    typename P::L B = as_arr<typename P::L>(Bg);
    for (u32 x = (u32)t.tid(); x < a0.nB; x += (u32)T::kNT) lo = B.k[x] < lo ? B.k[x] : lo;
  } else {
    typename P::G B = as_arr<typename P::G>(Bg);
    for (u32 x = (u32)t.tid(); x < a0.nB; x += (u32)T::kNT) lo = B.k[x] < lo ? B.k[x] : lo;
  }
  t.minmax64(lo, hi);
  return lo;
}

struct RoundMemo {  // team-uniform facts about the previous round
  float avgdeg;
  u32 k;  // the last k the learned rule proposed
};

PBH_INL float flog2p1(float x) { return __builtin_log2f(1.0f + x); }

// The 8 model features, identical in plain and speculative runs: heap size,
// |B_0|, key spread of B_0, the pivots p_0 and p_1 relative to the minimum
// key (a quantile sketch of the queue: the level boundaries), the minimum key
// itself, the mean out-degree of the previous round's vertices, and d.
template <class T, class SP, class A0>
PBH_INL void round_features(const T& t, const Geom& g, SP st, A0 B, u32 nB, const RoundMemo& memo, float* f) {
  u64 lo = KINF, hi = 0;
  for (u32 x = (u32)t.tid(); x < nB; x += (u32)T::kNT) {
    u64 k = B.k[x];
    lo = k < lo ? k : lo;
    hi = k > hi ? k : hi;
  }
  t.minmax64(lo, hi);
  u64 tot = st->deep_n;
  for (int i = 0; i < g.q; ++i) tot += (u64)st->L[i].nB + st->L[i].nS;
  const float spread = (float)(hi - lo);
  f[0] = flog2p1((float)tot);
  f[1] = flog2p1((float)nB);
  f[2] = flog2p1(spread);
  const u64 p0 = st->L[0].pk, p1 = st->L[1].pk;
  f[3] = p0 == KINF ? f[2] + 1.0f : flog2p1((float)(p0 - lo));
  f[4] = (g.q < 2 || p1 == KINF) ? f[3] + 1.0f : flog2p1((float)(p1 - lo));
  f[5] = flog2p1((float)lo) * 0.125f;
  f[6] = flog2p1(memo.avgdeg);
  f[7] = flog2p1((float)g.d);
}

// Rounds a float to bfloat16 (round to nearest even) and back: the model's
// weights are used at BF16 precision with FP32 accumulation.
PBH_INL float bf16r(float x) {
  u32 u = __builtin_bit_cast(u32, x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __builtin_bit_cast(float, u & 0xFFFF0000u);
}

PBH_INL float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }

// MLP 8 -> 64 -> 64 -> 1 with GELU (exact, x * Phi(x)); every parameter is
// used rounded to bfloat16, as in training; thread j computes hidden unit j of
// each layer (weights stored input-major, so the loads of
// one input row are contiguous), the output is reduced through LDS.  BF16
// weights, FP32 accumulation.  Returns y (k = 2^(s * y)).
template <class T>
PBH_INL float mlp_forward(const T& t, const float* m, const float* f) {
  const float* W1 = m;
  const float* b1 = W1 + NFEAT * MLP_H;
  const float* W2 = b1 + MLP_H;
  const float* b2 = W2 + MLP_H * MLP_H;
  const float* w3 = b2 + MLP_H;
  const float* b3 = w3 + MLP_H;
  const float* mu = b3 + 1;
  const float* sd = mu + NFEAT;
  float x[NFEAT];
#pragma unroll
  for (int i = 0; i < NFEAT; ++i) x[i] = (f[i] - mu[i]) / sd[i];
  for (int j = t.tid(); j < MLP_H; j += T::kNT) {
    float a = bf16r(b1[j]);
#pragma unroll
    for (int i = 0; i < NFEAT; ++i) a += bf16r(W1[i * MLP_H + j]) * x[i];
    t.sh->mlp_h[j] = gelu(a);
  }
  t.sync();
  if constexpr (T::kNT >= 256) {
    // four threads per hidden unit, each summing a quarter of the inputs
    const int j = t.tid() & (MLP_H - 1), qtr = t.tid() >> 6;
    if (t.tid() < 4 * MLP_H) {
      float a = 0.0f;
      for (int i = qtr * (MLP_H / 4); i < (qtr + 1) * (MLP_H / 4); ++i) a += bf16r(W2[i * MLP_H + j]) * t.sh->mlp_h[i];
      t.sh->mlp_p[t.tid()] = a;
    }
    t.sync();
    if (t.tid() < MLP_H) {
      float a = bf16r(b2[j]);
      for (int q = 0; q < 4; ++q) a += t.sh->mlp_p[q * MLP_H + j];
      t.sh->mlp_z[j] = bf16r(w3[j]) * gelu(a);
    }
  } else {
    for (int j = t.tid(); j < MLP_H; j += T::kNT) {
      float a = bf16r(b2[j]);
      for (int i = 0; i < MLP_H; ++i) a += bf16r(W2[i * MLP_H + j]) * t.sh->mlp_h[i];
      t.sh->mlp_z[j] = bf16r(w3[j]) * gelu(a);
    }
  }
  t.sync();
  float y = bf16r(b3[0]);
  if constexpr (T::kNT >= 64) {
    // every wavefront sums the 64 output terms with a butterfly of lane
    // exchanges (the same order in every lane), instead of each thread
    // reading all 64 from LDS one after another
    static_assert(MLP_H == 64, "one output term per lane");
    float z = t.sh->mlp_z[t.lane()];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) z += __shfl_xor(z, o, 64);
    y += z;
  } else {
    for (int j = 0; j < MLP_H; ++j) y += t.sh->mlp_z[j];
  }
  t.sync();
  return y * sd[NFEAT];
}

template <class T, class SP, class A0>
PBH_INL u32 propose_k(const T& t, const Geom& g, SP st, const SpecCfg& sc, A0 B, u32 nB, u64 round,
                      RoundMemo& memo) {
  u32 k = 1;
  if (sc.rule == 1) {
    k = sc.kfix;
  } else if (sc.rule == 3) {
    k = sc.kseq[round % sc.kseq_len];
  } else if (sc.rule == 2 && sc.kevery > 1 && round % sc.kevery != 0) {
    k = memo.k;  // between model runs the last proposal stands
  } else if (sc.rule == 2) {
    float f[NFEAT];
    round_features(t, g, st, B, nB, memo, f);
    float y = mlp_forward(t, sc.model, f) * sc.kscale;
    // fall back to the plain rule on anything that is not a finite number
    if (y == y && y > -64.0f && y < 64.0f) {
      float kk = __builtin_exp2f(y);
      k = kk < 1.0f ? 1u : (kk > (float)sc.kmax ? sc.kmax : (u32)(kk + 0.5f));
    }
  }
  k = k < 1 ? 1 : k;
  k = k > sc.kmax ? sc.kmax : k;
  k = k > (u32)KMAX_ROUND ? (u32)KMAX_ROUND : k;
  memo.k = k;
  return k;
}

// Records one training trace: features and the TRACE_K smallest (key, id) of
// B_0 in key order (by repeated team minima; traced rounds are sparse).
template <class T, class SP, class A0>
PBH_INL void record_trace(const T& t, const Geom& g, SP st, const SpecCfg& sc, A0 B, u32 nB,
                          const RoundMemo& memo) {
  float f[NFEAT];
  round_features(t, g, st, B, nB, memo, f);
  u32 slot = 0;
  if (t.tid() == 0) slot = t.atomic_add32(sc.trace_count, 1u);
  slot = t.sum(slot);
  if (slot >= sc.trace_cap) return;
  if (t.tid() == 0) {
    for (int i = 0; i < NFEAT; ++i) sc.trace_f[(u64)slot * NFEAT + i] = f[i];
    if (sc.trace_q) sc.trace_q[slot] = sc.qid;
  }
  u64 lastk = 0;
  u32 lastv = 0;
  bool have = false;
  for (int r = 0; r < TRACE_K; ++r) {
    u64 bk = KINF;
    u32 bv = VINF;
    for (u32 x = (u32)t.tid(); x < nB; x += (u32)T::kNT) {
      u64 k = B.k[x];
      u32 v = B.v[x];
      bool after = !have || k > lastk || (k == lastk && v > lastv);
      if (after && (k < bk || (k == bk && v < bv))) {
        bk = k;
        bv = v;
      }
    }
    t.minkv(bk, bv);
    if (t.tid() == 0) {
      sc.trace_k[(u64)slot * TRACE_K + r] = bk;
      sc.trace_v[(u64)slot * TRACE_K + r] = bv;
    }
    lastk = bk;
    lastv = bv;
    have = true;
  }
  t.sync();
}

// Round update list U (n pairs, global) -> one pair per id, sorted by id: keep
// the pairs whose key equals dist[id] (the minimum, by atomicMin), sort by id,
// drop equal neighbours (equal candidates from two sources).
template <class T, class GA>
PBH_INL u32 intake_list(const T& t, GA U, u32 n, GA W, const u64* dist, int idbits) {
  u32 out = 0;
  constexpr int RE = 4;  // elements per thread per pass, loads issued together
  for (u32 base = 0; base < n; base += (u32)T::kNT * RE) {
    u64 k[RE], c[RE];
    u32 v[RE];
#pragma unroll
    for (int r = 0; r < RE; ++r) {
      const u32 x = base + (u32)r * (u32)T::kNT + (u32)t.tid();
      k[r] = x < n ? U.k[x] : 0;
      v[r] = x < n ? U.v[x] : 0;
    }
#pragma unroll
    for (int r = 0; r < RE; ++r) {
      const u32 x = base + (u32)r * (u32)T::kNT + (u32)t.tid();
      c[r] = x < n ? t.load_cur(dist + v[r]) : ~k[r];
    }
    u32 cnt = 0;
#pragma unroll
    for (int r = 0; r < RE; ++r) cnt += c[r] == k[r] ? 1u : 0u;
    u32 tot;
    u32 o = out + t.scan_excl(cnt, &tot);
#pragma unroll
    for (int r = 0; r < RE; ++r)
      if (c[r] == k[r]) {
        W.k[o] = k[r];
        W.v[o] = v[r];
        ++o;
      }
    out += tot;
  }
  t.sync();
  bool inU = sort_by_id(t, W, U, out, idbits);
  GA S = inU ? U : W, D = inU ? W : U;
  u32 m = 0;
  for (u32 base = 0; base < out; base += (u32)T::kNT) {
    u32 x = base + (u32)t.tid();
    bool keep = x < out && (x == 0 || S.v[x - 1] != S.v[x]);
    u64 k = x < out ? S.k[x] : 0;
    u32 v = x < out ? S.v[x] : 0;
    u32 tot;
    u32 o = m + t.scan_excl(keep ? 1u : 0u, &tot);
    if (keep) {
      D.k[o] = k;
      D.v[o] = v;
    }
    m += tot;
  }
  t.sync();
  if (!inU) copy_arr(t, D, U, m);  // result always in U
  return m;
}

// intake_list with the filtered pairs sorted in LDS (two buffers L1, L2 of at
// least n pairs): the filter reads U and dist, the radix sort by id runs
// between L1 and L2, and the deduplicated list is written back to U.
template <class T, class GA, class LA>
PBH_INL u32 intake_list_lds(const T& t, GA U, u32 n, LA L1, LA L2, const u64* dist, int idbits) {
  u32 out = 0;
  constexpr int RE = 4;
  for (u32 base = 0; base < n; base += (u32)T::kNT * RE) {
    u64 k[RE], c[RE];
    u32 v[RE];
#pragma unroll
    for (int r = 0; r < RE; ++r) {
      const u32 x = base + (u32)r * (u32)T::kNT + (u32)t.tid();
      k[r] = x < n ? U.k[x] : 0;
      v[r] = x < n ? U.v[x] : 0;
    }
#pragma unroll
    for (int r = 0; r < RE; ++r) {
      const u32 x = base + (u32)r * (u32)T::kNT + (u32)t.tid();
      c[r] = x < n ? t.load_cur(dist + v[r]) : ~k[r];
    }
    u32 cnt = 0;
#pragma unroll
    for (int r = 0; r < RE; ++r) cnt += c[r] == k[r] ? 1u : 0u;
    u32 tot;
    u32 o = out + t.scan_excl(cnt, &tot);
#pragma unroll
    for (int r = 0; r < RE; ++r)
      if (c[r] == k[r]) {
        L1.k[o] = k[r];
        L1.v[o] = v[r];
        ++o;
      }
    out += tot;
  }
  t.sync();
  const bool in2 = sort_by_id(t, L1, L2, out, idbits);
  LA S = in2 ? L2 : L1;
  u32 m = 0;
  for (u32 base = 0; base < out; base += (u32)T::kNT) {
    u32 x = base + (u32)t.tid();
    bool keep = x < out && (x == 0 || S.v[x - 1] != S.v[x]);
    u64 k = x < out ? S.k[x] : 0;
    u32 v = x < out ? S.v[x] : 0;
    u32 tot;
    u32 o = m + t.scan_excl(keep ? 1u : 0u, &tot);
    if (keep) {
      U.k[o] = k;
      U.v[o] = v;
    }
    m += tot;
  }
  t.sync();
  return m;
}

// One speculative round: extract the `k` smallest of B_0, relax every out-edge
// of them, collect the improved (dist, v) pairs in the global list U.
template <class T, class P, class A0>
PBH_INL bool round_spec(const T& t, const Geom& g, typename P::SP st, const u64* off, const u32* tg,
                        const u32* wt, u64* dist, int idbits, u32 k, const SpecCfg& sc, SsspCounters* c,
                        RoundMemo* memo, u32* ulen) {
  using G = typename P::G;
  const Lvl a0 = lvl_load(st, 0);
  if (a0.nB == 0) return false;
  A0 B = as_arr<A0>(lbuf(g, 0, a0.bsel));
  const u32 take = k < a0.nB ? k : a0.nB;
  KV thr = take == a0.nB ? kv_inf() : select_kth(t, B, a0.nB, take);
  u32 n0, n1, n2;
  A0 X = as_arr<A0>(lbuf(g, 0, 2));
  partition3(t, B, a0.nB, thr, kv_inf(), X, as_arr<A0>(lbuf(g, 0, a0.bsel ^ 1)), X, &n0, &n1, &n2);
  if (sc.order)
    for (u32 j = (u32)t.tid(); j < take; j += (u32)T::kNT)
      if (c->extracted + j < sc.order_cap) sc.order[c->extracted + j] = X.v[j];
  prof_lap(t, st, PROF_EXTRACT);
  // out-degree prefix sums of the extracted vertices
  u32 E = 0;
  for (u32 base = 0; base < take; base += (u32)T::kNT) {
    u32 j = base + (u32)t.tid();
    u64 e0 = 0, e1 = 0;
    if (j < take) {
      u32 v = X.v[j];
      e0 = off[v];
      e1 = off[v + 1];
      t.sh->ex0[j] = e0;
    }
    u32 tot;
    u32 p = E + t.scan_excl((u32)(e1 - e0), &tot);
    if (j < take) t.sh->exd[j] = p;
    E += tot;
  }
  if (t.tid() == 0) t.sh->exd[take] = E;
  t.sync();
  G U{(decltype(G::k))sc.uk, (decltype(G::v))sc.uv};
  u32 nu = 0;
  // RE edges per thread per pass: their CSR loads and atomics are all in
  // flight before any result is waited for; one scan places the improvements.
  constexpr int RE = 8;
  for (u32 eb = 0; eb < E; eb += (u32)T::kNT * RE) {
    u64 ei[RE], cand[RE];
    u32 v[RE];
    bool imp[RE];
#pragma unroll
    for (int r = 0; r < RE; ++r) {
      const u32 e = eb + (u32)r * (u32)T::kNT + (u32)t.tid();
      ei[r] = 0;
      cand[r] = 0;
      if (e < E) {
        u32 lo = 0, hi = take;  // largest j with exd[j] <= e
        while (hi - lo > 1) {
          u32 mid = (lo + hi) >> 1;
          if (t.sh->exd[mid] <= e)
            lo = mid;
          else
            hi = mid;
        }
        ei[r] = t.sh->ex0[lo] + (e - t.sh->exd[lo]);
        cand[r] = X.k[lo];
      }
    }
#pragma unroll
    for (int r = 0; r < RE; ++r) {
      const bool in = eb + (u32)r * (u32)T::kNT + (u32)t.tid() < E;
      v[r] = in ? tg[ei[r]] : 0u;
      cand[r] += in ? (u64)wt[ei[r]] : 0ull;
    }
    u32 cnt = 0;
#pragma unroll
    for (int r = 0; r < RE; ++r) {
      const bool in = eb + (u32)r * (u32)T::kNT + (u32)t.tid() < E;
      imp[r] = in && cand[r] < t.atomic_min(dist + v[r], cand[r]);
      cnt += imp[r] ? 1u : 0u;
    }
    u32 tot;
    u32 p = nu + t.scan_excl(cnt, &tot);
#pragma unroll
    for (int r = 0; r < RE; ++r)
      if (imp[r]) {
        U.k[p] = cand[r];
        U.v[p] = v[r];
        ++p;
      }
    nu += tot;
  }
  t.sync();
  prof_lap(t, st, PROF_RELAX);
  if (sc.lcap != 0 && nu <= sc.lcap) {
    // the list fits in the LDS after the levels: sort it there
    using L = typename P::L;
    unsigned char* lb = reinterpret_cast<unsigned char*>(g.lk) + lvl_off(g.d, g.qlds) * 12ull;
    L L1, L2;
    L1.k = (decltype(L1.k))reinterpret_cast<u64*>(lb);
    L2.k = (decltype(L2.k))reinterpret_cast<u64*>(lb + (u64)sc.lcap * 8u);
    L1.v = (decltype(L1.v))reinterpret_cast<u32*>(lb + (u64)sc.lcap * 16u);
    L2.v = (decltype(L2.v))reinterpret_cast<u32*>(lb + (u64)sc.lcap * 20u);
    nu = intake_list_lds(t, U, nu, L1, L2, dist, idbits);
  } else {
    G Wt{(decltype(G::k))sc.tk, (decltype(G::v))sc.tv};
    nu = intake_list(t, U, nu, Wt, dist, idbits);
  }
  if (t.tid() == 0) {
    st->L[0].bsel = a0.bsel ^ 1;
    st->L[0].nB = n1;
    st->elems += 3ull * a0.nB + 3ull * nu;
    if (st->ell < 0 && n1 > 0) st->ell = 0;
  }
  t.sync();
  prof_lap(t, st, PROF_INTAKE);
  c->relax += E;
  c->updates += nu;
  c->extracted += take;
  memo->avgdeg = (float)E / (float)take;
  *ulen = nu;
  return true;
}

// parDijkstra: rounds until the heap is empty.  The extraction and the bulk
// update of a round share one Resolve(0) and the schedule: between them S_0 is
// empty and B_0 keeps at least d elements, so Algorithm 1's preconditions hold.
// Speculative rounds bulk-update their list U in pieces of at most d, each
// piece an operation followed by Resolve(0) and the schedule.
struct NoHook {
  template <class SP>
  PBH_INL void operator()(const Geom&, SP, const SsspCounters&) const {}
};

// `hook` sees the heap after every operation's Resolve schedule (the CPU
// tests use it to check invariants; the kernels pass NoHook).
// With `sy` (and lim < q), levels >= lim are resolved by their own workers
// (the deep-level service above).
// SPEC false: the plain rule only (one extraction per round, no traces) --
// the speculative rounds, the model and the update pieces are left out of
// the code, which lightens the kernel of plain runs.
template <class T, class P, class Hook = NoHook, class SY = NoDeepSync, bool SPEC = true>
PBH_INL void sssp_rounds(const T& t, const Geom& g, typename P::SP st, const u64* off, const u32* tg,
                         const u32* wt, u64* dist, u32 n, u32 src, int sched, const SpecCfg& sc, SsspCounters* cnt,
                         const Hook& hook = Hook(), SY* sy = nullptr, int lim = MAXL) {
  using G = typename P::G;
  DeepFront<T, P, SY> fr{sy, lim, false};
  const int idbits = bits_for(n);
  if (t.tid() == 0) {
    Arr S = lbuf(g, 0, 3);
    if (g.qlds > 0) {
      typename P::L s = as_arr<typename P::L>(S);
      s.k[0] = 0;
      s.v[0] = src;
    } else {
      typename P::G s = as_arr<typename P::G>(S);
      s.k[0] = 0;
      s.v[0] = src;
    }
    st->L[0].nS = 1;
    st->L[0].ssel = 0;
    st->ell = 0;
    st->prof_last = pbh_clock();
  }
  t.sync();
  SsspCounters c{0, 0, 1, 0, KINF, 0};
  RoundMemo memo{0.0f, 1u};
  u32 upos = 0, ulen = 0;
  for (;;) {
    // Resolve(0) and the schedule after the previous operation (the source's
    // insertion, a round's bulk update or a piece of it), then make sure B_0
    // holds the minimum if the heap is not empty.
    fr.drive(t, g, st, dist, sched, DRIVE_AFTER | DRIVE_ENSURE);
    prof_lap(t, st, PROF_DRIVE);
    if (st->err) break;
    hook(g, st, c);
    if (SPEC && upos < ulen) {  // next piece of the round's bulk update
      u32 len = ulen - upos < g.d ? ulen - upos : g.d;
      G U{(decltype(G::k))sc.uk, (decltype(G::v))sc.uv};
      if (g.qlds > 0) {
        typename P::L S = as_arr<typename P::L>(lbuf(g, 0, 3));
        for (u32 x = (u32)t.tid(); x < len; x += (u32)T::kNT) {
          S.k[x] = U.k[upos + x];
          S.v[x] = U.v[upos + x];
        }
      } else {
        G S = as_arr<G>(lbuf(g, 0, 3));
        for (u32 x = (u32)t.tid(); x < len; x += (u32)T::kNT) {
          S.k[x] = U.k[upos + x];
          S.v[x] = U.v[upos + x];
        }
      }
      t.sync();
      if (t.tid() == 0) {
        st->L[0].nS = len;
        st->L[0].ssel = 0;
        if (st->ell < 0) st->ell = 0;
      }
      t.sync();
      prof_lap(t, st, PROF_PIECE);
      upos += len;
      continue;
    }
    if (sc.max_rounds || sc.stop_key) {
      const u64 mn = b0_min_key<T, P>(t, g, st);
      if ((sc.max_rounds && c.rounds >= sc.max_rounds) || (sc.stop_key && mn != KINF && mn > sc.stop_key)) {
        c.last_key = mn;
        c.stopped = 1;
        break;
      }
    }
    // Every extraction consumes one insertion and every insertion comes from
    // one scanned edge (or the source), so rounds <= 1 + relax always holds.
    if (c.rounds > c.relax + 1) {
      if (t.tid() == 0) st->err = E_INTERNAL;
      t.sync();
      break;
    }
    prof_lap(t, st, PROF_OTHER);
    bool more;
    if (!SPEC || (sc.rule == 0 && !sc.trace_f)) {
      more = g.qlds > 0
                 ? round_body<T, P, typename P::L, !SPEC>(t, g, st, off, tg, wt, dist, idbits, &c.relax, &c.updates,
                                                          sc.order, sc.order_cap, c.extracted)
                 : round_body<T, P, typename P::G, !SPEC>(t, g, st, off, tg, wt, dist, idbits, &c.relax, &c.updates,
                                                          sc.order, sc.order_cap, c.extracted);
      c.extracted += more ? 1 : 0;
    } else if constexpr (SPEC) {
      const Lvl a0 = lvl_load(st, 0);
      Arr Bg = lbuf(g, 0, a0.bsel);
      u32 k;
      if (g.qlds > 0) {
        typename P::L B = as_arr<typename P::L>(Bg);
        if (sc.trace_f && a0.nB && c.rounds % sc.trace_every == 0) record_trace(t, g, st, sc, B, a0.nB, memo);
        k = propose_k(t, g, st, sc, B, a0.nB, c.rounds, memo);
        prof_lap(t, st, PROF_PROPOSE);
        more = round_spec<T, P, typename P::L>(t, g, st, off, tg, wt, dist, idbits, k, sc, &c, &memo, &ulen);
      } else {
        G B = as_arr<G>(Bg);
        if (sc.trace_f && a0.nB && c.rounds % sc.trace_every == 0) record_trace(t, g, st, sc, B, a0.nB, memo);
        k = propose_k(t, g, st, sc, B, a0.nB, c.rounds, memo);
        prof_lap(t, st, PROF_PROPOSE);
        more = round_spec<T, P, G>(t, g, st, off, tg, wt, dist, idbits, k, sc, &c, &memo, &ulen);
      }
      upos = 0;
    }
    fr.tick(t, c.rounds);
    if (!more) {
      // B_0 is empty only once the heap is (the refill above guarantees it).
      if (st->ell >= 0) {
        t.sync();
        if (t.tid() == 0) st->err = E_INTERNAL;
        t.sync();
      }
      break;
    }
    ++c.rounds;
  }
  fr.finish(t, g, st);
  *cnt = c;
}

// ---------------------------------------------------------------- pbh_* calls
struct PbhParams {
  Geom g;
  HeapState* gst;  // heap state in device memory, loaded into LDS per kernel
  u64* cur;        // current key of every id
  u32* bitmap;     // one bit per id, all zero between calls
  u32 nwords;
  u32 id_cap;
  int sched;
  int idbits;
  // bulk update
  const u64* keys;
  const u32* ids;
  u64 count;
  u64* ukeys;  // compacted update list
  u32* uids;
  // extract
  u64 k;
  u64* okeys;
  u32* oids;
};

// Could the next operation push elements out of the deepest allocated level?
// Then the caller adds a level first (growing the arena keeps the offsets of
// the existing levels).
template <class SP>
PBH_INL bool need_grow(const Geom& g, SP st) {
  const int q = g.q;
  u64 have = (u64)st->L[q - 1].nB + st->L[q - 1].nS;
  u64 in = (q == 1) ? (u64)g.d : capB(g.d, q - 2) + capS(g.d, q - 2);
  return have + in > nomB(g.d, q - 1);
}

// BulkUpdate of one call.  First pass: cur[id] = min(cur[id], key) with
// atomicMin (duplicates in the batch: the smallest key wins), ids whose key
// dropped are marked in a bitmap; compacting the bitmap gives the changed ids
// in increasing id order with their new keys, i.e. U sorted by value as
// Section 2.2 requires.  Then pieces of at most d go into S_0, each followed
// by Resolve(0) and the schedule.  Resumable: st->aux[0] = list length,
// aux[1] = list built, aux[3] = stopped because a level must be added,
// progress = list position reached.  All levels are in HBM (type P::G).
template <class T, class P>
PBH_INL void pbh_update_body(const T& t, const Geom& g, typename P::SP st, const PbhParams& p) {
  using G = typename P::G;
  if (st->aux[1] == 0) {
    u32 newly = 0;
    for (u64 x = (u64)t.tid(); x < p.count; x += (u64)T::kNT) {
      u32 id = p.ids[x];
      u64 k = p.keys[x];
      u64 old = t.atomic_min(p.cur + id, k);
      if (k < old) {
        t.atomic_or32(p.bitmap + (id >> 5), 1u << (id & 31));
        newly += (old == KINF);
      }
    }
    newly = t.sum(newly);
    t.fence();
    t.sync();
    u64 nu = 0;
    for (u32 wb = 0; wb < p.nwords; wb += (u32)T::kNT) {
      u32 w = wb + (u32)t.tid();
      u32 bits = 0;
      if (w < p.nwords) {
        bits = t.load32(p.bitmap + w);
        if (bits) p.bitmap[w] = 0u;
      }
      u32 tot;
      u64 o = nu + t.scan_excl((u32)__builtin_popcount(bits), &tot);
      while (bits) {
        u32 b = (u32)__builtin_ctz(bits);
        bits &= bits - 1;
        u32 id = w * 32u + b;
        p.uids[o] = id;
        p.ukeys[o] = t.load_cur(p.cur + id);
        ++o;
      }
      nu += tot;
    }
    t.sync();
    if (t.tid() == 0) {
      st->aux[0] = nu;
      st->aux[1] = 1;
      st->live += newly;
      st->progress = 0;
    }
    t.sync();
  }
  const u64 nu = st->aux[0];
  if (t.tid() == 0) st->aux[3] = 0;
  t.sync();
  for (u64 c0 = st->progress; c0 < nu;) {
    if (need_grow(g, st)) {
      if (t.tid() == 0) st->aux[3] = 1;
      t.sync();
      break;
    }
    u32 len = (u32)((nu - c0) < g.d ? (nu - c0) : g.d);
    G S = as_arr<G>(lbuf(g, 0, 3));
    for (u32 x = (u32)t.tid(); x < len; x += (u32)T::kNT) {
      S.k[x] = p.ukeys[c0 + x];
      S.v[x] = p.uids[c0 + x];
    }
    t.sync();
    if (t.tid() == 0) {
      st->L[0].nS = len;
      st->L[0].ssel = 0;
      if (st->ell < 0) st->ell = 0;
      st->elems += 2ull * len;
    }
    t.sync();
    drive<T, P>(t, g, st, p.cur, p.sched, DRIVE_AFTER);
    if (st->err) break;
    c0 += len;
    if (t.tid() == 0) st->progress = c0;
    t.sync();
  }
}

// Delete(e) of one call (Section 1.2) for a batch of ids (absent ids: no-op).
// The paper sends a DEL priority down the levels that removes the matching
// elements when they meet in a merge.  Here the id's current key is set to
// "absent" (KINF) instead: every merge and every move into B_0 already drops
// copies whose key is not the current one (the duplicate reading used for
// updates), so copies in deeper levels leave when they next meet a merge or
// move up.  B_0 must hold only live elements, so it is filtered at once; then
// Resolve(0) and the schedule run, as after any operation.  Resumable like
// the update: aux[1] = ids marked and B_0 filtered, aux[3] = stopped because a
// level must be added.
template <class T, class P>
PBH_INL void pbh_delete_body(const T& t, const Geom& g, typename P::SP st, const PbhParams& p) {
  using G = typename P::G;
  if (st->aux[1] == 0) {
    u32 gone = 0;
    for (u64 x = (u64)t.tid(); x < p.count; x += (u64)T::kNT)
      gone += t.atomic_exch(p.cur + p.ids[x], KINF) != KINF ? 1u : 0u;
    gone = t.sum(gone);
    t.fence();
    t.sync();
    const Lvl a0 = lvl_load(st, 0);
    u32 n0 = 0, n1 = 0, n2 = 0;
    if (a0.nB) {
      G B = as_arr<G>(lbuf(g, 0, a0.bsel)), O = as_arr<G>(lbuf(g, 0, a0.bsel ^ 1)), X = as_arr<G>(lbuf(g, 0, 2));
      partition3(t, B, a0.nB, kv_inf(), kv_inf(), O, X, X, &n0, &n1, &n2, p.cur);
    }
    if (t.tid() == 0) {
      if (a0.nB) {
        st->L[0].bsel = a0.bsel ^ 1;
        st->L[0].nB = n0;
        st->elems += (u64)a0.nB + n0;
      }
      st->live -= gone;
      st->aux[1] = 1;
      fix_ell(st, g.q);
    }
    t.sync();
  }
  if (t.tid() == 0) st->aux[3] = 0;
  t.sync();
  if (need_grow(g, st)) {
    if (t.tid() == 0) st->aux[3] = 1;
    t.sync();
    return;
  }
  drive<T, P>(t, g, st, p.cur, p.sched, DRIVE_AFTER);
}

// Batched ExtractMin of one call: repeatedly take the smallest min(k_left,
// |B_0|) elements of B_0 (B_0 <= p_0 < everything else, and B_0 holds only
// live elements), output them sorted by (key, id), mark their ids absent, then
// Resolve(0) and the schedule.  Resumable: progress = elements written,
// aux[2] = an extraction awaits its Resolve(0), aux[3] = stopped for growth,
// aux[4] = heap ran empty.
template <class T, class P>
PBH_INL void pbh_extract_body(const T& t, const Geom& g, typename P::SP st, const PbhParams& p) {
  using G = typename P::G;
  if (t.tid() == 0) {
    st->aux[3] = 0;
    st->aux[4] = 0;
  }
  t.sync();
  for (;;) {
    const bool pending = st->aux[2] != 0;  // the last extraction still needs its Resolve(0)
    const u64 outpos = st->progress;
    if (!pending && outpos >= p.k) break;
    if (need_grow(g, st)) {
      if (t.tid() == 0) st->aux[3] = 1;
      t.sync();
      break;
    }
    drive<T, P>(t, g, st, p.cur, p.sched, (pending ? DRIVE_AFTER : 0) | (outpos < p.k ? DRIVE_ENSURE : 0));
    if (t.tid() == 0) st->aux[2] = 0;
    t.sync();
    if (st->err || outpos >= p.k) break;
    const Lvl a0 = lvl_load(st, 0);
    if (a0.nB == 0) {
      t.sync();
      if (t.tid() == 0) {
        if (st->ell >= 0)
          st->err = E_INTERNAL;  // the refill leaves B_0 empty only when the heap is
        else
          st->aux[4] = 1;
      }
      t.sync();
      break;
    }
    u32 take = (u32)((p.k - outpos) < a0.nB ? (p.k - outpos) : a0.nB);
    G B = as_arr<G>(lbuf(g, 0, a0.bsel));
    KV thr = (take == a0.nB) ? kv_inf() : select_kth(t, B, a0.nB, take);
    u32 n0, n1, n2;
    G X = as_arr<G>(lbuf(g, 0, 2));
    partition3(t, B, a0.nB, thr, kv_inf(), X, as_arr<G>(lbuf(g, 0, a0.bsel ^ 1)), X, &n0, &n1, &n2);
    G R = sort_kv(t, X, B, take, p.idbits) ? B : X;
    for (u32 x = (u32)t.tid(); x < take; x += (u32)T::kNT) {
      u32 id = R.v[x];
      p.okeys[outpos + x] = R.k[x];
      p.oids[outpos + x] = id;
      t.store_cur(p.cur + id, KINF);
    }
    t.fence();
    t.sync();
    if (t.tid() == 0) {
      st->L[0].bsel ^= 1;
      st->L[0].nB = n1;
      st->live -= take;
      st->progress = outpos + take;
      st->elems += 6ull * a0.nB;
      st->aux[2] = 1;
    }
    t.sync();
  }
}

}  // namespace bkt
