// Device-wide engine of the parallel bucket heap (see wide.h).
//
// Kernels (256 threads per workgroup, tiles of 2048 elements):
//   k_merge<false> / k_scan / k_merge<true>
//       Merge of two id-sorted arrays with DeleteDuplicates (Section 2.1):
//       a counting pass (which also finds each tile's merge-path split
//       points), a scan of the tile counts, and a writing pass; in both passes
//       each thread walks 8 consecutive merge positions from one merge-path
//       search in LDS, and the writing pass stores its outputs through an
//       LDS transpose.  The counting pass can also count outputs <= a pivot
//       (the count in Resolve's EMPTY step) and the key range (the start of
//       Select), as per-workgroup partials folded by the scan, which then
//       publishes the step before the writing pass runs.
//   k_part<false> / k_scan (three arrays) / k_part<true>
//       Stable three-way split by two (key, id) pivots.
//   k_sel_pass / k_sel_collect
//       Select: radix selection on the 96-bit (key, id) value, 8 bits per
//       pass from the first bit where the keys differ, until at most 256
//       candidates remain; those are gathered and ranked.  The last
//       workgroup of a pass makes its pick, the last one of the gather ranks
//       the candidates; the split that follows reads the result on the
//       device, so Select and split are one host step.
//   k_intake / k_bits<false> / k_bits<true>
//       BulkUpdate intake: atomicMin on the current keys, a mark byte per id
//       whose key dropped, and their compaction into U sorted by id.
//   k_tsort / k_spart / k_smerge
//       Sorting the extracted minima by (key, id): tiles sorted in registers
//       and LDS (per-thread sort, then merge-path rounds), then merge passes.
//   k_absent, k_delete
//       Mark extracted or deleted ids absent.
// The few results the host needs after a step (sizes, the selected element)
// are written by the step's last kernel into host-mapped memory.
#include "wide.h"

#include <algorithm>
#include <chrono>
#include <cstddef>
#include <cstring>
#include <vector>

#include "pbh_team.h"

namespace bkt {
namespace {

using u8 = unsigned char;

constexpr int NT = 256;
constexpr int WE = 8;
constexpr u32 TILE = NT * WE;  // 2048
constexpr int SEL_BITS = 8;
constexpr int SEL_BINS = 1 << SEL_BITS;  // one bin per thread of the pick kernel
constexpr u32 CANDMAX = NT;              // candidates ranked by one workgroup
constexpr int GRID_STRIDE = 2048;        // workgroups of the grid-stride kernels
constexpr int GRID_HIST = 512;           // workgroups of a Select pass or gather (each flushes <= 256
                                         // atomics, and one on the shared pass counter: about 10 ns
                                         // each on one address, 2048 workgroups measured 20 us)

// Device-side state of a selection (read and written by the Select kernels)
// and the key range of the array it runs on.
struct Ctl {
  u64 kmin, kmax;
  u64 spk;
  u32 spv;
  int snb;      // leading bits of (key, id) fixed so far
  u32 srank;    // rank still sought among the elements with that prefix
  u32 scnt;     // elements with that prefix
  int sdone;    // few enough candidates: gather them
  int sfail;    // the gather ran before the passes were done
  int sbad;     // no bin held the rank (never expected)
  u32 sncand;
  u32 passdone;  // workgroups finished with the current pass (the last one picks)
  u32 npass;     // passes that did work since the last gather (profiling)
  u32 scandone;  // workgroups of a publishing k_scan finished (the last one publishes)
  u32 shist[SEL_BINS];
};

// What the host reads after a step.  The step's kernels write it in device
// memory; k_post then copies it into host-mapped coherent memory and writes
// the step's sequence number last, which the host polls.
struct Mail {
  u32 total;    // output size of a merge or of the mark compaction
  u32 num_le;   // merge outputs <= the counting pivot
  u32 part[4];  // three-way split sizes
  u64 newly;    // ids inserted by the intake
  u64 rk;       // selected element
  u32 rv;
  int sfail;    // the selection needs more passes
  int sbad;     // the selection found no element of the rank (never expected)
  u32 npass;    // Select passes of the step that did work (the others returned at once)
  u32 pad_;     // keeps seq the struct's last word
  u32 seq;      // number of the last step published (host copy only)
};
static_assert(offsetof(Mail, seq) + sizeof(u32) == sizeof(Mail) && sizeof(Mail) % 4 == 0,
              "k_post copies whole words and writes seq last");
constexpr u32 MAIL_WORDS = sizeof(Mail) / 4;

__device__ __forceinline__ u64 atomic_min64(u64* p, u64 v) {
  return __hip_atomic_fetch_min((u64 PBH_GLB*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u32 atomic_add32(u32* p, u32 v) {
  return __hip_atomic_fetch_add((u32 PBH_GLB*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive scan over the workgroup (NTH threads); *total = the sum.
// sw: LDS scratch of NTH/64 words.
template <int NTH>
__device__ __forceinline__ u32 block_scan(u32 x, u32* total, u32* sw) {
  u32 inc = wave_incl(x);
  const int w = (int)(threadIdx.x >> 6);
  if ((threadIdx.x & 63) == 63) sw[w] = inc;
  __syncthreads();
  u32 pre = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < NTH / 64; ++k) {
    u32 s = sw[k];
    pre += k < w ? s : 0u;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return pre + inc - x;
}
template <int NTH>
__device__ __forceinline__ u32 block_sum(u32 x, u32* sw) {
  u32 t;
  block_scan<NTH>(x, &t, sw);
  return t;
}
template <int NTH>
__device__ __forceinline__ void block_minmax(u64& lo, u64& hi, u64* swl, u64* swh) {
  wave_minmax64(lo, hi);
  const int w = (int)(threadIdx.x >> 6);
  if ((threadIdx.x & 63) == 0) {
    swl[w] = lo;
    swh[w] = hi;
  }
  __syncthreads();
  lo = swl[0];
  hi = swh[0];
#pragma unroll
  for (int k = 1; k < NTH / 64; ++k) {
    lo = swl[k] < lo ? swl[k] : lo;
    hi = swh[k] > hi ? swh[k] : hi;
  }
  __syncthreads();
}

// How many of the first `diag` elements of merge(A, B) come from A; ties go
// to A first.  ById compares ids, otherwise (key, id).
template <bool BYKV, class KP, class VP>
__device__ __forceinline__ u32 mpath(KP ak, VP av, u32 na, KP bk, VP bv, u32 nb, u32 diag) {
  u32 lo = diag > nb ? diag - nb : 0u, hi = diag < na ? diag : na;
  while (lo < hi) {
    u32 mid = (lo + hi) >> 1, jb = diag - 1 - mid;
    bool afirst;
    if constexpr (BYKV) {
      u64 ka = ak[mid], kb = bk[jb];
      afirst = ka < kb || (ka == kb && av[mid] <= bv[jb]);
    } else {
      afirst = av[mid] <= bv[jb];
    }
    if (afirst)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// The same split as mpath, found by one wavefront: each round every lane
// tests one of 64 evenly spaced probes and the ballot's popcount (the tests
// are true on a prefix) narrows the range 65-fold, so a split of arrays of
// millions costs about four dependent global loads instead of twenty-odd.
// All 64 lanes must call it with the same arguments.
template <bool BYKV, class KP, class VP>
__device__ __forceinline__ u32 mpath_wave(KP ak, VP av, u32 na, KP bk, VP bv, u32 nb, u32 diag) {
  const u32 lane = threadIdx.x & 63u;
  u32 lo = diag > nb ? diag - nb : 0u, hi = diag < na ? diag : na;
  while (lo < hi) {
    const u32 len = hi - lo;
    const bool small = len <= 64u;
    const u32 mid = small ? lo + lane : lo + (u32)(((u64)(lane + 1) * len) / 65u);
    bool afirst = false;
    if (!small || lane < len) {
      const u32 jb = diag - 1 - mid;
      if constexpr (BYKV) {
        const u64 ka = ak[mid], kb = bk[jb];
        afirst = ka < kb || (ka == kb && av[mid] <= bv[jb]);
      } else {
        afirst = av[mid] <= bv[jb];
      }
    }
    const u32 c = (u32)__popcll(__ballot(afirst));
    if (small) return lo + c;
    if (c == 0) {
      hi = lo + (u32)(len / 65u);
    } else {
      const u32 nlo = lo + (u32)(((u64)c * len) / 65u) + 1u;
      if (c < 64u) hi = lo + (u32)(((u64)(c + 1) * len) / 65u);
      lo = nlo;
    }
  }
  return lo;
}

// ------------------------------------------------------------------ merge by id

struct MArgs {
  const u64* ak;
  const u32* av;
  u32 na;
  const u64* bk;
  const u32* bv;
  u32 nb;
  u64* ck;
  u32* cv;
  const u64* cur;  // liveness for PREFER_LIVE and filterB (may be null)
  int prefer;
  int filterB;
  u64 pk;          // outputs <= (pk, pv) are counted
  u32 pv;
};

// The copy kept when A and B hold the same id (DeleteDuplicates).
__device__ __forceinline__ bool pair_keep(const MArgs& a, u64 ka, u64 kb, u32 v, u64* k) {
  if (a.prefer == PREFER_B) {
    *k = kb;
    return true;
  }
  if (a.prefer == PREFER_A || ka == kb) {
    *k = ka;
    return true;
  }
  if (a.cur) {
    u64 c = a.cur[v];
    *k = kb == c ? kb : ka;
    return ka == c || kb == c;
  }
  *k = ka < kb ? ka : kb;
  return true;
}

// Split searches per workgroup of the sort's partition kernel (one
// wavefront each).
constexpr u32 SPW = NT / 64;

// One tile of merge(A, B) by id with DeleteDuplicates: the outputs at merge
// positions [t*TILE, (t+1)*TILE), whose inputs are A[i0, i1) and B[j0, j1)
// (staged in LDS: ids, and keys in the writing pass).  Each thread takes WE
// consecutive merge positions: one merge-path search in LDS finds where they
// start, then a sequential walk merges them (ties: A first), so a copy of an
// id present in both inputs sits right after A's copy.  The pair is decided
// at A's slot (pair_keep) and B's slot is dropped; a partner just outside the
// tile is A[i0-1] or B[j1].  Counting pass: tcnt[t] = kept outputs; with
// KEYS it also stages the keys and counts the outputs <= (pk, pv) and their
// key range, as per-workgroup partials (thousands of workgroups updating the
// same word with atomics would serialise in the L2) that the scan folds.
// So the scan, which runs before the writing pass, has every result the host
// reads.  Writing pass: a scan of the threads' kept counts gives each output
// its place in the tile's output range; the outputs are transposed through
// LDS (reusing the input staging, at index o + o/8 so that the threads' runs
// of WE spread over the banks) and stored coalesced at toff[t] + o.  Stored
// straight from the walk, each store instruction would touch 64 cache lines
// (a thread's outputs are consecutive), which measured 1.6x slower.
struct Partials {
  u32* cnt;
  u64* lo;
  u64* hi;
};

template <bool WRITE, bool KEYS = WRITE>
__global__ __launch_bounds__(NT) void k_merge(MArgs a, const u32* part, u32* part_out, u32* tcnt, const u32* toff,
                                              Partials pt) {
  static_assert(KEYS || !WRITE, "the writing pass stages keys");
  constexpr u32 NONE = 0xFFFFFFFFu;  // exhausted input (ids are < 2^32 - 1)
  constexpr u32 PAD = WRITE ? TILE / 8 : 0;  // room for the transposed index o + o/8
  __shared__ u32 sv[TILE + PAD];
  __shared__ u64 sk[KEYS ? TILE + PAD : 1];
  __shared__ u32 sw[NT / 64];
  __shared__ u64 swl[NT / 64], swh[NT / 64];
  const u32 t = blockIdx.x, total = a.na + a.nb;
  const u32 d0 = t * TILE, d1 = min(d0 + TILE, total);
  u32 i0, i1;
  if constexpr (!WRITE) {
    // The counting pass finds its tile's split points itself (wavefronts 0
    // and 1, one 65-way search each) and records them for the writing pass.
    __shared__ u32 ssplit[2];
    const u32 wv = threadIdx.x >> 6;
    if (wv < 2) {
      const u64 dg = (u64)(t + wv) * TILE;
      const u32 diag = (u32)(dg < total ? dg : total);
      const u32 i = mpath_wave<false>((const u64*)nullptr, a.av, a.na, (const u64*)nullptr, a.bv, a.nb, diag);
      if ((threadIdx.x & 63u) == 0) ssplit[wv] = i;
    }
    __syncthreads();
    i0 = ssplit[0];
    i1 = ssplit[1];
    if (threadIdx.x == 0) {
      part_out[t] = i0;
      if (t + 1 == gridDim.x) part_out[t + 1] = i1;
    }
  } else {
    i0 = part[t];
    i1 = part[t + 1];
  }
  const u32 j0 = d0 - i0, j1 = d1 - i1;
  const u32 nA = i1 - i0, nT = d1 - d0, nB = nT - nA;
  {
    u64 lk[WE];
    u32 lv[WE];
#pragma unroll
    for (int q = 0; q < WE; ++q) {
      const u32 x = threadIdx.x + (u32)q * NT;
      const bool fromA = x < nA;
      const u32 g = fromA ? i0 + x : j0 + (x - nA);
      lv[q] = 0;
      lk[q] = 0;
      if (x < nT) {
        lv[q] = fromA ? a.av[g] : a.bv[g];
        if constexpr (KEYS) lk[q] = fromA ? a.ak[g] : a.bk[g];
      }
    }
#pragma unroll
    for (int q = 0; q < WE; ++q) {
      const u32 x = threadIdx.x + (u32)q * NT;
      if (x < nT) {
        sv[x] = lv[q];
        if constexpr (KEYS) sk[x] = lk[q];
      }
    }
  }
  const bool hasPrev = i0 > 0, hasNext = j1 < a.nb;
  const u32 aprev = hasPrev ? a.av[i0 - 1] : 0u, bnext = hasNext ? a.bv[j1] : 0u;
  __syncthreads();
  const u32* sA = sv;
  const u32* sB = sv + nA;
  const u32 p0 = min((u32)threadIdx.x * WE, nT), p1 = min(p0 + WE, nT);
  u32 i = mpath<false>((const u64*)nullptr, sA, nA, (const u64*)nullptr, sB, nB, p0);
  u32 j = p0 - i;
  u32 va = i < nA ? sA[i] : NONE, vb = j < nB ? sB[j] : NONE;
  bool havePrevA = i > 0 || hasPrev;
  u32 prevA = i > 0 ? sA[i - 1] : aprev;
  u64 ko[WE];
  u32 vo[WE];
  u32 keep = 0;
#pragma unroll
  for (int q = 0; q < WE; ++q) {
    ko[q] = 0;
    vo[q] = 0;
    if (p0 + (u32)q >= p1) continue;
    bool kp = true;
    if (va <= vb) {  // A's element (first on equal ids)
      const u32 v = va;
      u64 k = KEYS ? sk[i] : 0ull;
      const bool dup = j < nB ? vb == v : (hasNext && bnext == v);
      if (dup && (KEYS || a.prefer == PREFER_LIVE)) {
        const u64 ka = KEYS ? k : a.ak[i0 + i];
        const u64 kb = j < nB ? (KEYS ? sk[nA + j] : a.bk[j0 + j]) : a.bk[j1];
        kp = pair_keep(a, ka, kb, v, &k);
      }
      vo[q] = v;
      ko[q] = k;
      prevA = v;
      havePrevA = true;
      ++i;
      va = i < nA ? sA[i] : NONE;
    } else {  // B's element: dropped when A holds the id
      const u32 v = vb;
      const u64 k = KEYS ? sk[nA + j] : 0ull;
      kp = !(havePrevA && prevA == v);
      if (kp && a.filterB) kp = a.cur[v] == (KEYS ? k : a.bk[j0 + j]);
      vo[q] = v;
      ko[q] = k;
      ++j;
      vb = j < nB ? sB[j] : NONE;
    }
    keep |= (u32)kp << q;
  }
  const u32 nk = (u32)__builtin_popcount(keep);
  if constexpr (!WRITE) {
    const u32 tot = block_sum<NT>(nk, sw);
    if (threadIdx.x == 0) tcnt[t] = tot;
    if constexpr (KEYS) {
      // statistics of the kept outputs: how many are <= (pk, pv), and the
      // key range
      u32 nle = 0;
      u64 lo = KINF, hi = 0;
#pragma unroll
      for (int q = 0; q < WE; ++q)
        if ((keep >> q) & 1u) {
          nle += kv_le(KV{ko[q], vo[q]}, KV{a.pk, a.pv});
          lo = ko[q] < lo ? ko[q] : lo;
          hi = ko[q] > hi ? ko[q] : hi;
        }
      nle = block_sum<NT>(nle, sw);
      block_minmax<NT>(lo, hi, swl, swh);
      if (threadIdx.x == 0) {
        pt.cnt[t] = nle;
        pt.lo[t] = lo;
        pt.hi[t] = hi;
      }
    }
  } else {
    u32 tot;
    u32 o = block_scan<NT>(nk, &tot, sw);  // its barriers also end every walk's reads of sv / sk
#pragma unroll
    for (int q = 0; q < WE; ++q)
      if ((keep >> q) & 1u) {
        const u32 z = o + (o >> 3);
        sk[z] = ko[q];
        sv[z] = vo[q];
        ++o;
      }
    __syncthreads();
    const u32 base = toff[t];
#pragma unroll
    for (int q = 0; q < WE; ++q) {
      const u32 x = threadIdx.x + (u32)q * NT;
      if (x < tot) {
        const u32 z = x + (x >> 3);
        a.ck[base + x] = sk[z];
        a.cv[base + x] = sv[z];
      }
    }
  }
}

// A step published by the kernel that computes the last result the host
// reads (the scan of a merge, split or compaction, which also folds the
// merge's statistics), instead of by k_post after the step's last kernel:
// the host then reads the sizes and goes on while the step's writing pass,
// whose output it never reads, still runs (its next launches queue behind
// that pass on the stream).  mail == nullptr: the kernel does not publish.
struct Pub {
  const Mail* box;
  Mail* mail;
  u32 seq;
};

// Copies the box into the host-mapped mailbox and then writes the sequence
// number (as k_post).  Called by every thread of the publishing workgroup
// once its results are in the box: the wait and the barrier make this
// workgroup's stores reach the L2, which the agent-scope loads read.
__device__ __forceinline__ void publish(const Pub& p) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  const u32 l = threadIdx.x;
  if (l + 1 < MAIL_WORDS) {
    ((u32*)p.mail)[l] =
        __hip_atomic_load((const u32 PBH_GLB*)p.box + l, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence_system();
  }
  __syncthreads();
  if (l == 0) __hip_atomic_store(&p.mail->seq, p.seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Sums n partial counts into *sum (when sum != null) and folds the partial
// key ranges into ctl->kmin / kmax.  One workgroup.
__global__ __launch_bounds__(1024) void k_reduce(Partials pt, u32 n, u32* sum32, u64* sum64, Ctl* c) {
  __shared__ u32 sw[16];
  __shared__ u64 swl[16], swh[16];
  u64 tot = 0, lo = KINF, hi = 0;
  for (u32 x = threadIdx.x; x < n; x += 1024) {
    tot += pt.cnt[x];
    if (pt.lo) {
      lo = pt.lo[x] < lo ? pt.lo[x] : lo;
      hi = pt.hi[x] > hi ? pt.hi[x] : hi;
    }
  }
  const u32 s = block_sum<1024>((u32)tot, sw);
  block_minmax<1024>(lo, hi, swl, swh);
  if (threadIdx.x == 0) {
    if (sum32) *sum32 = s;
    if (sum64) *sum64 = s;
    if (pt.lo) {
      c->kmin = lo;
      c->kmax = hi;
    }
  }
}

// Exclusive scan of n tile counts (one workgroup of 1024); *total = the sum.
// blockIdx.x selects one of several count arrays spaced `stride` apart.
// With fold.cnt set (one workgroup only) it also folds n per-tile partials:
// *fold_sum = their count, ctl->kmin / kmax = their key range.  With
// pub.mail set, the last of the workgroups to finish publishes the step
// (ctl->scandone counts them; the totals are stored with agent-scope stores
// so that it reads every one).
__global__ __launch_bounds__(1024) void k_scan(const u32* cnt, u32 n, u32 stride, u32* off, u32* total, Ctl* ctl,
                                               Pub pub, Partials fold, u32* fold_sum) {
  __shared__ u32 sw[16];
  __shared__ u64 swl[16], swh[16];
  __shared__ int s_last;
  if (fold.cnt) {
    u32 c = 0;
    u64 lo = KINF, hi = 0;
    for (u32 x = threadIdx.x; x < n; x += 1024) {
      c += fold.cnt[x];
      lo = fold.lo[x] < lo ? fold.lo[x] : lo;
      hi = fold.hi[x] > hi ? fold.hi[x] : hi;
    }
    c = block_sum<1024>(c, sw);
    block_minmax<1024>(lo, hi, swl, swh);
    if (threadIdx.x == 0) {
      *fold_sum = c;
      ctl->kmin = lo;
      ctl->kmax = hi;
    }
  }
  cnt += (u64)blockIdx.x * stride;
  off += (u64)blockIdx.x * stride;
  u32 carry = 0;
  for (u32 b = 0; b < n; b += 1024) {
    u32 x = b + threadIdx.x;
    u32 v = x < n ? cnt[x] : 0u;
    u32 tot;
    u32 e = block_scan<1024>(v, &tot, sw);
    if (x < n) off[x] = carry + e;
    carry += tot;
  }
  if (threadIdx.x == 0)
    __hip_atomic_store((u32 PBH_GLB*)(total + blockIdx.x), carry, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (!pub.mail) return;
  if (gridDim.x > 1) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
      const u32 prev =
          __hip_atomic_fetch_add((u32 PBH_GLB*)&ctl->scandone, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_last = prev == gridDim.x - 1;
      if (s_last) __hip_atomic_store((u32 PBH_GLB*)&ctl->scandone, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (!s_last) return;
  }
  publish(pub);
}


// ------------------------------------------------------------------ three-way split

struct PArgs {
  const u64* k;
  const u32* v;
  u32 n;
  u64 p1k;
  u32 p1v;
  u64 p2k;
  u32 p2v;
  const u64* live;  // class-0 elements whose key is not live[id] are dropped
  u64* ok[3];
  u32* ov[3];
  // When set, the first pivot is min(the element Select published in this
  // box, (p1k, p1v)), and a failed Select (sfail / sbad) splits nothing.
  const Mail* sel;
};

// The first pivot: (p1k, p1v), or its minimum with the Select result; false:
// the Select failed, nothing is split.  (The arguments stay untouched: a
// modified copy of them, indexed by class, would live in scratch memory.)
__device__ __forceinline__ bool part_pivot(const PArgs& a, KV* p1) {
  *p1 = KV{a.p1k, a.p1v};
  if (!a.sel) return true;
  if (a.sel->sfail || a.sel->sbad) return false;
  const KV s{a.sel->rk, a.sel->rv};
  if (kv_less(s, *p1)) *p1 = s;
  return true;
}

__device__ __forceinline__ u32 pclass(const PArgs& a, KV p1, u64 k, u32 v) {
  KV e{k, v};
  u32 c = kv_le(e, p1) ? 0u : (kv_le(e, KV{a.p2k, a.p2v}) ? 1u : 2u);
  if (c == 0 && a.live && a.live[v] != k) c = 3;
  return c;
}

// Tile t = elements [t*TILE, (t+1)*TILE), visited in WE rounds of NT
// consecutive elements so that each round's outputs are written coalesced.
template <bool WRITE>
__global__ __launch_bounds__(NT) void k_part(PArgs a, u32* tc, const u32* toff, u32 stride) {
  __shared__ u32 sw[NT / 64];
  const u32 t = blockIdx.x;
  KV p1;
  const u32 n = part_pivot(a, &p1) ? a.n : 0u;  // a failed Select: every element counts as dropped
  const u64 base = (u64)t * TILE;
  u32 c01 = 0, c2 = 0;
  u32 run[3] = {0, 0, 0};
  if constexpr (WRITE) {
    run[0] = toff[t];
    run[1] = toff[stride + t];
    run[2] = toff[2 * stride + t];
  }
  u64 kk[WE];
  u32 vv[WE];
#pragma unroll
  for (int r = 0; r < WE; ++r) {
    const u64 x = base + (u64)r * NT + threadIdx.x;
    kk[r] = x < n ? a.k[x] : 0;
    vv[r] = x < n ? a.v[x] : 0;
  }
#pragma unroll
  for (int r = 0; r < WE; ++r) {
    const u64 x = base + (u64)r * NT + threadIdx.x;
    const u64 k = kk[r];
    const u32 v = vv[r];
    const u32 c = x < n ? pclass(a, p1, k, v) : 3u;
    if constexpr (!WRITE) {
      c01 += c == 0 ? 1u : (c == 1 ? 1u << 16 : 0u);
      c2 += c == 2;
    } else {
      u32 tot;
      u32 e = block_scan<NT>(c < 3 ? 1u << (10 * c) : 0u, &tot, sw);
      if (c < 3) {
        u32 pos = run[c] + ((e >> (10 * c)) & 1023u);
        a.ok[c][pos] = k;
        a.ov[c][pos] = v;
      }
      run[0] += tot & 1023u;
      run[1] += (tot >> 10) & 1023u;
      run[2] += (tot >> 20) & 1023u;
    }
  }
  if constexpr (!WRITE) {
    c01 = block_sum<NT>(c01, sw);
    c2 = block_sum<NT>(c2, sw);
    if (threadIdx.x == 0) {
      tc[t] = c01 & 0xFFFFu;
      tc[stride + t] = c01 >> 16;
      tc[2 * stride + t] = c2;
    }
  }
}

// ------------------------------------------------------------------ Select

__device__ __forceinline__ bool sel_match(u64 k, u32 v, u64 pk, u32 pv, int nb) {
  if (nb == 0) return true;
  if (nb <= 64) return (k >> (64 - nb)) == (pk >> (64 - nb));
  if (k != pk) return false;
  const int r = nb - 64;
  return (v >> (32 - r)) == (pv >> (32 - r));
}
// Bits [p, p + w) of the 96-bit value key * 2^32 + id.
__device__ __forceinline__ u32 sel_digit(u64 k, u32 v, int p, int w) {
  const u32 mask = (1u << w) - 1u;
  if (p >= 32) return (u32)(k >> (p - 32)) & mask;
  return (u32)(((k << 32) | v) >> p) & mask;
}

// Agent-scope atomic loads and stores: coherent across the XCDs' L2 caches
// within a launch, for words that workgroups of one launch hand to each
// other (a plain store can stay in one XCD's L2 until the kernel ends).
__device__ __forceinline__ u32 ld_a32(const u32* p) {
  return __hip_atomic_load((const u32 PBH_GLB*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u64 ld_a64(const u64* p) {
  return __hip_atomic_load((const u64 PBH_GLB*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_a32(u32* p, u32 v) {
  __hip_atomic_store((u32 PBH_GLB*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_a64(u64* p, u64 v) {
  __hip_atomic_store((u64 PBH_GLB*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Is this workgroup the last of the launch to get here?  Each thread first
// waits for its own memory operations (its atomics have then been performed),
// then one counter increment per workgroup; the last one sees gridDim.x - 1
// and resets the counter for the next launch.
__device__ __forceinline__ bool last_workgroup(u32* ctr, int* s_last) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    const u32 prev = __hip_atomic_fetch_add((u32 PBH_GLB*)ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *s_last = prev == gridDim.x - 1;
    if (*s_last) st_a32(ctr, 0u);
  }
  __syncthreads();
  return *s_last != 0;
}

// The starting prefix of a selection of rank r among n elements whose keys
// lie in [ctl->kmin, ctl->kmax]: the bits the keys share.
struct SelState {
  u64 pk;
  u32 pv;
  int nb;
  u32 rank, cnt;
  int done;
};
__device__ __forceinline__ SelState sel_start(const Ctl* c, u32 r, u32 n) {
  const u64 mn = c->kmin, mx = c->kmax;
  SelState q;
  if (mn == mx) {
    q.nb = 64;
    q.pk = mn;
  } else {
    q.nb = __builtin_clzll(mn ^ mx);
    q.pk = q.nb ? (mn >> (64 - q.nb)) << (64 - q.nb) : 0ull;
  }
  q.pv = 0;
  q.rank = r;
  q.cnt = n;
  q.done = n <= CANDMAX;
  return q;
}

// One radix pass of Select (rank r among A[0, n)): every workgroup histograms
// its share of the elements that match the prefix fixed so far (LDS, then one
// atomic per non-empty bin); the last workgroup to finish reads the total,
// moves the bin holding the rank into the prefix, writes the new state to ctl
// and clears the histogram.  The first pass (`first`) derives the starting
// prefix from the key range in ctl (every workgroup the same); later passes
// read the state, and return at once when the selection is done.
__global__ __launch_bounds__(NT) void k_sel_pass(const u64* K, const u32* V, u32 n, Ctl* c, u32 r, int first) {
  static_assert(SEL_BINS == NT, "one bin per thread");
  __shared__ u32 h[SEL_BINS];
  __shared__ u32 sw[NT / 64];
  __shared__ int s_last;
  SelState q;
  if (first) {
    q = sel_start(c, r, n);
    if (q.done) {  // few enough elements: no pass needed
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        c->spk = q.pk;
        c->spv = q.pv;
        c->snb = q.nb;
        c->srank = q.rank;
        c->scnt = q.cnt;
        c->sdone = 1;
        c->sbad = 0;
      }
      return;
    }
  } else {
    q.done = c->sdone;
    if (q.done) return;
    q.pk = c->spk;
    q.pv = c->spv;
    q.nb = c->snb;
    q.rank = c->srank;
    q.cnt = c->scnt;
  }
  const int w = 96 - q.nb < SEL_BITS ? 96 - q.nb : SEL_BITS;
  const int p = 96 - q.nb - w;
  // the ids take part only once the prefix or this pass's digit reaches
  // them; until then the pass reads the keys alone
  const bool needv = q.nb > 64 || p < 32;
  h[threadIdx.x] = 0;
  __syncthreads();
  const u64 step = (u64)gridDim.x * NT;
  for (u64 x0 = (u64)blockIdx.x * NT + threadIdx.x; x0 < n; x0 += 4 * step) {
    u64 k[4];
    u32 v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const u64 x = x0 + j * step;
      k[j] = x < n ? K[x] : KINF;
      v[j] = needv && x < n ? V[x] : 0u;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (x0 + j * step < n && sel_match(k[j], v[j], q.pk, q.pv, q.nb)) atomicAdd(&h[sel_digit(k[j], v[j], p, w)], 1u);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomic_add32(&c->shist[threadIdx.x], h[threadIdx.x]);
  if (!last_workgroup(&c->passdone, &s_last)) return;
  // the pick, by the last workgroup: bin b (one per thread) holds the rank
  if (threadIdx.x == 0) c->npass += 1;
  const u32 b = threadIdx.x;
  const u32 hb = ld_a32(&c->shist[b]);
  u32 tot;
  const u32 before = block_scan<NT>(hb, &tot, sw);
  if (hb && before < q.rank && q.rank <= before + hb) {
    u64 pk = q.pk;
    u32 pv = q.pv;
    if (p >= 32) {
      pk |= (u64)b << (p - 32);
    } else {
      u64 lo = ((pk & 0xFFFFFFFFull) << 32) | pv;
      lo |= (u64)b << p;
      pk = (pk & 0xFFFFFFFF00000000ull) | (lo >> 32);
      pv = (u32)lo;
    }
    c->spk = pk;
    c->spv = pv;
    c->snb = q.nb + w;
    c->srank = q.rank - before;
    c->scnt = hb;
    c->sdone = hb <= CANDMAX || q.nb + w == 96;
    c->sbad = 0;
  }
  if (threadIdx.x == 0 && (q.rank == 0 || q.rank > tot)) {
    c->sbad = 1;
    c->sdone = 1;
  }
  st_a32(&c->shist[b], 0u);
}

// Gathers the elements that match the selected prefix (at most CANDMAX) and,
// in the last workgroup to finish, ranks them by counting: the one with
// exactly rank-1 smaller candidates is the answer.  Publishes the outcome to
// the box (sfail: the passes were not done; sbad: a consistency check failed).
__global__ __launch_bounds__(NT) void k_sel_collect(const u64* K, const u32* V, u32 n, Ctl* c, u64* ck, u32* cv,
                                                    Mail* box) {
  __shared__ u64 sk[CANDMAX];
  __shared__ u32 sv[CANDMAX];
  __shared__ int s_last;
  const int done = c->sdone;
  if (!done) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      box->sfail = 1;
      box->sbad = 0;
      box->npass = c->npass;
      c->npass = 0;
    }
    return;
  }
  const u64 pk = c->spk;
  const u32 pv = c->spv;
  const int nb = c->snb;
  const u64 step = (u64)gridDim.x * NT;
  const bool needv = nb > 64;  // otherwise the match reads the keys alone, and a candidate's id is read when found
  if (!c->sbad)
    for (u64 x0 = (u64)blockIdx.x * NT + threadIdx.x; x0 < n; x0 += 4 * step) {
      u64 k[4];
      u32 v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const u64 x = x0 + j * step;
        k[j] = x < n ? K[x] : KINF;
        v[j] = needv && x < n ? V[x] : 0u;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (x0 + j * step < n && sel_match(k[j], v[j], pk, pv, nb)) {
          const u32 o = atomic_add32(&c->sncand, 1u);
          if (o < CANDMAX) {
            st_a64(ck + o, k[j]);
            st_a32(cv + o, needv ? v[j] : V[x0 + j * step]);
          }
        }
    }
  if (!last_workgroup(&c->passdone, &s_last)) return;
  const u32 nc0 = ld_a32(&c->sncand), m = nc0 < CANDMAX ? nc0 : CANDMAX;
  const u32 r = c->srank;
  if (threadIdx.x < m) {
    sk[threadIdx.x] = ld_a64(ck + threadIdx.x);
    sv[threadIdx.x] = ld_a32(cv + threadIdx.x);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    box->sfail = 0;
    box->sbad = (c->sbad || r == 0 || r > m || nc0 != c->scnt) ? 1 : 0;
    box->npass = c->npass;
    c->npass = 0;
    st_a32(&c->sncand, 0u);
  }
  if (threadIdx.x < m) {
    const u64 k = sk[threadIdx.x];
    const u32 v = sv[threadIdx.x];
    u32 below = 0;
    for (u32 y = 0; y < m; ++y) below += sk[y] < k || (sk[y] == k && sv[y] < v);
    if (below + 1 == r) {
      box->rk = k;
      box->rv = v;
    }
  }
}

__global__ __launch_bounds__(NT) void k_minmax(const u64* K, u32 n, Partials pt) {
  __shared__ u64 swl[NT / 64], swh[NT / 64];
  u64 lo = KINF, hi = 0;
  const u64 step = (u64)gridDim.x * NT;
  for (u64 x0 = (u64)blockIdx.x * NT + threadIdx.x; x0 < n; x0 += 4 * step) {
    u64 k[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) k[q] = x0 + q * step < n ? K[x0 + q * step] : KINF;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (x0 + q * step < n) {
        lo = k[q] < lo ? k[q] : lo;
        hi = k[q] > hi ? k[q] : hi;
      }
  }
  block_minmax<NT>(lo, hi, swl, swh);
  if (threadIdx.x == 0) {
    pt.cnt[blockIdx.x] = 0;
    pt.lo[blockIdx.x] = lo;
    pt.hi[blockIdx.x] = hi;
  }
}

// ------------------------------------------------------------------ publishing

// Copies a step's results (box, device memory) into the host-mapped mailbox,
// then writes the sequence number with a system-scope release.  Each lane
// fences its own word before the barrier, so every word is visible to the
// host before seq is.
__global__ __launch_bounds__(64) void k_post(const Mail* box, Mail* mail, u32 seq) {
  const u32 l = threadIdx.x;
  if (l + 1 < MAIL_WORDS) {
    ((u32*)mail)[l] = ((const u32*)box)[l];
    __threadfence_system();
  }
  __syncthreads();
  if (l == 0) __hip_atomic_store(&mail->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// ------------------------------------------------------------------ intake

// cur[id] = min(cur[id], key) for every pair (atomicMin); an id whose key
// dropped gets its mark byte set by a plain store (every writer stores the
// same 1, so no atomic is needed: a random atomic costs a round trip to the
// memory side, a byte store is merged in the L2).
__global__ __launch_bounds__(NT) void k_intake(const u64* keys, const u32* ids, u64 count, u64* cur, u8* marks,
                                               Partials pt) {
  __shared__ u32 sw[NT / 64];
  u32 newly = 0;
  const u64 step = (u64)gridDim.x * NT;
  for (u64 x0 = (u64)blockIdx.x * NT + threadIdx.x; x0 < count; x0 += 4 * step) {
    u32 id[4];
    u64 k[4], old[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const u64 x = x0 + q * step;
      id[q] = x < count ? ids[x] : 0u;
      k[q] = x < count ? keys[x] : KINF;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) old[q] = x0 + q * step < count ? atomic_min64(cur + id[q], k[q]) : KINF;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (k[q] < old[q]) {
        marks[id[q]] = 1;
        newly += old[q] == KINF;
      }
  }
  newly = block_sum<NT>(newly, sw);
  if (threadIdx.x == 0) pt.cnt[blockIdx.x] = newly;
}

// Mark compaction: marked ids in increasing order -> (cur[id], id); the
// marks are cleared.  Each thread takes 32 consecutive ids (two 16-byte loads)
// per round, turned into a 32-bit mask; tile t = ids [t*TILE*32, (t+1)*TILE*32)
// in WE rounds.  In the writing pass each round's marked ids are gathered in
// LDS in order (a scan of the masks' popcounts places them) and then written
// out coalesced, one output per thread, with cur[id] read alongside.
__device__ __forceinline__ u32 mark_mask(uint4 m) {
  const u32 w[4] = {m.x, m.y, m.z, m.w};
  u32 bits = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int b = 0; b < 4; ++b) bits |= (u32)(((w[j] >> (8 * b)) & 0xFFu) != 0u) << (4 * j + b);
  return bits;
}
template <bool WRITE>
__global__ __launch_bounds__(NT) void k_bits(u8* marks, u32 nwords, u32* tc, const u32* toff, const u64* cur,
                                             u64* uk, u32* uv) {
  __shared__ u32 sw[NT / 64];
  __shared__ u32 sid[WRITE ? NT * 32 : 1];
  const u32 t = blockIdx.x;
  u32 run = WRITE ? toff[t] : 0u, cnt = 0;
  uint4* m4 = (uint4*)marks;
  u32 bitsr[WE];
#pragma unroll
  for (int r = 0; r < WE; ++r) {
    const u64 w = (u64)t * TILE + (u64)r * NT + threadIdx.x;
    bitsr[r] = w < nwords ? mark_mask(m4[2 * w]) | (mark_mask(m4[2 * w + 1]) << 16) : 0u;
  }
#pragma unroll
  for (int r = 0; r < WE; ++r) {
    const u64 w = (u64)t * TILE + (u64)r * NT + threadIdx.x;
    u32 bits = bitsr[r];
    const u32 pc = (u32)__builtin_popcount(bits);
    if constexpr (!WRITE) {
      cnt += pc;
    } else {
      u32 tot;
      u32 o = block_scan<NT>(pc, &tot, sw);  // its barriers also end the previous round's reads of sid
      if (bits) {
        m4[2 * w] = make_uint4(0u, 0u, 0u, 0u);
        m4[2 * w + 1] = make_uint4(0u, 0u, 0u, 0u);
      }
      while (bits) {
        const u32 b = (u32)__builtin_ctz(bits);
        bits &= bits - 1;
        sid[o++] = (u32)w * 32u + b;
      }
      __syncthreads();
      for (u32 x = threadIdx.x; x < tot; x += NT) {
        const u32 id = sid[x];
        uv[run + x] = id;
        uk[run + x] = cur[id];
      }
      run += tot;
    }
  }
  if constexpr (!WRITE) {
    cnt = block_sum<NT>(cnt, sw);
    if (threadIdx.x == 0) tc[t] = cnt;
  }
}

// Delete of a batch of ids: cur[id] = KINF; each workgroup counts the ids
// that were present (the exchange returns the old key, so repeats in the
// batch count once).
__global__ __launch_bounds__(NT) void k_delete(const u32* ids, u64 count, u64* cur, Partials pt) {
  __shared__ u32 sw[NT / 64];
  u32 gone = 0;
  for (u64 x = (u64)blockIdx.x * NT + threadIdx.x; x < count; x += (u64)gridDim.x * NT)
    gone += __hip_atomic_exchange((u64 PBH_GLB*)(cur + ids[x]), KINF, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) !=
                    KINF
                ? 1u
                : 0u;
  gone = block_sum<NT>(gone, sw);
  if (threadIdx.x == 0) pt.cnt[blockIdx.x] = gone;
}

__global__ void k_absent(const u32* ids, u64 n, u64* cur) {
  for (u64 x = (u64)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (u64)gridDim.x * blockDim.x)
    cur[ids[x]] = KINF;
}

// ------------------------------------------------------------------ sort by (key, id)

// Compare-exchange by (key, id).
__device__ __forceinline__ void cx(u64& ka, u32& va, u64& kb, u32& vb) {
  if (ka > kb || (ka == kb && va > vb)) {
    const u64 tk = ka;
    const u32 tv = va;
    ka = kb;
    va = vb;
    kb = tk;
    vb = tv;
  }
}

// Sorts each tile of TILE (key, id) pairs by (key, id): every thread sorts
// its WE consecutive elements in registers (odd-even transposition), then
// rounds merge the runs of WE, 2WE, ..., TILE/2 pairwise in LDS (ping-pong
// buffers), each thread producing its WE consecutive outputs after one
// merge-path search.  About a quarter of the LDS accesses of a bitonic sort
// of the tile in LDS, and 8 barriers instead of 66.  Padding (KINF, VINF)
// sorts last and is not written.
__global__ __launch_bounds__(NT) void k_tsort(const u64* sk_, const u32* sv_, u32 n, u64* dk, u32* dv) {
  __shared__ u64 bk[2][TILE];
  __shared__ u32 bv[2][TILE];
  const u64 base = (u64)blockIdx.x * TILE;
  {
    u64 lk[WE];
    u32 lv[WE];
#pragma unroll
    for (int q = 0; q < WE; ++q) {
      const u64 g = base + threadIdx.x + (u64)q * NT;
      lk[q] = g < n ? sk_[g] : KINF;
      lv[q] = g < n ? sv_[g] : VINF;
    }
#pragma unroll
    for (int q = 0; q < WE; ++q) {
      bk[0][threadIdx.x + q * NT] = lk[q];
      bv[0][threadIdx.x + q * NT] = lv[q];
    }
  }
  __syncthreads();
  const u32 o0 = threadIdx.x * WE;
  u64 k[WE];
  u32 v[WE];
#pragma unroll
  for (int q = 0; q < WE; ++q) {
    k[q] = bk[0][o0 + q];
    v[q] = bv[0][o0 + q];
  }
#pragma unroll
  for (int r = 0; r < WE; ++r)
#pragma unroll
    for (int i = r & 1; i + 1 < WE; i += 2) cx(k[i], v[i], k[i + 1], v[i + 1]);
  int cur = 1;
  for (u32 L = WE; L < TILE; L *= 2, cur ^= 1) {
    // (buffer cur was last read two rounds ago, before the previous barrier)
#pragma unroll
    for (int q = 0; q < WE; ++q) {
      bk[cur][o0 + q] = k[q];
      bv[cur][o0 + q] = v[q];
    }
    __syncthreads();
    const u32 pb = (o0 / (2 * L)) * (2 * L), diag = o0 - pb;
    const u64* ak = bk[cur] + pb;
    const u32* av = bv[cur] + pb;
    const u64* bk2 = ak + L;
    const u32* bv2 = av + L;
    u32 i = mpath<true>(ak, av, L, bk2, bv2, L, diag), j = diag - i;
    u64 xa = i < L ? ak[i] : KINF, xb = j < L ? bk2[j] : KINF;
    u32 ya = i < L ? av[i] : VINF, yb = j < L ? bv2[j] : VINF;
#pragma unroll
    for (int q = 0; q < WE; ++q) {
      const bool ta = i < L && (j >= L || xa < xb || (xa == xb && ya <= yb));
      if (ta) {
        k[q] = xa;
        v[q] = ya;
        ++i;
        xa = i < L ? ak[i] : KINF;
        ya = i < L ? av[i] : VINF;
      } else {
        k[q] = xb;
        v[q] = yb;
        ++j;
        xb = j < L ? bk2[j] : KINF;
        yb = j < L ? bv2[j] : VINF;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < WE; ++q) {
    bk[cur][o0 + q] = k[q];
    bv[cur][o0 + q] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < WE; ++q) {
    const u32 x = threadIdx.x + (u32)q * NT;
    const u64 g = base + x;
    if (g < n) {
      dk[g] = bk[cur][x];
      dv[g] = bv[cur][x];
    }
  }
}

// Merge pass over sorted runs of length L (a multiple of TILE): runs 2p and
// 2p+1 are merged into [2pL, 2pL + 2L).  part[t] = A-elements before output
// tile t within its pair.
__device__ __forceinline__ void run_pair(u32 n, u32 L, u64 s, u32* base, u32* na, u32* nb) {
  const u64 b = (s / (2ull * L)) * 2ull * L;
  const u64 mid = b + L < n ? b + L : n, end = b + 2ull * L < n ? b + 2ull * L : n;
  *base = (u32)b;
  *na = (u32)(mid - b);
  *nb = (u32)(end - mid);
}

__global__ __launch_bounds__(NT) void k_spart(const u64* K, const u32* V, u32 n, u32 L, u32 ntiles, u32* part) {
  const u32 t = blockIdx.x * SPW + (threadIdx.x >> 6);
  if (t >= ntiles) return;
  u32 b, na, nb;
  run_pair(n, L, (u64)t * TILE, &b, &na, &nb);
  const u32 i = mpath_wave<true>(K + b, V + b, na, K + b + na, V + b + na, nb, t * TILE - b);
  if ((threadIdx.x & 63u) == 0) part[t] = i;
}

__global__ __launch_bounds__(NT) void k_smerge(const u64* K, const u32* V, u32 n, u32 L, const u32* part, u64* DK,
                                               u32* DV) {
  __shared__ u64 sk[TILE];
  __shared__ u32 sv[TILE];
  const u32 t = blockIdx.x;
  const u64 s = (u64)t * TILE;
  u32 b, na, nb;
  run_pair(n, L, s, &b, &na, &nb);
  const u32 d0 = (u32)(s - b);
  const u32 d1 = min(d0 + TILE, na + nb);
  const u32 i0 = part[t];
  const u32 i1 = d1 == na + nb ? na : part[t + 1];
  const u32 j0 = d0 - i0, j1 = d1 - i1;
  const u32 nA = i1 - i0, nT = d1 - d0, nB = j1 - j0;
  {
    u64 lk[WE];
    u32 lv[WE];
#pragma unroll
    for (int q = 0; q < WE; ++q) {
      const u32 x = threadIdx.x + (u32)q * NT;
      const u32 g = x < nA ? b + i0 + x : b + na + j0 + (x - nA);
      lk[q] = x < nT ? K[g] : 0;
      lv[q] = x < nT ? V[g] : 0;
    }
#pragma unroll
    for (int q = 0; q < WE; ++q) {
      const u32 x = threadIdx.x + (u32)q * NT;
      if (x < nT) {
        sk[x] = lk[q];
        sv[x] = lv[q];
      }
    }
  }
  __syncthreads();
  const u32 dd0 = min((u32)threadIdx.x * WE, nT), dd1 = min(dd0 + WE, nT);
  u32 i = mpath<true>(sk, sv, nA, sk + nA, sv + nA, nB, dd0), j = dd0 - i;
  u64 ko[WE];
  u32 vo[WE];
#pragma unroll
  for (int q = 0; q < WE; ++q) {
    ko[q] = 0;
    vo[q] = 0;
    if (dd0 + q < dd1) {
      bool takeA = i < nA;
      if (takeA && j < nB) {
        const u64 ka = sk[i], kb = sk[nA + j];
        takeA = ka < kb || (ka == kb && sv[i] <= sv[nA + j]);
      }
      if (takeA) {
        ko[q] = sk[i];
        vo[q] = sv[i];
        ++i;
      } else {
        ko[q] = sk[nA + j];
        vo[q] = sv[nA + j];
        ++j;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < WE; ++q)
    if (dd0 + q < dd1) {
      sk[dd0 + q] = ko[q];
      sv[dd0 + q] = vo[q];
    }
  __syncthreads();
  for (u32 x = threadIdx.x; x < nT; x += NT) {
    DK[s + x] = sk[x];
    DV[s + x] = sv[x];
  }
}

u32 cdiv(u64 a, u64 b) { return (u32)((a + b - 1) / b); }
u32 grid_for(u64 n) {
  u64 g = (n + NT - 1) / NT;
  return (u32)(g < 1 ? 1 : (g > GRID_STRIDE ? GRID_STRIDE : g));
}

}  // namespace

struct WideScratch {
  u32 d = 0;
  Ctl* ctl = nullptr;      // device
  Mail* box = nullptr;     // device: results of the current step
  Mail* mail_h = nullptr;  // host-mapped coherent mailbox (host view)
  Mail* mail_d = nullptr;  // its device address
  u32 seq = 0;             // steps published so far
  u8* marks = nullptr;     // one byte per id (32 per 32-id word), zero between calls
  u64 marks_n = 0;
  u32* part = nullptr;  // tile split points (maxtiles + 1)
  u32* tc = nullptr;    // tile counts, 3 arrays of maxtiles
  u32* toff = nullptr;  // tile offsets, 3 arrays of maxtiles
  u64* cand_k = nullptr;
  u32* cand_v = nullptr;
  u64* tmp_k = nullptr;  // sort scratch (4d elements)
  u32* tmp_v = nullptr;
  Partials pt{nullptr, nullptr, nullptr};  // one slot per tile / workgroup (maxtiles, >= GRID_STRIDE)
  u32 maxtiles = 0;
  hipStream_t s = 0;
  // Profiling (off by default): HIP events around every kernel launch of
  // the engine, with the kernel's kind and algorithmic bytes; totalled per
  // kind when the operation ends.
  bool profile = false;
  struct Rec {
    int kind;
    u64 bytes;
  };
  std::vector<hipEvent_t> ev;  // event pairs, created as needed
  std::vector<Rec> rec;        // launches of the current operation
  WideKernelStat kst[WK_COUNT] = {};
};

namespace {

#define WCHK(x)                               \
  do {                                        \
    if ((x) != hipSuccess) return E_DEVICE;   \
  } while (0)

int launch_ok() { return hipGetLastError() == hipSuccess ? 0 : E_DEVICE; }

// Runs launch() -- one kernel launch -- bracketed by HIP events while
// profiling is on.  Returns the launch's record index (bytes can be patched
// once a step's results are known) or -1.
template <class F>
int plaunch(WideScratch* w, int kind, u64 bytes, F&& launch) {
  if (!w->profile) {
    launch();
    return -1;
  }
  const size_t i = w->rec.size();
  while (w->ev.size() < 2 * (i + 1)) {
    hipEvent_t e = nullptr;
    // timing-only events: without the system-scope fence a record does not
    // write back the L2 (which would slow the very step being timed)
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
      launch();
      return -1;
    }
    w->ev.push_back(e);
  }
  (void)hipEventRecord(w->ev[2 * i], w->s);
  launch();
  (void)hipEventRecord(w->ev[2 * i + 1], w->s);
  w->rec.push_back(WideScratch::Rec{kind, bytes});
  return (int)i;
}

void patch_bytes(WideScratch* w, int idx, u64 bytes) {
  if (idx >= 0) w->rec[(size_t)idx].bytes = bytes;
}
void patch_kind(WideScratch* w, int idx, int kind) {
  if (idx >= 0) w->rec[(size_t)idx].kind = kind;
}

// Totals the current operation's timed launches per kind (the operation's
// work has ended, so the events have passed).
int prof_collect(WideScratch* w) {
  if (w->rec.empty()) return 0;
  WCHK(hipEventSynchronize(w->ev[2 * w->rec.size() - 1]));
  for (size_t i = 0; i < w->rec.size(); ++i) {
    float ms = 0.f;
    WCHK(hipEventElapsedTime(&ms, w->ev[2 * i], w->ev[2 * i + 1]));
    WideKernelStat& k = w->kst[w->rec[i].kind];
    k.launches += 1;
    k.bytes += w->rec[i].bytes;
    k.ms += ms;
  }
  w->rec.clear();
  return 0;
}

// Waits until the host sees step `want` published, by polling the mailbox's
// sequence number (a stream synchronisation would add the runtime's
// completion path and a system-scope cache write-back to every step).
// Should the number not arrive within a second, the stream is synchronised,
// which also reports a failed kernel (E_DEVICE); a step whose kernels all
// ended without the number arriving gives E_TIMEOUT.
int wait_mail(WideScratch* w, u32 want) {
  const auto t0 = std::chrono::steady_clock::now();
  for (u32 spin = 1;; ++spin) {
    if (__atomic_load_n(&w->mail_h->seq, __ATOMIC_ACQUIRE) == want) return 0;
    if ((spin & 4095u) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(1)) break;
  }
  WCHK(hipStreamSynchronize(w->s));
  return __atomic_load_n(&w->mail_h->seq, __ATOMIC_ACQUIRE) == want ? 0 : E_TIMEOUT;
}

// Ends a step whose kernels do not publish it: k_post publishes the box,
// then the host waits for it.
int fetch(WideScratch* w) {
  const u32 want = ++w->seq;
  plaunch(w, WK_OTHER, 2ull * sizeof(Mail),
          [&] { hipLaunchKernelGGL(k_post, dim3(1), dim3(64), 0, w->s, w->box, w->mail_d, want); });
  if (int rc = launch_ok()) return rc;
  return wait_mail(w, want);
}

// C = DeleteDuplicates(Merge(A, B)) by id; *num_le = outputs <= piv.
int wmerge(WideScratch* w, Arr A, u32 na, Arr B, u32 nb, Arr C, const u64* cur, int prefer, bool filterB, KV piv,
           u32* m, u32* num_le, bool stats = true) {
  const u64 total = (u64)na + nb;
  if (total == 0) {
    *m = 0;
    *num_le = 0;
    return 0;
  }
  const u32 nt = cdiv(total, TILE);
  if (nt > w->maxtiles) return E_INTERNAL;
  MArgs a{A.k, A.v, na, B.k, B.v, nb, C.k, C.v, cur, prefer, filterB ? 1 : 0, piv.k, piv.v};
  // With stats the counting pass also stages the keys and counts the outputs
  // <= piv and their key range; the scan folds those and publishes the step,
  // so the host goes on while the writing pass runs.
  if (stats)
    plaunch(w, WK_MERGE_COUNT, 12ull * total, [&] {
      hipLaunchKernelGGL((k_merge<false, true>), dim3(nt), dim3(NT), 0, w->s, a, (const u32*)nullptr, w->part, w->tc,
                         (const u32*)nullptr, w->pt);
    });
  else
    plaunch(w, WK_MERGE_COUNT, 4ull * total, [&] {
      hipLaunchKernelGGL((k_merge<false, false>), dim3(nt), dim3(NT), 0, w->s, a, (const u32*)nullptr, w->part,
                         w->tc, (const u32*)nullptr, w->pt);
    });
  const u32 want = ++w->seq;
  plaunch(w, WK_OTHER, (stats ? 28ull : 8ull) * nt, [&] {
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, w->s, w->tc, nt, 0u, w->toff, &w->box->total, w->ctl,
                       Pub{w->box, w->mail_d, want}, stats ? w->pt : Partials{nullptr, nullptr, nullptr},
                       &w->box->num_le);
  });
  const int iw = plaunch(w, WK_MERGE_WRITE, 12ull * total, [&] {
    hipLaunchKernelGGL((k_merge<true, true>), dim3(nt), dim3(NT), 0, w->s, a, (const u32*)w->part, (u32*)nullptr,
                       (u32*)nullptr, (const u32*)w->toff, w->pt);
  });
  if (int rc = launch_ok()) return rc;
  if (int rc = wait_mail(w, want)) return rc;
  *m = w->mail_h->total;
  *num_le = stats ? w->mail_h->num_le : 0u;
  patch_bytes(w, iw, 12ull * (total + *m));  // 12 B per input read + 12 B per output written
  return 0;
}

// Select(A, r) (rank r, 1-based) followed by the three-way split of A at
// (min(Select(A, r), cap), p2) into O0 / O1 / O2, as one host step: the
// split reads the selected element on the device.  *p1 = the split's first
// pivot.  The key range of A must be in ctl (from the merge that wrote A)
// unless have_range is false.
int wpartition3_sel(WideScratch* w, Arr A, u32 n, KV p1, KV p2, Arr O0, Arr O1, Arr O2, const u64* live, u32* n0,
                    u32* n1, u32* n2, const Mail* sel);
int wselpart(WideScratch* w, Arr A, u32 n, u32 r, bool have_range, KV cap, KV p2, Arr O0, Arr O1, Arr O2,
             const u64* live, KV* p1, u32* n0, u32* n1, u32* n2) {
  if (n == 0 || r == 0 || r > n) return E_INTERNAL;
  if (!have_range) {
    const u32 gm = grid_for(n);
    plaunch(w, WK_OTHER, 8ull * n, [&] { hipLaunchKernelGGL(k_minmax, dim3(gm), dim3(NT), 0, w->s, A.k, n, w->pt); });
    plaunch(w, WK_OTHER, 20ull * gm, [&] {
      hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, w->s, w->pt, gm, (u32*)nullptr, (u64*)nullptr, w->ctl);
    });
  }
  const u32 g = grid_for(n), gh = std::min<u32>(g, GRID_HIST);
  // Each pass fixes 8 more of the 96 bits, so 12 passes (4 rounds of 3)
  // always finish; two or three typically do (three when the keys crowd at
  // one end of their range, as decreased keys do).  Passes after the last
  // needed one return at once.
  for (int round = 0; round < 4; ++round) {
    int ip[3];
    for (int p = 0; p < 3; ++p)
      ip[p] = plaunch(w, WK_SEL_PASS, 8ull * n, [&] {
        hipLaunchKernelGGL(k_sel_pass, dim3(gh), dim3(NT), 0, w->s, A.k, A.v, n, w->ctl, r,
                           round == 0 && p == 0 ? 1 : 0);
      });
    const int ic = plaunch(w, WK_SEL_GATHER, 8ull * n, [&] {
      hipLaunchKernelGGL(k_sel_collect, dim3(gh), dim3(NT), 0, w->s, A.k, A.v, n, w->ctl, w->cand_k, w->cand_v,
                         w->box);
    });
    if (int rc = wpartition3_sel(w, A, n, cap, p2, O0, O1, O2, live, n0, n1, n2, w->box)) return rc;
    // passes after the last needed one, and a gather before the passes were
    // done, returned at once: they read nothing
    for (int p = (int)w->mail_h->npass; p < 3; ++p) patch_kind(w, ip[p], WK_IDLE), patch_bytes(w, ip[p], 0);
    if (w->mail_h->sfail) patch_kind(w, ic, WK_IDLE), patch_bytes(w, ic, 0);
    if (w->mail_h->sbad) return E_INTERNAL;
    if (!w->mail_h->sfail) {
      *p1 = cap;
      const KV s{w->mail_h->rk, w->mail_h->rv};
      if (kv_less(s, cap)) *p1 = s;
      return 0;
    }
  }
  return E_INTERNAL;
}

int wpartition3_sel(WideScratch* w, Arr A, u32 n, KV p1, KV p2, Arr O0, Arr O1, Arr O2, const u64* live, u32* n0,
                    u32* n1, u32* n2, const Mail* sel) {
  if (n == 0) {
    *n0 = *n1 = *n2 = 0;
    return 0;
  }
  const u32 nt = cdiv(n, TILE);
  if (nt > w->maxtiles) return E_INTERNAL;
  PArgs a{A.k, A.v, n, p1.k, p1.v, p2.k, p2.v, live, {O0.k, O1.k, O2.k}, {O0.v, O1.v, O2.v}, sel};
  plaunch(w, WK_SPLIT_COUNT, 12ull * n, [&] {
    hipLaunchKernelGGL(k_part<false>, dim3(nt), dim3(NT), 0, w->s, a, w->tc, (const u32*)nullptr, w->maxtiles);
  });
  // published by the scan: the sizes are known before the writing pass
  const u32 want = ++w->seq;
  plaunch(w, WK_OTHER, 24ull * nt, [&] {
    hipLaunchKernelGGL(k_scan, dim3(3), dim3(1024), 0, w->s, w->tc, nt, w->maxtiles, w->toff, w->box->part, w->ctl,
                       Pub{w->box, w->mail_d, want}, Partials{nullptr, nullptr, nullptr}, (u32*)nullptr);
  });
  plaunch(w, WK_SPLIT_WRITE, 24ull * n, [&] {
    hipLaunchKernelGGL(k_part<true>, dim3(nt), dim3(NT), 0, w->s, a, (u32*)nullptr, w->toff, w->maxtiles);
  });
  if (int rc = launch_ok()) return rc;
  if (int rc = wait_mail(w, want)) return rc;
  *n0 = w->mail_h->part[0];
  *n1 = w->mail_h->part[1];
  *n2 = w->mail_h->part[2];
  return 0;
}

int wpartition3(WideScratch* w, Arr A, u32 n, KV p1, KV p2, Arr O0, Arr O1, Arr O2, const u64* live, u32* n0,
                u32* n1, u32* n2) {
  return wpartition3_sel(w, A, n, p1, p2, O0, O1, O2, live, n0, n1, n2, nullptr);
}

// Sorts X[0, n) by (key, id) into D (n <= 4d; X is overwritten).
int wsort(WideScratch* w, Arr X, u32 n, u64* dk, u32* dv) {
  if (n == 0) return 0;
  const u32 nt = cdiv(n, TILE);
  if (nt > w->maxtiles) return E_INTERNAL;
  int passes = 0;
  for (u64 L = TILE; L < n; L *= 2) ++passes;
  // ping-pong so that the last pass lands in D
  Arr bufs[2] = {X, Arr{w->tmp_k, w->tmp_v}};
  Arr dst = passes == 0 ? Arr{dk, dv} : bufs[(passes & 1) ? 1 : 0];
  plaunch(w, WK_SORT_TILE, 24ull * n,
          [&] { hipLaunchKernelGGL(k_tsort, dim3(nt), dim3(NT), 0, w->s, X.k, X.v, n, dst.k, dst.v); });
  Arr src = dst;
  u64 L = TILE;
  for (int p = 0; p < passes; ++p, L *= 2) {
    Arr to = p == passes - 1 ? Arr{dk, dv} : (src.k == bufs[0].k ? bufs[1] : bufs[0]);
    plaunch(w, WK_OTHER, 4ull * nt, [&] {
      hipLaunchKernelGGL(k_spart, dim3(cdiv(nt, SPW)), dim3(NT), 0, w->s, src.k, src.v, n, (u32)L, nt, w->part);
    });
    plaunch(w, WK_SORT_MERGE, 24ull * n, [&] {
      hipLaunchKernelGGL(k_smerge, dim3(nt), dim3(NT), 0, w->s, src.k, src.v, n, (u32)L, w->part, to.k, to.v);
    });
    src = to;
  }
  return launch_ok();
}

// Resolve(i) of Algorithm 1 with the device-wide steps; the control flow is
// the one-workgroup engine's (resolve_t), step for step.
int wresolve(WideScratch* w, const Geom& g, HeapState* st, const u64* cur, int i) {
  Lvl a = st->L[i];
  const bool nx = i + 1 < g.q;
  Lvl b = nx ? st->L[i + 1] : Lvl{0, 0, 0, 0, KINF, VINF, 0};
  int ell = st->ell;
  KV pi{a.pk, a.pv}, pn{b.pk, b.pv};
  const u32 cB = (u32)nomB(g.d, i);
  u64 touched = 0;
  int rc = 0;
  if (a.nS > 0 || a.nB > cB) {
    Arr S = lbuf(g, i, 3 + a.ssel), B = lbuf(g, i, a.bsel), M = lbuf(g, i, a.bsel ^ 1);
    if ((u64)a.nS + a.nB > capB(g.d, i)) return E_INTERNAL;
    u32 m, num;
    // S_0 holds the latest updates, so at level 0 its copy of an id is the live one.
    if ((rc = wmerge(w, S, a.nS, B, a.nB, M, cur, i == 0 ? PREFER_A : PREFER_LIVE, false, pi, &m, &num))) return rc;
    touched += 2ull * (a.nS + a.nB) + m;
    a.bsel ^= 1;
    a.nS = 0;
    a.ssel = 0;
    const bool sel = num > cB;
    if (sel) num = cB;
    if (num < m) {
      if (!nx) return E_CAPACITY;
      Arr Lo = lbuf(g, i, a.bsel ^ 1), Hi = lbuf(g, i, 2);
      u32 n0, n1, n2;
      if (sel) {  // p_i <- Select(B_i, 2d*4^i), and the split at it
        if ((rc = wselpart(w, M, m, cB, true, kv_inf(), kv_inf(), Lo, Hi, Hi, nullptr, &pi, &n0, &n1, &n2))) return rc;
        touched += m;
      } else if ((rc = wpartition3(w, M, m, pi, kv_inf(), Lo, Hi, Hi, nullptr, &n0, &n1, &n2))) {
        return rc;
      }
      touched += 3ull * m;
      a.bsel ^= 1;
      a.nB = n0;
      if ((u64)b.nS + n1 > capS(g.d, i + 1)) return E_INTERNAL;
      Arr Sn = lbuf(g, i + 1, 3 + b.ssel), Sn2 = lbuf(g, i + 1, 3 + (b.ssel ^ 1));
      u32 ms, dummy;
      if ((rc = wmerge(w, Sn, b.nS, Hi, n1, Sn2, cur, PREFER_LIVE, false, kv_inf(), &ms, &dummy, false))) return rc;
      touched += 2ull * (b.nS + n1) + ms;
      b.ssel ^= 1;
      b.nS = ms;
      if (ell < i + 1) ell = i + 1;
    } else {
      a.nB = m;
    }
  }
  if (a.nB < cB && i < ell && nx) {
    Arr Bn = lbuf(g, i + 1, b.bsel), Sn = lbuf(g, i + 1, 3 + b.ssel), M2 = lbuf(g, i + 1, b.bsel ^ 1);
    if ((u64)b.nB + b.nS > capB(g.d, i + 1)) return E_INTERNAL;
    u32 m2, dummy;
    if ((rc = wmerge(w, Bn, b.nB, Sn, b.nS, M2, cur, PREFER_LIVE, false, kv_inf(), &m2, &dummy))) return rc;
    touched += 2ull * (b.nB + b.nS) + m2;
    b.nS = 0;
    b.ssel = 0;
    b.bsel ^= 1;
    b.nB = m2;
    if (m2 > 0) {
      const u32 r = cB - a.nB;
      Arr Up = lbuf(g, i, 2), Bk = lbuf(g, i + 1, b.bsel ^ 1), Sk = lbuf(g, i + 1, 3);
      u32 nu, nb1, ns1;
      // p_i <- min(Select(B_{i+1}, r), p_{i+1}), and the split at (p_i,
      // p_{i+1}); elements moving up into B_0 are checked for liveness here,
      // all at once.
      KV pnew = pn;
      if (r < m2) {
        if ((rc = wselpart(w, M2, m2, r, true, pn, pn, Up, Bk, Sk, i == 0 ? cur : nullptr, &pnew, &nu, &nb1, &ns1)))
          return rc;
        touched += m2;
      } else if ((rc = wpartition3(w, M2, m2, pnew, pn, Up, Bk, Sk, i == 0 ? cur : nullptr, &nu, &nb1, &ns1))) {
        return rc;
      }
      touched += 3ull * m2;
      b.bsel ^= 1;
      b.nB = nb1;
      b.nS = ns1;
      b.ssel = 0;
      Arr Bi = lbuf(g, i, a.bsel), Bi2 = lbuf(g, i, a.bsel ^ 1);
      u32 mb;
      if ((rc = wmerge(w, Bi, a.nB, Up, nu, Bi2, cur, i == 0 ? PREFER_B : PREFER_LIVE, false, kv_inf(), &mb,
                       &dummy, false)))
        return rc;
      touched += 2ull * (a.nB + nu) + mb;
      a.bsel ^= 1;
      a.nB = mb;
      pi = pnew;
    }
  }
  a.cnt++;
  a.pk = pi.k;
  a.pv = pi.v;
  st->L[i] = a;
  if (nx) st->L[i + 1] = b;
  st->elems += touched;
  fix_ell(st, g.q);
  return 0;
}

void wdrive(WideScratch* w, WideHeap* h, int what) {
  HostTeam t{nullptr};
  drive_with(t, h->g, h->st, h->sched, what, [&](int lvl) {
    int rc = wresolve(w, h->g, h->st, h->cur, lvl);
    if (rc) h->st->err = rc;
  });
}

int grow_if_needed(WideScratch* w, WideHeap* h) {
  while (need_grow(h->g, h->st)) {
    if (int rc = h->grow(h->ctx, &h->g)) return rc;
    if (int rc = wide_reserve(w, capB(h->g.d, h->g.q - 1))) return rc;
  }
  return 0;
}

}  // namespace

int wide_reserve(WideScratch* w, u64 elems) {
  u64 need = (elems + TILE - 1) / TILE + 2;
  if (need < (u64)GRID_STRIDE) need = GRID_STRIDE;
  if (need <= w->maxtiles) return 0;
  if (w->part) (void)hipFree(w->part);
  if (w->tc) (void)hipFree(w->tc);
  if (w->toff) (void)hipFree(w->toff);
  if (w->pt.cnt) (void)hipFree(w->pt.cnt);
  if (w->pt.lo) (void)hipFree(w->pt.lo);
  if (w->pt.hi) (void)hipFree(w->pt.hi);
  w->part = w->tc = w->toff = nullptr;
  w->pt = Partials{nullptr, nullptr, nullptr};
  w->maxtiles = 0;
  WCHK(hipMalloc(&w->part, (need + 1) * sizeof(u32)));
  WCHK(hipMalloc(&w->tc, 3 * need * sizeof(u32)));
  WCHK(hipMalloc(&w->toff, 3 * need * sizeof(u32)));
  WCHK(hipMalloc(&w->pt.cnt, need * sizeof(u32)));
  WCHK(hipMalloc(&w->pt.lo, need * sizeof(u64)));
  WCHK(hipMalloc(&w->pt.hi, need * sizeof(u64)));
  w->maxtiles = (u32)need;
  return 0;
}

int wide_create(WideScratch** out, u32 d) {
  WideScratch* w = new WideScratch;
  w->d = d;
  *out = w;
  WCHK(hipMalloc(&w->ctl, sizeof(Ctl)));
  WCHK(hipMalloc(&w->box, sizeof(Mail)));
  WCHK(hipMemset(w->box, 0, sizeof(Mail)));
  WCHK(hipHostMalloc(&w->mail_h, sizeof(Mail), hipHostMallocMapped | hipHostMallocCoherent));
  std::memset(w->mail_h, 0, sizeof(Mail));
  WCHK(hipHostGetDevicePointer((void**)&w->mail_d, w->mail_h, 0));
  WCHK(hipMalloc(&w->cand_k, CANDMAX * sizeof(u64)));
  WCHK(hipMalloc(&w->cand_v, CANDMAX * sizeof(u32)));
  WCHK(hipMalloc(&w->tmp_k, 4ull * d * sizeof(u64)));
  WCHK(hipMalloc(&w->tmp_v, 4ull * d * sizeof(u32)));
  WCHK(hipMemset(w->ctl, 0, sizeof(Ctl)));
  return wide_reserve(w, 4ull * d);
}

void wide_set_profiling(WideScratch* w, bool on) { w->profile = on; }

void wide_kernel_profile(const WideScratch* w, int kind, WideKernelStat* out) { *out = w->kst[kind]; }

const char* wide_kernel_name(int kind) {
  static const char* const names[WK_COUNT] = {
      "k_merge<true> (merge + DeleteDuplicates, writing pass)",
      "k_merge<false> (merge, counting pass)",
      "k_sel_pass (radix Select pass)",
      "k_sel_collect (Select gather and rank)",
      "k_part<false> (three-way split, counting pass)",
      "k_part<true> (three-way split, writing pass)",
      "k_intake (atomicMin on current keys + marks)",
      "k_bits<false> (mark compaction, counting pass)",
      "k_bits<true> (mark compaction, writing pass)",
      "k_tsort (tile sort of the extracted minima)",
      "k_smerge (merge pass of the extracted minima)",
      "k_delete / k_absent (ids marked absent)",
      "scans, reductions, result publishing",
      "Select passes and gathers that returned at once"};
  return kind >= 0 && kind < WK_COUNT ? names[kind] : nullptr;
}

void wide_destroy(WideScratch* w) {
  if (!w) return;
  (void)hipDeviceSynchronize();
  if (w->ctl) (void)hipFree(w->ctl);
  if (w->box) (void)hipFree(w->box);
  if (w->marks) (void)hipFree(w->marks);
  if (w->mail_h) (void)hipHostFree(w->mail_h);
  if (w->part) (void)hipFree(w->part);
  if (w->tc) (void)hipFree(w->tc);
  if (w->toff) (void)hipFree(w->toff);
  if (w->pt.cnt) (void)hipFree(w->pt.cnt);
  if (w->pt.lo) (void)hipFree(w->pt.lo);
  if (w->pt.hi) (void)hipFree(w->pt.hi);
  if (w->cand_k) (void)hipFree(w->cand_k);
  if (w->cand_v) (void)hipFree(w->cand_v);
  if (w->tmp_k) (void)hipFree(w->tmp_k);
  if (w->tmp_v) (void)hipFree(w->tmp_v);
  for (hipEvent_t e : w->ev) (void)hipEventDestroy(e);
  delete w;
}

// BulkUpdate (Section 2.2): cur[id] = min(cur[id], key) for every pair, the
// ids whose key dropped form U sorted by id; pieces of at most d go into S_0,
// each followed by Resolve(0) and the schedule.
int wide_bulk_update(WideScratch* w, WideHeap* h, const u64* keys, const u32* ids, u64 count) {
  HeapState* st = h->st;
  if (count == 0) return 0;
  // A batch of at most d pairs is one piece: the compaction writes it straight
  // into S_0 (empty between operations).
  const bool direct = count <= h->g.d;
  if (direct)
    if (int rc = grow_if_needed(w, h)) return rc;
  if (int rc = wide_reserve(w, capB(h->g.d, h->g.q - 1))) return rc;
  if (w->marks_n < 32ull * h->nwords) {
    if (w->marks) (void)hipFree(w->marks);
    w->marks = nullptr;
    w->marks_n = 0;
    WCHK(hipMalloc(&w->marks, 32ull * h->nwords));
    WCHK(hipMemsetAsync(w->marks, 0, 32ull * h->nwords, w->s));
    w->marks_n = 32ull * h->nwords;
  }
  const u32 gi = grid_for(count);
  // per pair: the pair (12 B) and the atomicMin on its current key (8 B)
  plaunch(w, WK_INTAKE, 20ull * count, [&] {
    hipLaunchKernelGGL(k_intake, dim3(gi), dim3(NT), 0, w->s, keys, ids, count, h->cur, w->marks, w->pt);
  });
  plaunch(w, WK_OTHER, 4ull * gi, [&] {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, w->s, Partials{w->pt.cnt, nullptr, nullptr}, gi,
                       (u32*)nullptr, &w->box->newly, w->ctl);
  });
  const u32 nt = cdiv(h->nwords, TILE);
  if (nt > w->maxtiles) return E_INTERNAL;
  const Arr S0 = lbuf(h->g, 0, 3);
  u64* uk = direct ? S0.k : h->ukeys;
  u32* uv = direct ? S0.v : h->uids;
  const u64 nmark = 32ull * h->nwords;  // one mark byte per id
  plaunch(w, WK_BITS_COUNT, nmark, [&] {
    hipLaunchKernelGGL(k_bits<false>, dim3(nt), dim3(NT), 0, w->s, w->marks, h->nwords, w->tc, (const u32*)nullptr,
                       (const u64*)h->cur, uk, uv);
  });
  // published by the scan: the count of U is known before the compaction
  const u32 want = ++w->seq;
  plaunch(w, WK_OTHER, 8ull * nt, [&] {
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, w->s, w->tc, nt, 0u, w->toff, &w->box->total, w->ctl,
                       Pub{w->box, w->mail_d, want}, Partials{nullptr, nullptr, nullptr}, (u32*)nullptr);
  });
  const int ib = plaunch(w, WK_BITS_WRITE, nmark, [&] {
    hipLaunchKernelGGL(k_bits<true>, dim3(nt), dim3(NT), 0, w->s, w->marks, h->nwords, (u32*)nullptr, w->toff,
                       (const u64*)h->cur, uk, uv);
  });
  if (int rc = launch_ok()) return rc;
  if (int rc = wait_mail(w, want)) return rc;
  const u64 nu = w->mail_h->total;
  // marks read, plus per output its current key read (8 B) and the pair written (12 B)
  patch_bytes(w, ib, nmark + 20ull * nu);
  st->live += w->mail_h->newly;
  for (u64 c0 = 0; c0 < nu;) {
    if (!direct)
      if (int rc = grow_if_needed(w, h)) return rc;
    const u32 len = (u32)((nu - c0) < h->g.d ? (nu - c0) : h->g.d);
    Arr S = lbuf(h->g, 0, 3);
    if (!direct) {
      WCHK(hipMemcpyAsync(S.k, h->ukeys + c0, len * sizeof(u64), hipMemcpyDeviceToDevice, w->s));
      WCHK(hipMemcpyAsync(S.v, h->uids + c0, len * sizeof(u32), hipMemcpyDeviceToDevice, w->s));
    }
    st->L[0].nS = len;
    st->L[0].ssel = 0;
    if (st->ell < 0) st->ell = 0;
    st->elems += 2ull * len;
    wdrive(w, h, DRIVE_AFTER);
    if (st->err) return st->err;
    c0 += len;
  }
  return prof_collect(w);
}

// Delete (Section 1.2) of a batch of ids: their current keys become absent,
// which every later merge and every move into B_0 treat as a dead copy; B_0
// is filtered at once (it holds only live elements), then Resolve(0) and the
// schedule.
int wide_delete(WideScratch* w, WideHeap* h, const u32* ids, u64 count) {
  HeapState* st = h->st;
  if (count == 0) return 0;
  if (int rc = wide_reserve(w, capB(h->g.d, h->g.q - 1))) return rc;
  const u32 gi = grid_for(count);
  plaunch(w, WK_ABSENT, 12ull * count,
          [&] { hipLaunchKernelGGL(k_delete, dim3(gi), dim3(NT), 0, w->s, ids, count, h->cur, w->pt); });
  plaunch(w, WK_OTHER, 4ull * gi, [&] {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, w->s, Partials{w->pt.cnt, nullptr, nullptr}, gi,
                       (u32*)nullptr, &w->box->newly, w->ctl);
  });
  if (int rc = launch_ok()) return rc;
  const Lvl a0 = st->L[0];
  if (a0.nB) {
    Arr B = lbuf(h->g, 0, a0.bsel), O = lbuf(h->g, 0, a0.bsel ^ 1), X = lbuf(h->g, 0, 2);
    u32 n0, n1, n2;
    if (int rc = wpartition3(w, B, a0.nB, kv_inf(), kv_inf(), O, X, X, h->cur, &n0, &n1, &n2)) return rc;
    st->L[0].bsel ^= 1;
    st->L[0].nB = n0;
    st->elems += (u64)a0.nB + n0;
  } else if (int rc = fetch(w)) {
    return rc;
  }
  st->live -= w->mail_h->newly;
  fix_ell(st, h->g.q);
  if (int rc = grow_if_needed(w, h)) return rc;
  wdrive(w, h, DRIVE_AFTER);
  if (st->err) return st->err;
  return prof_collect(w);
}

// Batched ExtractMin: repeatedly the smallest min(k_left, |B_0|) elements of
// B_0 (B_0 <= p_0 < everything else and holds only live elements) are split
// off, sorted by (key, id), written out and marked absent; then Resolve(0)
// and the schedule.
int wide_extract_min(WideScratch* w, WideHeap* h, u64 k, u64* okeys, u32* oids, u64* count_out) {
  HeapState* st = h->st;
  *count_out = 0;
  u64 out = 0;
  bool pending = false;
  if (int rc = wide_reserve(w, capB(h->g.d, h->g.q - 1))) return rc;
  for (;;) {
    if (!pending && out >= k) break;
    if (int rc = grow_if_needed(w, h)) return rc;
    wdrive(w, h, (pending ? DRIVE_AFTER : 0) | (out < k ? DRIVE_ENSURE : 0));
    pending = false;
    if (st->err) return st->err;
    if (out >= k) break;
    const Lvl a0 = st->L[0];
    if (a0.nB == 0) {
      if (st->ell >= 0) return E_INTERNAL;  // the refill leaves B_0 empty only when the heap is
      break;
    }
    const u32 take = (u32)((k - out) < a0.nB ? (k - out) : a0.nB);
    Arr B = lbuf(h->g, 0, a0.bsel), X = lbuf(h->g, 0, 2);
    KV thr = kv_inf();
    u32 n0, n1, n2;
    if (take < a0.nB) {
      if (int rc = wselpart(w, B, a0.nB, take, false, kv_inf(), kv_inf(), X, lbuf(h->g, 0, a0.bsel ^ 1), X, nullptr,
                            &thr, &n0, &n1, &n2))
        return rc;
    } else if (int rc = wpartition3(w, B, a0.nB, thr, kv_inf(), X, lbuf(h->g, 0, a0.bsel ^ 1), X, nullptr, &n0, &n1,
                                    &n2)) {
      return rc;
    }
    if (n0 != take) return E_INTERNAL;
    if (int rc = wsort(w, X, take, okeys + out, oids + out)) return rc;
    plaunch(w, WK_ABSENT, 12ull * take, [&] {
      hipLaunchKernelGGL(k_absent, dim3(grid_for(take)), dim3(NT), 0, w->s, (const u32*)(oids + out), (u64)take,
                         h->cur);
    });
    if (int rc = launch_ok()) return rc;
    st->L[0].bsel ^= 1;
    st->L[0].nB = n1;
    st->live -= take;
    st->elems += 6ull * a0.nB;
    out += take;
    pending = true;
  }
  WCHK(hipStreamSynchronize(w->s));
  *count_out = out;
  return prof_collect(w);
}

}  // namespace bkt
