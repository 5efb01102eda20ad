// Device-wide engine of the parallel bucket heap, for large bulk sizes d.
//
// With d in the hundreds of thousands, one Resolve moves tens of megabytes,
// which a single workgroup cannot stream at HBM speed.  This engine runs every
// step of Algorithm 1 (Merge with DeleteDuplicates, Select, the splits) as a
// grid-wide kernel over the whole device, and the host runs Resolve's control
// flow and the schedule (drive_with, shared with the one-workgroup kernels),
// reading back the few sizes each step produces.  The heap state (sizes,
// pivots, buffer selectors) lives on the host; the arrays live in the same
// level arena as the one-workgroup engine's.
#pragma once
#include <hip/hip_runtime.h>

#include "pbh_core.h"

namespace bkt {

struct WideScratch;

// What the engine needs from a heap handle.  `grow` adds one level to the
// arena (existing levels keep their offsets) and refreshes `g`.
struct WideHeap {
  Geom g;
  HeapState* st;  // host-side state, authoritative for this engine
  u64* cur;       // device: current key of every id (KINF = absent)
  u32 nwords;     // id capacity / 32, rounded up
  int sched;
  u64* ukeys;     // device: room for min(count, id_capacity) update pairs
  u32* uids;
  int (*grow)(void* ctx, Geom* g);
  void* ctx;
};

// Error codes: 0, E_CAPACITY, E_INTERNAL, E_DEVICE for a failed HIP call, or
// E_TIMEOUT for a step whose kernels ended without publishing its results.
constexpr int E_DEVICE = -4;

int wide_create(WideScratch** out, u32 d);
void wide_destroy(WideScratch* w);
// Makes room for arrays of up to `elems` elements (called after growth).
int wide_reserve(WideScratch* w, u64 elems);

// BulkUpdate of `count` pairs (device arrays, already validated).
int wide_bulk_update(WideScratch* w, WideHeap* h, const u64* keys, const u32* ids, u64 count);
// Delete of `count` ids (device array, already validated).
int wide_delete(WideScratch* w, WideHeap* h, const u32* ids, u64 count);
// Batched ExtractMin of up to k elements into device arrays okeys/oids,
// ascending by (key, id); *count_out = number written.
int wide_extract_min(WideScratch* w, WideHeap* h, u64 k, u64* okeys, u32* oids, u64* count_out);

// Kernel kinds of the engine, for profiling.
enum {
  WK_MERGE_WRITE, WK_MERGE_COUNT, WK_SEL_PASS, WK_SEL_GATHER, WK_SPLIT_COUNT, WK_SPLIT_WRITE, WK_INTAKE,
  WK_BITS_COUNT, WK_BITS_WRITE, WK_SORT_TILE, WK_SORT_MERGE, WK_ABSENT, WK_OTHER, WK_IDLE, WK_COUNT
};
struct WideKernelStat {
  u64 launches;
  u64 bytes;  // algorithmic bytes of those launches
  double ms;  // summed HIP-event time
};
// Totals per kernel kind over the launches timed so far (only launches made
// while profiling is on are timed: the events cost each launch some
// microseconds of host time).
void wide_kernel_profile(const WideScratch* w, int kind, WideKernelStat* out);
const char* wide_kernel_name(int kind);  // nullptr past the last kind
void wide_set_profiling(WideScratch* w, bool on);

}  // namespace bkt
