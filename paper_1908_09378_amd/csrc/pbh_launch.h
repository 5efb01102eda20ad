// Host-side interface between the C ABI (abi.hip) and the kernels (kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "pbh_core.h"

namespace bkt {

// Device statistics block written by the SSSP kernel.
struct SsspDevStats {
  u64 rounds, relax, updates, elems, extracted, last_key;
  long long err;
  long long ell;
  u64 resolves[MAXL];
  u64 prof[PROF_N];  // time accounting of a profiled run (HeapState::prof)
};

struct SsspParams {
  const u64* off;
  const u32* tg;
  const u32* wt;
  u64* dist;
  u32 n;
  u32 src;
  int sched;
  Geom g;  // lk/lv are set inside the kernel
  SsspDevStats* stats;
  SpecCfg spec;
  u32 prof;  // time accounting on (single queries only)
  // deep-level workers: levels >= deep_lim each have a workgroup of their own
  // (blocks 1 .. q - deep_lim of a cooperative launch); null = none
  DeepCtl* deep;
  int deep_lim;
  // bytes of LDS staging for merges of HBM levels, after the LDS levels in
  // the dynamic block (the round loop) or at its start (workers); 0 = none
  u32 stage;
  // 1: the large-heap form of the round loop (k_sssp_full: staging, deep
  // workers when `deep` is set); 0: the plain one-workgroup form (k_sssp)
  u32 full;
};


struct CsrCheck {
  u64 bad;        // any malformed entry
  u64 maxdeg;
};

hipError_t launch_fill_dist(u64* dist, u32 n, u32 src, hipStream_t s);
hipError_t launch_zero_u64(u64* p, u64 n, hipStream_t s);
hipError_t launch_check_csr(const u64* off, const u32* tg, u32 n, u64 m, CsrCheck* out, hipStream_t s);
hipError_t launch_sssp(int team, const SsspParams& p, size_t lds_bytes, hipStream_t s);
hipError_t launch_sssp_full(int team, const SsspParams& p, size_t lds_bytes, hipStream_t s);
size_t sssp_static_lds(int team);
hipError_t launch_sssp_multi(int team, const SsspParams* qs, u32 nq, u32* counter, size_t lds, int grid,
                             hipStream_t s);
hipError_t launch_fill_multi(const SsspParams* qs, u32 nq, u32 maxn, u32* counter, hipStream_t s);
int multi_occupancy(int team, size_t lds);
hipError_t launch_pbh_update(const PbhParams& p, hipStream_t s);
hipError_t launch_pbh_extract(const PbhParams& p, hipStream_t s);
hipError_t launch_pbh_delete(const PbhParams& p, hipStream_t s);
hipError_t launch_mlp_infer(int team, const float* X, u32 n, const float* blob, float* y, hipStream_t s);
// keys may be NULL (a delete batch: ids only).
hipError_t launch_check_update(const u64* keys, const u32* ids, u64 count, u32 id_cap, u64* bad,
                               hipStream_t s);

}  // namespace bkt
