// The large-heap form of the parDijkstra round loop for gfx950.
//
//  k_sssp_full     one query: block 0 runs the rounds, with HBM levels merged
//                  through the LDS staging area; with deep-level workers,
//                  block b >= 1 resolves level deep_lim + b - 1 (one
//                  cooperative launch).
//  k_sssp_multi    many independent queries in one persistent launch.
#include "round_loop.h"

namespace bkt {

// Block 0 runs the rounds; with deep-level workers, block b >= 1 is the
// worker of level deep_lim + b - 1.
template <int NT>
__global__ __launch_bounds__(NT) void k_sssp_full(SsspParams p) {
  extern __shared__ __align__(16) unsigned char dyn[];
  __shared__ TeamShared<NT / 64> ts;
  __shared__ HeapState st_lds;
  DevTeam<NT, true> t{(TeamShared<NT / 64> PBH_LDS*)&ts};
  if (blockIdx.x == 0)
    sssp_query<NT, true>(t, (HeapState PBH_LDS*)&st_lds, dyn, p);
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
  DevTeam<NT, true> t{(TeamShared<NT / 64> PBH_LDS*)&ts};
  for (;;) {
    if (threadIdx.x == 0) qnext = atomicAdd(counter, 1u);
    t.sync();
    const u32 qi = qnext;
    t.sync();
    if (qi >= nq) break;
    const SsspParams p = qs[qi];
    sssp_query<NT, true>(t, (HeapState PBH_LDS*)&st_lds, dyn, p);
  }
}

template <int NT>
static hipError_t full_go(const SsspParams& p, size_t lds, hipStream_t s) {
  if (lds > 65536 - sssp_static_lds(NT)) {
    hipError_t e =
        hipFuncSetAttribute((const void*)k_sssp_full<NT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  // the round loop and one workgroup per worker level, resident together
  SsspParams a = p;
  void* args[] = {&a};
  const u32 grid = 1u + (p.deep ? (u32)(p.g.q - p.deep_lim) : 0u);
  return hipLaunchCooperativeKernel((const void*)k_sssp_full<NT>, dim3(grid), dim3(NT), args, lds, s);
}

hipError_t launch_sssp_full(int team, const SsspParams& p, size_t lds_bytes, hipStream_t s) {
  switch (team) {
    case 64: return full_go<64>(p, lds_bytes, s);
    case 256: return full_go<256>(p, lds_bytes, s);
    case 1024: return full_go<1024>(p, lds_bytes, s);
    default: return hipErrorInvalidValue;
  }
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

}  // namespace bkt
