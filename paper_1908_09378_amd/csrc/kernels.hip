// Kernels of the parallel bucket heap and parDijkstra for gfx950.
//
//  k_sssp          one workgroup (one team) runs all parDijkstra rounds; the
//                  small top levels of the heap live in its LDS, deeper
//                  levels in HBM.  One kernel per query: no host round trip
//                  per round.  Two instantiations: every k rule, or the
//                  plain rule only (lighter).  (The large-heap form with
//                  deep-level workers and the batched launch are in
//                  kernels_full.hip.)
//  k_pbh_update    BulkUpdate of a host call (current keys + id bitmap,
//                  then pieces of at most d into S_0, each followed by
//                  Resolve(0) and the schedule).
//  k_pbh_extract   batched ExtractMin of a host call.
//  k_pbh_delete    Delete of a batch of ids of a host call.
//  k_fill_dist, k_check_csr, k_check_update: grid-wide helpers.
#include "round_loop.h"

namespace bkt {

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

// One query, one workgroup: the plain form of the round loop, with every k
// rule (k_sssp) or the plain rule only (k_sssp_plain, lighter).
template <int NT, bool SPEC>
__global__ __launch_bounds__(NT) void k_sssp(SsspParams p) {
  extern __shared__ __align__(16) unsigned char dyn[];
  __shared__ TeamShared<NT / 64> ts;
  __shared__ HeapState st_lds;
  DevTeam<NT> t{(TeamShared<NT / 64> PBH_LDS*)&ts};
  sssp_query<NT, false, SPEC>(t, (HeapState PBH_LDS*)&st_lds, dyn, p);
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

template <int NT, bool SPEC>
static hipError_t sssp_go(const SsspParams& p, size_t lds, hipStream_t s) {
  if (lds > 65536 - sssp_static_lds(NT)) {
    hipError_t e =
        hipFuncSetAttribute((const void*)k_sssp<NT, SPEC>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_sssp<NT, SPEC>), dim3(1), dim3(NT), lds, s, p);
  return hipGetLastError();
}

hipError_t launch_fill_multi(const SsspParams* qs, u32 nq, u32 maxn, u32* counter, hipStream_t s) {
  u32 bx = (maxn + 255) / 256;
  bx = bx < 1 ? 1 : (bx > 1024 ? 1024 : bx);
  hipLaunchKernelGGL(k_fill_multi, dim3(bx, nq > 0 ? nq : 1), dim3(256), 0, s, qs, nq, counter);
  return hipGetLastError();
}

hipError_t launch_sssp(int team, const SsspParams& p, size_t lds_bytes, hipStream_t s) {
  if (p.full) return launch_sssp_full(team, p, lds_bytes, s);
  const bool spec = p.spec.rule != 0 || p.spec.trace_f;
  switch (team) {
    case 64: return spec ? sssp_go<64, true>(p, lds_bytes, s) : sssp_go<64, false>(p, lds_bytes, s);
    case 256: return spec ? sssp_go<256, true>(p, lds_bytes, s) : sssp_go<256, false>(p, lds_bytes, s);
    case 1024: return spec ? sssp_go<1024, true>(p, lds_bytes, s) : sssp_go<1024, false>(p, lds_bytes, s);
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
