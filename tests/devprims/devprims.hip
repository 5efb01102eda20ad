// GPU unit tests of the team primitives of pbh_core.h (tests only): each
// kernel runs one primitive with one team on device arrays given by the test.
#include "../../paper_1908_09378_amd/csrc/pbh_core.h"

using namespace bkt;

struct DP {
  using L = ArrT<u64 PBH_LDS*, u32 PBH_LDS*>;
  using G = ArrT<u64 PBH_GLB*, u32 PBH_GLB*>;
  using SP = HeapState PBH_LDS*;
};
using GA = DP::G;

template <int NT>
__global__ __launch_bounds__(NT) void k_prim(int op, u64* ak, u32* av, u32 na, u64* bk, u32* bv, u32 nb,
                                             u64* ck, u32* cv, u64* c2k, u32* c2v, u64* c3k, u32* c3v,
                                             const u64* cur, u64* res) {
  __shared__ TeamShared<NT / 64> ts;
  DevTeam<NT> t{(TeamShared<NT / 64> PBH_LDS*)&ts};
  GA A{(u64 PBH_GLB*)ak, (u32 PBH_GLB*)av}, B{(u64 PBH_GLB*)bk, (u32 PBH_GLB*)bv};
  GA C{(u64 PBH_GLB*)ck, (u32 PBH_GLB*)cv}, C2{(u64 PBH_GLB*)c2k, (u32 PBH_GLB*)c2v},
      C3{(u64 PBH_GLB*)c3k, (u32 PBH_GLB*)c3v};
  if (op == 0) {  // exclusive scan of av[0..na) (one value per thread, tiles of NT)
    u32 run = 0;
    for (u32 b = 0; b < na; b += NT) {
      u32 x = b + threadIdx.x;
      u32 tot;
      u32 e = t.scan_excl(x < na ? av[x] : 0u, &tot);
      if (x < na) cv[x] = run + e;
      run += tot;
    }
    if (threadIdx.x == 0) res[0] = run;
  } else if (op == 1) {  // team min (key, id) and min/max key
    u64 mk = KINF, lo = KINF, hi = 0;
    u32 mv = VINF;
    for (u32 x = threadIdx.x; x < na; x += NT) {
      u64 k = ak[x];
      u32 v = av[x];
      if (k < mk || (k == mk && v < mv)) {
        mk = k;
        mv = v;
      }
      lo = k < lo ? k : lo;
      hi = k > hi ? k : hi;
    }
    t.minkv(mk, mv);
    t.minmax64(lo, hi);
    if (threadIdx.x == 0) {
      res[0] = mk;
      res[1] = mv;
      res[2] = lo;
      res[3] = hi;
    }
  } else if (op == 2) {  // merge + dedup
    u32 m = merge_dedup(t, A, na, B, nb, C, cur, cur != nullptr);
    if (threadIdx.x == 0) res[0] = m;
  } else if (op == 3) {  // partition3 by res[0..3] = (p1k, p1v, p2k, p2v)
    KV p1{res[0], (u32)res[1]}, p2{res[2], (u32)res[3]};
    t.sync();
    u32 n0, n1, n2;
    partition3(t, A, na, p1, p2, C, C2, C3, &n0, &n1, &n2);
    if (threadIdx.x == 0) {
      res[4] = n0;
      res[5] = n1;
      res[6] = n2;
    }
  } else if (op == 4) {  // select r = nb
    KV s = select_kth(t, A, na, nb);
    if (threadIdx.x == 0) {
      res[0] = s.k;
      res[1] = s.v;
    }
  } else if (op == 5) {  // sort by (key, id) with B as temporary, idbits = res[0]
    bool in_tmp = sort_kv(t, A, B, na, (int)res[0]);
    if (threadIdx.x == 0) res[1] = in_tmp;
  }
}

extern "C" int dp_run(int nt, int op, u64* ak, u32* av, u32 na, u64* bk, u32* bv, u32 nb, u64* ck, u32* cv,
                      u64* c2k, u32* c2v, u64* c3k, u32* c3v, const u64* cur, u64* res) {
  switch (nt) {
    case 64:
      hipLaunchKernelGGL(k_prim<64>, dim3(1), dim3(64), 0, 0, op, ak, av, na, bk, bv, nb, ck, cv, c2k, c2v, c3k,
                         c3v, cur, res);
      break;
    case 256:
      hipLaunchKernelGGL(k_prim<256>, dim3(1), dim3(256), 0, 0, op, ak, av, na, bk, bv, nb, ck, cv, c2k, c2v,
                         c3k, c3v, cur, res);
      break;
    case 1024:
      hipLaunchKernelGGL(k_prim<1024>, dim3(1), dim3(1024), 0, 0, op, ak, av, na, bk, bv, nb, ck, cv, c2k, c2v,
                         c3k, c3v, cur, res);
      break;
    default:
      return -1;
  }
  if (hipGetLastError() != hipSuccess) return -2;
  return hipDeviceSynchronize() == hipSuccess ? 0 : -3;
}
