// Oracle: plain, slow, obviously-correct CPU reference for the parallel bucket
// heap's priority-queue semantics and for the shortest-path distances that
// parDijkstra computes.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library includes, links or
// calls this file; only tests, the smoke check and the CPU-baseline leg of the
// benchmark load it.  It shares no code with the HIP path.
//
// Contents
//   * opq_*       : the priority-queue ADT of Section 1.2 (extractMin / update /
//                   delete, plus BulkUpdate = update for every element of a
//                   batch) as a sorted multiset std::set<(key, id)> plus cur[id].
//                   Readings of the paper:
//                     - an update whose key is not smaller than the id's current
//                       key is a no-op (the paper assumes updates only decrease
//                       priority, footnote in Section 1.2; duplicate resolution
//                       in Section 2.1 keeps the smaller priority), an update of
//                       an absent id inserts it;
//                     - ties in priority are broken by id, so the order is the
//                       total order on (key, id);
//                     - a batched extract of k returns the min(k, size) smallest
//                       elements in ascending order, i.e. k successive
//                       extractMins with no update in between;
//                     - delete(id) removes the element with that id if the
//                       queue holds it and is a no-op otherwise (Section 1.2);
//                       a batch of deletes is one delete per listed id.
//   * odijkstra   : Dijkstra's algorithm (Section 1.1) with a binary heap and
//                   lazy deletion, uint64 distances, UINT64_MAX = unreached,
//                   relaxation on strictly shorter distance.  Also reports the
//                   order in which vertices are settled, which is ascending
//                   (dist, id).
//   * obellman_ford : Bellman-Ford (Section 1.1): repeat relaxing every edge
//                   until nothing changes.  Brute force for tiny graphs.
//
// All functions validate their arguments and return negative numbers on bad
// input instead of aborting.
#include <cstdint>
#include <cstring>
#include <functional>
#include <queue>
#include <set>
#include <utility>
#include <vector>

namespace {

constexpr uint64_t kInf = UINT64_MAX;

struct Pq {
  std::vector<uint64_t> cur;                      // current key of each id, kInf = absent
  std::set<std::pair<uint64_t, uint32_t>> items;  // live (key, id) pairs
};

}  // namespace

extern "C" {

void* opq_create(uint32_t id_capacity) {
  Pq* q = new Pq;
  q->cur.assign(id_capacity, kInf);
  return q;
}

void opq_destroy(void* h) { delete static_cast<Pq*>(h); }

// Update(e) for every e in the batch, in order.  Returns the number of
// elements whose key changed (inserted or decreased), or -1 on bad input
// (id out of range or key == UINT64_MAX, which is reserved for "absent");
// on bad input nothing is modified.
int64_t opq_bulk_update(void* h, const uint64_t* keys, const uint32_t* ids, uint64_t count) {
  Pq* q = static_cast<Pq*>(h);
  for (uint64_t i = 0; i < count; ++i)
    if (ids[i] >= q->cur.size() || keys[i] == kInf) return -1;
  int64_t changed = 0;
  for (uint64_t i = 0; i < count; ++i) {
    uint32_t id = ids[i];
    uint64_t k = keys[i];
    if (k < q->cur[id]) {
      if (q->cur[id] != kInf) q->items.erase({q->cur[id], id});
      q->items.insert({k, id});
      q->cur[id] = k;
      ++changed;
    }
  }
  return changed;
}

// Delete(e) for every id of the batch: the element with that id leaves the
// queue if it is there.  Returns the number removed, or -1 on bad input (an
// id out of range; nothing is modified then).
int64_t opq_delete(void* h, const uint32_t* ids, uint64_t count) {
  Pq* q = static_cast<Pq*>(h);
  for (uint64_t i = 0; i < count; ++i)
    if (ids[i] >= q->cur.size()) return -1;
  int64_t removed = 0;
  for (uint64_t i = 0; i < count; ++i) {
    uint32_t id = ids[i];
    if (q->cur[id] == kInf) continue;
    q->items.erase({q->cur[id], id});
    q->cur[id] = kInf;
    ++removed;
  }
  return removed;
}

// Removes and returns the min(k, size) smallest (key, id), ascending.
uint64_t opq_extract_min(void* h, uint64_t k, uint64_t* keys_out, uint32_t* ids_out) {
  Pq* q = static_cast<Pq*>(h);
  uint64_t n = 0;
  while (n < k && !q->items.empty()) {
    auto it = q->items.begin();
    keys_out[n] = it->first;
    ids_out[n] = it->second;
    q->cur[it->second] = kInf;
    q->items.erase(it);
    ++n;
  }
  return n;
}

uint64_t opq_size(void* h) { return static_cast<Pq*>(h)->items.size(); }

// Copies cur[] (kInf for absent ids) into out[id_capacity].
void opq_cur(void* h, uint64_t* out) {
  Pq* q = static_cast<Pq*>(h);
  std::memcpy(out, q->cur.data(), q->cur.size() * sizeof(uint64_t));
}

// Checks a CSR graph: offsets[0]==0, non-decreasing, offsets[n]==m, targets < n.
static int csr_ok(const uint64_t* off, const uint32_t* tg, uint32_t n, uint64_t m) {
  if (n == 0 || off[0] != 0 || off[n] != m) return 0;
  for (uint32_t u = 0; u < n; ++u)
    if (off[u + 1] < off[u]) return 0;
  for (uint64_t e = 0; e < m; ++e)
    if (tg[e] >= n) return 0;
  return 1;
}

// Dijkstra from src.  dist[n] receives the distances (kInf = unreachable).
// If order != nullptr it receives the settled vertices in settle order and
// *nsettled their count.  *nrelax (if non-null) receives the number of edges
// scanned (sum of out-degrees of settled vertices).  Returns 0, or -1 on bad
// input.
int odijkstra(const uint64_t* off, const uint32_t* tg, const uint32_t* w, uint32_t n, uint64_t m,
              uint32_t src, uint64_t* dist, uint32_t* order, uint64_t* nsettled, uint64_t* nrelax) {
  if (!csr_ok(off, tg, n, m) || src >= n) return -1;
  for (uint32_t v = 0; v < n; ++v) dist[v] = kInf;
  std::vector<char> done(n, 0);
  using Item = std::pair<uint64_t, uint32_t>;
  std::priority_queue<Item, std::vector<Item>, std::greater<Item>> pq;
  dist[src] = 0;
  pq.push({0, src});
  uint64_t settled = 0, relax = 0;
  while (!pq.empty()) {
    Item top = pq.top();
    pq.pop();
    uint32_t u = top.second;
    if (done[u] || top.first != dist[u]) continue;  // stale entry
    done[u] = 1;
    if (order) order[settled] = u;
    ++settled;
    for (uint64_t e = off[u]; e < off[u + 1]; ++e) {
      ++relax;
      uint32_t v = tg[e];
      uint64_t cand = dist[u] + w[e];
      if (cand < dist[v]) {
        dist[v] = cand;
        pq.push({cand, v});
      }
    }
  }
  if (nsettled) *nsettled = settled;
  if (nrelax) *nrelax = relax;
  return 0;
}

// Bellman-Ford from src: sweep all edges until no distance changes (at most n
// sweeps since weights are non-negative).  Returns the number of sweeps, or -1
// on bad input.
int64_t obellman_ford(const uint64_t* off, const uint32_t* tg, const uint32_t* w, uint32_t n, uint64_t m,
                      uint32_t src, uint64_t* dist) {
  if (!csr_ok(off, tg, n, m) || src >= n) return -1;
  for (uint32_t v = 0; v < n; ++v) dist[v] = kInf;
  dist[src] = 0;
  int64_t sweeps = 0;
  bool changed = true;
  while (changed) {
    changed = false;
    ++sweeps;
    for (uint32_t u = 0; u < n; ++u) {
      if (dist[u] == kInf) continue;
      for (uint64_t e = off[u]; e < off[u + 1]; ++e) {
        uint64_t cand = dist[u] + w[e];
        if (cand < dist[tg[e]]) {
          dist[tg[e]] = cand;
          changed = true;
        }
      }
    }
    if (sweeps > (int64_t)n + 1) return -2;  // cannot happen with non-negative weights
  }
  return sweeps;
}

}  // extern "C"
