// Pattern-based partitioning (Section III.A, Fig. 1b: the patterns split into
// sub-patterns, one state machine each, every machine over the same input).
//
// A k-mer set whose automaton would exceed the device tables (more than 4096
// states), or the three-symbol tables (more than 1023), is split into parts
// whose automata fit a state budget.  The patterns are taken in sorted order,
// so patterns that share prefixes share trie nodes inside a part; a part is
// closed when the next pattern's new prefixes would take its trie (its
// Aho-Corasick automaton) past the budget.  A scan runs every part's ordinary
// pipeline over the same sequence, the parts spread over a few streams of the
// partition's own so that short inputs keep several parts on the GPU at
// once, then one kernel on the caller's stream scatters the parts' counts to
// the global pattern ids and forwards the parts' kept consistency failures
// to the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_set>
#include <vector>

#include "coex.h"
#include "dfa.hpp"

namespace coex {
// coex.hip: the kept failure word of (device, stream) (creating its workspace)
int stream_sticky(int dev, void* stream, uint32_t** out);
}  // namespace coex

namespace {

constexpr uint32_t kPartStreams = 4;  // the hardware queues a process gets by default

// Per-pattern counts of all parts (local order) to the caller's buffer, and
// the parts' streams' kept failures to the caller's stream's word.
__global__ void k_partition_finish(const uint64_t* local, const uint32_t* map, uint32_t n, uint64_t* counts,
                                   uint32_t* e0, uint32_t* e1, uint32_t* e2, uint32_t* e3, uint32_t* dst) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) counts[map[i]] = local[i];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    uint32_t e = 0;
    if (e0) e |= atomicExch(e0, 0u);
    if (e1) e |= atomicExch(e1, 0u);
    if (e2) e |= atomicExch(e2, 0u);
    if (e3) e |= atomicExch(e3, 0u);
    if (e) atomicOr(dst, e);
  }
}

}  // namespace

struct coex_partition {
  std::vector<coex_dfa*> parts;
  std::vector<std::vector<uint32_t>> ids;  // global id of each part's pattern i
  std::vector<uint32_t> offset;            // first local count of each part
  uint32_t n_patterns = 0;
  struct Dev {
    int device = -1;
    uint64_t* local = nullptr;
    uint32_t* map = nullptr;
    std::vector<hipStream_t> st;
    std::vector<hipEvent_t> done;
    hipEvent_t start = nullptr;
  };
  std::deque<Dev> devs;  // stable addresses as devices are added
  std::mutex mu;
  ~coex_partition() {
    for (coex_dfa* d : parts) coex_dfa_free(d);
    int cur = -1;
    (void)hipGetDevice(&cur);
    for (Dev& D : devs) {
      (void)hipSetDevice(D.device);
      for (hipStream_t s : D.st) (void)hipStreamSynchronize(s);
      if (D.local) (void)hipFree(D.local);
      if (D.map) (void)hipFree(D.map);
      for (hipStream_t s : D.st) (void)hipStreamDestroy(s);
      for (hipEvent_t e : D.done) (void)hipEventDestroy(e);
      if (D.start) (void)hipEventDestroy(D.start);
    }
    if (cur >= 0) (void)hipSetDevice(cur);
  }
};

namespace {

// The device side of a partition on `dev`: count buffers, id map, streams.
int device_state(coex_partition& P, int dev, coex_partition::Dev*& out) {
  std::lock_guard<std::mutex> lk(P.mu);
  for (auto& D : P.devs)
    if (D.device == dev) { out = &D; return COEX_OK; }
  coex_partition::Dev D;
  D.device = dev;
  const uint32_t n = std::max<uint32_t>(1, P.n_patterns);
  std::vector<uint32_t> map;
  for (const auto& v : P.ids) map.insert(map.end(), v.begin(), v.end());
  auto fail = [&](int rc) {
    if (D.local) (void)hipFree(D.local);
    if (D.map) (void)hipFree(D.map);
    for (hipStream_t s : D.st) (void)hipStreamDestroy(s);
    for (hipEvent_t e : D.done) (void)hipEventDestroy(e);
    if (D.start) (void)hipEventDestroy(D.start);
    return rc;
  };
  if (hipMalloc(&D.local, (size_t)n * 8) != hipSuccess) { D.local = nullptr; return fail(COEX_ENOMEM); }
  if (hipMalloc(&D.map, (size_t)n * 4) != hipSuccess) { D.map = nullptr; return fail(COEX_ENOMEM); }
  if (!map.empty() && hipMemcpy(D.map, map.data(), map.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
    return fail(COEX_EDEVICE);
  const uint32_t ns = std::min<uint32_t>(kPartStreams, std::max<uint32_t>(1, (uint32_t)P.parts.size()));
  for (uint32_t i = 0; i < ns; ++i) {
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return fail(COEX_EDEVICE);
    D.st.push_back(s);
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return fail(COEX_EDEVICE);
    D.done.push_back(e);
  }
  if (hipEventCreateWithFlags(&D.start, hipEventDisableTiming) != hipSuccess) return fail(COEX_EDEVICE);
  P.devs.push_back(D);
  out = &P.devs.back();
  return COEX_OK;
}

}  // namespace

extern "C" {

int coex_partition_kmers(const char* const* kmers, uint32_t n, uint32_t max_states, coex_partition** out) {
  if (!kmers || n == 0 || !out) return COEX_EINVAL;
  if (max_states == 0) max_states = coex::kMaxStatesStep3;
  if (max_states < 2 || max_states > coex::kMaxStates) return COEX_EINVAL;
  try {
    auto P = std::make_unique<coex_partition>();
    P->n_patterns = n;
    std::vector<uint32_t> order(n);
    for (uint32_t i = 0; i < n; ++i) {
      if (!kmers[i] || !kmers[i][0]) return COEX_EINVAL;
      order[i] = i;
    }
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t a, uint32_t b) { return std::string(kmers[a]) < std::string(kmers[b]); });
    // greedy parts: trie nodes (automaton states less the root) within budget
    std::unordered_set<std::string> prefixes;
    std::vector<uint32_t> cur;
    auto fresh = [&](const std::string& w) {
      uint32_t k = 0;
      for (size_t l = 1; l <= w.size(); ++l) k += prefixes.count(w.substr(0, l)) ? 0u : 1u;
      return k;
    };
    uint64_t nodes = 0;
    for (uint32_t id : order) {
      const std::string w(kmers[id]);
      uint32_t add = fresh(w);
      if (!cur.empty() && nodes + add + 1 > max_states) {
        P->ids.push_back(cur);
        cur.clear();
        prefixes.clear();
        nodes = 0;
        add = fresh(w);
      }
      if (add + 1 > max_states) return COEX_ETOOBIG;  // one pattern alone is past the budget
      for (size_t l = 1; l <= w.size(); ++l) prefixes.insert(w.substr(0, l));
      nodes += add;
      cur.push_back(id);
    }
    if (!cur.empty()) P->ids.push_back(cur);
    uint32_t off = 0;
    for (const auto& v : P->ids) {
      std::vector<const char*> ks;
      for (uint32_t id : v) ks.push_back(kmers[id]);
      coex_dfa* d = nullptr;
      const int rc = coex_compile_kmers(ks.data(), (uint32_t)ks.size(), &d);
      if (rc) return rc;
      P->parts.push_back(d);
      P->offset.push_back(off);
      off += (uint32_t)v.size();
    }
    *out = P.release();
    return COEX_OK;
  } catch (const std::bad_alloc&) {
    return COEX_ENOMEM;
  } catch (...) {
    return COEX_EINTERNAL;
  }
}

int coex_partition_info(const coex_partition* p, uint32_t* n_parts, uint32_t* n_patterns) {
  if (!p) return COEX_EINVAL;
  if (n_parts) *n_parts = (uint32_t)p->parts.size();
  if (n_patterns) *n_patterns = p->n_patterns;
  return COEX_OK;
}

int coex_partition_part(const coex_partition* p, uint32_t i, const coex_dfa** dfa, const uint32_t** ids,
                        uint32_t* n) {
  if (!p || i >= p->parts.size()) return COEX_EINVAL;
  if (dfa) *dfa = p->parts[i];
  if (ids) *ids = p->ids[i].data();
  if (n) *n = (uint32_t)p->ids[i].size();
  return COEX_OK;
}

int coex_count_partitioned(coex_partition* p, const coex_seq* seq, uint64_t* counts_dev, const coex_opts* opts,
                           void* stream) {
  if (!p || !seq || !counts_dev) return COEX_EINVAL;
  try {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return COEX_EDEVICE;
    coex_partition::Dev* D = nullptr;
    int rc = device_state(*p, dev, D);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (hipEventRecord(D->start, st) != hipSuccess) return COEX_EDEVICE;
    for (hipStream_t s : D->st)
      if (hipStreamWaitEvent(s, D->start, 0) != hipSuccess) return COEX_EDEVICE;
    for (size_t j = 0; j < p->parts.size(); ++j) {
      rc = coex_count(p->parts[j], seq, D->local + p->offset[j], opts, D->st[j % D->st.size()]);
      if (rc) return rc;
    }
    uint32_t* e[kPartStreams] = {nullptr, nullptr, nullptr, nullptr};
    for (size_t i = 0; i < D->st.size(); ++i) {
      if (hipEventRecord(D->done[i], D->st[i]) != hipSuccess) return COEX_EDEVICE;
      if (hipStreamWaitEvent(st, D->done[i], 0) != hipSuccess) return COEX_EDEVICE;
      rc = coex::stream_sticky(dev, D->st[i], &e[i]);
      if (rc) return rc;
    }
    uint32_t* dst = nullptr;
    rc = coex::stream_sticky(dev, stream, &dst);
    if (rc) return rc;
    const uint32_t blocks = std::min<uint32_t>(1024, (p->n_patterns + 255) / 256);
    hipLaunchKernelGGL(k_partition_finish, dim3(std::max(1u, blocks)), dim3(256), 0, st, D->local, D->map,
                       p->n_patterns, counts_dev, e[0], e[1], e[2], e[3], dst);
    if (hipGetLastError() != hipSuccess) return COEX_EDEVICE;
    return COEX_OK;
  } catch (const std::bad_alloc&) {
    return COEX_ENOMEM;
  } catch (...) {
    return COEX_EINTERNAL;
  }
}

void coex_partition_free(coex_partition* p) { delete p; }

}  // extern "C"
