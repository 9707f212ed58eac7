// Batched FastFCA-AS over many mixtures of uneven size (C ABI, declared in
// include/fastfca.h).  Each mixture is an ordinary context; mixtures of equal
// (I, J) form a group that advances in one launch of k_as_resident_batch over
// a table of (mixture, bin) tiles sorted by decreasing N (one workgroup per
// tile, or with the "queue" option persistent workgroups that take tiles
// from a device counter).  One batch step (all
// group launches) is captured once per iteration count into a HIP graph and
// replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "fca_internal.h"

using fca::DevState;
using fca::KernelSet;

namespace {

struct Group {
  int I, J;
  const KernelSet* ks;
  std::vector<int> members;  // mixture indices
  int n_max;                 // largest N of the members
  int ntiles;
  int waves;                 // 0: the members use the streaming kernels
  DevState* d_states;        // device copies of the members' DevState
  int2* d_tiles;             // (member slot, bin), sorted by decreasing N
  int* d_counter;            // the work queue's next tile ("queue" option)
  mutable int queued;        // the last launch took the work-queue form
};

thread_local std::string g_batch_init_error;

}  // namespace

// Groups run side by side on up to kLanes streams of their own (default
// priority), forked from and joined back into the caller's stream, so that
// the workgroups of one (I, J) group fill the CUs that another group's tail
// leaves idle.  Under graph capture the fork and join become the graph's
// dependencies.
constexpr int kLanes = 3;  // with the caller's stream, the four hardware queues of a process

struct fca_batch {
  hipStream_t stream;
  int nlanes;                      // streams in use (1: everything on `stream`)
  hipStream_t lane[kLanes];
  hipEvent_t fork;
  hipEvent_t join[kLanes];
  std::vector<int> order;          // groups by decreasing estimated work
  std::vector<fca_ctx*> ctx;
  std::vector<Group> groups;
  void* dev;  // one allocation for all group tables
  int use_graph;
  int use_queue;  // 1: persistent workgroups take tiles from a device counter
  int autotune;
  int forced_waves;
  bool tuned;
  std::map<int, hipGraphExec_t> graphs;  // per iteration count
  std::string err;
};

namespace {

fca_status bfail(fca_batch* b, fca_status st, const std::string& msg) {
  if (b) b->err = msg; else g_batch_init_error = msg;
  return st;
}

fca_status bhip(fca_batch* b, hipError_t e, const char* where) {
  return bfail(b, FCA_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

hipError_t launch_group(fca_batch* b, const Group& g, int waves, int n_iter, hipStream_t st) {
  if (waves == 0) {
    for (int m : g.members)
      for (int it = 0; it < n_iter; ++it) {
        hipError_t e = g.ks->as_iter_stream(b->ctx[m]->s, st);
        if (e != hipSuccess) return e;
      }
    return hipSuccess;
  }
  bool general = false;  // any member with K > 1 or another P update
  for (int m : g.members) general = general || b->ctx[m]->s.K > 1 || b->ctx[m]->s.p_update != 0;
  for (int done = 0; done < n_iter;) {
    const int step = (n_iter - done) > 1024 ? 1024 : (n_iter - done);
    hipError_t e = g.ks->as_batch_resident(g.d_states, g.d_tiles, g.ntiles, g.n_max, st, step, waves, general,
                                           b->use_queue ? g.d_counter : nullptr, &g.queued);
    if (e != hipSuccess) return e;
    done += step;
  }
  return hipSuccess;
}

hipError_t save_restore(fca_batch* b, const Group& g, bool save) {
  for (int m : g.members) {
    hipError_t e = fca::copy_state(b->ctx[m], save);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Per group: the waves per workgroup (or the streaming kernels) with the
// smallest marginal cost per iteration, measured like the per-context tuner.
fca_status tune(fca_batch* b) {
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) return bhip(b, e, "batch tuner events");
  for (Group& g : b->groups) {
    std::vector<int> cands;
    const bool k_ok = !(g.I > fca::kResMaxIK && b->ctx[g.members[0]]->s.K > 1);
    for (int w : {1, 2, 4})
      if (k_ok && g.ks->as_resident_fits(g.n_max, w, 1) && (b->forced_waves == 0 || b->forced_waves == w))
        cands.push_back(w);
    if (cands.empty()) { g.waves = 0; continue; }
    if (cands.size() == 1 || !b->autotune) { g.waves = cands[0]; continue; }
    long long points = 0;
    for (int m : g.members) points += (long long)b->ctx[m]->F * b->ctx[m]->N;
    const std::string disk_key = fca::tune_key_prefix() + " batch I=" + std::to_string(g.I) +
                                 " J=" + std::to_string(g.J) + " tiles=" + std::to_string(g.ntiles) +
                                 " nmax=" + std::to_string(g.n_max) + " points=" + std::to_string(points) +
                                 " K=" + std::to_string(b->ctx[g.members[0]]->s.K) +
                                 " forced=" + std::to_string(b->forced_waves);
    int cw = 0, unused = 0;
    if (fca::tune_cache_get(disk_key, &cw, &unused) && std::find(cands.begin(), cands.end(), cw) != cands.end()) {
      g.waves = cw;
      continue;
    }
    if ((e = save_restore(b, g, true)) != hipSuccess) break;
    float best = 1e30f;
    int best_w = cands[0];
    const int n1 = 4, n2 = 16;
    for (int w : cands) {
      float t[2] = {1e30f, 1e30f};
      for (int len = 0; len < 2 && e == hipSuccess; ++len)
        for (int trial = 0; trial < 2 && e == hipSuccess; ++trial) {
          if ((e = save_restore(b, g, false)) != hipSuccess) break;
          if ((e = hipEventRecord(e0, b->stream)) != hipSuccess) break;
          if ((e = launch_group(b, g, w, len ? n1 + n2 : n1, b->stream)) != hipSuccess) break;
          if ((e = hipEventRecord(e1, b->stream)) != hipSuccess) break;
          if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
          float ms = 0.f;
          if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
          t[len] = std::min(t[len], ms);
        }
      if (e != hipSuccess) break;
      const float per = std::max(0.f, (t[1] - t[0]) / n2);
      const float cost = t[0] - n1 * per + 30 * per;
      if (cost < best) { best = cost; best_w = w; }
    }
    if (e == hipSuccess) e = save_restore(b, g, false);
    if (e != hipSuccess) break;
    g.waves = best_w;
    fca::tune_cache_put(disk_key, best_w, 0);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return bhip(b, e, "batch tuner");
  b->tuned = true;
  return FCA_OK;
}

hipError_t launch_all(fca_batch* b, int n_iter) {
  if (b->nlanes <= 1) {
    for (const Group& g : b->groups) {
      hipError_t e = launch_group(b, g, g.waves, n_iter, b->stream);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  hipError_t e = hipEventRecord(b->fork, b->stream);
  for (int k = 0; k < b->nlanes && e == hipSuccess; ++k) e = hipStreamWaitEvent(b->lane[k], b->fork, 0);
  // the largest groups first, dealt round-robin over the lanes
  for (size_t r = 0; r < b->order.size() && e == hipSuccess; ++r) {
    const Group& g = b->groups[b->order[r]];
    e = launch_group(b, g, g.waves, n_iter, b->lane[r % b->nlanes]);
  }
  // join every lane, also after an error (a capture must end joined)
  for (int k = 0; k < b->nlanes; ++k) {
    hipError_t e2 = hipEventRecord(b->join[k], b->lane[k]);
    if (e2 == hipSuccess) e2 = hipStreamWaitEvent(b->stream, b->join[k], 0);
    if (e == hipSuccess) e = e2;
  }
  return e;
}

void drop_graphs(fca_batch* b) {
  for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  b->graphs.clear();
}

}  // namespace

extern "C" {

fca_status fca_batch_init(fca_batch** out, int n_mix, const int* F, const int* N, const int* I, const int* J,
                          const fca_c64* const* x, const float* const* v0, const float* const* lam0,
                          const fca_c64* const* P0, void* hip_stream) {
  if (!out) return bfail(nullptr, FCA_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (n_mix < 1) return bfail(nullptr, FCA_ERR_ARG, "n_mix must be positive");
  if (!F || !N || !I || !J || !x || !v0 || !lam0 || !P0)
    return bfail(nullptr, FCA_ERR_ARG, "size and pointer arrays must be non-NULL host arrays of n_mix entries");
  for (int m = 0; m < n_mix; ++m) {  // every host-side check before any device work
    std::string msg;
    const fca_status st = fca::validate_init(FCA_METHOD_AS, F[m], N[m], I[m], J[m], x[m], v0[m], lam0[m], P0[m],
                                             nullptr, &msg);
    if (st != FCA_OK) return bfail(nullptr, st, "mixture " + std::to_string(m) + ": " + msg);
  }
  fca_batch* b = new (std::nothrow) fca_batch();
  if (!b) return bfail(nullptr, FCA_ERR_HIP, "host allocation failed");
  b->stream = reinterpret_cast<hipStream_t>(hip_stream);
  b->nlanes = 0;
  b->fork = nullptr;
  for (int k = 0; k < kLanes; ++k) { b->lane[k] = nullptr; b->join[k] = nullptr; }
  b->dev = nullptr;
  b->use_graph = 1;
  b->use_queue = 0;
  b->autotune = 1;
  b->forced_waves = 0;
  b->tuned = false;
  for (int m = 0; m < n_mix; ++m) {
    fca_ctx* c = nullptr;
    fca_status st = fca_init(&c, FCA_METHOD_AS, F[m], N[m], I[m], J[m], x[m], v0[m], lam0[m], P0[m], nullptr, hip_stream);
    if (st != FCA_OK) {
      const std::string msg = "mixture " + std::to_string(m) + ": " + fca_last_error(nullptr);
      fca_batch_destroy(b);
      return bfail(nullptr, st, msg);
    }
    b->ctx.push_back(c);
  }
  // groups of equal (I, J)
  std::map<std::pair<int, int>, int> gid;
  for (int m = 0; m < n_mix; ++m) {
    const auto key = std::make_pair(I[m], J[m]);
    auto it = gid.find(key);
    if (it == gid.end()) {
      Group g{};
      g.I = I[m]; g.J = J[m]; g.ks = b->ctx[m]->ks; g.n_max = 0; g.ntiles = 0;
      gid[key] = (int)b->groups.size();
      b->groups.push_back(g);
      it = gid.find(key);
    }
    Group& g = b->groups[it->second];
    g.members.push_back(m);
    g.n_max = std::max(g.n_max, N[m]);
    g.ntiles += F[m];
  }
  // device tables: per group the members' DevState and the sorted tiles
  size_t bytes = 0;
  std::vector<size_t> off_s(b->groups.size()), off_t(b->groups.size());
  for (size_t k = 0; k < b->groups.size(); ++k) {
    off_s[k] = bytes; bytes += (sizeof(DevState) * b->groups[k].members.size() + 255) / 256 * 256;
    off_t[k] = bytes; bytes += (sizeof(int2) * (size_t)b->groups[k].ntiles + 255) / 256 * 256;
    bytes += 256;  // the group's queue counter
  }
  hipError_t e = hipMalloc(&b->dev, bytes);
  if (e != hipSuccess) {
    fca_batch_destroy(b);
    return bhip(nullptr, e, "hipMalloc");
  }
  for (size_t k = 0; k < b->groups.size(); ++k) {
    Group& g = b->groups[k];
    g.d_states = reinterpret_cast<DevState*>(static_cast<char*>(b->dev) + off_s[k]);
    g.d_tiles = reinterpret_cast<int2*>(static_cast<char*>(b->dev) + off_t[k]);
    g.d_counter = reinterpret_cast<int*>(static_cast<char*>(b->dev) + off_t[k] +
                                         (sizeof(int2) * (size_t)g.ntiles + 255) / 256 * 256);
    std::vector<DevState> hs;
    for (int m : g.members) hs.push_back(b->ctx[m]->s);
    std::vector<int2> ht;
    for (int slot = 0; slot < (int)g.members.size(); ++slot)
      for (int f = 0; f < F[g.members[slot]]; ++f) ht.push_back(make_int2(slot, f));
    std::stable_sort(ht.begin(), ht.end(), [&](const int2& a, const int2& c) {
      return N[g.members[a.x]] > N[g.members[c.x]];
    });
    e = hipMemcpy(g.d_states, hs.data(), sizeof(DevState) * hs.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(g.d_tiles, ht.data(), sizeof(int2) * ht.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      fca_batch_destroy(b);
      return bhip(nullptr, e, "batch table upload");
    }
  }
  // groups by decreasing work (tiles x frames x per-point cost), and the
  // side streams
  for (size_t k = 0; k < b->groups.size(); ++k) b->order.push_back((int)k);
  auto work = [&](int k) {
    const Group& g = b->groups[k];
    return (double)g.ntiles * g.n_max * (double)g.I * (g.I * g.I + g.J);
  };
  std::stable_sort(b->order.begin(), b->order.end(), [&](int a, int c) { return work(a) > work(c); });
  const int want = (int)std::min<size_t>(kLanes, b->groups.size());
  if (want > 1) {
    e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    for (int k = 0; k < want && e == hipSuccess; ++k) {
      e = hipStreamCreateWithFlags(&b->lane[k], hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming);
      if (e == hipSuccess) b->nlanes = k + 1;
    }
    if (e != hipSuccess) {
      fca_batch_destroy(b);
      return bhip(nullptr, e, "batch streams");
    }
  }
  *out = b;
  return FCA_OK;
}

fca_status fca_batch_iterate(fca_batch* b, int n_iter) {
  if (!b) return bfail(nullptr, FCA_ERR_ARG, "NULL batch");
  if (n_iter < 0) return bfail(b, FCA_ERR_ARG, "n_iter must be >= 0");
  if (n_iter == 0) return FCA_OK;
  if (!b->tuned) {
    fca_status st = tune(b);
    if (st != FCA_OK) return st;
  }
  for (fca_ctx* c : b->ctx) ++c->version;
  hipError_t e;
  if (b->use_graph && b->stream != nullptr) {
    auto it = b->graphs.find(n_iter);
    if (it == b->graphs.end()) {
      hipGraph_t graph;
      if ((e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return bhip(b, e, "hipStreamBeginCapture");
      hipError_t le = launch_all(b, n_iter);
      e = hipStreamEndCapture(b->stream, &graph);
      if (le != hipSuccess) return bhip(b, le, "batch launch under capture");
      if (e != hipSuccess) return bhip(b, e, "hipStreamEndCapture");
      hipGraphExec_t exec;
      e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) return bhip(b, e, "hipGraphInstantiate");
      it = b->graphs.emplace(n_iter, exec).first;
    }
    if ((e = hipGraphLaunch(it->second, b->stream)) != hipSuccess) return bhip(b, e, "hipGraphLaunch");
  } else {
    if ((e = launch_all(b, n_iter)) != hipSuccess) return bhip(b, e, "batch launch");
  }
  return FCA_OK;
}

fca_status fca_batch_context(fca_batch* b, int m, fca_ctx** ctx) {
  if (!b) return bfail(nullptr, FCA_ERR_ARG, "NULL batch");
  if (!ctx || m < 0 || m >= (int)b->ctx.size()) return bfail(b, FCA_ERR_ARG, "bad mixture index or NULL out");
  *ctx = b->ctx[m];
  return FCA_OK;
}

fca_status fca_batch_set_option(fca_batch* b, const char* key, long long value) {
  if (!b) return bfail(nullptr, FCA_ERR_ARG, "NULL batch");
  if (!key) return bfail(b, FCA_ERR_ARG, "NULL key");
  if (!std::strcmp(key, "graph")) {
    if (value != 0 && value != 1) return bfail(b, FCA_ERR_ARG, "graph must be 0 or 1");
    b->use_graph = (int)value;
  } else if (!std::strcmp(key, "queue")) {
    if (value != 0 && value != 1) return bfail(b, FCA_ERR_ARG, "queue must be 0 or 1");
    b->use_queue = (int)value;
    drop_graphs(b);
  } else if (!std::strcmp(key, "autotune")) {
    if (value != 0 && value != 1) return bfail(b, FCA_ERR_ARG, "autotune must be 0 or 1");
    b->autotune = (int)value;
    b->tuned = false;
    drop_graphs(b);
  } else if (!std::strcmp(key, "waves")) {
    if (value != 0 && value != 1 && value != 2 && value != 4)
      return bfail(b, FCA_ERR_ARG, "waves must be 0 (auto), 1, 2 or 4");
    b->forced_waves = (int)value;
    b->tuned = false;
    drop_graphs(b);
  } else if (!std::strcmp(key, "K")) {
    if (value < 1 || value > 64) return bfail(b, FCA_ERR_ARG, "K must be in 1..64");
    for (fca_ctx* c : b->ctx) c->s.K = (int)value;
    b->tuned = false;  // K > 1 changes which launch shapes fit at large I
    drop_graphs(b);
    for (Group& g : b->groups) {
      std::vector<DevState> hs;
      for (int m : g.members) hs.push_back(b->ctx[m]->s);
      hipError_t e = hipMemcpyAsync(g.d_states, hs.data(), sizeof(DevState) * hs.size(), hipMemcpyHostToDevice, b->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
      if (e != hipSuccess) return bhip(b, e, "batch table update");
    }
  } else {
    return bfail(b, FCA_ERR_ARG, std::string("unknown option '") + key + "'");
  }
  return FCA_OK;
}

fca_status fca_batch_get_option(fca_batch* b, const char* key, int group, long long* value) {
  if (!b) return bfail(nullptr, FCA_ERR_ARG, "NULL batch");
  if (!key || !value) return bfail(b, FCA_ERR_ARG, "NULL key or value");
  if (!std::strcmp(key, "groups")) { *value = (long long)b->groups.size(); return FCA_OK; }
  if (!std::strcmp(key, "queue")) { *value = b->use_queue; return FCA_OK; }
  if (group < 0 || group >= (int)b->groups.size()) return bfail(b, FCA_ERR_ARG, "bad group index");
  const Group& g = b->groups[group];
  if (!std::strcmp(key, "group_I")) *value = g.I;
  else if (!std::strcmp(key, "group_J")) *value = g.J;
  else if (!std::strcmp(key, "group_tiles")) *value = g.ntiles;
  else if (!std::strcmp(key, "group_waves")) *value = b->tuned ? g.waves : -1;
  else if (!std::strcmp(key, "group_queued")) *value = g.queued;
  else return bfail(b, FCA_ERR_ARG, std::string("unknown option '") + key + "'");
  return FCA_OK;
}

const char* fca_batch_last_error(const fca_batch* b) { return b ? b->err.c_str() : g_batch_init_error.c_str(); }

void fca_batch_destroy(fca_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  for (int k = 0; k < kLanes; ++k) {
    if (b->lane[k]) {
      (void)hipStreamSynchronize(b->lane[k]);
      (void)hipStreamDestroy(b->lane[k]);
    }
    if (b->join[k]) (void)hipEventDestroy(b->join[k]);
  }
  if (b->fork) (void)hipEventDestroy(b->fork);
  drop_graphs(b);
  for (fca_ctx* c : b->ctx) fca_destroy(c);
  if (b->dev) (void)hipFree(b->dev);
  delete b;
}

}  // extern "C"
