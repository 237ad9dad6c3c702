// Batched SIMP iterations over many independent problems.
//
// Problems with equal grids (and options that allow it) form groups of up to
// kMaxGroup: the members share one stream, and every pass of their CG
// iterations -- operator, vector updates, each smoothing pass, transfer and
// coarse solve of the V-cycle -- is one launch for the whole group (grouped
// launches, internal.h), so a group of small problems costs about one small
// problem's launch latency per pass instead of one per member.  The rest of a
// SIMP iteration (filter, operator set-up, warm start, sensitivities, OC) runs
// member by member on the group's stream.  Groups, and problems that cannot be
// grouped, run concurrently on their own streams, driven by a pool of host
// threads (largest first); each checks its own convergence between chunks of
// CG iterations and never waits for the others.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

using namespace topo;

namespace {
struct Unit {               // a group, or one problem on its own stream
  std::vector<int> members;  // problem indices
  hipStream_t stream = nullptr, cap = nullptr;
  hipGraph_t graph = nullptr;     // captured chunk of grouped CG iterations
  hipGraphExec_t exec = nullptr;  // ... and its executable
  int64_t ndof = 0;
};
}  // namespace

struct topo_batch {
  std::vector<topo_ctx *> ctx;
  std::vector<hipStream_t> streams;  // per-problem streams (set-up; ungrouped problems)
  std::vector<int64_t> ndof;
  std::vector<Unit> units;
  int device = 0;
  int threads = 1;
  // Order matters: a group member's context runs on the group's stream, and
  // destroying a context synchronises its current stream, so the group
  // streams are drained and every context handed back its own stream before
  // any context goes; streams are destroyed last.
  ~topo_batch() {
    for (Unit &u : units) {
      if (u.members.size() > 1 && u.stream) {
        (void)hipStreamSynchronize(u.stream);
        for (int i : u.members)
          if (i < (int)ctx.size() && i < (int)streams.size()) ctx_set_stream(ctx[i], streams[i]);
      }
      if (u.exec) (void)hipGraphExecDestroy(u.exec);
      if (u.graph) (void)hipGraphDestroy(u.graph);
      u.exec = nullptr;
      u.graph = nullptr;
    }
    for (topo_ctx *c : ctx) topo_destroy(c);
    for (Unit &u : units) {
      if (u.cap) (void)hipStreamDestroy(u.cap);
      if (u.members.size() > 1 && u.stream) (void)hipStreamDestroy(u.stream);
    }
    for (hipStream_t s : streams)
      if (s) (void)hipStreamDestroy(s);
  }
};

// Groups: problems whose grids agree (and whose contexts allow grouping) take
// the launch shapes of the first of them and are split into groups of at most
// kMaxGroup; everything else is a unit of its own.
static topo_status make_units(topo_batch *b, bool group) {
  const int n = (int)b->ctx.size();
  std::map<std::string, std::vector<int>> buckets;
  std::vector<int> alone;
  for (int i = 0; i < n; ++i) {
    std::string key = group ? group_key(b->ctx[i]) : std::string();
    if (key.empty()) {
      alone.push_back(i);
      continue;
    }
    const Grid g = ctx_grid(b->ctx[i]);
    // the grid and the context's own key prefix; shapes are aligned below
    buckets[std::to_string(g.nx) + "x" + std::to_string(g.ny) + "x" + std::to_string(g.nz)].push_back(i);
  }
  for (auto &kv : buckets) {
    std::vector<int> &v = kv.second;
    for (size_t j = 1; j < v.size(); ++j) group_adopt_shapes(b->ctx[v[j]], b->ctx[v[0]]);
    // members must agree on everything the grouped CG depends on
    std::vector<std::vector<int>> parts;
    for (int i : v) {
      bool placed = false;
      for (auto &p : parts)
        if ((int)p.size() < kMaxGroup && group_key(b->ctx[p[0]]) == group_key(b->ctx[i])) {
          p.push_back(i);
          placed = true;
          break;
        }
      if (!placed) parts.push_back({i});
    }
    for (auto &p : parts) {
      if (p.size() == 1) {
        alone.push_back(p[0]);
        continue;
      }
      Unit u;
      u.members = p;
      if (hipStreamCreateWithFlags(&u.stream, hipStreamNonBlocking) != hipSuccess ||
          hipStreamCreateWithFlags(&u.cap, hipStreamNonBlocking) != hipSuccess) {
        b->units.push_back(u);
        return set_error("stream creation failed for a problem group"), TOPO_EDEVICE;
      }
      for (int i : p) {
        ctx_set_stream(b->ctx[i], u.stream);
        u.ndof += b->ndof[i];
      }
      b->units.push_back(u);
    }
  }
  for (int i : alone) {
    Unit u;
    u.members = {i};
    u.stream = b->streams[i];
    u.ndof = b->ndof[i];
    b->units.push_back(u);
  }
  // largest work first (longest-processing-time order)
  std::stable_sort(b->units.begin(), b->units.end(), [](const Unit &a, const Unit &c) { return a.ndof > c.ndof; });
  return TOPO_OK;
}

extern "C" topo_status topo_setup_batch(const topo_problem *problems, int32_t n, const topo_opts *opts,
                                        int32_t n_threads, topo_batch **out) {
  if (!out) return set_error("out is NULL"), TOPO_EINVAL;
  *out = nullptr;
  if (!problems || n < 1) return set_error("need at least one problem"), TOPO_EINVAL;
  if (n_threads < 0 || n_threads > 64) return set_error("n_threads must lie in [0, 64]"), TOPO_EINVAL;
  topo_opts defaults;
  topo_default_opts(&defaults);
  if (!opts) opts = &defaults;
  topo_batch *b = new (std::nothrow) topo_batch();
  if (!b) return set_error("host allocation failed"), TOPO_ENOMEM;
  if (hipGetDevice(&b->device) != hipSuccess) {
    delete b;
    return set_error("no HIP device"), TOPO_EDEVICE;
  }
  b->threads = n_threads > 0 ? std::min<int>(n_threads, n) : std::min<int>(8, n);
  for (int i = 0; i < n; ++i) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      delete b;
      return set_error("stream creation failed for problem %d", i), TOPO_EDEVICE;
    }
    b->streams.push_back(s);
    topo_ctx *c = nullptr;
    topo_status st = topo_setup(&problems[i], opts, (void *)s, &c);
    if (st != TOPO_OK) {
      std::string msg = topo_last_error();
      delete b;
      return set_error("problem %d: %s", i, msg.c_str()), st;
    }
    b->ctx.push_back(c);
    int64_t nd = 0;
    (void)topo_sizes(c, nullptr, &nd, nullptr);
    b->ndof.push_back(nd);
  }
  topo_status st = make_units(b, opts->group_launch != 0);
  if (st != TOPO_OK) {
    delete b;
    return st;
  }
  *out = b;
  return TOPO_OK;
}

extern "C" void topo_destroy_batch(topo_batch *b) { delete b; }

extern "C" topo_status topo_batch_context(topo_batch *b, int32_t i, topo_ctx **out) {
  if (!b || !out || i < 0 || i >= (int32_t)b->ctx.size()) return set_error("invalid argument"), TOPO_EINVAL;
  *out = b->ctx[i];
  return TOPO_OK;
}

// n_iter SIMP iterations of a group: per iteration every member's pre-solve
// part, the grouped CG, every member's post-solve part
static topo_status iterate_group(topo_batch *b, Unit &u, double *const *d_x, int32_t n_iter, topo_iter_stats *h_stats) {
  const int m = (int)u.members.size();
  Group G;
  G.s = u.stream;
  for (int i : u.members) G.c.push_back(b->ctx[i]);
  std::vector<hipEvent_t> ev(6 * (size_t)m, nullptr);
  for (auto &e : ev)
    if (hipEventCreate(&e) != hipSuccess) return set_error("event creation failed"), TOPO_EDEVICE;
  std::vector<topo_solve_stats> ss(m);
  std::vector<double *> x(m);
  std::vector<topo_iter_stats *> o(m);
  for (int k = 0; k < m; ++k) x[k] = d_x[u.members[k]];
  topo_status result = TOPO_OK, st = TOPO_OK;
  for (int it = 0; it < n_iter && st == TOPO_OK; ++it) {
    // members in lockstep (the normal case) share every launch of the
    // iteration; otherwise only the CG iterations
    const bool shared = group_lockstep(G);
    for (int k = 0; k < m; ++k) o[k] = h_stats ? h_stats + (size_t)u.members[k] * n_iter + it : nullptr;
    if (shared) st = group_pre(G, x.data(), ev.data());
    for (int k = 0; k < m && st == TOPO_OK && !shared; ++k) st = iterate_pre(G.c[k], x[k], &ev[6 * k]);
    if (st != TOPO_OK) break;
    st = group_pcg(G, &u.graph, &u.exec, u.cap, ss.data());
    if (st == TOPO_ENOTCONVERGED) result = st, st = TOPO_OK;
    if (st != TOPO_OK) break;
    if (shared) st = group_post(G, x.data(), ss.data(), ev.data(), o.data());
    for (int k = 0; k < m && st == TOPO_OK && !shared; ++k) st = iterate_post(G.c[k], x[k], ss[k], &ev[6 * k], o[k]);
  }
  if (st == TOPO_OK && hipStreamSynchronize(u.stream) != hipSuccess) {
    set_error("stream synchronisation failed");
    st = TOPO_EDEVICE;
  }
  for (auto &e : ev) (void)hipEventDestroy(e);
  return st != TOPO_OK ? st : result;
}

extern "C" topo_status topo_iterate_batch(topo_batch *b, double *const *d_x, int32_t n_iter,
                                          topo_iter_stats *h_stats) {
  if (!b || !d_x || n_iter < 0) return set_error("invalid argument"), TOPO_EINVAL;
  const int n = (int)b->ctx.size();
  for (int i = 0; i < n; ++i)
    if (!d_x[i]) return set_error("d_x[%d] is NULL", i), TOPO_EINVAL;
  const int nu = (int)b->units.size();
  std::atomic<int> next{0};
  std::mutex mu;
  topo_status first = TOPO_OK;
  bool notconv = false;
  std::string msg;
  auto worker = [&]() {
    if (hipSetDevice(b->device) != hipSuccess) {
      std::lock_guard<std::mutex> g(mu);
      if (first == TOPO_OK) first = TOPO_EDEVICE, msg = "hipSetDevice failed in a worker thread";
      return;
    }
    for (;;) {
      const int k = next.fetch_add(1);
      if (k >= nu) return;
      Unit &u = b->units[k];
      topo_status st;
      if (u.members.size() == 1) {
        const int i = u.members[0];
        st = topo_iterate(b->ctx[i], d_x[i], n_iter, h_stats ? h_stats + (size_t)i * n_iter : nullptr);
      } else {
        st = iterate_group(b, u, d_x, n_iter, h_stats);
      }
      if (st == TOPO_ENOTCONVERGED) {
        std::lock_guard<std::mutex> g(mu);
        notconv = true;
      } else if (st != TOPO_OK) {
        std::lock_guard<std::mutex> g(mu);
        if (first == TOPO_OK) {
          first = st;
          msg = std::string("problem ") + std::to_string(u.members[0]) + ": " + topo_last_error();
        }
        next.store(nu);  // stop handing out work
        return;
      }
    }
  };
  std::vector<std::thread> pool;
  const int T = std::max(1, std::min(b->threads, nu));
  for (int t = 1; t < T; ++t) pool.emplace_back(worker);
  worker();
  for (auto &t : pool) t.join();
  if (first != TOPO_OK) return set_error("%s", msg.c_str()), first;
  if (notconv) return set_error("at least one problem's CG reached max_iters"), TOPO_ENOTCONVERGED;
  return TOPO_OK;
}
