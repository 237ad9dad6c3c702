// Batched SIMP iterations over many independent problems.
//
// Every problem keeps its own context (multigrid hierarchy, CG graphs, scalars)
// on its own HIP stream, so kernels of different problems run concurrently on
// the device: the small and mid-size grids of a batch are latency-bound one by
// one, and interleaving their streams fills the compute units.  A pool of host
// threads drives the problems (largest first, each thread taking the next
// problem when it finishes one), because every problem's CG loop checks its
// own convergence flag between graph-replayed chunks and must not wait for the
// others.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

using namespace topo;

struct topo_batch {
  std::vector<topo_ctx *> ctx;
  std::vector<hipStream_t> streams;
  std::vector<int64_t> ndof;
  int device = 0;
  int threads = 1;
  ~topo_batch() {
    for (topo_ctx *c : ctx) topo_destroy(c);
    for (hipStream_t s : streams)
      if (s) (void)hipStreamDestroy(s);
  }
};

extern "C" topo_status topo_setup_batch(const topo_problem *problems, int32_t n, const topo_opts *opts,
                                        int32_t n_threads, topo_batch **out) {
  if (!out) return set_error("out is NULL"), TOPO_EINVAL;
  *out = nullptr;
  if (!problems || n < 1) return set_error("need at least one problem"), TOPO_EINVAL;
  if (n_threads < 0 || n_threads > 64) return set_error("n_threads must lie in [0, 64]"), TOPO_EINVAL;
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
  *out = b;
  return TOPO_OK;
}

extern "C" void topo_destroy_batch(topo_batch *b) { delete b; }

extern "C" topo_status topo_batch_context(topo_batch *b, int32_t i, topo_ctx **out) {
  if (!b || !out || i < 0 || i >= (int32_t)b->ctx.size()) return set_error("invalid argument"), TOPO_EINVAL;
  *out = b->ctx[i];
  return TOPO_OK;
}

extern "C" topo_status topo_iterate_batch(topo_batch *b, double *const *d_x, int32_t n_iter,
                                          topo_iter_stats *h_stats) {
  if (!b || !d_x || n_iter < 0) return set_error("invalid argument"), TOPO_EINVAL;
  const int n = (int)b->ctx.size();
  for (int i = 0; i < n; ++i)
    if (!d_x[i]) return set_error("d_x[%d] is NULL", i), TOPO_EINVAL;
  // largest problems first (longest-processing-time order)
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return b->ndof[a] > b->ndof[c]; });
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
      if (k >= n) return;
      const int i = order[k];
      topo_status st = topo_iterate(b->ctx[i], d_x[i], n_iter, h_stats ? h_stats + (size_t)i * n_iter : nullptr);
      if (st == TOPO_ENOTCONVERGED) {
        std::lock_guard<std::mutex> g(mu);
        notconv = true;
      } else if (st != TOPO_OK) {
        std::lock_guard<std::mutex> g(mu);
        if (first == TOPO_OK) {
          first = st;
          msg = std::string("problem ") + std::to_string(i) + ": " + topo_last_error();
        }
        next.store(n);  // stop handing out work
        return;
      }
    }
  };
  std::vector<std::thread> pool;
  const int T = std::max(1, std::min(b->threads, n));
  for (int t = 1; t < T; ++t) pool.emplace_back(worker);
  worker();
  for (auto &t : pool) t.join();
  if (first != TOPO_OK) return set_error("%s", msg.c_str()), first;
  if (notconv) return set_error("at least one problem's CG reached max_iters"), TOPO_ENOTCONVERGED;
  return TOPO_OK;
}
