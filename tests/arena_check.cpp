// Host-only check of the served loop's arena allocator (server_arena.h):
// random allocations from both ends and releases against a bitmap, then the
// serving pattern (state slots low, one batch of workspace slots high,
// released together) must leave the free space in one piece.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "server_arena.h"

static int fail(const char* what, long step) {
  std::printf("FAIL %s at step %ld\n", what, step);
  return 1;
}

int main() {
  const int64_t U = 4000;
  mpc::Arena a;
  a.init(U);
  std::vector<char> used(U, 0);
  std::vector<std::pair<int64_t, int64_t>> live;
  std::srand(7);
  for (long step = 0; step < 100000; ++step) {
    if (live.empty() || std::rand() % 3) {
      const int64_t n = 1 + std::rand() % 50;
      const bool high = std::rand() & 1;
      const int64_t off = high ? a.alloc_high(n) : a.alloc(n);
      if (off >= 0) {
        for (int64_t i = off; i < off + n; ++i) {
          if (i < 0 || i >= U || used[i]) return fail("overlap or out of range", step);
          used[i] = 1;
        }
        live.push_back({off, n});
      } else {
        int64_t run = 0, best = 0;
        for (int64_t i = 0; i < U; ++i) {
          run = used[i] ? 0 : run + 1;
          if (run > best) best = run;
        }
        if (best >= n) return fail("refused although a free run fits", step);
      }
    } else {
      const size_t k = std::rand() % live.size();
      const auto p = live[k];
      live[k] = live.back();
      live.pop_back();
      for (int64_t i = p.first; i < p.first + p.second; ++i) used[i] = 0;
      a.release(p.first, p.second);
    }
    int64_t fu = 0;
    for (int64_t i = 0; i < U; ++i) fu += !used[i];
    if (fu != a.free_units()) return fail("free count", step);
  }
  // serving pattern: 2000 controllers' states (two sizes) interleaved with the
  // first batch's workspace, then batches of workspace alone
  mpc::Arena b;
  b.init(1 << 22);
  std::vector<std::pair<int64_t, int64_t>> ws;
  for (int c = 0; c < 2000; ++c) {
    if (b.alloc(c % 2 ? 7 : 11) < 0) return fail("state", c);
    const int64_t n = c % 2 ? 40 : 90, off = b.alloc_high(n);
    if (off < 0) return fail("workspace", c);
    ws.push_back({off, n});
  }
  for (int batch = 0; batch < 20; ++batch) {
    for (auto& p : ws) b.release(p.first, p.second);
    if (b.fragments() != 1) return fail("free space not in one piece after a batch", batch);
    ws.clear();
    for (int c = 0; c < 2000; ++c) {
      const int64_t n = c % 2 ? 40 : 90, off = b.alloc_high(n);
      if (off < 0) return fail("workspace", batch);
      ws.push_back({off, n});
    }
  }
  std::printf("arena ok\n");
  return 0;
}
