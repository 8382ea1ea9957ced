// Host-only checks of the planner and the staged work lists, built with the
// address and undefined-behaviour sanitizers by tests/test_host_sanitized.py.
// Exit status 0 when every check holds.

#include <cstdio>
#include <random>
#include <string>
#include <vector>

#include "../../paper_2004_11610_amd/csrc/planner.hpp"
#include "../../paper_2004_11610_amd/csrc/worklist.hpp"

using namespace spt;

static int failures = 0;
#define CHECK(cond, ...)                      \
  do {                                        \
    if (!(cond)) {                            \
      std::printf("FAIL %s:%d ", __FILE__, __LINE__); \
      std::printf(__VA_ARGS__);               \
      std::printf("\n");                      \
      ++failures;                             \
    }                                         \
  } while (0)

// every input column covered once by a block's retained range or the tail
static void check_partition(int64_t N, const std::vector<BlockGeom>& b, int64_t tail, bool two) {
  std::vector<int> cov(N, 0);
  for (int64_t m = 0; m < tail && m < N; ++m) cov[m] += 1;
  for (const BlockGeom& g : b) {
    CHECK(g.L % 2 == 0 && 0 <= g.c_lo && g.c_lo < g.c_hi && g.c_hi <= g.L, "block geometry");
    for (int c = g.c_lo; c < g.c_hi; ++c) {
      const int64_t m = c + (int64_t)g.m_off;
      CHECK(m >= 0 && m < N, "retained column out of range");
      if (m >= 0 && m < N) cov[m] += 1;
    }
  }
  for (int64_t m = 0; m < N; ++m) CHECK(cov[m] == 1, "N %lld column %lld covered %d times (two-sided %d)",
                                        (long long)N, (long long)m, cov[m], (int)two);
}

int main() {
  // planner over sizes and parameters
  const double eps1s[] = {1e-12, 1e-7, 1e-4};
  const double eps2s[] = {1e-3, 1e-2, 3e-2};
  std::vector<int64_t> Ns;
  for (int64_t N = 2; N < 600; ++N) Ns.push_back(N);
  for (int64_t N = 600; N < 70000; N = N * 5 / 4 + 7) Ns.push_back(N);
  for (double e1 : eps1s) {
    const double z = zeta_of_eps(e1);
    CHECK(z > 0 && z < 60, "zeta");
    for (double e2 : eps2s) {
      if (!(e2 > e1)) continue;
      for (int64_t N : Ns) {
        std::vector<BlockGeom> b;
        int64_t tail = 0;
        partition_one_sided(N, z, e2, 32, true, b, tail);
        check_partition(N, b, tail, false);
        partition_two_sided(N, z, e2, true, b, tail);
        check_partition(N, b, tail, true);
      }
    }
  }
  // staged batch product lists: random batches, all-windowed and none-windowed
  std::mt19937 rng(2004);
  int batches = 0;
  for (int trial = 0; trial < 900; ++trial) {
    const int count = 1 + (int)(rng() % 64);
    const int mode = trial % 3;  // 0 random, 1 every plan windowed, 2 none
    std::vector<BatchProductPlan> p(count);
    for (auto& q : p) {
      const int tiles = 1 + (int)(rng() % 800);
      q = BatchProductPlan{mode == 1 ? 1 : mode == 2 ? 0 : (int)(rng() % 2), (tiles + 3) / 4, tiles,
                           1 + (int64_t)(rng() % 300)};
    }
    for (int chunked = 0; chunked < 2; ++chunked) {
      BatchProductLists bl;
      build_batch_product_lists(p.data(), count, chunked != 0, bl);
      std::string why;
      CHECK(check_batch_product_launch(p.data(), count, bl.tile_launch, &why), "%s", why.c_str());
      CHECK(check_batch_product_launch(p.data(), count, bl.win_launch, &why), "%s", why.c_str());
      // the window launch pointed at the per-tile list (the pairing of a
      // fixed fault) is refused whenever the windowed plans have items
      if (chunked && !bl.win_items.empty()) {
        const BatchProductLaunch wrong{&bl.tile_items, (int)bl.win_items.size(), true, true};
        CHECK(!check_batch_product_launch(p.data(), count, wrong, &why),
              "window launch over the tile list accepted");
      }
      ++batches;
    }
  }
  // FFT item lists
  for (int trial = 0; trial < 2000; ++trial) {
    const int count = 1 + (int)(rng() % 8);
    std::vector<std::vector<FftItemBlock>> blocks(count);
    std::vector<int64_t> R(count);
    for (int i = 0; i < count; ++i) {
      R[i] = 1 + (int64_t)(rng() % 200);
      const int nb = 1 + (int)(rng() % 6);
      for (int b = 0; b < nb; ++b) {
        const bool four = rng() % 3 == 0;
        blocks[i].push_back(FftItemBlock{64 + (int)(rng() % 40000), four ? 1 : 0,
                                         four ? 1 + (int)(rng() % 40) : 0,
                                         four ? 1 + (int)(rng() % 40) : 0,
                                         four ? 1 : 1 << (int)(rng() % 7)});
      }
    }
    FftItemLists fl;
    build_fft_item_lists(blocks, R, fl);
    std::string why;
    CHECK(check_fft_item_lists(blocks, R, fl, &why), "%s", why.c_str());
    if (!fl.first.empty()) {  // a dropped item is caught
      FftItemLists bad = fl;
      bad.first.pop_back();
      CHECK(!check_fft_item_lists(blocks, R, bad, &why), "dropped item accepted");
    }
  }
  std::printf("planner sizes %zu, product batches %d, failures %d\n", Ns.size(), batches, failures);
  return failures == 0 ? 0 : 1;
}
