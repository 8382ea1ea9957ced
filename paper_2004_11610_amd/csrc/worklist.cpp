// Work lists of staged launches (host only): see worklist.hpp.

#include "worklist.hpp"

#include <algorithm>

namespace spt {

void build_batch_product_lists(const BatchProductPlan* plans, int count, bool chunked,
                               BatchProductLists& out) {
  out.tile_items.clear();
  out.win_items.clear();
  for (int i = 0; i < count; ++i) {
    const bool win = chunked && plans[i].windowed;
    std::vector<WorkItem>& it = win ? out.win_items : out.tile_items;
    const int n = win ? plans[i].n_groups : plans[i].n_tiles;
    for (int64_t r0 = 0; r0 < plans[i].R; r0 += 64) {
      while (it.size() % 8) it.push_back(WorkItem{i, -1, 0, 0});
      for (int t = 0; t < n; ++t) it.push_back(WorkItem{i, xcd_order(t, n), (int32_t)r0, 0});
    }
  }
  out.tile_launch = BatchProductLaunch{&out.tile_items, (int)out.tile_items.size(), false, chunked};
  out.win_launch = BatchProductLaunch{&out.win_items, (int)out.win_items.size(), true, chunked};
}

bool check_batch_product_launch(const BatchProductPlan* plans, int count,
                                const BatchProductLaunch& l, std::string* why) {
  auto fail = [&](const std::string& m) {
    if (why) *why = (l.window ? "window launch: " : "tile launch: ") + m;
    return false;
  };
  if (l.count == 0) return true;
  if (!l.list) return fail("no list");
  if (l.count < 0 || (size_t)l.count > l.list->size())
    return fail("reads " + std::to_string(l.count) + " items of a list of " +
                std::to_string(l.list->size()));
  for (int b = 0; b < l.count; ++b) {
    const WorkItem& it = (*l.list)[b];
    if (it.x < 0 || it.x >= count) return fail("item " + std::to_string(b) + ": plan out of range");
    const BatchProductPlan& p = plans[it.x];
    if (it.y < 0) continue;  // padding
    if (l.window != (l.chunked && p.windowed != 0))
      return fail("item " + std::to_string(b) + ": plan of the other product kernel");
    const int n = l.window ? p.n_groups : p.n_tiles;
    if (it.y >= n) return fail("item " + std::to_string(b) + ": tile or group out of range");
    if (it.z < 0 || it.z >= p.R || it.z % 64 != 0)
      return fail("item " + std::to_string(b) + ": first right-hand side out of range");
  }
  return true;
}

void build_fft_item_lists(const std::vector<std::vector<FftItemBlock>>& blocks,
                          const std::vector<int64_t>& R, FftItemLists& out) {
  std::vector<WorkItem> col, fft, row;
  for (size_t i = 0; i < blocks.size(); ++i) {
    const int r = (int)R[i];
    for (size_t b = 0; b < blocks[i].size(); ++b) {
      const FftItemBlock& B = blocks[i][b];
      if (B.four) {
        for (int rr = 0; rr < r; ++rr)
          for (int g = 0; g < B.n_col; ++g)
            col.push_back(WorkItem{item_head(ITEM_COL, (int)i), (int)b, rr, g});
        for (int rr = 0; rr < r; ++rr)
          for (int q = 0; q < B.n_row; ++q)
            row.push_back(WorkItem{item_head(ITEM_ROW, (int)i), (int)b, rr, q});
      } else {
        int lg = 0;
        while ((1 << (lg + 1)) <= B.batch) ++lg;
        for (int r0 = 0; r0 < r; r0 += B.batch)
          fft.push_back(WorkItem{item_head(ITEM_FFT, (int)i), (int)b, r0, lg});
      }
    }
  }
  out.first = col;
  out.first.insert(out.first.end(), fft.begin(), fft.end());
  out.second = row;
}

bool check_fft_item_lists(const std::vector<std::vector<FftItemBlock>>& blocks,
                          const std::vector<int64_t>& R, const FftItemLists& l,
                          std::string* why) {
  auto fail = [&](const std::string& m) {
    if (why) *why = m;
    return false;
  };
  // every (plan, block, right-hand side) transformed exactly once; COL/ROW
  // items only in their launch, and each group of a four-step transform once
  std::vector<std::vector<std::vector<int>>> seen(blocks.size());
  for (size_t i = 0; i < blocks.size(); ++i) {
    seen[i].resize(blocks[i].size());
    for (size_t b = 0; b < blocks[i].size(); ++b) {
      const FftItemBlock& B = blocks[i][b];
      seen[i][b].assign((size_t)R[i] * (B.four ? B.n_col + B.n_row : 1), 0);
    }
  }
  for (int launch = 0; launch < 2; ++launch) {
    const std::vector<WorkItem>& L = launch == 0 ? l.first : l.second;
    for (size_t n = 0; n < L.size(); ++n) {
      const WorkItem& it = L[n];
      const int kind = it.x & 15, p = it.x >> 4;
      if (p < 0 || (size_t)p >= blocks.size()) return fail("item plan out of range");
      if (it.y < 0 || (size_t)it.y >= blocks[p].size()) return fail("item block out of range");
      const FftItemBlock& B = blocks[p][it.y];
      if (it.z < 0 || it.z >= R[p]) return fail("item right-hand side out of range");
      if (kind == ITEM_FFT) {
        if (launch != 0 || B.four) return fail("single-workgroup item in the wrong launch");
        const int nb = 1 << it.w;
        if (nb != B.batch || it.z % nb) return fail("single-workgroup item: bad batch");
        for (int t = it.z; t < std::min<int64_t>(it.z + nb, R[p]); ++t) seen[p][it.y][t] += 1;
      } else if (kind == ITEM_COL || kind == ITEM_ROW) {
        if (!B.four) return fail("four-step item of a single-workgroup block");
        if ((kind == ITEM_COL) != (launch == 0)) return fail("four-step item in the wrong launch");
        const int lim = kind == ITEM_COL ? B.n_col : B.n_row;
        if (it.w < 0 || it.w >= lim) return fail("four-step item: group out of range");
        const int slot = kind == ITEM_COL ? it.w : B.n_col + it.w;
        seen[p][it.y][(size_t)it.z * (B.n_col + B.n_row) + slot] += 1;
      } else {
        return fail("unknown item kind");
      }
    }
  }
  for (size_t i = 0; i < blocks.size(); ++i)
    for (size_t b = 0; b < blocks[i].size(); ++b)
      for (int c : seen[i][b])
        if (c != 1) return fail("a transform or group covered " + std::to_string(c) + " times");
  return true;
}

}  // namespace spt
