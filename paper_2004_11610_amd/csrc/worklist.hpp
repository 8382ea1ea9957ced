// Work lists of staged launches (host only, no HIP): the items that a launch's
// workgroups read, built from plain plan descriptions so that they can be
// built and checked without a device.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace spt {

// one work item (the device reads it as an int4)
struct WorkItem {
  int32_t x, y, z, w;
};

// items of the FFT launches and of the persistent executor: x = kind | plan
// << 4; y = block (FFT/COL/ROW) or first row tile (SPMM); z = first right-hand
// side; w = log2 of the right-hand sides (FFT), column group (COL) or pair
// group (ROW)
enum : int { ITEM_FFT = 0, ITEM_COL = 1, ITEM_ROW = 2, ITEM_SPMM = 3 };
inline int item_head(int kind, int plan) { return kind | (plan << 4); }

// ---------------------------------------------------------------- staged batch: products
// A plan of a staged batch as the product launches see it.
struct BatchProductPlan {
  int32_t windowed;  // 1: the chunked windowed product takes this plan (split-bf16)
  int32_t n_groups;  // groups of WIN_TILES row tiles (windowed plans)
  int32_t n_tiles;   // row tiles of TILE_ROWS rows
  int64_t R;         // right-hand sides
};

// The two product launches of a staged batch.  Each launch reads only its own
// list, `count` items of it: workgroup b takes list[b].
//   tile launch (per-tile product): items {plan, tile, r0, 0} of the plans that
//     are not windowed, tile < n_tiles (tile -1: padding);
//   window launch (chunked windowed product): items {plan, group, r0, 0} of the
//     windowed plans, group < n_groups (group -1: padding).
// Items of one plan's chunk of 64 right-hand sides start at a multiple of 8
// (padding in between); tiles and groups in XCD order (xcd_order).
struct BatchProductLaunch {
  const std::vector<WorkItem>* list = nullptr;
  int count = 0;
  bool window = false;   // the chunked windowed product's launch
  bool chunked = false;  // the batch sends its windowed plans to that launch
};
struct BatchProductLists {
  std::vector<WorkItem> tile_items, win_items;
  BatchProductLaunch tile_launch, win_launch;
};
void build_batch_product_lists(const BatchProductPlan* plans, int count, bool chunked,
                               BatchProductLists& out);
// true when every launch reads only its own list, within its size, and every
// item's plan, tile or group and first right-hand side lie within that plan;
// otherwise false with the reason in *why
bool check_batch_product_launch(const BatchProductPlan* plans, int count,
                                const BatchProductLaunch& l, std::string* why);

// ---------------------------------------------------------------- staged FFT items
// A block as the FFT items see it.
struct FftItemBlock {
  int32_t P;           // half length
  int32_t four;        // 1: four-step transform (COL then ROW items)
  int32_t n_col, n_row;  // COL / ROW items per right-hand side
  int32_t batch;       // right-hand sides per single-workgroup item (a power of two)
};
// Items of the staged FFT launches of a plan or batch (kind | plan << 4 as in
// the persistent executor's items): the first launch takes the COL items and
// the single-workgroup FFT items, the second the ROW items.
struct FftItemLists {
  std::vector<WorkItem> first, second;
};
void build_fft_item_lists(const std::vector<std::vector<FftItemBlock>>& blocks,
                          const std::vector<int64_t>& R, FftItemLists& out);
bool check_fft_item_lists(const std::vector<std::vector<FftItemBlock>>& blocks,
                          const std::vector<int64_t>& R, const FftItemLists& l, std::string* why);

// workgroup b of n in XCD order: consecutive tiles on one XCD (a bijection of [0, n))
inline int xcd_order(int b, int n) {
  const int n8 = n >> 3;
  return b < 8 * n8 ? (b & 7) * n8 + (b >> 3) : b;
}

}  // namespace spt
