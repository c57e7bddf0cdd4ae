// Work-item schedule per window length, tap precision and RIR length, read by
// the host planner, and the grid of the persistent batch launch. Written by
// paper_1810_11359_amd/autotune.py from timings on the target GPU; until the
// tuner has run for a class, the entries repeat the untuned defaults.
//   min_item_taps  estimated taps of the smallest work item
//   balance_items  items a large call is split into (about eight per
//                  resident wave), which sets the item size of large calls
//   ns_max         the entry applies to RIRs of at most this many samples
//                  (first match in table order)
//   waves          workgroups per SIMD of a persistent batch launch
#pragma once

namespace ism {

struct ItemTuning {
  int wt;        // window cap in samples
  int half;      // 1: FP16 taps, 0: FP32 taps
  int ns_max;    // RIR length bucket (samples)
  double min_item_taps;
  double balance_items;
};

struct BatchTuning {
  int wt;
  int half;
  int waves;
};

constexpr ItemTuning kItemTuning[] = {
    {32, 1, 2147483647, 60000, 196608.0},
    {32, 0, 2147483647, 240000, 98304.0},
    {64, 1, 2147483647, 60000, 24576.0},
    {64, 0, 2147483647, 120000, 98304.0},
    {96, 1, 2147483647, 240000, 24576.0},
    {96, 0, 2147483647, 480000, 24576.0},
    {128, 1, 2147483647, 120000, 196608.0},
    {128, 0, 2147483647, 60000, 24576.0},
};

constexpr BatchTuning kBatchTuning[] = {
    {64, 0, 7},
    {64, 1, 7},
};

}  // namespace ism
