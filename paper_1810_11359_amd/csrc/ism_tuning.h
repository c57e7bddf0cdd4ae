// Work-item schedule per window length and tap precision, read by the host
// planner. Written by paper_1810_11359_amd/autotune.py from timings on the
// target GPU (AMD Radeon Graphics).
//   min_item_taps  estimated taps of the smallest work item
//   balance_items  items a large call is split into (about eight per
//                  resident wave), which sets the item size of large calls
//
// Score: geometric mean over the class's workloads of kernel time relative
// to the fastest pair on that workload (1.0 = fastest everywhere).
// W=32 fp16 (room_4x5x3_32rcv_8k): best 60000 / 196608, score 1.0000, default 1.2e5 / 49152 score 1.0303
// W=32 fp32 (room_4x5x3_32rcv_8k): best 240000 / 98304, score 1.0000, default 1.2e5 / 49152 score 1.0635
// W=64 fp16 (room_4x5x3_32rcv_16k, batch_256_rooms_16k): best 60000 / 24576, score 1.0136, default 1.2e5 / 49152 score 1.0495
// W=64 fp32 (room_4x5x3_32rcv_16k, batch_256_rooms_16k): best 120000 / 98304, score 1.0032, default 1.2e5 / 49152 score 1.0157
// W=96 fp16 (room_6x9x3.5_uca64_48k): best 240000 / 24576, score 1.0000, default 1.2e5 / 49152 score 1.0085
// W=96 fp32 (room_6x9x3.5_uca64_48k): best 480000 / 24576, score 1.0000, default 1.2e5 / 49152 score 1.0065
// W=128 fp16 (room_4x5x3_16rcv_32k): best 120000 / 196608, score 1.0000, default 1.2e5 / 49152 score 1.0096
// W=128 fp32 (room_4x5x3_16rcv_32k): best 60000 / 24576, score 1.0000, default 1.2e5 / 49152 score 1.0146
#pragma once

namespace ism {

struct ItemTuning {
  int wt;        // window length in samples
  int half;      // 1: FP16 taps, 0: FP32 taps
  double min_item_taps;
  double balance_items;
};

constexpr ItemTuning kItemTuning[] = {
    {32, 1, 60000, 196608.0},
    {32, 0, 240000, 98304.0},
    {64, 1, 60000, 24576.0},
    {64, 0, 120000, 98304.0},
    {96, 1, 240000, 24576.0},
    {96, 0, 480000, 24576.0},
    {128, 1, 120000, 196608.0},
    {128, 0, 60000, 24576.0},
};

}  // namespace ism
