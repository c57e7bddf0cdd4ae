// Work-item schedule per window length, tap precision and RIR length, read by
// the host planner, and the grid of the persistent batch launch. Written by
// paper_1810_11359_amd/autotune.py from timings on the target GPU (AMD Radeon Graphics).
//   min_item_taps  estimated taps of the smallest work item
//   balance_items  items a large call is split into (about eight per
//                  resident wave), which sets the item size of large calls
//   ns_max         the entry applies to RIRs of at most this many samples
//                  (first match in table order)
//   waves          workgroups per SIMD of a persistent batch launch
//
// Score: geometric mean over the bucket's workloads of kernel time relative
// to the fastest pair on that workload (1.0 = fastest everywhere).
// W=32 fp16 nS<=8192 (room_t60_0.51_8k): best 60000 / 49152, score 1.0000, default 1.2e5 / 49152 score 1.2346
// W=32 fp16 nS<=32768 (room_t60_1.76_8k): best 120000 / 98304, score 1.0000, default 1.2e5 / 49152 score 1.0088
// W=32 fp16 nS<=2147483647 (room_t60_1.76_8k): best 120000 / 98304, score 1.0000, default 1.2e5 / 49152 score 1.0088
// W=32 fp32 nS<=8192 (room_t60_0.51_8k): best 60000 / 196608, score 1.0000, default 1.2e5 / 49152 score 1.0651
// W=32 fp32 nS<=32768 (room_t60_1.76_8k): best 120000 / 196608, score 1.0000, default 1.2e5 / 49152 score 1.0313
// W=32 fp32 nS<=2147483647 (room_t60_1.76_8k): best 120000 / 196608, score 1.0000, default 1.2e5 / 49152 score 1.0313
// W=64 fp16 nS<=8192 (room_t60_0.26_16k, batch_96_rooms_16k): best 120000 / 24576, score 1.0381, default 1.2e5 / 49152 score 1.0558
// W=64 fp16 nS<=32768 (room_t60_1.28_16k, batch_160_rooms_16k): best 240000 / 49152, score 1.0000, default 1.2e5 / 49152 score 1.0306
// W=64 fp16 nS<=2147483647 (room_t60_2.27_16k): best 480000 / 24576, score 1.0000, default 1.2e5 / 49152 score 1.0066
// W=64 fp32 nS<=8192 (room_t60_0.26_16k, batch_96_rooms_16k): best 60000 / 24576, score 1.0351, default 1.2e5 / 49152 score 1.0450
// W=64 fp32 nS<=32768 (room_t60_1.28_16k, batch_160_rooms_16k): best 120000 / 196608, score 1.0000, default 1.2e5 / 49152 score 1.0172
// W=64 fp32 nS<=2147483647 (room_t60_2.27_16k): best 240000 / 98304, score 1.0000, default 1.2e5 / 49152 score 1.0026
// W=96 fp16 nS<=8192 (room_t60_0.09_48k): best 60000 / 24576, score 1.0000, default 1.2e5 / 49152 score 1.2619
// W=96 fp16 nS<=32768 (room_t60_0.43_48k): best 60000 / 196608, score 1.0000, default 1.2e5 / 49152 score 1.0061
// W=96 fp16 nS<=2147483647 (room_t60_1.59_48k): best 240000 / 24576, score 1.0000, default 1.2e5 / 49152 score 1.0177
// W=96 fp32 nS<=8192 (room_t60_0.09_48k): best 60000 / 49152, score 1.0000, default 1.2e5 / 49152 score 1.2549
// W=96 fp32 nS<=32768 (room_t60_0.43_48k): best 120000 / 196608, score 1.0000, default 1.2e5 / 49152 score 1.0176
// W=96 fp32 nS<=2147483647 (room_t60_1.59_48k): best 240000 / 24576, score 1.0000, default 1.2e5 / 49152 score 1.0214
// W=128 fp16 nS<=8192 (room_t60_0.13_32k): best 60000 / 49152, score 1.0000, default 1.2e5 / 49152 score 1.0559
// W=128 fp16 nS<=32768 (room_t60_0.64_32k): best 120000 / 196608, score 1.0000, default 1.2e5 / 49152 score 1.0069
// W=128 fp16 nS<=2147483647 (room_t60_1.76_32k): best 240000 / 24576, score 1.0000, default 1.2e5 / 49152 score 1.0078
// W=128 fp32 nS<=8192 (room_t60_0.13_32k): best 60000 / 49152, score 1.0000, default 1.2e5 / 49152 score 1.1039
// W=128 fp32 nS<=32768 (room_t60_0.64_32k): best 240000 / 49152, score 1.0000, default 1.2e5 / 49152 score 1.0315
// W=128 fp32 nS<=2147483647 (room_t60_1.76_32k): best 240000 / 98304, score 1.0000, default 1.2e5 / 49152 score 1.0254
// W=64 fp16 batch: best 7 waves per SIMD, 4: 1.0660, 5: 1.0235, 6: 1.0050, 7: 1.0000, 8: 1.0021
// W=64 fp32 batch: best 8 waves per SIMD, 4: 1.0558, 5: 1.0156, 6: 1.0017, 7: 1.0008, 8: 1.0000
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
    {32, 1, 8192, 60000, 49152.0},
    {32, 1, 32768, 120000, 98304.0},
    {32, 1, 2147483647, 120000, 98304.0},
    {32, 0, 8192, 60000, 196608.0},
    {32, 0, 32768, 120000, 196608.0},
    {32, 0, 2147483647, 120000, 196608.0},
    {64, 1, 8192, 120000, 24576.0},
    {64, 1, 32768, 240000, 49152.0},
    {64, 1, 2147483647, 480000, 24576.0},
    {64, 0, 8192, 60000, 24576.0},
    {64, 0, 32768, 120000, 196608.0},
    {64, 0, 2147483647, 240000, 98304.0},
    {96, 1, 8192, 60000, 24576.0},
    {96, 1, 32768, 60000, 196608.0},
    {96, 1, 2147483647, 240000, 24576.0},
    {96, 0, 8192, 60000, 49152.0},
    {96, 0, 32768, 120000, 196608.0},
    {96, 0, 2147483647, 240000, 24576.0},
    {128, 1, 8192, 60000, 49152.0},
    {128, 1, 32768, 120000, 196608.0},
    {128, 1, 2147483647, 240000, 24576.0},
    {128, 0, 8192, 60000, 49152.0},
    {128, 0, 32768, 240000, 49152.0},
    {128, 0, 2147483647, 240000, 98304.0},
};

constexpr BatchTuning kBatchTuning[] = {
    {64, 1, 7},
    {64, 0, 8},
};

}  // namespace ism
