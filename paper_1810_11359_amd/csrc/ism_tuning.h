// Work-item schedule per window length, tap precision and RIR length, read by
// the host planner, and the grid of the persistent batch launch. Written by
// paper_1810_11359_amd/autotune.py from timings on the target GPU (AMD Radeon Graphics).
//   min_item_taps  estimated taps of the smallest work item
//   balance_items  items a large call is split into (about eight per
//                  resident wave), which sets the item size of large calls
//   ns_max         the entry applies to RIRs of at most this many samples
//                  (first match in table order)
//   waves          workgroups per SIMD of a persistent batch launch
//   item_taps      largest work item of a batch job (estimated taps)
//
// Score: geometric mean over the bucket's workloads of kernel time relative
// to the fastest pair on that workload (1.0 = fastest everywhere).
// W=32 fp16 nS<=8192 (room_t60_0.51_8k): best 480000 / 98304, score 1.0000, default 1.2e5 / 49152 score 1.0301
// W=32 fp16 nS<=32768 (room_t60_1.76_8k): best 120000 / 24576, score 1.0000, default 1.2e5 / 49152 score 1.0053
// W=32 fp16 nS<=2147483647 (room_t60_1.76_8k): best 120000 / 24576, score 1.0000, default 1.2e5 / 49152 score 1.0053
// W=32 fp32 nS<=8192 (room_t60_0.51_8k): best 240000 / 196608, score 1.0000, default 1.2e5 / 49152 score 1.0248
// W=32 fp32 nS<=32768 (room_t60_1.76_8k): best 240000 / 24576, score 1.0000, default 1.2e5 / 49152 score 1.0079
// W=32 fp32 nS<=2147483647 (room_t60_1.76_8k): best 240000 / 24576, score 1.0000, default 1.2e5 / 49152 score 1.0079
// W=64 fp16 nS<=8192 (room_t60_0.26_16k, batch_96_rooms_16k): best 480000 / 49152, score 1.0034, default 1.2e5 / 49152 score 1.0312
// W=64 fp16 nS<=32768 (room_t60_1.28_16k, batch_160_rooms_16k): best 120000 / 49152, score 1.0030, default 1.2e5 / 49152 score 1.0030
// W=64 fp16 nS<=2147483647 (room_t60_2.27_16k): best 60000 / 196608, score 1.0000, default 1.2e5 / 49152 score 1.0004
// W=64 fp32 nS<=8192 (room_t60_0.26_16k, batch_96_rooms_16k): best 480000 / 24576, score 1.0016, default 1.2e5 / 49152 score 1.0093
// W=64 fp32 nS<=32768 (room_t60_1.28_16k, batch_160_rooms_16k): best 120000 / 49152, score 1.0002, default 1.2e5 / 49152 score 1.0002
// W=64 fp32 nS<=2147483647 (room_t60_2.27_16k): best 240000 / 196608, score 1.0000, default 1.2e5 / 49152 score 1.0008
// W=96 fp16 nS<=8192 (room_t60_0.09_48k): best 120000 / 98304, score 1.0000, default 1.2e5 / 49152 score 1.0189
// W=96 fp16 nS<=32768 (room_t60_0.43_48k): best 480000 / 24576, score 1.0000, default 1.2e5 / 49152 score 1.0128
// W=96 fp16 nS<=2147483647 (room_t60_1.59_48k): best 240000 / 196608, score 1.0000, default 1.2e5 / 49152 score 1.0055
// W=96 fp32 nS<=8192 (room_t60_0.09_48k): best 480000 / 98304, score 1.0000, default 1.2e5 / 49152 score 1.0006
// W=96 fp32 nS<=32768 (room_t60_0.43_48k): best 480000 / 49152, score 1.0000, default 1.2e5 / 49152 score 1.0045
// W=96 fp32 nS<=2147483647 (room_t60_1.59_48k): best 120000 / 196608, score 1.0000, default 1.2e5 / 49152 score 1.0166
// W=128 fp16 nS<=8192 (room_t60_0.13_32k): best 480000 / 49152, score 1.0000, default 1.2e5 / 49152 score 1.0245
// W=128 fp16 nS<=32768 (room_t60_0.64_32k): best 120000 / 98304, score 1.0000, default 1.2e5 / 49152 score 1.0003
// W=128 fp16 nS<=2147483647 (room_t60_1.76_32k): best 480000 / 49152, score 1.0000, default 1.2e5 / 49152 score 1.0185
// W=128 fp32 nS<=8192 (room_t60_0.13_32k): best 240000 / 24576, score 1.0000, default 1.2e5 / 49152 score 1.0777
// W=128 fp32 nS<=32768 (room_t60_0.64_32k): best 120000 / 98304, score 1.0000, default 1.2e5 / 49152 score 1.0033
// W=128 fp32 nS<=2147483647 (room_t60_1.76_32k): best 240000 / 24576, score 1.0000, default 1.2e5 / 49152 score 1.0206
// W=64 fp16 batch: best 6 waves per SIMD, items <= 500000 taps; (4, 120000): 1.0820, (4, 250000): 1.0685, (4, 500000): 1.0620, (5, 120000): 1.0355, (5, 250000): 1.0236, (5, 500000): 1.0159, (6, 120000): 1.0170, (6, 250000): 1.0050, (6, 500000): 1.0000, (7, 120000): 1.0152, (7, 250000): 1.0107, (7, 500000): 1.0174, (8, 120000): 1.0154, (8, 250000): 1.0142, (8, 500000): 1.0217
// W=64 fp32 batch: best 6 waves per SIMD, items <= 500000 taps; (4, 120000): 1.0648, (4, 250000): 1.0546, (4, 500000): 1.0473, (5, 120000): 1.0243, (5, 250000): 1.0143, (5, 500000): 1.0089, (6, 120000): 1.0127, (6, 250000): 1.0059, (6, 500000): 1.0000, (7, 120000): 1.0108, (7, 250000): 1.0130, (7, 500000): 1.0185, (8, 120000): 1.0132, (8, 250000): 1.0123, (8, 500000): 1.0239
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
  double item_taps;
};

constexpr ItemTuning kItemTuning[] = {
    {32, 1, 8192, 480000, 98304.0},
    {32, 1, 32768, 120000, 24576.0},
    {32, 1, 2147483647, 120000, 24576.0},
    {32, 0, 8192, 240000, 196608.0},
    {32, 0, 32768, 240000, 24576.0},
    {32, 0, 2147483647, 240000, 24576.0},
    {64, 1, 8192, 480000, 49152.0},
    {64, 1, 32768, 120000, 49152.0},
    {64, 1, 2147483647, 60000, 196608.0},
    {64, 0, 8192, 480000, 24576.0},
    {64, 0, 32768, 120000, 49152.0},
    {64, 0, 2147483647, 240000, 196608.0},
    {96, 1, 8192, 120000, 98304.0},
    {96, 1, 32768, 480000, 24576.0},
    {96, 1, 2147483647, 240000, 196608.0},
    {96, 0, 8192, 480000, 98304.0},
    {96, 0, 32768, 480000, 49152.0},
    {96, 0, 2147483647, 120000, 196608.0},
    {128, 1, 8192, 480000, 49152.0},
    {128, 1, 32768, 120000, 98304.0},
    {128, 1, 2147483647, 480000, 49152.0},
    {128, 0, 8192, 240000, 24576.0},
    {128, 0, 32768, 120000, 98304.0},
    {128, 0, 2147483647, 240000, 24576.0},
};

constexpr BatchTuning kBatchTuning[] = {
    {64, 1, 6, 500000},
    {64, 0, 6, 500000},
};

}  // namespace ism
