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
// W=32 fp16 nS<=8192 (room_t60_0.51_8k): best 60000 / 49152, score 1.0000, default 1.2e5 / 49152 score 1.0350
// W=32 fp16 nS<=32768 (room_t60_1.76_8k): best 120000 / 98304, score 1.0000, default 1.2e5 / 49152 score 1.0028
// W=32 fp16 nS<=2147483647 (room_t60_1.76_8k): best 120000 / 98304, score 1.0000, default 1.2e5 / 49152 score 1.0028
// W=32 fp32 nS<=8192 (room_t60_0.51_8k): best 480000 / 196608, score 1.0000, default 1.2e5 / 49152 score 1.0535
// W=32 fp32 nS<=32768 (room_t60_1.76_8k): best 120000 / 49152, score 1.0000, default 1.2e5 / 49152 score 1.0000
// W=32 fp32 nS<=2147483647 (room_t60_1.76_8k): best 120000 / 49152, score 1.0000, default 1.2e5 / 49152 score 1.0000
// W=64 fp16 nS<=8192 (room_t60_0.26_16k, batch_96_rooms_16k): best 480000 / 196608, score 1.0265, default 1.2e5 / 49152 score 1.0475
// W=64 fp16 nS<=32768 (room_t60_1.28_16k, batch_160_rooms_16k): best 120000 / 49152, score 1.0041, default 1.2e5 / 49152 score 1.0041
// W=64 fp16 nS<=2147483647 (room_t60_2.27_16k): best 240000 / 49152, score 1.0000, default 1.2e5 / 49152 score 1.0114
// W=64 fp32 nS<=8192 (room_t60_0.26_16k, batch_96_rooms_16k): best 240000 / 24576, score 1.0298, default 1.2e5 / 49152 score 1.0309
// W=64 fp32 nS<=32768 (room_t60_1.28_16k, batch_160_rooms_16k): best 120000 / 98304, score 1.0061, default 1.2e5 / 49152 score 1.0119
// W=64 fp32 nS<=2147483647 (room_t60_2.27_16k): best 120000 / 49152, score 1.0000, default 1.2e5 / 49152 score 1.0000
// W=96 fp16 nS<=8192 (room_t60_0.09_48k): best 120000 / 49152, score 1.0000, default 1.2e5 / 49152 score 1.0000
// W=96 fp16 nS<=32768 (room_t60_0.43_48k): best 480000 / 196608, score 1.0000, default 1.2e5 / 49152 score 1.0190
// W=96 fp16 nS<=2147483647 (room_t60_1.59_48k): best 240000 / 196608, score 1.0000, default 1.2e5 / 49152 score 1.0005
// W=96 fp32 nS<=8192 (room_t60_0.09_48k): best 120000 / 49152, score 1.0000, default 1.2e5 / 49152 score 1.0000
// W=96 fp32 nS<=32768 (room_t60_0.43_48k): best 480000 / 49152, score 1.0000, default 1.2e5 / 49152 score 1.0293
// W=96 fp32 nS<=2147483647 (room_t60_1.59_48k): best 240000 / 196608, score 1.0000, default 1.2e5 / 49152 score 1.0095
// W=128 fp16 nS<=8192 (room_t60_0.13_32k): best 120000 / 196608, score 1.0000, default 1.2e5 / 49152 score 1.0084
// W=128 fp16 nS<=32768 (room_t60_0.64_32k): best 240000 / 24576, score 1.0000, default 1.2e5 / 49152 score 1.0149
// W=128 fp16 nS<=2147483647 (room_t60_1.76_32k): best 240000 / 98304, score 1.0000, default 1.2e5 / 49152 score 1.0155
// W=128 fp32 nS<=8192 (room_t60_0.13_32k): best 120000 / 196608, score 1.0000, default 1.2e5 / 49152 score 1.0633
// W=128 fp32 nS<=32768 (room_t60_0.64_32k): best 480000 / 49152, score 1.0000, default 1.2e5 / 49152 score 1.0116
// W=128 fp32 nS<=2147483647 (room_t60_1.76_32k): best 240000 / 196608, score 1.0000, default 1.2e5 / 49152 score 1.0148
// W=64 fp16 batch: best 6 waves per SIMD, items <= 500000 taps; (4, 120000): 1.1133, (4, 250000): 1.0950, (4, 500000): 1.0922, (5, 120000): 1.0367, (5, 250000): 1.0270, (5, 500000): 1.0213, (6, 120000): 1.0175, (6, 250000): 1.0030, (6, 500000): 1.0000, (7, 120000): 1.0160, (7, 250000): 1.0047, (7, 500000): 1.0164, (8, 120000): 1.0082, (8, 250000): 1.0082, (8, 500000): 1.0170
// W=64 fp32 batch: best 6 waves per SIMD, items <= 250000 taps; (4, 120000): 1.0939, (4, 250000): 1.0810, (4, 500000): 1.0756, (5, 120000): 1.0303, (5, 250000): 1.0158, (5, 500000): 1.0148, (6, 120000): 1.0135, (6, 250000): 1.0000, (6, 500000): 1.0003, (7, 120000): 1.0092, (7, 250000): 1.0070, (7, 500000): 1.0190, (8, 120000): 1.0100, (8, 250000): 1.0106, (8, 500000): 1.0187
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
    {32, 1, 8192, 60000, 49152.0},
    {32, 1, 32768, 120000, 98304.0},
    {32, 1, 2147483647, 120000, 98304.0},
    {32, 0, 8192, 480000, 196608.0},
    {32, 0, 32768, 120000, 49152.0},
    {32, 0, 2147483647, 120000, 49152.0},
    {64, 1, 8192, 480000, 196608.0},
    {64, 1, 32768, 120000, 49152.0},
    {64, 1, 2147483647, 240000, 49152.0},
    {64, 0, 8192, 240000, 24576.0},
    {64, 0, 32768, 120000, 98304.0},
    {64, 0, 2147483647, 120000, 49152.0},
    {96, 1, 8192, 120000, 49152.0},
    {96, 1, 32768, 480000, 196608.0},
    {96, 1, 2147483647, 240000, 196608.0},
    {96, 0, 8192, 120000, 49152.0},
    {96, 0, 32768, 480000, 49152.0},
    {96, 0, 2147483647, 240000, 196608.0},
    {128, 1, 8192, 120000, 196608.0},
    {128, 1, 32768, 240000, 24576.0},
    {128, 1, 2147483647, 240000, 98304.0},
    {128, 0, 8192, 120000, 196608.0},
    {128, 0, 32768, 480000, 49152.0},
    {128, 0, 2147483647, 240000, 196608.0},
};

constexpr BatchTuning kBatchTuning[] = {
    {64, 1, 6, 500000},
    {64, 0, 6, 250000},
};

}  // namespace ism
