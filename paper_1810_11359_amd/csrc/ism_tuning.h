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
// W=32 fp16 nS<=8192 (room_t60_0.51_8k): best 60000 / 98304, score 1.0000, default 1.2e5 / 49152 score 1.2394
// W=32 fp16 nS<=32768 (room_t60_1.76_8k): best 120000 / 98304, score 1.0000, default 1.2e5 / 49152 score 1.0026
// W=32 fp16 nS<=2147483647 (room_t60_1.76_8k): best 120000 / 98304, score 1.0000, default 1.2e5 / 49152 score 1.0026
// W=32 fp32 nS<=8192 (room_t60_0.51_8k): best 60000 / 98304, score 1.0000, default 1.2e5 / 49152 score 1.0533
// W=32 fp32 nS<=32768 (room_t60_1.76_8k): best 120000 / 49152, score 1.0000, default 1.2e5 / 49152 score 1.0000
// W=32 fp32 nS<=2147483647 (room_t60_1.76_8k): best 120000 / 49152, score 1.0000, default 1.2e5 / 49152 score 1.0000
// W=64 fp16 nS<=8192 (room_t60_0.26_16k, batch_96_rooms_16k): best 120000 / 24576, score 1.0285, default 1.2e5 / 49152 score 1.0336
// W=64 fp16 nS<=32768 (room_t60_1.28_16k, batch_160_rooms_16k): best 120000 / 196608, score 1.0014, default 1.2e5 / 49152 score 1.0219
// W=64 fp16 nS<=2147483647 (room_t60_2.27_16k): best 240000 / 196608, score 1.0000, default 1.2e5 / 49152 score 1.0072
// W=64 fp32 nS<=8192 (room_t60_0.26_16k, batch_96_rooms_16k): best 120000 / 98304, score 1.0582, default 1.2e5 / 49152 score 1.0589
// W=64 fp32 nS<=32768 (room_t60_1.28_16k, batch_160_rooms_16k): best 120000 / 196608, score 1.0022, default 1.2e5 / 49152 score 1.0145
// W=64 fp32 nS<=2147483647 (room_t60_2.27_16k): best 240000 / 196608, score 1.0000, default 1.2e5 / 49152 score 1.0085
// W=96 fp16 nS<=8192 (room_t60_0.09_48k): best 60000 / 24576, score 1.0000, default 1.2e5 / 49152 score 1.2479
// W=96 fp16 nS<=32768 (room_t60_0.43_48k): best 60000 / 49152, score 1.0000, default 1.2e5 / 49152 score 1.0140
// W=96 fp16 nS<=2147483647 (room_t60_1.59_48k): best 240000 / 49152, score 1.0000, default 1.2e5 / 49152 score 1.0073
// W=96 fp32 nS<=8192 (room_t60_0.09_48k): best 60000 / 24576, score 1.0000, default 1.2e5 / 49152 score 1.2646
// W=96 fp32 nS<=32768 (room_t60_0.43_48k): best 120000 / 196608, score 1.0000, default 1.2e5 / 49152 score 1.0014
// W=96 fp32 nS<=2147483647 (room_t60_1.59_48k): best 240000 / 98304, score 1.0000, default 1.2e5 / 49152 score 1.0110
// W=128 fp16 nS<=8192 (room_t60_0.13_32k): best 60000 / 196608, score 1.0000, default 1.2e5 / 49152 score 1.0995
// W=128 fp16 nS<=32768 (room_t60_0.64_32k): best 240000 / 196608, score 1.0000, default 1.2e5 / 49152 score 1.0131
// W=128 fp16 nS<=2147483647 (room_t60_1.76_32k): best 240000 / 98304, score 1.0000, default 1.2e5 / 49152 score 1.0097
// W=128 fp32 nS<=8192 (room_t60_0.13_32k): best 60000 / 98304, score 1.0000, default 1.2e5 / 49152 score 1.2114
// W=128 fp32 nS<=32768 (room_t60_0.64_32k): best 240000 / 24576, score 1.0000, default 1.2e5 / 49152 score 1.0073
// W=128 fp32 nS<=2147483647 (room_t60_1.76_32k): best 240000 / 196608, score 1.0000, default 1.2e5 / 49152 score 1.0084
// W=64 fp16 batch: best 6 waves per SIMD, items <= 500000 taps; (4, 120000): 1.1100, (4, 250000): 1.0953, (4, 500000): 1.0925, (5, 120000): 1.0375, (5, 250000): 1.0242, (5, 500000): 1.0153, (6, 120000): 1.0101, (6, 250000): 1.0039, (6, 500000): 1.0000, (7, 120000): 1.0117, (7, 250000): 1.0100, (7, 500000): 1.0180, (8, 120000): 1.0117, (8, 250000): 1.0077, (8, 500000): 1.0166
// W=64 fp32 batch: best 6 waves per SIMD, items <= 500000 taps; (4, 120000): 1.0957, (4, 250000): 1.0878, (4, 500000): 1.0799, (5, 120000): 1.0364, (5, 250000): 1.0244, (5, 500000): 1.0148, (6, 120000): 1.0153, (6, 250000): 1.0043, (6, 500000): 1.0000, (7, 120000): 1.0102, (7, 250000): 1.0113, (7, 500000): 1.0179, (8, 120000): 1.0128, (8, 250000): 1.0167, (8, 500000): 1.0281
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
    {32, 1, 8192, 60000, 98304.0},
    {32, 1, 32768, 120000, 98304.0},
    {32, 1, 2147483647, 120000, 98304.0},
    {32, 0, 8192, 60000, 98304.0},
    {32, 0, 32768, 120000, 49152.0},
    {32, 0, 2147483647, 120000, 49152.0},
    {64, 1, 8192, 120000, 24576.0},
    {64, 1, 32768, 120000, 196608.0},
    {64, 1, 2147483647, 240000, 196608.0},
    {64, 0, 8192, 120000, 98304.0},
    {64, 0, 32768, 120000, 196608.0},
    {64, 0, 2147483647, 240000, 196608.0},
    {96, 1, 8192, 60000, 24576.0},
    {96, 1, 32768, 60000, 49152.0},
    {96, 1, 2147483647, 240000, 49152.0},
    {96, 0, 8192, 60000, 24576.0},
    {96, 0, 32768, 120000, 196608.0},
    {96, 0, 2147483647, 240000, 98304.0},
    {128, 1, 8192, 60000, 196608.0},
    {128, 1, 32768, 240000, 196608.0},
    {128, 1, 2147483647, 240000, 98304.0},
    {128, 0, 8192, 60000, 98304.0},
    {128, 0, 32768, 240000, 24576.0},
    {128, 0, 2147483647, 240000, 196608.0},
};

constexpr BatchTuning kBatchTuning[] = {
    {64, 1, 6, 500000},
    {64, 0, 6, 500000},
};

}  // namespace ism
