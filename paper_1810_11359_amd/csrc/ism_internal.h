// Internal types shared by the host planner (ism_host.cpp) and the HIP kernels
// (ism_device.hip). Not part of the public ABI.
#pragma once

#include <stdint.h>

namespace ism {

// Tiles partition the integer delays k0 = floor(x) of the images: tile t owns
// the images with k0 in [t*TILE, (t+1)*TILE) and writes output samples
// [t*TILE, (t+1)*TILE) plus two margins, the W/2 - 1 samples before and the
// W/2 samples after, which belong to the neighbouring tiles.
constexpr int TILE = 256;
// Most tiles per RIR: ceil((ISM_MAX_SAMPLES + 128/2 - 1) / TILE).
constexpr int MAX_TILES = 1025;
// Dispatch positions per block of the plan's coarse first-item table.
constexpr int PLAN_BLK = 16;
// Batch margin records are addressed in units of MARG_UNIT floats (window caps
// are multiples of it); a record of a job with window cap WT holds WT floats.
constexpr int MARG_UNIT = 32;
// Window caps: the kernels are built for caps WT = 32, 64, ..., 256 samples.
// An even integer window W in {32, 64, 96, 128} runs with compile-time tap
// constants (exact mode); any other W <= 256 runs with the next cap and
// per-call constants, masking the taps outside |j - f| < W/2 (general mode).
constexpr int MAX_WINDOW = 256;
// Per-tap constants of a general-mode window, 8 floats per tap jj of the cap:
// FP32 taps (-sigma, sigma j, cos(2 pi j / W), sin(2 pi j / W), 0 ...),
// FP16 taps (c0, c1, ..., c5, 0, 0) of the tap's interpolant.
constexpr int WC_STRIDE = 8;
// Reduce kernels: a run of at least RED_SLICE_MIN partials or margins of one
// sample is summed as RED_SLICES consecutive slices (each in order from its
// first term, then the slice sums in order); shorter runs term by term. The
// order depends on the run length only; launches whose runs are all shorter
// use one thread per sample, others RED_SLICES threads per sample.
constexpr int RED_SLICES = 4;
constexpr int RED_SLICE_MIN = 64;
// Window classes (cap, mode) one batch may hold: one persistent launch each.
constexpr int kMaxBatchClasses = 8;
// Work items per tile are capped so the per-tile chunk count fits a byte.
constexpr int MAX_CHUNKS = 255;
// Waves per SIMD the accumulate kernels are built for (their LDS and VGPR
// budget); the planner sizes the tail taper of a launch with it.
constexpr int kAccWavesPerSimd = 7;

// Per-call room constants, passed by value as a kernel argument. Lengths are in
// metres, delays in samples. Float-float pairs (hi, lo) carry double-precision
// host values into FP32-only device arithmetic. The per-axis arrays are in
// table-axis order: table axis k is room axis perm[k], with the room's
// shortest side last (the innermost enumeration axis, whose columns then
// hold the most images).
struct RoomArgs {
  int perm[3];             // room axis of each table axis
  float L_hi[3], L_lo[3];  // room size
  float beta[6];           // x0, x1, y0, y1, z0, z1 (high part of a float-float pair)
  float beta_lo[6];        // low parts: beta = beta + beta_lo to about 48 bits
  int lo[3];               // first lattice index ceil(-N/2) per axis
  int N[3];                // lattice size per axis
  int off[3];              // offset of each axis in the per-RIR table
  int n_tab;               // Nx + Ny + Nz
  float q_hi, q_lo;        // fs / c [samples per metre]
  float kappa;             // fs / (4 pi c): A = gain * kappa / x with x in samples
  float half_w;            // WT / 2, WT the window cap (layout of tiles and margins)
  float win_hw;            // W / 2, W = t_w fs the window [samples]
  float inv_win;           // 1 / W
  int gen;                 // 1: general-mode window (per-call tap constants, masked taps)
  int n_samples;           // nS
  int k_end;               // nS + W/2 - 1: images with k0 >= k_end add nothing
  int n_src, n_rcv;
  float period[3];         // 2 L q: displacement step between images of one parity [samples]
  float inv_period[3];     // 1 / period
  float dir_a, dir_b;      // receiver polar pattern a + b cos(theta) (b = 1 - a); polar calls only
};

// Work decomposition of one call. Items are ordered by tile (last tile first,
// where the images are densest), then by RIR, then by chunk. Tile t owns the
// images with k0 in [t*TILE, min((t+1)*TILE, k_end)); that shell is split into
// chunks[t] slabs along the x displacement.
// The first item of dispatch position pos (tile n_tiles - 1 - pos) is
// first_blk[pos / PLAN_BLK] plus n_rir * chunks of the positions before pos in
// its block (plan_first_item); the compact form keeps the plan a kernel argument.
struct PlanArgs {
  int n_tiles;
  int n_rir;
  uint32_t first_blk[(MAX_TILES + PLAN_BLK) / PLAN_BLK + 1];
  uint8_t chunks[MAX_TILES];  // chunks per tile (by tile index)
};

// Per-RIR table entry for one lattice index of one axis: square of the
// displacement from the receiver to the image coordinate, in samples^2
// (float-float, low part not renormalised), the axis factor of the
// reflection gain, and (polar calls) the displacement times the receiver's
// unit orientation along this axis, in samples (0 otherwise).
struct AxisEntry {
  float sq_hi, sq_lo, gain, proj;
};

// Per-RIR offsets of the two image families of each axis, in samples: even
// n = 2m sits at m*period + e_even, odd n = 2m - 1 at m*period + e_odd.
struct AxisOrigin {
  float e_even[3], e_odd[3];
};

// Batch mode: one entry per job (room) of a batch, uploaded once per prepared
// batch. Pointers are device pointers owned by the caller.
struct JobDev {
  RoomArgs ra;  // dir_a = 1, dir_b = 0 for omnidirectional jobs
  const float *src;
  const float *rcv;
  float *out;
  const float *orient;  // receiver orientations, or null (omnidirectional)
  float *wc;            // general-mode window constants [WT][WC_STRIDE], or null
  uint64_t tab_base;    // first table entry of the job's first RIR
  uint32_t rir_base;    // batch-wide index of the job's first RIR
  uint32_t pad;
};

// Batch-wide RIR index -> (job, RIR within the job).
struct BatchRir {
  uint32_t job, rir;
};

// One work item of a batch (same meaning as in single-room mode). slot is the
// partial tile written when the tile is split (chunks > 1), else 0xffffffff;
// mslot is the offset of its margin record in units of MARG_UNIT floats.
struct BatchItem {
  uint32_t job, rir;
  uint16_t tile;
  uint8_t chunk, chunks;
  uint32_t slot;
  uint32_t mslot;
};

// One output tile of a batch RIR: its own partials (slots first ..
// first + chunks - 1 when chunks > 1) and the margin records of the items of
// the previous and next tile (nprev records from offset mprev, nnext from
// mnext, in units of MARG_UNIT floats, consecutive records WT floats apart;
// counts are 0 where there is no such tile).
struct BatchReduce {
  uint32_t job, rir;
  uint16_t tile, chunks;
  uint32_t first;
  uint32_t mprev, mnext;
  uint16_t nprev, nnext;
};

// Enumeration check (test entry ism_debug_enumerate): one record per image a
// work item owns, with the lattice index n per room axis, k0 = floor(x), the
// delay fraction fq in units of 2^-24 and the Eq. (4) amplitude in FP32.
struct DumpRec {
  int32_t rir;
  int32_t n[3];
  int32_t k0;
  uint32_t fq;
  float A;
  uint32_t pad;
};
struct DumpArgs {
  DumpRec *rec;
  uint32_t *count;  // records produced (may exceed cap; only cap are stored)
  uint32_t cap;
};

// Workspace layout of one FFT filter call (offsets in bytes): block size B,
// transform size N = 2B, RIR partitions P, pieces per input block R, segment
// length L, input and output block counts.
struct FftPlan {
  int B, N, P, R, n_in_blocks, n_out_blocks, L;
  size_t off_tw, off_H, off_X, off_Y, off_z, bytes;
};

}  // namespace ism
