// Moving-source filtering (Sec. 3.4): a source signal x is cut into n_pos
// consecutive segments of seg_len = ceil(n_x / n_pos) samples (the last one
// shorter when n_pos does not divide n_x); segment p is convolved with the RIR
// of trajectory point p to each microphone and the results are added at the
// segment's offset (overlap-add). Equivalently, for microphone m,
//   y_m[n] = sum_k x[n - k] h_{p(n - k), m}[k],   p(i) = floor(i / seg_len),
// a filter that changes with the segment of the input sample. The paper runs
// this with batched FFTs; here it is a direct sum: the RIRs of one point are
// short next to the signal, the sum has no plan or work area, and every
// output is added in a fixed order (bitwise reproducible).
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace ism {

constexpr int FT = 256;       // threads per block
constexpr int FR = 4;         // consecutive outputs per thread
constexpr int FN = FT * FR;   // outputs per block
constexpr int FK = 256;       // filter taps per chunk
constexpr int FJ = 64;        // taps per sub-chunk (the unit a wave skips)
constexpr int FW = 64 * FR;   // outputs per wave
constexpr int XPAD = 1;       // zero slot in front of the staged input window (aligns the 16-byte reads)

// XCDs of the device: consecutive workgroups are dispatched to them in turn.
constexpr int kXcds = 8;

// grid = ceil(n_y / FN) x n_mic blocks, one dimension. Block b runs on XCD
// b % 8; it takes logical block (b % 8) * ceil(G / 8) + b / 8 (G blocks in
// all), so each XCD works through a contiguous run of output blocks of one
// microphone, which read the same RIR chunks: that reuse stays in the XCD's
// L2 instead of being fetched once per XCD. Logical block L covers outputs
// [(L % gx) FN, +FN) of microphone L / gx. For each chunk of FK taps and each segment
// the chunk's input window touches, the block stages the window (input
// samples of other segments zeroed) and the segment's FK taps in LDS; a
// thread keeps its 4 outputs in registers and slides a 4-sample input window
// down the taps (one 16-byte input read and one 16-byte tap read per 16
// FMAs). A wave skips each sub-chunk of FJ taps whose inputs, for its FW
// outputs, all lie outside the staged segment (or whose taps are past the
// RIR's end): those products are all zero, so skipping them leaves every sum
// unchanged and removes most of the work on zeroed samples, since a wave's
// input range is short next to a segment.
__global__ __launch_bounds__(FT) void filter_kernel(const float *__restrict__ x, int n_x,
                                                    const float *__restrict__ rir, int n_mic, int n_rir,
                                                    int seg_len, float *__restrict__ y, int n_y, int gx) {
  const int G = gx * n_mic;
  const int per_xcd = (G + kXcds - 1) / kXcds;
  const int L = (int)(blockIdx.x % kXcds) * per_xcd + (int)(blockIdx.x / kXcds);
  if (L >= G) return;  // uniform over the block
  const int m = L / gx;
  const int n0 = (L % gx) * FN;
  const int tid = threadIdx.x;
  __shared__ __attribute__((aligned(16))) float xs[XPAD + FN + FK];
  __shared__ __attribute__((aligned(16))) float hs[FK];
  float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
  if (tid < XPAD) xs[tid] = 0.0f;
  // input index of window slot w: i = n0 - kc - FK + 1 + w; output n = n0 + FR tid + r
  // with tap k = kc + j reads slot FR tid + r + FK - 1 - j
  const int base = XPAD + FR * tid + FK - 1;
  // first output of this thread's wave (uniform over the wave)
  const int nw = __builtin_amdgcn_readfirstlane(n0 + FW * (tid / 64));
  typedef float f4 __attribute__((ext_vector_type(4)));
  for (int kc = 0; kc < n_rir; kc += FK) {
    const int i_lo = n0 - kc - FK + 1;
    const int lo = max(i_lo, 0), hi = min(n0 + FN - 1 - kc, n_x - 1);
    if (lo > hi) continue;  // uniform over the block
    for (int p = lo / seg_len; p <= hi / seg_len; ++p) {
      const int s0 = p * seg_len, s1 = min(s0 + seg_len, n_x);
      __syncthreads();  // the previous segment's window is used up
      for (int w = tid; w < FN + FK - 1; w += FT) {
        const int i = i_lo + w;
        xs[XPAD + w] = (i >= s0 && i < s1) ? x[i] : 0.0f;
      }
      const float *h = rir + ((size_t)p * n_mic + m) * n_rir;
      for (int j = tid; j < FK; j += FT) hs[j] = (kc + j < n_rir) ? h[kc + j] : 0.0f;
      __syncthreads();
      for (int jb = 0; jb < FK; jb += FJ) {
        // the wave's outputs [nw, nw + FW) read inputs [ilo, ihi] for these taps
        const int ilo = nw - kc - jb - FJ + 1, ihi = nw + FW - 1 - kc - jb;
        if (ihi < s0 || ilo >= s1 || kc + jb >= n_rir) continue;  // uniform over the wave
        const f4 v = *reinterpret_cast<const f4 *>(&xs[base - jb]);
        float v0 = v.x, v1 = v.y, v2 = v.z, v3 = v.w;
        // two-level sums: the FJ products of a sub-chunk, then the sub-chunk
        // sums, so rounding grows as sqrt(FJ) + sqrt(n_rir / FJ) instead of
        // sqrt(n_rir) over an output's n_rir products
        float b0 = 0.0f, b1 = 0.0f, b2 = 0.0f, b3 = 0.0f;
#pragma unroll 4
        for (int j = jb; j < jb + FJ; j += 4) {
          const f4 t = *reinterpret_cast<const f4 *>(&hs[j]);
          // u.w, u.z, u.y, u.x = inputs one, two, three, four slots before v0
          const f4 u = *reinterpret_cast<const f4 *>(&xs[base - j - 4]);
          b0 = __builtin_fmaf(v0, t.x, b0); b0 = __builtin_fmaf(u.w, t.y, b0);
          b0 = __builtin_fmaf(u.z, t.z, b0); b0 = __builtin_fmaf(u.y, t.w, b0);
          b1 = __builtin_fmaf(v1, t.x, b1); b1 = __builtin_fmaf(v0, t.y, b1);
          b1 = __builtin_fmaf(u.w, t.z, b1); b1 = __builtin_fmaf(u.z, t.w, b1);
          b2 = __builtin_fmaf(v2, t.x, b2); b2 = __builtin_fmaf(v1, t.y, b2);
          b2 = __builtin_fmaf(v0, t.z, b2); b2 = __builtin_fmaf(u.w, t.w, b2);
          b3 = __builtin_fmaf(v3, t.x, b3); b3 = __builtin_fmaf(v2, t.y, b3);
          b3 = __builtin_fmaf(v1, t.z, b3); b3 = __builtin_fmaf(v0, t.w, b3);
          v3 = u.w; v2 = u.z; v1 = u.y; v0 = u.x;
        }
        a0 += b0;
        a1 += b1;
        a2 += b2;
        a3 += b3;
      }
    }
  }
  const int nb = n0 + FR * tid;
  float *ym = y + (size_t)m * n_y;
  if (nb < n_y) ym[nb] = a0;
  if (nb + 1 < n_y) ym[nb + 1] = a1;
  if (nb + 2 < n_y) ym[nb + 2] = a2;
  if (nb + 3 < n_y) ym[nb + 3] = a3;
}

int launch_filter(const float *x, int n_x, const float *rir, int n_pos, int n_mic, int n_rir, float *y,
                  hipStream_t st) {
  const int seg_len = (n_x + n_pos - 1) / n_pos;
  const int n_y = n_x + n_rir - 1;
  const int gx = (n_y + FN - 1) / FN;
  if ((int64_t)gx * n_mic > (int64_t)0x7fffff00) return -2;  // block count beyond a grid dimension
  const int G = gx * n_mic;
  const int per_xcd = (G + kXcds - 1) / kXcds;
  hipLaunchKernelGGL(filter_kernel, dim3((unsigned)(per_xcd * kXcds)), dim3(FT), 0, st, x, n_x, rir, n_mic, n_rir,
                     seg_len, y, n_y, gx);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace ism
