// Moving-source filtering (Sec. 3.4) by partitioned FFT convolution: the
// paper filters the signal through the trajectory's RIRs with batched FFTs;
// this is that path, written for gfx950 (radix-2 Stockham transforms in LDS).
//
// The signal x is cut into segments of L = ceil(n_x / n_pos) samples and
// segment p goes through RIR p (y_m[n] = sum_k x[n - k] h_{p(n-k), m}[k]).
// With blocks of B samples (N = 2B point transforms):
//   - RIR partition q of point p and microphone m, h_{p,m}[qB, qB + B), has
//     the spectrum H[p][m][q];
//   - input block i, x[iB, iB + B), is split into pieces, one per segment it
//     touches (samples of other segments zeroed); piece r (segment p0(i) + r)
//     has the spectrum X[i][r];
//   - piece (i, r) times partition q is the linear convolution of two B-sample
//     sequences placed at (i + q) B: 2B - 1 samples, exact in an N-point
//     circular convolution. Output block b collects, in the frequency domain,
//     Y[m][b] = sum_q sum_r X[b - q][r] H[p(b - q, r)][m][q] (q, then r, in
//     increasing order), and
//   - y_m[bB + t] = z_b[t] + z_{b-1}[B + t], z_b = IFFT(Y[m][b]) (overlap-add).
// Every sum has a fixed order, so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "ism_internal.h"
#include "ism_math.h"

namespace ism {

constexpr int FFT_MAX = 8192;   // largest transform (points)
constexpr int FFT_THREADS = 256;

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(__builtin_fmaf(a.x, b.x, -a.y * b.y), __builtin_fmaf(a.x, b.y, a.y * b.x));
}

// tw[t] = exp(-2 pi i t / N), t < N/2
__global__ __launch_bounds__(256) void fft_twiddle_kernel(float2 *__restrict__ tw, int N) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < N / 2; t += gridDim.x * blockDim.x) {
    float s, c;
    sincospi_acc(-2.0f * (float)t / (float)N, s, c);
    tw[t] = make_float2(c, s);
  }
}

// N-point transform (N a power of two, <= FFT_MAX) of a[0 .. N) in LDS, with
// b[0 .. N) as scratch, by radix-2 Stockham stages: stage of span Ns reads
// a[j], a[j + N/2] and writes the butterfly of twiddle exp(-+2 pi i k /
// (2 Ns)), k = j mod Ns, to positions 2 (j - k) + k and + Ns; after log2 N
// stages the result is in natural order. inverse: conjugate twiddles (no
// 1/N). Returns the buffer that holds the result.
__device__ float2 *lds_fft(float2 *a, float2 *b, int N, const float2 *__restrict__ tw, bool inverse) {
  for (int Ns = 1; Ns < N; Ns <<= 1) {
    __syncthreads();
    const int step = N / (2 * Ns);
    for (int j = threadIdx.x; j < N / 2; j += blockDim.x) {
      const int k = j & (Ns - 1);
      float2 w = tw[k * step];
      if (inverse) w.y = -w.y;
      const float2 u = a[j], v = cmul(a[j + N / 2], w);
      const int o = 2 * (j - k) + k;
      b[o] = make_float2(u.x + v.x, u.y + v.y);
      b[o + Ns] = make_float2(u.x - v.x, u.y - v.y);
    }
    float2 *t = a;
    a = b;
    b = t;
  }
  __syncthreads();
  return a;
}

// Spectra of the RIR partitions: block (p * n_mic + m) * P + q.
__global__ __launch_bounds__(FFT_THREADS) void fft_rir_kernel(const float *__restrict__ rir, int n_rir, int B,
                                                            int N, int P, const float2 *__restrict__ tw,
                                                            float2 *__restrict__ H) {
  __shared__ float2 buf[2][FFT_MAX];
  const int row = blockIdx.x;
  const int q = row % P;
  const float *h = rir + (size_t)(row / P) * n_rir + (size_t)q * B;
  const int len = min(B, n_rir - q * B);
  for (int t = threadIdx.x; t < N; t += blockDim.x) buf[0][t] = make_float2(t < len ? h[t] : 0.0f, 0.0f);
  const float2 *r = lds_fft(buf[0], buf[1], N, tw, false);
  float2 *o = H + (size_t)row * N;
  for (int t = threadIdx.x; t < N; t += blockDim.x) o[t] = r[t];
}

// Segment of input block i's piece r, or -1 when the piece is empty.
__device__ __forceinline__ int piece_segment(int i, int r, int B, int L, int n_x, int n_pos) {
  const int lo = i * B, hi = min(lo + B, n_x);  // samples [lo, hi)
  const int p = lo / L + r;
  if (p >= n_pos || p * L >= hi) return -1;
  return p;
}

// Spectra of the input pieces: block i * R + r.
__global__ __launch_bounds__(FFT_THREADS) void fft_input_kernel(const float *__restrict__ x, int n_x, int n_pos,
                                                              int L, int B, int N, int R,
                                                              const float2 *__restrict__ tw, float2 *__restrict__ X) {
  __shared__ float2 buf[2][FFT_MAX];
  const int i = blockIdx.x / R, r = blockIdx.x % R;
  const int p = piece_segment(i, r, B, L, n_x, n_pos);
  float2 *o = X + (size_t)blockIdx.x * N;
  if (p < 0) {  // uniform over the block; the spectrum is never read
    return;
  }
  const int s0 = p * L, s1 = min(s0 + L, n_x);
  for (int t = threadIdx.x; t < N; t += blockDim.x) {
    const int n = i * B + t;
    buf[0][t] = make_float2((t < B && n >= s0 && n < s1) ? x[n] : 0.0f, 0.0f);
  }
  const float2 *res = lds_fft(buf[0], buf[1], N, tw, false);
  for (int t = threadIdx.x; t < N; t += blockDim.x) o[t] = res[t];
}

// Y[m][b][k] = sum over q, then r of X[b - q][r][k] H[p][m][q][k].
// grid = (N / 256, n_out_blocks, n_mic).
__global__ __launch_bounds__(256) void spectrum_mac_kernel(const float2 *__restrict__ X, const float2 *__restrict__ H,
                                                           int n_x, int n_pos, int n_mic, int L, int B, int N, int P,
                                                           int R, int n_in_blocks, float2 *__restrict__ Y) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y, m = blockIdx.z;
  float2 acc = make_float2(0.0f, 0.0f);
  for (int q = 0; q < P; ++q) {
    const int i = b - q;
    if (i < 0) break;
    if (i >= n_in_blocks) continue;
    for (int r = 0; r < R; ++r) {
      const int p = piece_segment(i, r, B, L, n_x, n_pos);
      if (p < 0) continue;  // uniform over the block
      const float2 xv = X[((size_t)i * R + r) * N + k];
      const float2 hv = H[(((size_t)p * n_mic + m) * P + q) * N + k];
      acc.x = __builtin_fmaf(xv.x, hv.x, acc.x);
      acc.x = __builtin_fmaf(-xv.y, hv.y, acc.x);
      acc.y = __builtin_fmaf(xv.x, hv.y, acc.y);
      acc.y = __builtin_fmaf(xv.y, hv.x, acc.y);
    }
  }
  Y[((size_t)m * gridDim.y + b) * N + k] = acc;
}

// z[m][b] = real part of IFFT(Y[m][b]) / N; block m * n_out_blocks + b.
__global__ __launch_bounds__(FFT_THREADS) void ifft_block_kernel(const float2 *__restrict__ Y, int N,
                                                               const float2 *__restrict__ tw, float *__restrict__ z) {
  __shared__ float2 buf[2][FFT_MAX];
  const float2 *in = Y + (size_t)blockIdx.x * N;
  for (int t = threadIdx.x; t < N; t += blockDim.x) buf[0][t] = in[t];
  const float2 *res = lds_fft(buf[0], buf[1], N, tw, true);
  const float inv_n = 1.0f / (float)N;
  float *o = z + (size_t)blockIdx.x * N;
  for (int t = threadIdx.x; t < N; t += blockDim.x) o[t] = res[t].x * inv_n;
}

// y[m][bB + t] = z[m][b][t] + z[m][b - 1][B + t]; grid = (ceil(n_y / 256), n_mic).
__global__ __launch_bounds__(256) void overlap_add_kernel(const float *__restrict__ z, int B, int N, int n_out_blocks,
                                                          float *__restrict__ y, int n_y) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  const int m = blockIdx.y;
  if (n >= n_y) return;
  const int b = n / B, t = n % B;
  const float *zm = z + (size_t)m * n_out_blocks * N;
  float v = zm[(size_t)b * N + t];
  if (b > 0) v += zm[(size_t)(b - 1) * N + B + t];
  y[(size_t)m * n_y + n] = v;
}

static size_t fft_align(size_t v) { return (v + 255) & ~(size_t)255; }

// Block size: B = 4096 for RIRs of 16384 taps and more, else a quarter of
// the next power of two of n_rir (at least 256). R: pieces per input block.
// Returns false when the pieces per block exceed max_pieces.
bool fft_plan(int n_x, int n_pos, int n_mic, int n_rir, int max_pieces, FftPlan &f) {
  int np2 = 1;
  while (np2 < n_rir) np2 <<= 1;
  f.B = np2 >= 16384 ? 4096 : (np2 / 4 < 256 ? 256 : np2 / 4);
  f.N = 2 * f.B;
  f.P = (n_rir + f.B - 1) / f.B;
  f.L = (n_x + n_pos - 1) / n_pos;
  f.R = (f.B + f.L - 1) / f.L + 1;  // segments one block can touch
  if (f.R > n_pos) f.R = n_pos;
  if (f.R > max_pieces) return false;
  f.n_in_blocks = (n_x + f.B - 1) / f.B;
  const int64_t n_y = (int64_t)n_x + n_rir - 1;
  if ((n_y + f.B - 1) / f.B > 65535) return false;  // one grid dimension per output block
  f.n_out_blocks = (int)((n_y + f.B - 1) / f.B);
  size_t o = 0;
  f.off_tw = o;
  o = fft_align(o + sizeof(float2) * (size_t)(f.N / 2));
  f.off_H = o;
  o = fft_align(o + sizeof(float2) * (size_t)n_pos * n_mic * f.P * f.N);
  f.off_X = o;
  o = fft_align(o + sizeof(float2) * (size_t)f.n_in_blocks * f.R * f.N);
  f.off_Y = o;
  o = fft_align(o + sizeof(float2) * (size_t)n_mic * f.n_out_blocks * f.N);
  f.off_z = o;
  o = fft_align(o + sizeof(float) * (size_t)n_mic * f.n_out_blocks * f.N);
  f.bytes = o;
  return true;
}

int launch_filter_fft(const float *x, int n_x, const float *rir, int n_pos, int n_mic, int n_rir, float *y,
                      const FftPlan &f, void *ws, hipStream_t st) {
  char *w = (char *)ws;
  float2 *tw = (float2 *)(w + f.off_tw), *H = (float2 *)(w + f.off_H), *X = (float2 *)(w + f.off_X),
         *Y = (float2 *)(w + f.off_Y);
  float *z = (float *)(w + f.off_z);
  hipLaunchKernelGGL(fft_twiddle_kernel, dim3((f.N / 2 + 255) / 256), dim3(256), 0, st, tw, f.N);
  hipLaunchKernelGGL(fft_rir_kernel, dim3((unsigned)((size_t)n_pos * n_mic * f.P)), dim3(FFT_THREADS), 0, st, rir,
                     n_rir, f.B, f.N, f.P, tw, H);
  hipLaunchKernelGGL(fft_input_kernel, dim3((unsigned)(f.n_in_blocks * f.R)), dim3(FFT_THREADS), 0, st, x, n_x,
                     n_pos, f.L, f.B, f.N, f.R, tw, X);
  hipLaunchKernelGGL(spectrum_mac_kernel, dim3(f.N / 256, f.n_out_blocks, n_mic), dim3(256), 0, st, X, H, n_x, n_pos,
                     n_mic, f.L, f.B, f.N, f.P, f.R, f.n_in_blocks, Y);
  hipLaunchKernelGGL(ifft_block_kernel, dim3((unsigned)(n_mic * f.n_out_blocks)), dim3(FFT_THREADS), 0, st, Y, f.N,
                     tw, z);
  const int n_y = n_x + n_rir - 1;
  hipLaunchKernelGGL(overlap_add_kernel, dim3((n_y + 255) / 256, n_mic), dim3(256), 0, st, z, f.B, f.N,
                     f.n_out_blocks, y, n_y);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace ism
