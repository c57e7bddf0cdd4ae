// Moving-source filtering (Sec. 3.4) by partitioned FFT convolution: the
// paper filters the signal through the trajectory's RIRs with batched FFTs;
// this is that path, written for gfx950 (real transforms through half-size
// complex Stockham transforms in LDS).
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

// Transforms: the real N-point transform of each block (N = 2B, the second
// half zero) is taken as an M = N/2-point complex transform of the packed
// sequence z[n] = x[2n] + i x[2n+1], then split into the spectrum of x: with
// W = exp(-2 pi i / N),
//   X[k] = (Z[k] + conj Z[M-k]) / 2 + W^k (Z[k] - conj Z[M-k]) / (2i), 0 < k < M,
//   X[0] = Re Z[0] + Im Z[0], X[M] = Re Z[0] - Im Z[0] (both real),
// stored as M complex bins, bin 0 holding (X[0], X[M]). The inverse runs the
// same steps backwards (Z[k] = E[k] + i O[k] from Y[k] and conj Y[M-k], then
// an inverse M-point transform scaled by 1/M gives y[2n] + i y[2n+1]).
// The complex transforms are Stockham passes of radix 8 (then one of radix 4
// or 2), each thread holding its butterflies' points in registers between
// two barriers; the data stay in LDS (M complex per transform).
constexpr int FFT_THREADS = 256;

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(__builtin_fmaf(a.x, b.x, -a.y * b.y), __builtin_fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// a times -i (forward) or +i (inverse)
__device__ __forceinline__ float2 rot_i(float2 a, bool inv) {
  return inv ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// T[n] = exp(-2 pi i n / N), n < N
__global__ __launch_bounds__(256) void fft_twiddle_kernel(float2 *__restrict__ tw, int N) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < N; t += gridDim.x * blockDim.x) {
    float s, c;
    sincospi_acc(-2.0f * (float)t / (float)N, s, c);
    tw[t] = make_float2(c, s);
  }
}

// R-point DFT of v in place (R = 2, 4, 8), kernel exp(-+2 pi i t s / R).
template <int R>
__device__ __forceinline__ void dft_small(float2 *v, bool inv) {
  if constexpr (R == 2) {
    const float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    const float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]), t2 = cadd(v[1], v[3]),
                 t3 = rot_i(csub(v[1], v[3]), inv);
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  } else {
    // DFTs of the even and odd points, combined with exp(-+2 pi i s / 8)
    float2 e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
    dft_small<4>(e, inv);
    dft_small<4>(o, inv);
    constexpr float h = 0.70710678118654752f;  // 1 / sqrt(2)
    const float2 o1 = inv ? make_float2(h * (o[1].x - o[1].y), h * (o[1].x + o[1].y))
                          : make_float2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
    const float2 o2 = rot_i(o[2], inv);
    const float2 o3 = inv ? make_float2(-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y))
                          : make_float2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
}

// Threads per transform and transforms per block for M-point transforms.
template <int M> struct FftShape {
  static constexpr int TPF = M / 8 < FFT_THREADS ? M / 8 : FFT_THREADS;
  static constexpr int FPB = FFT_THREADS / TPF;
};

// One Stockham pass of radix R and span Ns over the M points at a (LDS): the
// butterfly j (k = j mod Ns) takes a[j + t M/R], t < R, twiddles point t by
// exp(-+2 pi i t k / (R Ns)) (table T of the N = 2M-point roots: index 2 t k
// M / (R Ns)), and writes its DFT to a[(j - k) R + k + s Ns]. The twiddles
// are fetched first, all LDS reads of the pass happen before the first
// barrier and all writes after it.
template <int M, int R>
__device__ __forceinline__ void fft_pass(float2 *a, int tid, const float2 *__restrict__ T, int Ns, bool inv) {
  constexpr int TPF = FftShape<M>::TPF;
  constexpr int NB = M / R / TPF;  // butterflies per thread
  static_assert(NB >= 1 && NB * R * TPF == M, "pass shape");
  const int step2 = 2 * (M / (R * Ns));
  float2 w[NB][R];
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const int k = (tid + u * TPF) & (Ns - 1);
#pragma unroll
    for (int t = 1; t < R; ++t) w[u][t] = T[t * k * step2];
  }
  float2 v[NB][R];
#pragma unroll
  for (int u = 0; u < NB; ++u)
#pragma unroll
    for (int t = 0; t < R; ++t) v[u][t] = a[tid + u * TPF + t * (M / R)];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const int j = tid + u * TPF;
    const int k = j & (Ns - 1);
#pragma unroll
    for (int t = 1; t < R; ++t) v[u][t] = cmul(v[u][t], inv ? make_float2(w[u][t].x, -w[u][t].y) : w[u][t]);
    dft_small<R>(v[u], inv);
    const int o = (j - k) * R + k;
#pragma unroll
    for (int s = 0; s < R; ++s) a[o + s * Ns] = v[u][s];
  }
  __syncthreads();
}

// M-point complex transform into a (LDS), natural order in and out; point n
// of the input is load(n). The first pass (radix 8, span 1: no twiddles)
// reads its points through load and writes a; the later passes work in a.
template <int M, class Load>
__device__ __forceinline__ void fft_m(Load &&load, float2 *a, int tid, const float2 *__restrict__ T, bool inv) {
  constexpr int LOG = __builtin_ctz(M);
  static_assert(LOG >= 6, "at least two radix-8 passes");
  constexpr int TPF = FftShape<M>::TPF;
  constexpr int NB = M / 8 / TPF;
  {
    float2 v[NB][8];
#pragma unroll
    for (int u = 0; u < NB; ++u)
#pragma unroll
      for (int t = 0; t < 8; ++t) v[u][t] = load(tid + u * TPF + t * (M / 8));
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      dft_small<8>(v[u], inv);
      const int j = tid + u * TPF;
#pragma unroll
      for (int s = 0; s < 8; ++s) a[8 * j + s] = v[u][s];
    }
    __syncthreads();
  }
  int Ns = 8;
#pragma unroll
  for (int p = 1; p < LOG / 3; ++p) {
    fft_pass<M, 8>(a, tid, T, Ns, inv);
    Ns *= 8;
  }
  if constexpr (LOG % 3 == 1) fft_pass<M, 2>(a, tid, T, Ns, inv);
  if constexpr (LOG % 3 == 2) fft_pass<M, 4>(a, tid, T, Ns, inv);
}

// Spectrum bins k < M of the real sequence packed in a (after fft_m) to o.
template <int M>
__device__ __forceinline__ void real_split(const float2 *a, int tid, const float2 *__restrict__ T,
                                           float2 *__restrict__ o) {
  constexpr int TPF = FftShape<M>::TPF;
  for (int k = tid; k < M; k += TPF) {
    if (k == 0) {
      o[0] = make_float2(a[0].x + a[0].y, a[0].x - a[0].y);
      continue;
    }
    const float2 zk = a[k], zm = make_float2(a[M - k].x, -a[M - k].y);  // conj Z[M-k]
    const float2 e = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y + zm.y));
    const float2 d = csub(zk, zm);
    const float2 od = make_float2(0.5f * d.y, -0.5f * d.x);  // d / (2i)
    o[k] = cadd(e, cmul(T[k], od));
  }
}

// Point k of the packed sequence Z whose inverse transform gives a real
// block, from its packed spectrum Y (M bins, bin 0 holding bins 0 and M).
template <int M>
__device__ __forceinline__ float2 real_merge(const float2 *__restrict__ Y, int k, const float2 *__restrict__ T) {
  if (k == 0) {
    const float2 y0 = Y[0];
    return make_float2(0.5f * (y0.x + y0.y), 0.5f * (y0.x - y0.y));
  }
  const float2 yk = Y[k], ym = make_float2(Y[M - k].x, -Y[M - k].y);  // conj Y[M-k]
  const float2 e = make_float2(0.5f * (yk.x + ym.x), 0.5f * (yk.y + ym.y));
  const float2 w = make_float2(T[k].x, -T[k].y);  // exp(+2 pi i k / N)
  const float2 d = csub(yk, ym);
  const float2 od = cmul(make_float2(0.5f * d.x, 0.5f * d.y), w);
  return make_float2(e.x - od.y, e.y + od.x);  // e + i od
}

// Spectra of the RIR partitions: transform row = (p * n_mic + m) * P + q.
template <int M>
__global__ __launch_bounds__(FFT_THREADS) void fft_rir_kernel(const float *__restrict__ rir, int n_rir, int P,
                                                            int n_rows, const float2 *__restrict__ T,
                                                            float2 *__restrict__ H) {
  constexpr int TPF = FftShape<M>::TPF, FPB = FftShape<M>::FPB;
  __shared__ float2 buf[FPB][M];
  const int f = threadIdx.x / TPF, tid = threadIdx.x % TPF;
  const int row = blockIdx.x * FPB + f;
  const int q = row % P;
  const float *h = rir + (size_t)(row / P) * n_rir + (size_t)q * M;  // B = M samples per partition
  const int len = row < n_rows ? min(M, n_rir - q * M) : 0;
  fft_m<M>([&](int n) {
    const int i0 = 2 * n, i1 = 2 * n + 1;
    return make_float2(i0 < len ? h[i0] : 0.0f, i1 < len ? h[i1] : 0.0f);
  }, buf[f], tid, T, false);
  if (row < n_rows) real_split<M>(buf[f], tid, T, H + (size_t)row * M);
}

// Segment of input block i's piece r, or -1 when the piece is empty.
__device__ __forceinline__ int piece_segment(int i, int r, int B, int L, int n_x, int n_pos) {
  const int lo = i * B, hi = min(lo + B, n_x);  // samples [lo, hi)
  const int p = lo / L + r;
  if (p >= n_pos || p * L >= hi) return -1;
  return p;
}

// Spectra of the input pieces: transform i * R + r (empty pieces are skipped:
// their spectra are never read).
template <int M>
__global__ __launch_bounds__(FFT_THREADS) void fft_input_kernel(const float *__restrict__ x, int n_x, int n_pos,
                                                              int L, int R, int n_rows, const float2 *__restrict__ T,
                                                              float2 *__restrict__ X) {
  constexpr int TPF = FftShape<M>::TPF, FPB = FftShape<M>::FPB;
  __shared__ float2 buf[FPB][M];
  const int f = threadIdx.x / TPF, tid = threadIdx.x % TPF;
  const int row = blockIdx.x * FPB + f;
  const int i = row / R, r = row % R;
  const int p = row < n_rows ? piece_segment(i, r, M, L, n_x, n_pos) : -1;
  // samples of the block (B = M) inside segment p: [lo, hi) relative to the block
  const int lo = p >= 0 ? max(p * L - i * M, 0) : 0;
  const int hi = p >= 0 ? min(min(p * L + L, n_x) - i * M, M) : 0;
  const float *xb = x + (size_t)i * M;
  fft_m<M>([&](int n) {
    const int t0 = 2 * n, t1 = 2 * n + 1;
    return make_float2(t0 >= lo && t0 < hi ? xb[t0] : 0.0f, t1 >= lo && t1 < hi ? xb[t1] : 0.0f);
  }, buf[f], tid, T, false);
  if (p >= 0) real_split<M>(buf[f], tid, T, X + (size_t)row * M);
}

// Y[m][b][k] = sum over q, then r of X[b - q][r][k] H[p][m][q][k], k < M
// (bin 0 holds the two real bins 0 and M: their products are taken apart).
// grid = (M / 256, n_out_blocks, n_mic).
__global__ __launch_bounds__(256) void spectrum_mac_kernel(const float2 *__restrict__ X, const float2 *__restrict__ H,
                                                           int n_x, int n_pos, int n_mic, int L, int B, int M, int P,
                                                           int R, int n_in_blocks, float2 *__restrict__ Y) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y, m = blockIdx.z;
  const float2 *__restrict__ Xk = X + k;
  const float2 *__restrict__ Hk = H + (size_t)m * P * M + k;
  float2 acc = make_float2(0.0f, 0.0f);
  // input blocks i = b - q that exist: q in [q0, q1]; the pieces of block i
  // are the segments p0(i), p0(i) + 1, ... up to the first empty one
  const int q0 = max(0, b - (n_in_blocks - 1)), q1 = min(P - 1, b);
  for (int q = q0; q <= q1; ++q) {
    const int i = b - q;
    const int lo = i * B, hi = min(lo + B, n_x);
    const int p0 = lo / L;
    for (int r = 0; r < R; ++r) {
      const int p = p0 + r;
      if (p >= n_pos || p * L >= hi) break;  // uniform over the block
      const float2 xv = Xk[((size_t)i * R + r) * M];
      const float2 hv = Hk[((size_t)p * n_mic * P + q) * M];
      if (k == 0) {
        acc.x = __builtin_fmaf(xv.x, hv.x, acc.x);
        acc.y = __builtin_fmaf(xv.y, hv.y, acc.y);
      } else {
        acc.x = __builtin_fmaf(xv.x, hv.x, acc.x);
        acc.x = __builtin_fmaf(-xv.y, hv.y, acc.x);
        acc.y = __builtin_fmaf(xv.x, hv.y, acc.y);
        acc.y = __builtin_fmaf(xv.y, hv.x, acc.y);
      }
    }
  }
  Y[((size_t)m * gridDim.y + b) * M + k] = acc;
}

// z[m][b] = IFFT(Y[m][b]) (N real samples); transform row = m * n_out_blocks + b.
template <int M>
__global__ __launch_bounds__(FFT_THREADS) void ifft_block_kernel(const float2 *__restrict__ Y, int n_rows,
                                                               const float2 *__restrict__ T, float *__restrict__ z) {
  constexpr int TPF = FftShape<M>::TPF, FPB = FftShape<M>::FPB;
  __shared__ float2 buf[FPB][M];
  const int f = threadIdx.x / TPF, tid = threadIdx.x % TPF;
  const int row = blockIdx.x * FPB + f;
  const bool live = row < n_rows;
  const float2 *Yr = Y + (size_t)(live ? row : 0) * M;
  fft_m<M>([&](int n) { return live ? real_merge<M>(Yr, n, T) : make_float2(0.0f, 0.0f); }, buf[f], tid, T, true);
  if (live) {
    constexpr float inv_m = 1.0f / (float)M;
    const float2 *a = buf[f];
    float2 *o = reinterpret_cast<float2 *>(z + (size_t)row * 2 * M);
    for (int n = tid; n < M; n += TPF) o[n] = make_float2(a[n].x * inv_m, a[n].y * inv_m);
  }
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
  o = fft_align(o + sizeof(float2) * (size_t)f.N);
  f.off_H = o;
  o = fft_align(o + sizeof(float2) * (size_t)n_pos * n_mic * f.P * f.B);
  f.off_X = o;
  o = fft_align(o + sizeof(float2) * (size_t)f.n_in_blocks * f.R * f.B);
  f.off_Y = o;
  o = fft_align(o + sizeof(float2) * (size_t)n_mic * f.n_out_blocks * f.B);
  f.off_z = o;
  o = fft_align(o + sizeof(float) * (size_t)n_mic * f.n_out_blocks * f.N);
  f.bytes = o;
  return true;
}

template <int M>
static int launch_fft_m(const float *x, int n_x, const float *rir, int n_pos, int n_mic, int n_rir, float *y,
                        const FftPlan &f, char *w, hipStream_t st) {
  constexpr int FPB = FftShape<M>::FPB;
  float2 *T = (float2 *)(w + f.off_tw), *H = (float2 *)(w + f.off_H), *X = (float2 *)(w + f.off_X),
         *Y = (float2 *)(w + f.off_Y);
  float *z = (float *)(w + f.off_z);
  hipLaunchKernelGGL(fft_twiddle_kernel, dim3((f.N + 255) / 256), dim3(256), 0, st, T, f.N);
  const int rir_rows = n_pos * n_mic * f.P;
  hipLaunchKernelGGL(fft_rir_kernel<M>, dim3((rir_rows + FPB - 1) / FPB), dim3(FFT_THREADS), 0, st, rir, n_rir, f.P,
                     rir_rows, T, H);
  const int in_rows = f.n_in_blocks * f.R;
  hipLaunchKernelGGL(fft_input_kernel<M>, dim3((in_rows + FPB - 1) / FPB), dim3(FFT_THREADS), 0, st, x, n_x, n_pos,
                     f.L, f.R, in_rows, T, X);
  hipLaunchKernelGGL(spectrum_mac_kernel, dim3(M / 256, f.n_out_blocks, n_mic), dim3(256), 0, st, X, H, n_x, n_pos,
                     n_mic, f.L, f.B, M, f.P, f.R, f.n_in_blocks, Y);
  const int out_rows = n_mic * f.n_out_blocks;
  hipLaunchKernelGGL(ifft_block_kernel<M>, dim3((out_rows + FPB - 1) / FPB), dim3(FFT_THREADS), 0, st, Y, out_rows,
                     T, z);
  const int n_y = n_x + n_rir - 1;
  hipLaunchKernelGGL(overlap_add_kernel, dim3((n_y + 255) / 256, n_mic), dim3(256), 0, st, z, f.B, f.N,
                     f.n_out_blocks, y, n_y);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_filter_fft(const float *x, int n_x, const float *rir, int n_pos, int n_mic, int n_rir, float *y,
                      const FftPlan &f, void *ws, hipStream_t st) {
  char *w = (char *)ws;
  switch (f.B) {  // M = B complex points per transform
    case 256: return launch_fft_m<256>(x, n_x, rir, n_pos, n_mic, n_rir, y, f, w, st);
    case 512: return launch_fft_m<512>(x, n_x, rir, n_pos, n_mic, n_rir, y, f, w, st);
    case 1024: return launch_fft_m<1024>(x, n_x, rir, n_pos, n_mic, n_rir, y, f, w, st);
    case 2048: return launch_fft_m<2048>(x, n_x, rir, n_pos, n_mic, n_rir, y, f, w, st);
    case 4096: return launch_fft_m<4096>(x, n_x, rir, n_pos, n_mic, n_rir, y, f, w, st);
    default: return -1;
  }
}

}  // namespace ism
