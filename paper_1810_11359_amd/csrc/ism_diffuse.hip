// Diffuse reverberation tail (Sec. 2.2, Eq. (8); Sec. 3.3): after t_diff the
// RIR is logistic noise times the square root of an exponential power envelope,
//   P(t) = A 10^(-6 (t - t_diff) / T60)      (-60 dB of power in T60, Sabine),
// whose level A is estimated from the ISM part of the same RIR: the mean of
// h[k]^2 / 10^(-6 (t_k - t_diff) / T60) over the last fifth of the ISM part.
// The noise of sample k of RIR i is the unit-variance logistic variate of one
// 32-bit word of the Philox4x32-10 counter-based generator (Salmon et al.,
// SC'11) with counter (k / 4, i, 0, 0) and key (seed low, seed high), word
// k % 4: any sample can be drawn independently, so the tail is one pass of
// independent threads and a result does not depend on the launch shape.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

namespace ism {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Philox4x32 with 10 rounds: a round maps (c0, c1, c2, c3) with key (k0, k1)
// to (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)); the key
// advances by two Weyl increments before every round but the first.
__device__ __forceinline__ u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint32_t hi0 = __umulhi(M0, c.x), lo0 = M0 * c.x;
    const uint32_t hi1 = __umulhi(M1, c.z), lo1 = M1 * c.z;
    c = u32x4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
  }
  return c;
}

// Unit-variance logistic variate of a word x: log(u / (1 - u)) sqrt(3)/pi at
// u = (x + 1/2) / 2^32, with u and 1 - u both formed from exact integers.
__device__ __forceinline__ float logistic_from_bits(uint32_t x) {
  const float a = (float)x + 0.5f;
  const float b = (float)(0xFFFFFFFFu - x) + 0.5f;
  constexpr float kScale = 0.69314718055994531f * 0.55132889542179204f;  // ln 2 * sqrt(3)/pi
  return (__log2f(a) - __log2f(b)) * kScale;
}

// grid = n_seg x n_rir blocks (block b: RIR b / n_seg, segment b % n_seg of
// 256 SPT samples); each block recomputes the level A of its RIR (a
// fixed-order block sum over the window) and writes SPT samples per thread:
// the ISM part copied for k < k_diff, the tail after it.
constexpr int SPT = 4;
__global__ __launch_bounds__(256) void diffuse_kernel(const float *__restrict__ ism, int k_diff, int k_w,
                                                      float *__restrict__ out, int n_samples, int n_seg, float fs,
                                                      float t_diff, float t60, uint32_t key0, uint32_t key1) {
  const int rir = (int)(blockIdx.x / (unsigned)n_seg);
  const int seg = (int)(blockIdx.x % (unsigned)n_seg);
  const float *h = ism + (size_t)rir * k_diff;
  // power envelope shape at sample k: exp2(c1 (k / fs - t_diff))
  const float c1 = -6.0f * 3.32192809488736235f / t60;
  __shared__ float red[256];
  float acc = 0.0f;
  for (int k = k_w + (int)threadIdx.x; k < k_diff; k += 256) {
    const float v = h[k];
    acc += v * v * exp2f(-c1 * ((float)k / fs - t_diff));
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const float A = red[0] / (float)(k_diff - k_w);
  float *o = out + (size_t)rir * n_samples;
  const int k0 = (seg * 256 + (int)threadIdx.x) * SPT;  // SPT consecutive samples, one Philox block
  if (k0 >= n_samples) return;
  const u32x4 bits = philox4x32_10(u32x4{(uint32_t)(k0 / 4), (uint32_t)rir, 0u, 0u}, key0, key1);
#pragma unroll
  for (int j = 0; j < SPT; ++j) {
    const int k = k0 + j;
    if (k >= n_samples) break;
    float v;
    if (k < k_diff) {
      v = h[k];
    } else {
      const float env = exp2f(c1 * ((float)k / fs - t_diff));
      v = logistic_from_bits(bits[j]) * sqrtf(A * env);
    }
    o[k] = v;
  }
}

int launch_diffuse(const float *ism, int k_diff, float *out, int n_samples, int n_rir, double fs, double t_diff,
                   double t60, uint64_t seed, hipStream_t st) {
  const int k_w = k_diff - (k_diff / 5 > 1 ? k_diff / 5 : 1);
  const int n_seg = (n_samples + 256 * SPT - 1) / (256 * SPT);
  const uint64_t blocks = (uint64_t)n_seg * (uint64_t)n_rir;
  if (blocks == 0 || blocks > 0x7fffffffu) return -1;
  hipLaunchKernelGGL(diffuse_kernel, dim3((unsigned)blocks), dim3(256), 0, st, ism, k_diff, k_w, out, n_samples,
                     n_seg, (float)fs, (float)t_diff, (float)t60, (uint32_t)(seed & 0xFFFFFFFFu),
                     (uint32_t)(seed >> 32));
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace ism
