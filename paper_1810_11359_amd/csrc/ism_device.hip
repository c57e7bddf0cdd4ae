// HIP kernels of the Image Source Method for gfx950 (MI355X).
//
// Three kernels per call:
//   tables_kernel      per (RIR, axis, lattice index): displacement of the image
//                      coordinate from the receiver in samples (float-float) and
//                      the axis factor of the reflection gain (Sec. 2.1, Eq. (1)
//                      and the gain rule below it). Also flags invalid pairs.
//   accumulate_kernel  per work item (RIR, output tile, slab of the image shell):
//                      enumerates exactly the lattice images whose window can
//                      reach the tile, computes each image's delay and amplitude
//                      (Eq. (2)-(4)) and adds its Hann-windowed-sinc taps (Eq. (6))
//                      into wave-private FP32 LDS tiles (Eq. (5)).
//   reduce_kernel      sums, in a fixed order, the partial tiles of tiles that
//                      were split over several work items.
//
// Arithmetic is FP32 only; delays use error-free transformations so that the
// fractional delay keeps ~1e-7 sample accuracy at 1e5-sample distances.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "ism_internal.h"

namespace ism {

// ---------------------------------------------------------------------------
// Float-float building blocks (Dekker / Knuth error-free transformations).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
  s = a + b;
  float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
__device__ __forceinline__ void fast_two_sum(float a, float b, float &s, float &e) {  // |a| >= |b|
  s = a + b;
  e = b - (s - a);
}
__device__ __forceinline__ void two_prod(float a, float b, float &p, float &e) {
  p = a * b;
  e = __builtin_fmaf(a, b, -p);
}
__device__ __forceinline__ void ff_mul(float ah, float al, float bh, float bl, float &ch, float &cl) {
  float p, e;
  two_prod(ah, bh, p, e);
  e = __builtin_fmaf(ah, bl, e);
  e = __builtin_fmaf(al, bh, e);
  fast_two_sum(p, e, ch, cl);
}
// b^e for e >= 0 by binary powering in float-float (0^0 = 1).
__device__ float ff_pow(float b, int e) {
  float rh = 1.0f, rl = 0.0f, bh = b, bl = 0.0f;
  while (e > 0) {
    if (e & 1) ff_mul(rh, rl, bh, bl, rh, rl);
    e >>= 1;
    if (e) ff_mul(bh, bl, bh, bl, bh, bl);
  }
  return rh + rl;
}
// a^2 of a float-float value, as float-float.
__device__ __forceinline__ void ff_sq(float h, float l, float &sh, float &sl) {
  two_prod(h, h, sh, sl);
  sl = __builtin_fmaf(2.0f * h, l, sl);
}
// (ah, al) - (bh, bl), renormalised.
__device__ __forceinline__ void ff_sub(float ah, float al, float bh, float bl, float &ch, float &cl) {
  float s, e;
  two_sum(ah, -bh, s, e);
  e += al - bl;
  fast_two_sum(s, e, ch, cl);
}

// ---------------------------------------------------------------------------
// Compile-time constants of the tap loop (evaluated in double by the compiler).
// ---------------------------------------------------------------------------
constexpr double kPi = 3.14159265358979323846;

constexpr double cx_sin(double x) {  // |x| <= pi: Taylor series to double accuracy
  double term = x, sum = x;
  for (int k = 1; k < 30; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double cx_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 30; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}

// For an even integer window of WT samples and fractional delay f in (0, 1),
// the taps of one image are j = JLO .. JLO + WT - 1 (JLO = 1 - WT/2) relative to
// k0 = floor(x). With v = j - f:
//   sin(pi v) = sigma_j sin(pi f),            sigma_j = (-1)^(j+1)
//   1 + cos(2 pi v / W) = 1 + cos(th_j) cos(phi) + sin(th_j) sin(phi),
//                         th_j = 2 pi j / W, phi = 2 pi f / W,
// so tap_j = [C/2 + (C/2 cos phi) cos th_j + (C/2 sin phi) sin th_j] / (sigma_j (j - f))
// with C = A sin(pi f) / pi. Only sigma_j, sigma_j j, cos th_j, sin th_j depend on j.
template <int WT>
struct TapConsts {
  float sig[WT], sig_j[WT], cth[WT], sth[WT];
};
template <int WT>
constexpr TapConsts<WT> make_tap_consts() {
  TapConsts<WT> t{};
  for (int jj = 0; jj < WT; ++jj) {
    const int j = jj + 1 - WT / 2;
    const double sg = (j % 2 == 0) ? -1.0 : 1.0;
    const double th = 2.0 * kPi * j / WT;  // in (-pi, pi]
    t.sig[jj] = (float)sg;
    t.sig_j[jj] = (float)(sg * j);
    t.cth[jj] = (float)cx_cos(th);
    t.sth[jj] = (float)cx_sin(th);
  }
  return t;
}

// FP16 taps. Away from the centre (j <= -2 or j >= 3) the tap of an image is
// C g_j(t) with t = f - 1/2 in [-1/2, 1/2) and
//   g_j = (1 + cos(2 pi (j - f) / W)) sigma_j / (2 (j - f)),
// which is analytic on the interval (its nearest pole is 2.5 away in t). Each
// g_j is replaced by its cubic interpolant at the four Chebyshev nodes of
// [-1/2, 1/2] (interpolation error < 2e-4 of max|g_j|), evaluated in packed
// FP16 two taps at a time. The four central taps keep the exact FP32 form.
constexpr bool poly_tap(int j) { return j <= -2 || j >= 3; }

template <int WT>
struct PolyConsts {
  float c[4][WT];  // monomial coefficients in t, rounded to FP16 where used
};
constexpr double g_tap(int j, double t, int wt) {
  const double v = j - (t + 0.5);
  const double sg = (j % 2 == 0) ? -1.0 : 1.0;
  return (1.0 + cx_cos(2.0 * kPi * v / wt)) * sg / (2.0 * v);
}
template <int WT>
constexpr PolyConsts<WT> make_poly_consts() {
  PolyConsts<WT> P{};
  for (int jj = 0; jj < WT; ++jj) {
    const int j = jj + 1 - WT / 2;
    if (!poly_tap(j)) continue;
    double x[4] = {}, y[4] = {};
    for (int k = 0; k < 4; ++k) {
      x[k] = 0.5 * cx_cos((2.0 * k + 1.0) * kPi / 8.0);
      y[k] = g_tap(j, x[k], WT);
    }
    // Newton divided differences, then expansion to monomials
    double d[4] = {y[0], y[1], y[2], y[3]};
    for (int lvl = 1; lvl < 4; ++lvl)
      for (int k = 3; k >= lvl; --k) d[k] = (d[k] - d[k - 1]) / (x[k] - x[k - lvl]);
    double m[4] = {d[3], 0.0, 0.0, 0.0};  // coefficients of the running polynomial, highest first
    int deg = 0;
    for (int k = 2; k >= 0; --k) {  // m(t) = m(t) * (t - x[k]) + d[k]
      double nm[4] = {0.0, 0.0, 0.0, 0.0};
      for (int q = 0; q <= deg; ++q) {
        nm[q] += m[q];
        nm[q + 1] -= m[q] * x[k];
      }
      ++deg;
      nm[deg] += d[k];
      for (int q = 0; q < 4; ++q) m[q] = nm[q];
    }
    for (int q = 0; q < 4; ++q) P.c[3 - q][jj] = (float)m[q];  // c[k] multiplies t^k
  }
  return P;
}

// sin(pi h) / pi for h in [0, 1/2]: Taylor series of sin to the h^13 term
// (truncation < 2e-10 at h = 1/2), Horner in h^2.
__device__ __forceinline__ float sinpi_over_pi(float h) {
  constexpr float c1 = (float)(-kPi * kPi / 6.0);
  constexpr float c2 = (float)(kPi * kPi * kPi * kPi / 120.0);
  constexpr float c3 = (float)(-kPi * kPi * kPi * kPi * kPi * kPi / 5040.0);
  constexpr float c4 = (float)(kPi * kPi * kPi * kPi * kPi * kPi * kPi * kPi / 362880.0);
  constexpr float c5 = (float)(-kPi * kPi * kPi * kPi * kPi * kPi * kPi * kPi * kPi * kPi / 39916800.0);
  constexpr float c6 = (float)(kPi * kPi * kPi * kPi * kPi * kPi * kPi * kPi * kPi * kPi * kPi * kPi / 6227020800.0);
  const float u = h * h;
  float p = __builtin_fmaf(u, c6, c5);
  p = __builtin_fmaf(u, p, c4);
  p = __builtin_fmaf(u, p, c3);
  p = __builtin_fmaf(u, p, c2);
  p = __builtin_fmaf(u, p, c1);
  p = __builtin_fmaf(u, p, 1.0f);
  return h * p;
}
// cos and sin of a small angle |phi| <= 0.2 (Taylor, truncation < 3e-12).
__device__ __forceinline__ void small_sincos(float phi, float &s, float &c) {
  const float u = phi * phi;
  float pc = __builtin_fmaf(u, (float)(1.0 / 40320.0), (float)(-1.0 / 720.0));
  pc = __builtin_fmaf(u, pc, (float)(1.0 / 24.0));
  pc = __builtin_fmaf(u, pc, -0.5f);
  c = __builtin_fmaf(u, pc, 1.0f);
  float ps = __builtin_fmaf(u, (float)(1.0 / 362880.0), (float)(-1.0 / 5040.0));
  ps = __builtin_fmaf(u, ps, (float)(1.0 / 120.0));
  ps = __builtin_fmaf(u, ps, (float)(-1.0 / 6.0));
  s = __builtin_fmaf(phi * u, ps, phi);
}

// ---------------------------------------------------------------------------
// Kernel 1: per-RIR axis tables.
// ---------------------------------------------------------------------------
// Table entry e (axis a, lattice index n) of the RIR with source s, receiver r.
__device__ __forceinline__ AxisEntry table_entry(const RoomArgs &ra, const float *__restrict__ s3,
                                                 const float *__restrict__ r3, int e) {
  const int a = e < ra.off[1] ? 0 : (e < ra.off[2] ? 1 : 2);
  const int n = ra.lo[a] + (e - ra.off[a]);
  const float s = s3[a], r = r3[a];
  // Eq. (1): even n -> n L + s, odd n -> (n + 1) L - s.
  const bool odd = (n & 1) != 0;
  const float m = (float)(odd ? n + 1 : n);
  float p, pe;
  two_prod(m, ra.L_hi[a], p, pe);
  pe = __builtin_fmaf(m, ra.L_lo[a], pe);
  float t, te;
  two_sum(odd ? -s : s, -r, t, te);  // exact
  float u, ue;
  two_sum(p, t, u, ue);
  ue += pe + te;
  fast_two_sum(u, ue, u, ue);
  // times fs / c: displacement in samples
  float v, ve;
  two_prod(u, ra.q_hi, v, ve);
  ve = __builtin_fmaf(u, ra.q_lo, ve);
  ve = __builtin_fmaf(ue, ra.q_hi, ve);
  fast_two_sum(v, ve, v, ve);
  // Gain factor: the path from image n crosses |floor(n/2)| copies of the wall
  // at 0 and |ceil(n/2)| copies of the wall at L along this axis.
  const int e0 = abs(n >> 1), e1 = abs((n + 1) >> 1);
  const float g = ff_pow(ra.beta[2 * a], e0) * ff_pow(ra.beta[2 * a + 1], e1);
  return AxisEntry{v, ve, g, 0.0f};
}

// Validity of a pair (both points strictly inside, distinct) and the family
// offsets of its axes.
__device__ __forceinline__ int rir_header(const RoomArgs &ra, const float *__restrict__ s3,
                                          const float *__restrict__ r3, AxisOrigin &o) {
  bool ok = true, same = true;
  for (int b = 0; b < 3; ++b) {
    const float sb = s3[b], rb = r3[b];
    ok = ok && sb > 0.0f && (sb - ra.L_hi[b]) < ra.L_lo[b] && rb > 0.0f && (rb - ra.L_hi[b]) < ra.L_lo[b];
    same = same && (sb == rb);
    o.e_even[b] = (sb - rb) * ra.q_hi;
    o.e_odd[b] = (-sb - rb) * ra.q_hi;
  }
  return (ok && !same) ? 1 : 0;
}

__global__ __launch_bounds__(256) void tables_kernel(RoomArgs ra, const float *__restrict__ src,
                                                     const float *__restrict__ rcv, AxisEntry *__restrict__ tab,
                                                     AxisOrigin *__restrict__ origin, int *__restrict__ valid,
                                                     int n_rir) {
  const int64_t total = (int64_t)n_rir * ra.n_tab;
  for (int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gid < total;
       gid += (int64_t)gridDim.x * blockDim.x) {
    const int rir = (int)(gid / ra.n_tab);
    const int e = (int)(gid % ra.n_tab);
    const float *s3 = src + 3 * (rir / ra.n_rcv);
    const float *r3 = rcv + 3 * (rir % ra.n_rcv);
    tab[gid] = table_entry(ra, s3, r3, e);
    if (e == 0) {
      AxisOrigin o;
      valid[rir] = rir_header(ra, s3, r3, o);
      origin[rir] = o;
    }
  }
}

// Batch mode: one block per batch-wide RIR.
__global__ __launch_bounds__(256) void tables_batch_kernel(const JobDev *__restrict__ jobs,
                                                           const BatchRir *__restrict__ rirs,
                                                           AxisEntry *__restrict__ tab,
                                                           AxisOrigin *__restrict__ origin,
                                                           int *__restrict__ valid) {
  const BatchRir br = rirs[blockIdx.x];
  const JobDev &jb = jobs[br.job];
  const RoomArgs ra = jb.ra;
  const float *s3 = jb.src + 3 * (br.rir / ra.n_rcv);
  const float *r3 = jb.rcv + 3 * (br.rir % ra.n_rcv);
  AxisEntry *t = tab + jb.tab_base + (size_t)br.rir * ra.n_tab;
  for (int e = threadIdx.x; e < ra.n_tab; e += blockDim.x) t[e] = table_entry(ra, s3, r3, e);
  if (threadIdx.x == 0) {
    AxisOrigin o;
    valid[blockIdx.x] = rir_header(ra, s3, r3, o);
    origin[blockIdx.x] = o;
  }
}

// ---------------------------------------------------------------------------
// Wave-level helpers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Image displacements along one axis are strictly increasing in the lattice
// index n: even n = 2m at m P + e_even, odd n = 2m - 1 at m P + e_odd (P = 2 L q).
// first_ge returns the table index (n - lo) of the first n with displacement
// >= b, or N if there is none. Float rounding can move the answer by one index
// only for images within ~1e-3 samples of b; callers widen their bounds by a
// sample so such images lie outside the band that matters.
struct AxisRange {
  int lo, N;
  float inv_p, e_even, e_odd;
};
__device__ __forceinline__ int family_first(float b, float e, float inv_p, int m_lo, int m_hi) {
  // smallest m in [m_lo, m_hi] with m P + e >= b, or m_hi + 1
  const float mf = ceilf((b - e) * inv_p);
  if (!(mf > (float)m_lo)) return m_lo;  // also -inf
  if (mf > (float)(m_hi + 1)) return m_hi + 1;
  return (int)mf;
}
__device__ __forceinline__ int first_ge(const AxisRange &a, float b) {
  const int hi = a.lo + a.N;  // exclusive
  int best = hi;
  const int me_lo = (a.lo + 1) >> 1, me_hi = (hi - 1) >> 1;  // even n = 2m in [lo, hi)
  if (me_lo <= me_hi) {
    const int m = family_first(b, a.e_even, a.inv_p, me_lo, me_hi);
    if (m <= me_hi) best = min(best, 2 * m);
  }
  const int mo_lo = (a.lo + 2) >> 1, mo_hi = hi >> 1;  // odd n = 2m - 1 in [lo, hi)
  if (mo_lo <= mo_hi) {
    const int m = family_first(b, a.e_odd, a.inv_p, mo_lo, mo_hi);
    if (m <= mo_hi) best = min(best, 2 * m - 1);
  }
  return best - a.lo;
}

// ---------------------------------------------------------------------------
// Kernel 2: enumeration of the image shell of one tile + windowed-sinc taps.
//
// Each wave accumulates into its own FP32 tile in LDS with plain
// read-add-write, one tap at a time: within one instruction the active lanes
// hold images with distinct first-tap positions (enforced by a byte claim per
// position), and a compiler barrier between taps keeps every lane's
// read-modify-write of tap j ahead of any lane's access for tap j + 1, so
// overlapping windows of different lanes never race. At the end the wave tiles
// are summed in a fixed order, which makes results bitwise reproducible.
// ---------------------------------------------------------------------------
constexpr int QCAP = 256;  // per-wave queue of candidate images

// Work of one item: the taps of the images of the shell slab (chunk c of C) of
// output tile tile_id of one RIR, written to dst (the RIR's samples of the
// tile, or a partial tile when C > 1).
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

template <int WT, int NW, bool HALF>
__device__ __forceinline__ void accumulate_item(const RoomArgs &ra, const int tile_id, const int C, const int c,
                                                const AxisEntry *__restrict__ tab, const AxisOrigin &org,
                                                const bool valid, float *__restrict__ dst) {
  constexpr int JLO = 1 - WT / 2;
  constexpr int JHI = WT / 2;
  constexpr int MARGIN = WT;
  constexpr int SPAN = TILE + 2 * MARGIN;
  constexpr TapConsts<WT> K = make_tap_consts<WT>();

  __shared__ float tile[NW][SPAN];
  __shared__ uint8_t claim[NW][SPAN];
  __shared__ uint32_t queue[NW][QCAP];
  __shared__ float col_sh[NW][64], col_sl[NW][64], col_g[NW][64];
  __shared__ int nx_pref[NW][64], nx_nylo[NW][64];

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int T0 = tile_id * TILE;
  const int T1 = min(T0 + TILE, ra.n_samples);

  if (!valid) {
    for (int k = threadIdx.x; k < T1 - T0; k += NW * 64) dst[k] = __builtin_nanf("");
    return;
  }
  const AxisEntry *__restrict__ tx = tab + ra.off[0];
  const AxisEntry *__restrict__ ty = tab + ra.off[1];
  const AxisEntry *__restrict__ tz = tab + ra.off[2];
  const AxisRange ax{ra.lo[0], ra.N[0], ra.inv_period[0], org.e_even[0], org.e_odd[0]};
  const AxisRange ay{ra.lo[1], ra.N[1], ra.inv_period[1], org.e_even[1], org.e_odd[1]};
  const AxisRange az{ra.lo[2], ra.N[2], ra.inv_period[2], org.e_even[2], org.e_odd[2]};

  float *__restrict__ wt = tile[wave];
  uint8_t *__restrict__ wc = claim[wave];
  for (int i = lane; i < SPAN; i += 64) wt[i] = 0.0f;

  // Images whose window reaches the tile have delay x in (T0 - W/2, T1 - 1 + W/2);
  // the enumeration bounds are widened by two samples on each side and every
  // candidate is then filtered exactly on its integer delay.
  const float R1 = (float)(T1 - 1) + ra.half_w + 2.0f;
  const float R0 = (float)T0 - ra.half_w - 2.0f;
  float r1h, r1l, r0h = 0.0f, r0l = 0.0f;
  two_prod(R1, R1, r1h, r1l);
  if (R0 > 0.0f) two_prod(R0, R0, r0h, r0l);

  // Slab of the shell along the x displacement owned by this chunk.
  float dlo = -INFINITY, dhi = INFINITY;
  if (c > 0) dlo = -R1 + (2.0f * R1) * ((float)c / (float)C);
  if (c < C - 1) dhi = -R1 + (2.0f * R1) * ((float)(c + 1) / (float)C);
  const int nx_a = max(first_ge(ax, dlo), first_ge(ax, -R1));
  const int nx_b = min(first_ge(ax, dhi), first_ge(ax, R1));

  // Image held by this lane, with its tap parameters.
  bool has = false;
  float f = 0.0f, C2 = 0.0f, CP = 0.0f, CQ = 0.0f;
  int base = 0;

  // Claim positions, add the taps of the winning lanes (distinct bases).
  auto tap_round = [&]() {
    volatile uint8_t *vc = wc;
    if (has) vc[base] = (uint8_t)lane;
    wave_sync();
    const bool win = has && vc[base] == (uint8_t)lane;
    // Each tap: issue the LDS read, compute the tap while it is in flight, add,
    // write back. The scheduling barrier keeps taps in this order (bounded
    // register use, hence more waves to hide the LDS round trip).
    if (win && !HALF) {
      float *t = wt + base;
#pragma unroll
      for (int jj = 0; jj < WT; ++jj) {
        const float o = t[jj];
        // ties this tap's arithmetic to its place in the chain (no instruction)
        __asm__ volatile("" : "+v"(f), "+v"(CP), "+v"(CQ), "+v"(C2) :: "memory");
        const float u = __builtin_fmaf(-K.sig[jj], f, K.sig_j[jj]);
        const float r = __builtin_amdgcn_rcpf(u);
        float w = __builtin_fmaf(K.cth[jj], CP, C2);
        w = __builtin_fmaf(K.sth[jj], CQ, w);
        t[jj] = __builtin_fmaf(w, r, o);
        __asm__ volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    if (win && HALF) {
      constexpr PolyConsts<WT> P = make_poly_consts<WT>();
      float *t = wt + base;
      const _Float16 th = (_Float16)(f - 0.5f);
      half2_t tt = {th, th};
      const float Cc = 2.0f * C2;
#pragma unroll
      for (int jj = 0; jj < WT; ++jj) {
        const int j = jj + 1 - WT / 2;
        if (!poly_tap(j)) {
          const float o = t[jj];
          __asm__ volatile("" : "+v"(f), "+v"(CP), "+v"(CQ), "+v"(C2) :: "memory");
          const float u = __builtin_fmaf(-K.sig[jj], f, K.sig_j[jj]);
          const float r = __builtin_amdgcn_rcpf(u);
          float w = __builtin_fmaf(K.cth[jj], CP, C2);
          w = __builtin_fmaf(K.sth[jj], CQ, w);
          t[jj] = __builtin_fmaf(w, r, o);
          __asm__ volatile("" ::: "memory");
          __builtin_amdgcn_sched_barrier(0);
        } else if (jj + 1 < WT && poly_tap(j + 1) && ((j <= -2) ? (j - JLO) % 2 == 0 : (j - 3) % 2 == 0)) {
          // taps jj and jj + 1 in one packed register
          const half2_t c3 = {(_Float16)P.c[3][jj], (_Float16)P.c[3][jj + 1]};
          const half2_t c2 = {(_Float16)P.c[2][jj], (_Float16)P.c[2][jj + 1]};
          const half2_t c1 = {(_Float16)P.c[1][jj], (_Float16)P.c[1][jj + 1]};
          const half2_t c0 = {(_Float16)P.c[0][jj], (_Float16)P.c[0][jj + 1]};
          const float o0 = t[jj];
          __asm__ volatile("" : "+v"(tt) :: "memory");
          half2_t pv = __builtin_elementwise_fma(c3, tt, c2);
          pv = __builtin_elementwise_fma(pv, tt, c1);
          pv = __builtin_elementwise_fma(pv, tt, c0);
          t[jj] = __builtin_fmaf((float)pv.x, Cc, o0);
          __asm__ volatile("" ::: "memory");
          const float o1 = t[jj + 1];
          t[jj + 1] = __builtin_fmaf((float)pv.y, Cc, o1);
          __asm__ volatile("" ::: "memory");
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    has = has && !win;
    wave_sync();
  };

  for (int nx0 = nx_a; nx0 < nx_b; nx0 += 64) {
    // lanes = x indices: y range of the columns that reach the outer sphere
    const int nxi = nx0 + lane;
    int ny_lo = 0, ny_cnt = 0;
    if (nxi < nx_b) {
      const AxisEntry ex = tx[nxi];
      float qh, ql, rh, rl;
      ff_sq(ex.d_hi, ex.d_lo, qh, ql);
      ff_sub(r1h, r1l, qh, ql, rh, rl);
      if (rh > 0.0f) {
        const float R = __builtin_sqrtf(rh) + 1.0f;
        ny_lo = first_ge(ay, -R);
        ny_cnt = first_ge(ay, R) - ny_lo;
      }
    }
    const int incl_y = wave_incl_scan(ny_cnt);
    const int ncols = __builtin_amdgcn_readlane(incl_y, 63);
    nx_pref[wave][lane] = incl_y - ny_cnt;
    nx_nylo[wave][lane] = ny_lo;
    wave_sync();

    for (int cb = wave; cb * 64 < ncols; cb += NW) {
      // lanes = columns (nx, ny): z ranges of the shell
      const int g = cb * 64 + lane;
      int z1 = 0, n1 = 0, z2 = 0, n2 = 0;
      if (g < ncols) {
        int i = 0;
#pragma unroll
        for (int step = 32; step > 0; step >>= 1)
          if (i + step < 64 && nx_pref[wave][i + step] <= g) i += step;
        const AxisEntry ex = tx[nx0 + i];
        const AxisEntry ey = ty[nx_nylo[wave][i] + (g - nx_pref[wave][i])];
        float ah, al, bh, bl, sh, sl;
        ff_sq(ex.d_hi, ex.d_lo, ah, al);
        ff_sq(ey.d_hi, ey.d_lo, bh, bl);
        two_sum(ah, bh, sh, sl);
        sl += al + bl;
        fast_two_sum(sh, sl, sh, sl);
        col_sh[wave][lane] = sh;
        col_sl[wave][lane] = sl;
        col_g[wave][lane] = ex.gain * ey.gain;
        float rh, rl;
        ff_sub(r1h, r1l, sh, sl, rh, rl);
        if (rh > 0.0f) {
          const float zmax = __builtin_sqrtf(rh) + 1.0f;
          float zmin = 0.0f;
          if (R0 > 0.0f) {
            float hh, hl;
            ff_sub(r0h, r0l, sh, sl, hh, hl);
            if (hh > 0.0f) zmin = fmaxf(__builtin_sqrtf(hh) - 1.0f, 0.0f);
          }
          if (zmin > 0.0f) {
            z1 = first_ge(az, -zmax);
            n1 = max(first_ge(az, -zmin) - z1, 0);
            z2 = first_ge(az, zmin);
            n2 = max(first_ge(az, zmax) - z2, 0);
          } else {
            z1 = first_ge(az, -zmax);
            n1 = max(first_ge(az, zmax) - z1, 0);
          }
        }
      }
      const int cnt = n1 + n2;
      const int incl = wave_incl_scan(cnt);
      const int total = __builtin_amdgcn_readlane(incl, 63);
      const int excl = incl - cnt;

      for (int q0 = 0; q0 < total; q0 += QCAP) {
        // lanes write their candidates with wave-wide index in [q0, q0 + QCAP)
        const int i_lo = max(0, q0 - excl), i_hi = min(cnt, q0 + QCAP - excl);
        for (int i = i_lo; i < i_hi; ++i) {
          const int nz = (i < n1) ? z1 + i : z2 + (i - n1);
          queue[wave][excl + i - q0] = ((uint32_t)lane << 16) | (uint32_t)nz;
        }
        wave_sync();
        const int qn = min(QCAP, total - q0);
        int qpos = 0;
        while (qpos < qn) {
          // refill the lanes without an image from the queue (lanes = images)
          const bool need = !has;
          const uint64_t need_mask = __ballot(need);
          const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(need_mask >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)need_mask, 0u));
          if (need && qpos + rank < qn) {
            const uint32_t ent = queue[wave][qpos + rank];
            const int cl = (int)(ent >> 16);
            const int nz = (int)(ent & 0xffffu);
            const AxisEntry ez = tz[nz];
            float ph, pl, s, se, Sh, Sl;
            ff_sq(ez.d_hi, ez.d_lo, ph, pl);
            two_sum(col_sh[wave][cl], ph, s, se);
            se += col_sl[wave][cl] + pl;
            fast_two_sum(s, se, Sh, Sl);
            // x = sqrt(S) in samples (Eq. (2)-(3)): one Newton correction in float-float
            const float x0 = __builtin_amdgcn_sqrtf(Sh);
            const float rx = __builtin_amdgcn_rcpf(x0);
            const float xl = (__builtin_fmaf(-x0, x0, Sh) + Sl) * (0.5f * rx);
            float kf = floorf(x0);
            float fr = (x0 - kf) + xl;
            if (fr < 0.0f) {
              fr += 1.0f;
              kf -= 1.0f;
            }
            if (fr >= 1.0f) {
              fr -= 1.0f;
              kf += 1.0f;
            }
            const int k0 = (int)kf;
            base = k0 + JLO - T0 + MARGIN;
            has = (x0 < 1.0e9f) && (k0 + JHI >= T0) && (k0 + JLO <= T1 - 1) && base >= 0 && base + WT <= SPAN;
            // Eq. (4) amplitude and the per-image factors of the taps
            const float A = col_g[wave][cl] * ez.gain * ra.kappa * rx;
            f = fmaxf(fr, 0x1p-100f);
            const float Cc = A * sinpi_over_pi(fminf(f, 1.0f - f));
            float sp, cp;
            small_sincos(f * ra.two_pi_over_w, sp, cp);
            C2 = 0.5f * Cc;
            CP = C2 * cp;
            CQ = C2 * sp;
          }
          qpos += __builtin_popcountll(need_mask);
          tap_round();
        }
        wave_sync();
      }
    }
    wave_sync();
  }
  // images still waiting after their queue ran out
  while (__ballot(has) != 0) tap_round();

  __syncthreads();
  for (int k = threadIdx.x; k < T1 - T0; k += NW * 64) {
    float v = 0.0f;
#pragma unroll
    for (int w = 0; w < NW; ++w) v += tile[w][MARGIN + k];
    dst[k] = v;
  }
}

// Single-room launch: the item index decodes through the per-tile chunk counts.
template <int WT, int NW, bool HALF>
__global__ __launch_bounds__(NW * 64) void accumulate_kernel(RoomArgs ra, PlanArgs pa,
                                                             const AxisEntry *__restrict__ tab_all,
                                                             const AxisOrigin *__restrict__ origin,
                                                             const int *__restrict__ valid, float *__restrict__ out,
                                                             float *__restrict__ part) {
  const uint32_t item = blockIdx.x;
  int pos = 0;
  {
    int lo = 0, hi = pa.n_tiles;  // largest pos with first_item[pos] <= item
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (pa.first_item[mid] <= item) lo = mid;
      else hi = mid;
    }
    pos = lo;
  }
  const int tile_id = pa.n_tiles - 1 - pos;
  const int C = pa.chunks[tile_id];
  const uint32_t rel = item - pa.first_item[pos];
  const int rir = (int)(rel / (uint32_t)C);
  const int c = (int)(rel % (uint32_t)C);
  float *dst = (C == 1) ? out + (size_t)rir * ra.n_samples + (size_t)tile_id * TILE : part + (size_t)item * TILE;
  const AxisOrigin org = origin[rir];
  accumulate_item<WT, NW, HALF>(ra, tile_id, C, c, tab_all + (size_t)rir * ra.n_tab, org, valid[rir] != 0, dst);
}

// Batch launch: every item names its job; the job table carries the room.
template <int WT, int NW, bool HALF>
__global__ __launch_bounds__(NW * 64) void accumulate_batch_kernel(const JobDev *__restrict__ jobs,
                                                                   const BatchItem *__restrict__ items,
                                                                   const AxisEntry *__restrict__ tab_all,
                                                                   const AxisOrigin *__restrict__ origin,
                                                                   const int *__restrict__ valid,
                                                                   float *__restrict__ part) {
  const BatchItem it = items[blockIdx.x];
  const JobDev &jb = jobs[it.job];
  const RoomArgs ra = jb.ra;
  const uint32_t grir = jb.rir_base + it.rir;
  float *dst = (it.slot == 0xffffffffu) ? jb.out + (size_t)it.rir * ra.n_samples + (size_t)it.tile * TILE
                                        : part + (size_t)it.slot * TILE;
  const AxisOrigin org = origin[grir];
  accumulate_item<WT, NW, HALF>(ra, it.tile, it.chunks, it.chunk, tab_all + jb.tab_base + (size_t)it.rir * ra.n_tab, org,
                          valid[grir] != 0, dst);
}

// ---------------------------------------------------------------------------
// Kernel 3: ordered sum of the partial tiles of split tiles.
// grid = (rir, dispatch position of the tile, 256-sample segment)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void reduce_kernel(RoomArgs ra, PlanArgs pa, const float *__restrict__ part,
                                                     float *__restrict__ out) {
  const int pos = blockIdx.y;
  const int tile_id = pa.n_tiles - 1 - pos;
  const int C = pa.chunks[tile_id];
  if (C <= 1) return;
  const int rir = blockIdx.x;
  const int T0 = tile_id * TILE;
  const int T1 = min(T0 + TILE, ra.n_samples);
  const int k = blockIdx.z * 256 + threadIdx.x;
  if (k >= T1 - T0) return;
  const size_t first = (size_t)pa.first_item[pos] + (size_t)rir * C;
  float v = 0.0f;
  for (int cc = 0; cc < C; ++cc) v += part[(first + cc) * TILE + k];
  out[(size_t)rir * ra.n_samples + T0 + k] = v;
}

// Batch mode: grid = (split tile, 256-sample segment).
__global__ __launch_bounds__(256) void reduce_batch_kernel(const JobDev *__restrict__ jobs,
                                                           const BatchReduce *__restrict__ red,
                                                           const float *__restrict__ part) {
  const BatchReduce br = red[blockIdx.x];
  const JobDev &jb = jobs[br.job];
  const int n_samples = jb.ra.n_samples;
  const int T0 = (int)br.tile * TILE;
  const int T1 = min(T0 + TILE, n_samples);
  const int k = blockIdx.y * 256 + threadIdx.x;
  if (k >= T1 - T0) return;
  float v = 0.0f;
  for (int cc = 0; cc < br.chunks; ++cc) v += part[((size_t)br.first + cc) * TILE + k];
  jb.out[(size_t)br.rir * n_samples + T0 + k] = v;
}

// ---------------------------------------------------------------------------
// Launchers (called from ism_host.cpp).
// ---------------------------------------------------------------------------
int launch_tables(const RoomArgs &ra, const float *src, const float *rcv, AxisEntry *tab, AxisOrigin *origin,
                  int *valid, int n_rir, hipStream_t st) {
  const int64_t total = (int64_t)n_rir * ra.n_tab;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65535) blocks = 65535;
  hipLaunchKernelGGL(tables_kernel, dim3((unsigned)blocks), dim3(256), 0, st, ra, src, rcv, tab, origin, valid,
                     n_rir);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int WT, bool HALF>
static int launch_acc_w(const RoomArgs &ra, const PlanArgs &pa, uint32_t n_items, const AxisEntry *tab,
                        const AxisOrigin *origin, const int *valid, float *out, float *part, hipStream_t st) {
  constexpr int NW = 4;
  hipLaunchKernelGGL((accumulate_kernel<WT, NW, HALF>), dim3(n_items), dim3(NW * 64), 0, st, ra, pa, tab, origin,
                     valid, out, part);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

bool supported_window(int wt) { return wt == 32 || wt == 64 || wt == 96 || wt == 128; }

int launch_accumulate(int wt, bool half, const RoomArgs &ra, const PlanArgs &pa, uint32_t n_items,
                      const AxisEntry *tab, const AxisOrigin *origin, const int *valid, float *out, float *part,
                      hipStream_t st) {
#define ISM_ACC(W)                                                                             \
  case W:                                                                                      \
    return half ? launch_acc_w<W, true>(ra, pa, n_items, tab, origin, valid, out, part, st)    \
                : launch_acc_w<W, false>(ra, pa, n_items, tab, origin, valid, out, part, st);
  switch (wt) {
    ISM_ACC(32)
    ISM_ACC(64)
    ISM_ACC(96)
    ISM_ACC(128)
    default: return -2;
  }
#undef ISM_ACC
}

template <int WT, bool HALF>
static int launch_acc_batch_w(const JobDev *jobs, const BatchItem *items, uint32_t n_items, const AxisEntry *tab,
                              const AxisOrigin *origin, const int *valid, float *part, hipStream_t st) {
  constexpr int NW = 4;
  hipLaunchKernelGGL((accumulate_batch_kernel<WT, NW, HALF>), dim3(n_items), dim3(NW * 64), 0, st, jobs, items, tab,
                     origin, valid, part);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_batch(const JobDev *jobs, const BatchRir *rirs, uint32_t n_rir, const BatchItem *items,
                 const uint32_t *class_first, const uint32_t *class_count, const int *class_wt, int n_classes,
                 bool half, const BatchReduce *red, uint32_t n_red, AxisEntry *tab, AxisOrigin *origin, int *valid,
                 float *part, hipStream_t st, hipEvent_t ev_start, hipEvent_t ev_stop) {
  hipLaunchKernelGGL(tables_batch_kernel, dim3(n_rir), dim3(256), 0, st, jobs, rirs, tab, origin, valid);
  if (hipGetLastError() != hipSuccess) return -1;
  if (ev_start && hipEventRecord(ev_start, st) != hipSuccess) return -1;
  for (int k = 0; k < n_classes; ++k) {
    if (class_count[k] == 0) continue;
    const BatchItem *it = items + class_first[k];
    int rc = -2;
#define ISM_BACC(W)                                                                                     \
  case W:                                                                                               \
    rc = half ? launch_acc_batch_w<W, true>(jobs, it, class_count[k], tab, origin, valid, part, st)     \
              : launch_acc_batch_w<W, false>(jobs, it, class_count[k], tab, origin, valid, part, st);   \
    break;
    switch (class_wt[k]) {
      ISM_BACC(32)
      ISM_BACC(64)
      ISM_BACC(96)
      ISM_BACC(128)
      default: break;
    }
#undef ISM_BACC
    if (rc != 0) return -1;
  }
  if (ev_stop && hipEventRecord(ev_stop, st) != hipSuccess) return -1;
  if (n_red > 0) {
    hipLaunchKernelGGL(reduce_batch_kernel, dim3(n_red, TILE / 256), dim3(256), 0, st, jobs, red, part);
    if (hipGetLastError() != hipSuccess) return -1;
  }
  return 0;
}

int launch_reduce(const RoomArgs &ra, const PlanArgs &pa, int n_rir, const float *part, float *out,
                  hipStream_t st) {
  hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)n_rir, (unsigned)pa.n_tiles, TILE / 256), dim3(256), 0, st, ra,
                     pa, part, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace ism
