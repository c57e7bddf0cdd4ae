// HIP kernels of the Image Source Method for gfx950 (MI355X).
//
// Three kernels per call:
//   tables_kernel      per (RIR, axis, lattice index): displacement of the image
//                      coordinate from the receiver in samples (float-float) and
//                      the axis factor of the reflection gain (Sec. 2.1, Eq. (1)
//                      and the gain rule below it); for directional receivers
//                      also the displacement's share of the projection onto the
//                      receiver's orientation. Also flags invalid pairs.
//   accumulate_kernel  per work item (RIR, output tile, slab of the image shell):
//                      enumerates exactly the lattice images whose window can
//                      reach the tile, computes each image's delay and amplitude
//                      (Eq. (2)-(4), times the receiver's polar pattern when
//                      directional) and adds its Hann-windowed-sinc taps
//                      (Eq. (6): FP32, packed FP16, or read from the table of
//                      Eq. (9)) into wave-private FP32 LDS tiles (Eq. (5)).
//   reduce_kernel      sums, in a fixed order, the partial tiles of tiles that
//                      were split over several work items.
//
// Geometry and accumulation are FP32 only; delays use error-free
// transformations so that the fractional delay keeps ~1e-7 sample accuracy at
// 1e5-sample distances.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdio.h>

#include <type_traits>

#include "ism.h"
#include "ism_internal.h"
#include "ism_math.h"

namespace ism {

// Bits of a staged record that carry the tile-local base of an image (its
// integer delay minus the tile start), and the mask that extracts them.
constexpr int kBaseBits = (TILE <= 256) ? 8 : 9;
constexpr uint32_t kBaseMask = (1u << kBaseBits) - 1u;
static_assert(TILE <= (1 << kBaseBits), "tile-local bases must fit the record");
// The delay fraction of the table-tap record (and of the FP32 record where
// cq_base is false), in units of 2^-kFracBits.
constexpr int kFracBits = 32 - kBaseBits;
// Whether the FP32 record of window cap wt carries the base in CQ's low
// mantissa bits (else beside the fraction): all but general windows of the
// 32-sample cap.
constexpr bool cq_base(int wt, bool gen) { return !(gen && wt == 32); }

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
// (b + bl)^e for e >= 0 by binary powering in float-float (0^0 = 1): the
// reflection coefficient keeps its double-precision value, so the gain of an
// image many reflections deep is accurate to a few FP32 ulp.
__device__ float ff_pow(float b, float b_lo, int e) {
  float rh = 1.0f, rl = 0.0f, bh = b, bl = b_lo;
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

// FP16 taps. For one image with fractional delay f, tap j (Eq. (6) at
// v = j - f) is A s_j(t) with t = f - 1/2 in [-1/2, 1/2) and
//   s_j(t) = sinc(j - f) (1 + cos(2 pi (j - f) / W)) / 2,
// an entire function of t. Each s_j is replaced by its interpolant of degree
// SPD at the Chebyshev nodes of [-1/2, 1/2] (interpolation error < 6e-5),
// written as c0 + t q(t), q = c1 + c2 t + ... + c5 t^4. A tap then adds
// A c0 in FP32 and q(t) (A t), with q evaluated in packed FP16 (two taps per
// register) and the product and sum in FP32. FP16 rounding of q and t bounds
// the tap error by ~6e-4 A at the central taps and ~2.5e-4 A elsewhere.
constexpr int SPD = 5;
template <int WT>
struct SincPoly {
  float c[SPD + 1][WT];  // c[k][jj] multiplies t^k for tap j = jj + 1 - W/2
};
constexpr double s_tap(int j, double t, int wt) {
  const double f = t + 0.5;  // in (0, 1) at the nodes, so j - f != 0
  const double v = j - f;
  const double sg = (j % 2 == 0) ? -1.0 : 1.0;  // sin(pi v) = sg sin(pi f)
  return sg * cx_sin(kPi * f) / (kPi * v) * 0.5 * (1.0 + cx_cos(2.0 * kPi * v / wt));
}
template <int WT>
constexpr SincPoly<WT> make_sinc_poly() {
  constexpr int NP = SPD + 1;
  SincPoly<WT> P{};
  for (int jj = 0; jj < WT; ++jj) {
    const int j = jj + 1 - WT / 2;
    double x[NP] = {}, y[NP] = {};
    for (int k = 0; k < NP; ++k) {
      x[k] = 0.5 * cx_cos((2.0 * k + 1.0) * kPi / (2.0 * NP));
      y[k] = s_tap(j, x[k], WT);
    }
    // Newton divided differences, then expansion to monomials
    double d[NP] = {};
    for (int k = 0; k < NP; ++k) d[k] = y[k];
    for (int lvl = 1; lvl < NP; ++lvl)
      for (int k = NP - 1; k >= lvl; --k) d[k] = (d[k] - d[k - 1]) / (x[k] - x[k - lvl]);
    double m[NP] = {};  // coefficients of the running polynomial, highest first
    m[0] = d[NP - 1];
    int deg = 0;
    for (int k = NP - 2; k >= 0; --k) {  // m(t) = m(t) * (t - x[k]) + d[k]
      double nm[NP] = {};
      for (int q = 0; q <= deg; ++q) {
        nm[q] += m[q];
        nm[q + 1] -= m[q] * x[k];
      }
      ++deg;
      nm[deg] += d[k];
      for (int q = 0; q < NP; ++q) m[q] = nm[q];
    }
    for (int q = 0; q < NP; ++q) P.c[SPD - q][jj] = (float)m[q];
  }
  return P;
}

// Monomial coefficients of the degree-SPD interpolant at the Chebyshev nodes
// of [-1/2, 1/2]: c = V^-1 y for the node values y, V the Vandermonde matrix
// of the nodes (inverted in double by the compiler, Gauss-Jordan with partial
// pivoting). Used for general-mode FP16 windows, whose interpolants are
// computed per call.
struct ChebFit {
  float node[SPD + 1];
  float vinv[SPD + 1][SPD + 1];  // vinv[k][i]: coefficient of t^k per unit value at node i
  float sin_pi_f[SPD + 1];       // sin(pi f_i) / pi at f_i = node_i + 1/2
};
constexpr ChebFit make_cheb_fit() {
  constexpr int NP = SPD + 1;
  ChebFit F{};
  double x[NP] = {}, a[NP][2 * NP] = {};
  for (int i = 0; i < NP; ++i) x[i] = 0.5 * cx_cos((2.0 * i + 1.0) * kPi / (2.0 * NP));
  for (int i = 0; i < NP; ++i) {  // [V | I], V[i][k] = x_i^k
    double pw = 1.0;
    for (int k = 0; k < NP; ++k) {
      a[i][k] = pw;
      pw *= x[i];
    }
    a[i][NP + i] = 1.0;
  }
  for (int c = 0; c < NP; ++c) {
    int piv = c;
    for (int r = c + 1; r < NP; ++r)
      if ((a[r][c] < 0 ? -a[r][c] : a[r][c]) > (a[piv][c] < 0 ? -a[piv][c] : a[piv][c])) piv = r;
    for (int k = 0; k < 2 * NP; ++k) {
      const double t = a[c][k];
      a[c][k] = a[piv][k];
      a[piv][k] = t;
    }
    const double d = a[c][c];
    for (int k = 0; k < 2 * NP; ++k) a[c][k] /= d;
    for (int r = 0; r < NP; ++r)
      if (r != c) {
        const double m = a[r][c];
        for (int k = 0; k < 2 * NP; ++k) a[r][k] -= m * a[c][k];
      }
  }
  // V^-1 maps node values to coefficients: c_k = sum_i (V^-1)[k][i] y_i
  for (int k = 0; k < NP; ++k)
    for (int i = 0; i < NP; ++i) F.vinv[k][i] = (float)a[k][NP + i];
  for (int i = 0; i < NP; ++i) {
    F.node[i] = (float)x[i];
    F.sin_pi_f[i] = (float)(cx_sin(kPi * (x[i] + 0.5)) / kPi);  // pi (x + 1/2) in (0, pi)
  }
  return F;
}
__constant__ ChebFit kChebFit = make_cheb_fit();

// Constants of tap jj (j = jj + 1 - WT/2) of a general-mode window of W
// samples under cap WT, for FP32 (half == 0) or FP16 (half == 1) taps, into
// e[0 .. WC_STRIDE). FP16: the interpolant of s_j(t) = tap value at
// f = t + 1/2 (Eq. (6), 0 where |j - f| >= W/2) at the Chebyshev nodes.
__device__ void window_const_entry(float W, int WT, int half, int jj, float *e) {
  const int j = jj + 1 - WT / 2;
  const float sg = (j & 1) ? 1.0f : -1.0f;  // sin(pi (j - f)) = sg sin(pi f)
  for (int k = 0; k < WC_STRIDE; ++k) e[k] = 0.0f;
  if (!half) {
    float sn, cs;
    sincospi_acc(2.0f * (float)j / W, sn, cs);
    e[0] = cq_base(WT, true) ? -sg : -sg * 0x1p-32f;  // times f, or times float(F) = f 2^32
    e[1] = sg * (float)j;
    e[2] = cs;
    e[3] = sn;
    return;
  }
  float y[SPD + 1];
  for (int i = 0; i <= SPD; ++i) {
    const float f = kChebFit.node[i] + 0.5f;
    const float v = (float)j - f;
    float sn, cs;
    sincospi_acc(2.0f * v / W, sn, cs);
    y[i] = (__builtin_fabsf(v) < 0.5f * W) ? sg * kChebFit.sin_pi_f[i] / v * 0.5f * (1.0f + cs) : 0.0f;
  }
  for (int k = 0; k <= SPD; ++k) {
    float ck = 0.0f;
    for (int i = 0; i <= SPD; ++i) ck = __builtin_fmaf(kChebFit.vinv[k][i], y[i], ck);
    e[k] = ck;
  }
}

// Lookup-table taps (Eq. (9)): the windowed sinc of Eq. (6) tabulated at Q
// points per sample, L[n] = (1 + cos(2 pi n / (Q W))) / 2 sinc(n / Q) for
// n = -QW/2 .. QW/2, and each tap interpolated linearly between the two
// entries around its delay. For tap j of an image with fraction f = (fl + fr)/Q
// (fl an integer in [0, Q), fr in [0, 1)), v = j - f lies between entries
// n0 = Q j - fl - 1 and n0 + 1, with weight 1 - fr on the upper one. All taps
// of one image share fl, so the table is stored phase-major: entry
// (ph, m) = (L[i], L[i + 1] - L[i]) with i = n0 + QW/2 = Q m + ph,
// ph = Q - 1 - fl and m = j + W/2 - 1; the lanes of an image read consecutive
// entries of one row.
constexpr int kLutQ = 16;
template <int WT>
struct alignas(16) LutPairs {
  float p[kLutQ][WT][2];
};
constexpr double lut_entry(int i, int wt) {  // L[i - QW/2]
  const int n = i - kLutQ * wt / 2;
  const double hann = 0.5 * (1.0 + cx_cos(2.0 * kPi * n / (kLutQ * wt)));  // angle in [-pi, pi]
  if (n == 0) return hann;
  // sin(pi n / Q) with n = Q m + r, 0 <= r < Q: (-1)^m sin(pi r / Q), keeping
  // the series argument in [0, pi)
  const int r = ((n % kLutQ) + kLutQ) % kLutQ;
  const int m = (n - r) / kLutQ;
  const double s = ((m & 1) ? -1.0 : 1.0) * cx_sin(kPi * r / kLutQ);
  const double v = (double)n / kLutQ;
  return hann * s / (kPi * v);
}
template <int WT>
constexpr LutPairs<WT> make_lut_pairs() {
  LutPairs<WT> t{};
  double L[kLutQ * WT + 1] = {};
  for (int i = 0; i <= kLutQ * WT; ++i) L[i] = lut_entry(i, WT);
  L[kLutQ * WT] = 0.0;  // the window's end (1 + cos(pi) = 0)
  for (int ph = 0; ph < kLutQ; ++ph)
    for (int m = 0; m < WT; ++m) {
      const int i = kLutQ * m + ph;
      t.p[ph][m][0] = (float)L[i];
      t.p[ph][m][1] = (float)(L[i + 1] - L[i]);
    }
  return t;
}

// ---------------------------------------------------------------------------
// Kernel 1: per-RIR axis tables.
// ---------------------------------------------------------------------------
// Table entry e (axis a, lattice index n) of the RIR with source s, receiver r.
__device__ __forceinline__ AxisEntry table_entry(const RoomArgs &ra, const float *__restrict__ s3,
                                                 const float *__restrict__ r3, int e,
                                                 const float *__restrict__ o3 = nullptr) {
  const int a = e < ra.off[1] ? 0 : (e < ra.off[2] ? 1 : 2);
  const int n = ra.lo[a] + (e - ra.off[a]);
  const float s = s3[ra.perm[a]], r = r3[ra.perm[a]];
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
  const float g = ff_pow(ra.beta[2 * a], ra.beta_lo[2 * a], e0) * ff_pow(ra.beta[2 * a + 1], ra.beta_lo[2 * a + 1], e1);
  // the enumeration only needs the square of the displacement
  float sq, sqe;
  ff_sq(v, ve, sq, sqe);
  // receiver orientation (polar calls): the displacement's share of the
  // projection onto the unit orientation, whose three shares add up to
  // |d| cos(theta) in samples
  float proj = 0.0f;
  if (o3) {
    const float inv = __builtin_amdgcn_rsqf(o3[0] * o3[0] + o3[1] * o3[1] + o3[2] * o3[2]);
    proj = v * (o3[ra.perm[a]] * inv);
  }
  return AxisEntry{sq, sqe, g, proj};
}

// Validity of a pair (both points strictly inside, distinct) and the family
// offsets of its axes.
__device__ __forceinline__ int rir_header(const RoomArgs &ra, const float *__restrict__ s3,
                                          const float *__restrict__ r3, AxisOrigin &o) {
  bool ok = true, same = true;
  for (int b = 0; b < 3; ++b) {
    const float sb = s3[ra.perm[b]], rb = r3[ra.perm[b]];
    ok = ok && sb > 0.0f && (sb - ra.L_hi[b]) < ra.L_lo[b] && rb > 0.0f && (rb - ra.L_hi[b]) < ra.L_lo[b];
    same = same && (sb == rb);
    o.e_even[b] = (sb - rb) * ra.q_hi;
    o.e_odd[b] = (-sb - rb) * ra.q_hi;
  }
  return (ok && !same) ? 1 : 0;
}

__global__ __launch_bounds__(256) void tables_kernel(RoomArgs ra, const float *__restrict__ src,
                                                     const float *__restrict__ rcv,
                                                     const float *__restrict__ orient, AxisEntry *__restrict__ tab,
                                                     AxisOrigin *__restrict__ origin, int *__restrict__ valid,
                                                     int n_rir) {
  const int64_t total = (int64_t)n_rir * ra.n_tab;
  for (int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gid < total;
       gid += (int64_t)gridDim.x * blockDim.x) {
    const int rir = (int)(gid / ra.n_tab);
    const int e = (int)(gid % ra.n_tab);
    const float *s3 = src + 3 * (rir / ra.n_rcv);
    const float *r3 = rcv + 3 * (rir % ra.n_rcv);
    tab[gid] = table_entry(ra, s3, r3, e, orient ? orient + 3 * (rir % ra.n_rcv) : nullptr);
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
  const float *o3 = jb.orient ? jb.orient + 3 * (br.rir % ra.n_rcv) : nullptr;
  for (int e = threadIdx.x; e < ra.n_tab; e += blockDim.x) t[e] = table_entry(ra, s3, r3, e, o3);
  if (threadIdx.x == 0) {
    AxisOrigin o;
    valid[blockIdx.x] = rir_header(ra, s3, r3, o);
    origin[blockIdx.x] = o;
  }
}

// ---------------------------------------------------------------------------
// Wave-level helpers.
// ---------------------------------------------------------------------------
// Inclusive prefix sum over the 64 lanes with DPP lane shifts (no LDS):
// Hillis-Steele within each row of 16 lanes, then the row totals are carried
// into the later rows by the row broadcasts of lanes 15 and 31.
__device__ __forceinline__ int wave_incl_scan(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1, 3
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2, 3
  return v;
}
// Inclusive running maximum over the 64 lanes of non-negative values, same
// lane pattern as wave_incl_scan.
__device__ __forceinline__ int wave_incl_max(int v) {
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false));
  return v;
}
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Image displacements along one axis are strictly increasing in the lattice
// index n: even n = 2m at m P + e_even, odd n = 2m - 1 at m P + e_odd (P = 2 L q).
// The table index (n - lo) of the first n with displacement >= b is therefore
// the number of images below b, which first_ge counts family by family:
// family f holds M_f images m = m0_f .. m0_f + M_f - 1, of which
// clamp(ceil((b - e_f) / P) - m0_f, 0, M_f) lie below b. Float rounding can
// move the count by one only for images within ~1e-2 samples of b; callers
// widen their bounds by a sample so such images lie outside the band that
// matters. first_ge is monotone in b and a pure function of it, so equal
// bounds split a range exactly.
struct AxisRange {
  float inv_p;            // 1 / P
  float c_even, c_odd;    // -(e_f / P + m0_f)
  float n_even, n_odd;    // M_f
};
__device__ __forceinline__ AxisRange axis_range(int lo, int N, float inv_p, float e_even, float e_odd) {
  const int hi = lo + N;  // exclusive
  const int me0 = (lo + 1) >> 1, me1 = (hi - 1) >> 1;  // even n = 2m in [lo, hi)
  const int mo0 = (lo + 2) >> 1, mo1 = hi >> 1;        // odd n = 2m - 1 in [lo, hi)
  AxisRange a;
  a.inv_p = inv_p;
  a.c_even = -__builtin_fmaf(e_even, inv_p, (float)me0);
  a.c_odd = -__builtin_fmaf(e_odd, inv_p, (float)mo0);
  a.n_even = (float)max(me1 - me0 + 1, 0);
  a.n_odd = (float)max(mo1 - mo0 + 1, 0);
  return a;
}
__device__ __forceinline__ int first_ge(const AxisRange &a, float b) {
  const float ce = fminf(fmaxf(ceilf(__builtin_fmaf(b, a.inv_p, a.c_even)), 0.0f), a.n_even);
  const float co = fminf(fmaxf(ceilf(__builtin_fmaf(b, a.inv_p, a.c_odd)), 0.0f), a.n_odd);
  return (int)(ce + co);
}

// ---------------------------------------------------------------------------
// Kernel 2: enumeration of the image shell of one tile + windowed-sinc taps.
//
// Work item = (RIR, output tile, slab of the image shell along x). The wave
// walks the columns (nx, ny) that cross the shell, numbers their z candidates
// and hands them to a consumer that turns candidates into image
// parameters (delay, amplitude; lanes = images) and adds their taps.
//
// Tap consumer (lanes = taps, both precisions): the candidates' parameters
// are staged in LDS; each half-wave then takes one staged image per step and
// its 32 lanes add W/32 taps each into the half-wave's own FP32 tile. All
// addresses of one step are distinct and consecutive, so there are no bank
// conflicts and no lost updates; steps of a half-wave reach LDS in program
// order. FP32 taps divide by the sinc argument; FP16 taps evaluate a
// per-tap polynomial in packed FP16.
//
// Items end with a fixed-order sum of the tiles, so results are bitwise
// reproducible.
// ---------------------------------------------------------------------------
typedef int int4v __attribute__((ext_vector_type(4)));
typedef float float2v __attribute__((ext_vector_type(2)));

// Per-wave LDS of the shell enumeration. The candidates of a batch of 64
// columns are numbered 0 .. total-1, column by column; column lane c holds
// positions [excl_c, excl_c + n1_c + n2_c), its first run of z indices
// (z1_c ..) then its second (z2_c ..).
struct EnumLds {
  int mark[64];        // per chunk of 64 positions: column lane + 1 where a column starts
  int4v col_run[64];   // (excl + n1, z1 - excl, z2 - n1 - excl, gain bits): position p
                       // of the column has z index p + (p < excl + n1 ? z1 - excl : z2 - n1 - excl)
  float2v col_s[64];   // column part of the squared distance (float-float)
  // per x lane of the row batch: (first column << 11) | first y table index
  // (column counts stay below 64 * 2048 = 2^17, table indices below 2^11)
  uint32_t nx_col[64];
};
static_assert(ISM_MAX_N_IMG <= 2048, "nx_col packs y table indices in 11 bits");

// Wave-uniform geometry of one work item.
struct ItemGeom {
  int T0, T1;                    // output samples [T0, T1) of the tile (empty past nS)
  int K1;                        // owned integer delays: k0 in [T0, K1)
  float R0, R1;                  // shell radii in samples, widened by 2
  float r1h, r1l, r0h, r0l;      // their squares (float-float)
  int nx_a, nx_b;                // x table indices of the slab
};

__device__ __forceinline__ ItemGeom item_geom(const RoomArgs &ra, const AxisRange &ax, int tile_id, int C, int c) {
  ItemGeom g;
  g.T0 = tile_id * TILE;
  g.T1 = min(g.T0 + TILE, ra.n_samples);
  g.K1 = min(g.T0 + TILE, ra.k_end);
  // The owned images have delay x in [T0, K1); the enumeration bounds are
  // widened by two samples on each side and every candidate is then filtered
  // exactly on its integer delay.
  g.R1 = (float)g.K1 + 2.0f;
  g.R0 = (float)g.T0 - 2.0f;
  two_prod(g.R1, g.R1, g.r1h, g.r1l);
  g.r0h = 0.0f;
  g.r0l = 0.0f;
  if (g.R0 > 0.0f) two_prod(g.R0, g.R0, g.r0h, g.r0l);
  // Slab of the shell along the x displacement owned by chunk c of C.
  float dlo = -INFINITY, dhi = INFINITY;
  if (c > 0) dlo = -g.R1 + (2.0f * g.R1) * ((float)c / (float)C);
  if (c < C - 1) dhi = -g.R1 + (2.0f * g.R1) * ((float)(c + 1) / (float)C);
  g.nx_a = max(first_ge(ax, dlo), first_ge(ax, -g.R1));
  g.nx_b = min(first_ge(ax, dhi), first_ge(ax, g.R1));
  return g;
}

// Walks the shell of the item. For every batch of 64 columns with candidates
// it fills es.col_run and es.col_s and calls consume(total, excl, cnt): total
// candidates in the batch, and on column lane c its first position excl and
// its count cnt. The column gain in col_run is the product of the x and y
// gain factors times gscale.
// DUMP (enumeration check): col_xy receives each column's x and y table
// indices, (x << 16) | y.
template <bool POLAR, bool DUMP, class Consume>
__device__ __forceinline__ void enumerate_shell(const ItemGeom &g, const AxisEntry *__restrict__ tx,
                                                const AxisEntry *__restrict__ ty, const AxisRange &ay,
                                                const AxisRange &az, const float gscale, EnumLds &es,
                                                float *__restrict__ col_p, uint32_t *__restrict__ col_xy,
                                                Consume &&consume) {
  const int lane = threadIdx.x & 63;
  for (int nx0 = g.nx_a; nx0 < g.nx_b; nx0 += 64) {
    // lanes = x indices: y range of the columns that reach the outer sphere
    const int nxi = nx0 + lane;
    int ny_lo = 0, ny_cnt = 0;
    if (nxi < g.nx_b) {
      const AxisEntry ex = tx[nxi];
      float rh, rl;
      ff_sub(g.r1h, g.r1l, ex.sq_hi, ex.sq_lo, rh, rl);
      if (rh > 0.0f) {
        const float R = __builtin_sqrtf(rh) + 1.0f;
        ny_lo = first_ge(ay, -R);
        ny_cnt = first_ge(ay, R) - ny_lo;
      }
    }
    const int incl_y = wave_incl_scan(ny_cnt);
    const int ncols = __builtin_amdgcn_readlane(incl_y, 63);
    const int col0 = incl_y - ny_cnt;  // first column of this x lane
    es.nx_col[lane] = ((uint32_t)col0 << 11) | (uint32_t)ny_lo;

    int xcarry = 0;
    for (int cb = 0; cb * 64 < ncols; ++cb) {
      // lanes = columns (nx, ny): z ranges of the shell
      const int gcol = cb * 64 + lane;
      // x lane of the column: the last x lane with columns starting at or
      // before it (each marks its first column in the batch; a running
      // maximum carries the marks forward, as for the candidates)
      es.mark[lane] = 0;
      wave_sync();
      if (ny_cnt > 0 && (uint32_t)(col0 - cb * 64) < 64u) es.mark[col0 - cb * 64] = lane + 1;
      wave_sync();
      const int xm = max(wave_incl_max(es.mark[lane]), xcarry);
      xcarry = __builtin_amdgcn_readlane(xm, 63);
      int z1 = 0, n1 = 0, z2 = 0, n2 = 0;
      float cg = 0.0f;
      if (gcol < ncols) {
        const int i = max(xm - 1, 0);
        const uint32_t xc = es.nx_col[i];
        const AxisEntry ex = tx[nx0 + i];
        const int iy = (int)(xc & 0x7ffu) + (gcol - (int)(xc >> 11));
        const AxisEntry ey = ty[iy];
        if constexpr (DUMP) col_xy[lane] = ((uint32_t)(nx0 + i) << 16) | (uint32_t)iy;
        float sh, sl;
        two_sum(ex.sq_hi, ey.sq_hi, sh, sl);
        sl += ex.sq_lo + ey.sq_lo;
        fast_two_sum(sh, sl, sh, sl);
        es.col_s[lane] = float2v{sh, sl};
        if constexpr (POLAR) col_p[lane] = ex.proj + ey.proj;  // column part of |d| cos(theta)
        cg = (ex.gain * ey.gain) * gscale;
        float rh, rl;
        ff_sub(g.r1h, g.r1l, sh, sl, rh, rl);
        if (rh > 0.0f) {
          const float zmax = __builtin_sqrtf(rh) + 1.0f;
          float zmin = 0.0f;
          if (g.R0 > 0.0f) {
            float hh, hl;
            ff_sub(g.r0h, g.r0l, sh, sl, hh, hl);
            if (hh > 0.0f) zmin = fmaxf(__builtin_sqrtf(hh) - 1.0f, 0.0f);
          }
          // displacements in [-zmax, -zmin) and [zmin, zmax): two runs of the
          // table (contiguous when zmin = 0)
          z1 = first_ge(az, -zmax);
          n1 = first_ge(az, -zmin) - z1;
          z2 = first_ge(az, zmin);
          n2 = first_ge(az, zmax) - z2;
        }
      }
      const int cnt = n1 + n2;
      const int incl = wave_incl_scan(cnt);
      const int total = __builtin_amdgcn_readlane(incl, 63);
      const int excl = incl - cnt;
      es.col_run[lane] = int4v{excl + n1, z1 - excl, z2 - n1 - excl, __float_as_int(cg)};
      if (total > 0) {
        wave_sync();
        consume(total, excl, cnt);
        wave_sync();
      }
    }
    wave_sync();
  }
}

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));

// Parameters of one image candidate (column part cs of the squared distance,
// column gain cgain, z table row ez). ok is false when the
// tile does not own the image. base = k0 - T0 is the tile-local LDS index of its
// tap j = 1 - W/2 (the LDS tile starts at sample T0 + 1 - W/2). rec is the
// staged record of the taps, which also carries the base:
//   FP32: (f, CP, CQ', C/2) with f the fraction in [2^-24, 1 - 2^-24],
//         C = A sin(pi f)/pi, CP = C/2 cos(2 pi f/W), and CQ' the value
//         CQ = C/2 sin(2 pi f/W) with the base in its 8 low mantissa bits.
//         That changes CQ by less than 2^-15 of itself; CQ enters tap j as
//         CQ sin(2 pi j/W) / (j - f) and |CQ| <= C/2 sin(2 pi/W) (W >= 4), so
//         a tap moves by less than 2^-15 sin(2 pi/W) A/(2 pi): 4.8e-7 A at
//         W = 64, 9.5e-7 A at W = 32. General windows of the 32-sample cap
//         (any W < 32, where that bound grows towards 4.9e-6 A) keep the
//         fraction and the base in one word instead (cq_base false):
//         (F, CP, CQ, C/2) with F = fq 2^8 + base, fq the fraction rounded
//         to 24 bits, and f = float(F) 2^-32 for the taps and the factors;
//   FP16: (t, A') with t = f - 1/2 in FP32 and A' the amplitude with the
//         base in its 8 low mantissa bits (relative change < 2^-15);
//   LUT:  (F, A) with F = fq 2^8 + base (bits of a uint32), fq the fraction
//         in units of 2^-24, and A in FP32.
// The column gain cgain carries the constant factor of A: fs / (4 pi c)
// for FP16 and LUT, and fs / (4 pi c) / (2 pi) for FP32, whose record holds C/2.
template <bool HALF> struct StageRec { typedef f4v type; };
template <> struct StageRec<true> { typedef float2v type; };
template <bool HALF>
struct ImageParams {
  bool ok;
  int base;
  typename StageRec<HALF>::type rec;
};
template <bool HALF>
__device__ __forceinline__ float column_gain_scale(const RoomArgs &ra) {
  return HALF ? ra.kappa : ra.kappa * (float)(0.5 / kPi);
}
template <int WT, bool HALF, bool LUT, bool POLAR, bool GEN = false>
__device__ __forceinline__ ImageParams<HALF || LUT> image_params(const RoomArgs &ra, const ItemGeom &g,
                                                                 const float2v cs, const float cgain,
                                                                 const AxisEntry ez, const float cp) {
  ImageParams<HALF || LUT> p;
  // S = column part + z part in float-float (Sh + Sl, not renormalised)
  float Sh, Sl;
  two_sum(cs.x, ez.sq_hi, Sh, Sl);
  Sl += cs.y + ez.sq_lo;
  // x = sqrt(S) in samples (Eq. (2)-(3)): one Newton correction in float-float
  const float x0 = __builtin_amdgcn_sqrtf(Sh);
  const float rx = __builtin_amdgcn_rcpf(x0);
  const float xl = (__builtin_fmaf(-x0, x0, Sh) + Sl) * (0.5f * rx);
  // k0 = floor(x), f = x - k0: |xl| is a few ulps of x0 at most, so the
  // fraction (x0 - floor(x0)) + xl lies in (-1, 2) and one floor moves it into
  // [0, 1); the clamp catches a tiny negative fraction that rounds up to 1.
  float kf = floorf(x0);
  float fr = (x0 - kf) + xl;
  const float d = floorf(fr);
  fr = fminf(fr - d, 0x1.fffffep-1f);
  kf += d;
  const int k0 = (int)kf;
  p.base = k0 - g.T0;
  p.ok = (x0 < 1.0e9f) && (uint32_t)p.base < (uint32_t)(g.K1 - g.T0);
  // Eq. (4) amplitude (times the constant factor carried by the column gain)
  float A = (cgain * ez.gain) * rx;
  // receiver polar pattern a + b cos(theta), cos(theta) = (d . o) / |d|
  if constexpr (POLAR) A *= __builtin_fmaf(ra.dir_b, (cp + ez.proj) * rx, ra.dir_a);
  if constexpr (HALF) {
    const float t = fr - 0.5f;
    const uint32_t Ab = (__float_as_uint(A) & ~kBaseMask) | ((uint32_t)p.base & kBaseMask);
    p.rec = float2v{t, __uint_as_float(Ab)};
  } else if constexpr (LUT) {
    // 24-bit fraction (as in the FP32 record) with the base in the low byte;
    // its top 4 bits are the table phase, the next 20 the interpolation weight
    const uint32_t fq = min((uint32_t)__builtin_rintf(fr * (float)(1u << kFracBits)), (1u << kFracBits) - 1u);
    p.rec = float2v{__uint_as_float((fq << kBaseBits) | ((uint32_t)p.base & kBaseMask)), A};
  } else {
    // f at least 2^-24 (fr is at most 1 - 2^-24 already): no tap sits on the
    // image itself, where the sinc's numerator and denominator both vanish.
    // Packed beside the base, f is rounded to 24 bits (the delay moves by at
    // most 3e-8 samples) and float(F) 2^-32 stays in [2^-24, 1 - 2^-24].
    constexpr bool CQB = cq_base(WT, GEN);
    uint32_t F = 0;
    float f;
    if constexpr (CQB) {
      f = fmaxf(fr, 0x1p-24f);
    } else {
      const uint32_t fq = min(max((uint32_t)__builtin_rintf(fr * (float)(1u << kFracBits)), 1u), (1u << kFracBits) - 2u);
      F = (fq << kBaseBits) | ((uint32_t)p.base & kBaseMask);
      f = (float)F * 0x1p-32f;
    }
    // The hardware sine and cosine take the angle in turns; their relative
    // error (< 1e-6, also for the tiny angles of f near 0 or 1) enters each
    // tap of the image once. sin(pi f) is taken as sin(pi min(f, 1 - f)).
    const float C2 = A * __builtin_amdgcn_sinf(0.5f * fminf(f, 1.0f - f));
    const float turn = f * (GEN ? ra.inv_win : 1.0f / (float)WT);  // phi = 2 pi f / W in turns
    const float CQ = C2 * __builtin_amdgcn_sinf(turn);
    const float CP = C2 * __builtin_amdgcn_cosf(turn);
    if constexpr (CQB) {
      const uint32_t Qb = (__float_as_uint(CQ) & ~kBaseMask) | ((uint32_t)p.base & kBaseMask);
      p.rec = f4v{f, CP, __uint_as_float(Qb), C2};
    } else {
      p.rec = f4v{__uint_as_float(F), CP, CQ, C2};
    }
  }
  return p;
}

// Per-tap constants, indexed by jj = j - (1 - W/2).
__constant__ TapConsts<32> kTap32 = make_tap_consts<32>();
__constant__ TapConsts<64> kTap64 = make_tap_consts<64>();
__constant__ TapConsts<96> kTap96 = make_tap_consts<96>();
__constant__ TapConsts<128> kTap128 = make_tap_consts<128>();
template <int WT> __device__ __forceinline__ const TapConsts<WT> &tap_table();
template <> __device__ __forceinline__ const TapConsts<32> &tap_table<32>() { return kTap32; }
template <> __device__ __forceinline__ const TapConsts<64> &tap_table<64>() { return kTap64; }
template <> __device__ __forceinline__ const TapConsts<96> &tap_table<96>() { return kTap96; }
template <> __device__ __forceinline__ const TapConsts<128> &tap_table<128>() { return kTap128; }
__constant__ SincPoly<32> kPoly32 = make_sinc_poly<32>();
__constant__ SincPoly<64> kPoly64 = make_sinc_poly<64>();
__constant__ SincPoly<96> kPoly96 = make_sinc_poly<96>();
__constant__ SincPoly<128> kPoly128 = make_sinc_poly<128>();
template <int WT> __device__ __forceinline__ const SincPoly<WT> &poly_table();
template <> __device__ __forceinline__ const SincPoly<32> &poly_table<32>() { return kPoly32; }
template <> __device__ __forceinline__ const SincPoly<64> &poly_table<64>() { return kPoly64; }
template <> __device__ __forceinline__ const SincPoly<96> &poly_table<96>() { return kPoly96; }
template <> __device__ __forceinline__ const SincPoly<128> &poly_table<128>() { return kPoly128; }
// Compile-time checks of the tables: entries within [-0.25, 1], 1 at v = 0,
// and 0 (to FP32 rounding) at the other integers, where the sinc vanishes.
template <int WT>
constexpr bool lut_sane(const LutPairs<WT> &t) {
  for (int ph = 0; ph < kLutQ; ++ph)
    for (int m = 0; m < WT; ++m) {
      const double e = t.p[ph][m][0];
      if (!(e >= -0.25 && e <= 1.0)) return false;
      const int n = kLutQ * m + ph - kLutQ * WT / 2;
      if (n == 0 && e != 1.0) return false;
      if (n != 0 && n % kLutQ == 0 && (e > 1e-7 || e < -1e-7)) return false;
    }
  return true;
}
static_assert(lut_sane(make_lut_pairs<32>()) && lut_sane(make_lut_pairs<64>()), "table of Eq. (9)");
static_assert(lut_sane(make_lut_pairs<96>()) && lut_sane(make_lut_pairs<128>()), "table of Eq. (9)");
__constant__ LutPairs<32> kLut32 = make_lut_pairs<32>();
__constant__ LutPairs<64> kLut64 = make_lut_pairs<64>();
__constant__ LutPairs<96> kLut96 = make_lut_pairs<96>();
__constant__ LutPairs<128> kLut128 = make_lut_pairs<128>();
template <int WT> __device__ __forceinline__ const LutPairs<WT> &lut_table();
template <> __device__ __forceinline__ const LutPairs<32> &lut_table<32>() { return kLut32; }
template <> __device__ __forceinline__ const LutPairs<64> &lut_table<64>() { return kLut64; }
template <> __device__ __forceinline__ const LutPairs<96> &lut_table<96>() { return kLut96; }
template <> __device__ __forceinline__ const LutPairs<128> &lut_table<128>() { return kLut128; }


// Output of a work item whose taps are in LDS tiles t0 (+ t1): the tile's own
// samples go to dst, the W/2 - 1 samples before and the W/2 after to marg
// (layout: left margin, then right margin; W - 1 values).
template <int WT, int NT>
__device__ __forceinline__ void write_item(float (*tile)[TILE + WT - 1], int n_own, float *__restrict__ dst,
                                           float *__restrict__ marg, int tid, int nthreads) {
  constexpr int LM = WT / 2 - 1;
  for (int k = tid; k < n_own; k += nthreads) {
    float v = tile[0][LM + k];
#pragma unroll
    for (int w = 1; w < NT; ++w) v += tile[w][LM + k];
    dst[k] = v;
  }
  for (int i = tid; i < WT - 1; i += nthreads) {
    const int ti = i < LM ? i : TILE + i;
    float v = tile[0][ti];
#pragma unroll
    for (int w = 1; w < NT; ++w) v += tile[w][ti];
    marg[i] = v;
  }
}
template <int WT>
__device__ __forceinline__ void write_invalid(int n_own, float *__restrict__ dst, float *__restrict__ marg, int tid,
                                              int nthreads) {
  for (int k = tid; k < n_own; k += nthreads) dst[k] = __builtin_nanf("");
  for (int i = tid; i < WT - 1; i += nthreads) marg[i] = __builtin_nanf("");
}

// One work item on one wave (lanes = taps). Each step takes NQ staged images,
// one per group of LPG = 64 / NQ lanes; lane l of group g adds the taps
// j = 1 - W/2 + l + LPG m (m < TPL = W / LPG) of its image into the group's
// own LDS tile. dst receives the own samples of the tile (or a partial tile
// when C > 1), marg the margins. HALF selects the FP16 tap arithmetic, LUT
// the table taps; accumulation is FP32 in all modes.
// DUMP: the enumeration check. No taps; every owned image is written to
// dump->rec as a DumpRec of RIR rir (amplitude and fraction as the table
// taps compute them).
// GEN: general-mode window (WT is the cap, W = 2 ra.win_hw): the per-lane tap
// constants come from wc ([WT][WC_STRIDE], written for this window by
// window_consts_kernel) and FP32 taps with |j - f| >= W/2 are masked.
template <int WT, bool HALF, int NQ, bool LUT = false, bool POLAR = false, bool DUMP = false, bool GEN = false>
__device__ __forceinline__ void accumulate_item(const RoomArgs &ra, const int tile_id, const int C, const int c,
                                                const AxisEntry *__restrict__ tab, const AxisOrigin &org,
                                                const bool valid, float *__restrict__ dst, float *__restrict__ marg,
                                                const DumpArgs *dump = nullptr, const int rir = 0,
                                                const float *__restrict__ wc = nullptr) {
  static_assert(!(GEN && (LUT || DUMP)), "general-mode windows take FP32 or FP16 taps");
  constexpr int LSPAN = TILE + WT - 1;
  constexpr int LPG = 64 / NQ;          // lanes per image
  constexpr int TPL = WT / LPG;         // taps per lane per step
  constexpr int NPAIR = (TPL + 1) / 2;  // packed FP16 tap pairs per lane
  // staged images: up to 64 new + NQ - 1 carried, + the read-ahead of a step
  constexpr int SCAP = 64 + 3 * NQ;
  static_assert(WT % LPG == 0, "window must be a multiple of the lanes per image");

  __shared__ float tile[NQ][LSPAN];
  static_assert(!(HALF && LUT), "one tap mode");
  constexpr bool NARROW = HALF || LUT;  // 8-byte stage record
  typedef typename StageRec<NARROW>::type Rec;
  __shared__ Rec stp[SCAP];  // staged records (ImageParams::rec)
  __shared__ EnumLds es;
  __shared__ float col_p[POLAR ? 64 : 1];  // polar calls: column part of |d| cos(theta)
  __shared__ uint32_t col_xy[DUMP ? 64 : 1];  // enumeration check: column table indices

  const int lane = threadIdx.x & 63;
  const int h = lane / LPG, l = lane % LPG;  // image group, lane within it
  const int n_own = min(TILE, ra.n_samples - tile_id * TILE);  // may be <= 0 past nS
  if (!valid) {
    if constexpr (!DUMP) write_invalid<WT>(n_own, dst, marg, lane, 64);
    return;
  }
  const AxisEntry *__restrict__ tx = tab + ra.off[0];
  const AxisEntry *__restrict__ ty = tab + ra.off[1];
  const AxisEntry *__restrict__ tz = tab + ra.off[2];
  const AxisRange ax = axis_range(ra.lo[0], ra.N[0], ra.inv_period[0], org.e_even[0], org.e_odd[0]);
  const AxisRange ay = axis_range(ra.lo[1], ra.N[1], ra.inv_period[1], org.e_even[1], org.e_odd[1]);
  const AxisRange az = axis_range(ra.lo[2], ra.N[2], ra.inv_period[2], org.e_even[2], org.e_odd[2]);
  const ItemGeom g = item_geom(ra, ax, tile_id, C, c);

  // per-lane tap constants
  float nsg[TPL], sgj[TPL], cth[TPL], sth[TPL];  // FP32 taps
  float pc0[TPL];                                // FP16 taps: c0 of each tap
  half2_t pq[NPAIR][SPD];                        // and c1..c5 of tap pairs (2p, 2p + 1)
  if constexpr (GEN && HALF) {
#pragma unroll
    for (int m = 0; m < TPL; ++m) pc0[m] = wc[WC_STRIDE * (l + LPG * m)];
#pragma unroll
    for (int pr = 0; pr < NPAIR; ++pr)
#pragma unroll
      for (int k = 0; k < SPD; ++k) {
        const int m0 = 2 * pr, m1 = 2 * pr + 1;
        const float a = wc[WC_STRIDE * (l + LPG * m0) + k + 1];
        const float b = m1 < TPL ? wc[WC_STRIDE * (l + LPG * m1) + k + 1] : 0.0f;
        pq[pr][k] = half2_t{(_Float16)a, (_Float16)b};
      }
  } else if constexpr (GEN) {
#pragma unroll
    for (int m = 0; m < TPL; ++m) {
      const float4 e = *reinterpret_cast<const float4 *>(wc + WC_STRIDE * (l + LPG * m));
      nsg[m] = e.x;
      sgj[m] = e.y;
      cth[m] = e.z;
      sth[m] = e.w;
    }
  } else if constexpr (HALF && !DUMP) {
    const SincPoly<WT> &P = poly_table<WT>();
#pragma unroll
    for (int m = 0; m < TPL; ++m) pc0[m] = P.c[0][l + LPG * m];
#pragma unroll
    for (int pr = 0; pr < NPAIR; ++pr)
#pragma unroll
      for (int k = 0; k < SPD; ++k) {
        const int m0 = 2 * pr, m1 = 2 * pr + 1;
        const float a = P.c[k + 1][l + LPG * m0];
        const float b = m1 < TPL ? P.c[k + 1][l + LPG * m1] : 0.0f;
        pq[pr][k] = half2_t{(_Float16)a, (_Float16)b};
      }
  } else if constexpr (!LUT && !DUMP) {
    const TapConsts<WT> &K = tap_table<WT>();
#pragma unroll
    for (int m = 0; m < TPL; ++m) {
      nsg[m] = -K.sig[l + LPG * m];
      sgj[m] = K.sig_j[l + LPG * m];
      cth[m] = K.cth[l + LPG * m];
      sth[m] = K.sth[l + LPG * m];
    }
  }
  for (int i = lane; i < NQ * LSPAN; i += 64) (&tile[0][0])[i] = 0.0f;
  float *const th = &tile[h][l];
  // LUT taps: the table is copied into LDS once per work item (8 KB at
  // W = 64; it costs occupancy, but LDS reads of a row's consecutive pairs
  // beat the vector-memory path, 0.68 against 0.89 ms on the 32-receiver
  // call); lrow is this lane's first entry of row 0 (rows are WT pairs apart)
  __shared__ __attribute__((aligned(16))) float lds_lut[LUT ? kLutQ * WT * 2 : 4];
  const float hw = ra.win_hw;  // general mode: taps with |j - f| >= W/2 are masked
  if constexpr (LUT) {
    const float *gl = &lut_table<WT>().p[0][0][0];
    for (int i = lane; i < kLutQ * WT * 2; i += 64) lds_lut[i] = gl[i];
    wave_sync();
  }
  const float *const lrow = &lds_lut[LUT ? 2 * l : 0];

  // One step: staged image (record P) on this lane group, taps l + LPG m.
  // The empty asm consumes the record as one value where the step starts,
  // which keeps its LDS read a single wide read (16 bytes for FP32, 8 for
  // FP16) issued ahead.
  auto step = [&](const Rec P) {
    __asm__ volatile("" ::"v"(P));
    uint32_t bw;  // record word that carries the base
    if constexpr (NARROW || !cq_base(WT, GEN)) bw = __float_as_uint(HALF ? P.y : P.x);
    else bw = __float_as_uint(P.z);
    const int b = (int)(bw & kBaseMask);
    float *t = th + b;
    if constexpr (HALF) {
      // tap = A (c0 + t q(t)), q in packed FP16 two taps at a time, the
      // rest in FP32 (t q(t) + c0 as one mixed-precision FMA)
      const float tf = P.x, A = P.y;
      const half2_t tt = {(_Float16)tf, (_Float16)tf};
#pragma unroll
      for (int pr = 0; pr < NPAIR; ++pr) {
        half2_t q = pq[pr][SPD - 1];
#pragma unroll
        for (int k = SPD - 2; k >= 0; --k) q = __builtin_elementwise_fma(q, tt, pq[pr][k]);
        const int m0 = 2 * pr, m1 = 2 * pr + 1;
        t[LPG * m0] = __builtin_fmaf(A, __builtin_fmaf(tf, (float)q.x, pc0[m0]), t[LPG * m0]);
        if (m1 < TPL) t[LPG * m1] = __builtin_fmaf(A, __builtin_fmaf(tf, (float)q.y, pc0[m1]), t[LPG * m1]);
      }
    } else if constexpr (LUT) {
      // tap = A (L[i] + (1 - fr) (L[i + 1] - L[i])) from row ph of the table
      const uint32_t F = __float_as_uint(P.x);
      const float A = P.y;
      const int ph = (kLutQ - 1) - (int)(F >> 28);
      const float al = 1.0f - (float)((F >> kBaseBits) & ((1u << (28 - kBaseBits)) - 1u)) *
                                  (1.0f / (float)(1u << (28 - kBaseBits)));
      const float *const row = lrow + 2 * WT * ph;
#pragma unroll
      for (int m = 0; m < TPL; ++m) {
        const float2v e = *reinterpret_cast<const float2v *>(row + 2 * LPG * m);
        t[LPG * m] = __builtin_fmaf(A, __builtin_fmaf(al, e.y, e.x), t[LPG * m]);
      }
    } else if constexpr (GEN) {
      // general window: no half-period symmetry between the lane's taps; a
      // tap outside |j - f| < W/2 gets a zero reciprocal
      const float fs = cq_base(WT, GEN) ? P.x : (float)__float_as_uint(P.x);  // f, or f 2^32
#pragma unroll
      for (int m = 0; m < TPL; ++m) {
        float w = __builtin_fmaf(cth[m], P.y, P.w);
        w = __builtin_fmaf(sth[m], P.z, w);
        const float u = __builtin_fmaf(nsg[m], fs, sgj[m]);  // sigma (j - f)
        const float r = __builtin_fabsf(u) < hw ? __builtin_amdgcn_rcpf(u) : 0.0f;
        t[LPG * m] = __builtin_fmaf(w, r, t[LPG * m]);
      }
    } else {
      // When TPL is even, tap m + TPL/2 sits half a window period after tap
      // m, where the Hann term flips sign: its numerator is 2 (C/2) - w_m.
      float w[TPL];
#pragma unroll
      for (int m = 0; m < TPL; ++m) {
        if (TPL % 2 == 0 && m >= TPL / 2) {
          w[m] = __builtin_fmaf(2.0f, P.w, -w[m - TPL / 2]);
        } else {
          w[m] = __builtin_fmaf(cth[m], P.y, P.w);
          w[m] = __builtin_fmaf(sth[m], P.z, w[m]);
        }
      }
      const float fs = P.x;  // f
#pragma unroll
      for (int m = 0; m < TPL; ++m) {
        const float u = __builtin_fmaf(nsg[m], fs, sgj[m]);
        const float r = __builtin_amdgcn_rcpf(u);
        t[LPG * m] = __builtin_fmaf(w[m], r, t[LPG * m]);
      }
    }
  };
  // staged record k (read as one 16-byte access: see step)
  auto rec = [&](int k) { return stp[k]; };

  int ns = 0;  // staged images (wave-uniform)
  enumerate_shell<POLAR, DUMP>(g, tx, ty, ay, az, column_gain_scale<NARROW || DUMP>(ra), es, col_p, col_xy,
                               [&](int total, int excl, int cnt) {
    // Chunks of 64 candidate positions; lane i takes position q0 + i. Its
    // column is the last one starting at or before it: each column marks its
    // first position in the chunk, a running maximum over the lanes carries
    // the marks forward, and the last lane's column carries into the next
    // chunk (columns start in increasing order).
    int carry = 0;
    auto locate = [&](int q0, int &cl, int &nz, float &cg) {
      es.mark[lane] = 0;
      wave_sync();
      const int r = excl - q0;
      if (cnt > 0 && (uint32_t)r < 64u) es.mark[r] = lane + 1;
      wave_sync();
      const int m = max(wave_incl_max(es.mark[lane]), carry);
      carry = __builtin_amdgcn_readlane(m, 63);
      cl = max(m - 1, 0);
      const int4v cr = es.col_run[cl];
      const int pos = q0 + lane;
      nz = min(max(pos + (pos < cr.x ? cr.y : cr.z), 0), ra.N[2] - 1);
      cg = __int_as_float(cr.w);
    };
    // the next chunk's column and z table row are found ahead of its use
    int cl, nz;
    float cg;
    locate(0, cl, nz, cg);
    AxisEntry ez{0.0f, 0.0f, 0.0f, 0.0f};
    if (lane < total) ez = tz[nz];
    for (int q = 0; q < total; q += 64) {
      const int cl_c = cl;
      const float cg_c = cg;
      const AxisEntry ez_c = ez;
      const int nz_c = nz;
      if (q + 64 < total) {
        locate(q + 64, cl, nz, cg);
        if (q + 64 + lane < total) ez = tz[nz];
      }
      if constexpr (DUMP) {
        // delay and amplitude exactly as the table taps compute them
        ImageParams<true> p;
        p.ok = false;
        if (q + lane < total) p = image_params<WT, false, true, POLAR>(ra, g, es.col_s[cl_c], cg_c, ez_c, 0.0f);
        const uint64_t okm = __ballot(p.ok);
        const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(okm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)okm, 0u));
        uint32_t first = 0;
        if (lane == 0 && okm != 0) first = atomicAdd(dump->count, (uint32_t)__builtin_popcountll(okm));
        first = (uint32_t)__builtin_amdgcn_readlane((int)first, 0);
        if (p.ok && first + (uint32_t)rank < dump->cap) {
          const uint32_t xy = col_xy[cl_c];
          // lattice index per table axis, then per room axis (table axis k is room axis perm[k])
          const int t0 = ra.lo[0] + (int)(xy >> 16), t1 = ra.lo[1] + (int)(xy & 0xffffu), t2 = ra.lo[2] + nz_c;
          DumpRec d;
          d.rir = rir;
          d.n[0] = ra.perm[0] == 0 ? t0 : (ra.perm[1] == 0 ? t1 : t2);
          d.n[1] = ra.perm[0] == 1 ? t0 : (ra.perm[1] == 1 ? t1 : t2);
          d.n[2] = ra.perm[0] == 2 ? t0 : (ra.perm[1] == 2 ? t1 : t2);
          d.k0 = g.T0 + p.base;
          d.fq = (__float_as_uint(p.rec.x) >> kBaseBits) << (kBaseBits - 8);  // units of 2^-24
          d.A = p.rec.y;
          d.pad = 0;
          dump->rec[first + (uint32_t)rank] = d;
        }
        wave_sync();
        continue;
      }
      // lanes = candidates: parameters, then compaction into the stage
      ImageParams<NARROW> p;
      p.ok = false;
      if (q + lane < total)
        p = image_params<WT, HALF, LUT, POLAR, GEN>(ra, g, es.col_s[cl_c], cg_c, ez_c, POLAR ? col_p[cl_c] : 0.0f);
      const uint64_t okm = __ballot(p.ok);
      const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(okm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)okm, 0u));
      if (p.ok) stp[ns + rank] = p.rec;
      ns += __builtin_popcountll(okm);
      wave_sync();
      // lanes = taps: NQ staged images per step, one per lane group; the next
      // step's record is read ahead of this step's tile update (reads ahead
      // stay inside the stage: indices < NQ (np + 1) + h <= SCAP)
      const int np = ns / NQ;
      Rec PA = rec(h);
      for (int s = 0; s < np; s += 2) {
        const Rec PB = rec(NQ * (s + 1) + h);
        __builtin_amdgcn_sched_barrier(0);  // keep the read-ahead in front of the step
        step(PA);
        if (s + 1 < np) {
          PA = rec(NQ * (s + 2) + h);
          __builtin_amdgcn_sched_barrier(0);
          step(PB);
        }
      }
      // carry the remaining images to the front of the stage (the ranges do
      // not overlap when np > 0)
      const int rem = ns - NQ * np;
      if (np > 0 && rem > 0) {
        Rec P{};
        if (lane < rem) P = stp[NQ * np + lane];
        wave_sync();
        if (lane < rem) stp[lane] = P;
      }
      ns = rem;
      wave_sync();
    }
  });
  if constexpr (DUMP) return;
  if (h < ns) step(stp[h]);  // last images, fewer than NQ

  wave_sync();
  write_item<WT, NQ>(tile, n_own, dst, marg, lane, 64);
}

// First work item of dispatch position pos (see PlanArgs).
__device__ __forceinline__ uint32_t plan_first_item(const PlanArgs &pa, int pos) {
  uint32_t f = pa.first_blk[pos / PLAN_BLK];
  for (int p = pos - pos % PLAN_BLK; p < pos; ++p) f += (uint32_t)pa.n_rir * pa.chunks[pa.n_tiles - 1 - p];
  return f;
}

// Work item of a single-room launch: the item index decodes through the
// per-tile chunk counts.
struct SingleItem {
  int pos, tile_id, C, rir, c;
  uint32_t first;  // first item of the dispatch position
};
__device__ __forceinline__ SingleItem decode_item(const PlanArgs &pa, uint32_t item) {
  // largest dispatch position pos whose first item is <= item: the block by
  // binary search over first_blk, then the position within the block
  const int nblk = (pa.n_tiles + PLAN_BLK - 1) / PLAN_BLK;
  int lo = 0, hi = nblk;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pa.first_blk[mid] <= item) lo = mid;
    else hi = mid;
  }
  int pos = lo * PLAN_BLK;
  uint32_t first = pa.first_blk[lo];
  const int pend = min(pa.n_tiles, pos + PLAN_BLK);
  for (;;) {
    const uint32_t next = first + (uint32_t)pa.n_rir * pa.chunks[pa.n_tiles - 1 - pos];
    if (pos + 1 >= pend || next > item) break;
    first = next;
    ++pos;
  }
  SingleItem si;
  si.pos = pos;
  si.first = first;
  si.tile_id = pa.n_tiles - 1 - pos;
  si.C = pa.chunks[si.tile_id];
  const uint32_t rel = item - first;
  si.rir = (int)(rel / (uint32_t)si.C);
  si.c = (int)(rel % (uint32_t)si.C);
  return si;
}

template <int WT, bool HALF, int NQ, bool LUT, bool POLAR, bool GEN>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kAccWavesPerSimd))) void accumulate_kernel(RoomArgs ra, PlanArgs pa,
                                                             const AxisEntry *__restrict__ tab_all,
                                                             const AxisOrigin *__restrict__ origin,
                                                             const int *__restrict__ valid, float *__restrict__ out,
                                                             float *__restrict__ part, float *__restrict__ marg,
                                                             const float *__restrict__ wc) {
  const uint32_t item = blockIdx.x;
  const SingleItem si = decode_item(pa, item);
  // (for a tile past nS, dst is never written: the tile has no own samples)
  float *dst = (si.C == 1) ? out + (size_t)si.rir * ra.n_samples + (size_t)si.tile_id * TILE
                           : part + (size_t)item * TILE;
  const AxisOrigin org = origin[si.rir];
  accumulate_item<WT, HALF, NQ, LUT, POLAR, false, GEN>(ra, si.tile_id, si.C, si.c,
                                                        tab_all + (size_t)si.rir * ra.n_tab, org, valid[si.rir] != 0,
                                                        dst, marg + (size_t)item * WT, nullptr, 0, wc);
}

// Per-tap constants of a general-mode window (one thread per tap of the cap).
__global__ __launch_bounds__(256) void window_consts_kernel(float W, int WT, int half, float *__restrict__ wc) {
  const int jj = threadIdx.x;
  if (jj < WT) window_const_entry(W, WT, half, jj, wc + WC_STRIDE * jj);
}
// Batch mode: one block per job; jobs without general-mode constants exit.
__global__ __launch_bounds__(256) void window_consts_batch_kernel(const JobDev *__restrict__ jobs, int half) {
  const JobDev &jb = jobs[blockIdx.x];
  if (!jb.wc) return;
  const int WT = (int)(2.0f * jb.ra.half_w);
  const int jj = threadIdx.x;
  if (jj < WT) window_const_entry(2.0f * jb.ra.win_hw, WT, half, jj, jb.wc + WC_STRIDE * jj);
}

// Enumeration check: the items of a single-room launch, images only.
template <int WT>
__global__ __launch_bounds__(64) void enumerate_dump_kernel(RoomArgs ra, PlanArgs pa,
                                                            const AxisEntry *__restrict__ tab_all,
                                                            const AxisOrigin *__restrict__ origin,
                                                            const int *__restrict__ valid, DumpArgs dump) {
  const SingleItem si = decode_item(pa, blockIdx.x);
  const AxisOrigin org = origin[si.rir];
  accumulate_item<WT, false, 2, false, false, true>(ra, si.tile_id, si.C, si.c, tab_all + (size_t)si.rir * ra.n_tab,
                                                    org, valid[si.rir] != 0, nullptr, nullptr, &dump, si.rir);
}

__global__ void fill_u32_kernel(uint32_t *p, uint32_t v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Batch launch: persistent. The grid holds at most the resident waves; each
// workgroup (one wave) takes item blockIdx.x first, then the next unclaimed
// item of the largest-first list from the class's queue counter (which the
// run sets to the grid size before the launch), until the list is exhausted.
// Without a queue (queue == null) a workgroup takes every gridDim.x-th item.
// Every item names its job; the job table carries the room.
template <int WT, bool HALF, int NQ, bool LUT, bool POLAR, bool GEN>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kAccWavesPerSimd))) void accumulate_batch_kernel(
    const JobDev *__restrict__ jobs, const BatchItem *__restrict__ items, uint32_t n_items, uint32_t *queue,
    const AxisEntry *__restrict__ tab_all, const AxisOrigin *__restrict__ origin, const int *__restrict__ valid,
    float *__restrict__ part, float *__restrict__ marg) {
  const int lane = threadIdx.x & 63;
  uint32_t item = blockIdx.x;
  while (item < n_items) {
    const BatchItem it = items[item];
    const JobDev &jb = jobs[it.job];
    const RoomArgs ra = jb.ra;
    const uint32_t grir = jb.rir_base + it.rir;
    float *dst = (it.slot == 0xffffffffu) ? jb.out + (size_t)it.rir * ra.n_samples + (size_t)it.tile * TILE
                                          : part + (size_t)it.slot * TILE;
    const AxisOrigin org = origin[grir];
    accumulate_item<WT, HALF, NQ, LUT, POLAR, false, GEN>(ra, it.tile, it.chunks, it.chunk,
                                                         tab_all + jb.tab_base + (size_t)it.rir * ra.n_tab, org,
                                                         valid[grir] != 0, dst,
                                                         marg + (size_t)it.mslot * MARG_UNIT, nullptr, 0, jb.wc);
    if (queue) {
      uint32_t next = 0;
      if (lane == 0) next = atomicAdd(queue, 1u);
      item = (uint32_t)__builtin_amdgcn_readlane((int)next, 0);
    } else {
      item += gridDim.x;
    }
  }
}

// ---------------------------------------------------------------------------
// Kernel 3: ordered completion of the output tiles. Sample k of tile t is
//   (own sum) + (right margins of the items of tile t-1) + (left margins of
//   the items of tile t+1),
// where the own sum is the ordered sum of the tile's partials when it was
// split and the value already in the output otherwise. Every term is added in
// a fixed order, so results do not depend on scheduling.
// grid = (rir, dispatch position of the tile, segment of the tile)
// ---------------------------------------------------------------------------
// v + x[0] + x[stride] + ... + x[(n - 1) stride], added in that order; the
// loads of a group of 32 (then 8) are issued together, so a tile split into
// many items costs few memory round trips (the order of the additions, and
// so the result, does not depend on the grouping).
template <int B>
__device__ __forceinline__ float ordered_block(float v, const float *__restrict__ x, size_t stride) {
  float t[B];
#pragma unroll
  for (int u = 0; u < B; ++u) t[u] = x[(size_t)u * stride];
#pragma unroll
  for (int u = 0; u < B; ++u) v += t[u];
  return v;
}
__device__ __forceinline__ float ordered_sum(float v, const float *__restrict__ x, size_t stride, int n) {
  int cc = 0;
  for (; cc + 32 <= n; cc += 32) v = ordered_block<32>(v, x + (size_t)cc * stride, stride);
  for (; cc + 8 <= n; cc += 8) v = ordered_block<8>(v, x + (size_t)cc * stride, stride);
  if (cc < n) {  // the last (fewer than 8) terms, loaded together
    const int m = n - cc;
    float t[7];
#pragma unroll
    for (int u = 0; u < 7; ++u)
      if (u < m) t[u] = x[(size_t)(cc + u) * stride];
#pragma unroll
    for (int u = 0; u < 7; ++u)
      if (u < m) v += t[u];
  }
  return v;
}

// A run of n terms added to v in the fixed order of the reduce (the run
// length alone decides it): fewer than RED_SLICE_MIN terms one by one, longer
// runs as RED_SLICES consecutive slices, each summed in order from its first term,
// whose sums are then added to v in slice order. Launches with a long run
// take RED_SLICES threads per sample (a block covers RED_SAMPLES samples):
// each thread sums one slice and the sample's first thread adds the slice
// sums; the others take one thread per sample and add term by term (all
// their runs are short). n is uniform over the block (its barriers are);
// active: this thread's sample takes the run.
constexpr int RED_SAMPLES = 256 / RED_SLICES;
static_assert(TILE % RED_SAMPLES == 0, "reduce blocks tile the tile");
__device__ __forceinline__ float run_sum(float v, const float *__restrict__ x, size_t stride, int n, bool active,
                                         int slice, int ks, float (*red)[RED_SAMPLES]) {
  if (n < RED_SLICE_MIN) {
    if (active && slice == 0) v = ordered_sum(v, x, stride, n);
    return v;
  }
  const int m = (n + RED_SLICES - 1) / RED_SLICES;
  const int a = slice * m, len = min(m, n - a);
  red[slice][ks] = active ? ordered_sum(0.0f, x + (size_t)a * stride, stride, len) : 0.0f;
  __syncthreads();
  if (active && slice == 0) {
#pragma unroll
    for (int i = 0; i < RED_SLICES; ++i) v += red[i][ks];
  }
  __syncthreads();
  return v;
}

template <bool SLICED>
__global__ __launch_bounds__(256) void reduce_kernel(RoomArgs ra, PlanArgs pa, const float *__restrict__ part,
                                                     const float *__restrict__ marg, float *__restrict__ out) {
  constexpr int SPB = SLICED ? RED_SAMPLES : 256;  // samples per block
  __shared__ float red[SLICED ? RED_SLICES : 1][SLICED ? RED_SAMPLES : 1];
  const int pos = blockIdx.y;
  const int tile_id = pa.n_tiles - 1 - pos;
  const int C = pa.chunks[tile_id];
  const int rir = blockIdx.x;
  const int T0 = tile_id * TILE;
  const int ks = (int)threadIdx.x % SPB, slice = (int)threadIdx.x / SPB;
  const int k0 = blockIdx.z * SPB, k = k0 + ks;
  const int W = (int)(2.0f * ra.half_w);
  const int LM = W / 2 - 1;
  // block-uniform: which runs exist for some sample of this block
  const bool has_l = tile_id > 0 && k0 < W / 2;                    // right margin of tile t-1
  const bool has_r = tile_id + 1 < pa.n_tiles && k0 + SPB > TILE - LM;  // left margin of tile t+1
  if (C <= 1 && !has_l && !has_r) return;
  const bool in = k < ra.n_samples - T0 && k < TILE;
  const bool zl = in && has_l && k < W / 2;
  const bool zr = in && has_r && k >= TILE - LM;
  auto add = [&](float v, const float *x, size_t stride, int n, bool active) {
    if constexpr (SLICED) return run_sum(v, x, stride, n, active, slice, ks, red);
    else return active ? ordered_sum(v, x, stride, n) : v;  // n < RED_SLICE_MIN
  };
  float *o = out + (size_t)rir * ra.n_samples + T0 + k;
  float v = 0.0f;
  if (C > 1) {
    const size_t first = (size_t)plan_first_item(pa, pos) + (size_t)rir * C;
    v = add(0.0f, part + first * TILE + k, TILE, C, in);
  } else if (in && slice == 0 && (zl || zr)) {
    v = *o;
  }
  if (has_l) {  // tile t-1 is dispatched at pos + 1
    const int Cp = pa.chunks[tile_id - 1];
    const size_t first = (size_t)plan_first_item(pa, pos + 1) + (size_t)rir * Cp;
    v = add(v, marg + first * W + LM + k, W, Cp, zl);
  }
  if (has_r) {  // tile t+1 is dispatched at pos - 1
    const int Cn = pa.chunks[tile_id + 1];
    const size_t first = (size_t)plan_first_item(pa, pos - 1) + (size_t)rir * Cn;
    v = add(v, marg + first * W + (k - (TILE - LM)), W, Cn, zr);
  }
  if (in && slice == 0 && (C > 1 || zl || zr)) *o = v;
}

// Batch mode: grid = (output tile of a batch RIR, segment of the tile).
template <bool SLICED>
__global__ __launch_bounds__(256) void reduce_batch_kernel(const JobDev *__restrict__ jobs,
                                                           const BatchReduce *__restrict__ red_tab,
                                                           const float *__restrict__ part,
                                                           const float *__restrict__ marg) {
  constexpr int SPB = SLICED ? RED_SAMPLES : 256;
  __shared__ float red[SLICED ? RED_SLICES : 1][SLICED ? RED_SAMPLES : 1];
  const BatchReduce br = red_tab[blockIdx.x];
  const JobDev &jb = jobs[br.job];
  const int n_samples = jb.ra.n_samples;
  const int T0 = (int)br.tile * TILE;
  const int ks = (int)threadIdx.x % SPB, slice = (int)threadIdx.x / SPB;
  const int k0 = blockIdx.y * SPB, k = k0 + ks;
  const int W = (int)(2.0f * jb.ra.half_w);
  const int LM = W / 2 - 1;
  const bool has_l = br.nprev > 0 && k0 < W / 2;
  const bool has_r = br.nnext > 0 && k0 + SPB > TILE - LM;
  if (br.chunks <= 1 && !has_l && !has_r) return;
  const bool in = k < n_samples - T0 && k < TILE;
  const bool zl = in && has_l && k < W / 2;
  const bool zr = in && has_r && k >= TILE - LM;
  auto add = [&](float v, const float *x, size_t stride, int n, bool active) {
    if constexpr (SLICED) return run_sum(v, x, stride, n, active, slice, ks, red);
    else return active ? ordered_sum(v, x, stride, n) : v;  // n < RED_SLICE_MIN
  };
  float *o = jb.out + (size_t)br.rir * n_samples + T0 + k;
  float v = 0.0f;
  if (br.chunks > 1) {
    v = add(0.0f, part + (size_t)br.first * TILE + k, TILE, br.chunks, in);
  } else if (in && slice == 0 && (zl || zr)) {
    v = *o;
  }
  if (has_l) v = add(v, marg + (size_t)br.mprev * MARG_UNIT + LM + k, W, br.nprev, zl);
  if (has_r) v = add(v, marg + (size_t)br.mnext * MARG_UNIT + (k - (TILE - LM)), W, br.nnext, zr);
  if (in && slice == 0 && (br.chunks > 1 || zl || zr)) *o = v;
}

// The fixed order of run_sum on one thread: the slices of a long run summed
// one after the other (each from its first term), then added in order.
__device__ __forceinline__ float run_sum_serial(float v, const float *__restrict__ x, size_t stride, int n) {
  if (n < RED_SLICE_MIN) return ordered_sum(v, x, stride, n);
  const int m = (n + RED_SLICES - 1) / RED_SLICES;
  for (int i = 0; i < RED_SLICES; ++i) v += ordered_sum(0.0f, x + (size_t)(i * m) * stride, stride, min(m, n - i * m));
  return v;
}

// Batch mode, tiles that were not split: their own samples are final, and
// only the W - 1 margin samples (the first W/2 and the last W/2 - 1) take the
// neighbours' margins, in the order of reduce_batch_kernel. One 64-lane block
// per reduce entry.
__global__ __launch_bounds__(64) void reduce_margins_kernel(const JobDev *__restrict__ jobs,
                                                            const BatchReduce *__restrict__ red_tab,
                                                            const float *__restrict__ marg) {
  const BatchReduce br = red_tab[blockIdx.x];
  const JobDev &jb = jobs[br.job];
  const int n_samples = jb.ra.n_samples;
  const int T0 = (int)br.tile * TILE;
  const int W = (int)(2.0f * jb.ra.half_w);
  const int LM = W / 2 - 1;
  for (int i = (int)threadIdx.x; i < W - 1; i += 64) {
    const int k = i < W / 2 ? i : TILE - LM + (i - W / 2);
    if (k >= n_samples - T0) continue;
    const bool zl = br.nprev > 0 && k < W / 2;
    const bool zr = br.nnext > 0 && k >= TILE - LM;
    if (!zl && !zr) continue;
    float *o = jb.out + (size_t)br.rir * n_samples + T0 + k;
    float v = *o;
    if (zl) v = run_sum_serial(v, marg + (size_t)br.mprev * MARG_UNIT + LM + k, W, br.nprev);
    if (zr) v = run_sum_serial(v, marg + (size_t)br.mnext * MARG_UNIT + (k - (TILE - LM)), W, br.nnext);
    *o = v;
  }
}

// ---------------------------------------------------------------------------
// Launchers (called from ism_host.cpp).
// ---------------------------------------------------------------------------
// Staged images per step (lane groups of 64 / NQ lanes). Two (half-waves) is
// the measured best: four images per step halve the broadcast reads per tap
// but need four LDS tiles and more registers per wave, and ran 12 % slower.
constexpr int images_per_step(int wt, bool half) { return (void)wt, (void)half, 2; }
int launch_tables(const RoomArgs &ra, const float *src, const float *rcv, const float *orient, AxisEntry *tab,
                  AxisOrigin *origin, int *valid, int n_rir, hipStream_t st) {
  const int64_t total = (int64_t)n_rir * ra.n_tab;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65535) blocks = 65535;
  hipLaunchKernelGGL(tables_kernel, dim3((unsigned)blocks), dim3(256), 0, st, ra, src, rcv, orient, tab, origin,
                     valid, n_rir);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int WT, bool HALF, bool LUT, bool POLAR, bool GEN>
static int launch_acc_w(const RoomArgs &ra, const PlanArgs &pa, uint32_t n_items, const AxisEntry *tab,
                        const AxisOrigin *origin, const int *valid, float *out, float *part, float *marg,
                        const float *wc, hipStream_t st) {
  hipLaunchKernelGGL((accumulate_kernel<WT, HALF, images_per_step(WT, HALF), LUT, POLAR, GEN>), dim3(n_items),
                     dim3(64), 0, st, ra, pa, tab, origin, valid, out, part, marg, wc);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_dump(int wt, const RoomArgs &ra, const PlanArgs &pa, uint32_t n_items, const AxisEntry *tab,
                const AxisOrigin *origin, const int *valid, DumpArgs dump, hipStream_t st) {
  hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, st, dump.count, 0u, 1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    fprintf(stderr, "ism_debug_enumerate: fill launch: %s\n", hipGetErrorString(e));
    return -1;
  }
  switch (wt) {
    case 32: hipLaunchKernelGGL(enumerate_dump_kernel<32>, dim3(n_items), dim3(64), 0, st, ra, pa, tab, origin, valid, dump); break;
    case 64: hipLaunchKernelGGL(enumerate_dump_kernel<64>, dim3(n_items), dim3(64), 0, st, ra, pa, tab, origin, valid, dump); break;
    case 96: hipLaunchKernelGGL(enumerate_dump_kernel<96>, dim3(n_items), dim3(64), 0, st, ra, pa, tab, origin, valid, dump); break;
    case 128: hipLaunchKernelGGL(enumerate_dump_kernel<128>, dim3(n_items), dim3(64), 0, st, ra, pa, tab, origin, valid, dump); break;
    case 160: hipLaunchKernelGGL(enumerate_dump_kernel<160>, dim3(n_items), dim3(64), 0, st, ra, pa, tab, origin, valid, dump); break;
    case 192: hipLaunchKernelGGL(enumerate_dump_kernel<192>, dim3(n_items), dim3(64), 0, st, ra, pa, tab, origin, valid, dump); break;
    case 224: hipLaunchKernelGGL(enumerate_dump_kernel<224>, dim3(n_items), dim3(64), 0, st, ra, pa, tab, origin, valid, dump); break;
    case 256: hipLaunchKernelGGL(enumerate_dump_kernel<256>, dim3(n_items), dim3(64), 0, st, ra, pa, tab, origin, valid, dump); break;
    default: return -2;
  }
  e = hipGetLastError();
  if (e != hipSuccess) {
    fprintf(stderr, "ism_debug_enumerate: enumeration launch: %s\n", hipGetErrorString(e));
    return -1;
  }
  return 0;
}

bool supported_window(int wt, bool gen) {
  if (gen) return wt >= 32 && wt <= MAX_WINDOW && wt % 32 == 0;
  return wt == 32 || wt == 64 || wt == 96 || wt == 128;
}

int launch_window_consts(float W, int wt, bool half, float *wc, hipStream_t st) {
  hipLaunchKernelGGL(window_consts_kernel, dim3(1), dim3(MAX_WINDOW), 0, st, W, wt, half ? 1 : 0, wc);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Calls the kernel instance of a window class: exact windows W in {32, 64,
// 96, 128} with every tap mode, general-mode caps 32 .. 256 with FP32 or FP16
// taps. fn is a generic lambda taking the template arguments as values.
template <class Fn>
static int dispatch_window(int wt, bool gen, bool half, bool lut, bool polar, Fn &&fn) {
  if (half && lut) return -2;
  auto by_mode = [&](auto W, auto G) -> int {
    constexpr bool kG = decltype(G)::value;
    if (half) return polar ? fn(W, std::true_type{}, std::false_type{}, std::true_type{}, G)
                           : fn(W, std::true_type{}, std::false_type{}, std::false_type{}, G);
    if constexpr (!kG) {
      if (lut) return polar ? fn(W, std::false_type{}, std::true_type{}, std::true_type{}, G)
                            : fn(W, std::false_type{}, std::true_type{}, std::false_type{}, G);
    } else {
      if (lut) return -2;
    }
    return polar ? fn(W, std::false_type{}, std::false_type{}, std::true_type{}, G)
                 : fn(W, std::false_type{}, std::false_type{}, std::false_type{}, G);
  };
  using F = std::false_type;
  using T = std::true_type;
  if (!gen) {
    switch (wt) {
      case 32: return by_mode(std::integral_constant<int, 32>{}, F{});
      case 64: return by_mode(std::integral_constant<int, 64>{}, F{});
      case 96: return by_mode(std::integral_constant<int, 96>{}, F{});
      case 128: return by_mode(std::integral_constant<int, 128>{}, F{});
      default: return -2;
    }
  }
  switch (wt) {
    case 32: return by_mode(std::integral_constant<int, 32>{}, T{});
    case 64: return by_mode(std::integral_constant<int, 64>{}, T{});
    case 96: return by_mode(std::integral_constant<int, 96>{}, T{});
    case 128: return by_mode(std::integral_constant<int, 128>{}, T{});
    case 160: return by_mode(std::integral_constant<int, 160>{}, T{});
    case 192: return by_mode(std::integral_constant<int, 192>{}, T{});
    case 224: return by_mode(std::integral_constant<int, 224>{}, T{});
    case 256: return by_mode(std::integral_constant<int, 256>{}, T{});
    default: return -2;
  }
}

// polar: directional receivers (any tap mode; half and lut exclusive).
int launch_accumulate(int wt, bool gen, bool half, bool lut, bool polar, const RoomArgs &ra, const PlanArgs &pa,
                      uint32_t n_items, const AxisEntry *tab, const AxisOrigin *origin, const int *valid, float *out,
                      float *part, float *marg, const float *wc, hipStream_t st) {
  return dispatch_window(wt, gen, half, lut, polar, [&](auto W, auto H, auto L, auto P, auto G) -> int {
    return launch_acc_w<decltype(W)::value, decltype(H)::value, decltype(L)::value, decltype(P)::value,
                        decltype(G)::value>(ra, pa, n_items, tab, origin, valid, out, part, marg, wc, st);
  });
}

// grid: workgroups of the persistent launch (at most n_items; the planner
// sizes it from the tuned workgroups per SIMD).
template <int WT, bool HALF, bool LUT, bool POLAR, bool GEN>
static int launch_acc_batch_w(const JobDev *jobs, const BatchItem *items, uint32_t n_items, uint32_t grid,
                              uint32_t *queue, const AxisEntry *tab, const AxisOrigin *origin, const int *valid,
                              float *part, float *marg, hipStream_t st) {
  hipLaunchKernelGGL((accumulate_batch_kernel<WT, HALF, images_per_step(WT, HALF), LUT, POLAR, GEN>),
                     dim3(grid), dim3(64), 0, st, jobs, items, n_items, queue, tab, origin, valid, part, marg);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// queue[k] = the first item of class k not taken by a workgroup's first pick.
__global__ void queue_init_kernel(uint32_t *queue, uint4 a, uint4 b) {
  const uint32_t v[kMaxBatchClasses] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
  if (threadIdx.x < kMaxBatchClasses) queue[threadIdx.x] = v[threadIdx.x];
}

int launch_batch(const JobDev *jobs, int n_jobs, bool any_gen, const BatchRir *rirs, uint32_t n_rir,
                 const BatchItem *items, const uint32_t *class_first, const uint32_t *class_count,
                 const uint32_t *class_grid, const int *class_wt, const int *class_gen, int n_classes, bool half, bool lut, bool polar,
                 const BatchReduce *red, uint32_t n_red, uint32_t n_red_split, bool long_runs, AxisEntry *tab,
                 AxisOrigin *origin, int *valid, float *part, float *marg, uint32_t *queue, hipStream_t st,
                 hipEvent_t ev_start, hipEvent_t ev_stop) {
  hipLaunchKernelGGL(tables_batch_kernel, dim3(n_rir), dim3(256), 0, st, jobs, rirs, tab, origin, valid);
  if (hipGetLastError() != hipSuccess) return -1;
  if (any_gen) {
    hipLaunchKernelGGL(window_consts_batch_kernel, dim3(n_jobs), dim3(MAX_WINDOW), 0, st, jobs, half ? 1 : 0);
    if (hipGetLastError() != hipSuccess) return -1;
  }
  if (queue) {
    uint32_t fp[kMaxBatchClasses] = {};
    for (int k = 0; k < n_classes && k < kMaxBatchClasses; ++k) fp[k] = class_grid[k];
    hipLaunchKernelGGL(queue_init_kernel, dim3(1), dim3(64), 0, st, queue, make_uint4(fp[0], fp[1], fp[2], fp[3]),
                       make_uint4(fp[4], fp[5], fp[6], fp[7]));
    if (hipGetLastError() != hipSuccess) return -1;
  }
  if (ev_start && hipEventRecord(ev_start, st) != hipSuccess) return -1;
  for (int k = 0; k < n_classes; ++k) {
    if (class_count[k] == 0) continue;
    const BatchItem *it = items + class_first[k];
    uint32_t *qk = queue ? queue + k : nullptr;
    const int rc = dispatch_window(class_wt[k], class_gen[k] != 0, half, lut, polar,
                                   [&](auto W, auto H, auto L, auto P, auto G) -> int {
                                     return launch_acc_batch_w<decltype(W)::value, decltype(H)::value,
                                                               decltype(L)::value, decltype(P)::value,
                                                               decltype(G)::value>(jobs, it, class_count[k],
                                                                                   class_grid[k], qk, tab, origin,
                                                                                   valid, part, marg, st);
                                   });
    if (rc != 0) return -1;
  }
  if (ev_stop && hipEventRecord(ev_stop, st) != hipSuccess) return -1;
  if (n_red_split > 0) {
    // split tiles, whole tiles; runs of RED_SLICE_MIN terms or more: RED_SLICES threads per sample
    if (long_runs)
      hipLaunchKernelGGL(reduce_batch_kernel<true>, dim3(n_red_split, TILE / RED_SAMPLES), dim3(256), 0, st, jobs, red,
                         part, marg);
    else
      hipLaunchKernelGGL(reduce_batch_kernel<false>, dim3(n_red_split, TILE / 256), dim3(256), 0, st, jobs, red, part,
                         marg);
    if (hipGetLastError() != hipSuccess) return -1;
  }
  if (n_red > n_red_split) {  // the other tiles: their margin samples only
    hipLaunchKernelGGL(reduce_margins_kernel, dim3(n_red - n_red_split), dim3(64), 0, st, jobs, red + n_red_split,
                       marg);
    if (hipGetLastError() != hipSuccess) return -1;
  }
  return 0;
}

int launch_reduce(const RoomArgs &ra, const PlanArgs &pa, int n_rir, const float *part, const float *marg,
                  float *out, hipStream_t st) {
  int max_c = 0;  // longest run: the most items of any tile (its own, or a neighbour's margins)
  for (int t = 0; t < pa.n_tiles; ++t) max_c = max(max_c, (int)pa.chunks[t]);
  if (max_c >= RED_SLICE_MIN)
    hipLaunchKernelGGL(reduce_kernel<true>, dim3((unsigned)n_rir, (unsigned)pa.n_tiles, TILE / RED_SAMPLES), dim3(256),
                       0, st, ra, pa, part, marg, out);
  else
    hipLaunchKernelGGL(reduce_kernel<false>, dim3((unsigned)n_rir, (unsigned)pa.n_tiles, TILE / 256), dim3(256), 0, st,
                       ra, pa, part, marg, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace ism
