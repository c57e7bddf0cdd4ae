/*
 * FP64 reference ("oracle") for the Image Source Method room impulse response.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the GPU library.
 *
 * Written from the paper (gpuRIR, Diaz-Guerra et al.), Sec. 2:
 *   Sec. 2.1  lattice of images, Eq. (1) positions, Eq. (2)-(3) distance and
 *             delay, Eq. (4) amplitude, Eq. (5) RIR as a sum of delayed impulses;
 *   Sec. 2.2  Eq. (6) Hann-windowed sinc replacing the impulse (cut-off fs/2),
 *             signed reflection coefficients, Eq. (7) Sabine's formula;
 *   Sec. 3.5  Eq. (9) the windowed sinc tabulated at Q points per sample and
 *             read by linear interpolation (the lookup-table variant);
 *   Sec. 4    directional receivers (pattern and orientation; no formula in
 *             the paper: the first-order family a + (1 - a) cos(theta)).
 * Readings where the paper is silent (wall exponents, grid size, taps before
 * t = 0) are stated at the function that takes them.
 *
 * Parity pins: see tests/test_oracle_pins.py. No function here is unpinned.
 */
#include "ism_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>

static const double PI = 3.14159265358979323846;

int64_t oracle_n_samples(double t_max, double fs) {
  double v = t_max * fs;
  double r = nearbyint(v);
  if (fabs(v - r) <= 1e-9 * fabs(v)) return (int64_t)r;
  return (int64_t)ceil(v);
}

/* Eq. (7): T60 = 0.161 V / sum_i S_i alpha_i with alpha_i = 1 - beta_i^2.
 * With one beta for all six walls, sum_i S_i alpha_i = S (1 - beta^2), hence
 * beta = sqrt(1 - 0.161 V / (S T60)). The constant is the paper's, as printed. */
int oracle_beta_from_t60(const double L[3], double t60, double beta_out[6]) {
  if (!(t60 > 0.0)) return -1;
  double V = L[0] * L[1] * L[2];
  double S = 2.0 * (L[0] * L[1] + L[0] * L[2] + L[1] * L[2]);
  double alpha = 0.161 * V / (S * t60);
  if (alpha > 1.0) return -2;
  double b = sqrt(1.0 - alpha);
  for (int i = 0; i < 6; ++i) beta_out[i] = b;
  return 0;
}

/* Reading of "images per dimension for a simulation time without lost
 * reflections" (Sec. 4): images come in pairs at 2 m L +- x_s; keeping every
 * pair index |m| <= K with K = ceil(c t / (2 L)) keeps every image closer than
 * c t, and in the lattice indexing of Sec. 2.1 that is N = 4 K + 2. */
void oracle_n_img_for_time(const double L[3], double c, double t, int n_out[3]) {
  for (int a = 0; a < 3; ++a) n_out[a] = 4 * (int)ceil(c * t / (2.0 * L[a])) + 2;
}

double oracle_time_for_attenuation(double t60, double att_db) { return t60 * att_db / 60.0; }

/* Lattice bounds of Sec. 2.1: ceil(-N/2) <= n < ceil(N/2). */
static int lat_lo(int N) { return (int)ceil(-N / 2.0); }
static int lat_hi(int N) { return (int)ceil(N / 2.0); }

/* Eq. (1): coordinate of image n along one axis. */
static double image_coord(int n, double L, double s) {
  if (n % 2 == 0) return n * L + s;
  return (n + 1) * L - s;
}

/* beta^e by repeated multiplication, so that 0^0 = 1 and a signed beta keeps
 * its sign pattern exactly. */
static double ipow(double b, int e) {
  double r = 1.0;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

/* Reading of the gain of Sec. 2.1 ("product of the reflection coefficients of
 * each wall crossed"): along an axis, the path from image n crosses |n| walls,
 * |floor(n/2)| of them copies of the wall at 0 and |ceil(n/2)| copies of the
 * wall at L. */
static double axis_gain(int n, double b0, double b1) {
  int e0 = abs((int)floor(n / 2.0));
  int e1 = abs((int)ceil(n / 2.0));
  return ipow(b0, e0) * ipow(b1, e1);
}

typedef struct {
  double gain, d, x, A;
  double to_image[3]; /* p_n - p_r: from the receiver to the image */
} image_t;

/* One image: Eq. (1) position, Eq. (2) distance (reading: the norm is taken to
 * the image, p_r - p_n), Eq. (3) delay in samples, Eq. (4) amplitude. */
static image_t make_image(const oracle_room *room, const double src[3], const double rcv[3], int nx,
                          int ny, int nz) {
  const int n[3] = {nx, ny, nz};
  image_t im;
  double g = 1.0, d2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    double p = image_coord(n[a], room->L[a], src[a]);
    double diff = rcv[a] - p;
    d2 += diff * diff;
    im.to_image[a] = -diff;
    g *= axis_gain(n[a], room->beta[2 * a], room->beta[2 * a + 1]);
  }
  im.gain = g;
  im.d = sqrt(d2);
  im.x = im.d / room->c * room->fs;
  im.A = g / (4.0 * PI * im.d);
  return im;
}

/* Eq. (6) sampled at t = (k - x)/fs with f_c = fs/2 and W = T_w fs samples:
 * 0.5 (1 + cos(2 pi v / W)) sin(pi v)/(pi v), v = k - x, for |v| < W/2. */
static double windowed_sinc(double v, double W) {
  double hann = 0.5 * (1.0 + cos(2.0 * PI * v / W));
  double sinc = (v == 0.0) ? 1.0 : sin(PI * v) / (PI * v);
  return hann * sinc;
}

/* Eq. (9): LUT[n] = 0.5 (1 + cos(2 pi n / (Q W))) sinc(pi n / Q) for
 * n = -QW/2 .. QW/2, i.e. Eq. (6) at v = n / Q; sinc(pi u) = sin(pi u)/(pi u).
 * Stored at index n + QW/2. Returns NULL when QW/2 is not an integer. */
static double *make_lut(double W, int q) {
  const double half = q * W / 2.0;
  const int64_t h = (int64_t)llround(half);
  if (q < 1 || h < 1 || fabs(half - (double)h) > 1e-9 * half) return NULL;
  double *lut = (double *)malloc(sizeof(double) * (size_t)(2 * h + 1));
  if (!lut) return NULL;
  for (int64_t n = -h; n <= h; ++n) {
    double hann = 0.5 * (1.0 + cos(2.0 * PI * (double)n / (q * W)));
    double u = (double)n / q;
    double sinc = (n == 0) ? 1.0 : sin(PI * u) / (PI * u);
    lut[n + h] = hann * sinc;
  }
  return lut;
}

/* Sec. 3.5: the tap at v (|v| < W/2) by linear interpolation between the two
 * table entries around v Q: n0 = floor(v Q), a = v Q - n0,
 * tap = LUT[n0] + a (LUT[n0 + 1] - LUT[n0]). */
static double lut_tap(const double *lut, double W, int q, double v) {
  const int64_t h = (int64_t)llround(q * W / 2.0);
  const double p = v * q;
  int64_t n0 = (int64_t)floor(p);
  if (n0 < -h) n0 = -h;          /* only p = -QW/2 exactly */
  if (n0 > h - 1) n0 = h - 1;    /* only p = +QW/2 exactly */
  const double a = p - (double)n0;
  return lut[n0 + h] + a * (lut[n0 + 1 + h] - lut[n0 + h]);
}

int oracle_lut_taps(const double *v, int64_t n, double W, int q, double *out) {
  double *lut = make_lut(W, q);
  if (!lut) return -1;
  for (int64_t i = 0; i < n; ++i)
    out[i] = (fabs(v[i]) < W / 2.0) ? lut_tap(lut, W, q, v[i]) : 0.0;
  free(lut);
  return 0;
}

/* Eq. (5) with Eq. (6) in place of the impulse, restricted to k in
 * [k_begin, k_end). Taps that would fall before k = 0 or after the last sample
 * are dropped (reading: no wrap-around, no shift). With lut != NULL each tap
 * is read from the table of Eq. (9) (q points per sample) instead. With
 * orient != NULL the receiver is directional (the library of Sec. 4 takes a
 * polar pattern and an orientation; the paper gives no formula). Reading: the
 * first-order family, each image's amplitude times a + (1 - a) cos(theta),
 * theta the angle between orient and the direction from the receiver to the
 * image. */
static int rir_window(const oracle_room *room, const double src[3], const double rcv[3], int64_t k_begin,
                      int64_t k_end, const double *lut, int q, const double *orient, double pattern_a,
                      double *out) {
  const double W = room->t_w * room->fs;
  double onorm = 0.0;
  if (orient) {
    onorm = sqrt(orient[0] * orient[0] + orient[1] * orient[1] + orient[2] * orient[2]);
    if (!(onorm > 0.0)) return -1;
  }
  for (int64_t k = k_begin; k < k_end; ++k) out[k - k_begin] = 0.0;
  for (int nx = lat_lo(room->n[0]); nx < lat_hi(room->n[0]); ++nx)
    for (int ny = lat_lo(room->n[1]); ny < lat_hi(room->n[1]); ++ny)
      for (int nz = lat_lo(room->n[2]); nz < lat_hi(room->n[2]); ++nz) {
        image_t im = make_image(room, src, rcv, nx, ny, nz);
        if (!(im.d > 0.0)) return -1;
        if (orient) {
          double cos_theta = (im.to_image[0] * orient[0] + im.to_image[1] * orient[1] +
                              im.to_image[2] * orient[2]) / (im.d * onorm);
          im.A *= pattern_a + (1.0 - pattern_a) * cos_theta;
        }
        int64_t first = (int64_t)floor(im.x - W / 2.0) + 1; /* smallest k > x - W/2 */
        int64_t last = (int64_t)ceil(im.x + W / 2.0) - 1;   /* largest k < x + W/2  */
        if (first < k_begin) first = k_begin;
        if (last > k_end - 1) last = k_end - 1;
        for (int64_t k = first; k <= last; ++k) {
          double v = (double)k - im.x;
          if (fabs(v) < W / 2.0)
            out[k - k_begin] += im.A * (lut ? lut_tap(lut, W, q, v) : windowed_sinc(v, W));
        }
      }
  return 0;
}

int oracle_rir_window(const oracle_room *room, const double src[3], const double rcv[3],
                      int64_t k_begin, int64_t k_end, double *out) {
  return rir_window(room, src, rcv, k_begin, k_end, NULL, 0, NULL, 1.0, out);
}

typedef struct {
  const oracle_room *room;
  const double *src, *rcv;
  int n_src, n_rcv;
  int64_t k_begin, k_end;
  const double *lut;
  int q;
  const double *orient; /* [n_rcv][3] or NULL */
  double pattern_a;
  double *out;
  int next, status;
  pthread_mutex_t lock;
} batch_t;

static void *batch_worker(void *arg) {
  batch_t *b = (batch_t *)arg;
  const int64_t len = b->k_end - b->k_begin;
  for (;;) {
    pthread_mutex_lock(&b->lock);
    int p = b->next++;
    pthread_mutex_unlock(&b->lock);
    if (p >= b->n_src * b->n_rcv) break;
    int s = p / b->n_rcv, r = p % b->n_rcv;
    int st = rir_window(b->room, b->src + 3 * s, b->rcv + 3 * r, b->k_begin, b->k_end, b->lut, b->q,
                        b->orient ? b->orient + 3 * r : NULL, b->pattern_a, b->out + (int64_t)p * len);
    if (st != 0) {
      pthread_mutex_lock(&b->lock);
      if (b->status == 0) b->status = st;
      pthread_mutex_unlock(&b->lock);
    }
  }
  return NULL;
}

static int rir_batch(const oracle_room *room, const double *src, int n_src, const double *rcv, int n_rcv,
                     int64_t k_begin, int64_t k_end, int q, const double *orient, double pattern_a,
                     int n_threads, double *out) {
  if (n_src < 0 || n_rcv < 0 || k_begin < 0 || k_end < k_begin || q < 0) return -1;
  if (n_threads < 1) n_threads = 1;
  double *lut = NULL;
  if (q > 0) {
    lut = make_lut(room->t_w * room->fs, q);
    if (!lut) return -1;
  }
  batch_t b;
  b.lut = lut;
  b.q = q;
  b.orient = orient;
  b.pattern_a = pattern_a;
  b.room = room;
  b.src = src;
  b.rcv = rcv;
  b.n_src = n_src;
  b.n_rcv = n_rcv;
  b.k_begin = k_begin;
  b.k_end = k_end;
  b.out = out;
  b.next = 0;
  b.status = 0;
  pthread_mutex_init(&b.lock, NULL);
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)n_threads);
  int started = 0;
  for (int i = 0; i < n_threads; ++i)
    if (pthread_create(&th[i], NULL, batch_worker, &b) == 0) ++started;
  if (started == 0) batch_worker(&b);
  for (int i = 0; i < started; ++i) pthread_join(th[i], NULL);
  free(th);
  free(lut);
  pthread_mutex_destroy(&b.lock);
  return b.status;
}

int oracle_rir_batch_lut(const oracle_room *room, const double *src, int n_src, const double *rcv,
                         int n_rcv, int64_t k_begin, int64_t k_end, int q, int n_threads, double *out) {
  return rir_batch(room, src, n_src, rcv, n_rcv, k_begin, k_end, q, NULL, 1.0, n_threads, out);
}

int oracle_rir_batch(const oracle_room *room, const double *src, int n_src, const double *rcv,
                     int n_rcv, int64_t k_begin, int64_t k_end, int n_threads, double *out) {
  return rir_batch(room, src, n_src, rcv, n_rcv, k_begin, k_end, 0, NULL, 1.0, n_threads, out);
}

int oracle_rir_batch_polar(const oracle_room *room, const double *src, int n_src, const double *rcv,
                           int n_rcv, const double *orient, double pattern_a, int64_t k_begin, int64_t k_end,
                           int q, int n_threads, double *out) {
  if (!orient || !(pattern_a >= 0.0 && pattern_a <= 1.0)) return -1;
  return rir_batch(room, src, n_src, rcv, n_rcv, k_begin, k_end, q, orient, pattern_a, n_threads, out);
}

int64_t oracle_image_list(const oracle_room *room, const double src[3], const double rcv[3],
                          int32_t *idx, double *vals, int64_t cap) {
  int64_t i = 0;
  for (int nx = lat_lo(room->n[0]); nx < lat_hi(room->n[0]); ++nx)
    for (int ny = lat_lo(room->n[1]); ny < lat_hi(room->n[1]); ++ny)
      for (int nz = lat_lo(room->n[2]); nz < lat_hi(room->n[2]); ++nz, ++i) {
        if (idx == NULL || vals == NULL || i >= cap) continue;
        image_t im = make_image(room, src, rcv, nx, ny, nz);
        idx[3 * i] = nx;
        idx[3 * i + 1] = ny;
        idx[3 * i + 2] = nz;
        vals[4 * i] = im.gain;
        vals[4 * i + 1] = im.d;
        vals[4 * i + 2] = im.x;
        vals[4 * i + 3] = im.A;
      }
  return i;
}

int64_t oracle_count_taps(const oracle_room *room, const double src[3], const double rcv[3]) {
  const double W = room->t_w * room->fs;
  const int64_t nS = oracle_n_samples(room->t_max, room->fs);
  int64_t taps = 0;
  for (int nx = lat_lo(room->n[0]); nx < lat_hi(room->n[0]); ++nx)
    for (int ny = lat_lo(room->n[1]); ny < lat_hi(room->n[1]); ++ny)
      for (int nz = lat_lo(room->n[2]); nz < lat_hi(room->n[2]); ++nz) {
        image_t im = make_image(room, src, rcv, nx, ny, nz);
        int64_t first = (int64_t)floor(im.x - W / 2.0) + 1;
        int64_t last = (int64_t)ceil(im.x + W / 2.0) - 1;
        if (first < 0) first = 0;
        if (last > nS - 1) last = nS - 1;
        for (int64_t k = first; k <= last; ++k)
          if (fabs((double)k - im.x) < W / 2.0) ++taps;
      }
  return taps;
}
