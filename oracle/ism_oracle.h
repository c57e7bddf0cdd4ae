/*
 * FP64 reference ("oracle") for the Image Source Method room impulse response.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. It shares no code,
 * header, table or constant with the GPU library under paper_1810_11359_amd/.
 *
 * It evaluates the plain definition of the ISM sum (Sec. 2.1, Eq. (1)-(5), with
 * the Hann-windowed sinc of Eq. (6) in place of the Dirac impulse) in double
 * precision with libm sin/cos, in the paper's own order: for every image of the
 * lattice, position -> distance -> delay -> amplitude -> windowed-sinc taps.
 *
 * All entry points are plain C, take host pointers and return a status
 * (0 = ok, negative = invalid argument) or a count.
 */
#ifndef ISM_ORACLE_H
#define ISM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double L[3];      /* room size Lx, Ly, Lz [m]                                 */
  double beta[6];   /* reflection coefficients x0, x1, y0, y1, z0, z1; x0 is the
                       wall in the plane x = 0, x1 the wall in the plane x = Lx */
  int n[3];         /* images per dimension Nx, Ny, Nz (Sec. 2.1)               */
  double c;         /* speed of sound [m/s]                                     */
  double fs;        /* sampling rate [Hz]                                       */
  double t_max;     /* RIR length [s]                                           */
  double t_w;       /* window length T_w of Eq. (6) [s]                         */
} oracle_room;

/* Number of output samples: ceil(t_max*fs), snapped to the nearest integer when
 * t_max*fs is within 1e-9 (relative) of it. */
int64_t oracle_n_samples(double t_max, double fs);

/* Uniform reflection coefficient for a target T60 by Sabine's formula, Eq. (7)
 * with alpha = 1 - beta^2. Returns -2 when the target is infeasible (alpha > 1). */
int oracle_beta_from_t60(const double L[3], double t60, double beta_out[6]);

/* Images per dimension such that no image closer than c*t is left out of the
 * lattice: N = 4*ceil(c*t/(2L)) + 2 per axis. */
void oracle_n_img_for_time(const double L[3], double c, double t, int n_out[3]);

/* Time at which an exponential (Sabine) decay of the given T60 reaches att_db of
 * attenuation: t60 * att_db / 60. */
double oracle_time_for_attenuation(double t60, double att_db);

/* h[k] for k in [k_begin, k_end) of the RIR between src and rcv (k_begin >= 0,
 * k_end <= number of samples). out has k_end - k_begin doubles. Returns -1 if
 * an image coincides with the receiver. */
int oracle_rir_window(const oracle_room *room, const double src[3], const double rcv[3],
                      int64_t k_begin, int64_t k_end, double *out);

/* Windows [k_begin, k_end) of the RIRs of every (src, rcv) pair, src-major:
 * out[(s*n_rcv + r)*(k_end-k_begin) + k - k_begin]. Runs on n_threads POSIX
 * threads (one pair at a time per thread). Returns the first failing status. */
int oracle_rir_batch(const oracle_room *room, const double *src, int n_src,
                     const double *rcv, int n_rcv, int64_t k_begin, int64_t k_end,
                     int n_threads, double *out);

/* As oracle_rir_batch, with every tap read from the table of Eq. (9) at q
 * points per sample by linear interpolation (Sec. 3.5) when q > 0 (q = 0: the
 * exact Eq. (6)). Returns -1 when q W / 2 is not an integer. */
int oracle_rir_batch_lut(const oracle_room *room, const double *src, int n_src, const double *rcv,
                         int n_rcv, int64_t k_begin, int64_t k_end, int q, int n_threads, double *out);

/* As oracle_rir_batch with directional receivers: every image's amplitude
 * times a + (1 - a) cos(theta), theta the angle between orient[r] (the
 * receiver's orientation, [n_rcv][3], any nonzero length) and the direction
 * from the receiver to the image; a = pattern_a in [0, 1]. Returns -1 for a
 * null orient, a pattern outside [0, 1] or a zero orientation. q > 0: table
 * taps as for oracle_rir_batch_lut. */
int oracle_rir_batch_polar(const oracle_room *room, const double *src, int n_src, const double *rcv,
                           int n_rcv, const double *orient, double pattern_a, int64_t k_begin, int64_t k_end,
                           int q, int n_threads, double *out);

/* Table taps of Sec. 3.5 at the offsets v[0..n) (v = k - x in samples, 0 for
 * |v| >= W/2), table of Eq. (9) at q points per sample. Returns -1 when
 * q W / 2 is not an integer. */
int oracle_lut_taps(const double *v, int64_t n, double W, int q, double *out);

/* Every lattice image in the order nx, ny, nz (outermost first). When idx/vals
 * are non-null, writes up to cap entries: idx[3*i..] = (nx, ny, nz) and
 * vals[4*i..] = (gain, distance d [m], delay x = d*fs/c [samples],
 * amplitude A = gain/(4 pi d)). Returns the lattice size. */
int64_t oracle_image_list(const oracle_room *room, const double src[3], const double rcv[3],
                          int32_t *idx, double *vals, int64_t cap);

/* Exact number of window taps inside the output: sum over lattice images of
 * #{k in [0, nS) : |k - x| < W/2}, W = t_w*fs. */
int64_t oracle_count_taps(const oracle_room *room, const double src[3], const double rcv[3]);

#ifdef __cplusplus
}
#endif
#endif
