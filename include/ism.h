/*
 * ism.h - C ABI of the MI355X (gfx950) Image Source Method library (libism.so).
 *
 * The library computes room impulse responses (RIRs) of a shoebox room with the
 * Image Source Method of Allen and Berkley as restated in the gpuRIR paper
 * (Diaz-Guerra et al.), Sec. 2.1: for every (source, receiver) pair it sums,
 * over the lattice of image sources, a Hann-windowed sinc (Sec. 2.2, Eq. (6))
 * of amplitude beta_n / (4 pi d_n) (Eq. (4)) delayed by d_n / c (Eq. (3)).
 *
 * Conventions shared by every entry point:
 *  - Plain C types only. "host" pointers are CPU memory, "device" pointers are
 *    memory of the current HIP device. The caller owns every buffer; the
 *    library allocates nothing in the simulate calls and keeps no global
 *    mutable state, so calls are reentrant.
 *  - Every call returns an int status: ISM_OK (0) or a negative ISM_E_* code.
 *    All argument checks run before any launch; a call that fails them leaves
 *    every output untouched. No C++ exception crosses this boundary.
 *  - GPU calls are asynchronous on the given HIP stream (NULL = the default
 *    stream). A launch failure is reported as ISM_E_DEVICE.
 */
#ifndef ISM_H
#define ISM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ISM_ABI_VERSION 1

enum {
  ISM_OK = 0,
  ISM_E_INVALID_ARG = -1,    /* null pointer, non-positive size, NaN, ...          */
  ISM_E_INFEASIBLE_T60 = -2, /* Sabine's formula needs an absorption above 1       */
  ISM_E_OUT_OF_ROOM = -3,    /* a position not strictly inside the room            */
  ISM_E_WORKSPACE = -4,      /* workspace missing or smaller than required         */
  ISM_E_DEVICE = -5,         /* HIP launch or runtime error                        */
  ISM_E_TOO_LARGE = -6,      /* problem exceeds a documented limit (see below)     */
  ISM_E_UNSUPPORTED = -7     /* valid request the library does not implement       */
};

/* Arithmetic used for the windowed-sinc taps. Geometry, delays and the
 * accumulation are FP32 in every mode.
 * ISM_FP32_LUT: each tap is read from a table of the windowed sinc of Eq. (6)
 *   at Q = 16 points per sample (Eq. (9), Sec. 3.5) and interpolated linearly
 *   between the two entries around its delay, in FP32. The interpolation
 *   moves a tap by at most 1.6e-3 of its amplitude from Eq. (6) (the linear
 *   interpolation bound h^2/8 max|s''| with h = 1/16). All calls accept it. */
typedef enum { ISM_FP32 = 0, ISM_FP16 = 1, ISM_BF16 = 2, ISM_FP32_LUT = 3 } ism_precision;

/* One shoebox room and its simulation parameters (Sec. 2.1, Sec. 4). */
typedef struct {
  double room[3];  /* Lx, Ly, Lz [m], > 0                                            */
  double beta[6];  /* reflection coefficients in [-1, 1], order x0, x1, y0, y1, z0, z1;
                      x0 is the wall in the plane x = 0, x1 the wall in x = Lx       */
  int n_img[3];    /* images per dimension N_a >= 1; lattice index n_a runs over
                      ceil(-N_a/2) <= n_a < ceil(N_a/2) (Sec. 2.1)                  */
  double c;        /* speed of sound [m/s], > 0                                     */
  double fs;       /* sampling rate [Hz], > 0                                       */
  double t_max;    /* RIR length [s], > 0; nS = ism_n_samples(t_max, fs)            */
  double t_w;      /* Hann window length T_w of Eq. (6) [s], > 0; W = t_w*fs samples,
                      cut-off frequency fs/2                                        */
} ism_room;

/* Limits of the library (ISM_E_TOO_LARGE beyond them). */
#define ISM_MAX_SAMPLES (256 * 1024) /* nS per RIR                                     */
#define ISM_MAX_N_IMG 2048           /* N_a per axis                                   */
#define ISM_MAX_PAIRS (1 << 22)      /* n_src * n_rcv per call                         */

/* Human-readable name of a status code (static storage, never NULL). */
const char *ism_status_string(int status);

/* ISM_ABI_VERSION of the loaded library. */
int ism_abi_version(void);

/* ---- Host helpers (Sec. 4: helper functions of the library) ---------------- */

/* Uniform reflection coefficient for all six walls giving reverberation time
 * t60 by Sabine's formula (Sec. 2.2, Eq. (7)) with alpha = 1 - beta^2:
 * beta = sqrt(1 - 0.161 V / (S t60)). beta_out: host [6].
 * ISM_E_INFEASIBLE_T60 when 0.161 V / (S t60) > 1. */
int ism_beta_from_t60(const double room[3], double t60, double beta_out[6]);

/* Images per dimension so that no image closer than c*t is left out of the
 * lattice: N_a = 4 ceil(c t / (2 L_a)) + 2. n_out: host [3]. */
int ism_n_img_for_time(const double room[3], double c, double t, int n_out[3]);

/* Time at which the exponential energy decay of reverberation time t60
 * reaches att_db decibels of attenuation: t60 * att_db / 60. */
int ism_time_for_attenuation(double t60, double att_db, double *t_out);

/* Samples per RIR: ceil(t_max*fs), snapped to the nearest integer when t_max*fs
 * lies within 1e-9 (relative) of it. Returns -1 for invalid input. */
int64_t ism_n_samples(double t_max, double fs);

/* ---- Validation -------------------------------------------------------------- */

/* Checks every field of *room (finite, positive sizes, |beta| <= 1, limits). */
int ism_check_room(const ism_room *room);

/* Checks host positions src [n_src][3], rcv [n_rcv][3] (float32): each strictly
 * inside the room (0 < p_a < L_a) -> else ISM_E_OUT_OF_ROOM; a source equal to
 * a receiver -> ISM_E_INVALID_ARG (its direct path has zero length). */
int ism_check_positions(const ism_room *room, const float *src, int n_src, const float *rcv, int n_rcv);

/* ---- Work measure -------------------------------------------------------------- */

/* Exact number of window taps the simulation evaluates, summed over all pairs:
 * sum over (src, rcv, lattice image) of #{k in [0, nS) : |k - x| < W/2},
 * x = d fs / c, computed on the host in double precision from host positions. */
int ism_count_taps(const ism_room *room, const float *src, int n_src, const float *rcv, int n_rcv,
                   int64_t *taps_out);

/* ---- Work schedule ------------------------------------------------------------------ */

/* How a call splits its work into work items (units of the accumulation
 * kernel: one RIR, one 256-sample output tile, one slab of the image shell
 * that tile owns). The split changes the summation order, so results agree
 * across schedules within rounding (<= 1e-6 of the RIR peak), not bitwise; a
 * given schedule always gives the same bits. NULL means the tuned default. A
 * field left at 0 (tail_rounds: < 0) keeps its default. Used by tuning and
 * tests; the library reads no environment variables. */
typedef struct {
  double item_taps;     /* > 0: every work item holds about this many estimated taps,
                           with no tail taper                                         */
  double min_item_taps; /* > 0: smallest work item (replaces the tuned value)         */
  double balance_items; /* > 0: items a large call is split into (replaces the tuned
                           value; sets the item size of large calls)                  */
  double tail_rounds;   /* single calls: the items dispatched once less than this many
                           rounds of resident waves of work remain are cut smaller so
                           the launch ends evenly; 0 = no taper, < 0 = default (1)    */
  double batch_waves;   /* batches: workgroups per SIMD of each persistent launch
                           (1 .. 16; the grid is 1024 times this); 0 = tuned value */
} ism_schedule;

/* ---- GPU simulation -------------------------------------------------------------- */

/* Device workspace (bytes) that ism_simulate needs for this room, pair count
 * and precision. The size depends only on these arguments. */
int ism_workspace_size(const ism_room *room, int n_src, int n_rcv, int precision, size_t *bytes);

/* RIRs of every (source, receiver) pair of one room: the problem statement of
 * Sec. 4 (room, reflection coefficients, positions, fs, RIR length, window)
 * with positions given in host memory.
 *   src   host float32 [n_src][3], rcv host float32 [n_rcv][3] (positions [m]),
 *         checked as by ism_check_positions before any launch (a position not
 *         strictly inside the room -> ISM_E_OUT_OF_ROOM, a source equal to a
 *         receiver -> ISM_E_INVALID_ARG) and copied into the workspace, so the
 *         host arrays may be reused as soon as the call returns;
 *   out   device float32 [n_src][n_rcv][nS], row-major, fully overwritten;
 *   ws    device workspace of at least ism_workspace_size() bytes;
 *   stream  hipStream_t or NULL.
 * A call that fails any check returns its status and leaves out untouched.
 * Kernels run asynchronously on stream; results are those of ism_simulate. */
int ism_simulate_host(const ism_room *room, const float *src, int n_src, const float *rcv, int n_rcv,
                      int precision, float *out, void *ws, size_t ws_bytes, void *stream);

/* RIRs of every (source, receiver) pair of one room, positions in device memory
 * (an extension of ism_simulate_host for callers whose positions are already
 * on the GPU).
 *   src   device float32 [n_src][3], rcv device float32 [n_rcv][3] (positions [m]);
 *   out   device float32 [n_src][n_rcv][nS], row-major, fully overwritten;
 *   ws    device workspace of at least ism_workspace_size() bytes (contents
 *         need not be initialised; overwritten);
 *   stream  hipStream_t or NULL.
 * Room, counts, precision and workspace are checked before any launch.
 * Positions live on the device, so they are checked there: a pair whose
 * source or receiver is not strictly inside the room, or whose source equals
 * its receiver, gets an RIR filled with NaN (ism_simulate_host returns a
 * status instead). The summation order is fixed, so repeated calls with the
 * same arguments give bitwise identical results.
 * Asynchronous; out and ws must stay valid until the stream reaches it. */
int ism_simulate(const ism_room *room, const float *src, int n_src, const float *rcv, int n_rcv,
                 int precision, float *out, void *ws, size_t ws_bytes, void *stream);

/* ism_simulate, plus per-kernel timing: records the caller's HIP events
 * ev_start immediately before and ev_stop immediately after the tap
 * accumulation kernel (the dominant kernel), on the same stream. Either event
 * may be NULL. The events are caller-owned (hipEventCreate); the library only
 * records them. Same arguments, checks and results as ism_simulate. */
int ism_simulate_timed(const ism_room *room, const float *src, int n_src, const float *rcv, int n_rcv,
                       int precision, float *out, void *ws, size_t ws_bytes, void *stream, void *ev_start,
                       void *ev_stop);

/* ism_simulate_timed with an explicit work schedule (see ism_schedule; NULL =
 * default, the same as ism_simulate_timed). The workspace must hold
 * ism_workspace_size_ex() bytes for the same schedule. */
int ism_workspace_size_ex(const ism_room *room, int n_src, int n_rcv, int precision, const ism_schedule *sched,
                          size_t *bytes);
int ism_simulate_ex(const ism_room *room, const float *src, int n_src, const float *rcv, int n_rcv, int precision,
                    const ism_schedule *sched, float *out, void *ws, size_t ws_bytes, void *stream, void *ev_start,
                    void *ev_stop);

/* ism_simulate with directional receivers (the paper's library takes each
 * receiver's polar pattern and orientation, Sec. 4; it gives no formula).
 * Reading: the first-order pattern family, each image's amplitude (Eq. (4))
 * times a + (1 - a) cos(theta), theta the angle between the receiver's
 * orientation and the direction from the receiver to the image. a = 1 is
 * omnidirectional (same result as ism_simulate), 0.75 subcardioid, 0.5
 * cardioid, 0.25 hypercardioid, 0 bidirectional (figure of eight).
 *   orient: device float32 [n_rcv][3], one orientation per receiver in room
 *           axes; need not be unit length (normalised here); a zero vector
 *           gives NaN RIRs for that receiver;
 *   pattern: a in [0, 1], the same for every receiver;
 *   precision: ISM_FP32, ISM_FP16 or ISM_FP32_LUT (the pattern scales each
 *           image's amplitude before its taps, in FP32; ISM_BF16 returns
 *           ISM_E_UNSUPPORTED as for ism_simulate);
 *   the other arguments, the workspace (ism_workspace_size with the same
 *   room, counts and precision) and the errors as for ism_simulate, all
 *   checked before any launch; ISM_E_INVALID_ARG for a null orient or a
 *   pattern outside [0, 1]. Asynchronous. */
int ism_simulate_polar(const ism_room *room, const float *src, int n_src, const float *rcv, int n_rcv,
                       const float *orient, double pattern, int precision, float *out, void *ws, size_t ws_bytes,
                       void *stream);

/* ---- Diffuse reverberation tail (Sec. 2.2, Eq. (8); Sec. 3.3) --------------- */

/* Device workspace (bytes) that ism_simulate_diffuse needs; depends only on
 * these arguments. */
int ism_diffuse_workspace_size(const ism_room *room, double t_diff, double t60, int n_src, int n_rcv,
                               int precision, size_t *bytes);

/* RIRs whose early part is the ISM and whose late part is a noise tail with an
 * exponential power envelope (Sec. 2.2, Eq. (8); Sec. 3.3).
 *   room    t_max is the full RIR length (nS = ism_n_samples(t_max, fs)); n_img
 *           is the image lattice of the ISM part (ism_n_img_for_time(room, c,
 *           t_diff) covers every image arriving before t_diff);
 *   t_diff  switch time [s], 0 < t_diff <= t_max: samples k < k_diff =
 *           ism_n_samples(t_diff, fs) are the ISM RIR computed as ism_simulate
 *           with t_max = t_diff (same precision rules);
 *   t60     reverberation time of the envelope [s], > 0;
 *   seed    selects the noise streams.
 * For k >= k_diff, sample k of RIR i (i = source * n_rcv + receiver) is
 *   z_ik * sqrt(A_i * 10^(-6 (k/fs - t_diff) / t60)),
 * where A_i is the mean of h_i[k]^2 / 10^(-6 (k/fs - t_diff) / t60) over the
 * last fifth of the ISM part (samples [k_diff - max(1, k_diff / 5), k_diff)),
 * and z_ik is the unit-variance logistic variate log(u / (1 - u)) sqrt(3)/pi,
 * u = (x + 1/2) / 2^32, of the 32-bit word x = word k % 4 of Philox4x32-10
 * (Salmon et al., SC'11) at counter (k / 4, i, 0, 0) and key (seed low 32 bits,
 * seed high 32 bits). Draws depend only on (seed, i, k).
 *   src, rcv, out, ws, stream: as for ism_simulate (out is [n_src][n_rcv][nS]);
 *   ws of at least ism_diffuse_workspace_size() bytes.
 * Errors: ISM_E_INVALID_ARG for t_diff or t60 out of range, otherwise as
 * ism_simulate, all before any launch. Asynchronous. */
int ism_simulate_diffuse(const ism_room *room, double t_diff, double t60, uint64_t seed, const float *src,
                         int n_src, const float *rcv, int n_rcv, int precision, float *out, void *ws,
                         size_t ws_bytes, void *stream);

/* ism_simulate_diffuse, plus the events of ism_simulate_timed recorded around
 * the tap accumulation kernel of the ISM part. Same arguments, checks and
 * results as ism_simulate_diffuse. */
int ism_simulate_diffuse_timed(const ism_room *room, double t_diff, double t60, uint64_t seed, const float *src,
                               int n_src, const float *rcv, int n_rcv, int precision, float *out, void *ws,
                               size_t ws_bytes, void *stream, void *ev_start, void *ev_stop);

/* ism_simulate_diffuse with directional receivers (Sec. 4; pattern and
 * orientation as for ism_simulate_polar). The ISM part is the directional RIR
 * that ism_simulate_polar gives for T_max = t_diff; the tail is drawn as for
 * ism_simulate_diffuse, at the level A estimated from that directional ISM
 * part (reading: the diffuse field itself is not directional).
 *   orient, pattern: as for ism_simulate_polar; the other arguments, the
 *   workspace (ism_diffuse_workspace_size) and the errors as for
 *   ism_simulate_diffuse, all checked before any launch. Asynchronous. */
int ism_simulate_diffuse_polar(const ism_room *room, double t_diff, double t60, uint64_t seed, const float *src,
                               int n_src, const float *rcv, int n_rcv, const float *orient, double pattern,
                               int precision, float *out, void *ws, size_t ws_bytes, void *stream);

/* ---- Moving source (Sec. 3.4) -------------------------------------------------- */

/* Filters a source signal through the RIRs of a trajectory by overlap-add:
 * x is cut into n_pos segments of seg_len = ceil(n_x / n_pos) samples
 * (segment p = samples [p seg_len, min((p+1) seg_len, n_x))), segment p is
 * convolved with the RIR of trajectory point p to each microphone and added
 * at its offset, i.e. y[m][n] = sum_k x[n - k] rir[p(n - k)][m][k] with
 * p(i) = floor(i / seg_len).
 *   x    device float32 [n_x];
 *   rir  device float32 [n_pos][n_mic][n_rir] (the output layout of
 *        ism_simulate with the trajectory points as sources and the
 *        microphones as receivers);
 *   y    device float32 [n_mic][n_x + n_rir - 1], fully overwritten.
 * 1 <= n_pos <= n_x, n_mic <= 65535, n_rir >= 1. Allocates nothing; the sum
 * order is fixed (bitwise reproducible). Asynchronous on stream.
 * Errors: ISM_E_INVALID_ARG, ISM_E_TOO_LARGE before any launch. */
int ism_filter_trajectory(const float *x, int n_x, const float *rir, int n_pos, int n_mic, int n_rir, float *y,
                          void *stream);

/* Filter methods of ism_filter_trajectory_ex. */
enum {
  ISM_FILTER_AUTO = 0,   /* FFT for RIRs of 1024 taps and more (when every input
                            block of the FFT path touches at most 4 segments),
                            direct otherwise                                   */
  ISM_FILTER_DIRECT = 1, /* the direct sum of ism_filter_trajectory            */
  ISM_FILTER_FFT = 2     /* partitioned FFT convolution (the paper's batched
                            FFTs, Sec. 3.4)                                     */
};

/* Device workspace (bytes) of ism_filter_trajectory_ex for these sizes and
 * method: 0 for the direct sum; for the FFT path the spectra of every RIR
 * partition (about twice the RIR data), of the input blocks and of the
 * output blocks. ISM_E_UNSUPPORTED for ISM_FILTER_FFT when one block of the
 * signal would touch more than 16 segments (segments much shorter than the
 * block); errors otherwise as for ism_filter_trajectory. */
int ism_filter_workspace_size(int n_x, int n_pos, int n_mic, int n_rir, int method, size_t *bytes);

/* ism_filter_trajectory (same x, rir, y layouts and result definition) with a
 * choice of method. The FFT path cuts x into blocks of B samples (B = 4096
 * for RIRs of 16384 taps and more, else a quarter of the next power of two of
 * n_rir, at least 256), splits each block at segment boundaries, multiplies
 * the spectra of the pieces with those of the B-tap partitions of their
 * segment's RIR (2B-point real FP32 transforms, computed as B-point complex
 * Stockham transforms in LDS), adds the
 * products of each output block in a fixed order and overlap-adds the
 * inverse transforms: results are bitwise reproducible and agree with the
 * direct sum to FP32 transform rounding. Its cost per output sample grows
 * with log B and n_rir / B instead of n_rir.
 *   ws: ism_filter_workspace_size() bytes (may be NULL for the direct sum).
 * Errors: as for ism_filter_trajectory, ISM_E_WORKSPACE, ISM_E_UNSUPPORTED;
 * all before any launch. Asynchronous on stream. */
int ism_filter_trajectory_ex(const float *x, int n_x, const float *rir, int n_pos, int n_mic, int n_rir, int method,
                             float *y, void *ws, size_t ws_bytes, void *stream);

/* ---- Batches of rooms --------------------------------------------------------- */

/* One job of a batch: one room with its own sources, receivers and output. */
typedef struct {
  ism_room room;
  const float *src; /* device float32 [n_src][3] */
  int n_src;
  const float *rcv; /* device float32 [n_rcv][3] */
  int n_rcv;
  float *out;       /* device float32 [n_src][n_rcv][nS(room)], caller-owned, overwritten */
  const float *orient; /* NULL: omnidirectional receivers; else device float32 [n_rcv][3]
                          receiver orientations, as for ism_simulate_polar      */
  double pattern;   /* polar pattern a in [0, 1] when orient is set (ignored otherwise) */
} ism_job;

/* Host-side record of a prepared batch, filled by ism_batch_prepare and read by
 * ism_batch_run. Caller-owned plain memory; its contents are private. */
typedef struct {
  uint64_t opaque[40];
} ism_batch;

/* Device workspace (bytes) for a batch of n_jobs jobs (host array), for
 * ism_batch_prepare and for ism_simulate_batch. */
int ism_batch_workspace_size(const ism_job *jobs, int n_jobs, int precision, size_t *bytes);

/* Plans a batch on the host (every job checked as in ism_simulate; the first
 * failing job's status is returned), uploads the job and work tables into ws
 * (a blocking host-to-device copy on stream), and fills *batch. After it
 * returns, jobs may be freed; the device pointers inside them must stay valid
 * for every ism_batch_run of this batch. Work items of all jobs are ordered by
 * decreasing estimated work, so rooms of very different sizes share one launch
 * per window length (Sec. 3 discusses why uneven image counts made the paper
 * process one room per call). */
int ism_batch_prepare(const ism_job *jobs, int n_jobs, int precision, void *ws, size_t ws_bytes, void *stream,
                      ism_batch *batch);

/* Simulates every job of a prepared batch on stream: kernel launches only (no
 * host-device copies, no allocation), so it can be captured in a HIP graph and
 * replayed. Work items are sized from the batch's total work: each job is
 * planned as a single call with item_taps = t = min(B, max(min_item_taps,
 * batch taps / balance_items)) of its class, B the tuned largest batch item
 * of the class, or, for a batch of less than t taps per resident wave, with
 * its taps over the resident waves (at least 1e4); the schedule's item_taps
 * replaces both when given. A
 * job's result therefore agrees within rounding (<= 1e-6 of the RIR peak)
 * with the job alone and with ism_simulate; it is bitwise that of
 * ism_simulate_ex with the same item_taps, and a batch of one job (of fewer
 * than B x balance_items estimated taps) is bitwise ism_simulate_ex with
 * tail_rounds = 0. */
int ism_batch_run(const ism_batch *batch, void *stream);

/* ism_batch_run that also records the caller's HIP events ev_start before the
 * first and ev_stop after the last tap-accumulation launch (either may be NULL). */
int ism_batch_run_timed(const ism_batch *batch, void *stream, void *ev_start, void *ev_stop);

/* ism_batch_workspace_size and ism_batch_prepare with an explicit work
 * schedule for every job (tail_rounds is ignored: batches do not taper). */
int ism_batch_workspace_size_ex(const ism_job *jobs, int n_jobs, int precision, const ism_schedule *sched,
                                size_t *bytes);
int ism_batch_prepare_ex(const ism_job *jobs, int n_jobs, int precision, const ism_schedule *sched, void *ws,
                         size_t ws_bytes, void *stream, ism_batch *batch);

/* Many rooms in one call, positions in host memory (the batched form of
 * ism_simulate_host; Sec. 3 on rooms of uneven image counts). Here src, rcv
 * and orient of each job are HOST float32 arrays ([n_src][3], [n_rcv][3],
 * [n_rcv][3] or NULL); out stays a device array. Every job is checked as by
 * ism_check_room / ism_check_positions (and its pattern) before any launch:
 * the first failing job's status is returned and no output is touched. The
 * positions are copied into ws with the batch tables (one host-to-device copy
 * on stream, complete when the call returns), then the kernels of
 * ism_batch_run are launched asynchronously. ws: ism_batch_workspace_size()
 * bytes of the same jobs. Results are those of ism_batch_run. */
int ism_simulate_batch(const ism_job *jobs, int n_jobs, int precision, void *ws, size_t ws_bytes, void *stream);

/* ---- Without allocation --------------------------------------------------------- */

/* Size of the device array ism_simulate_noalloc uses as its workspace: 64 MiB
 * (the 32-receiver, 0.7 s, 16 kHz room of 4 x 5 x 3 m needs 38 MiB). */
#define ISM_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)

/* ism_simulate for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): no
 * workspace argument; the call uses a fixed array of
 * ISM_NOALLOC_SCRATCH_BYTES in the library's device memory instead (one per
 * GPU, held until the process ends, looked up once per device). It calls no
 * allocating routine. Same arguments (device positions), results and checks as
 * ism_simulate; a call whose ism_workspace_size exceeds the array returns
 * ISM_E_TOO_LARGE before any launch. Every call on a GPU shares that GPU's
 * array, so calls that overlap on one GPU (other streams, other host threads)
 * race: order them, e.g. on one stream. Nothing in the array needs clearing
 * between calls (every byte read is written earlier in the same call). */
int ism_simulate_noalloc(const ism_room *room, const float *src, int n_src, const float *rcv, int n_rcv,
                         int precision, float *out, void *stream);

#ifdef __cplusplus
}
#endif
#endif
