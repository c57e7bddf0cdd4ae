// C ABI of libism.so (declared in include/ism.h): argument checks, FP64 host
// planning, workspace layout and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <memory>
#include <thread>
#include <vector>

#include "ism.h"
#include "ism_debug.h"
#include "ism_internal.h"
#include "ism_tuning.h"

namespace ism {
int launch_tables(const RoomArgs &ra, const float *src, const float *rcv, const float *orient, AxisEntry *tab,
                  AxisOrigin *origin, int *valid, int n_rir, hipStream_t st);
int launch_accumulate(int wt, bool gen, bool half, bool lut, bool polar, const RoomArgs &ra, const PlanArgs &pa,
                      uint32_t n_items, const AxisEntry *tab, const AxisOrigin *origin, const int *valid, float *out,
                      float *part, float *marg, const float *wc, hipStream_t st);
int launch_reduce(const RoomArgs &ra, const PlanArgs &pa, int n_rir, const float *part, const float *marg,
                  float *out, hipStream_t st);
bool supported_window(int wt, bool gen);
int launch_window_consts(float W, int wt, bool half, float *wc, hipStream_t st);
int launch_dump(int wt, const RoomArgs &ra, const PlanArgs &pa, uint32_t n_items, const AxisEntry *tab,
                const AxisOrigin *origin, const int *valid, DumpArgs dump, hipStream_t st);
int launch_batch(const JobDev *jobs, int n_jobs, bool any_gen, const BatchRir *rirs, uint32_t n_rir,
                 const BatchItem *items, const uint32_t *class_first, const uint32_t *class_count,
                 const uint32_t *class_grid, const int *class_wt, const int *class_gen, int n_classes, bool half, bool lut, bool polar,
                 const BatchReduce *red, uint32_t n_red, uint32_t n_red_split, bool long_runs, AxisEntry *tab,
                 AxisOrigin *origin, int *valid, float *part, float *marg, uint32_t *queue, hipStream_t st,
                 hipEvent_t ev_start, hipEvent_t ev_stop);
int launch_diffuse(const float *ism, int k_diff, float *out, int n_samples, int n_rir, double fs, double t_diff,
                   double t60, uint64_t seed, hipStream_t st);
int launch_filter(const float *x, int n_x, const float *rir, int n_pos, int n_mic, int n_rir, float *y,
                  hipStream_t st);
bool fft_plan(int n_x, int n_pos, int n_mic, int n_rir, int max_pieces, FftPlan &f);
int launch_filter_fft(const float *x, int n_x, const float *rir, int n_pos, int n_mic, int n_rir, float *y,
                      const FftPlan &f, void *ws, hipStream_t st);
}  // namespace ism

using namespace ism;

namespace {

constexpr double kPi = 3.14159265358979323846;

// A failed HIP runtime call: names it on stderr and maps it to ISM_E_DEVICE.
int device_error(const char *where, hipError_t e) {
  fprintf(stderr, "libism: %s: %s\n", where, hipGetErrorString(e));
  return ISM_E_DEVICE;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int lattice_lo(int N) { return -(N / 2); }       // ceil(-N/2)
int lattice_hi(int N) { return (N + 1) / 2; }    // ceil(N/2), exclusive

void split(double v, float &hi, float &lo) {
  hi = (float)v;
  lo = (float)(v - (double)hi);
}

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// Window length W = t_w * fs in samples when it is an even integer (within
// 1e-9 relative); 0 otherwise.
int even_window(const ism_room &r) {
  const double W = r.t_w * r.fs;
  const double k = std::nearbyint(W);
  if (std::fabs(W - k) > 1e-9 * W) return 0;
  const long iw = (long)k;
  if (iw < 2 || (iw & 1)) return 0;
  return (int)iw;
}

// Kernel class of a window of W = t_w fs samples (Eq. (6)): exact mode for an
// even integer W in {32, 64, 96, 128} (cap WT = W), else general mode with
// the cap WT = the next multiple of 32 (at least 32, at most MAX_WINDOW).
int window_class(const ism_room &r, int &wt, bool &gen, double &W) {
  W = r.t_w * r.fs;
  const int ev = even_window(r);
  if (ev == 32 || ev == 64 || ev == 96 || ev == 128) {
    wt = ev;
    gen = false;
    W = ev;
    return ISM_OK;
  }
  if (W > MAX_WINDOW * (1.0 + 1e-9)) return ISM_E_TOO_LARGE;
  W = std::min(W, (double)MAX_WINDOW);
  wt = std::max(32, 32 * (int)std::ceil(W / 32.0 - 1e-9));
  gen = true;
  return ISM_OK;
}

struct Plan {
  RoomArgs ra;
  PlanArgs pa;
  double tile_taps[MAX_TILES];  // estimated taps of each tile's image shell
  double total_taps;            // over all RIRs
  int wt;     // window cap WT (kernel layout)
  bool gen;   // general-mode window (per-call tap constants)
  double win; // W = t_w fs
  bool half;
  bool lut;  // table taps (Eq. (9)); FP32 arithmetic otherwise
  int n_rir;
  uint32_t n_items;
  bool any_split;
  size_t off_valid, off_origin, off_tab, off_part, off_marg, off_wc, off_pos, ws_bytes;
};

// Work-item size in estimated taps. A launch should hold about balance_items
// items (some eight per resident wave) so that the largest-first order keeps
// every CU busy to the end; small calls keep items of min_item_taps. Both come
// from the tuning table (ism_tuning.h) for the window and precision unless the
// call's schedule (ism_schedule) replaces them.
constexpr double kMinItemTaps = 1.2e5;
constexpr double kBalanceItems = 49152.0;
double item_target(double total_taps, int wt, bool half, int64_t n_samples, const ism_schedule *sc) {
  double min_taps = kMinItemTaps, balance = kBalanceItems;
  for (const ItemTuning &t : kItemTuning)
    if (t.wt == wt && t.half == (half ? 1 : 0) && n_samples <= t.ns_max) {
      min_taps = t.min_item_taps;
      balance = t.balance_items;
      break;
    }
  if (sc && sc->min_item_taps > 0.0) min_taps = std::max(1e3, sc->min_item_taps);
  if (sc && sc->balance_items > 0.0) balance = std::max(1.0, sc->balance_items);
  return std::max(min_taps, total_taps / balance);
}

// Largest work item of a batch job (the tuned value of its window class and
// precision; classes the tuner has no batch workload for take kBatchItemTaps).
constexpr double kBatchItemTaps = 2.5e5;
double batch_item_taps(int wt, bool half) {
  for (const BatchTuning &t : kBatchTuning)
    if (t.wt == wt && t.half == (half ? 1 : 0)) return t.item_taps;
  return kBatchItemTaps;
}

// Waves of the accumulate kernel resident on the device at once (256 CUs x
// 4 SIMDs x the waves per SIMD the kernel is built for), and the default
// rounds of them over which a single call tapers its tail.
constexpr double kResidentWaves = 256.0 * 4.0 * kAccWavesPerSimd;
constexpr double kTailRounds = 1.0;

// Small calls: a call whose work does not give every resident wave an item
// of the tuned size is spread over them instead, total / resident waves per
// item but at least kSmallItemTaps, which is also the taper's lowest item (a
// single 4800-sample RIR, 1e7 taps, measured 27 us per accumulate launch with
// 1e4-tap items against 35 us with the earlier floor of an eighth of 1.2e5
// and 103 us with 1.2e5-tap items).
constexpr double kSmallItemTaps = 1e4;
double small_call_floor(double total_taps) { return std::max(kSmallItemTaps, total_taps / kResidentWaves); }

bool valid_schedule(const ism_schedule *sc) {
  if (!sc) return true;
  const double v[5] = {sc->item_taps, sc->min_item_taps, sc->balance_items, sc->tail_rounds, sc->batch_waves};
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return sc->item_taps >= 0.0 && sc->min_item_taps >= 0.0 && sc->balance_items >= 0.0 && sc->batch_waves >= 0.0 &&
         sc->batch_waves <= 16.0;
}

// sched: the call's schedule (null = the tuned default).
// taper: cut the items dispatched last (single calls; a batch's tail is the
// largest-first order over all its jobs' items instead).
int make_plan(const ism_room *r, int n_src, int n_rcv, int precision, Plan &p, const ism_schedule *sched = nullptr,
              bool taper = true) {
  int st = ism_check_room(r);
  if (st != ISM_OK) return st;
  if (!valid_schedule(sched)) return ISM_E_INVALID_ARG;
  if (n_src < 1 || n_rcv < 1) return ISM_E_INVALID_ARG;
  if ((int64_t)n_src * n_rcv > ISM_MAX_PAIRS) return ISM_E_TOO_LARGE;
  if (precision != ISM_FP32 && precision != ISM_FP16 && precision != ISM_FP32_LUT)
    return precision == ISM_BF16 ? ISM_E_UNSUPPORTED : ISM_E_INVALID_ARG;
  p.half = precision == ISM_FP16;
  p.lut = precision == ISM_FP32_LUT;
  st = window_class(*r, p.wt, p.gen, p.win);
  if (st != ISM_OK) return st;
  // table taps are built for the exact windows only
  if (!supported_window(p.wt, p.gen) || (p.gen && p.lut)) return ISM_E_UNSUPPORTED;
  const int64_t nS = ism_n_samples(r->t_max, r->fs);
  const double W = (double)p.wt;
  const double q = r->fs / r->c;

  RoomArgs &ra = p.ra;
  std::memset(&ra, 0, sizeof(ra));
  // table axes: room axes by decreasing length (stable), shortest innermost
  int perm[3] = {0, 1, 2};
  std::stable_sort(perm, perm + 3, [&](int a, int b) { return r->room[a] > r->room[b]; });
  int off = 0;
  for (int k = 0; k < 3; ++k) {
    const int a = perm[k];
    ra.perm[k] = a;
    split(r->room[a], ra.L_hi[k], ra.L_lo[k]);
    ra.lo[k] = lattice_lo(r->n_img[a]);
    ra.N[k] = r->n_img[a];
    ra.off[k] = off;
    off += r->n_img[a];
    ra.period[k] = (float)(2.0 * r->room[a] * q);
    ra.inv_period[k] = (float)(1.0 / (2.0 * r->room[a] * q));
    split(r->beta[2 * a], ra.beta[2 * k], ra.beta_lo[2 * k]);
    split(r->beta[2 * a + 1], ra.beta[2 * k + 1], ra.beta_lo[2 * k + 1]);
  }
  ra.n_tab = off;
  split(q, ra.q_hi, ra.q_lo);
  ra.kappa = (float)(r->fs / (4.0 * kPi * r->c));
  ra.half_w = (float)(W / 2.0);
  ra.win_hw = (float)(p.win / 2.0);
  ra.inv_win = (float)(1.0 / p.win);
  ra.gen = p.gen ? 1 : 0;
  ra.n_samples = (int)nS;
  ra.k_end = (int)nS + p.wt / 2 - 1;
  ra.n_src = n_src;
  ra.n_rcv = n_rcv;

  // Work split: tile t owns the images with k0 in [t TILE, min((t+1) TILE, k_end));
  // its estimated taps are the owned shell volume over the image density
  // 1 / (Lx Ly Lz) (one image per mirrored room copy), times W.
  p.n_rir = n_src * n_rcv;
  PlanArgs &pa = p.pa;
  std::memset(&pa, 0, sizeof(pa));
  pa.n_tiles = (ra.k_end + TILE - 1) / TILE;
  if (pa.n_tiles > MAX_TILES) return ISM_E_TOO_LARGE;
  pa.n_rir = p.n_rir;
  const double cell = r->room[0] * r->room[1] * r->room[2] * q * q * q;
  const double lattice = (double)r->n_img[0] * r->n_img[1] * r->n_img[2];
  p.total_taps = 0.0;
  for (int t = 0; t < pa.n_tiles; ++t) {
    const double x0 = (double)t * TILE, x1 = std::min((double)(t + 1) * TILE, (double)ra.k_end);
    const double imgs = std::min(4.0 / 3.0 * kPi * (x1 * x1 * x1 - x0 * x0 * x0) / cell, lattice);
    p.tile_taps[t] = imgs * W;
    p.total_taps += p.tile_taps[t] * p.n_rir;
  }
  // an explicit item size is used as given
  const bool fixed = sched && sched->item_taps > 0.0;
  double target = fixed ? std::max(1e3, sched->item_taps) : item_target(p.total_taps, p.wt, p.half, nS, sched);
  if (!fixed && p.total_taps < kResidentWaves * target) target = std::min(target, small_call_floor(p.total_taps));
  // Tail taper: tiles are dispatched last first, and the items of a tile
  // dispatched when the work left (this tile included) is below tail_rounds
  // rounds of the resident waves are cut to that work over tail_rounds x the
  // resident waves, down to target / 8 but not below kSmallItemTaps, so the
  // last waves of a launch finish close together instead of one full-size
  // item after another.
  const double tail_rounds =
      (fixed || !taper) ? 0.0 : (sched && sched->tail_rounds >= 0.0 ? sched->tail_rounds : kTailRounds);
  const double floor_taps = std::min(target, std::max(kSmallItemTaps, target / 8.0));
  p.any_split = false;
  double rem = p.total_taps;
  for (int pos = 0; pos < pa.n_tiles; ++pos) {
    const int t = pa.n_tiles - 1 - pos;
    const double taps = p.tile_taps[t];
    double tt = target;
    if (tail_rounds > 0.0) tt = std::max(floor_taps, std::min(target, rem / (tail_rounds * kResidentWaves)));
    int ch = (int)std::ceil(taps / tt);
    ch = std::max(1, std::min(ch, MAX_CHUNKS));
    pa.chunks[t] = (uint8_t)ch;
    if (ch > 1) p.any_split = true;
    rem -= taps * p.n_rir;
  }
  uint64_t acc = 0;
  for (int pos = 0; pos < pa.n_tiles; ++pos) {
    if (pos % PLAN_BLK == 0) pa.first_blk[pos / PLAN_BLK] = (uint32_t)acc;
    acc += (uint64_t)p.n_rir * pa.chunks[pa.n_tiles - 1 - pos];
    if (acc > 0x7fffffffULL) return ISM_E_TOO_LARGE;
  }
  pa.first_blk[(pa.n_tiles + PLAN_BLK - 1) / PLAN_BLK] = (uint32_t)acc;
  p.n_items = (uint32_t)acc;

  p.off_valid = 0;
  p.off_origin = align_up(sizeof(int) * (size_t)p.n_rir);
  p.off_tab = align_up(p.off_origin + sizeof(AxisOrigin) * (size_t)p.n_rir);
  p.off_part = align_up(p.off_tab + sizeof(AxisEntry) * (size_t)p.n_rir * ra.n_tab);
  p.off_marg = align_up(p.off_part + (p.any_split ? sizeof(float) * (size_t)p.n_items * TILE : 0));
  // general-mode window constants
  p.off_wc = align_up(p.off_marg + sizeof(float) * (size_t)p.n_items * p.wt);
  // host-position calls copy src then rcv here
  p.off_pos = align_up(p.off_wc + (p.gen ? sizeof(float) * WC_STRIDE * (size_t)p.wt : 0));
  p.ws_bytes = align_up(p.off_pos + sizeof(float) * 3 * ((size_t)n_src + (size_t)n_rcv));
  return ISM_OK;
}

}  // namespace

extern "C" {

const char *ism_status_string(int status) {
  switch (status) {
    case ISM_OK: return "ok";
    case ISM_E_INVALID_ARG: return "invalid argument";
    case ISM_E_INFEASIBLE_T60: return "T60 infeasible by Sabine's formula (absorption > 1)";
    case ISM_E_OUT_OF_ROOM: return "position not strictly inside the room";
    case ISM_E_WORKSPACE: return "workspace missing or too small";
    case ISM_E_DEVICE: return "HIP device error";
    case ISM_E_TOO_LARGE: return "problem exceeds a library limit";
    case ISM_E_UNSUPPORTED: return "request not supported by the library";
    default: return "unknown status";
  }
}

int ism_abi_version(void) { return ISM_ABI_VERSION; }

int ism_beta_from_t60(const double room[3], double t60, double beta_out[6]) {
  if (!room || !beta_out) return ISM_E_INVALID_ARG;
  if (!finite_pos(room[0]) || !finite_pos(room[1]) || !finite_pos(room[2]) || !finite_pos(t60)) return ISM_E_INVALID_ARG;
  const double V = room[0] * room[1] * room[2];
  const double S = 2.0 * (room[0] * room[1] + room[0] * room[2] + room[1] * room[2]);
  const double alpha = 0.161 * V / (S * t60);  // Eq. (7) with one alpha for all walls
  if (alpha > 1.0) return ISM_E_INFEASIBLE_T60;
  const double b = std::sqrt(1.0 - alpha);  // alpha = 1 - beta^2
  for (int i = 0; i < 6; ++i) beta_out[i] = b;
  return ISM_OK;
}

int ism_n_img_for_time(const double room[3], double c, double t, int n_out[3]) {
  if (!room || !n_out) return ISM_E_INVALID_ARG;
  if (!finite_pos(c) || !finite_pos(t)) return ISM_E_INVALID_ARG;
  for (int a = 0; a < 3; ++a) {
    if (!finite_pos(room[a])) return ISM_E_INVALID_ARG;
    const double k = std::ceil(c * t / (2.0 * room[a]));
    if (k > (ISM_MAX_N_IMG - 2) / 4) return ISM_E_TOO_LARGE;
    n_out[a] = 4 * (int)k + 2;
  }
  return ISM_OK;
}

int ism_time_for_attenuation(double t60, double att_db, double *t_out) {
  if (!t_out || !finite_pos(t60) || !std::isfinite(att_db) || att_db < 0.0) return ISM_E_INVALID_ARG;
  *t_out = t60 * att_db / 60.0;
  return ISM_OK;
}

int64_t ism_n_samples(double t_max, double fs) {
  if (!finite_pos(t_max) || !finite_pos(fs)) return -1;
  const double v = t_max * fs;
  if (v > 9.0e15) return -1;
  const double r = std::nearbyint(v);
  if (std::fabs(v - r) <= 1e-9 * v) return (int64_t)r;
  return (int64_t)std::ceil(v);
}

int ism_check_room(const ism_room *r) {
  if (!r) return ISM_E_INVALID_ARG;
  for (int a = 0; a < 3; ++a) {
    if (!finite_pos(r->room[a])) return ISM_E_INVALID_ARG;
    if (r->n_img[a] < 1) return ISM_E_INVALID_ARG;
    if (r->n_img[a] > ISM_MAX_N_IMG) return ISM_E_TOO_LARGE;
  }
  for (int i = 0; i < 6; ++i)
    if (!std::isfinite(r->beta[i]) || std::fabs(r->beta[i]) > 1.0) return ISM_E_INVALID_ARG;
  if (!finite_pos(r->c) || !finite_pos(r->fs) || !finite_pos(r->t_max) || !finite_pos(r->t_w)) return ISM_E_INVALID_ARG;
  const int64_t nS = ism_n_samples(r->t_max, r->fs);
  if (nS < 1) return ISM_E_INVALID_ARG;
  if (nS > ISM_MAX_SAMPLES) return ISM_E_TOO_LARGE;
  return ISM_OK;
}

int ism_check_positions(const ism_room *room, const float *src, int n_src, const float *rcv, int n_rcv) {
  int st = ism_check_room(room);
  if (st != ISM_OK) return st;
  if (!src || !rcv || n_src < 1 || n_rcv < 1) return ISM_E_INVALID_ARG;
  auto inside = [&](const float *p) {
    for (int a = 0; a < 3; ++a)
      if (!(std::isfinite(p[a]) && p[a] > 0.0f && (double)p[a] < room->room[a])) return false;
    return true;
  };
  for (int i = 0; i < n_src; ++i)
    if (!inside(src + 3 * i)) return ISM_E_OUT_OF_ROOM;
  for (int i = 0; i < n_rcv; ++i)
    if (!inside(rcv + 3 * i)) return ISM_E_OUT_OF_ROOM;
  for (int i = 0; i < n_src; ++i)
    for (int j = 0; j < n_rcv; ++j)
      if (src[3 * i] == rcv[3 * j] && src[3 * i + 1] == rcv[3 * j + 1] && src[3 * i + 2] == rcv[3 * j + 2])
        return ISM_E_INVALID_ARG;
  return ISM_OK;
}

int ism_count_taps(const ism_room *room, const float *src, int n_src, const float *rcv, int n_rcv,
                   int64_t *taps_out) {
  if (!taps_out) return ISM_E_INVALID_ARG;
  int st = ism_check_room(room);
  if (st != ISM_OK) return st;
  if (!src || !rcv || n_src < 1 || n_rcv < 1) return ISM_E_INVALID_ARG;
  const double W = room->t_w * room->fs, hw = W / 2.0;
  const double q = room->fs / room->c;
  const int64_t nS = ism_n_samples(room->t_max, room->fs);
  const int n_pairs = n_src * n_rcv;
  std::atomic<int> next{0};
  std::atomic<int64_t> total{0};
  auto worker = [&]() {
    for (;;) {
      const int pidx = next.fetch_add(1);
      if (pidx >= n_pairs) return;
      const float *s = src + 3 * (pidx / n_rcv);
      const float *r = rcv + 3 * (pidx % n_rcv);
      // per-axis squared displacements (samples^2) of every lattice index
      std::vector<double> d2[3];
      for (int a = 0; a < 3; ++a) {
        for (int n = lattice_lo(room->n_img[a]); n < lattice_hi(room->n_img[a]); ++n) {
          const double coord = (n % 2 == 0) ? n * room->room[a] + s[a] : (n + 1) * room->room[a] - s[a];
          const double dd = (coord - r[a]) * q;
          d2[a].push_back(dd * dd);
        }
      }
      int64_t cnt = 0;
      for (double dx : d2[0])
        for (double dy : d2[1])
          for (double dz : d2[2]) {
            const double x = std::sqrt(dx + dy + dz);
            int64_t first = (int64_t)std::floor(x - hw) + 1;
            int64_t last = (int64_t)std::ceil(x + hw) - 1;
            if (first < 0) first = 0;
            if (last > nS - 1) last = nS - 1;
            if (last >= first) cnt += last - first + 1;
          }
      total.fetch_add(cnt);
    }
  };
  const unsigned hc = std::max(1u, std::min(std::thread::hardware_concurrency(), (unsigned)n_pairs));
  std::vector<std::thread> th;
  for (unsigned i = 1; i < hc; ++i) th.emplace_back(worker);
  worker();
  for (auto &t : th) t.join();
  *taps_out = total.load();
  return ISM_OK;
}

int ism_workspace_size_ex(const ism_room *room, int n_src, int n_rcv, int precision, const ism_schedule *sched,
                          size_t *bytes) {
  if (!bytes) return ISM_E_INVALID_ARG;
  Plan p;
  const int st = make_plan(room, n_src, n_rcv, precision, p, sched);
  if (st != ISM_OK) return st;
  *bytes = p.ws_bytes;
  return ISM_OK;
}

int ism_workspace_size(const ism_room *room, int n_src, int n_rcv, int precision, size_t *bytes) {
  return ism_workspace_size_ex(room, n_src, n_rcv, precision, nullptr, bytes);
}

int ism_simulate(const ism_room *room, const float *src, int n_src, const float *rcv, int n_rcv, int precision,
                 float *out, void *ws, size_t ws_bytes, void *stream) {
  return ism_simulate_ex(room, src, n_src, rcv, n_rcv, precision, nullptr, out, ws, ws_bytes, stream, nullptr,
                         nullptr);
}

// Launches the ISM kernels of a plan: tables, taps, completion of the tiles.
// ws holds at least p.ws_bytes; out is device [n_rir][nS].
// orient: device [n_rcv][3] receiver orientations for a polar call (p.ra.dir_a,
// dir_b set), else null.
static int run_plan(const Plan &p, const float *src, const float *rcv, float *out, void *ws, void *stream,
                    void *ev_start, void *ev_stop, const float *orient = nullptr) {
  hipStream_t s = (hipStream_t)stream;
  char *w = (char *)ws;
  int *valid = (int *)(w + p.off_valid);
  AxisOrigin *origin = (AxisOrigin *)(w + p.off_origin);
  AxisEntry *tab = (AxisEntry *)(w + p.off_tab);
  float *part = p.any_split ? (float *)(w + p.off_part) : nullptr;
  float *marg = (float *)(w + p.off_marg);
  float *wc = p.gen ? (float *)(w + p.off_wc) : nullptr;
  if (launch_tables(p.ra, src, rcv, orient, tab, origin, valid, p.n_rir, s) != 0) return ISM_E_DEVICE;
  if (wc && launch_window_consts((float)p.win, p.wt, p.half, wc, s) != 0) return ISM_E_DEVICE;
  if (ev_start && hipEventRecord((hipEvent_t)ev_start, s) != hipSuccess) return ISM_E_DEVICE;
  if (launch_accumulate(p.wt, p.gen, p.half, p.lut, orient != nullptr, p.ra, p.pa, p.n_items, tab, origin, valid, out,
                        part, marg, wc, s) != 0)
    return ISM_E_DEVICE;
  if (ev_stop && hipEventRecord((hipEvent_t)ev_stop, s) != hipSuccess) return ISM_E_DEVICE;
  // split tiles and the margins between neighbouring tiles
  if ((p.any_split || p.pa.n_tiles > 1) && launch_reduce(p.ra, p.pa, p.n_rir, part, marg, out, s) != 0)
    return ISM_E_DEVICE;
  return ISM_OK;
}

int ism_simulate_ex(const ism_room *room, const float *src, int n_src, const float *rcv, int n_rcv, int precision,
                    const ism_schedule *sched, float *out, void *ws, size_t ws_bytes, void *stream, void *ev_start,
                    void *ev_stop) {
  Plan p;
  const int st = make_plan(room, n_src, n_rcv, precision, p, sched);
  if (st != ISM_OK) return st;
  if (!src || !rcv || !out) return ISM_E_INVALID_ARG;
  if (!ws || ws_bytes < p.ws_bytes) return ISM_E_WORKSPACE;
  return run_plan(p, src, rcv, out, ws, stream, ev_start, ev_stop);
}

int ism_simulate_timed(const ism_room *room, const float *src, int n_src, const float *rcv, int n_rcv,
                       int precision, float *out, void *ws, size_t ws_bytes, void *stream, void *ev_start,
                       void *ev_stop) {
  return ism_simulate_ex(room, src, n_src, rcv, n_rcv, precision, nullptr, out, ws, ws_bytes, stream, ev_start,
                         ev_stop);
}

int ism_simulate_host(const ism_room *room, const float *src, int n_src, const float *rcv, int n_rcv,
                      int precision, float *out, void *ws, size_t ws_bytes, void *stream) {
  Plan p;
  int st = make_plan(room, n_src, n_rcv, precision, p);
  if (st != ISM_OK) return st;
  if (!src || !rcv || !out) return ISM_E_INVALID_ARG;
  st = ism_check_positions(room, src, n_src, rcv, n_rcv);
  if (st != ISM_OK) return st;
  if (!ws || ws_bytes < p.ws_bytes) return ISM_E_WORKSPACE;
  // positions into the workspace: pageable host memory, so the call returns
  // once the host arrays have been read
  hipStream_t s = (hipStream_t)stream;
  float *pos = (float *)((char *)ws + p.off_pos);
  if (hipMemcpyAsync(pos, src, sizeof(float) * 3 * (size_t)n_src, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(pos + 3 * (size_t)n_src, rcv, sizeof(float) * 3 * (size_t)n_rcv, hipMemcpyHostToDevice, s) !=
          hipSuccess)
    return ISM_E_DEVICE;
  return run_plan(p, pos, pos + 3 * (size_t)n_src, out, ws, stream, nullptr, nullptr);
}

int ism_debug_enumerate(const ism_room *room, const float *src, int n_src, const float *rcv, int n_rcv,
                        const ism_schedule *sched, void *records, uint32_t cap, uint32_t *count, void *ws,
                        size_t ws_bytes, void *stream) {
  Plan p;
  const int st = make_plan(room, n_src, n_rcv, ISM_FP32, p, sched);
  if (st != ISM_OK) return st;
  if (!src || !rcv || !count || (cap > 0 && !records)) return ISM_E_INVALID_ARG;
  if (!ws || ws_bytes < p.ws_bytes) return ISM_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  char *w = (char *)ws;
  int *valid = (int *)(w + p.off_valid);
  AxisOrigin *origin = (AxisOrigin *)(w + p.off_origin);
  AxisEntry *tab = (AxisEntry *)(w + p.off_tab);
  if (launch_tables(p.ra, src, rcv, nullptr, tab, origin, valid, p.n_rir, s) != 0) {
    fprintf(stderr, "ism_debug_enumerate: tables launch failed\n");
    return ISM_E_DEVICE;
  }
  DumpArgs d{(DumpRec *)records, count, cap};
  if (launch_dump(p.wt, p.ra, p.pa, p.n_items, tab, origin, valid, d, s) != 0) return ISM_E_DEVICE;
  return ISM_OK;
}

int ism_simulate_polar(const ism_room *room, const float *src, int n_src, const float *rcv, int n_rcv,
                       const float *orient, double pattern, int precision, float *out, void *ws, size_t ws_bytes,
                       void *stream) {
  Plan p;
  const int st = make_plan(room, n_src, n_rcv, precision, p);
  if (st != ISM_OK) return st;
  if (!src || !rcv || !out || !orient) return ISM_E_INVALID_ARG;
  if (!(pattern >= 0.0 && pattern <= 1.0)) return ISM_E_INVALID_ARG;
  if (!ws || ws_bytes < p.ws_bytes) return ISM_E_WORKSPACE;
  p.ra.dir_a = (float)pattern;
  p.ra.dir_b = (float)(1.0 - pattern);
  return run_plan(p, src, rcv, out, ws, stream, nullptr, nullptr, orient);
}

// ---- Diffuse tail (Sec. 2.2, Eq. (8); Sec. 3.3) ------------------------------
// The ISM part is planned as a call with t_max = t_diff; its RIRs go to the
// workspace after the plan's own arrays, and the diffuse kernel writes the
// full RIRs (ISM part copied, tail drawn) to out.
static int diffuse_plan(const ism_room *r, double t_diff, double t60, int n_src, int n_rcv, int precision, Plan &p,
                        int64_t &n_full, size_t &off_ism, size_t &ws_bytes) {
  if (!r) return ISM_E_INVALID_ARG;
  if (!(t_diff > 0.0) || !(t60 > 0.0) || !std::isfinite(t_diff) || !std::isfinite(t60)) return ISM_E_INVALID_ARG;
  const int rs = ism_check_room(r);
  if (rs != ISM_OK) return rs;
  if (!(t_diff <= r->t_max)) return ISM_E_INVALID_ARG;
  ism_room ri = *r;
  ri.t_max = t_diff;
  const int st = make_plan(&ri, n_src, n_rcv, precision, p);
  if (st != ISM_OK) return st;
  n_full = ism_n_samples(r->t_max, r->fs);
  if (p.ra.n_samples > n_full) return ISM_E_INVALID_ARG;
  off_ism = align_up(p.ws_bytes);
  ws_bytes = off_ism + sizeof(float) * (size_t)p.n_rir * (size_t)p.ra.n_samples;
  return ISM_OK;
}

int ism_diffuse_workspace_size(const ism_room *room, double t_diff, double t60, int n_src, int n_rcv, int precision,
                               size_t *bytes) {
  if (!bytes) return ISM_E_INVALID_ARG;
  Plan p;
  int64_t n_full;
  size_t off_ism, ws;
  const int st = diffuse_plan(room, t_diff, t60, n_src, n_rcv, precision, p, n_full, off_ism, ws);
  if (st != ISM_OK) return st;
  *bytes = ws;
  return ISM_OK;
}

int ism_simulate_diffuse(const ism_room *room, double t_diff, double t60, uint64_t seed, const float *src, int n_src,
                         const float *rcv, int n_rcv, int precision, float *out, void *ws, size_t ws_bytes,
                         void *stream) {
  return ism_simulate_diffuse_timed(room, t_diff, t60, seed, src, n_src, rcv, n_rcv, precision, out, ws, ws_bytes,
                                    stream, nullptr, nullptr);
}

// Diffuse RIRs; orient != null makes the receivers directional (pattern a).
static int simulate_diffuse(const ism_room *room, double t_diff, double t60, uint64_t seed, const float *src,
                            int n_src, const float *rcv, int n_rcv, const float *orient, double pattern,
                            int precision, float *out, void *ws, size_t ws_bytes, void *stream, void *ev_start,
                            void *ev_stop) {
  Plan p;
  int64_t n_full;
  size_t off_ism, need;
  const int st = diffuse_plan(room, t_diff, t60, n_src, n_rcv, precision, p, n_full, off_ism, need);
  if (st != ISM_OK) return st;
  if (!src || !rcv || !out) return ISM_E_INVALID_ARG;
  if (orient && !(pattern >= 0.0 && pattern <= 1.0)) return ISM_E_INVALID_ARG;
  if (!ws || ws_bytes < need) return ISM_E_WORKSPACE;
  if (orient) {
    p.ra.dir_a = (float)pattern;
    p.ra.dir_b = (float)(1.0 - pattern);
  }
  float *ism = (float *)((char *)ws + off_ism);
  const int rs = run_plan(p, src, rcv, ism, ws, stream, ev_start, ev_stop, orient);
  if (rs != ISM_OK) return rs;
  if (launch_diffuse(ism, p.ra.n_samples, out, (int)n_full, p.n_rir, room->fs, t_diff, t60, seed,
                     (hipStream_t)stream) != 0)
    return ISM_E_DEVICE;
  return ISM_OK;
}

int ism_simulate_diffuse_timed(const ism_room *room, double t_diff, double t60, uint64_t seed, const float *src,
                               int n_src, const float *rcv, int n_rcv, int precision, float *out, void *ws,
                               size_t ws_bytes, void *stream, void *ev_start, void *ev_stop) {
  return simulate_diffuse(room, t_diff, t60, seed, src, n_src, rcv, n_rcv, nullptr, 1.0, precision, out, ws,
                          ws_bytes, stream, ev_start, ev_stop);
}

int ism_simulate_diffuse_polar(const ism_room *room, double t_diff, double t60, uint64_t seed, const float *src,
                               int n_src, const float *rcv, int n_rcv, const float *orient, double pattern,
                               int precision, float *out, void *ws, size_t ws_bytes, void *stream) {
  if (!orient) return ISM_E_INVALID_ARG;
  return simulate_diffuse(room, t_diff, t60, seed, src, n_src, rcv, n_rcv, orient, pattern, precision, out, ws,
                          ws_bytes, stream, nullptr, nullptr);
}

// ---- batches ------------------------------------------------------------------

namespace {

constexpr int kMaxClasses = kMaxBatchClasses;

struct BatchState {  // stored in ism_batch::opaque
  uint64_t ws;
  uint64_t off_jobs, off_rirs, off_items, off_red, off_pos, off_valid, off_origin, off_tab, off_part, off_marg,
      off_queue, off_wc;
  uint32_t n_rir, n_red, n_classes, mode;  // mode: 0 FP32, 1 FP16, 2 table taps
  uint32_t polar, n_jobs, any_gen, long_runs;  // polar: directional kernels; any_gen: general-mode windows;
                                               // long_runs: a tile of RED_SLICE_MIN items or more
  uint32_t n_red_split, pad;                    // reduce entries of split tiles (they come first)
  uint32_t class_first[kMaxClasses], class_count[kMaxClasses], class_grid[kMaxClasses];
  int32_t class_wt[kMaxClasses], class_gen[kMaxClasses];
};
static_assert(sizeof(BatchState) <= sizeof(ism_batch), "ism_batch too small");

struct BatchPlan {
  std::vector<JobDev> jobs;
  std::vector<BatchRir> rirs;
  std::vector<BatchItem> items;
  std::vector<BatchReduce> red;
  std::vector<size_t> pos_off;  // per job: offset (floats) of its src, rcv, orient in the position area
  BatchState st;
  size_t ws_bytes;
};

// Largest-first order without a comparison sort: items go into buckets of
// their estimated cost, eight per octave, filled from the most expensive down
// (stable: jobs, tiles, RIRs and chunks keep their order inside a bucket).
constexpr int kCostBuckets = 512;
int cost_bucket(double cost) {
  const int b = (int)std::floor(8.0 * std::log2(cost + 1.0));
  return std::max(0, std::min(kCostBuckets - 1, b));
}

// Plans a batch. With fill == false only the counts and the workspace layout
// are computed (ism_batch_workspace_size); with fill == true the job, RIR,
// item and reduce tables are built as well (ism_batch_prepare).
int plan_batch(const ism_job *jobs, int n_jobs, int precision, const ism_schedule *sched, BatchPlan &bp,
               bool fill) {
  if (!jobs || n_jobs < 1) return ISM_E_INVALID_ARG;
  std::memset(&bp.st, 0, sizeof(bp.st));
  // Each job is planned as a single call without the tail taper (tapering
  // every job would only fragment small jobs; the batch's own tail is the
  // largest-first order over all its items), with an item size taken from
  // the whole batch (pass 0).
  std::vector<Plan> plans(n_jobs);
  bool polar = false;
  for (int j = 0; j < n_jobs; ++j) {
    if (!jobs[j].src || !jobs[j].rcv || !jobs[j].out) return ISM_E_INVALID_ARG;
    if (jobs[j].orient) {
      if (!(jobs[j].pattern >= 0.0 && jobs[j].pattern <= 1.0)) return ISM_E_INVALID_ARG;
      polar = true;
    }
  }
  // with any directional job the batch runs the directional kernels; the
  // others take the pattern a = 1, b = 0, whose factor is exactly 1
  // pass 0: every job's estimated work. The batch fills the device with all
  // of it, so its items are sized from the batch's total as a single call
  // sizes them from its own (max(min_item_taps, total / balance_items) of
  // the job's class), capped at the tuned batch item size: many small items
  // cost margin and partial writes, a few large ones leave an uneven tail;
  // a batch with less work than that per resident wave gets items of its
  // work over the resident waves (at least kSmallItemTaps).
  double batch_taps = 0.0;
  for (int j = 0; j < n_jobs; ++j) {
    Plan &p = plans[j];
    const int stt = make_plan(&jobs[j].room, jobs[j].n_src, jobs[j].n_rcv, precision, p, sched, false);
    if (stt != ISM_OK) return stt;
    batch_taps += p.total_taps;
  }
  // pass 1: plans, window classes and counts
  int n_classes = 0;
  int class_wt[kMaxClasses] = {}, class_gen[kMaxClasses] = {};
  std::vector<int> job_cls(n_jobs);
  uint64_t tab_entries = 0, n_rir = 0, n_items = 0, slots = 0, n_red = 0, marg_units = 0, wc_floats = 0,
           max_chunks = 0;
  std::vector<uint64_t> bucket_count((size_t)kMaxClasses * kCostBuckets, 0);
  for (int j = 0; j < n_jobs; ++j) {
    Plan &p = plans[j];
    if (!(sched && sched->item_taps > 0.0)) {
      ism_schedule js{};
      if (sched) js = *sched;
      const double t = std::min(batch_item_taps(p.wt, p.half), item_target(batch_taps, p.wt, p.half, p.ra.n_samples, sched));
      // a batch too small to give every resident wave an item of that size is
      // spread over them instead (the small-call rule of single calls)
      js.item_taps = batch_taps < kResidentWaves * t ? std::min(t, small_call_floor(batch_taps)) : t;
      const int stt = make_plan(&jobs[j].room, jobs[j].n_src, jobs[j].n_rcv, precision, p, &js, false);
      if (stt != ISM_OK) return stt;
    }
    int cls = -1;
    for (int k = 0; k < n_classes; ++k)
      if (class_wt[k] == p.wt && class_gen[k] == (p.gen ? 1 : 0)) cls = k;
    if (cls < 0) {
      if (n_classes == kMaxClasses) return ISM_E_UNSUPPORTED;
      cls = n_classes++;
      class_wt[cls] = p.wt;
      class_gen[cls] = p.gen ? 1 : 0;
    }
    job_cls[j] = cls;
    if (p.gen) wc_floats += (uint64_t)WC_STRIDE * p.wt;
    for (int t = 0; t < p.pa.n_tiles; ++t) {
      const uint64_t C = p.pa.chunks[t];
      max_chunks = std::max(max_chunks, C);
      n_items += C * p.n_rir;
      marg_units += C * p.n_rir * (uint64_t)(p.wt / MARG_UNIT);
      if (C > 1) slots += C * p.n_rir;
      bucket_count[(size_t)cls * kCostBuckets + cost_bucket(p.tile_taps[t] / C)] += C * p.n_rir;
    }
    n_red += (uint64_t)p.pa.n_tiles * p.n_rir;
    tab_entries += (uint64_t)p.n_rir * p.ra.n_tab;
    n_rir += (uint64_t)p.n_rir;
  }
  if (n_rir > 0x7fffffffULL || n_items > 0x7fffffffULL || slots > 0xffffffffULL || n_red > 0x7fffffffULL ||
      marg_units > 0xffffffffULL)
    return ISM_E_TOO_LARGE;
  // item positions: classes in order, each class from its most expensive bucket down
  std::vector<uint64_t> bucket_next((size_t)kMaxClasses * kCostBuckets, 0);
  uint64_t acc = 0;
  for (int k = 0; k < n_classes; ++k) {
    bp.st.class_first[k] = (uint32_t)acc;
    for (int b = kCostBuckets - 1; b >= 0; --b) {
      bucket_next[(size_t)k * kCostBuckets + b] = acc;
      acc += bucket_count[(size_t)k * kCostBuckets + b];
    }
    bp.st.class_count[k] = (uint32_t)(acc - bp.st.class_first[k]);
    bp.st.class_wt[k] = class_wt[k];
    bp.st.class_gen[k] = class_gen[k];
    // persistent grid: the tuned workgroups per SIMD (or the schedule's)
    int waves = kAccWavesPerSimd;
    for (const BatchTuning &t : kBatchTuning)
      if (t.wt == class_wt[k] && t.half == (precision == ISM_FP16 ? 1 : 0)) waves = t.waves;
    if (sched && sched->batch_waves > 0.0) waves = std::max(1, (int)std::lround(sched->batch_waves));
    bp.st.class_grid[k] = (uint32_t)std::min<uint64_t>(bp.st.class_count[k], 1024ull * (uint64_t)waves);
  }
  bp.st.n_jobs = (uint32_t)n_jobs;
  bp.st.any_gen = wc_floats > 0 ? 1u : 0u;
  bp.st.long_runs = max_chunks >= (uint64_t)RED_SLICE_MIN ? 1u : 0u;
  bp.st.n_classes = (uint32_t)n_classes;
  bp.st.mode = precision == ISM_FP16 ? 1u : precision == ISM_FP32_LUT ? 2u : 0u;
  bp.st.polar = polar ? 1u : 0u;
  bp.st.n_rir = (uint32_t)n_rir;
  bp.st.n_red = (uint32_t)n_red;
  size_t o = 0;
  bp.st.off_jobs = o;
  o = align_up(o + sizeof(JobDev) * (size_t)n_jobs);
  bp.st.off_rirs = o;
  o = align_up(o + sizeof(BatchRir) * (size_t)n_rir);
  bp.st.off_items = o;
  o = align_up(o + sizeof(BatchItem) * (size_t)n_items);
  bp.st.off_red = o;
  o = align_up(o + sizeof(BatchReduce) * (size_t)n_red);
  // positions of every job (ism_simulate_batch copies host positions here)
  bp.st.off_pos = o;
  bp.pos_off.resize(n_jobs);
  size_t pos_floats = 0;
  for (int j = 0; j < n_jobs; ++j) {
    bp.pos_off[j] = pos_floats;
    pos_floats += 3 * ((size_t)jobs[j].n_src + (size_t)jobs[j].n_rcv * (jobs[j].orient ? 2 : 1));
  }
  o = align_up(o + sizeof(float) * pos_floats);
  bp.st.off_valid = o;
  o = align_up(o + sizeof(int) * n_rir);
  bp.st.off_origin = o;
  o = align_up(o + sizeof(AxisOrigin) * n_rir);
  bp.st.off_tab = o;
  o = align_up(o + sizeof(AxisEntry) * tab_entries);
  bp.st.off_part = o;
  o = align_up(o + sizeof(float) * (size_t)slots * TILE);
  bp.st.off_marg = o;
  o = align_up(o + sizeof(float) * MARG_UNIT * (size_t)marg_units);
  // work-queue counters of the persistent launches, one per window class
  bp.st.off_queue = o;
  o = align_up(o + sizeof(uint32_t) * kMaxClasses);
  // general-mode window constants, one block per such job
  bp.st.off_wc = o;
  o = align_up(o + sizeof(float) * (size_t)wc_floats);
  bp.ws_bytes = o;
  if (!fill) return ISM_OK;

  // pass 2: tables. Margin records are numbered in (job, tile, RIR, chunk)
  // order, so the records of one (tile, RIR) are contiguous.
  bp.jobs.resize(n_jobs);
  bp.rirs.resize(n_rir);
  bp.items.resize(n_items);
  bp.red.resize(n_red);
  uint64_t rir_base = 0, tab_base = 0, mslot = 0, red_i = 0, wc_base = 0;
  uint32_t slot = 0;
  for (int j = 0; j < n_jobs; ++j) {
    const Plan &p = plans[j];
    const ism_job &jb = jobs[j];
    JobDev &d = bp.jobs[j];
    std::memset(&d, 0, sizeof(d));
    d.ra = p.ra;
    d.ra.dir_a = jb.orient ? (float)jb.pattern : 1.0f;
    d.ra.dir_b = jb.orient ? (float)(1.0 - jb.pattern) : 0.0f;
    d.src = jb.src;
    d.rcv = jb.rcv;
    d.out = jb.out;
    d.orient = jb.orient;
    d.tab_base = tab_base;
    d.rir_base = (uint32_t)rir_base;
    if (p.gen) {  // device address filled in by prepare_batch (ws base unknown here)
      d.wc = (float *)(uintptr_t)(wc_base + 1);
      wc_base += (uint64_t)WC_STRIDE * p.wt;
    }
    for (int r = 0; r < p.n_rir; ++r) bp.rirs[rir_base + r] = BatchRir{(uint32_t)j, (uint32_t)r};
    const int nt = p.pa.n_tiles;
    // margin records (units of MARG_UNIT floats, wu units each): the first
    // record of (tile t, RIR r) is mfirst_t + r * chunks[t] * wu
    const uint64_t wu = (uint64_t)(p.wt / MARG_UNIT);
    std::vector<uint64_t> mfirst(nt);
    for (int t = 0; t < nt; ++t) {
      mfirst[t] = mslot;
      mslot += (uint64_t)p.pa.chunks[t] * p.n_rir * wu;
    }
    for (int t = 0; t < nt; ++t) {
      const int C = p.pa.chunks[t];
      uint64_t &pos = bucket_next[(size_t)job_cls[j] * kCostBuckets + cost_bucket(p.tile_taps[t] / C)];
      for (int r = 0; r < p.n_rir; ++r) {
        BatchReduce &rd = bp.red[red_i++];
        std::memset(&rd, 0, sizeof(rd));
        rd.job = (uint32_t)j;
        rd.rir = (uint32_t)r;
        rd.tile = (uint16_t)t;
        rd.chunks = (uint16_t)C;
        rd.first = C > 1 ? slot : 0xffffffffu;
        if (t > 0) {
          rd.mprev = (uint32_t)(mfirst[t - 1] + (uint64_t)r * p.pa.chunks[t - 1] * wu);
          rd.nprev = p.pa.chunks[t - 1];
        }
        if (t + 1 < nt) {
          rd.mnext = (uint32_t)(mfirst[t + 1] + (uint64_t)r * p.pa.chunks[t + 1] * wu);
          rd.nnext = p.pa.chunks[t + 1];
        }
        for (int c = 0; c < C; ++c)
          bp.items[pos++] = BatchItem{(uint32_t)j, (uint32_t)r, (uint16_t)t, (uint8_t)c, (uint8_t)C,
                                      C > 1 ? slot + (uint32_t)c : 0xffffffffu,
                                      (uint32_t)(mfirst[t] + ((uint64_t)r * C + c) * wu)};
        if (C > 1) slot += (uint32_t)C;
      }
    }
    tab_base += (uint64_t)p.n_rir * p.ra.n_tab;
    rir_base += (uint64_t)p.n_rir;
  }
  if (mslot > 0xffffffffULL) return ISM_E_TOO_LARGE;
  // split tiles first (their whole tile is summed), then the tiles whose own
  // samples are already final (only their margin samples change)
  const auto mid = std::stable_partition(bp.red.begin(), bp.red.end(),
                                         [](const BatchReduce &r) { return r.chunks > 1; });
  bp.st.n_red_split = (uint32_t)(mid - bp.red.begin());
  return ISM_OK;
}

}  // namespace

int ism_batch_workspace_size_ex(const ism_job *jobs, int n_jobs, int precision, const ism_schedule *sched,
                                size_t *bytes) {
  if (!bytes) return ISM_E_INVALID_ARG;
  BatchPlan bp;
  const int st = plan_batch(jobs, n_jobs, precision, sched, bp, false);
  if (st != ISM_OK) return st;
  *bytes = bp.ws_bytes;
  return ISM_OK;
}

int ism_batch_workspace_size(const ism_job *jobs, int n_jobs, int precision, size_t *bytes) {
  return ism_batch_workspace_size_ex(jobs, n_jobs, precision, nullptr, bytes);
}

namespace {
// Plans a batch and uploads its tables (and, with host_pos, the jobs' host
// positions) into ws with one host-to-device copy on stream.
int prepare_batch(const ism_job *jobs, int n_jobs, int precision, const ism_schedule *sched, void *ws,
                  size_t ws_bytes, void *stream, bool host_pos, ism_batch *batch) {
  if (!batch) return ISM_E_INVALID_ARG;
  BatchPlan bp;
  int st = plan_batch(jobs, n_jobs, precision, sched, bp, true);
  if (st != ISM_OK) return st;
  if (host_pos) {
    for (int j = 0; j < n_jobs; ++j) {
      st = ism_check_positions(&jobs[j].room, jobs[j].src, jobs[j].n_src, jobs[j].rcv, jobs[j].n_rcv);
      if (st != ISM_OK) return st;
      if (jobs[j].orient)
        for (int i = 0; i < jobs[j].n_rcv; ++i) {
          const float *o = jobs[j].orient + 3 * i;
          if (!(std::isfinite(o[0]) && std::isfinite(o[1]) && std::isfinite(o[2])) ||
              (o[0] == 0.0f && o[1] == 0.0f && o[2] == 0.0f))
            return ISM_E_INVALID_ARG;
        }
    }
  }
  if (!ws || ws_bytes < bp.ws_bytes) return ISM_E_WORKSPACE;
  // one contiguous host image of the metadata, copied with a single transfer
  // (alignment gaps between the tables are left uninitialised)
  std::unique_ptr<char[]> host_buf(new char[bp.st.off_valid]);
  char *const host = host_buf.get();
  if (host_pos) {
    // the jobs' device view points into the position area of ws
    float *dpos = (float *)((char *)ws + bp.st.off_pos);
    float *hpos = (float *)(host + bp.st.off_pos);
    for (int j = 0; j < n_jobs; ++j) {
      const ism_job &jb = jobs[j];
      JobDev &d = bp.jobs[j];
      size_t o = bp.pos_off[j];
      std::memcpy(hpos + o, jb.src, sizeof(float) * 3 * (size_t)jb.n_src);
      d.src = dpos + o;
      o += 3 * (size_t)jb.n_src;
      std::memcpy(hpos + o, jb.rcv, sizeof(float) * 3 * (size_t)jb.n_rcv);
      d.rcv = dpos + o;
      o += 3 * (size_t)jb.n_rcv;
      if (jb.orient) {
        std::memcpy(hpos + o, jb.orient, sizeof(float) * 3 * (size_t)jb.n_rcv);
        d.orient = dpos + o;
      }
    }
  }
  for (JobDev &d : bp.jobs)  // general-mode window constants: offsets into ws
    if (d.wc) d.wc = (float *)((char *)ws + bp.st.off_wc) + ((uintptr_t)d.wc - 1);
  std::memcpy(host + bp.st.off_jobs, bp.jobs.data(), sizeof(JobDev) * bp.jobs.size());
  std::memcpy(host + bp.st.off_rirs, bp.rirs.data(), sizeof(BatchRir) * bp.rirs.size());
  std::memcpy(host + bp.st.off_items, bp.items.data(), sizeof(BatchItem) * bp.items.size());
  if (!bp.red.empty()) std::memcpy(host + bp.st.off_red, bp.red.data(), sizeof(BatchReduce) * bp.red.size());
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(ws, host, bp.st.off_valid, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return device_error("batch tables upload", e);
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return device_error("batch tables upload (synchronize)", e);
  bp.st.ws = (uint64_t)(uintptr_t)ws;
  std::memset(batch, 0, sizeof(*batch));
  std::memcpy(batch, &bp.st, sizeof(bp.st));
  return ISM_OK;
}
}  // namespace

int ism_batch_prepare_ex(const ism_job *jobs, int n_jobs, int precision, const ism_schedule *sched, void *ws,
                         size_t ws_bytes, void *stream, ism_batch *batch) {
  return prepare_batch(jobs, n_jobs, precision, sched, ws, ws_bytes, stream, false, batch);
}

int ism_batch_prepare(const ism_job *jobs, int n_jobs, int precision, void *ws, size_t ws_bytes, void *stream,
                      ism_batch *batch) {
  return prepare_batch(jobs, n_jobs, precision, nullptr, ws, ws_bytes, stream, false, batch);
}

int ism_simulate_batch(const ism_job *jobs, int n_jobs, int precision, void *ws, size_t ws_bytes, void *stream) {
  ism_batch b;
  const int st = prepare_batch(jobs, n_jobs, precision, nullptr, ws, ws_bytes, stream, true, &b);
  if (st != ISM_OK) return st;
  return ism_batch_run(&b, stream);
}

int ism_batch_run(const ism_batch *batch, void *stream) { return ism_batch_run_timed(batch, stream, nullptr, nullptr); }

int ism_batch_run_timed(const ism_batch *batch, void *stream, void *ev_start, void *ev_stop) {
  if (!batch) return ISM_E_INVALID_ARG;
  BatchState b;
  std::memcpy(&b, batch, sizeof(b));
  if (!b.ws || b.n_rir == 0 || b.n_classes == 0 || b.n_classes > (uint32_t)kMaxClasses || b.n_red_split > b.n_red)
    return ISM_E_INVALID_ARG;
  char *w = (char *)(uintptr_t)b.ws;
  const int rc = launch_batch((const JobDev *)(w + b.off_jobs), (int)b.n_jobs, b.any_gen != 0,
                              (const BatchRir *)(w + b.off_rirs), b.n_rir,
                              (const BatchItem *)(w + b.off_items), b.class_first, b.class_count, b.class_grid,
                              b.class_wt, b.class_gen, (int)b.n_classes, b.mode == 1, b.mode == 2, b.polar != 0,
                              (const BatchReduce *)(w + b.off_red), b.n_red, b.n_red_split, b.long_runs != 0,
                              (AxisEntry *)(w + b.off_tab), (AxisOrigin *)(w + b.off_origin),
                              (int *)(w + b.off_valid), (float *)(w + b.off_part), (float *)(w + b.off_marg),
                              (uint32_t *)(w + b.off_queue), (hipStream_t)stream,
                              (hipEvent_t)ev_start, (hipEvent_t)ev_stop);
  return rc == 0 ? ISM_OK : ISM_E_DEVICE;
}

}  // extern "C"

// ---- Moving-source filtering (Sec. 3.4) --------------------------------------
namespace {
constexpr int kFftMaxPieces = 16;  // segments one FFT input block may touch
constexpr int kAutoMaxPieces = 4;

int filter_args(const float *x, int n_x, const float *rir, int n_pos, int n_mic, int n_rir, const float *y) {
  if (!x || !rir || !y) return ISM_E_INVALID_ARG;
  if (n_x < 1 || n_pos < 1 || n_mic < 1 || n_rir < 1 || n_pos > n_x) return ISM_E_INVALID_ARG;
  if (n_mic > 65535 || (int64_t)n_x + n_rir - 1 > (int64_t)0x7fffffff) return ISM_E_TOO_LARGE;
  return ISM_OK;
}

// Resolves the method (auto: FFT for RIRs of 1024 taps and more when an input
// block touches at most kAutoMaxPieces segments) and the FFT plan.
int filter_method(int n_x, int n_pos, int n_mic, int n_rir, int method, FftPlan &f, int &resolved) {
  if (method != ISM_FILTER_AUTO && method != ISM_FILTER_DIRECT && method != ISM_FILTER_FFT) return ISM_E_INVALID_ARG;
  resolved = ISM_FILTER_DIRECT;
  if (method == ISM_FILTER_DIRECT) return ISM_OK;
  const bool ok = fft_plan(n_x, n_pos, n_mic, n_rir, method == ISM_FILTER_FFT ? kFftMaxPieces : kAutoMaxPieces, f);
  if (method == ISM_FILTER_FFT) {
    if (!ok) return ISM_E_UNSUPPORTED;
    resolved = ISM_FILTER_FFT;
  } else if (ok && n_rir >= 1024) {
    resolved = ISM_FILTER_FFT;
  }
  return ISM_OK;
}
}  // namespace

int ism_filter_workspace_size(int n_x, int n_pos, int n_mic, int n_rir, int method, size_t *bytes) {
  if (!bytes) return ISM_E_INVALID_ARG;
  if (n_x < 1 || n_pos < 1 || n_mic < 1 || n_rir < 1 || n_pos > n_x) return ISM_E_INVALID_ARG;
  if (n_mic > 65535 || (int64_t)n_x + n_rir - 1 > (int64_t)0x7fffffff) return ISM_E_TOO_LARGE;
  FftPlan f;
  int m = 0;
  const int st = filter_method(n_x, n_pos, n_mic, n_rir, method, f, m);
  if (st != ISM_OK) return st;
  *bytes = m == ISM_FILTER_FFT ? f.bytes : 0;
  return ISM_OK;
}

int ism_filter_trajectory_ex(const float *x, int n_x, const float *rir, int n_pos, int n_mic, int n_rir, int method,
                             float *y, void *ws, size_t ws_bytes, void *stream) {
  int st = filter_args(x, n_x, rir, n_pos, n_mic, n_rir, y);
  if (st != ISM_OK) return st;
  FftPlan f;
  int m = 0;
  st = filter_method(n_x, n_pos, n_mic, n_rir, method, f, m);
  if (st != ISM_OK) return st;
  if (m == ISM_FILTER_DIRECT) return ism_filter_trajectory(x, n_x, rir, n_pos, n_mic, n_rir, y, stream);
  if (!ws || ws_bytes < f.bytes) return ISM_E_WORKSPACE;
  if (launch_filter_fft(x, n_x, rir, n_pos, n_mic, n_rir, y, f, ws, (hipStream_t)stream) != 0) return ISM_E_DEVICE;
  return ISM_OK;
}

int ism_filter_trajectory(const float *x, int n_x, const float *rir, int n_pos, int n_mic, int n_rir, float *y,
                          void *stream) {
  if (!x || !rir || !y) return ISM_E_INVALID_ARG;
  if (n_x < 1 || n_pos < 1 || n_mic < 1 || n_rir < 1 || n_pos > n_x) return ISM_E_INVALID_ARG;
  if (n_mic > 65535 || (int64_t)n_x + n_rir - 1 > (int64_t)0x7fffffff) return ISM_E_TOO_LARGE;
  const int rc = launch_filter(x, n_x, rir, n_pos, n_mic, n_rir, y, (hipStream_t)stream);
  if (rc == -2) return ISM_E_TOO_LARGE;
  if (rc != 0) return ISM_E_DEVICE;
  return ISM_OK;
}
