/*
 * ism_debug.h - check entry of libism.so: the image enumeration of the GPU
 * path, exposed so that tests can compare it exactly with a plain
 * enumeration of the lattice. Not needed to compute RIRs.
 */
#ifndef ISM_DEBUG_H
#define ISM_DEBUG_H

#include <stddef.h>
#include <stdint.h>

#include "ism.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One image as the accumulation kernel sees it (32 bytes). */
typedef struct {
  int32_t rir;     /* source * n_rcv + receiver                                      */
  int32_t n[3];    /* lattice index per room axis (x, y, z), Sec. 2.1               */
  int32_t k0;      /* floor(x), x = d fs / c the delay in samples (Eq. (3))          */
  uint32_t fq;     /* x - k0 rounded to units of 2^-24 (as the table taps use it)    */
  float amp;       /* Eq. (4) amplitude beta_n / (4 pi d_n), FP32                   */
  uint32_t pad;
} ism_image_record;

/* Runs the image enumeration of ism_simulate_ex (same room, positions, plan and
 * schedule, FP32 mode) without computing taps, and writes one record per image
 * that some work item owns: every lattice image whose integer delay k0 lies in
 * [0, nS + W/2 - 1), i.e. every image with a tap inside the RIR, once.
 *   src, rcv  device float32 [n][3] as for ism_simulate;
 *   sched     as for ism_simulate_ex (NULL = default);
 *   records   device array of cap ism_image_record, in no particular order;
 *   count     device uint32: set to the number of images found (records beyond
 *             cap are counted but not stored);
 *   ws        workspace of ism_workspace_size_ex(room, n_src, n_rcv, ISM_FP32,
 *             sched) bytes.
 * Errors as for ism_simulate_ex, before any launch. Asynchronous on stream. */
int ism_debug_enumerate(const ism_room *room, const float *src, int n_src, const float *rcv, int n_rcv,
                        const ism_schedule *sched, void *records, uint32_t cap, uint32_t *count, void *ws,
                        size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif
