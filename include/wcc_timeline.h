/* wcc_timeline.h -- per-wave timestamps of the half-step kernels.
 *
 * Diagnostic library only: libwcc_timeline.so exports the whole C ABI of
 * wcc.h and wcc2d.h, built from the same kernel sources, plus the calls
 * below; its half-step kernels also record, for every wave, the constant
 * 100 MHz clock and the shader clock counter at entry and exit and the
 * hardware placement (HW_ID and XCC_ID registers).  The product library
 * libwcc.so does not contain them.  The records answer what the kernel trace
 * cannot: how long each wave lives, how many waves share a SIMD over the
 * launch, and the shader clock the waves ran at (the ratio of the two clocks),
 * against which an instruction-issue roof is priced.
 *
 * One record array per kernel family: suffix 1d (the 64-cell wave-tile
 * kernels, launch variants 0..3), 1d_wide (128-cell tiles, variant 4), 2d
 * (the 2D kernels).  Records are indexed by the global wave index
 * (block index x waves per block + wave in block) for the first
 * WCC_TIMELINE_WAVES waves of a launch; each launch overwrites the records of
 * its waves, so after a run they hold its last launch.  The record stamped
 * at exit by a kernel that does not stamp at entry (the state wave-speed
 * kernel of a write) keeps the entry fields of the last clear.
 *
 * Both calls copy synchronously (host <-> device, null stream) on the current
 * device: call them with no half-step in flight.  Return 0 on success, a HIP
 * error code otherwise; the read returns 1 for dst == NULL or a buffer below
 * WCC_TIMELINE_WAVES * sizeof(wcc_timeline_rec) bytes.
 */
#ifndef WCC_TIMELINE_H
#define WCC_TIMELINE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WCC_TIMELINE_WAVES 16384

typedef struct {
  uint64_t t0, t1;   /* constant 100 MHz clock at kernel entry / exit of the wave */
  uint64_t c0, c1;   /* shader clock counter at entry / exit */
  uint32_t hw_id;    /* HW_ID: bits 3:0 wave slot, 5:4 SIMD, 11:8 CU, 12 SH, 13 and up SE */
  uint32_t xcc_id;   /* XCC_ID: bits 3:0 the XCD */
  uint32_t pad[2];
} wcc_timeline_rec;  /* 48 bytes */

/* Zero the records of one kernel family. */
int wcc_timeline_clear_1d(void);
int wcc_timeline_clear_1d_wide(void);
int wcc_timeline_clear_2d(void);

/* Copy the WCC_TIMELINE_WAVES records of one kernel family to host memory
 * `dst` of `bytes` bytes (caller-owned). */
int wcc_timeline_read_1d(void* dst, size_t bytes);
int wcc_timeline_read_1d_wide(void* dst, size_t bytes);
int wcc_timeline_read_2d(void* dst, size_t bytes);

#ifdef __cplusplus
}
#endif

#endif /* WCC_TIMELINE_H */
