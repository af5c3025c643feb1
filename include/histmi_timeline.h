/*
 * histmi_timeline.h -- the per-workgroup timeline of the diagnostic build.
 *
 * libhistmi_timeline.so is libhistmi.so with its kernel compiled with HISTMI_TIMELINE: the
 * same C ABI (include/histmi.h), the same steps, plus one store per recorded event.  Thread
 * 0 of each of the first `workgroups` workgroups of a launch records up to `per_workgroup`
 * events in a device array, each one 64-bit word:
 *   bits [56,64) phase, [40,56) segment (or a count, see below), [0,40) the device's
 *   constant 100 MHz clock (s_memrealtime);
 * phases: 0 entry, 2 segment set up (decision taken, table staged), 3 tile counted,
 * 4 flushed, 5 finalizer start, 6 merged, 7 finalizer done, 8 exit, 9 flush start, 10 table
 * summed, 11 atomics issued, 12 sequencer lock taken, 13 sequencer batch decided (segment
 * field: chunks decided), 14 lock released, 15 sequencer batch loaded (chunks present).
 * Unused words are 0.  Workgroups of consecutive launches write over each other: reset,
 * run one launch, synchronize, read.  Used by paper_1011_0235_amd/timeline.py to break a
 * launch down into the steps of the paper's Table 1 (Sec. III.A).  The default library does
 * not export these calls.
 */
#ifndef HISTMI_TIMELINE_H
#define HISTMI_TIMELINE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Size of the device array: workgroups recorded x events per workgroup (never fails with
 * non-null pointers; returns hipSuccess, 0). */
int hist_timeline_shape(uint32_t *workgroups, uint32_t *per_workgroup);
/* Copy the whole array (bytes = workgroups x per_workgroup x 8) to host memory; synchronous.
 * Returns a HIP error code (0 on success; invalid value for a wrong size). */
int hist_timeline_read(uint64_t *host, size_t bytes);
/* Zero the array; synchronous.  Returns a HIP error code. */
int hist_timeline_reset(void);

#ifdef __cplusplus
}
#endif

#endif
