/*
 * swept_debug.h -- entry points of the counting build libswept_count.so,
 * the same sources compiled with SWEPT_COUNT_UPDATES.  The normal library
 * libswept.so does not export them.
 *
 * In that build the stage kernels (the banded and continuous-band
 * schedules, for single fields, unequal tilings and batches) count every
 * point update they compute, in a device counter.  The swept rule computes
 * each (point, sub-timestep level) of a run exactly once and nothing else
 * (paper, Section 3), so a run of nsteps steps on a ring of n points
 * (the two-fold cover for odd nx) adds exactly n * nsteps * (sub-timesteps
 * per step).  The lane-frame kernel, the adjoint and the naive schedules
 * are not counted.  The counting slows the kernels; it is for tests only.
 */
#ifndef SWEPT_DEBUG_H
#define SWEPT_DEBUG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Wait for the library's stream, then store the count of point updates
 * since the last reset in *count (host pointer) and, if reset != 0, zero the
 * counter.  SWEPT_ENOTINIT before swept_init, SWEPT_EINVAL for a null
 * pointer, SWEPT_EHIP if a HIP call fails.
 */
int swept_debug_update_count(uint64_t *count, int32_t reset);

#ifdef __cplusplus
}
#endif

#endif /* SWEPT_DEBUG_H */
