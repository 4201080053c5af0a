/*
 * hipmsat_probe.h -- bandwidth probes for MI355X (gfx950): the memory-system
 * ceilings the solve loop's kernels are measured against.  Measurement aids
 * only, with no part in the method; built as libhipmsat_probe.so beside the
 * solver library.
 *
 * Both probes enqueue `iters` timed launches on `stream` (a hipStream_t, NULL =
 * the null stream) after one untimed launch, bracket them with HIP events on
 * that stream, synchronise it, and return the average milliseconds per launch
 * in *ms.  Pointers are DEVICE memory on the current device, owned by the
 * caller; nothing is kept after the call.  Return 0 on success, else a
 * nonzero code with hmsp_last_error() holding a message (thread-local).
 */
#ifndef HIPMSAT_PROBE_H
#define HIPMSAT_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Streaming copy of `bytes` (a multiple of 16, at most 2^43; src and dst
 * 16-byte aligned, not overlapping): one 16-byte load and store per thread,
 * the grid covering the buffers once.  Moves 2 * bytes per launch (read +
 * write).
 */
int32_t hmsp_copy(const void* src, void* dst, int64_t bytes, int32_t iters, void* stream, double* ms);

/*
 * Gather-sum over random rows, the access pattern of the transposed pass:
 * out[o][c] = sum over k < deg of src[idx[o deg + k]][c], for o < n_idx / deg
 * and rows of row_floats floats (1, 2, 4, 8, 16, 32 or 64: 4 to 256 bytes).
 * Each lane owns `vec` consecutive floats of a row (1, 2 or 4, at most
 * row_floats); an output's deg (8 or 16) index loads are issued together, then
 * its deg row loads.  src: [rows][row_floats] FP32; idx: n_idx uint32 row
 * indices (a multiple of 16), each below `rows` (the caller guarantees it;
 * the probe does not check); out: [n_idx / deg][row_floats] FP32.  Per
 * launch it reads 4 n_idx index bytes and 4 n_idx row_floats gathered bytes
 * and writes 4 (n_idx / deg) row_floats.
 */
int32_t hmsp_gather(const float* src, int64_t rows, int32_t row_floats, const uint32_t* idx, int64_t n_idx,
                    int32_t deg, int32_t vec, float* out, int32_t iters, void* stream, double* ms);

/*
 * Grid barrier: one cooperative launch of `blocks` 256-thread workgroups (all
 * resident at once) running `rounds` barrier rounds; in each, every
 * workgroup adds one to a device counter (agent-scope release) and polls it
 * (agent-scope acquire) until all have arrived, as a persistent kernel must
 * between passes whose data cross the XCDs.  *us receives the average
 * microseconds per round.  Every wait is bounded: a workgroup that polls
 * 2^20 times, or sees that another gave up, sets an abort flag and leaves
 * (*gave_up = 1; the time is then not a barrier's).  Uses 256 bytes of
 * stream-ordered device memory.
 */
int32_t hmsp_grid_barrier(int32_t blocks, int32_t rounds, void* stream, double* us, int32_t* gave_up);

/*
 * Launch gap: `kernels` launches, one after the other on `stream`, of a
 * kernel of `blocks` 256-thread workgroups that does nothing, enqueued
 * directly (graph = 0) or replayed from a captured graph (graph = 1); *us
 * receives the average microseconds per launch (each waits for the one
 * before, as the passes of a step do).
 */
int32_t hmsp_launch_gap(int32_t blocks, int32_t kernels, int32_t graph, void* stream, double* us);

/* Message of the last failed probe call on this thread ("" if none). */
const char* hmsp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HIPMSAT_PROBE_H */
