/*
 * Mixed batches: several codes (of uneven length) decoded in one call, and
 * per-code layout autotuning.
 *
 * ldpc_decode_multi forks the jobs of one call onto a pool of library
 * streams (default priority, created once per device and kept until the
 * process ends) and joins them back into the caller's stream with events, so
 * the frames of different codes run concurrently and the whole call can be
 * captured into one HIP graph (it enqueues no memset and never
 * synchronises).  Every frame keeps its own early stop.
 */
#ifndef LDPC_MULTI_H
#define LDPC_MULTI_H

#include "ldpc.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One sub-batch: the arguments of one ldpc_decode_batch call without the
 * workspace and the stream. */
typedef struct {
    const ldpc_code *code;
    int32_t n_frames;
    const void *llr_in;
    ldpc_decode_params params;
    uint8_t *hard_out;
    float *llr_out;      /* may be NULL */
    int32_t *iters_out;
    uint8_t *syndrome_ok;
} ldpc_job;

/* Workspace bytes for the jobs together (each job's ldpc_decode_workspace_size,
 * 256-byte aligned, concatenated in job order). */
ldpc_status ldpc_multi_workspace_size(const ldpc_job *jobs, int32_t n_jobs, size_t *bytes);

/*
 * Decode every job (all codes on one device).  Results equal n_jobs separate
 * ldpc_decode_batch calls.  Jobs are spread over up to 4 library streams,
 * the longest (frames x edges x max_iter) first; with one job, the caller's
 * stream is used directly.  Errors as ldpc_decode_batch, checked for every
 * job before anything is launched.
 */
ldpc_status ldpc_decode_multi(const ldpc_job *jobs, int32_t n_jobs, void *workspace, size_t workspace_bytes,
                              void *stream);

/*
 * The same jobs in ONE persistent launch: 1024-thread workgroups, one per
 * CU, take work items from a device counter until none is left; a work item
 * is 1024 / T frames of one job (T: threads of the code's packed register
 * shape, 256, 512 or 1024), each frame in its own LDS region, the frames of
 * an item sharing the workgroup's barriers (a frame that has stopped idles
 * until the item's last frame stops).  Jobs with the longest frames
 * (edges x max_iter) are taken first.  Results equal ldpc_decode_multi's.
 * Every job with frames must run the packed kernel in 6-bit int8
 * single-scan (AUTO or REG layout; LDPC_EUNSUPPORTED otherwise); at most 8
 * jobs with frames.  Early stop folds into the gathers (as in
 * ldpc_decode_batch) only when every job has early_stop, no posterior
 * output and max_iter >= 1; otherwise every job takes the separate
 * syndrome pass.  Workspace: ldpc_multi_persistent_workspace_size() bytes
 * (the work-item counter, zeroed by a kernel before the launch, so the call
 * is capturable); allocates nothing, never synchronises.
 */
ldpc_status ldpc_multi_persistent_workspace_size(const ldpc_job *jobs, int32_t n_jobs, size_t *bytes);
ldpc_status ldpc_decode_multi_persistent(const ldpc_job *jobs, int32_t n_jobs, void *workspace,
                                         size_t workspace_bytes, void *stream);

/*
 * Time every layout that can run (msg, sched) of *p on this code (REG, REG1,
 * LDS, HBM, FRAMES; each on n_frames zero-LLR frames with early stop off and
 * p->max_iter iterations, best of 3 after a warm-up), allocating device
 * memory for the trial, and make AUTO use the fastest one for this (msg,
 * sched, msg_bits) on this handle from now on.  A later AUTO call whose
 * parameters the tuned layout cannot run (another frame count's workspace
 * form, say) falls back to the built-in policy.  Synchronises the device.
 *  best_layout  out: LDPC_LAYOUT_* chosen.
 *  best_ms      out: its time per call in milliseconds (may be NULL).
 *  n_tried      out: layouts timed (may be NULL).
 */
ldpc_status ldpc_autotune(ldpc_code *code, int32_t n_frames, const ldpc_decode_params *p, int32_t *best_layout,
                          float *best_ms, int32_t *n_tried);

#ifdef __cplusplus
}
#endif
#endif /* LDPC_MULTI_H */
