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
 * ldpc_decode_batch calls.  The job whose workgroups each take the most LDS,
 * if that is more than half of a CU's (one frame per CU: its workgroups can
 * only start on empty CUs), is launched first on the caller's stream; the
 * others are spread over up to 4 library streams, the longest (frames x
 * edges x max_iter) first; with one job, the caller's stream is used
 * directly.  Errors as ldpc_decode_batch, checked for every job before
 * anything is launched.
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
 * form, say) falls back to the built-in policy.
 *
 * When REG runs the packed two-rows-per-lane kernel (ldpc_code_info's
 * pk_slots > 0), REG is timed with each packed shape worth trying: per
 * threads-per-workgroup and lanes-per-row pair (which set the frames a CU
 * holds), the instantiated shape covering the code with the fewest slots and
 * rows, the handle's own shape first.  If REG wins, its fastest shape becomes
 * the handle's (ldpc_code_query reports it), else the handle keeps its own.
 * The packed shape belongs to the handle: it serves every later call that
 * runs the packed kernel, whatever its parameters (results do not depend on
 * it; the built-in AUTO policy and ldpc_decode_multi_persistent, which needs
 * a shape of 256, 512 or 1024 threads, read it).  Changing it replaces the
 * handle's device arrays, so no other call may use the handle while
 * ldpc_autotune runs.  Synchronises the device.  On an error the handle
 * keeps a valid packed shape.
 *  best_layout  out: LDPC_LAYOUT_* chosen.
 *  best_ms      out: its time per call in milliseconds (may be NULL).
 *  n_tried      out: configurations timed, (layout, packed shape) pairs
 *               (may be NULL).
 */
ldpc_status ldpc_autotune(ldpc_code *code, int32_t n_frames, const ldpc_decode_params *p, int32_t *best_layout,
                          float *best_ms, int32_t *n_tried);

/*
 * The packed shapes ldpc_autotune times on this code, the handle's current
 * one first: (slots per lane, rows per thread, threads per workgroup)
 * triples, the fields ldpc_code_info reports as pk_slots,
 * pk_rows_per_thread and pk_threads (a shape with fewer slots than the
 * longest row splits every row over a lane pair).  None (count 0) when the
 * code has no packed shape.  Works on host-only handles.
 *  shapes  out: [cap][3]; the first min(cap, count) triples are written.
 *  count   out: triples in all.
 */
ldpc_status ldpc_code_packed_shapes(const ldpc_code *code, int32_t *shapes, int32_t cap, int32_t *count);

/*
 * Make one of ldpc_code_packed_shapes() the handle's packed shape (to install
 * a shape ldpc_autotune chose earlier without timing again, say).  Rebuilds
 * the per-edge records on the host and replaces the handle's device copies
 * (allocates; synchronous).  Decoding results do not depend on the shape.  No
 * other call may use the handle meanwhile, and work queued earlier with it
 * must have finished.  LDPC_EUNSUPPORTED for a triple not in the list,
 * LDPC_EINVAL for a host-only handle, LDPC_ENOMEM / LDPC_EDEVICE (the handle
 * keeps its shape).
 */
ldpc_status ldpc_code_set_packed_shape(ldpc_code *code, int32_t slots, int32_t rows_per_thread, int32_t threads);

#ifdef __cplusplus
}
#endif
#endif /* LDPC_MULTI_H */
