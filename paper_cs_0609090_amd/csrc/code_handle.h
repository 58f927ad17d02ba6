// The code handle behind the opaque ldpc_code of the C ABI (host side),
// shared by the decoder runtime and the channel-simulation entry points.
#pragma once

#include <array>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/ldpc.h"
#include "code_facts.h"

struct ldpc_code {
    int32_t device = 0;
    int32_t M = 0, N = 0;
    int64_t E = 0;
    int32_t D = 0, Mp = 0, dummy = 0;
    int32_t min_row_deg = 0, max_col_deg = 0;
    ldpc::CodeFacts facts;  // degree histograms and block structure (ldpc_code_query)
    int32_t lds_limit = 65536;
    uint32_t *d_ell = nullptr;
    int32_t *d_vc_ptr = nullptr;
    uint32_t *d_vc_slot = nullptr;
    // register-resident shape (0 = none)
    int32_t regD = 0, regR = 0, regP = 0;
    uint32_t *d_ell_reg = nullptr;
    // packed two-rows-per-lane INT8 shape (0 = none); uses regP's packing
    int32_t pkD = 0, pkR = 0, pkT = 0;  // slots per lane, rows per thread, threads per workgroup
    int32_t pkS = 1;                    // lanes per row (2: a row's slots split over a lane pair)
    int32_t pkBias = 0;  // accumulator field bias of the packed kernel
    uint32_t *d_pk_idx = nullptr;
    uint32_t *d_pk_idx16 = nullptr;  // the records for int16 Z_old (8-bit messages; accumulator
                                     // fields of 16 bits or more), else null
    // persistent multi-code launch: frames per 1024-thread workgroup (0: not
    // supported), LDS bytes of one frame's region, and the records of every
    // region one set after another (null when one region: d_pk_idx serves)
    int32_t pkGroups = 0;
    uint32_t pkRegion = 0;
    uint32_t *d_pk_grp = nullptr;
    uint32_t *d_pk_slot = nullptr;  // [N] posterior slot of each variable
    uint32_t *d_pk_shift = nullptr;  // accumulator field shift of every edge (bytes), one set for all regions
    // frames-across-lanes binary32 path: CSR rows and, per edge, {variable,
    // position of the edge in variable-major order}
    int32_t *d_row_ptr = nullptr;
    uint32_t *d_row_ent = nullptr;
    uint32_t *d_vc_csr = nullptr;  // [E + 64] row-order edge of each variable-major position
    int32_t cu_count = 256;
    // host copy of H (CSR), kept for the encoder, which is built on first use
    std::vector<int32_t> h_row_ptr, h_col_idx;
    // systematic encoder (0 = not built yet / none; see ldpc_sim.h)
    std::mutex enc_mu;
    bool enc_built = false;
    int32_t enc_kind = 0;         // LDPC_ENC_*
    int32_t enc_K = 0;            // information bits
    int32_t enc_rank = 0;         // parity bits (rank of H)
    int32_t enc_words = 0;        // 32-bit words per packed row of the dense parity map
    std::vector<int32_t> h_info_pos;  // [N]: K information columns (ascending), then the parity columns
    int32_t *d_info_pos = nullptr;    // device copy
    uint32_t *d_enc_rows = nullptr;   // dense: [rank][words] parity map over the information bits
    std::string enc_error;
    // learned decoder: check-degree classes (distinct row degrees, ascending)
    int32_t learn_classes = 0;
    std::vector<int32_t> learn_degrees;
    int32_t *d_row_cls = nullptr;  // [M] class of each row
    // layout used by LDPC_LAYOUT_AUTO per (msg, sched, message width), index
    // tuned_slot(); 0 = the built-in policy (set by ldpc_autotune, read
    // atomically).  A tuned layout that cannot plan a later call falls back to
    // the built-in policy for that call.
    int32_t tuned_layout[18] = {};
};

namespace ldpc {
// index of (msg, sched, msg_bits) in ldpc_code::tuned_layout
inline int tuned_slot(const ldpc_decode_params *p) {
    const int w = p->msg_bits <= 6 ? 0 : p->msg_bits - 6;  // 0, 6 -> 0; 7 -> 1; 8 -> 2
    return (p->msg * 2 + p->sched) * 3 + w;
}

// Makes `dev` the current device for the guard's lifetime.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// ldpc_decode_batch: every check, then (when `launch`) the kernels on `stream`
ldpc_status decode_job(const ldpc_code *c, int32_t n_frames, const void *llr_in, const ldpc_decode_params *p,
                       uint8_t *hard_out, float *llr_out, int32_t *iters_out, uint8_t *syndrome_ok,
                       void *workspace, size_t workspace_bytes, void *stream, bool launch);

struct PersistJob;
// One job of a persistent multi-code launch: the checks of decode_job, then
// that the call runs the 6-bit int8 packed kernel with a shape the persistent
// kernel holds; fills the job's arguments (items and order are the caller's).
ldpc_status persist_job(const ldpc_code *c, int32_t n_frames, const void *llr_in, const ldpc_decode_params *p,
                        uint8_t *hard_out, float *llr_out, int32_t *iters_out, uint8_t *syndrome_ok,
                        PersistJob *out);

// Packed shapes worth timing on this code (the handle's own first): per
// threads-per-workgroup and lanes-per-row pair, the instantiated shape that
// covers the code with the fewest slots and rows.  Empty without a packed shape.
std::vector<std::array<int, 4>> pk_candidates(const ldpc_code *c);
// Makes (D, R, T, S) the handle's packed shape: rebuilds its records and slot
// placement and replaces the device copies.  On failure the handle keeps its
// shape and arrays.  No call may use the handle meanwhile, and no kernel
// launched with the old arrays may still be running.
ldpc_status pk_install(ldpc_code *c, int D, int R, int T, int S);

// error state of the calling thread (ldpc_last_error), set by every entry point
ldpc_status set_error(ldpc_status st, const std::string &msg);
void clear_error();

// Device allocations of the library's own buffers (code handles, the encoder,
// autotuning trials).  Failure injection for tests of the error paths: with
// the environment variable LDPC_FAIL_ALLOC=k (k >= 1), the k-th allocation
// after the last reset_alloc_count() on the calling thread fails as an
// out-of-memory error would, without touching the device.  Entry points that
// allocate reset the count when they start.
hipError_t dev_malloc(void **p, size_t bytes);
void reset_alloc_count();
}  // namespace ldpc
