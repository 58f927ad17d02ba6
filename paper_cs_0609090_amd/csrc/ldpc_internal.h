// Library-private declarations shared by the runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace ldpc {

constexpr int kWave = 64;     // CDNA wavefront width
constexpr int kQmax = 31;     // 6-bit message range: extrinsics saturate to +-31
constexpr int kZoldMax = 62;  // stored Z_{n} saturates to +-62 (see ss_int.hip)
// b-bit messages (Sec. V, b = 6..8): extrinsics saturate to Q = 2^(b-1) - 1 and
// the stored Z_old to 2Q, which keeps sat_Q(sat_2Q(Z) - L) = sat_Q(Z - L) for |L| <= Q

enum Msg : int { MSG_FP32 = 0, MSG_INT8 = 1, MSG_1BIT = 2 };

// Device copy of a parity-check matrix in padded slot-major (ELL) form.
// Slot j of row m lives at index j * Mp + m, so the 64 rows of a wavefront
// touch 64 consecutive entries of every per-slot array.
struct DevCode {
    int32_t M, N;
    int32_t Mp;          // rows rounded up to a multiple of 64
    int32_t D;           // slots per row (max row degree)
    int32_t dummy;       // variable index of padding slots: multiple of 6, >= N
    const uint32_t *ell; // [D][Mp] variable index of each slot (dummy for padding)
    const int32_t *vc_ptr;   // [N+1] edges of variable n: vc_slot[vc_ptr[n] .. vc_ptr[n+1])
    const uint32_t *vc_slot; // [E] slot index (j*Mp + m) of each edge, ascending m
    const uint32_t *ell_reg; // [regD][regR*1024] index for the register-resident kernel (or null)
    const uint32_t *pk_idx;  // [pkR/2][pkD][T] x {zold_a, zold_b, acc_a, acc_b} LDS byte addresses for the packed
                             // kernel (or null); the set for 16-bit Z_old with 8-bit messages
    const uint32_t *pk_slot; // [N] posterior slot of each variable (packed kernel)
    const uint32_t *pk_shift; // [pkR/2][ceil(ceil(pkD/2)/4)][T] x 4 words: the field shift of each record's
                              // accumulator word, bytes (a, b) of slot 2i and then 2i+1 in word i
};

// Everything a decode kernel needs; passed by value in the kernel arguments.
struct DecodeArgs {
    DevCode c;
    int32_t n_frames;
    int32_t max_iter;
    int32_t early_stop;
    const void *llr_in;      // [F][N] int8 or float
    int32_t a8, b_int;       // fixed-point normalisation: max(((m*a8+128)>>8) - b, 0)
    float alpha, beta;       // binary32 normalisation: max(alpha*m - beta, 0)
    double step;             // LLR value of one fixed-point unit
    uint8_t *hard_out;
    float *llr_out;          // nullable
    int32_t *iters_out;
    uint8_t *ok_out;
    uint8_t *ws;             // caller workspace (device), per-frame stride below
    uint64_t ws_stride;
    // layout plan
    int32_t zpack;           // Z accumulator fields per 32-bit LDS word: 1, 2 or 3
    int32_t zbias;           // packed kernel: bias of each accumulator field (Z + zbias)
    uint32_t off_zold;       // LDS byte offsets
    uint32_t off_zacc;
    uint32_t off_msg;
    uint32_t off_z;
    uint32_t off_aux;
    uint64_t ws_off_msg;     // workspace byte offsets inside one frame's stride
    uint64_t ws_off_z;
    // fixed point: per-iteration (a, b) pairs [wsched_T][2] replacing a8/b_int
    // (null: the constant pair), and the message width
    const float *wsched;
    int32_t wsched_T;
    int32_t qmax;            // Q: extrinsic bound (31, 63, 127)
    int32_t zmax;            // 2Q: bound of the stored Z_old
};

// Fixed-point pair of iteration `it` from the schedule: row min(it, T) - 1,
// a8 = round(256 a), b = round(b / step) (half away from zero, binary64 as
// for the constant pair), clamped to [0, 256] and [0, 255].
__device__ __forceinline__ void sched_pair(const DecodeArgs &a, int it, int &a8, int &b) {
    const int r = min(it, a.wsched_T) - 1;
    const double xa = (double)a.wsched[2 * r] * 256.0;
    const double xb = (double)a.wsched[2 * r + 1] / a.step;
    // clamped in binary64 first (NaN goes to 0), so the conversions are in range
    a8 = __builtin_amdgcn_readfirstlane((int)fmin(fmax(round(xa), 0.0), 256.0));
    b = __builtin_amdgcn_readfirstlane((int)fmin(fmax(round(xb), 0.0), 255.0));
}

struct LaunchCfg {
    int dmax;        // register-array bucket: 8, 16, 32 or 64 slots
    int threads;     // workgroup size (multiple of 64)
    size_t lds;      // dynamic LDS bytes
    bool msg_lds;    // message state in LDS (else workspace)
    bool z_lds;      // posterior array in LDS (else workspace)
};

// Kernel launchers, one per family (defined next to their kernels).
hipError_t launch_ss_int(const DecodeArgs &a, int msg, const LaunchCfg &cfg, hipStream_t s);
hipError_t launch_ss_f32(const DecodeArgs &a, const LaunchCfg &cfg, hipStream_t s);
// binary32 single-scan, frames across lanes; workspace of one call (the
// batch runs in chunks of fl_chunk_frames frames, 0 = code too large)
int fl_chunk_frames(int N, int64_t E);
size_t fl_workspace_bytes(int N, int64_t E, int n_frames, int max_iter);
// frames each lane of that decoder holds (1 or 4) for a call of n_frames
int fl_frames_per_lane(int N, int64_t E, int n_frames, int max_row_deg);
constexpr int kFlThreads = 256;  // threads per workgroup of the frames-across-lanes kernels
// two-scan baseline (int8 or binary32), frames across lanes
int ts_fl_chunk_frames(int N, int64_t E, bool int8);
size_t ts_fl_workspace_bytes(int N, int64_t E, int n_frames, int max_iter, bool int8);
int ts_fl_frames_per_lane(int N, int64_t E, bool int8, int n_frames, int max_row_deg);
hipError_t launch_two_scan_fl(const DecodeArgs &d, bool int8, const int32_t *row_ptr, const uint32_t *row_ent,
                              const uint32_t *vc_csr, int64_t E, int max_row_deg, int cu_count, hipStream_t s);
hipError_t launch_ss_f32_fl(const DecodeArgs &a, const int32_t *row_ptr, const uint32_t *row_ent, int64_t E,
                            int max_row_deg, int cu_count, const float *weights, int weight_iters,
                            const int32_t *row_cls, int n_classes, hipStream_t s);
hipError_t launch_two_scan(const DecodeArgs &a, int msg, const LaunchCfg &cfg, hipStream_t s);
hipError_t launch_ss_reg(const DecodeArgs &a, int msg, int D, int R, int P, size_t lds, hipStream_t s);
// qb: message bits (6; 7 and 8 for INT8 with one or two accumulator fields per word)
hipError_t launch_ss_pk(const DecodeArgs &a, int D, int R, int T, int S, bool onebit, int qb, size_t lds,
                        hipStream_t s);
void pk_shapes(int *out, int cap, int *count);   // (D, R, T, lanes per row) quadruples

// Persistent multi-code launch of the packed kernel (ldpc_decode_multi_persistent).
constexpr int kPersistThreads = 1024;  // threads per workgroup
constexpr int kMaxPersistJobs = 8;
struct PersistJob {
    DecodeArgs a;          // the job's decode arguments
    const uint32_t *recs;  // per-edge records of the workgroup's frame regions: region g at recs + g * rec_words
    uint32_t rec_words;    // 32-bit words of one region's records
    uint32_t region;       // LDS bytes of one frame's region (multiple of 16)
    int32_t shape;         // pk_shape_id() of the job's packed shape
    int32_t first;         // first work item of the job (items are numbered job after job)
};
struct PersistArgs {
    PersistJob job[kMaxPersistJobs];
    int32_t njobs, nitems;  // jobs in use; work items in all (an item: kPersistThreads / T frames of a job)
    int32_t *counter;       // device work-item counter (zeroed by the launcher)
    uint32_t off_item;      // LDS byte offset of the word that hands a work item to the workgroup
};
int pk_shape_id(int D, int R, int T, int S);  // index of an instantiated packed shape, -1 if none
hipError_t launch_ss_pk_persist(const PersistArgs &pa, bool fused, size_t lds, int grid, hipStream_t s);
bool reg_shape_available(int D, int R, int P);
void reg_shapes(int *out, int cap, int *count);  // (D, R, P) triples
constexpr int kRegThreads = 1024;
hipError_t launch_check_input(const void *llr, int64_t count, int msg, int qmax, int32_t *bad,
                              hipStream_t s);

// Launch bound (threads) of each register-array bucket.
__host__ __device__ constexpr int launch_bound_for(int dmax) {
    return dmax <= 16 ? 1024 : (dmax <= 32 ? 512 : 256);
}

}  // namespace ldpc
