// C ABI of the decoder library (declared in include/ldpc.h): code handles,
// argument validation, the per-call layout plan and kernel dispatch.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/ldpc.h"
#include "ldpc_internal.h"

#include "code_handle.h"

namespace {

thread_local std::string g_err;

// LDS per workgroup assumed for host-only handles: one gfx950 CU (160 KiB).
constexpr int kHostOnlyLds = 160 * 1024;
constexpr int kQmax6 = 31;  // Q of the default 6-bit messages

ldpc_status fail(ldpc_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

using ldpc::DeviceGuard;

}  // namespace

// Workspace of ldpc_decode_batch_noalloc: a device global of the code object,
// so every GPU the library runs on holds its own copy (at its own address)
// until the process ends.  Host code never passes this name to a kernel (on
// the host it is only a stand-in); it takes the device address that
// hipGetSymbolAddress returns for the current device (resolve_scratch).
static __device__ __align__(256) uint8_t scratch[LDPC_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device ordinal (null: not yet)

// With `device` current: the device address of that device's `scratch`,
// looked up once per device and kept.
ldpc_status resolve_scratch(int device, void **out) {
    if (device < 0 || device >= kMaxDevices) return fail(LDPC_EUNSUPPORTED, "device ordinal above 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(LDPC_EDEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return LDPC_OK;
}

// Per-call layout plan (which state lives in LDS, which in the workspace).
struct Plan {
    ldpc::LaunchCfg cfg{};
    int family = 0;  // 0: single-scan int8/1-bit, 1: single-scan fp32, 2: two-scan, 3: register-resident,
                     // 4: packed, 5: fp32 frames across lanes, 6: two-scan frames across lanes
    int zpack = 1;
    uint32_t off_zold = 0, off_zacc = 0, off_msg = 0, off_z = 0, off_aux = 0;
    uint64_t ws_off_msg = 0, ws_off_z = 0, ws_stride = 0;
    size_t check_bytes = 0;  // LDPC_F_CHECK_INPUT scratch at the end of the workspace
};

ldpc_status validate_params(const ldpc_decode_params *p) {
    if (!p) return fail(LDPC_EINVAL, "params is NULL");
    if (p->max_iter < 0) return fail(LDPC_EINVAL, "max_iter < 0");
    if (!(p->alpha > 0.0f && p->alpha <= 1.0f)) return fail(LDPC_EINVAL, "alpha outside (0, 1]");
    if (!(p->beta >= 0.0f) || !std::isfinite(p->beta)) return fail(LDPC_EINVAL, "beta < 0 or not finite");
    if (p->msg < LDPC_MSG_FP32 || p->msg > LDPC_MSG_1BIT) return fail(LDPC_EINVAL, "unknown msg type");
    if (p->sched != LDPC_SINGLE_SCAN && p->sched != LDPC_TWO_SCAN)
        return fail(LDPC_EINVAL, "unknown schedule");
    if (p->msg != LDPC_MSG_FP32 && !(p->llr_step > 0.0f && std::isfinite(p->llr_step)))
        return fail(LDPC_EINVAL, "llr_step must be > 0 for fixed-point messages");
    if (p->sched == LDPC_TWO_SCAN && p->msg == LDPC_MSG_1BIT)
        return fail(LDPC_EUNSUPPORTED, "two-scan has no 1-bit form (Sec. V compresses single-scan)");
    const uint32_t layout = (p->flags >> LDPC_F_LAYOUT_SHIFT) & 0xFu;
    if (layout > LDPC_LAYOUT_FRAMES) return fail(LDPC_EINVAL, "unknown layout override");
    if (p->weights && p->weight_iters < 1) return fail(LDPC_EINVAL, "weight_iters must be >= 1 with weights");
    if (p->weight_classes != 0 && p->weight_classes != 1) return fail(LDPC_EINVAL, "weight_classes must be 0 or 1");
    if (p->msg_bits != 0 && (p->msg_bits < 6 || p->msg_bits > 8))
        return fail(LDPC_EINVAL, "msg_bits must be 0, 6, 7 or 8");
    if (p->msg_bits > 6 && (p->msg != LDPC_MSG_INT8 || p->sched != LDPC_SINGLE_SCAN))
        return fail(LDPC_EUNSUPPORTED, "7-8 bit messages: INT8 single-scan only");
    if (p->weights && p->sched != LDPC_SINGLE_SCAN)
        return fail(LDPC_EUNSUPPORTED, "per-iteration weights: single-scan only");
    return LDPC_OK;
}

// Q of the call's fixed-point messages: 2^(b-1) - 1 for b = msg_bits (6 by default).
int qmax_of(const ldpc_decode_params *p) { return (1 << ((p->msg_bits ? p->msg_bits : 6) - 1)) - 1; }

ldpc_status plan_layout(const ldpc_code *c, const ldpc_decode_params *p, uint32_t layout, Plan *pl);

ldpc_status make_plan(const ldpc_code *c, const ldpc_decode_params *p, Plan *pl) {
    const uint32_t layout = (p->flags >> LDPC_F_LAYOUT_SHIFT) & 0xFu;
    if (layout == LDPC_LAYOUT_AUTO && !p->weights) {  // a layout chosen by ldpc_autotune
        const int32_t t = __atomic_load_n(&c->tuned_layout[ldpc::tuned_slot(p)], __ATOMIC_RELAXED);
        if (t > 0) {
            Plan tp;
            if (plan_layout(c, p, (uint32_t)t, &tp) == LDPC_OK) {
                *pl = tp;
                return LDPC_OK;
            }
            g_err.clear();  // the tuned layout cannot run this call: the built-in policy decides
        }
    }
    return plan_layout(c, p, layout, pl);
}

ldpc_status plan_layout(const ldpc_code *c, const ldpc_decode_params *p, uint32_t layout, Plan *pl) {
    const int D = c->D, Mp = c->Mp;
    const size_t nz = (size_t)c->dummy + 1;
    const size_t limit = (size_t)c->lds_limit;
    const size_t aux = 16;
    int dmax = D <= 8 ? 8 : (D <= 16 ? 16 : (D <= 32 ? 32 : 64));
    pl->cfg.dmax = dmax;
    pl->cfg.threads = std::min(ldpc::launch_bound_for(dmax), Mp);
    const bool allow_lds = layout == LDPC_LAYOUT_AUTO || layout == LDPC_LAYOUT_LDS;
    const bool allow_hbm = layout == LDPC_LAYOUT_AUTO || layout == LDPC_LAYOUT_HBM;

    const bool reg_layout = layout == LDPC_LAYOUT_REG || layout == LDPC_LAYOUT_REG1;
    const int qmax = qmax_of(p);
    if (p->weights && p->msg != LDPC_MSG_FP32 && p->weight_classes == 0 && c->learn_classes > 1)
        return fail(LDPC_EUNSUPPORTED,
                    "per-class pairs are FP32 only; fixed point takes one pair per iteration (weight_classes = 1)");
    // 7-8 bit messages: the packed kernel when its accumulator words hold one or
    // two fields (the 10-bit fields of three per word are sized for 6 bits),
    // else the generic LDS/HBM kernel
    const bool wide_pk_ok = p->msg == LDPC_MSG_INT8 && c->pkD > 0 && c->regP <= 2;
    if (qmax != kQmax6 && layout == LDPC_LAYOUT_REG1)
        return fail(LDPC_EUNSUPPORTED, "7-8 bit messages: no one-row register kernel (use REG, LDS or HBM)");
    if (qmax != kQmax6 && layout == LDPC_LAYOUT_REG && !wide_pk_ok)
        return fail(LDPC_EUNSUPPORTED, "7-8 bit messages: this code's packed accumulator has 10-bit fields "
                                       "(three per word); use the LDS/HBM kernel");
    // AUTO for fixed point (measured on MI355X, 50 iterations): the packed
    // two-rows-per-lane kernel pays off from 16 rows per thread (M > 8192),
    // from 8 rows per thread for rows of up to 7 slots (two frames per CU) and
    // for the 1-bit state, for rows wider than 8 slots that fill a wide packed
    // shape (22 slots on a lane pair) and with its 256-thread shapes for small codes; otherwise the
    // one-row register kernel is faster, and other codes of at most 1024
    // checks run best LDS-resident with one thread per row (the register
    // kernels give every frame 1024 threads).
    const bool small_pk = c->pkD > 0 && c->pkT <= 256;  // packed shape with small workgroups
    const bool wide_pk = c->pkD * c->pkS > 8 && 5 * c->D >= 4 * c->pkD * c->pkS;  // wide rows filling >= 80% of the slots
    const bool small_auto = layout == LDPC_LAYOUT_AUTO && c->M <= 1024 && !small_pk;
    if (p->sched == LDPC_SINGLE_SCAN && p->msg != LDPC_MSG_FP32 && !small_auto &&
        (qmax == kQmax6 || wide_pk_ok) && (layout == LDPC_LAYOUT_AUTO || reg_layout)) {
        const bool packed = c->pkD > 0 && layout != LDPC_LAYOUT_REG1 &&
                            (layout == LDPC_LAYOUT_REG || c->pkR >= 16 || wide_pk || small_pk ||
                             (c->pkR >= 8 && (p->msg == LDPC_MSG_1BIT || c->pkD <= 7)));
        const bool ok = packed || (c->regD > 0 && qmax == kQmax6);
        // int16 Z_old for 8-bit messages
        const size_t zold = align_up(nz * (qmax > 63 ? 2 : 1), 16);
        const size_t zacc_pk = align_up(4 * ((size_t)c->dummy / c->regP + 1 + 64), 16);
        if (ok && packed && zold + zacc_pk + aux > limit) {
            if (reg_layout) return fail(LDPC_EUNSUPPORTED, "the packed kernel's LDS state does not fit");
        } else if (ok) {
            pl->family = packed ? 4 : 3;
            // the packed kernel adds 64 private accumulator words for padding slots
            const size_t zacc = align_up(4 * ((size_t)c->dummy / c->regP + 1 + (packed ? 64 : 0)), 16);
            pl->zpack = c->regP;
            pl->off_zold = 0;
            pl->off_zacc = (uint32_t)zold;
            pl->off_aux = (uint32_t)(zold + zacc);
            pl->cfg.lds = zold + zacc + aux;
            pl->cfg.threads = packed ? c->pkT : ldpc::kRegThreads;
            pl->ws_stride = 0;
            return LDPC_OK;
        }
        if (reg_layout)
            return fail(LDPC_EUNSUPPORTED, "no register-resident shape for this code and message type");
    }
    if (reg_layout) return fail(LDPC_EUNSUPPORTED, "register layout is single-scan INT8/1BIT only");
    if (p->weights && p->msg == LDPC_MSG_FP32) {  // the weighted binary32 decoder runs frames across lanes
        if (layout != LDPC_LAYOUT_AUTO && layout != LDPC_LAYOUT_FRAMES)
            return fail(LDPC_EUNSUPPORTED, "per-iteration weights need the frames-across-lanes layout");
        if (ldpc::fl_chunk_frames(c->N, c->E) <= 0)
            return fail(LDPC_EUNSUPPORTED, "code too large for the frames-across-lanes layout");
        pl->family = 5;
        return LDPC_OK;
    }
    if (layout == LDPC_LAYOUT_FRAMES) {
        if (p->sched == LDPC_TWO_SCAN) {
            if (ldpc::ts_fl_chunk_frames(c->N, c->E, p->msg == LDPC_MSG_INT8) <= 0)
                return fail(LDPC_EUNSUPPORTED, "code too large for the frames-across-lanes layout");
            pl->family = 6;
            return LDPC_OK;
        }
        if (p->msg != LDPC_MSG_FP32)
            return fail(LDPC_EUNSUPPORTED, "frames-across-lanes single-scan is FP32 only");
        if (ldpc::fl_chunk_frames(c->N, c->E) <= 0)
            return fail(LDPC_EUNSUPPORTED, "code too large for the frames-across-lanes layout");
        pl->family = 5;
        return LDPC_OK;
    }

    if (p->sched == LDPC_SINGLE_SCAN && p->msg != LDPC_MSG_FP32) {
        pl->family = 0;
        const size_t zold = align_up(nz * (qmax > 63 ? 2 : 1), 16);  // int16 Z_old for 8-bit messages
        const size_t msg = align_up(p->msg == LDPC_MSG_INT8 ? (size_t)D * Mp
                                                             : (size_t)D * (Mp / 64) * 8 + 2 * (size_t)Mp,
                                    16);
        const int span = qmax * (c->max_col_deg + 1);  // bound on |partial Z| (Eq. 3 sums)
        for (int pass = 0; pass < 2; ++pass) {
            const bool msg_lds = pass == 0;
            if ((msg_lds && !allow_lds) || (!msg_lds && !allow_hbm)) continue;
            for (int P = 1; P <= 3; ++P) {
                if (P == 2 && span > 32767) continue;
                if (P == 3 && span > 511) continue;
                const size_t zacc = align_up(4 * ((size_t)c->dummy / P + 1), 16);
                const size_t total = zold + zacc + aux + (msg_lds ? msg : 0);
                if (total > limit) continue;
                pl->zpack = P;
                pl->off_zold = 0;
                pl->off_zacc = (uint32_t)zold;
                pl->off_aux = (uint32_t)(zold + zacc);
                pl->off_msg = (uint32_t)(zold + zacc + aux);
                pl->cfg.lds = total;
                pl->cfg.msg_lds = msg_lds;
                pl->cfg.z_lds = true;
                pl->ws_stride = msg_lds ? 0 : align_up(msg, 256);
                pl->ws_off_msg = 0;
                return LDPC_OK;
            }
        }
        return fail(LDPC_EUNSUPPORTED, "posterior arrays of this code do not fit in LDS");
    }
    // binary32 single-scan and the two-scan baseline: message array + posterior array
    size_t msg, zb;
    if (p->sched == LDPC_SINGLE_SCAN) {
        pl->family = 1;
        msg = align_up((size_t)4 * D * Mp, 16);
        zb = align_up(4 * nz, 16);
        // messages that do not fit on chip stream through HBM frames-across-lanes
        if (layout == LDPC_LAYOUT_AUTO && zb + msg + aux > limit && ldpc::fl_chunk_frames(c->N, c->E) > 0) {
            pl->family = 5;
            return LDPC_OK;
        }
    } else {
        pl->family = 2;
        const size_t esz = p->msg == LDPC_MSG_INT8 ? 1 : 4;
        msg = align_up(2 * esz * (size_t)D * Mp, 16);
        zb = align_up((p->msg == LDPC_MSG_INT8 ? 2 : 4) * nz, 16);
        // per-edge arrays that do not fit on chip stream through HBM frames-across-lanes
        if (layout == LDPC_LAYOUT_AUTO && zb + msg + aux > limit &&
            ldpc::ts_fl_chunk_frames(c->N, c->E, p->msg == LDPC_MSG_INT8) > 0) {
            pl->family = 6;
            return LDPC_OK;
        }
    }
    const bool opts[3][2] = {{true, true}, {false, true}, {false, false}};
    for (auto &o : opts) {
        const bool ml = o[0], zl = o[1];
        if ((ml && !allow_lds) || (!ml && !allow_hbm)) continue;
        const size_t total = (zl ? zb : 0) + (ml ? msg : 0) + aux;
        if (total > limit) continue;
        pl->cfg.msg_lds = ml;
        pl->cfg.z_lds = zl;
        pl->cfg.lds = total;
        pl->off_z = 0;
        pl->off_msg = (uint32_t)(zl ? zb : 0);
        pl->off_aux = (uint32_t)((zl ? zb : 0) + (ml ? msg : 0));
        pl->ws_off_msg = 0;
        pl->ws_off_z = ml ? 0 : align_up(msg, 256);
        pl->ws_stride = align_up((ml ? 0 : align_up(msg, 256)) + (zl ? 0 : zb), 256);
        return LDPC_OK;
    }
    return fail(LDPC_EUNSUPPORTED, "no layout fits the requested override");
}

__global__ void check_input_kernel(const void *llr, int64_t count, int msg, int qmax, int32_t *bad) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        bool b;
        if (msg == ldpc::MSG_FP32) {
            b = !isfinite(static_cast<const float *>(llr)[i]);
        } else {
            const int v = static_cast<const int8_t *>(llr)[i];
            b = v < -qmax || v > qmax;
        }
        if (b) atomicOr(bad, 1);
    }
}

__global__ void zero_word_kernel(int32_t *p) { *p = 0; }

// Bank-aware placement of variables into posterior slots for the packed
// kernel.  Slot s keeps Z_old in LDS byte s (bank (s/4) mod 32) and its
// accumulator in word s/P, field s%P (bank (zacc_off/4 + s/P) mod 32).  Each
// LDS instruction of the row loop touches the variables of one slot of 64
// consecutive rows, served 32 lanes at a time by the 32 banks; the greedy
// gives every variable (highest degree first) the free slot whose two banks
// are least used by the half-wavefronts that will touch it, so each half's 32
// gathers and 32 atomics spread over the banks.
std::vector<uint32_t> pk_slot_assignment(int M, int N, const int32_t *row_ptr, const int32_t *col_idx,
                                         int pkD, int pkR, int T, int S, int P, uint32_t zacc_off) {
    const int RP = pkR / 2, nwave = T / 32;  // half-wavefront groups
    const int ngroups = RP * 2 * pkD * nwave;
    std::vector<int32_t> gptr((size_t)N + 1, 0);
    auto each_edge = [&](auto &&fn) {
        for (int pp = 0; pp < RP; ++pp)
            for (int h = 0; h < 2; ++h)
                for (int j = 0; j < pkD; ++j)
                    for (int w = 0; w < nwave; ++w) {
                        const int g = ((pp * 2 + h) * pkD + j) * nwave + w;
                        for (int l = 0; l < 32; ++l) {
                            // lane w*32+l: row (pp + h*RP)*(T/S) + lane/S, its slots from (lane%S)*pkD
                            const int lane = w * 32 + l;
                            const int m = (pp + h * RP) * (T / S) + lane / S, jr = (lane % S) * pkD + j;
                            if (m < M && jr < row_ptr[m + 1] - row_ptr[m]) fn(col_idx[row_ptr[m] + jr], g);
                        }
                    }
    };
    each_edge([&](int n, int) { gptr[n + 1]++; });
    for (int n = 0; n < N; ++n) gptr[n + 1] += gptr[n];
    std::vector<int32_t> gidx(gptr[N]);
    {
        std::vector<int32_t> fill(gptr.begin(), gptr.end() - 1);
        each_edge([&](int n, int g) { gidx[fill[n]++] = g; });
    }
    std::vector<std::vector<uint32_t>> freel(32 * 32);
    for (int sl = N - 1; sl >= 0; --sl) {
        const int gb = (sl >> 2) & 31, ab = (int)(((zacc_off >> 2) + (uint32_t)sl / (uint32_t)P) & 31u);
        freel[gb * 32 + ab].push_back((uint32_t)sl);
    }
    std::vector<uint16_t> gcnt((size_t)ngroups * 32, 0), acnt((size_t)ngroups * 32, 0);
    std::vector<int32_t> order(N);
    for (int n = 0; n < N; ++n) order[n] = n;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return gptr[a + 1] - gptr[a] > gptr[b + 1] - gptr[b]; });
    std::vector<uint32_t> slot(N);
    for (int v : order) {
        int gs[32] = {0}, as[32] = {0};
        for (int k = gptr[v]; k < gptr[v + 1]; ++k) {
            const uint16_t *gc = &gcnt[(size_t)gidx[k] * 32], *ac = &acnt[(size_t)gidx[k] * 32];
            for (int b = 0; b < 32; ++b) {
                gs[b] += gc[b];
                as[b] += ac[b];
            }
        }
        int best = -1;
        int64_t bestscore = INT64_MAX;
        for (int cb = 0; cb < 1024; ++cb) {
            if (freel[cb].empty()) continue;
            const int64_t sc = (int64_t)(gs[cb >> 5] + as[cb & 31]) * (1 << 20) - (int64_t)freel[cb].size();
            if (sc < bestscore) {
                bestscore = sc;
                best = cb;
            }
        }
        const uint32_t sl = freel[best].back();
        freel[best].pop_back();
        slot[v] = sl;
        for (int k = gptr[v]; k < gptr[v + 1]; ++k) {
            gcnt[(size_t)gidx[k] * 32 + (best >> 5)]++;
            acnt[(size_t)gidx[k] * 32 + (best & 31)]++;
        }
    }
    return slot;
}

// Device workspace of the decode itself, then with the LDPC_F_CHECK_INPUT
// word (256 bytes at the next 256-byte boundary) when that flag is set.
size_t decode_workspace(const ldpc_code *c, const ldpc_decode_params *p, const Plan &pl, int32_t n_frames) {
    return pl.family == 5   ? ldpc::fl_workspace_bytes(c->N, c->E, n_frames, p->max_iter)
           : pl.family == 6 ? ldpc::ts_fl_workspace_bytes(c->N, c->E, n_frames, p->max_iter,
                                                          p->msg == LDPC_MSG_INT8)
                            : (size_t)pl.ws_stride * (size_t)n_frames;
}
size_t total_workspace(const ldpc_code *c, const ldpc_decode_params *p, const Plan &pl, int32_t n_frames) {
    const size_t b = decode_workspace(c, p, pl, n_frames);
    return (p->flags & LDPC_F_CHECK_INPUT) ? align_up(b, 256) + 256 : b;
}

}  // namespace

namespace ldpc {
// error state of the calling thread, for the other entry points of the library
ldpc_status set_error(ldpc_status st, const std::string &msg) { return fail(st, msg); }
void clear_error() { g_err.clear(); }

namespace {
thread_local long g_alloc_count = 0;
}
void reset_alloc_count() { g_alloc_count = 0; }
hipError_t dev_malloc(void **p, size_t bytes) {
    ++g_alloc_count;
    if (const char *f = std::getenv("LDPC_FAIL_ALLOC")) {
        if (std::atol(f) == g_alloc_count) {
            *p = nullptr;
            return hipErrorOutOfMemory;
        }
    }
    return hipMalloc(p, bytes);
}
}  // namespace ldpc

namespace ldpc {
hipError_t launch_check_input(const void *llr, int64_t count, int msg, int qmax, int32_t *bad, hipStream_t s) {
    hipLaunchKernelGGL(zero_word_kernel, dim3(1), dim3(1), 0, s, bad);
    if (count > 0) {
        const int64_t blocks = std::min<int64_t>((count + 255) / 256, 4096);
        hipLaunchKernelGGL(check_input_kernel, dim3((unsigned)blocks), dim3(256), 0, s, llr, count, msg, qmax, bad);
    }
    return hipGetLastError();
}
}  // namespace ldpc

// Host arrays of the packed kernel for shape (Dk slots per lane, R rows per
// thread, T threads, S lanes per row): the slot placement; the per-edge
// records {zold_a, zold_b, acc_a, acc_b} of slot j of rows a = p*T/S + t/S,
// b = (p + R/2)*T/S + t/S (lane t holds the row slots (t%S)*D + j): LDS byte
// addresses of the saturated posterior and of the accumulator word; the set
// for int16 Z_old (7-8 bit messages), and one set per LDS region of the
// persistent launch; and the field shifts of the accumulator words, one byte
// per edge, shared by every set: word i of row pair p holds slots 2i and
// 2i + 1 (bytes: row a, row b, row a, row b), four words per 16-byte entry
// [p][i / 4][t].
struct PkHost {
    std::vector<uint32_t> idx, idx16, grp, slot, shift;
    int groups = 0;
    uint32_t region = 0;
};

static void pk_build_host(const ldpc_code *c, const int32_t *row_ptr, const int32_t *col_idx, int Dk, int R, int T,
                          int S, int lds_dev, PkHost *out) {
    const int M = c->M, N = c->N;
    std::vector<uint32_t> &pk_idx = out->idx, &pk_idx16 = out->idx16, &pk_grp = out->grp, &pk_slot = out->slot;
    const int RP = R / 2, Pk = c->regP;
    const int fbits = Pk == 1 ? 32 : (Pk == 2 ? 16 : 10);
    const uint32_t nwords = (uint32_t)c->dummy / (uint32_t)Pk + 1;
    pk_slot = pk_slot_assignment(M, N, row_ptr, col_idx, Dk, R, T, S, Pk,
                                 (uint32_t)align_up((size_t)c->dummy + 1, 16));
    // zb: bytes per stored Z_old (1; 2 for the int16 Z_old of 8-bit messages,
    // whose accumulator words then start after the wider Z_old array)
    auto build = [&](std::vector<uint32_t> &rec, uint32_t zb) {
        const uint32_t zacc_off = (uint32_t)align_up(((size_t)c->dummy + 1) * zb, 16);
        auto acc_of_slot = [&](uint32_t sl) -> uint32_t {
            return zacc_off + sl / (uint32_t)Pk * 4u;
        };
        rec.assign((size_t)RP * Dk * T * 4, 0u);
        for (int pp = 0; pp < RP; ++pp)
            for (int j = 0; j < Dk; ++j)
                for (int t = 0; t < T; ++t)
                    for (int h = 0; h < 2; ++h) {
                        const int m = (pp + h * RP) * (T / S) + t / S, jr = (t % S) * Dk + j;
                        uint32_t *r = &rec[(((size_t)pp * Dk + j) * T + t) * 4];
                        if (m < M && jr < row_ptr[m + 1] - row_ptr[m]) {
                            const uint32_t sl = pk_slot[col_idx[row_ptr[m] + jr]];
                            r[h] = sl * zb;
                            r[2 + h] = acc_of_slot(sl);
                        } else {  // padding: shared Z_old, a private accumulator word per lane
                            r[h] = (uint32_t)c->dummy * zb;
                            r[2 + h] = zacc_off + (nwords + (uint32_t)(t & 63)) * 4u;
                        }
                    }
    };
    build(pk_idx, 1);
    // field shifts (padding slots: 0, their words are private)
    const int NQ = ((Dk + 1) / 2 + 3) / 4;
    out->shift.assign((size_t)RP * NQ * T * 4, 0u);
    for (int pp = 0; pp < RP; ++pp)
        for (int j = 0; j < Dk; ++j)
            for (int t = 0; t < T; ++t)
                for (int h = 0; h < 2; ++h) {
                    const int m = (pp + h * RP) * (T / S) + t / S, jr = (t % S) * Dk + j;
                    if (m >= M || jr >= row_ptr[m + 1] - row_ptr[m]) continue;
                    const uint32_t sl = pk_slot[col_idx[row_ptr[m] + jr]];
                    const uint32_t sh = sl % (uint32_t)Pk * (uint32_t)fbits;
                    const int i = j / 2;
                    out->shift[(((size_t)pp * NQ + i / 4) * T + t) * 4 + i % 4] |= sh << (8 * (2 * (j % 2) + h));
                }
    // 7-8 bit messages need accumulator fields of 16 bits or more
    if (Pk <= 2) build(pk_idx16, 2);
    // the persistent launch: 1024 / T frames per workgroup, each in its
    // own LDS region of the 6-bit plan's size; one record set per region
    // (the records hold absolute LDS addresses)
    const size_t region = align_up((size_t)c->dummy + 1, 16) +
                          align_up(4 * ((size_t)c->dummy / Pk + 1 + 64), 16) + 16;
    const int G = ldpc::kPersistThreads % T == 0 ? ldpc::kPersistThreads / T : 0;
    if (G >= 1 && (size_t)G * region + 16 <= (size_t)lds_dev) {
        out->groups = G;
        out->region = (uint32_t)region;
        if (G > 1) {
            std::vector<uint32_t> one;
            build(one, 1);
            pk_grp.reserve(one.size() * G);
            for (int g = 0; g < G; ++g) {
                const uint32_t off = (uint32_t)(g * region);
                for (size_t i = 0; i < one.size(); i += 4) {
                    pk_grp.push_back(one[i] + off);
                    pk_grp.push_back(one[i + 1] + off);
                    pk_grp.push_back(one[i + 2] + off);
                    pk_grp.push_back(one[i + 3] + off);
                }
            }
        }
    }
}

// Device copies of a packed shape's host arrays, replacing the handle's
// previous ones (freed) on success; on failure the handle keeps its arrays
// and whatever was allocated here is freed.  The device is current.
static ldpc_status pk_upload(ldpc_code *c, const PkHost &h) {
    uint32_t *di = nullptr, *di16 = nullptr, *dg = nullptr, *ds = nullptr, *dh = nullptr;
    hipError_t e = ldpc::dev_malloc((void **)&di, h.idx.size() * sizeof(uint32_t));
    if (e == hipSuccess) e = ldpc::dev_malloc((void **)&ds, h.slot.size() * sizeof(uint32_t));
    if (e == hipSuccess) e = ldpc::dev_malloc((void **)&dh, h.shift.size() * sizeof(uint32_t));
    if (e == hipSuccess && !h.idx16.empty()) e = ldpc::dev_malloc((void **)&di16, h.idx16.size() * sizeof(uint32_t));
    if (e == hipSuccess && !h.grp.empty()) e = ldpc::dev_malloc((void **)&dg, h.grp.size() * sizeof(uint32_t));
    const bool allocated = e == hipSuccess;
    if (allocated) e = hipMemcpy(di, h.idx.data(), h.idx.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ds, h.slot.data(), h.slot.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dh, h.shift.data(), h.shift.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess && di16)
        e = hipMemcpy(di16, h.idx16.data(), h.idx16.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess && dg) e = hipMemcpy(dg, h.grp.data(), h.grp.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        for (uint32_t *q : {di, di16, dg, ds, dh})
            if (q) (void)hipFree(q);
        (void)hipGetLastError();
        return allocated ? fail(LDPC_EDEVICE, "copy of the packed layout to the device failed")
                         : fail(LDPC_ENOMEM, "device allocation failed");
    }
    for (uint32_t *q : {c->d_pk_idx, c->d_pk_idx16, c->d_pk_grp, c->d_pk_slot, c->d_pk_shift})
        if (q) (void)hipFree(q);
    c->d_pk_shift = dh;
    c->d_pk_idx = di;
    c->d_pk_idx16 = di16;
    c->d_pk_grp = dg;
    c->d_pk_slot = ds;
    c->pkGroups = h.groups;
    c->pkRegion = h.region;
    return LDPC_OK;
}

namespace ldpc {

std::vector<std::array<int, 4>> pk_candidates(const ldpc_code *c) {
    std::vector<std::array<int, 4>> out;
    if (c->pkD <= 0) return out;
    out.push_back({c->pkD, c->pkR, c->pkT, c->pkS});
    int pks[4 * 64], n = 0;
    pk_shapes(pks, 64, &n);
    n = std::min(n, 64);
    // per (threads, lanes per row): the covering shape with the fewest slots,
    // then the fewest rows per thread (more of either is padding only); rows
    // padded to more than twice max(D, 8) slots are not tried, nor lane pairs
    // for rows that fit one lane
    for (int i = 0; i < n; ++i) {
        const int d = pks[4 * i], r = pks[4 * i + 1], t = pks[4 * i + 2], l = pks[4 * i + 3];
        if (d * l < c->D || (int64_t)r * (t / l) < c->M || d * l > 2 * std::max(c->D, 8)) continue;
        if (l > 1 && d >= c->D) continue;
        bool best = true;
        for (int k = 0; k < n && best; ++k) {
            const int d2 = pks[4 * k], r2 = pks[4 * k + 1], t2 = pks[4 * k + 2], l2 = pks[4 * k + 3];
            if (k == i || t2 != t || l2 != l || d2 * l2 < c->D || (int64_t)r2 * (t2 / l2) < c->M) continue;
            if (d2 < d || (d2 == d && r2 < r)) best = false;
        }
        if (!best || (d == c->pkD && r == c->pkR && t == c->pkT && l == c->pkS)) continue;
        out.push_back({d, r, t, l});
    }
    return out;
}

ldpc_status pk_install(ldpc_code *c, int D, int R, int T, int S) {
    if (c->device < 0) return fail(LDPC_EINVAL, "host-only handle");
    PkHost h;
    pk_build_host(c, c->h_row_ptr.data(), c->h_col_idx.data(), D, R, T, S, c->lds_limit, &h);
    DeviceGuard g(c->device);
    if (!g.ok) return fail(LDPC_EDEVICE, "hipSetDevice failed");
    const ldpc_status st = pk_upload(c, h);
    if (st != LDPC_OK) return st;
    c->pkD = D;
    c->pkR = R;
    c->pkT = T;
    c->pkS = S;
    return LDPC_OK;
}

}  // namespace ldpc

extern "C" {

const char *ldpc_last_error(void) { return g_err.c_str(); }

const char *ldpc_version(void) { return "ldpc-singlescan-gfx950 0.1"; }

ldpc_status ldpc_code_create(int32_t M, int32_t N, int64_t nnz, const int32_t *row_ptr,
                             const int32_t *col_idx, int32_t device, ldpc_code **out) {
    if (!out) return fail(LDPC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!row_ptr || (nnz > 0 && !col_idx)) return fail(LDPC_EINVAL, "row_ptr/col_idx is NULL");
    if (M < 1 || N < 1) return fail(LDPC_EBADCODE, "M and N must be >= 1");
    if (N > (1 << 30)) return fail(LDPC_EUNSUPPORTED, "N too large");
    if (row_ptr[0] != 0 || (int64_t)row_ptr[M] != nnz) return fail(LDPC_EBADCODE, "row_ptr[0] != 0 or row_ptr[M] != nnz");
    int D = 0, dmin = 1 << 30;
    std::vector<int32_t> row_cols;
    for (int m = 0; m < M; ++m) {
        const int d = row_ptr[m + 1] - row_ptr[m];
        if (d < 0) return fail(LDPC_EBADCODE, "row_ptr decreases at row " + std::to_string(m));
        if (d < 2) return fail(LDPC_EBADCODE, "row " + std::to_string(m) + " has degree < 2");
        D = std::max(D, d);
        dmin = std::min(dmin, d);
        row_cols.assign(col_idx + row_ptr[m], col_idx + row_ptr[m + 1]);
        std::sort(row_cols.begin(), row_cols.end());
        for (int j = 0; j < d; ++j) {
            if (row_cols[j] < 0 || row_cols[j] >= N)
                return fail(LDPC_EBADCODE, "column index out of range in row " + std::to_string(m));
            if (j > 0 && row_cols[j] == row_cols[j - 1])
                return fail(LDPC_EBADCODE, "duplicate column in row " + std::to_string(m));
        }
    }
    if (D > 64) return fail(LDPC_EUNSUPPORTED, "row degree above 64");

    ldpc_code *c = new ldpc_code();
    c->device = device;
    c->M = M;
    c->N = N;
    c->E = nnz;
    c->D = D;
    c->Mp = (M + 63) / 64 * 64;
    c->dummy = (N + 5) / 6 * 6;
    c->min_row_deg = dmin;
    c->h_row_ptr.assign(row_ptr, row_ptr + M + 1);
    c->h_col_idx.assign(col_idx, col_idx + nnz);
    ldpc::analyse_code(M, N, row_ptr, col_idx, &c->facts);
    std::vector<int32_t> row_cls(M);
    {
        std::vector<int32_t> degs(M);
        for (int m = 0; m < M; ++m) degs[m] = row_ptr[m + 1] - row_ptr[m];
        c->learn_degrees = degs;
        std::sort(c->learn_degrees.begin(), c->learn_degrees.end());
        c->learn_degrees.erase(std::unique(c->learn_degrees.begin(), c->learn_degrees.end()), c->learn_degrees.end());
        c->learn_classes = (int32_t)c->learn_degrees.size();
        for (int m = 0; m < M; ++m)
            row_cls[m] = (int32_t)(std::lower_bound(c->learn_degrees.begin(), c->learn_degrees.end(), degs[m]) -
                                   c->learn_degrees.begin());
    }
    const size_t slots = (size_t)c->D * c->Mp;
    std::vector<uint32_t> ell(slots, (uint32_t)c->dummy);
    std::vector<int32_t> vc_ptr((size_t)N + 1, 0);
    for (int64_t e = 0; e < nnz; ++e) vc_ptr[col_idx[e] + 1]++;
    for (int n = 0; n < N; ++n) {
        c->max_col_deg = std::max(c->max_col_deg, vc_ptr[n + 1]);
        vc_ptr[n + 1] += vc_ptr[n];
    }
    std::vector<uint32_t> vc_slot((size_t)std::max<int64_t>(nnz, 1));
    // + 64 padding entries (variable 0, position 0): a row's slots load unconditionally
    std::vector<uint32_t> row_ent((size_t)2 * (nnz + 64), 0u);
    std::vector<uint32_t> vc_csr((size_t)nnz + 64, 0u);
    std::vector<int32_t> fill(vc_ptr.begin(), vc_ptr.end() - 1);
    for (int m = 0; m < M; ++m)
        for (int j = 0; j < row_ptr[m + 1] - row_ptr[m]; ++j) {
            const int n = col_idx[row_ptr[m] + j];
            const uint32_t slot = (uint32_t)((size_t)j * c->Mp + m);
            ell[slot] = (uint32_t)n;
            row_ent[2 * (size_t)(row_ptr[m] + j)] = (uint32_t)n;
            row_ent[2 * (size_t)(row_ptr[m] + j) + 1] = (uint32_t)fill[n];
            vc_csr[fill[n]] = (uint32_t)(row_ptr[m] + j);
            vc_slot[fill[n]++] = slot;  // rows visited in ascending order
        }

    // register-resident shape: smallest instantiated (slots, rows/thread, packing)
    // covering the code whose posterior arrays fit the LDS budget
    int lds_dev = kHostOnlyLds;
    if (device >= 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && v > 0)
            lds_dev = v;
    }
    {
        int shapes[3 * 64], cnt = 0;
        ldpc::reg_shapes(shapes, 64, &cnt);
        const int span = 31 * (c->max_col_deg + 1);
        int bestD = 1 << 30, bestR = 1 << 30, bestP = 0;
        for (int i = 0; i < cnt && i < 64; ++i) {
            const int d = shapes[3 * i], r = shapes[3 * i + 1], pk = shapes[3 * i + 2];
            if (d < D || (int64_t)r * ldpc::kRegThreads < M) continue;
            if (pk == 2 && span > 32767) continue;
            if (pk == 3 && (span > 511 || c->dummy + 1 >= 98303)) continue;
            const size_t need = align_up((size_t)c->dummy + 1, 16) +
                                align_up(4 * ((size_t)c->dummy / pk + 1), 16) + 16;
            if (need > (size_t)lds_dev) continue;
            if (d < bestD || (d == bestD && r < bestR) || (d == bestD && r == bestR && pk < bestP)) {
                bestD = d;
                bestR = r;
                bestP = pk;
            }
        }
        if (bestP) {
            c->regD = bestD;
            c->regR = bestR;
            c->regP = bestP;
            // packed kernel: any instantiated (slots, even rows/thread) covering the
            // code; its accumulator addressing comes from the per-edge records
            int pks[4 * 64], pcnt = 0;
            ldpc::pk_shapes(pks, 64, &pcnt);
            int pD = 1 << 30, pR = 1 << 30, pT = 0, pS = 1;
            // it also keeps 64 private accumulator words for padding slots
            const size_t need_pk = align_up((size_t)c->dummy + 1, 16) +
                                   align_up(4 * ((size_t)c->dummy / bestP + 1 + 64), 16) + 16;
            // rows of more than 16 entries on a lane pair when a shape allows it
            // (512 threads, two frames per CU, instead of 768), other rows on one
            // lane; then fewest
            // slots per row, fewest padded rows, fewest rows per thread
            auto rank = [&](int d, int r, int t, int l) {
                return std::make_tuple((D > 16) == (l == 2) ? 0 : 1, d * l, (int64_t)r * (t / l), r);
            };
            for (int i = 0; i < pcnt && i < 64 && need_pk <= (size_t)lds_dev; ++i) {
                const int d = pks[4 * i], r = pks[4 * i + 1], t = pks[4 * i + 2], l = pks[4 * i + 3];
                if (d * l < D || (int64_t)r * (t / l) < M) continue;
                if (pT == 0 || rank(d, r, t, l) < rank(pD, pR, pT, pS)) {
                    pD = d;
                    pR = r;
                    pT = t;
                    pS = l;
                }
            }
            // 10-bit fields are biased by 319 or 575 (both 63 mod 256: the low
            // byte of a field clamped to bias +- 62 is then Z_old + 63)
            const int pbias = bestP == 1 ? 0 : bestP == 2 ? 32768 : span <= 319 ? 319 : span <= 448 ? 575 : -1;
            if (pD < (1 << 30) && pbias >= 0) {
                c->pkD = pD;
                c->pkR = pR;
                c->pkT = pT;
                c->pkS = pS;
                c->pkBias = pbias;
            }
        }
    }
    // host-side layouts of the register kernels (built for host-only handles
    // too, so that planning and the host checks cover the same code)
    std::vector<uint32_t> ell_reg;
    if (c->regD > 0) {
        const size_t Mr = (size_t)c->regR * ldpc::kRegThreads;
        ell_reg.assign((size_t)c->regD * Mr, (uint32_t)c->dummy);
        for (int m = 0; m < M; ++m)
            for (int j = 0; j < row_ptr[m + 1] - row_ptr[m]; ++j)
                ell_reg[(size_t)j * Mr + m] = (uint32_t)col_idx[row_ptr[m] + j];
    }
    PkHost pkh;
    if (c->pkD > 0) {
        pk_build_host(c, row_ptr, col_idx, c->pkD, c->pkR, c->pkT, c->pkS, lds_dev, &pkh);
        c->pkGroups = pkh.groups;
        c->pkRegion = pkh.region;
    }
    if (device < 0) {  // host-only handle: planning and queries, no decoding
        c->lds_limit = kHostOnlyLds;
        *out = c;
        g_err.clear();
        return LDPC_OK;
    }
    DeviceGuard g(device);
    if (!g.ok) {
        delete c;
        return fail(LDPC_EDEVICE, "hipSetDevice failed");
    }
    if (device < kMaxDevices) {  // the allocation-free entry point's scratch: resolved once per device
        void *sp = nullptr;
        if (resolve_scratch(device, &sp) != LDPC_OK) {
            delete c;
            return LDPC_EDEVICE;
        }
    }
    ldpc::reset_alloc_count();
    int lds = 0, cus = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
        c->lds_limit = lds;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        c->cu_count = cus;
    hipError_t e1 = ldpc::dev_malloc((void **)&c->d_ell, slots * sizeof(uint32_t));
    hipError_t e7 = ldpc::dev_malloc((void **)&c->d_row_ptr, ((size_t)M + 1) * sizeof(int32_t));
    hipError_t e8 = ldpc::dev_malloc((void **)&c->d_row_ent, row_ent.size() * sizeof(uint32_t));
    hipError_t e9 = ldpc::dev_malloc((void **)&c->d_vc_csr, vc_csr.size() * sizeof(uint32_t));
    hipError_t e10 = ldpc::dev_malloc((void **)&c->d_row_cls, sizeof(int32_t) * std::max<size_t>(row_cls.size(), 1));
    hipError_t e2 = ldpc::dev_malloc((void **)&c->d_vc_ptr, vc_ptr.size() * sizeof(int32_t));
    hipError_t e3 = ldpc::dev_malloc((void **)&c->d_vc_slot, vc_slot.size() * sizeof(uint32_t));
    hipError_t e4 = hipSuccess;
    if (!ell_reg.empty()) e4 = ldpc::dev_malloc((void **)&c->d_ell_reg, ell_reg.size() * sizeof(uint32_t));
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess || e7 != hipSuccess ||
        e8 != hipSuccess || e9 != hipSuccess || e10 != hipSuccess) {
        ldpc_code_destroy(c);
        (void)hipGetLastError();
        return fail(LDPC_ENOMEM, "device allocation failed");
    }
    if (hipMemcpy(c->d_ell, ell.data(), slots * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->d_vc_ptr, vc_ptr.data(), vc_ptr.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->d_vc_slot, vc_slot.data(), vc_slot.size() * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->d_row_ptr, row_ptr, ((size_t)M + 1) * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->d_row_ent, row_ent.data(), row_ent.size() * sizeof(uint32_t), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(c->d_vc_csr, vc_csr.data(), vc_csr.size() * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->d_row_cls, row_cls.data(), sizeof(int32_t) * row_cls.size(), hipMemcpyHostToDevice) !=
            hipSuccess ||
        (c->d_ell_reg && hipMemcpy(c->d_ell_reg, ell_reg.data(), ell_reg.size() * sizeof(uint32_t),
                                   hipMemcpyHostToDevice) != hipSuccess)) {
        ldpc_code_destroy(c);
        return fail(LDPC_EDEVICE, "copy of the code to the device failed");
    }
    if (c->pkD > 0) {
        const ldpc_status st = pk_upload(c, pkh);
        if (st != LDPC_OK) {
            const std::string msg = g_err;
            ldpc_code_destroy(c);
            return fail(st, msg);
        }
    }
    *out = c;
    g_err.clear();
    return LDPC_OK;
}

ldpc_status ldpc_code_destroy(ldpc_code *code) {
    if (!code) return LDPC_OK;
    if (code->device < 0) {
        delete code;
        return LDPC_OK;
    }
    DeviceGuard g(code->device);
    if (code->d_ell) (void)hipFree(code->d_ell);
    if (code->d_vc_ptr) (void)hipFree(code->d_vc_ptr);
    if (code->d_vc_slot) (void)hipFree(code->d_vc_slot);
    if (code->d_row_ptr) (void)hipFree(code->d_row_ptr);
    if (code->d_row_ent) (void)hipFree(code->d_row_ent);
    if (code->d_vc_csr) (void)hipFree(code->d_vc_csr);
    if (code->d_info_pos) (void)hipFree(code->d_info_pos);
    if (code->d_row_cls) (void)hipFree(code->d_row_cls);
    if (code->d_enc_rows) (void)hipFree(code->d_enc_rows);
    if (code->d_ell_reg) (void)hipFree(code->d_ell_reg);
    if (code->d_pk_idx) (void)hipFree(code->d_pk_idx);
    if (code->d_pk_idx16) (void)hipFree(code->d_pk_idx16);
    if (code->d_pk_grp) (void)hipFree(code->d_pk_grp);
    if (code->d_pk_slot) (void)hipFree(code->d_pk_slot);
    if (code->d_pk_shift) (void)hipFree(code->d_pk_shift);
    delete code;
    return LDPC_OK;
}

ldpc_status ldpc_code_query(const ldpc_code *c, ldpc_code_info *o) {
    if (!c || !o) return fail(LDPC_EINVAL, "NULL argument");
    std::memset(o, 0, sizeof(*o));
    o->M = c->M;
    o->N = c->N;
    o->E = c->E;
    o->min_row_deg = c->min_row_deg;
    o->max_row_deg = c->D;
    o->max_col_deg = c->max_col_deg;
    o->slots_per_row = c->D;
    o->rows_padded = c->Mp;
    o->device = c->device;
    o->addr_bytes_single = c->E * 4;
    o->addr_bytes_two = c->E * 8;
    o->msg_bits_int8 = c->E * 8;
    int lg = 0;
    while ((1 << lg) < c->D) ++lg;
    o->msg_bits_1bit = c->E + (int64_t)c->M * (5 + 5 + lg);
    o->lds_bytes_per_cu = c->lds_limit;
    o->reg_slots = c->regD;
    o->reg_rows_per_thread = c->regR;
    o->reg_zpack = c->regP;
    o->pk_slots = c->pkD;
    o->pk_rows_per_thread = c->pkR;
    o->pk_threads = c->pkT;
    for (int d = 0; d <= 64; ++d) {
        o->row_deg_hist[d] = c->facts.row_hist[d];
        o->col_deg_hist[d] = c->facts.col_hist[d];
    }
    o->structure = c->facts.structure;
    o->qc_lift = c->facts.qc_lift;
    o->ira_group = c->facts.ira_group;
    const int64_t E = c->E, N = c->N, M = c->M, Eb = (E + 7) / 8;
    o->var_values_single = N;
    o->var_values_two = E;
    o->msg_bytes_int8 = E;
    o->msg_bytes_1bit = Eb + 2 * M;
    o->msg_bytes_fp32 = 4 * E;
    o->post_bytes_int = 2 * N;
    o->post_bytes_fp32 = 4 * N;
    o->stream_bytes_int8 = 2 * E + 5 * N;
    o->stream_bytes_1bit = 2 * Eb + 4 * M + 5 * N;
    o->stream_bytes_fp32 = 8 * E + 12 * N;
    o->stream_bytes_two_int8 = 4 * E + 3 * N;
    o->stream_bytes_two_fp32 = 16 * E + 8 * N;
    return LDPC_OK;
}

ldpc_status ldpc_decode_workspace_size(const ldpc_code *c, int32_t n_frames,
                                       const ldpc_decode_params *p, size_t *bytes) {
    if (!c || !bytes) return fail(LDPC_EINVAL, "NULL argument");
    if (n_frames < 0) return fail(LDPC_EINVAL, "n_frames < 0");
    ldpc_status st = validate_params(p);
    if (st != LDPC_OK) return st;
    Plan pl;
    st = make_plan(c, p, &pl);
    if (st != LDPC_OK) return st;
    *bytes = total_workspace(c, p, pl, n_frames);
    return LDPC_OK;
}

ldpc_status ldpc_decode_plan(const ldpc_code *c, int32_t n_frames, const ldpc_decode_params *p,
                             ldpc_plan_info *out) {
    if (!c || !out) return fail(LDPC_EINVAL, "NULL argument");
    if (n_frames < 0) return fail(LDPC_EINVAL, "n_frames < 0");
    ldpc_status st = validate_params(p);
    if (st != LDPC_OK) return st;
    Plan pl;
    st = make_plan(c, p, &pl);
    if (st != LDPC_OK) return st;
    ldpc_plan_info o{};
    o.kernel = pl.family;  // the ldpc_kernel values are the plan families
    const bool frames = pl.family == 5 || pl.family == 6;
    o.layout = pl.family == 4 ? LDPC_LAYOUT_REG
               : pl.family == 3 ? LDPC_LAYOUT_REG1
               : frames         ? LDPC_LAYOUT_FRAMES
               : pl.cfg.msg_lds ? LDPC_LAYOUT_LDS
                                : LDPC_LAYOUT_HBM;
    o.threads = frames ? ldpc::kFlThreads : pl.cfg.threads;
    o.lds_bytes = frames ? 0 : (int32_t)pl.cfg.lds;
    o.frames_per_lane =
        pl.family == 5   ? ldpc::fl_frames_per_lane(c->N, c->E, n_frames, c->D)
        : pl.family == 6 ? ldpc::ts_fl_frames_per_lane(c->N, c->E, p->msg == LDPC_MSG_INT8, n_frames, c->D)
                         : 0;
    o.workspace_bytes = total_workspace(c, p, pl, n_frames);
    *out = o;
    return LDPC_OK;
}

ldpc_status ldpc_decode_batch(const ldpc_code *c, int32_t n_frames, const void *llr_in,
                              const ldpc_decode_params *p, uint8_t *hard_out, float *llr_out,
                              int32_t *iters_out, uint8_t *syndrome_ok, void *workspace,
                              size_t workspace_bytes, void *stream) {
    return ldpc::decode_job(c, n_frames, llr_in, p, hard_out, llr_out, iters_out, syndrome_ok, workspace,
                            workspace_bytes, stream, true);
}

ldpc_status ldpc_decode_batch_noalloc(const ldpc_code *c, int32_t n_frames, const void *llr_in,
                                      const ldpc_decode_params *p, uint8_t *hard_out, float *llr_out,
                                      int32_t *iters_out, uint8_t *syndrome_ok, void *stream) {
    if (!c) return fail(LDPC_EINVAL, "code is NULL");
    size_t need = 0;
    ldpc_status st = ldpc_decode_workspace_size(c, n_frames, p, &need);
    if (st != LDPC_OK) return st;
    if (need > (size_t)LDPC_NOALLOC_SCRATCH_BYTES)
        return fail(LDPC_EUNSUPPORTED, "the call needs " + std::to_string(need) +
                                           " bytes of workspace; the static scratch holds " +
                                           std::to_string((size_t)LDPC_NOALLOC_SCRATCH_BYTES) +
                                           " (use ldpc_decode_batch with a workspace, or fewer frames)");
    if (c->device < 0) return fail(LDPC_EINVAL, "host-only handle (device < 0) cannot decode");
    void *ws = nullptr;
    if (need > 0) {
        DeviceGuard g(c->device);
        if (!g.ok) return fail(LDPC_EDEVICE, "hipSetDevice failed");
        st = resolve_scratch(c->device, &ws);
        if (st != LDPC_OK) return st;
    }
    return ldpc::decode_job(c, n_frames, llr_in, p, hard_out, llr_out, iters_out, syndrome_ok, ws,
                            ws ? (size_t)LDPC_NOALLOC_SCRATCH_BYTES : 0, stream, true);
}

}  // extern "C"

namespace {
// The kernel arguments of one decode call (plan already made).
void fill_args(const ldpc_code *c, int32_t n_frames, const void *llr_in, const ldpc_decode_params *p, const Plan &pl,
               uint8_t *hard_out, float *llr_out, int32_t *iters_out, uint8_t *syndrome_ok, void *workspace,
               ldpc::DecodeArgs *out) {
    ldpc::DecodeArgs &a = *out;
    a.c.M = c->M;
    a.c.N = c->N;
    a.c.Mp = c->Mp;
    a.c.D = c->D;
    a.c.dummy = c->dummy;
    a.c.ell = c->d_ell;
    a.c.vc_ptr = c->d_vc_ptr;
    a.c.vc_slot = c->d_vc_slot;
    a.c.ell_reg = c->d_ell_reg;
    a.c.pk_idx = qmax_of(p) > 63 ? c->d_pk_idx16 : c->d_pk_idx;  // int16 Z_old for 8-bit messages
    a.c.pk_slot = c->d_pk_slot;
    a.c.pk_shift = c->d_pk_shift;
    a.n_frames = n_frames;
    a.max_iter = p->max_iter;
    a.early_stop = p->early_stop ? 1 : 0;
    a.llr_in = llr_in;
    a.a8 = (int32_t)std::lround((double)p->alpha * 256.0);
    // offsets of 255 steps and more all zero every b-bit message (b <= 8):
    // capped there so that the conversion stays in range
    a.b_int = p->msg == LDPC_MSG_FP32
                  ? 0
                  : (int32_t)std::lround(std::fmin((double)p->beta / (double)p->llr_step, 255.0));
    a.alpha = p->alpha;
    a.beta = p->beta;
    a.step = (double)p->llr_step;
    a.hard_out = hard_out;
    a.llr_out = llr_out;
    a.iters_out = iters_out;
    a.ok_out = syndrome_ok;
    a.ws = static_cast<uint8_t *>(workspace);
    a.ws_stride = pl.ws_stride;
    a.zpack = pl.zpack;
    a.zbias = c->pkBias;
    a.off_zold = pl.off_zold;
    a.off_zacc = pl.off_zacc;
    a.off_msg = pl.off_msg;
    a.off_z = pl.off_z;
    a.off_aux = pl.off_aux;
    a.ws_off_msg = pl.ws_off_msg;
    a.ws_off_z = pl.ws_off_z;
    a.wsched = p->msg == LDPC_MSG_FP32 ? nullptr : p->weights;  // binary32 takes its pairs below
    a.wsched_T = p->weight_iters;
    a.qmax = qmax_of(p);
    a.zmax = 2 * a.qmax;
}
}  // namespace

namespace ldpc {

ldpc_status decode_job(const ldpc_code *c, int32_t n_frames, const void *llr_in, const ldpc_decode_params *p,
                       uint8_t *hard_out, float *llr_out, int32_t *iters_out, uint8_t *syndrome_ok,
                       void *workspace, size_t workspace_bytes, void *stream, bool launch) {
    if (!c) return fail(LDPC_EINVAL, "code is NULL");
    if (n_frames < 0) return fail(LDPC_EINVAL, "n_frames < 0");
    ldpc_status st = validate_params(p);
    if (st != LDPC_OK) return st;
    if (n_frames > 0 && (!llr_in || !hard_out || !iters_out || !syndrome_ok))
        return fail(LDPC_EINVAL, "llr_in, hard_out, iters_out and syndrome_ok are required");
    Plan pl;
    st = make_plan(c, p, &pl);
    if (st != LDPC_OK) return st;
    const size_t check_off = align_up(decode_workspace(c, p, pl, n_frames), 256);
    const size_t need = total_workspace(c, p, pl, n_frames);
    if (need > 0 && (!workspace || workspace_bytes < need))
        return fail(LDPC_EINVAL, "workspace missing or smaller than ldpc_decode_workspace_size()");
    if (workspace && (reinterpret_cast<uintptr_t>(workspace) & 255u))
        return fail(LDPC_EINVAL, "workspace must be 256-byte aligned");
    if (c->device < 0) return fail(LDPC_EINVAL, "host-only handle (device < 0) cannot decode");
    if (n_frames == 0 || !launch) return LDPC_OK;

    DeviceGuard g(c->device);
    if (!g.ok) return fail(LDPC_EDEVICE, "hipSetDevice failed");
    hipStream_t s = static_cast<hipStream_t>(stream);

    if (p->flags & LDPC_F_CHECK_INPUT) {
        int32_t *bad = reinterpret_cast<int32_t *>(static_cast<uint8_t *>(workspace) + check_off);
        hipError_t e = ldpc::launch_check_input(llr_in, (int64_t)n_frames * c->N, p->msg, qmax_of(p), bad, s);
        int32_t hbad = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return fail(LDPC_EDEVICE, std::string("input check failed: ") + hipGetErrorString(e));
        if (hbad) return fail(LDPC_EINVAL, "llr_in holds non-finite or out-of-range values");
    }

    ldpc::DecodeArgs a{};
    fill_args(c, n_frames, llr_in, p, pl, hard_out, llr_out, iters_out, syndrome_ok, workspace, &a);

    hipError_t e;
    if (pl.family == 0)
        e = ldpc::launch_ss_int(a, p->msg, pl.cfg, s);
    else if (pl.family == 3)
        e = ldpc::launch_ss_reg(a, p->msg, c->regD, c->regR, c->regP, pl.cfg.lds, s);
    else if (pl.family == 4)
        e = ldpc::launch_ss_pk(a, c->pkD, c->pkR, c->pkT, c->pkS, p->msg == LDPC_MSG_1BIT,
                               p->msg_bits ? p->msg_bits : 6, pl.cfg.lds, s);
    else if (pl.family == 1)
        e = ldpc::launch_ss_f32(a, pl.cfg, s);
    else if (pl.family == 6)
        e = ldpc::launch_two_scan_fl(a, p->msg == LDPC_MSG_INT8, c->d_row_ptr, c->d_row_ent, c->d_vc_csr, c->E,
                                     c->D, c->cu_count, s);
    else if (pl.family == 5)
        e = ldpc::launch_ss_f32_fl(a, c->d_row_ptr, c->d_row_ent, c->E, c->D, c->cu_count, p->weights,
                                   p->weight_iters, c->d_row_cls, p->weight_classes == 1 ? 1 : c->learn_classes, s);
    else
        e = ldpc::launch_two_scan(a, p->msg, pl.cfg, s);
    if (e != hipSuccess) return fail(LDPC_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return LDPC_OK;
}


ldpc_status persist_job(const ldpc_code *c, int32_t n_frames, const void *llr_in, const ldpc_decode_params *p,
                        uint8_t *hard_out, float *llr_out, int32_t *iters_out, uint8_t *syndrome_ok,
                        PersistJob *out) {
    if (!c) return fail(LDPC_EINVAL, "code is NULL");
    ldpc_status st = validate_params(p);
    if (st != LDPC_OK) return st;
    if (p->msg != LDPC_MSG_INT8 || p->sched != LDPC_SINGLE_SCAN || qmax_of(p) != kQmax6)
        return fail(LDPC_EUNSUPPORTED, "the persistent launch runs 6-bit int8 single-scan only");
    Plan pl;
    st = make_plan(c, p, &pl);
    if (st != LDPC_OK) return st;
    const int shape = pk_shape_id(c->pkD, c->pkR, c->pkT, c->pkS);
    if (pl.family != 4 || c->pkGroups < 1 || shape < 0)
        return fail(LDPC_EUNSUPPORTED, "the persistent launch needs the packed kernel with a shape of 256, 512 "
                                       "or 1024 threads (this call plans another kernel)");
    // the remaining checks of a decode call (the packed kernel needs no workspace)
    st = decode_job(c, n_frames, llr_in, p, hard_out, llr_out, iters_out, syndrome_ok, nullptr, 0, nullptr, false);
    if (st != LDPC_OK) return st;
    if ((size_t)c->pkRegion != align_up(pl.cfg.lds, 16))
        return fail(LDPC_EUNSUPPORTED, "persistent launch: LDS region mismatch");
    PersistJob &j = *out;
    j = PersistJob{};
    fill_args(c, n_frames, llr_in, p, pl, hard_out, llr_out, iters_out, syndrome_ok, nullptr, &j.a);
    j.recs = c->pkGroups > 1 ? c->d_pk_grp : c->d_pk_idx;
    j.rec_words = (uint32_t)((size_t)(c->pkR / 2) * c->pkD * c->pkT * 4);
    j.region = c->pkRegion;
    j.shape = shape;
    return LDPC_OK;
}

}  // namespace ldpc
