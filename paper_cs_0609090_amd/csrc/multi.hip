// Mixed batches (several codes in one call) and per-code layout autotuning;
// C ABI declared in include/ldpc_multi.h.
//
// A mixed call runs every job's ordinary decode kernels, but on a pool of
// library streams forked from and joined back into the caller's stream with
// events: kernels of different codes share the chip (a 128-frame job of a
// long code fills half of the CUs with one workgroup per frame, the short
// codes fill the rest), and the fork/join pattern is capturable, so a caller
// can record the whole mixed call into one HIP graph and replay it.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ldpc_multi.h"
#include "code_handle.h"
#include "ldpc_internal.h"

namespace {

constexpr int kPool = 4;  // library streams per device

struct Pool {
    std::mutex mu;  // held while a call enqueues its fork/join
    hipStream_t s[kPool] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kPool] = {};
};

std::mutex g_pools_mu;
std::vector<std::unique_ptr<Pool>> g_pools;  // by device ordinal; kept until the process ends

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// The pool of `dev` (created on first use, with `dev` current).
ldpc_status pool_for(int dev, Pool **out) {
    std::lock_guard<std::mutex> lk(g_pools_mu);
    if ((int)g_pools.size() <= dev) g_pools.resize(dev + 1);
    if (!g_pools[dev]) {
        auto p = std::make_unique<Pool>();
        hipError_t e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming);
        for (int i = 0; i < kPool && e == hipSuccess; ++i) {
            e = hipStreamCreateWithFlags(&p->s[i], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&p->join[i], hipEventDisableTiming);
        }
        if (e != hipSuccess)  // the partial pool is leaked: creation failing leaves the device unusable anyway
            return ldpc::set_error(LDPC_EDEVICE, std::string("stream pool: ") + hipGetErrorString(e));
        g_pools[dev] = std::move(p);
    }
    *out = g_pools[dev].get();
    return LDPC_OK;
}

std::string job_prefix(int j) { return "job " + std::to_string(j) + ": "; }

// Per-job workspace sizes and offsets (256-byte aligned, in job order).
ldpc_status job_layout(const ldpc_job *jobs, int32_t n_jobs, std::vector<size_t> *off, size_t *total) {
    if (n_jobs < 0) return ldpc::set_error(LDPC_EINVAL, "n_jobs < 0");
    if (n_jobs > 0 && !jobs) return ldpc::set_error(LDPC_EINVAL, "jobs is NULL");
    off->assign(n_jobs, 0);
    size_t t = 0;
    int dev = -1;
    for (int j = 0; j < n_jobs; ++j) {
        const ldpc_job &b = jobs[j];
        if (!b.code) return ldpc::set_error(LDPC_EINVAL, job_prefix(j) + "code is NULL");
        if (b.params.flags & LDPC_F_CHECK_INPUT)
            return ldpc::set_error(LDPC_EINVAL, job_prefix(j) +
                                                    "LDPC_F_CHECK_INPUT synchronises; check inputs with "
                                                    "ldpc_decode_batch");
        if (b.n_frames > 0) {
            if (dev >= 0 && b.code->device != dev)
                return ldpc::set_error(LDPC_EINVAL, job_prefix(j) + "codes of one call must share a device");
            dev = b.code->device;
        }
        size_t need = 0;
        ldpc_status st = ldpc_decode_workspace_size(b.code, b.n_frames, &b.params, &need);
        if (st != LDPC_OK) return ldpc::set_error(st, job_prefix(j) + ldpc_last_error());
        t = align256(t);
        (*off)[j] = t;
        t += need;
    }
    *total = t;
    return LDPC_OK;
}

double job_work(const ldpc_job &b) {
    return (double)b.n_frames * (double)b.code->E * (double)std::max(b.params.max_iter, 1);
}

// Deterministic pseudo-random channel values for autotuning trials (the
// timing of the decoders does not depend on them with early stop off).
__global__ void trial_llr_kernel(void *out, int64_t count, int fp32) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        uint32_t h = (uint32_t)i * 0x9E3779B1u;
        h ^= h >> 15;
        h *= 0x85EBCA77u;
        h ^= h >> 13;
        if (fp32)
            static_cast<float *>(out)[i] = (float)(h % 4001u) * (1.0f / 250.0f) - 4.0f;  // [-4, 12]
        else
            static_cast<int8_t *>(out)[i] = (int8_t)((int)(h % 42u) - 10);  // [-10, 31]
    }
}

}  // namespace

extern "C" {

ldpc_status ldpc_multi_workspace_size(const ldpc_job *jobs, int32_t n_jobs, size_t *bytes) {
    if (!bytes) return ldpc::set_error(LDPC_EINVAL, "bytes is NULL");
    std::vector<size_t> off;
    return job_layout(jobs, n_jobs, &off, bytes);
}

ldpc_status ldpc_decode_multi(const ldpc_job *jobs, int32_t n_jobs, void *workspace, size_t workspace_bytes,
                              void *stream) {
    std::vector<size_t> off;
    size_t total = 0;
    ldpc_status st = job_layout(jobs, n_jobs, &off, &total);
    if (st != LDPC_OK) return st;
    if (total > 0 && (!workspace || workspace_bytes < total))
        return ldpc::set_error(LDPC_EINVAL, "workspace missing or smaller than ldpc_multi_workspace_size()");
    if (workspace && (reinterpret_cast<uintptr_t>(workspace) & 255u))
        return ldpc::set_error(LDPC_EINVAL, "workspace must be 256-byte aligned");
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    std::vector<int> active;
    for (int j = 0; j < n_jobs; ++j) {
        const ldpc_job &b = jobs[j];
        st = ldpc::decode_job(b.code, b.n_frames, b.llr_in, &b.params, b.hard_out, b.llr_out, b.iters_out,
                              b.syndrome_ok, ws ? ws + off[j] : nullptr, ws ? workspace_bytes - off[j] : 0,
                              stream, false);
        if (st != LDPC_OK) return ldpc::set_error(st, job_prefix(j) + ldpc_last_error());
        if (b.n_frames > 0 && b.params.max_iter >= 0) active.push_back(j);
    }
    auto launch = [&](int j, void *s) {
        const ldpc_job &b = jobs[j];
        ldpc_status r = ldpc::decode_job(b.code, b.n_frames, b.llr_in, &b.params, b.hard_out, b.llr_out,
                                         b.iters_out, b.syndrome_ok, ws ? ws + off[j] : nullptr,
                                         ws ? workspace_bytes - off[j] : 0, s, true);
        return r == LDPC_OK ? r : ldpc::set_error(r, job_prefix(j) + ldpc_last_error());
    };
    if (active.empty()) return LDPC_OK;
    if (active.size() == 1) return launch(active[0], stream);

    const int dev = jobs[active[0]].code->device;
    ldpc::DeviceGuard g(dev);
    if (!g.ok) return ldpc::set_error(LDPC_EDEVICE, "hipSetDevice failed");
    Pool *pool = nullptr;
    st = pool_for(dev, &pool);
    if (st != LDPC_OK) return st;

    // A job whose workgroups each take more than half of a CU's LDS (one
    // frame per CU) can start a workgroup only on an empty CU; launched at the
    // same time as the others, it waits until their workgroups leave whole
    // CUs free (measured: the N=64800 job of the mixed workload ran 4.1 ms
    // instead of 1.1).  The largest such job goes first, on the caller's
    // stream, ahead of the forked ones; the rest go longest first onto the
    // least loaded library stream.
    int lead = -1, lead_lds = 0;
    for (size_t k = 0; k < active.size(); ++k) {
        const ldpc_job &b = jobs[active[k]];
        ldpc_plan_info pi{};
        if (ldpc_decode_plan(b.code, b.n_frames, &b.params, &pi) != LDPC_OK) continue;
        if (2 * (int64_t)pi.lds_bytes > (int64_t)b.code->lds_limit && pi.lds_bytes > lead_lds) {
            lead = active[k];
            lead_lds = pi.lds_bytes;
        }
    }
    if (lead >= 0) active.erase(std::find(active.begin(), active.end(), lead));
    std::stable_sort(active.begin(), active.end(),
                     [&](int x, int y) { return job_work(jobs[x]) > job_work(jobs[y]); });
    double load[kPool] = {0, 0, 0, 0};
    std::vector<int> where(active.size());
    int used = 0;
    for (size_t k = 0; k < active.size(); ++k) {
        const int i = (int)(std::min_element(load, load + kPool) - load);
        where[k] = i;
        load[i] += job_work(jobs[active[k]]);
        used = std::max(used, i + 1);
    }

    std::lock_guard<std::mutex> lk(pool->mu);
    hipStream_t caller = static_cast<hipStream_t>(stream);
    hipError_t e = hipEventRecord(pool->fork, caller);
    if (e != hipSuccess) return ldpc::set_error(LDPC_EDEVICE, std::string("fork: ") + hipGetErrorString(e));
    ldpc_status first = LDPC_OK;
    std::string first_msg;
    if (lead >= 0) {  // after the fork point, so the forked jobs do not wait for it
        first = launch(lead, caller);
        if (first != LDPC_OK) first_msg = ldpc_last_error();
    }
    for (int i = 0; i < used && e == hipSuccess; ++i) e = hipStreamWaitEvent(pool->s[i], pool->fork, 0);
    if (e != hipSuccess) return ldpc::set_error(LDPC_EDEVICE, std::string("fork: ") + hipGetErrorString(e));
    for (size_t k = 0; k < active.size(); ++k) {
        ldpc_status r = launch(active[k], pool->s[where[k]]);
        if (r != LDPC_OK && first == LDPC_OK) {
            first = r;
            first_msg = ldpc_last_error();
        }
    }
    // join every forked stream, also after a failed launch, so the caller's
    // stream (or its capture) is left consistent
    for (int i = 0; i < used; ++i) {
        hipError_t ej = hipEventRecord(pool->join[i], pool->s[i]);
        if (ej == hipSuccess) ej = hipStreamWaitEvent(caller, pool->join[i], 0);
        if (ej != hipSuccess && e == hipSuccess) e = ej;
    }
    if (first != LDPC_OK) return ldpc::set_error(first, first_msg);
    if (e != hipSuccess) return ldpc::set_error(LDPC_EDEVICE, std::string("join: ") + hipGetErrorString(e));
    ldpc::clear_error();
    return LDPC_OK;
}

ldpc_status ldpc_multi_persistent_workspace_size(const ldpc_job *jobs, int32_t n_jobs, size_t *bytes) {
    if (!bytes) return ldpc::set_error(LDPC_EINVAL, "bytes is NULL");
    std::vector<size_t> off;
    size_t total = 0;
    ldpc_status st = job_layout(jobs, n_jobs, &off, &total);
    if (st != LDPC_OK) return st;
    *bytes = 256;  // the work-item counter
    return LDPC_OK;
}

ldpc_status ldpc_decode_multi_persistent(const ldpc_job *jobs, int32_t n_jobs, void *workspace,
                                         size_t workspace_bytes, void *stream) {
    std::vector<size_t> off;
    size_t total = 0;
    ldpc_status st = job_layout(jobs, n_jobs, &off, &total);
    if (st != LDPC_OK) return st;
    if (!workspace || workspace_bytes < 256)
        return ldpc::set_error(LDPC_EINVAL, "workspace missing or smaller than "
                                            "ldpc_multi_persistent_workspace_size()");
    if (reinterpret_cast<uintptr_t>(workspace) & 255u)
        return ldpc::set_error(LDPC_EINVAL, "workspace must be 256-byte aligned");
    std::vector<int> active;
    for (int j = 0; j < n_jobs; ++j)
        if (jobs[j].n_frames > 0) active.push_back(j);
    if ((int)active.size() > ldpc::kMaxPersistJobs)
        return ldpc::set_error(LDPC_EUNSUPPORTED, "the persistent launch takes at most 8 jobs with frames");
    ldpc::PersistArgs pa{};
    size_t lds = 0;
    bool fused = true;
    for (size_t k = 0; k < active.size(); ++k) {
        const ldpc_job &b = jobs[active[k]];
        st = ldpc::persist_job(b.code, b.n_frames, b.llr_in, &b.params, b.hard_out, b.llr_out, b.iters_out,
                               b.syndrome_ok, &pa.job[k]);
        if (st != LDPC_OK) return ldpc::set_error(st, job_prefix(active[k]) + ldpc_last_error());
        lds = std::max(lds, (size_t)b.code->pkGroups * b.code->pkRegion);
        fused = fused && b.params.early_stop && b.llr_out == nullptr && b.params.max_iter >= 1;
    }
    for (int j = 0; j < n_jobs; ++j)  // jobs without frames are validated too
        if (jobs[j].n_frames == 0) {
            const ldpc_job &b = jobs[j];
            ldpc::PersistJob tmp;
            st = ldpc::persist_job(b.code, 0, b.llr_in, &b.params, b.hard_out, b.llr_out, b.iters_out,
                                   b.syndrome_ok, &tmp);
            if (st != LDPC_OK) return ldpc::set_error(st, job_prefix(j) + ldpc_last_error());
        }
    if (active.empty()) return LDPC_OK;
    const ldpc_code *c0 = jobs[active[0]].code;
    if (lds + 16 > (size_t)c0->lds_limit)
        return ldpc::set_error(LDPC_EUNSUPPORTED, "the jobs' LDS regions do not fit one workgroup");
    // longest frames first (so the last items are short), work items job after job
    std::vector<int> order(active.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        const ldpc_job &a = jobs[active[x]], &b = jobs[active[y]];
        return (double)a.code->E * a.params.max_iter > (double)b.code->E * b.params.max_iter;
    });
    ldpc::PersistArgs sorted{};
    int items = 0;
    for (size_t k = 0; k < order.size(); ++k) {
        sorted.job[k] = pa.job[order[k]];
        sorted.job[k].first = items;
        const int G = jobs[active[order[k]]].code->pkGroups;
        items += (jobs[active[order[k]]].n_frames + G - 1) / G;
    }
    sorted.njobs = (int)order.size();
    sorted.nitems = items;
    sorted.counter = static_cast<int32_t *>(workspace);
    sorted.off_item = (uint32_t)((lds + 15) / 16 * 16);
    ldpc::DeviceGuard g(c0->device);
    if (!g.ok) return ldpc::set_error(LDPC_EDEVICE, "hipSetDevice failed");
    const int grid = std::min(items, std::max(c0->cu_count, 1));
    hipError_t e = ldpc::launch_ss_pk_persist(sorted, fused, sorted.off_item + 16, grid,
                                             static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return ldpc::set_error(LDPC_EDEVICE, std::string("persistent launch: ") + hipGetErrorString(e));
    ldpc::clear_error();
    return LDPC_OK;
}

ldpc_status ldpc_autotune(ldpc_code *code, int32_t n_frames, const ldpc_decode_params *p, int32_t *best_layout,
                          float *best_ms, int32_t *n_tried) {
    if (!code || !p || !best_layout) return ldpc::set_error(LDPC_EINVAL, "NULL argument");
    if (n_frames < 1) return ldpc::set_error(LDPC_EINVAL, "n_frames < 1");
    if (p->weights) return ldpc::set_error(LDPC_EINVAL, "autotuning is for decoding without per-iteration weights");
    if (code->device < 0) return ldpc::set_error(LDPC_EINVAL, "host-only handle (device < 0)");
    static const int kCand[] = {LDPC_LAYOUT_REG, LDPC_LAYOUT_REG1, LDPC_LAYOUT_LDS, LDPC_LAYOUT_HBM,
                                LDPC_LAYOUT_FRAMES};
    ldpc_decode_params q[5];
    size_t need[5];
    bool feasible[5];
    size_t ws_max = 0;
    int nfeas = 0;
    {  // the parameters themselves must be valid under the automatic layout
        ldpc_decode_params a = *p;
        a.flags &= ~(0xFu << LDPC_F_LAYOUT_SHIFT);
        ldpc_status st = ldpc_decode_workspace_size(code, n_frames, &a, &need[0]);
        if (st != LDPC_OK) return st;
    }
    for (int i = 0; i < 5; ++i) {
        q[i] = *p;
        q[i].early_stop = 0;
        q[i].flags = (p->flags & ~(0xFu << LDPC_F_LAYOUT_SHIFT) & ~LDPC_F_CHECK_INPUT) |
                     ((uint32_t)kCand[i] << LDPC_F_LAYOUT_SHIFT);
        feasible[i] = ldpc_decode_workspace_size(code, n_frames, &q[i], &need[i]) == LDPC_OK;
        if (feasible[i]) {
            ws_max = std::max(ws_max, need[i]);
            ++nfeas;
        }
    }
    if (nfeas == 0) return ldpc::set_error(LDPC_EUNSUPPORTED, "no layout can run these parameters");

    ldpc::DeviceGuard g(code->device);
    if (!g.ok) return ldpc::set_error(LDPC_EDEVICE, "hipSetDevice failed");
    // REG on a handle with a packed shape runs the packed kernel: its other
    // shapes (threads per workgroup, hence frames per CU) are timed as well
    const std::vector<std::array<int, 4>> shapes =
        feasible[0] && code->pkD > 0 ? ldpc::pk_candidates(code) : std::vector<std::array<int, 4>>();
    const std::array<int, 4> orig = {code->pkD, code->pkR, code->pkT, code->pkS};
    std::array<int, 4> best_shape = orig;
    const bool fp32 = p->msg == LDPC_MSG_FP32;
    const size_t cnt = (size_t)n_frames * (size_t)code->N;
    void *llr = nullptr, *ws = nullptr;
    uint8_t *hard = nullptr, *ok = nullptr;
    int32_t *iters = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ldpc::reset_alloc_count();
    // a shape change frees arrays that work queued earlier may still read
    hipError_t e = shapes.size() > 1 ? hipDeviceSynchronize() : hipSuccess;
    if (e == hipSuccess) e = ldpc::dev_malloc(&llr, cnt * (fp32 ? 4 : 1));
    if (e == hipSuccess) e = ldpc::dev_malloc(reinterpret_cast<void **>(&hard), cnt);
    if (e == hipSuccess) e = ldpc::dev_malloc(reinterpret_cast<void **>(&iters), 4 * (size_t)n_frames);
    if (e == hipSuccess) e = ldpc::dev_malloc(reinterpret_cast<void **>(&ok), (size_t)n_frames);
    if (e == hipSuccess && ws_max > 0) e = ldpc::dev_malloc(&ws, ws_max);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    ldpc_status st = LDPC_OK;
    std::string msg;
    int best = 0, tried = 0;
    float best_t = 0.0f;
    if (e == hipSuccess) {
        const int64_t blocks = std::min<int64_t>(((int64_t)cnt + 255) / 256, 4096);
        hipLaunchKernelGGL(trial_llr_kernel, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, s, llr,
                           (int64_t)cnt, fp32 ? 1 : 0);
        e = hipGetLastError();
    }
    // makes a packed shape the handle's (nothing to do when it already is)
    auto install = [&](const std::array<int, 4> &sh) -> ldpc_status {
        if (sh[0] == code->pkD && sh[1] == code->pkR && sh[2] == code->pkT && sh[3] == code->pkS) return LDPC_OK;
        if (s && (e = hipStreamSynchronize(s)) != hipSuccess) return LDPC_EDEVICE;
        return ldpc::pk_install(code, sh[0], sh[1], sh[2], sh[3]);
    };
    for (int i = 0; i < 5 && e == hipSuccess && st == LDPC_OK; ++i) {
        if (!feasible[i]) continue;
        const size_t nsh = kCand[i] == LDPC_LAYOUT_REG && !shapes.empty() ? shapes.size() : 1;
        for (size_t k = 0; k < nsh && e == hipSuccess && st == LDPC_OK; ++k) {
            if (nsh > 1) {
                st = install(shapes[k]);
                if (st != LDPC_OK) {
                    msg = e != hipSuccess ? std::string("autotune: ") + hipGetErrorString(e) : ldpc_last_error();
                    break;
                }
            }
            float t_min = 0.0f;
            for (int rep = 0; rep < 4 && st == LDPC_OK && e == hipSuccess; ++rep) {
                e = hipEventRecord(e0, s);
                if (e != hipSuccess) break;
                st = ldpc::decode_job(code, n_frames, llr, &q[i], hard, nullptr, iters, ok, ws, ws_max, s, true);
                if (st != LDPC_OK) {
                    msg = ldpc_last_error();
                    break;
                }
                e = hipEventRecord(e1, s);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.0f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (rep > 0 && (rep == 1 || ms < t_min)) t_min = ms;  // rep 0 is the warm-up
            }
            if (st != LDPC_OK || e != hipSuccess) break;
            ++tried;
            if (best == 0 || t_min < best_t) {
                best = kCand[i];
                best_t = t_min;
                if (nsh > 1) best_shape = shapes[k];
            }
        }
    }
    if (e != hipSuccess && st == LDPC_OK) {
        st = LDPC_EDEVICE;
        msg = std::string("autotune: ") + hipGetErrorString(e);
    }
    // the winning packed shape when REG won, else the handle's own
    if (shapes.size() > 1) {
        const hipError_t e_keep = e;
        e = hipSuccess;
        const ldpc_status sti = install(st == LDPC_OK && best == LDPC_LAYOUT_REG ? best_shape : orig);
        if (sti != LDPC_OK && st == LDPC_OK) {
            st = sti;
            msg = e != hipSuccess ? std::string("autotune: ") + hipGetErrorString(e) : ldpc_last_error();
        }
        if (e == hipSuccess) e = e_keep;
    }
    if (s) (void)hipStreamSynchronize(s);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    if (ws) (void)hipFree(ws);
    if (ok) (void)hipFree(ok);
    if (iters) (void)hipFree(iters);
    if (hard) (void)hipFree(hard);
    if (llr) (void)hipFree(llr);
    if (st != LDPC_OK) return ldpc::set_error(st, msg);
    __atomic_store_n(&code->tuned_layout[ldpc::tuned_slot(p)], best, __ATOMIC_RELAXED);
    *best_layout = best;
    if (best_ms) *best_ms = best_t;
    if (n_tried) *n_tried = tried;
    ldpc::clear_error();
    return LDPC_OK;
}

ldpc_status ldpc_code_packed_shapes(const ldpc_code *code, int32_t *shapes, int32_t cap, int32_t *count) {
    if (!code || !count || cap < 0 || (cap > 0 && !shapes)) return ldpc::set_error(LDPC_EINVAL, "NULL argument");
    const std::vector<std::array<int, 4>> c = ldpc::pk_candidates(code);
    for (size_t i = 0; i < c.size() && (int64_t)i < cap; ++i) {
        shapes[3 * i] = c[i][0];
        shapes[3 * i + 1] = c[i][1];
        shapes[3 * i + 2] = c[i][2];
    }
    *count = (int32_t)c.size();
    ldpc::clear_error();
    return LDPC_OK;
}

ldpc_status ldpc_code_set_packed_shape(ldpc_code *code, int32_t slots, int32_t rows_per_thread, int32_t threads) {
    if (!code) return ldpc::set_error(LDPC_EINVAL, "NULL argument");
    if (code->device < 0) return ldpc::set_error(LDPC_EINVAL, "host-only handle (device < 0)");
    for (const std::array<int, 4> &sh : ldpc::pk_candidates(code))
        if (sh[0] == slots && sh[1] == rows_per_thread && sh[2] == threads) {
            ldpc::reset_alloc_count();
            const ldpc_status st = ldpc::pk_install(code, sh[0], sh[1], sh[2], sh[3]);
            if (st != LDPC_OK) return ldpc::set_error(st, ldpc_last_error());
            ldpc::clear_error();
            return LDPC_OK;
        }
    return ldpc::set_error(LDPC_EUNSUPPORTED, "not one of ldpc_code_packed_shapes() for this code");
}

}  // extern "C"
