// Single-scan min-sum in binary32 with frames across lanes (Sec. IV, Eq. 3).
//
// Lane f of a wavefront decodes frame f of a group of 64, and every lane of
// a wavefront works on the same check row or variable, so the code's
// addressing is wave-uniform (scalar loads) and every per-frame array is
// stored frame-minor: element (i, f) at i*Fp + f.  A wavefront's access to
// one posterior or one message is then one contiguous 256-byte transaction,
// whatever the code's wiring.  That keeps codes whose binary32 state does
// not fit on chip streaming through HBM at full line efficiency.
//
// One iteration is two passes over the whole batch:
//   check pass     t_j = Z^(k-1)[n_j] - L^(k-1)_j, min1/argmin/min2 of |t_j|,
//                  sign parity; L^(k)_j = sign_j * (j == argmin ? B : A) with
//                  A = max(alpha*min1 - beta, 0), B likewise from min2 (the
//                  product rounded before the subtraction).
//   variable pass  Z^(k)[n] = Z^(0)[n] + sum of L^(k) over M(n), added in
//                  ascending check order: the fixed order of a sequential
//                  decoder that visits the rows in order, so the result does
//                  not depend on scheduling.
// Messages are stored in variable-major edge order (the order of the
// variable-to-check index), so the check pass writes each message to the
// position the variable pass streams it from.
//
// Syndrome early stop (Sec. III stopping rule): the check pass of iteration
// k+1 also forms the syndrome of the hard decisions of Z^(k) and marks the
// frames with an unsatisfied row; the variable pass of iteration k+1 then
// freezes, for good, the posteriors of every frame whose syndrome passed at
// some iteration <= k, which reproduces a per-frame decoder that stops at the
// first iteration whose syndrome is zero.
#include "fl_common.h"

namespace ldpc {
namespace {

using namespace fl;

struct FlArgs {
    int32_t M, N, F, Fp, G;  // Fp = 64 * V * G frames (V per lane, 64 lanes per wavefront)
    int32_t rwaves;          // wavefronts per frame group in the strided passes
    uint32_t ebytes;         // bytes of the message array (E * Fp * 4 < 2^31)
    float alpha, beta;
    const int32_t *row_ptr;  // [M+1]
    const uint32_t *row_ent; // [E + 64][2] per check-to-variable edge: {variable, message position}
                             // (64 padding entries: a row's slots load unconditionally)
    const int32_t *vc_ptr;   // [N+1] message positions of variable n: vc_ptr[n] .. vc_ptr[n+1]
    float *z0;               // [N][Fp]
    float *zbuf[2];          // [N][Fp] posteriors of odd / even iterations
    float *L;                // [E][Fp] messages, variable-major edge order
    int32_t *fail;           // [K+1][Fp] 1 = syndrome of Z^(k) not satisfied
    int32_t *conv;           // [Fp] first iteration whose syndrome passed
    const float *W;          // null, or [Tw][C][2] (a, b) per iteration and row-degree class
    int32_t Tw, C;
    const int32_t *row_cls;  // [M] class of each row (with W)
};

__device__ __forceinline__ float norm_f(float m, float alpha, float beta) {
    const float v = __fsub_rn(__fmul_rn(alpha, m), beta);
    return v > 0.0f ? v : 0.0f;
}

// Check pass of iteration k (UPDATE), or the syndrome of zold alone.
//   syn_row >= 0: record rows failing the syndrome of zold in fail[syn_row]
//   conv_k  >= 1: first fold fail[conv_k] into conv (one wavefront)
// FIRST: L^(k-1) = 0 (iteration 1), the message array is not read.
// V frames per lane (1 or 4: consecutive frames, one 16-byte access each).
template <int DMAX, bool UPDATE, bool FIRST, int V>
__global__ void __launch_bounds__(kBlock) fl_check(FlArgs a, const float *__restrict__ zold, int syn_row,
                                                   int conv_k, int it) {
    const int lane = threadIdx.x & 63;
    const int w = wave_id();
    const int Fp = a.Fp;
    if (conv_k >= 1 && w == 0) fold_conv(a.conv, a.fail, conv_k, Fp, lane);
    if (w >= a.rwaves * a.G) return;
    const int g = w % a.G;
    const int r0 = w / a.G;
    const uint32_t f0 = (uint32_t)((g * 64 + lane) * V);  // first frame of the lane
    const uint32_t fo = f0 * 4u;                          // lane offset in bytes
    const uint32_t rowb = (uint32_t)Fp * 4u;              // bytes per element row
    const Buf zb(zold, (uint32_t)a.N * rowb), lb(a.L, a.ebytes);
    const auto *rp = cptr(a.row_ptr);
    const auto *re = cptr(a.row_ent);
    for (int m = r0; m < a.M; m += a.rwaves) {
        const int e0 = rp[m];
        const int d = rp[m + 1] - e0;
        float z[DMAX][V], t[DMAX][V];
        uint32_t pos[DMAX], var[DMAX];
        // the row's index entries (scalar loads), then all its data loads, then
        // the arithmetic, with no branch between them (slots j >= d are out of
        // range and masked)
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
            const uint32_t nv = re[2 * (e0 + j)], np = re[2 * (e0 + j) + 1];
            var[j] = j < d ? nv * rowb : kOutOfRange;
            pos[j] = j < d ? np * rowb : kOutOfRange;
        }
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
            zb.ldv<V, 0>(z[j], fo, var[j]);
            if (UPDATE) {
                if (FIRST) {
#pragma unroll
                    for (int c = 0; c < V; ++c) t[j][c] = 0.0f;
                } else {
                    lb.ldv<V, kNonTemporal>(t[j], fo, pos[j]);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < V; ++c) {  // each frame on its own
            int syn = 0, par = 0;
            float min1 = INFINITY, min2 = INFINITY;
            int idx = 0;
#pragma unroll
            for (int j = 0; j < DMAX; ++j) {
                const bool in = j < d;
                syn ^= (in && !(z[j][c] > 0.0f)) ? 1 : 0;
                if (UPDATE) {
                    const float tj = __fsub_rn(z[j][c], t[j][c]);
                    t[j][c] = tj;
                    par ^= (in && tj < 0.0f) ? 1 : 0;
                    const float av = in ? fabsf(tj) : INFINITY;
                    min2 = fminf(min2, fmaxf(min1, av));
                    idx = av < min1 ? j : idx;
                    min1 = fminf(min1, av);
                }
            }
            if (syn_row >= 0 && syn) a.fail[(size_t)syn_row * Fp + f0 + c] = 1;
            if (UPDATE) {
                float wa = a.alpha, wb = a.beta;
                if (a.W) {  // per-iteration, per-class pair
                    const auto *Wt = cptr(a.W) + (size_t)(min(it, a.Tw) - 1) * a.C * 2;
                    const int cl = a.C > 1 ? cptr(a.row_cls)[m] : 0;  // one column: a pair per iteration
                    wa = Wt[2 * cl];
                    wb = Wt[2 * cl + 1];
                }
                const float A = norm_f(min1, wa, wb);
                const float B = norm_f(min2, wa, wb);
#pragma unroll
                for (int j = 0; j < DMAX; ++j) {
                    const float mag = j == idx ? B : A;
                    const bool neg = (par ^ (t[j][c] < 0.0f ? 1 : 0)) != 0;
                    t[j][c] = neg ? -mag : mag;  // L^(k)_j
                }
            }
        }
        if (UPDATE) {
#pragma unroll
            for (int j = 0; j < DMAX; ++j) lb.stv<V, kNonTemporal>(t[j], fo, pos[j]);
        }
    }
}

// Variable pass of iteration k: znew = z0 + messages in ascending check
// order; frames frozen by the early stop copy zold instead.
template <bool FREEZE, int V>
__global__ void __launch_bounds__(kBlock) fl_var(FlArgs a, const float *__restrict__ zold, float *__restrict__ znew,
                                                 int fail_row) {
    const int lane = threadIdx.x & 63;
    const int w = wave_id();
    const int Fp = a.Fp;
    if (w >= a.rwaves * a.G) return;
    const int g = w % a.G;
    const uint32_t f0 = (uint32_t)((g * 64 + lane) * V);
    const uint32_t fo = f0 * 4u;
    const uint32_t rowb = (uint32_t)Fp * 4u;
    const uint32_t nb = (uint32_t)a.N * rowb;
    const Buf zo(zold, nb), zn(znew, nb), z0(a.z0, nb), lb(a.L, a.ebytes);
    bool frozen[V];
    bool all_frozen = true, any_frozen = false;
#pragma unroll
    for (int c = 0; c < V; ++c) {
        frozen[c] = FREEZE && (a.conv[f0 + c] != kNotConverged || a.fail[(size_t)fail_row * Fp + f0 + c] == 0);
        all_frozen = all_frozen && frozen[c];
        any_frozen = any_frozen || frozen[c];
    }
    // frozen frames copy Z_old: a lane whose frames are all frozen loads no
    // messages, a lane with none frozen no copy (out-of-range offsets move no
    // data and need no branch)
    const uint32_t fs = (FREEZE && all_frozen) ? kOutOfRange : fo;
    const uint32_t fc = (FREEZE && any_frozen) ? fo : kOutOfRange;
    const auto *vp = cptr(a.vc_ptr);
    for (int n = w / a.G; n < a.N; n += a.rwaves) {
        const uint32_t o = (uint32_t)n * rowb;
        const int e0 = vp[n], e1 = vp[n + 1];
        float s[V], cp[V], l[4][V];
        z0.ldv<V, kNonTemporal>(s, fs, o);
        if (FREEZE) zo.ldv<V, 0>(cp, fc, o);
        // messages four at a time, the first four issued with z0; slots past
        // the variable's last edge are out of range and skipped (no +0.0 is
        // added, so each sum is exactly the ordered one)
        for (int e = e0; e < e1; e += 4) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                lb.ldv<V, kNonTemporal>(l[i], fs, e + i < e1 ? (uint32_t)(e + i) * rowb : kOutOfRange);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int c = 0; c < V; ++c) s[c] = e + i < e1 ? __fadd_rn(s[c], l[i][c]) : s[c];
        }
        if (FREEZE) {
#pragma unroll
            for (int c = 0; c < V; ++c) s[c] = frozen[c] ? cp[c] : s[c];
        }
        zn.stv<V, 0>(s, fo, o);
    }
}

template <int DMAX, int V>
hipError_t run(const DecodeArgs &d, const FlArgs &a, int K, unsigned grid, hipStream_t s) {
    const bool es = d.early_stop != 0;
    const dim3 tgrid((unsigned)((a.N + 63) / 64), (unsigned)(a.Fp / 64));
    hipLaunchKernelGGL(transpose_in<float>, tgrid, dim3(kBlock), 0, s, static_cast<const float *>(d.llr_in), a.z0,
                       a.N, a.F, a.Fp);
    const int64_t nfail = (int64_t)(K + 1) * a.Fp;
    hipLaunchKernelGGL(init_flags, dim3((unsigned)((std::max<int64_t>(nfail, a.Fp) + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, s, a.fail, nfail, a.conv, a.Fp);
    const float *zold = a.z0;
    for (int k = 1; k <= K; ++k) {
        float *znew = a.zbuf[k & 1];
        // syndrome of Z^(k-1) (k >= 2), fold fail[k-2] into conv (k >= 3)
        const int syn_row = (es && k >= 2) ? k - 1 : -1;
        const int conv_k = (es && k >= 3) ? k - 2 : 0;
        if (k == 1)
            hipLaunchKernelGGL((fl_check<DMAX, true, true, V>), dim3(grid), dim3(kBlock), 0, s, a, zold, syn_row,
                               conv_k, k);
        else
            hipLaunchKernelGGL((fl_check<DMAX, true, false, V>), dim3(grid), dim3(kBlock), 0, s, a, zold, syn_row,
                               conv_k, k);
        if (es && k >= 2)
            hipLaunchKernelGGL((fl_var<true, V>), dim3(grid), dim3(kBlock), 0, s, a, zold, znew, k - 1);
        else
            hipLaunchKernelGGL((fl_var<false, V>), dim3(grid), dim3(kBlock), 0, s, a, zold, znew, 0);
        zold = znew;
    }
    // syndrome of the final posteriors, then the outputs
    hipLaunchKernelGGL((fl_check<DMAX, false, false, V>), dim3(grid), dim3(kBlock), 0, s, a, zold, K,
                       (es && K >= 3) ? K - 2 : 0, K);
    hipLaunchKernelGGL(frame_out, dim3((unsigned)((a.F + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, a.fail, a.conv,
                       a.F, a.Fp, K, d.early_stop, d.iters_out, d.ok_out);
    hipLaunchKernelGGL(transpose_out<float>, tgrid, dim3(kBlock), 0, s, zold, a.N, a.F, a.Fp, 1.0, d.hard_out,
                       d.llr_out);
    return hipGetLastError();
}

}  // namespace

// Frames per call chunk: every frame-minor array of a chunk below 2 GiB.
int fl_chunk_frames(int N, int64_t E) { return fl::chunk_frames(std::max<int64_t>(E, N) * 4); }

namespace {
// Frames per lane and per chunk of a call: four per lane (16-byte accesses)
// once a chunk holds at least 256 frames, chunks then a multiple of 256.
struct FlPlan {
    int V, chunk;
};
FlPlan fl_plan(int N, int64_t E, int n_frames) {
    const int chunk = fl_chunk_frames(N, E);
    if (std::min(n_frames, chunk) >= 256) return {4, chunk / 256 * 256};
    return {1, chunk};
}
size_t round_frames(int F, int V) { return (size_t)((F + 64 * V - 1) / (64 * V)) * 64 * V; }
}  // namespace

// Rows above 16 entries keep one frame per lane: four frames of a 32-slot
// row need all 256 registers of a lane, and the occupancy lost costs more than
// the wider accesses gain.  The frame padding of the plan stays.
int fl_frames_per_lane(int N, int64_t E, int n_frames, int max_row_deg) {
    return (fl_plan(N, E, n_frames).V == 4 && max_row_deg <= 16) ? 4 : 1;
}

size_t fl_workspace_bytes(int N, int64_t E, int n_frames, int max_iter) {
    const FlPlan pl = fl_plan(N, E, n_frames);
    const int fr = std::min(n_frames, std::max(pl.chunk, 1));
    const size_t Fp = round_frames(fr, pl.V);
    return 3 * fl::al256((size_t)N * Fp * 4) + fl::al256((size_t)E * Fp * 4) +
           fl::al256((size_t)(max_iter + 1) * Fp * 4) + fl::al256(Fp * 4);
}

hipError_t launch_ss_f32_fl(const DecodeArgs &d, const int32_t *row_ptr, const uint32_t *row_ent, int64_t E,
                            int max_row_deg, int cu_count, const float *weights, int weight_iters,
                            const int32_t *row_cls, int n_classes, hipStream_t s) {
    const FlPlan pl = fl_plan(d.c.N, E, d.n_frames);
    const int chunk = pl.chunk;
    if (chunk <= 0 || max_row_deg > 64) return hipErrorInvalidValue;
    for (int c0 = 0; c0 < d.n_frames; c0 += chunk) {
        const int F = std::min(chunk, d.n_frames - c0);
        DecodeArgs dc = d;
        dc.n_frames = F;
        dc.llr_in = static_cast<const float *>(d.llr_in) + (size_t)c0 * d.c.N;
        dc.hard_out = d.hard_out + (size_t)c0 * d.c.N;
        dc.llr_out = d.llr_out ? d.llr_out + (size_t)c0 * d.c.N : nullptr;
        dc.iters_out = d.iters_out + c0;
        dc.ok_out = d.ok_out + c0;
        FlArgs a{};
        a.M = d.c.M;
        a.N = d.c.N;
        a.F = F;
        const int V = fl_frames_per_lane(d.c.N, E, d.n_frames, max_row_deg);
        a.Fp = (int)round_frames(F, pl.V);
        a.G = a.Fp / (64 * V);
        a.alpha = d.alpha;
        a.beta = d.beta;
        a.row_ptr = row_ptr;
        a.row_ent = row_ent;
        a.vc_ptr = d.c.vc_ptr;
        a.W = weights;
        a.Tw = weight_iters;
        a.C = n_classes;
        a.row_cls = row_cls;
        const size_t Fp = (size_t)a.Fp;
        a.ebytes = (uint32_t)((size_t)E * Fp * 4);
        uint8_t *p = d.ws;
        a.z0 = reinterpret_cast<float *>(p);
        p += fl::al256((size_t)a.N * Fp * 4);
        a.zbuf[0] = reinterpret_cast<float *>(p);
        p += fl::al256((size_t)a.N * Fp * 4);
        a.zbuf[1] = reinterpret_cast<float *>(p);
        p += fl::al256((size_t)a.N * Fp * 4);
        a.L = reinterpret_cast<float *>(p);
        p += fl::al256((size_t)E * Fp * 4);
        a.fail = reinterpret_cast<int32_t *>(p);
        p += fl::al256((size_t)(d.max_iter + 1) * Fp * 4);
        a.conv = reinterpret_cast<int32_t *>(p);
        unsigned grid;
        wave_layout(cu_count, a.G, std::max(a.M, a.N), &a.rwaves, &grid);
        const int K = d.max_iter;
        hipError_t e;
        if (V == 4)
            e = max_row_deg <= 8 ? run<8, 4>(dc, a, K, grid, s) : run<16, 4>(dc, a, K, grid, s);
        else
            e = max_row_deg <= 8    ? run<8, 1>(dc, a, K, grid, s)
                : max_row_deg <= 16 ? run<16, 1>(dc, a, K, grid, s)
                : max_row_deg <= 32 ? run<32, 1>(dc, a, K, grid, s)
                                    : run<64, 1>(dc, a, K, grid, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace ldpc
